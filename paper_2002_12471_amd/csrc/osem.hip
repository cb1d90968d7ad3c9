// Kernels of one OS-LM-MLEM sub-iteration (Eq. 7-8).
//
//   forward      h_j(q) = sum over paths from q of  w G(E_j; E') K(u_j - u_end)
//                (the system row of event j), stored as a row of H, and the
//                partial sums of f_q h_j(q) over each pixel group
//   mean         mean_j = sum_q f_q h_j(q)  (denominator of Eq. 8)
//   backproject  b_q = sum_j h_j(q) / mean_j over a chunk of rows, one
//                column slice per thread: every output has one owner, so no
//                atomics and a fixed summation order
//   update       f_q <- f_q * b_q / sens_q  (Eq. 7)
//
// The forward kernel is the hot loop.  A workgroup owns one tile of up to EV
// events of one angle, sorted by detector position, and up to 256 emission
// pixels (one per lane).  For every path end in the tile's rank range it reads the
// (alpha, beta) pair of each lane's path once and reuses it for all EV
// events; per event the term is one FMA for the exponent, one exp2 and one
// FMA into the accumulator.  The event factor
//     K'_js = K(u_j - u_s) / Z_K * 2^(-c2 (E_j - e_c)^2)
// is computed once per (event, path end) into LDS and read back as a
// broadcast; the energy factor 2^(-c2 (E_j - e_c)^2) / Z_K is precomputed per
// event at ingest.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "lmosem_int.h"

namespace lmo {

constexpr int kRch = 128;   // path-end ranks staged in LDS per pass

// Per-event wave sums of a tile, EV values per lane, by halving exchanges:
// at each step a lane pairs with a partner that differs in one lane bit,
// keeps half of its values (the upper half when that bit is set), and adds
// the partner's copy of the half it kept.  The lane bits are taken in the
// order 3, 2, 0, 1, 4, 5, whose partners are a row mirror, a half-row
// mirror, two quad permutations (all DPP operands of the add) and shuffles
// across rows; each pairing flips its bit and only bits not yet used, so the
// two partners always hold the same events.  After log2(EV) halving steps a
// lane holds one event, its index read from the used bits (first one most
// significant); plain sums over the remaining bits finish the wave total.
template <int B>
__device__ __forceinline__ float partner(float v) {
    if constexpr (B == 3) return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false));
    else if constexpr (B == 2) return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false));
    else if constexpr (B == 0) return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
    else if constexpr (B == 1) return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
    else return __shfl_xor(v, 1 << B, 64);
}

constexpr int kSumBits[6] = {3, 2, 0, 1, 4, 5};

template <int S, int N, int EV>
__device__ __forceinline__ void halve_events(float (&v)[EV], int lane, int &e) {
    if constexpr (S < 6) {
        constexpr int B = kSumBits[S];
        if constexpr (N > 1) {
            const bool up = (lane >> B) & 1;
#pragma unroll
            for (int i = 0; i < N / 2; ++i) {
                const float send = up ? v[i] : v[i + N / 2];
                const float keep = up ? v[i + N / 2] : v[i];
                v[i] = keep + partner<B>(send);
            }
            e = 2 * e + (up ? 1 : 0);
            halve_events<S + 1, N / 2, EV>(v, lane, e);
        } else {
            v[0] += partner<B>(v[0]);
            halve_events<S + 1, 1, EV>(v, lane, e);
        }
    }
}

// the writer lanes: every bit not used for halving is 0
template <int EV>
constexpr int writer_mask() {
    int m = 0, n = EV;
    for (int s = 0; s < 6; ++s) {
        if (n > 1) n /= 2;
        else m |= 1 << kSumBits[s];
    }
    return m;
}

// buffer resource word 3 of the gfx9 family (raw, untyped 32-bit access)
constexpr int kBufferWord3 = 0x00020000;

// the (alpha, beta) entries of four consecutive ranks of each lane's column
__device__ __forceinline__ void load_group(__amdgpu_buffer_rsrc_t rs, uint32_t lane_off, uint32_t row0,
                                           uint32_t rstride, float2 (&v)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
        v[i] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, lane_off, row0 + i * rstride, 0));
}

// the terms of NR (of four loaded) ranks for all EV events: exponent FMA,
// exp2, accumulate
template <int EV, int NR = 4>
__device__ __forceinline__ void term_group(const float2 (&v)[4], const float *Kg, const float (&et)[EV],
                                           float (&acc)[EV]) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const float4 *kr = reinterpret_cast<const float4 *>(Kg + i * EV);
        float4 k4[EV / 4];
#pragma unroll
        for (int e4 = 0; e4 < EV / 4; ++e4) k4[e4] = kr[e4];
        float x[EV];
#pragma unroll
        for (int e = 0; e < EV; ++e) x[e] = fmaf(v[i].y, et[e], v[i].x);
#pragma unroll
        for (int e = 0; e < EV; ++e) x[e] = __builtin_amdgcn_exp2f(x[e]);
#pragma unroll
        for (int e4 = 0; e4 < EV / 4; ++e4) {
            acc[4 * e4 + 0] = fmaf(k4[e4].x, x[4 * e4 + 0], acc[4 * e4 + 0]);
            acc[4 * e4 + 1] = fmaf(k4[e4].y, x[4 * e4 + 1], acc[4 * e4 + 1]);
            acc[4 * e4 + 2] = fmaf(k4[e4].z, x[4 * e4 + 2], acc[4 * e4 + 2]);
            acc[4 * e4 + 3] = fmaf(k4[e4].w, x[4 * e4 + 3], acc[4 * e4 + 3]);
        }
    }
}

// the last group of a chunk, with its 1 to 4 ranks (a wave-uniform count):
// rank by rank behind scalar branches
template <int EV>
__device__ __forceinline__ void term_tail(const float2 (&v)[4], const float *Kg, const float (&et)[EV],
                                          float (&acc)[EV], int nr_last) {
    const float2 v0[4] = {v[0], v[0], v[0], v[0]};
    term_group<EV, 1>(v0, Kg, et, acc);
#pragma unroll
    for (int i = 1; i < 4; ++i) {
        if (i < nr_last) {
            const float2 vi[4] = {v[i], v[i], v[i], v[i]};
            term_group<EV, 1>(vi, Kg + i * EV, et, acc);
        }
    }
}

template <int EV>
__device__ __forceinline__ void forward_item(const Geo &g, const Tile *__restrict__ tiles, int n_tiles,
                                             int logical, const float2 *__restrict__ T,
                                             const double *__restrict__ us_sorted,
                                             const float *__restrict__ su, const float *__restrict__ se,
                                             const float *__restrict__ efac, const float *__restrict__ f,
                                             float *__restrict__ H, float *__restrict__ pmean, int row_base,
                                             int n_rows, float *Ks, float *red, int tid, int wave, int lane) {
    const int grp = logical / n_tiles;
    const Tile tl = tiles[logical - grp * n_tiles];
    const int gw = 64 * g.fwd_waves;   // pixels per group = threads per workgroup
    const int q = grp * gw + tid;
    const bool wave_on = grp * gw + wave * 64 < g.n_qpad;

    float et[EV], acc[EV];
#pragma unroll
    for (int e = 0; e < EV; ++e) {
        et[e] = e < tl.n ? se[tl.e0 + e] : 0.0f;
        acc[e] = 0.0f;
    }
    // the table rows of a chunk of ranks as a buffer resource: the per-lane
    // column offset is the VGPR offset and the rank row the SGPR offset, so a
    // table load needs no vector address arithmetic; loads past the angle's
    // rows (the prefetch one group beyond a tile's last rank) return 0 and are
    // unused
    const uint32_t rstride = (uint32_t)g.n_qpad * (uint32_t)sizeof(float2);
    const float2 *Ta = T + (size_t)tl.angle * g.n_rpad * g.n_qpad;
    const uint32_t lane_off = (uint32_t)(wave_on ? q : 0) * (uint32_t)sizeof(float2);
    const double *us = us_sorted + (size_t)tl.angle * g.n_p;
    const float inv2s2 = (float)(1.0 / (2.0 * g.sig_u * g.sig_u));
    const float edge = expf(-4.5f);

    // the staging thread's event (fixed: the group width is a multiple of
    // EV) with its position in FP64 (both positions are O(10 cm)) and its
    // energy factor, read once per tile
    const int e_st = tid & (EV - 1), r_st = tid / EV, r_step = gw / EV;
    const bool e_ok = e_st < tl.n;
    const double u_st = e_ok ? ((double)su[tl.e0 + e_st] - 0.5 * g.n_bins) * g.bin_cm : 0.0;
    const float ef_st = e_ok ? efac[tl.e0 + e_st] : 0.0f;
    for (int rc = tl.r0; rc < tl.r1; rc += kRch) {
        const int nr = min(kRch, tl.r1 - rc);
        const int nr4 = (nr + 3) & ~3;      // ranks rounded up to whole groups of 4 (K' = 0 past nr)
        __syncthreads();
        for (int r = r_st; r < nr4; r += r_step) {
            float kv = 0.0f;
            if (e_ok && r < nr) {
                // offset in FP64, response in FP32
                const float d = (float)(u_st - us[rc + r]);
                const float gk = __expf(-d * d * inv2s2) - edge;
                kv = gk > 0.0f ? gk * ef_st : 0.0f;
            }
            Ks[r * EV + e_st] = kv;
        }
        __syncthreads();
        if (wave_on) {
            // groups of 4 ranks in two alternating register sets: the next
            // group's entries are loaded while this one is computed.  With 8
            // events per tile the chunk's last group computes only its own 1
            // to 4 ranks; with more (where the separate tail costs registers
            // and waves) it runs whole, its padding ranks meeting K' = 0.
            // Loads past the tile read padding rows of the table, unused.
            constexpr bool kExactTail = EV == 8;
            const int n_full = __builtin_amdgcn_readfirstlane(kExactTail ? (nr - 1) >> 2 : nr4 >> 2);
            const int nr_last = __builtin_amdgcn_readfirstlane(nr - 4 * n_full);
            const uint64_t left = (uint64_t)(g.n_rpad - rc) * rstride;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<float2 *>(Ta + (size_t)rc * g.n_qpad), (short)0,
                (int)(uint32_t)std::min<uint64_t>(left, 0xFFFFFFFFull), kBufferWord3);
            float2 a[4], b[4];
            load_group(rs, lane_off, 0u, rstride, a);
            int gi = 0;
            for (; gi + 1 < n_full; gi += 2) {
                load_group(rs, lane_off, (uint32_t)(gi + 1) * 4u * rstride, rstride, b);
                term_group<EV>(a, Ks + gi * 4 * EV, et, acc);
                load_group(rs, lane_off, (uint32_t)(gi + 2) * 4u * rstride, rstride, a);
                term_group<EV>(b, Ks + (gi + 1) * 4 * EV, et, acc);
            }
            if constexpr (kExactTail) {
                if (gi < n_full) {   // one full group in a, then the last group
                    load_group(rs, lane_off, (uint32_t)(gi + 1) * 4u * rstride, rstride, b);
                    term_group<EV>(a, Ks + gi * 4 * EV, et, acc);
                    term_tail<EV>(b, Ks + (gi + 1) * 4 * EV, et, acc, nr_last);
                } else {             // a holds the last group
                    term_tail<EV>(a, Ks + gi * 4 * EV, et, acc, nr_last);
                }
            } else {
                if (gi < n_full) term_group<EV>(a, Ks + gi * 4 * EV, et, acc);
            }
        }
    }

    if (wave_on) {
        float *Hq = H + (size_t)(tl.e0 - row_base) * g.n_qpad + q;
#pragma unroll
        for (int e = 0; e < EV; ++e)
            if (e < tl.n) Hq[(size_t)e * g.n_qpad] = acc[e];
    }
    const float fq = (wave_on && q < g.n_q) ? f[(size_t)tl.real * g.n_qpad + q] : 0.0f;
    {
        float v[EV];
#pragma unroll
        for (int e = 0; e < EV; ++e) v[e] = fq * acc[e];
        int e = 0;
        halve_events<0, EV, EV>(v, lane, e);
        if ((lane & writer_mask<EV>()) == 0) red[wave * EV + e] = v[0];
    }
    __syncthreads();
    if (tid < tl.n) {
        float s;
        if (g.fwd_waves == 4) {
            s = (red[tid] + red[EV + tid]) + (red[2 * EV + tid] + red[3 * EV + tid]);
        } else {
            s = red[tid];
            for (int w = 1; w < g.fwd_waves; ++w) s += red[w * EV + tid];
        }
        pmean[(size_t)grp * n_rows + (tl.e0 - row_base) + tid] = s;
    }
}

// Map the dispatch index to a logical (pixel group, tile) item so that each
// XCD (workgroups are dealt to the 8 XCDs round-robin) runs one contiguous run
// of items: consecutive tiles of one angle and pixel group then share that
// XCD's L2 copy of the path-table slice they read.  (A persistent kernel that
// drained per-XCD work queues was measured slower than this hardware-
// scheduled grid on this workload.)
__device__ inline int xcd_logical(int p, int n) {
    constexpr int kXcd = 8;
    const int x = p % kXcd, k = p / kXcd;
    const int m = n / kXcd, rem = n % kXcd;
    return x * m + min(x, rem) + k;
}

// (the 8-event kernel fits 64 VGPRs without spilling: eight waves per SIMD,
// measured 1-2 % faster than the seven its unbounded allocation allows; the
// wider tiles spill when pressed below their own counts)
template <int EV>
__global__ __launch_bounds__(256, EV == 8 ? 8 : 1) void k_forward(Geo g, const Tile *__restrict__ tiles, int n_tiles,
                                                 const float2 *__restrict__ T,
                                                 const double *__restrict__ us_sorted,
                                                 const float *__restrict__ su,
                                                 const float *__restrict__ se,
                                                 const float *__restrict__ efac,
                                                 const float *__restrict__ f,
                                                 float *__restrict__ H, float *__restrict__ pmean,
                                                 int row_base, int n_rows) {
    __shared__ __align__(16) float Ks[kRch * EV];
    __shared__ float red[4 * EV];
    const int n_groups = forward_groups(g);
    const int logical = xcd_logical(blockIdx.x, n_tiles * n_groups);
    const int tid = threadIdx.x;
    forward_item<EV>(g, tiles, n_tiles, logical, T, us_sorted, su, se, efac, f, H, pmean, row_base, n_rows, Ks,
                     red, tid, tid >> 6, tid & 63);
}

// pixel groups of the forward launch (one group per workgroup)
__host__ __device__ int forward_groups(const Geo &g) { return (g.n_qpad + 64 * g.fwd_waves - 1) / (64 * g.fwd_waves); }

// a launch, with the kernel's own start and end events when ke is given
template <typename K, typename... A>
static hipError_t launch(K kernel, dim3 grid, dim3 block, hipStream_t st, const KernelEvents *ke, A... args) {
    if (ke)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, ke->start, ke->stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
    return hipGetLastError();
}

// nothing to launch: the events still bracket an (empty) interval
static hipError_t no_launch(const KernelEvents *ke, hipStream_t st) {
    if (!ke) return hipSuccess;
    hipError_t e = hipEventRecord(ke->start, st);
    return e == hipSuccess ? hipEventRecord(ke->stop, st) : e;
}

template <int EV>
static hipError_t launch_ev(const Geo &g, const Tables &t, const Tile *tiles, int n_tiles, const float *ev_u,
                            const float *ev_e, const float *efac, const float *f, float *H, float *pmean,
                            int row_base, int n_rows, hipStream_t st, const KernelEvents *ke) {
    const int n_work = n_tiles * forward_groups(g);
    return launch(k_forward<EV>, dim3(n_work), dim3(64 * g.fwd_waves), st, ke, g, tiles, n_tiles,
                  (const float2 *)t.T, (const double *)t.us_sorted, ev_u, ev_e, efac, f, H, pmean, row_base, n_rows);
}

hipError_t launch_forward(int ev_tile, const Geo &g, const Tables &t, const Tile *tiles, int n_tiles,
                          const float *ev_u, const float *ev_e, const float *efac, const float *f, float *H,
                          float *pmean, int row_base, int n_rows, hipStream_t st, const KernelEvents *ke) {
    if (n_tiles <= 0) return no_launch(ke, st);
    switch (ev_tile) {
    case 16:
        return launch_ev<16>(g, t, tiles, n_tiles, ev_u, ev_e, efac, f, H, pmean, row_base, n_rows, st, ke);
    case 32:
        return launch_ev<32>(g, t, tiles, n_tiles, ev_u, ev_e, efac, f, H, pmean, row_base, n_rows, st, ke);
    default:
        return launch_ev<8>(g, t, tiles, n_tiles, ev_u, ev_e, efac, f, H, pmean, row_base, n_rows, st, ke);
    }
}

__global__ void k_mean(const float *__restrict__ pmean, int n_groups, int n_rows,
                       float *__restrict__ mean, float *__restrict__ inv,
                       unsigned long long *__restrict__ skipped) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    int dead = 0;
    if (j < n_rows) {
        // the partials in batches of 8 loads in flight, added in group order
        float s = 0.0f;
        for (int k0 = 0; k0 < n_groups; k0 += 8) {
            float p[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) p[u] = k0 + u < n_groups ? pmean[(size_t)(k0 + u) * n_rows + j] : 0.0f;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u < n_groups) s += p[u];
        }
        mean[j] = s;
        dead = !(s > 1e-30f);
        inv[j] = dead ? 0.0f : 1.0f / s;
    }
    const unsigned long long m = __ballot(dead);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(skipped, (unsigned long long)__popcll(m));
}

hipError_t launch_mean(const float *pmean, int n_groups, int n_rows, float *mean, float *inv,
                       unsigned long long *skipped, hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mean, dim3((n_rows + 255) / 256), dim3(256), 0, st, pmean, n_groups, n_rows,
                       mean, inv, skipped);
    return hipGetLastError();
}

// Cached system rows (the rows do not depend on f): the event mean
// mean[j] = sum_q f[real(j)][q] H[j][q] over whole padded rows (padding is zero
// in both) and its inverse (0, and counted, when the mean is not positive).
// LPR lanes per row (64, or 16 for short rows so that a wave takes four rows
// at once), float4 loads and a butterfly sum; bound by reading H.  Each lane
// issues a batch of row loads (4 for short rows, which is all of them, 8
// otherwise) before the first multiply, so a wave has a whole brain-sized
// row in flight instead of one float4 per round trip; loads past the row end
// are zeroed.  The row's realisation is looked up in offsets staged in LDS;
// a short row's loads are issued before the lookup, so it hides under them
// (a batch of many short realisations has a lookup per few hundred bytes).
constexpr int kRowRealLds = 1024;   // realisation offsets kept in LDS (more: read from memory)

template <int N>
__device__ __forceinline__ void row_batch(const float4 *h, int k0, int step, int n4, float4 (&x)[N]) {
#pragma unroll
    for (int u = 0; u < N; ++u) {
        const int k = k0 + u * step;
        const float4 v = h[min(k, n4 - 1)];
        x[u] = k < n4 ? v : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}

template <int LPR>
__global__ __launch_bounds__(256) void k_row_dot(Geo g, const int *__restrict__ rrange, int n_real, int n_rows,
                                                 const float *__restrict__ H, const float *__restrict__ f,
                                                 float *__restrict__ mean, float *__restrict__ inv,
                                                 unsigned long long *__restrict__ skipped) {
    constexpr int kRowsPerBlock = 256 / LPR;
    constexpr int kLoads = LPR == 16 ? 4 : 8;
    __shared__ int rr_s[kRowRealLds + 1];
    const bool rr_in_lds = n_real <= kRowRealLds;
    if (rr_in_lds)
        for (int i = threadIdx.x; i <= n_real; i += 256) rr_s[i] = rrange[i];
    __syncthreads();
    const int *rr = rr_in_lds ? rr_s : rrange;
    const int sub = threadIdx.x % LPR;
    const int n4 = g.n_qpad / 4;
    for (int j = blockIdx.x * kRowsPerBlock + threadIdx.x / LPR; j < n_rows; j += gridDim.x * kRowsPerBlock) {
        const float4 *h = reinterpret_cast<const float4 *>(H + (size_t)j * g.n_qpad);
        float4 x[kLoads];
        // short rows: the whole row is one batch, issued before the lookup
        if constexpr (LPR == 16) row_batch(h, sub, LPR, n4, x);
        int lo = 0, hi = n_real;   // realisation r with rrange[r] <= j < rrange[r+1]
        while (hi - lo > 1) { const int m = (lo + hi) >> 1; if (rr[m] <= j) lo = m; else hi = m; }
        const float4 *fr = reinterpret_cast<const float4 *>(f + (size_t)lo * g.n_qpad);
        float s4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int k0 = sub; k0 < n4; k0 += kLoads * LPR) {
            if (LPR != 16 || k0 != sub) row_batch(h, k0, LPR, n4, x);   // (short rows take one pass)
            float4 y[kLoads];
            row_batch(fr, k0, LPR, n4, y);
#pragma unroll
            for (int u = 0; u < kLoads; ++u) {
                float &a = s4[u & 3];
                a = fmaf(x[u].x, y[u].x, a);
                a = fmaf(x[u].y, y[u].y, a);
                a = fmaf(x[u].z, y[u].z, a);
                a = fmaf(x[u].w, y[u].w, a);
            }
        }
        float s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
#pragma unroll
        for (int off = LPR / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        if (sub == 0) {
            const bool dead = !(s > 1e-30f);
            mean[j] = s;
            inv[j] = dead ? 0.0f : 1.0f / s;
            if (dead) atomicAdd(skipped, 1ull);
        }
    }
}

hipError_t launch_row_dot(const Geo &g, const int *rrange, int n_real, int n_rows, const float *H, const float *f,
                          float *mean, float *inv, unsigned long long *skipped, hipStream_t st,
                          const KernelEvents *ke) {
    if (n_rows <= 0) return no_launch(ke, st);
    if (g.n_qpad / 4 <= 64)   // rows of at most 256 floats: 16 lanes each
        return launch(k_row_dot<16>, dim3(std::min((n_rows + 15) / 16, 16384)), dim3(256), st, ke, g, rrange, n_real,
                      n_rows, H, f, mean, inv, skipped);
    return launch(k_row_dot<64>, dim3(std::min((n_rows + 3) / 4, 16384)), dim3(256), st, ke, g, rrange, n_real, n_rows,
                  H, f, mean, inv, skipped);
}

// pb[c][q] = sum_{j in chunk c} H[j][q] inv[j]; four columns per thread,
// blockDim.x threads per block along the row.
__global__ __launch_bounds__(256) void k_backproject(Geo g, const Chunk *__restrict__ chunks,
                                                     const float *__restrict__ H,
                                                     const float *__restrict__ inv,
                                                     float *__restrict__ pb) {
    const Chunk c = chunks[blockIdx.y];
    const int q4 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (q4 >= g.n_qpad) return;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const float *Hp = H + (size_t)c.j0 * g.n_qpad + q4;
#pragma unroll 8
    for (int j = c.j0; j < c.j1; ++j) {
        const float4 h = *reinterpret_cast<const float4 *>(Hp);
        const float w = inv[j];
        acc.x = fmaf(h.x, w, acc.x);
        acc.y = fmaf(h.y, w, acc.y);
        acc.z = fmaf(h.z, w, acc.z);
        acc.w = fmaf(h.w, w, acc.w);
        Hp += g.n_qpad;
    }
    *reinterpret_cast<float4 *>(pb + (size_t)blockIdx.y * g.n_qpad + q4) = acc;
}

// The backprojection with the event means formed first (the forward path,
// so that no separate means kernel runs): each block adds its chunk's
// pixel-group partials in group order, as k_mean does, into LDS; the first
// column block also writes the means, their inverses and the dead-event
// count; then the rows are weighted from LDS.
__global__ __launch_bounds__(256) void k_backproject_means(Geo g, const Chunk *__restrict__ chunks,
                                                           const float *__restrict__ H,
                                                           const float *__restrict__ pmean, int n_groups,
                                                           int n_rows, float *__restrict__ mean,
                                                           float *__restrict__ inv,
                                                           unsigned long long *__restrict__ skipped,
                                                           float *__restrict__ pb) {
    __shared__ float w_s[kMaxChunkRows];
    const Chunk c = chunks[blockIdx.y];
    const int n = c.j1 - c.j0;   // at most kMaxChunkRows (the plan's chunk size)
    for (int i0 = 0; i0 < n; i0 += blockDim.x) {
        const int i = i0 + threadIdx.x, j = c.j0 + i;
        int dead = 0;
        if (i < n) {
            float s = 0.0f;
            for (int k0 = 0; k0 < n_groups; k0 += 8) {
                float p[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) p[u] = k0 + u < n_groups ? pmean[(size_t)(k0 + u) * n_rows + j] : 0.0f;
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (k0 + u < n_groups) s += p[u];
            }
            dead = !(s > 1e-30f);
            const float w = dead ? 0.0f : 1.0f / s;
            w_s[i] = w;
            if (blockIdx.x == 0) {
                mean[j] = s;
                inv[j] = w;
            }
        }
        const unsigned long long m = __ballot(dead);
        if (blockIdx.x == 0 && (threadIdx.x & 63) == 0 && m) atomicAdd(skipped, (unsigned long long)__popcll(m));
    }
    __syncthreads();
    const int q4 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (q4 >= g.n_qpad) return;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const float *Hp = H + (size_t)c.j0 * g.n_qpad + q4;
#pragma unroll 8
    for (int i = 0; i < n; ++i) {
        const float4 h = *reinterpret_cast<const float4 *>(Hp);
        const float w = w_s[i];
        acc.x = fmaf(h.x, w, acc.x);
        acc.y = fmaf(h.y, w, acc.y);
        acc.z = fmaf(h.z, w, acc.z);
        acc.w = fmaf(h.w, w, acc.w);
        Hp += g.n_qpad;
    }
    *reinterpret_cast<float4 *>(pb + (size_t)blockIdx.y * g.n_qpad + q4) = acc;
}

// the fewest blocks of up to 256 threads that cover the row's float4
// columns, each a whole number of waves with as few idle lanes as that
// allows (brain64's 368 columns: two blocks of 192 rather than 256 + 112)
static dim3 backproject_block(const Geo &g) {
    const int n4 = g.n_qpad / 4;
    const int nb = (n4 + 255) / 256;
    return dim3((unsigned)(((n4 + nb - 1) / nb + 63) / 64 * 64));
}

hipError_t launch_backproject(const Geo &g, const Chunk *chunks, int n_chunks, const float *H,
                              const float *inv, float *pb, hipStream_t st, const KernelEvents *ke) {
    if (n_chunks <= 0) return no_launch(ke, st);
    const dim3 blk = backproject_block(g);
    const dim3 grid((unsigned)((g.n_qpad / 4 + blk.x - 1) / blk.x), (unsigned)n_chunks);
    return launch(k_backproject, grid, blk, st, ke, g, chunks, H, inv, pb);
}

hipError_t launch_backproject_means(const Geo &g, const Chunk *chunks, int n_chunks, int chunk_rows,
                                    const float *H, const float *pmean, int n_groups, int n_rows, float *mean,
                                    float *inv, unsigned long long *skipped, float *pb, hipStream_t st,
                                    const KernelEvents *ke) {
    if (chunk_rows > kMaxChunkRows) return hipErrorInvalidValue;
    if (n_chunks <= 0) return no_launch(ke, st);
    const dim3 blk = backproject_block(g);
    const dim3 grid((unsigned)((g.n_qpad / 4 + blk.x - 1) / blk.x), (unsigned)n_chunks);
    return launch(k_backproject_means, grid, blk, st, ke, g, chunks, H, pmean, n_groups, n_rows, mean, inv, skipped,
                  pb);
}

// f[r][q] <- f[r][q] * b / sens with b summed over realisation r's chunks:
// 64 pixels per block, the chunks split over kUpdWaves waves (4 accumulators
// each, so a brain-sized subset's ~100 chunk partials take two rounds of
// loads) and the wave partials added in a fixed order.
constexpr int kUpdWaves = 16;

__global__ __launch_bounds__(64 * kUpdWaves) void k_update(Geo g, const int *__restrict__ crange,
                                                          const float *__restrict__ pb,
                                                          const float *__restrict__ sens, float *__restrict__ f) {
    constexpr int W = kUpdWaves;
    __shared__ float part[W][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q = blockIdx.x * 64 + lane;
    const int r = blockIdx.y;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    if (q < g.n_q) {
        const int c0 = crange[r], c1 = crange[r + 1];
        int c = c0 + wv;
        for (; c + 3 * W < c1; c += 4 * W) {
            a0 += pb[(size_t)c * g.n_qpad + q];
            a1 += pb[(size_t)(c + W) * g.n_qpad + q];
            a2 += pb[(size_t)(c + 2 * W) * g.n_qpad + q];
            a3 += pb[(size_t)(c + 3 * W) * g.n_qpad + q];
        }
        for (; c < c1; c += W) a0 += pb[(size_t)c * g.n_qpad + q];
    }
    part[wv][lane] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (wv == 0 && q < g.n_q) {
        float b4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            b4[k] = 0.0f;
#pragma unroll
            for (int w = k; w < W; w += 4) b4[k] += part[w][lane];
        }
        const float b = (b4[0] + b4[1]) + (b4[2] + b4[3]);
        const float s = sens[q];
        float *fp = f + (size_t)r * g.n_qpad + q;
        if (s > 0.0f) *fp = (*fp * b) / s;
    }
}

hipError_t launch_update(const Geo &g, const int *crange, int n_real, const float *pb,
                         const float *sens, float *f, hipStream_t st) {
    hipLaunchKernelGGL(k_update, dim3((g.n_q + 63) / 64, n_real), dim3(64 * kUpdWaves), 0, st, g, crange, pb, sens,
                       f);
    return hipGetLastError();
}

// out[r][q] = sum over realisation r's chunks of pb[c][q]
__global__ void k_sum_real(Geo g, const int *__restrict__ crange, const float *__restrict__ pb,
                           float *__restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (q >= g.n_qpad) return;
    float b = 0.0f;
    for (int c = crange[r]; c < crange[r + 1]; ++c) b += pb[(size_t)c * g.n_qpad + q];
    out[(size_t)r * g.n_qpad + q] = q < g.n_q ? b : 0.0f;
}

hipError_t launch_sum_real(const Geo &g, const int *crange, int n_real, const float *pb, float *out,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_sum_real, dim3((g.n_qpad + 255) / 256, n_real), dim3(256), 0, st, g, crange, pb,
                       out);
    return hipGetLastError();
}

// ll[r] += sum_{rows of r} log mean_j - sum_q f_q sens_q  (one block per realisation)
__global__ __launch_bounds__(256) void k_loglik(Geo g, const int *__restrict__ rrange,
                                                const float *__restrict__ mean,
                                                const float *__restrict__ f,
                                                const float *__restrict__ sens, double *__restrict__ ll) {
    __shared__ double red[256];
    const int r = blockIdx.x, tid = threadIdx.x;
    double s = 0.0;
    for (int j = rrange[r] + tid; j < rrange[r + 1]; j += 256) {
        const float m = mean[j];
        if (m > 1e-30f) s += log((double)m);
    }
    for (int q = tid; q < g.n_q; q += 256) s -= (double)f[(size_t)r * g.n_qpad + q] * (double)sens[q];
    red[tid] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) ll[r] += red[0];
}

hipError_t launch_loglik(const Geo &g, const int *rrange, int n_real, const float *mean, const float *f,
                         const float *sens, double *ll, hipStream_t st) {
    hipLaunchKernelGGL(k_loglik, dim3(n_real), dim3(256), 0, st, g, rrange, mean, f, sens, ll);
    return hipGetLastError();
}

// compact activity f[r][q] from images [r][ny][nx] (stride 0: one shared image);
// a null image means 1 on the support
__global__ void k_gather_image(Geo g, const int *__restrict__ p_pix, const float *__restrict__ img,
                               int64_t stride, float *__restrict__ f) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (q >= g.n_qpad) return;
    float v = 0.0f;
    if (q < g.n_q) v = img ? img[(size_t)r * stride + p_pix[q]] : 1.0f;
    f[(size_t)r * g.n_qpad + q] = v;
}

hipError_t launch_gather_image(const Geo &g, const Tables &t, const float *img, int n_real,
                               int64_t img_stride, float *f, int, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_image, dim3((g.n_qpad + 255) / 256, n_real), dim3(256), 0, st, g, t.p_pix,
                       img, img_stride, f);
    return hipGetLastError();
}

// images [r][ny][nx] from compact f (0 off the emission set)
__global__ void k_scatter_image(Geo g, const int *__restrict__ q_of_pix, const float *__restrict__ f,
                                float *__restrict__ img) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (p >= g.n_pix) return;
    const int q = q_of_pix[p];
    img[(size_t)r * g.n_pix + p] = (q >= 0 && q < g.n_q) ? f[(size_t)r * g.n_qpad + q] : 0.0f;
}

// q_of_pix is stored right after p_pix in the same allocation
hipError_t launch_scatter_image(const Geo &g, const Tables &t, const float *f, int n_real, float *img,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_image, dim3((g.n_pix + 255) / 256, n_real), dim3(256), 0, st, g,
                       t.p_pix + g.n_p, f, img);
    return hipGetLastError();
}

__global__ void k_scatter_rows(const float *__restrict__ src, const int *__restrict__ orig, int n,
                               float *__restrict__ dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[orig[k]] = src[k];
}

hipError_t launch_scatter_rows(const float *src, const int *orig, int n, float *dst, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_rows, dim3((n + 255) / 256), dim3(256), 0, st, src, orig, n, dst);
    return hipGetLastError();
}

__global__ void k_gather_rows(const float *__restrict__ src, const int *__restrict__ orig, int n,
                              float *__restrict__ dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[orig[k]];
}

hipError_t launch_gather_rows(const float *src, const int *orig, int n, float *dst, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows, dim3((n + 255) / 256), dim3(256), 0, st, src, orig, n, dst);
    return hipGetLastError();
}

__global__ void k_fill(float *__restrict__ p, size_t n, float v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill(float *p, size_t n, float v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

__global__ void k_fill_d(double *__restrict__ p, size_t n, double v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_d(double *p, size_t n, double v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// count support pixels whose value is negative or not finite
__global__ void k_check_image(Geo g, const int *__restrict__ p_pix, const float *__restrict__ img,
                              int *__restrict__ bad) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    int b = 0;
    if (q < g.n_q) {
        const float v = img[p_pix[q]];
        b = !(v >= 0.0f && v <= 3.4e38f);
    }
    const unsigned long long m = __ballot(b);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(bad, (int)__popcll(m));
}

hipError_t launch_check_image(const Geo &g, const Tables &t, const float *img, int *bad, hipStream_t st) {
    hipLaunchKernelGGL(k_check_image, dim3((g.n_q + 255) / 256), dim3(256), 0, st, g, t.p_pix, img, bad);
    return hipGetLastError();
}

}  // namespace lmo
