// Learned scatter surrogate: features, exact training targets, inference.
//
// The surrogate replaces the first-order scatter part of the system row,
//     S(q; a, u, E) = sum_{s != q} w(q,s,a) K(u - u_s) G(E; E'(q,s,a)),
// by one network evaluation per (event, emission pixel), for the pairs whose
// event lies outside q's own position response (|u - u_q| >= 3 sig_u).  Inside
// it (the near field, where the scatter ends crowd around q and the sum is
// dominated by a few nearby pixels) the sum is taken exactly from a banded
// table of q's near path ends; the primary term is always exact.
//
// Network inputs (all O(1)) for pixel q, angle a, event position u (cm) and
// energy E (keV), with q at (u_q, d_q) in the detector frame (d toward the
// detector):
//     (u - u_q) / 2               event position relative to q's own
//     (E - 130) / 30              energy
//     (d_in - d_q) / 10           where the event's detector line enters the
//     (d_out - d_q) / 10            body (mu > 0) and leaves it, relative to q
//                                   (both 0 when the line misses the body)
//     ck / 2                      response-weighted attenuation of the line:
//                                   sum_s mu(s) pixel_cm k(u - u_s)
//     L_a(q), L_a^back(q)         attenuation from q toward and away from the detector
//     10 mu(q)                    attenuation coefficient at q
// with k(x) = exp(-x^2 / 2 sig_u^2) - e^-4.5 on |x| < 3 sig_u.
// Target: y = ln(S / S0 + 1e-4) with S0 = 1 / (pixel_cm sigma_E); inverse
// S = S0 max(e^y - 1e-4, 0).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "lmosem_int.h"
#include "mlp_infer.h"
#include "paths.h"

namespace lmo {

constexpr float kTargetFloor = 1e-4f;

// unnormalised truncated position response k(x)
__device__ inline double k_resp(const Geo &g, double x) {
    return fmax(exp(-x * x / (2.0 * g.sig_u * g.sig_u)) - exp(-4.5), 0.0);
}

// FP32 position response (the exact forward kernel evaluates it in
// FP32 too)
__device__ inline float k_resp_f(float d, float inv2s2) {
    return fmaxf(__expf(-d * d * inv2s2) - 0.011108996538242306f, 0.0f);   // e^-4.5
}

struct SurrTables {
    const float *Ldet, *Lback;   // [n_angles][n_p]
    const float *prim;           // [n_angles][n_p] alpha of the primary path
    const int *p_pix;
    const float *mu;
    const double *cs;
    const int *s_sorted;         // [n_angles][n_p]
    const double *us_sorted;     // [n_angles][n_p]
    const float *mu_sorted;      // [n_angles][n_p]
    float inv_nx, inv_nq;        // 1 / nx and 1 / n_q, rounded to FP32 on the host
};

// Column features of the detector line {r : r . t_a = u}: its extent inside
// the body along n_a, by boundary-to-boundary traversal from its entry into
// the grid, and its response-weighted attenuation over the reachable ranks.
// out = (d_in, d_out, ck, hit).
__device__ float4 column(const Geo &g, const SurrTables &st, int a, double u, int2 *reach_ranks = nullptr) {
    const double nx = st.cs[2 * a], ny = st.cs[2 * a + 1];
    const double tx = -ny, ty = nx;
    double d_in = 0.0, d_out = 0.0;
    bool hit = false;
    const double hx = 0.5 * g.nx * g.dx, hy = 0.5 * g.ny * g.dx;
    const double px = u * tx, py = u * ty;          // foot of the line; d = parameter along n
    double t0 = -1e300, t1 = 1e300;
    bool miss = false;
    const double p[2] = {px, py}, dir[2] = {nx, ny}, h[2] = {hx, hy};
    for (int k = 0; k < 2; ++k) {
        if (fabs(dir[k]) < 1e-300) {
            if (p[k] <= -h[k] || p[k] >= h[k]) miss = true;
        } else {
            double lo = (-h[k] - p[k]) / dir[k], hi = (h[k] - p[k]) / dir[k];
            if (lo > hi) { const double sw = lo; lo = hi; hi = sw; }
            t0 = fmax(t0, lo);
            t1 = fmin(t1, hi);
        }
    }
    if (!miss && t1 > t0) {
        double t = t0;
        const double ex = px + t0 * nx, ey = py + t0 * ny;
        const double eps = 1e-9 * g.dx;   // entry pixel, nudged inside along the direction
        int i = (int)floor((ex + eps * nx) / g.dx + 0.5 * g.nx);
        int j = (int)floor((ey + eps * ny) / g.dx + 0.5 * g.ny);
        i = min(max(i, 0), g.nx - 1);
        j = min(max(j, 0), g.ny - 1);
        const int sx = nx > 0 ? 1 : (nx < 0 ? -1 : 0), sy = ny > 0 ? 1 : (ny < 0 ? -1 : 0);
        const double inf = 1e300;
        double tmx = sx ? ((i + (sx > 0 ? 1 : 0) - 0.5 * g.nx) * g.dx - px) / nx : inf;
        double tmy = sy ? ((j + (sy > 0 ? 1 : 0) - 0.5 * g.ny) * g.dx - py) / ny : inf;
        const double tdx = sx ? g.dx / fabs(nx) : inf, tdy = sy ? g.dx / fabs(ny) : inf;
        for (int guard = 0; guard < 4 * (g.nx + g.ny) + 8; ++guard) {
            const double tn = fmin(fmin(tmx, tmy), t1);
            if (tn > t && st.mu[j * g.nx + i] > 0.0f) {
                if (!hit) d_in = t;
                d_out = tn;
                hit = true;
            }
            t = tn;
            if (t >= t1) break;
            if (tmx <= tmy) { i += sx; tmx += tdx; } else { j += sy; tmy += tdy; }
            if (i < 0 || i >= g.nx || j < 0 || j >= g.ny) break;
        }
    }
    const double *us = st.us_sorted + (size_t)a * g.n_p;
    const float *mus = st.mu_sorted + (size_t)a * g.n_p;
    const double reach = 3.0 * g.sig_u;
    int lo = 0, hi = g.n_p;   // first rank with us > u - reach
    while (lo < hi) { const int m = (lo + hi) >> 1; if (us[m] > u - reach) hi = m; else lo = m + 1; }
    int lo2 = lo, hi2 = g.n_p;   // first rank with us >= u + reach
    while (lo2 < hi2) { const int m = (lo2 + hi2) >> 1; if (us[m] >= u + reach) hi2 = m; else lo2 = m + 1; }
    const float inv2s2 = (float)(1.0 / (2.0 * g.sig_u * g.sig_u));
    float ck = 0.0f;
    for (int r = lo; r < lo2; ++r) ck = fmaf(mus[r], k_resp_f((float)(u - us[r]), inv2s2), ck);
    if (reach_ranks) *reach_ranks = make_int2(lo, lo2);
    return make_float4((float)d_in, (float)d_out, ck * (float)g.dx, hit ? 1.0f : 0.0f);
}

// k / d for 0 <= k <= 2^24 (exact in float; pixel indices of grids up to
// 4096 x 4096, pair indices of a batch) through a float reciprocal: the
// estimate's relative error is below 2^-23, so it is off by at most one,
// which one comparison each way corrects
__device__ inline int div_small(int k, int d, float inv_d) {
    int qt = (int)((float)k * inv_d);
    qt += (qt + 1) * d <= k ? 1 : 0;
    qt -= qt * d > k ? 1 : 0;
    return qt;
}

__device__ inline void pixel_frame(const Geo &g, const SurrTables &st, int q, int a, double &uq, double &dq) {
    const int pix = st.p_pix[q];
    const int py = div_small(pix, g.nx, st.inv_nx), px = pix - py * g.nx;
    const double cx = (px - 0.5 * (g.nx - 1)) * g.dx, cy = (py - 0.5 * (g.ny - 1)) * g.dx;
    const double nx = st.cs[2 * a], ny = st.cs[2 * a + 1];
    uq = cx * -ny + cy * nx;
    dq = nx * cx + ny * cy;
}

__device__ inline void features(const Geo &g, const SurrTables &st, int q, int a, double u, double e, float4 col,
                                float *x) {
    double uq, dq;
    pixel_frame(g, st, q, a, uq, dq);
    const bool hit = col.w > 0.5f;
    // (scales as FP64 products: within an FP64 rounding of the quotients)
    x[0] = (float)((u - uq) * 0.5);
    x[1] = (float)((e - 130.0) * (1.0 / 30.0));
    x[2] = hit ? (float)(((double)col.x - dq) * 0.1) : 0.0f;
    x[3] = hit ? (float)(((double)col.y - dq) * 0.1) : 0.0f;
    x[4] = col.z / 2.0f;
    x[5] = st.Ldet[(size_t)a * g.n_p + q];
    x[6] = st.Lback[(size_t)a * g.n_p + q];
    x[7] = 10.0f * st.mu[st.p_pix[q]];
}

// Training samples: features and the exact target, with every path weight
// evaluated from the per-angle line integrals and scatter-point factors (the
// function the table build uses), in FP64.
__global__ void k_surr_samples(Geo g, SurrTables st, const int *__restrict__ q_of_pix,
                               const double *__restrict__ Ld, const double *__restrict__ Bt,
                               const int32_t *__restrict__ pixel, const int32_t *__restrict__ angle,
                               const float *__restrict__ u_bin, const float *__restrict__ energy, int64_t n,
                               float *__restrict__ X, float *__restrict__ target, float *__restrict__ scatter) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int q = q_of_pix[pixel[k]];
    const int a = angle[k];
    const double u = ((double)u_bin[k] - 0.5 * g.n_bins) * g.bin_cm;
    const double e = (double)energy[k];
    const double nx = st.cs[2 * a], ny = st.cs[2 * a + 1];
    const double *us = st.us_sorted + (size_t)a * g.n_p;
    const double reach = 3.0 * g.sig_u;
    const double gnorm = 1.0 / (sqrt(2.0 * M_PI) * g.sig_e * g.zk);   // G and K normalisers
    int lo = 0, hi = g.n_p;   // first rank with us > u - reach
    while (lo < hi) { const int m = (lo + hi) >> 1; if (us[m] > u - reach) hi = m; else lo = m + 1; }
    double s = 0.0;
    for (int r = lo; r < g.n_p && us[r] < u + reach; ++r) {
        const int sp = st.s_sorted[(size_t)a * g.n_p + r];
        if (sp == q) continue;   // the primary path
        const double gk = k_resp(g, u - us[r]);
        if (gk <= 0.0) continue;
        const PathW pw = path_weight(g, st.p_pix, Ld, Bt, nx, ny, a, q, sp);
        const double de = e - pw.ep;
        s += gk * pw.w * exp(-de * de / (2.0 * g.sig_e * g.sig_e)) * gnorm;
    }
    float x[8];
    features(g, st, q, a, u, e, column(g, st, a, u), x);
#pragma unroll
    for (int i = 0; i < 8; ++i) X[k * 8 + i] = x[i];
    const double s0 = 1.0 / (g.dx * g.sig_e);
    target[k] = (float)log(s / s0 + (double)kTargetFloor);
    if (scatter) scatter[k] = (float)s;
}

// per event: column features of its detector line and the rank range
// [r0, r1) of path ends its position response reaches
__global__ void k_event_column(Geo g, SurrTables st, const int *__restrict__ ev_angle, const float *__restrict__ su,
                               int n, float4 *__restrict__ col, int2 *__restrict__ rr) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double u = ((double)su[j] - 0.5 * g.n_bins) * g.bin_cm;
    int2 r;
    col[j] = column(g, st, ev_angle[j], u, &r);
    rr[j] = r;
}

// Inference, step 1: for rows [j0, j0 + rows) of the sub-iteration and every
// emission pixel q, the network inputs, rounded to bf16 here as the network
// would round them (16 bytes per pair).
__global__ void k_surr_pairs(Geo g, SurrTables st, const int *__restrict__ ev_angle, const float *__restrict__ su,
                             const float *__restrict__ se, const float4 *__restrict__ col, int row_base, int j0,
                             int rows, uint16_t *__restrict__ X) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;   // pairs per launch <= 2^23
    if (k >= rows * g.n_q) return;
    const int lr = div_small(k, g.n_q, st.inv_nq);
    const int jr = j0 + lr, q = k - lr * g.n_q;
    const int j = row_base + jr;   // index into the sorted events
    const int a = ev_angle[j];
    const double u = ((double)su[j] - 0.5 * g.n_bins) * g.bin_cm;
    const float et = se[j];   // E - e_c
    float x[8];
    features(g, st, q, a, u, (double)et + g.e_c, col[j - row_base], x);
    uint4 packed;
    uint32_t *w = reinterpret_cast<uint32_t *>(&packed);
#pragma unroll
    for (int i = 0; i < 4; ++i)   // two inputs per word, the lower-numbered in the low half
        w[i] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{x[2 * i], x[2 * i + 1]}, bf16x2));
    reinterpret_cast<uint4 *>(X)[k] = packed;
}

// Inference, step 2: the network over the batch's pairs, reading the bf16
// inputs and writing S0 max(e^y - 1e-4, 0) into H for every pair (step 3
// then overwrites the near field's pairs with their exact values).
struct PairSource {
    const uint16_t *X;
    float *H;
    int j0, n_q, n_qpad;
    float s0, inv_nq;   // inv_nq = 1 / n_q: pair -> (row, pixel) without an integer division
    __device__ uint2 inputs(int64_t p, int gi) const { return *reinterpret_cast<const uint2 *>(X + p * 8 + 4 * gi); }
    // a wave's first pair as the start of its row of H and its pixel; the
    // wave's 32 pairs then step along the row and on into the next rows
    struct Out {
        int64_t row;
        int q;
    };
    __device__ Out out_base(int64_t p0) const {
        const int k = (int)p0;   // < 2^23 pairs per batch: exact in FP32, and the quotient is off by at most one
        int lr = (int)((float)k * inv_nq);
        lr += (lr + 1) * n_q <= k ? 1 : 0;
        lr -= lr * n_q > k ? 1 : 0;
        return Out{(int64_t)(j0 + lr) * n_qpad, k - lr * n_q};
    }
    __device__ void output(const Out &o, int i, float y) const {
        int64_t row = o.row;
        int q = o.q + i;
        while (q >= n_q) {   // once at most when n_q >= 32
            q -= n_q;
            row += n_qpad;
        }
        H[row + q] = s0 * fmaxf(__expf(y) - kTargetFloor, 0.0f);
    }
};

// Inference, step 3: the near field, exact.  The emission pixels within the
// event's own position response (|u - u_q| < 3 sig_u) are exactly the
// emission pixels among the path ends it reaches (its rank range), so one
// block per event row walks that range: the event's position response at
// every reached path end is staged in LDS first (one exp and an FP64 offset
// per path end instead of per term), then each group of 16 lanes takes one
// such pixel q, its lanes share the scatter terms of the reached ends (all
// inside q's band, stored contiguously per q, so the group's loads are
// contiguous), and the group's first lane adds the primary term and writes
// H over the network's value.  Ranges longer than the staging buffer fall
// back to evaluating the response per term.
constexpr int kNearStage = 2048;

__global__ __launch_bounds__(256) void k_surr_near(Geo g, SurrTables st, const float2 *__restrict__ band, int band_w,
                                                   const int *__restrict__ band_lo, const int *__restrict__ ev_angle,
                                                   const float *__restrict__ su, const float *__restrict__ se,
                                                   const float *__restrict__ efac, const int2 *__restrict__ rr,
                                                   int row_base, int j0, int rows, float *__restrict__ H) {
    __shared__ float Kr[kNearStage];
    const int lr = blockIdx.x;   // row within the batch
    if (lr >= rows) return;
    const int jr = j0 + lr, j = row_base + jr;
    const int a = ev_angle[j];
    const double u = ((double)su[j] - 0.5 * g.n_bins) * g.bin_cm;
    const float et = se[j];
    const int2 r = rr[jr];
    const double *us = st.us_sorted + (size_t)a * g.n_p;
    const int *ss = st.s_sorted + (size_t)a * g.n_p;
    const float inv2s2 = (float)(1.0 / (2.0 * g.sig_u * g.sig_u));
    const bool staged = r.y - r.x <= kNearStage;
    if (staged)
        for (int i = threadIdx.x; i < r.y - r.x; i += blockDim.x) Kr[i] = k_resp_f((float)(u - us[r.x + i]), inv2s2);
    __syncthreads();
    const int grp = threadIdx.x >> 4, l = threadIdx.x & 15;
    // every group runs the same number of passes, so the 16-lane sums below
    // always see all of their lanes
    for (int rank0 = r.x; rank0 < r.y; rank0 += 16) {
        const int rank = rank0 + grp;
        const int q = rank < r.y ? ss[rank] : g.n_q;
        float h = 0.0f;
        if (q < g.n_q) {
            const int lo = band_lo[(size_t)a * g.n_p + q];
            const float2 *bq = band + ((size_t)a * g.n_qpad + q) * band_w;
            const int b0 = max(r.x - lo, 0), b1 = min(r.y - lo, band_w);
            if (staged) {
                const float *kq = Kr + (lo - r.x);
#pragma unroll 4
                for (int b = b0 + l; b < b1; b += 16) {
                    const float2 ab = bq[b];
                    h = fmaf(kq[b], __builtin_amdgcn_exp2f(fmaf(ab.y, et, ab.x)), h);
                }
            } else {
                for (int b = b0 + l; b < b1; b += 16) {
                    const float2 ab = bq[b];
                    h = fmaf(k_resp_f((float)(u - us[lo + b]), inv2s2), __builtin_amdgcn_exp2f(fmaf(ab.y, et, ab.x)),
                             h);
                }
            }
        }
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) h += __shfl_xor(h, off, 64);
        if (l == 0 && q < g.n_q) {
            const float beta0 = (float)(2.0 * g.c2 * (g.e0 - g.e_c));
            const float kp = staged ? Kr[rank - r.x] : k_resp_f((float)(u - us[rank]), inv2s2);
            h += kp * __builtin_amdgcn_exp2f(fmaf(beta0, et, st.prim[(size_t)a * g.n_p + q]));
            H[(size_t)jr * g.n_qpad + q] = h * efac[j];
        }
    }
}

// partial means with one pixel group: pmean[j] = sum_q f[real(j)][q] H[j][q]
__global__ void k_row_mean(Geo g, const int *__restrict__ rrange, int n_real, int rows, const float *__restrict__ H,
                           const float *__restrict__ f, float *__restrict__ pmean) {
    const int j = blockIdx.x;
    if (j >= rows) return;
    int lo = 0, hi = n_real;   // realisation r with rrange[r] <= j < rrange[r+1]
    while (hi - lo > 1) { const int m = (lo + hi) >> 1; if (rrange[m] <= j) lo = m; else hi = m; }
    const float *fr = f + (size_t)lo * g.n_qpad;
    float s = 0.0f;
    for (int q = threadIdx.x; q < g.n_q; q += 64) s = fmaf(fr[q], H[(size_t)j * g.n_qpad + q], s);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) pmean[j] = s;
}

// the fused network over a batch of pairs, one workgroup per CU as for
// lmosem_net_forward
static hipError_t launch_mlp_pairs(Net *net, const PairSource &src, int64_t pairs, hipStream_t st) {
    const uint16_t *fw = nullptr;
    const float *fb = nullptr;
    net_fused_weights(net, &fw, &fb);
    const int64_t tiles = (pairs + kFusedTile - 1) / kFusedTile;
    const unsigned grid = (unsigned)std::min<int64_t>(tiles, 256);
    hipLaunchKernelGGL(k_mlp_infer<PairSource>, dim3(grid), dim3(kFusedThreads), 0, st, fw, fb, src, pairs);
    return hipGetLastError();
}

hipError_t surrogate_samples(const Geo &g, const Tables &t, const int32_t *pixel, const int32_t *angle,
                             const float *u_bin, const float *energy, int64_t n, float *X, float *target,
                             float *scatter, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    SurrTables s{t.Ldet, t.Lback, t.prim, t.p_pix, t.mu, t.cs, t.s_sorted, t.us_sorted,
                 t.mu_sorted, 1.0f / (float)g.nx, 1.0f / (float)g.n_q};
    hipLaunchKernelGGL(k_surr_samples, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, g, s, t.p_pix + g.n_p,
                       t.Ld, t.Bt, pixel, angle, u_bin, energy, n, X, target, scatter);
    return hipGetLastError();
}

// System rows of one sub-iteration with the surrogate scatter term:
// H[j][q] = primary(q; A_j) + S_net(q; A_j), and the partial means (one group).
hipError_t surrogate_rows(const Geo &g, const Tables &t, Net *net, const int *ev_angle, const float *su,
                          const float *se, const float *efac, const float *f, const int *rrange, int n_real,
                          int row_base, int rows, float *H, float *pmean, float *col, uint16_t *X,
                          int64_t pair_cap, hipStream_t st, const LaunchWrap *wrap_net) {
    if (rows <= 0) return hipSuccess;
    // the network's output walks a wave's pairs along rows of n_q pixels
    // (contexts never have an empty emission set; this keeps that walk finite)
    if (g.n_q <= 0) return hipErrorInvalidValue;
    SurrTables s{t.Ldet, t.Lback, t.prim, t.p_pix, t.mu, t.cs, t.s_sorted, t.us_sorted,
                 t.mu_sorted, 1.0f / (float)g.nx, 1.0f / (float)g.n_q};
    float4 *col4 = reinterpret_cast<float4 *>(col);
    int2 *rr = reinterpret_cast<int2 *>(col4 + rows);   // the workspace holds 6 words per event
    hipError_t e;
    hipLaunchKernelGGL(k_event_column, dim3((rows + 63) / 64), dim3(64), 0, st, g, s, ev_angle + row_base,
                       su + row_base, rows, col4, rr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int rows_per = (int)std::max<int64_t>(1, pair_cap / g.n_q);
    for (int j0 = 0; j0 < rows; j0 += rows_per) {
        const int nr = std::min(rows_per, rows - j0);
        const int64_t pairs = (int64_t)nr * g.n_q;
        hipLaunchKernelGGL(k_surr_pairs, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, st, g, s, ev_angle, su,
                           se, col4, row_base, j0, nr, X);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const PairSource src{X, H, j0, g.n_q, g.n_qpad, (float)(1.0 / (g.dx * g.sig_e)), 1.0f / (float)g.n_q};
        auto run_net = [&]() { return launch_mlp_pairs(net, src, pairs, st); };
        if ((e = wrap_net ? (*wrap_net)(run_net) : run_net()) != hipSuccess) return e;
    }
    // the near field of every row in one launch, over the network's values
    // (one block per row: a launch per batch of rows left most of the
    // GPU's block slots empty)
    hipLaunchKernelGGL(k_surr_near, dim3((unsigned)rows), dim3(256), 0, st, g, s, t.band, t.band_w, t.band_lo,
                       ev_angle, su, se, efac, rr, row_base, 0, rows, H);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_row_mean, dim3(rows), dim3(64), 0, st, g, rrange, n_real, rows, H, f, pmean);
    return hipGetLastError();
}

}  // namespace lmo
