// Event ingest: validation, ordering and tile planning.
//
// Events are ordered by (subset, realisation, angle, detector position):
// subsets are visited in order by the OS iteration (Sec. 2.2, subsets by
// detector angle), all realisations of one subset run in the same launches,
// and within one angle neighbouring positions share the path ends their
// position responses reach, so a tile of consecutive events reads one
// contiguous slice of the path table.
#include <hip/hip_runtime.h>
#include <hipcub/device/device_radix_sort.hpp>
#include <math.h>

#include <algorithm>
#include <cstdio>

#include "lmosem_int.h"

namespace lmo {

__global__ void k_validate(Geo g, int64_t n, const int32_t *__restrict__ angle,
                           const float *__restrict__ u_bin, const float *__restrict__ energy,
                           int *__restrict__ bad) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int local = 0;
    if (j < n) {
        int a = angle[j];
        float u = u_bin[j], e = energy[j];
        bool ok = a >= 0 && a < g.n_angles && u >= 0.0f && u < (float)g.n_bins &&
                  (double)e >= g.win_lo && (double)e <= g.win_hi;
        local = ok ? 0 : 1;
    }
    // one atomic per wave
    unsigned long long m = __ballot(local);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(bad, (int)__popcll(m));
}

hipError_t validate_events(const Geo &g, const lmosem_events &ev, int64_t *bad_host, int *bad_dev,
                           hipStream_t st) {
    hipError_t e = hipMemsetAsync(bad_dev, 0, sizeof(int), st);
    if (e != hipSuccess) return e;
    if (ev.n > 0) {
        hipLaunchKernelGGL(k_validate, dim3((unsigned)((ev.n + 255) / 256)), dim3(256), 0, st, g, ev.n,
                           ev.angle, ev.u_bin, ev.energy_kev, bad_dev);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    int h = 0;
    if ((e = hipMemcpyAsync(&h, bad_dev, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    *bad_host = h;
    return hipSuccess;
}

// key = (group << 32) | position bits; group = (subset * R + realisation) * N_A + angle
__global__ void k_keys(Geo g, int64_t n, int n_real, const int64_t *__restrict__ offs,
                       const int32_t *__restrict__ angle, const float *__restrict__ u_bin,
                       int force_subset, uint64_t *__restrict__ keys, int *__restrict__ idx) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int lo = 0, hi = n_real;           // realisation r with offs[r] <= j < offs[r+1]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (offs[mid] <= j) lo = mid; else hi = mid;
    }
    int a = angle[j];
    int sub = force_subset >= 0 ? force_subset : a % g.n_subsets;
    uint64_t grp = ((uint64_t)sub * n_real + lo) * g.n_angles + a;
    float u = u_bin[j];
    uint32_t bits = u > 0.0f ? __float_as_uint(u) : 0u;   // positions are >= 0: bits sort like values
    keys[j] = (grp << 32) | bits;
    idx[j] = (int)j;
}

__global__ void k_gather_events(Geo g, int64_t n, const uint64_t *__restrict__ keys,
                                const int *__restrict__ idx, const float *__restrict__ u_bin,
                                const float *__restrict__ energy, const int32_t *__restrict__ angle,
                                int *__restrict__ sa, float *__restrict__ su,
                                float *__restrict__ se, float *__restrict__ efac, int *__restrict__ orig,
                                int *__restrict__ counts) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int j = idx[k];
    sa[k] = angle[j];
    su[k] = u_bin[j];
    const double x = (double)energy[j] - g.e_c;
    se[k] = (float)x;
    efac[k] = (float)(exp2(-g.c2 * x * x) / g.zk);
    orig[k] = j;
    atomicAdd(&counts[keys[k] >> 32], 1);
}

// Rank ranges of the tiles, and per tile the number of terms the forward
// kernel evaluates and the number with a non-zero position response.
__global__ void k_tile_ranks(Geo g, Tile *__restrict__ tiles, int n_tiles,
                             const double *__restrict__ us_sorted, const float *__restrict__ su,
                             long long *__restrict__ terms, long long *__restrict__ useful) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    Tile tl = tiles[t];
    const double *us = us_sorted + (size_t)tl.angle * g.n_p;
    const double reach = 3.0 * g.sig_u;
    auto first_above = [&](double v) {      // first rank with us > v
        int lo = 0, hi = g.n_p;
        while (lo < hi) { int m = (lo + hi) >> 1; if (us[m] > v) hi = m; else lo = m + 1; }
        return lo;
    };
    auto first_at_least = [&](double v) {   // first rank with us >= v
        int lo = 0, hi = g.n_p;
        while (lo < hi) { int m = (lo + hi) >> 1; if (us[m] >= v) hi = m; else lo = m + 1; }
        return lo;
    };
    double u_first = ((double)su[tl.e0] - 0.5 * g.n_bins) * g.bin_cm;
    double u_last = ((double)su[tl.e0 + tl.n - 1] - 0.5 * g.n_bins) * g.bin_cm;
    tl.r0 = first_above(u_first - reach);
    tl.r1 = max(tl.r0, first_at_least(u_last + reach));
    tiles[t] = tl;
    long long use = 0;
    for (int e = 0; e < tl.n; ++e) {
        double u = ((double)su[tl.e0 + e] - 0.5 * g.n_bins) * g.bin_cm;
        use += first_at_least(u + reach) - first_above(u - reach);
    }
    terms[t] = (long long)(tl.r1 - tl.r0) * tl.n * g.n_q;
    useful[t] = use * g.n_q;
}

hipError_t launch_event_keys(const Geo &g, int64_t n, int n_real, const int64_t *offs_dev, const int32_t *angle,
                             const float *u_bin, int force_subset, uint64_t *keys, int *idx, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, n, n_real, offs_dev, angle,
                       u_bin, force_subset, keys, idx);
    return hipGetLastError();
}

hipError_t launch_gather_events(const Geo &g, int64_t n, const uint64_t *keys, const int *idx, const lmosem_events &ev,
                                int *sa, float *su, float *se, float *efac, int *orig, int *counts, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_events, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, n, keys, idx,
                       ev.u_bin, ev.energy_kev, ev.angle, sa, su, se, efac, orig, counts);
    return hipGetLastError();
}

hipError_t launch_tile_ranks(const Geo &g, Tile *tiles, int n_tiles, const double *us_sorted, const float *su,
                             long long *terms, long long *useful, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_ranks, dim3((unsigned)((n_tiles + 127) / 128)), dim3(128), 0, st, g, tiles, n_tiles,
                       us_sorted, su, terms, useful);
    return hipGetLastError();
}

int sort_key_bits(int n_groups) {
    int hi_bits = 1;
    while ((1ll << hi_bits) < (long long)n_groups) ++hi_bits;
    return 32 + hi_bits;
}

hipError_t sort_pairs_bytes(int64_t n, int n_groups, size_t &bytes) {
    bytes = 0;
    if (n <= 0) return hipSuccess;
    return hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                              (const int *)nullptr, (int *)nullptr, (int)n, 0,
                                              sort_key_bits(n_groups), (hipStream_t)nullptr);
}

hipError_t sort_pairs(void *tmp, size_t tmp_bytes, const uint64_t *keys, uint64_t *keys2, const int *idx, int *idx2,
                      int64_t n, int n_groups, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    return hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, keys2, idx, idx2, (int)n, 0,
                                              sort_key_bits(n_groups), st);
}

void host_tiles(const Geo &g, const std::vector<int> &counts, int n_angles_used, int ev_tile, std::vector<Tile> &tiles) {
    tiles.clear();
    int64_t pos = 0;
    for (int a = 0; a < n_angles_used; ++a) {
        const int c = counts[a];
        for (int k = 0; k < c; k += ev_tile) tiles.push_back(Tile{(int)(pos + k), std::min(ev_tile, c - k), a, 0, 0, 0});
        pos += c;
    }
}

hipError_t sort_events(const Geo &g, const Tables &tb, const lmosem_events &ev,
                       const std::vector<int64_t> &offs, int force_subset, EvSet &set,
                       hipStream_t st, std::string &err) {
    hipError_t e = hipSuccess;
    const int64_t n = ev.n;
    const int n_real = (int)offs.size() - 1;
    const int n_groups = g.n_subsets * n_real * g.n_angles;
    uint64_t *keys = nullptr, *keys2 = nullptr;
    int *idx = nullptr, *idx2 = nullptr, *counts = nullptr;
    int64_t *offs_d = nullptr;
    void *tmp = nullptr;
    auto cleanup = [&]() {
        hipFree(keys); hipFree(keys2); hipFree(idx); hipFree(idx2); hipFree(counts);
        hipFree(offs_d); hipFree(tmp);
    };
#define CK(call, what) do { e = (call); if (e != hipSuccess) { err = std::string(what) + ": " + hipGetErrorString(e); cleanup(); return e; } } while (0)
    set.n = n;
    set.n_real = n_real;
    size_t nn = (size_t)std::max<int64_t>(n, 1);
    CK(hipMalloc(&set.ang, sizeof(int) * nn), "alloc events");
    CK(hipMalloc(&set.u, sizeof(float) * nn), "alloc events");
    CK(hipMalloc(&set.e, sizeof(float) * nn), "alloc events");
    CK(hipMalloc(&set.orig, sizeof(int) * nn), "alloc events");
    CK(hipMalloc(&set.efac, sizeof(float) * nn), "alloc events");
    CK(hipMalloc(&counts, sizeof(int) * std::max(n_groups, 1)), "alloc counts");
    CK(hipMemsetAsync(counts, 0, sizeof(int) * std::max(n_groups, 1), st), "clear counts");
    if (n > 0) {
        CK(hipMalloc(&keys, sizeof(uint64_t) * n), "alloc keys");
        CK(hipMalloc(&keys2, sizeof(uint64_t) * n), "alloc keys");
        CK(hipMalloc(&idx, sizeof(int) * n), "alloc idx");
        CK(hipMalloc(&idx2, sizeof(int) * n), "alloc idx");
        CK(hipMalloc(&offs_d, sizeof(int64_t) * offs.size()), "alloc offsets");
        CK(hipMemcpyAsync(offs_d, offs.data(), sizeof(int64_t) * offs.size(), hipMemcpyHostToDevice, st),
           "upload offsets");
        unsigned blocks = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(k_keys, dim3(blocks), dim3(256), 0, st, g, n, n_real, offs_d, ev.angle,
                           ev.u_bin, force_subset, keys, idx);
        CK(hipGetLastError(), "keys");
        int hi_bits = 1;
        while ((1ll << hi_bits) < (long long)n_groups) ++hi_bits;
        size_t tmp_bytes = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys, keys2, idx, idx2, (int)n, 0,
                                              32 + hi_bits, st), "sort size");
        CK(hipMalloc(&tmp, tmp_bytes), "alloc sort");
        CK(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, keys2, idx, idx2, (int)n, 0,
                                              32 + hi_bits, st), "sort");
        hipLaunchKernelGGL(k_gather_events, dim3(blocks), dim3(256), 0, st, g, n, keys2, idx2, ev.u_bin,
                           ev.energy_kev, ev.angle, set.ang, set.u, set.e, set.efac, set.orig, counts);
        CK(hipGetLastError(), "gather events");
    }
    set.counts.assign(std::max(n_groups, 1), 0);
    CK(hipMemcpyAsync(set.counts.data(), counts, sizeof(int) * std::max(n_groups, 1), hipMemcpyDeviceToHost, st),
       "download counts");
    CK(hipStreamSynchronize(st), "ingest");
    cleanup();
#undef CK
    return plan_tiles(g, tb, set, set.ev_tile, set.chunk_rows, st, err);
}

// Tiles of ev_tile consecutive events per (subset, realisation, angle) group
// and backprojection chunks of chunk_rows rows per (subset, realisation), from
// the group counts of the sorted set; replaces any earlier plan.
hipError_t plan_tiles(const Geo &g, const Tables &tb, EvSet &set, int ev_tile, int chunk_rows,
                      hipStream_t st, std::string &err) {
    hipError_t e = hipSuccess;
    long long *terms_d = nullptr, *useful_d = nullptr;
    auto cleanup = [&]() { hipFree(terms_d); hipFree(useful_d); };
#define CK(call, what) do { e = (call); if (e != hipSuccess) { err = std::string(what) + ": " + hipGetErrorString(e); cleanup(); return e; } } while (0)
    hipFree(set.tiles); hipFree(set.chunks); hipFree(set.crange); hipFree(set.rrange);
    set.tiles = nullptr; set.chunks = nullptr; set.crange = nullptr; set.rrange = nullptr;
    set.ev_tile = ev_tile;
    set.chunk_rows = chunk_rows;
    const int n_real = set.n_real;
    const std::vector<int> &cnt = set.counts;
    const int EV = ev_tile, CH = chunk_rows;
    std::vector<Tile> tiles;
    std::vector<Chunk> chunks;
    std::vector<int> crange, rrange;
    set.row_off.assign(g.n_subsets + 1, 0);
    set.tile_off.assign(g.n_subsets + 1, 0);
    set.chunk_off.assign(g.n_subsets + 1, 0);
    set.max_rows = 0;
    set.max_chunks = 0;
    int64_t pos = 0;
    for (int i = 0; i < g.n_subsets; ++i) {
        set.row_off[i] = (int)pos;
        set.tile_off[i] = (int)tiles.size();
        set.chunk_off[i] = (int)chunks.size();
        for (int r = 0; r < n_real; ++r) {
            crange.push_back((int)chunks.size() - set.chunk_off[i]);
            rrange.push_back((int)(pos - set.row_off[i]));
            int64_t real_start = pos;
            for (int a = 0; a < g.n_angles; ++a) {
                int c = cnt[((size_t)i * n_real + r) * g.n_angles + a];
                for (int k = 0; k < c; k += EV)
                    tiles.push_back(Tile{(int)(pos + k), std::min(EV, c - k), a, r, 0, 0});
                pos += c;
            }
            for (int64_t j = real_start; j < pos; j += CH)
                chunks.push_back(Chunk{(int)(j - set.row_off[i]),
                                       (int)(std::min<int64_t>(pos, j + CH) - set.row_off[i]), r, 0});
        }
        crange.push_back((int)chunks.size() - set.chunk_off[i]);
        rrange.push_back((int)(pos - set.row_off[i]));
        set.max_rows = std::max(set.max_rows, (int)(pos - set.row_off[i]));
        set.max_chunks = std::max(set.max_chunks, (int)chunks.size() - set.chunk_off[i]);
    }
    set.row_off[g.n_subsets] = (int)pos;
    set.tile_off[g.n_subsets] = (int)tiles.size();
    set.chunk_off[g.n_subsets] = (int)chunks.size();
    size_t nt = std::max<size_t>(tiles.size(), 1), nc = std::max<size_t>(chunks.size(), 1);
    CK(hipMalloc(&set.tiles, sizeof(Tile) * nt), "alloc tiles");
    CK(hipMalloc(&set.chunks, sizeof(Chunk) * nc), "alloc chunks");
    CK(hipMalloc(&set.crange, sizeof(int) * crange.size()), "alloc ranges");
    CK(hipMalloc(&set.rrange, sizeof(int) * rrange.size()), "alloc ranges");
    CK(hipMalloc(&terms_d, sizeof(long long) * nt), "alloc counters");
    CK(hipMalloc(&useful_d, sizeof(long long) * nt), "alloc counters");
    if (!tiles.empty())
        CK(hipMemcpyAsync(set.tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, st),
           "upload tiles");
    if (!chunks.empty())
        CK(hipMemcpyAsync(set.chunks, chunks.data(), sizeof(Chunk) * chunks.size(), hipMemcpyHostToDevice,
                          st), "upload chunks");
    CK(hipMemcpyAsync(set.crange, crange.data(), sizeof(int) * crange.size(), hipMemcpyHostToDevice, st),
       "upload ranges");
    CK(hipMemcpyAsync(set.rrange, rrange.data(), sizeof(int) * rrange.size(), hipMemcpyHostToDevice, st),
       "upload ranges");
    std::vector<long long> terms(nt, 0), useful(nt, 0);
    if (!tiles.empty()) {
        hipLaunchKernelGGL(k_tile_ranks, dim3((unsigned)((tiles.size() + 127) / 128)), dim3(128), 0, st, g,
                           set.tiles, (int)tiles.size(), tb.us_sorted, set.u, terms_d, useful_d);
        CK(hipGetLastError(), "tile ranks");
        CK(hipMemcpyAsync(terms.data(), terms_d, sizeof(long long) * tiles.size(), hipMemcpyDeviceToHost, st),
           "download counters");
        CK(hipMemcpyAsync(useful.data(), useful_d, sizeof(long long) * tiles.size(), hipMemcpyDeviceToHost,
                          st), "download counters");
    }
    CK(hipStreamSynchronize(st), "tile plan");
    set.terms_sub.assign(g.n_subsets, 0);
    set.useful_sub.assign(g.n_subsets, 0);
    for (int i = 0; i < g.n_subsets; ++i)
        for (int t = set.tile_off[i]; t < set.tile_off[i + 1]; ++t) {
            set.terms_sub[i] += terms[t];
            set.useful_sub[i] += useful[t];
        }
    cleanup();
#undef CK
    return hipSuccess;
}

}  // namespace lmo
