// Per-event means (lmosem_forward) without any device allocation.
//
// Every buffer of the call -- the estimate on the emission set, the sorted
// events, the tile plan, the event means and, in turn, the sort's keys and
// temporary storage and then the system rows of one chunk of tiles -- is
// carved from one file-scope device array.  The array lives as long as the
// process on every GPU the library runs on; each call overwrites it (the
// counters that must start at zero are cleared), so calls that overlap on
// one GPU race, whatever their contexts.  The forward projection runs as in
// lmosem_forward, chunk by chunk of whole tiles, so each event's mean is the
// same sum in the same order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "lmosem_int.h"

namespace lmo {

namespace {
constexpr size_t kScratchSize = size_t(64) << 20;
constexpr int kMaxDevices = 64;
}  // namespace

const size_t kScratchBytes = kScratchSize;

// The scratch memory itself.  Host code never passes this name to a kernel
// or a copy (it is a host-side stand-in there): it uses the device address
// that scratch_address looks up.
static __device__ __align__(256) unsigned char scratch[kScratchSize];

hipError_t scratch_address(void **ptr) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

namespace {

// Byte offsets of the call's buffers in the scratch array.  The transient
// region holds the sort's keys, indices and temporary storage, and after the
// sort the system rows and partial means of one chunk of tiles.
struct Layout {
    size_t f, counts, offs, ang, u, e, efac, orig, mean, inv, tiles, terms, useful;
    size_t trans, keys, keys2, idx, idx2, tmp, tmp_bytes, sort_end;
    int max_tiles;
    int64_t chunk_rows;   // rows of one chunk that fit after the transient offset
    size_t need;          // bytes the call needs
};

size_t up(size_t x) { return (x + 255) & ~size_t(255); }

hipError_t layout(const Geo &g, int64_t n, int ev_tile, Layout &L) {
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = up(o + bytes); return at; };
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    L.f = take(sizeof(float) * g.n_qpad);
    L.counts = take(sizeof(int) * g.n_angles);
    L.offs = take(sizeof(int64_t) * 2);
    L.ang = take(sizeof(int) * nn);
    L.u = take(sizeof(float) * nn);
    L.e = take(sizeof(float) * nn);
    L.efac = take(sizeof(float) * nn);
    L.orig = take(sizeof(int) * nn);
    L.mean = take(sizeof(float) * nn);
    L.inv = take(sizeof(float) * nn);
    L.max_tiles = (int)std::min<int64_t>((int64_t)(nn + ev_tile - 1) / ev_tile + g.n_angles, 0x7fffffff);
    L.tiles = take(sizeof(Tile) * L.max_tiles);
    L.terms = take(sizeof(long long) * L.max_tiles);
    L.useful = take(sizeof(long long) * L.max_tiles);
    L.trans = o;
    L.keys = take(sizeof(uint64_t) * nn);
    L.keys2 = take(sizeof(uint64_t) * nn);
    L.idx = take(sizeof(int) * nn);
    L.idx2 = take(sizeof(int) * nn);
    hipError_t e = sort_pairs_bytes(n, g.n_angles, L.tmp_bytes);
    if (e != hipSuccess) return e;
    L.tmp = take(std::max<size_t>(L.tmp_bytes, 1));
    L.sort_end = o;
    // a chunk: rows x n_qpad system-row floats, then the partial means of its
    // pixel groups (groups x rows floats)
    const size_t per_row = sizeof(float) * ((size_t)g.n_qpad + (size_t)forward_groups(g));
    const size_t room = kScratchSize > L.trans + 256 ? kScratchSize - L.trans - 256 : 0;
    L.chunk_rows = (int64_t)(room / per_row);
    L.need = std::max(L.sort_end, L.trans + 256 + per_row * (size_t)ev_tile);
    return hipSuccess;
}

}  // namespace

hipError_t forward_noalloc_bytes(const Geo &g, int64_t n, int ev_tile, size_t &need) {
    Layout L;
    hipError_t e = layout(g, n, ev_tile, L);
    need = L.need;
    return e;
}

hipError_t forward_noalloc(const Geo &g, const Tables &t, const lmosem_events &ev, int ev_tile, const float *image,
                           float *mean_out, unsigned long long *skipped, hipStream_t st, int64_t &terms,
                           int64_t &useful) {
    terms = useful = 0;
    void *base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return e;
    Layout L;
    if ((e = layout(g, ev.n, ev_tile, L)) != hipSuccess) return e;
    if (L.need > kScratchSize || L.chunk_rows < ev_tile) return hipErrorInvalidValue;   // rejected by the caller
    char *b = static_cast<char *>(base);
    float *f = reinterpret_cast<float *>(b + L.f);
    int *counts = reinterpret_cast<int *>(b + L.counts);
    int64_t *offs = reinterpret_cast<int64_t *>(b + L.offs);
    int *ang = reinterpret_cast<int *>(b + L.ang), *orig = reinterpret_cast<int *>(b + L.orig);
    float *u = reinterpret_cast<float *>(b + L.u), *en = reinterpret_cast<float *>(b + L.e);
    float *efac = reinterpret_cast<float *>(b + L.efac);
    float *mean = reinterpret_cast<float *>(b + L.mean), *inv = reinterpret_cast<float *>(b + L.inv);
    Tile *tiles = reinterpret_cast<Tile *>(b + L.tiles);
    long long *terms_d = reinterpret_cast<long long *>(b + L.terms), *useful_d = reinterpret_cast<long long *>(b + L.useful);
    uint64_t *keys = reinterpret_cast<uint64_t *>(b + L.keys), *keys2 = reinterpret_cast<uint64_t *>(b + L.keys2);
    int *idx = reinterpret_cast<int *>(b + L.idx), *idx2 = reinterpret_cast<int *>(b + L.idx2);
    void *tmp = b + L.tmp;
    const int n = (int)ev.n;

    if ((e = launch_gather_image(g, t, image, 1, 0, f, 0, st)) != hipSuccess) return e;
    if (n == 0) return hipStreamSynchronize(st);
    // order the events by (angle, position), as lmosem_forward's ingest does
    // with every event in subset 0 and one realisation
    const int64_t offs_h[2] = {0, (int64_t)n};
    // the per-angle counters start at zero (a fill kernel: all-zero bits)
    if ((e = launch_fill(reinterpret_cast<float *>(counts), (size_t)g.n_angles, 0.0f, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(offs, offs_h, sizeof offs_h, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    if ((e = launch_event_keys(g, n, 1, offs, ev.angle, ev.u_bin, 0, keys, idx, st)) != hipSuccess) return e;
    if ((e = sort_pairs(tmp, L.tmp_bytes, keys, keys2, idx, idx2, n, g.n_angles, st)) != hipSuccess) return e;
    if ((e = launch_gather_events(g, n, keys2, idx2, ev, ang, u, en, efac, orig, counts, st)) != hipSuccess) return e;
    std::vector<int> cnt(g.n_angles);
    if ((e = hipMemcpyAsync(cnt.data(), counts, sizeof(int) * g.n_angles, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    std::vector<Tile> th;
    host_tiles(g, cnt, g.n_angles, ev_tile, th);
    const int nt = (int)th.size();
    if (nt > L.max_tiles) return hipErrorInvalidValue;
    if ((e = hipMemcpyAsync(tiles, th.data(), sizeof(Tile) * nt, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    if ((e = launch_tile_ranks(g, tiles, nt, t.us_sorted, u, terms_d, useful_d, st)) != hipSuccess) return e;
    // the forward projection chunk by chunk of whole tiles, in the transient
    // region (the sort's buffers are dead by now in stream order)
    float *H = reinterpret_cast<float *>(b + L.trans);
    const int64_t rows_max = L.chunk_rows;
    float *pmean = reinterpret_cast<float *>(b + L.trans + up(sizeof(float) * (size_t)rows_max * g.n_qpad));
    const int groups = forward_groups(g);
    for (int t0 = 0; t0 < nt;) {
        const int row_base = th[t0].e0;
        int rows = 0, t1 = t0;
        while (t1 < nt && rows + th[t1].n <= rows_max) rows += th[t1++].n;
        if ((e = launch_forward(ev_tile, g, t, tiles + t0, t1 - t0, u, en, efac, f, H, pmean, row_base, rows, st)) !=
            hipSuccess)
            return e;
        if ((e = launch_mean(pmean, groups, rows, mean + row_base, inv + row_base, skipped, st)) != hipSuccess) return e;
        t0 = t1;
    }
    if ((e = launch_scatter_rows(mean, orig, n, mean_out, st)) != hipSuccess) return e;
    std::vector<long long> tv(nt), uv(nt);
    if ((e = hipMemcpyAsync(tv.data(), terms_d, sizeof(long long) * nt, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(uv.data(), useful_d, sizeof(long long) * nt, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return e;
    for (int k = 0; k < nt; ++k) { terms += tv[k]; useful += uv[k]; }
    return hipSuccess;
}

}  // namespace lmo
