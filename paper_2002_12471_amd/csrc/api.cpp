// Host runtime and C ABI of the gfx950 list-mode OSEM library (include/lmosem.h).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lmosem_int.h"

using namespace lmo;

struct lmosem_ctx {
    lmosem_config cfg{};
    Geo g{};
    Tables t{};
    hipStream_t st = nullptr;
    std::string err;
    bool poisoned = false;
    int ev_tile = 8;
    int pixel_waves = 0;          // pixel tile of sets loaded from now on (waves of 64); 0: g.fwd_waves
    int *bad_dev = nullptr;
    unsigned long long *skipped_dev = nullptr;
    bool surrogate = false;        // scatter_model 2: network scatter term
    lmo::Net *net = nullptr;       // attached network (not owned)
    int64_t terms = 0, useful = 0;
    double table_ms = 0.0;
    int64_t table_bytes = 0;
    // the path table (or near-field band), sensitivities and primary weights
    // are built at the first call that needs them (binned work does not)
    bool paths_ready = false;
    // HIP graphs: one captured iteration per prepared set, replayed on an
    // internal stream ordered after the caller's stream by events
    bool graphs = true;
    hipStream_t gst = nullptr;
    hipEvent_t g_in = nullptr, g_out = nullptr;
    // per-kernel timing (HIP events around each launch while enabled)
    bool timing = false;
    struct Pending { hipEvent_t a, b; int kind; };
    std::vector<Pending> pending;
    int64_t launches[4] = {0, 0, 0, 0};
    double ms[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t net_pairs = 0;     // pairs of the timed network launches
    // device memory: the cap (0 = none) on what the context holds, and the
    // bytes held by its live event sets
    int64_t mem_cap = 0;
    int64_t set_bytes = 0;
    bool inject_failure = false;   // the next launch reports a HIP failure (testing hook)
};

// Workspace of one prepared event set.
struct lmosem_evset {
    EvSet s;
    float *H = nullptr;       // [max_rows][n_qpad]
    float *pmean = nullptr;   // [n_groups][max_rows]
    float *mean = nullptr;    // [max_rows]
    float *inv = nullptr;     // [max_rows]
    float *pb = nullptr;      // [max_chunks][n_qpad]
    float *f = nullptr;       // [n_real][n_qpad]
    double *ll = nullptr;     // [n_real]
    // one iteration captured as a graph: [with log-likelihood + 2 * from cached rows]
    hipGraphExec_t exec[4] = {nullptr, nullptr, nullptr, nullptr};
    float *Hc = nullptr;      // cached system rows [n][n_qpad] (lmosem_cache_rows), zero padded
    bool rows_valid = false;  // Hc holds every row
    int use_graph = -1;       // autotuned choice (1 replay graphs, 0 launch directly), -1 = context setting
    float *col = nullptr;     // surrogate: per-sub-iteration event column features [max_rows][4] + ranks [max_rows][2]
    uint16_t *X = nullptr;    // surrogate: network inputs [pair_cap][8], bf16
    size_t pb_chunks = 0;     // chunk rows allocated in pb
    size_t pmean_groups = 0;  // pixel groups allocated in pmean
    int64_t bytes = 0;        // device bytes held by the set (counted in its context's set_bytes)
};

namespace {

// The context's geometry with the set's forward pixel tile (waves of 64
// pixels per workgroup), which the autotuner may choose per set.
Geo set_geo(const lmosem_ctx *c, const lmosem_evset *s) {
    Geo g = c->g;
    if (s && s->s.fwd_waves > 0) g.fwd_waves = s->s.fwd_waves;
    return g;
}

constexpr int64_t kPairCap = 1 << 23;   // (event, pixel) pairs per surrogate network batch (128 MB of inputs)

lmosem_status set_err(lmosem_ctx *c, lmosem_status s, const std::string &msg) {
    if (c) {
        c->err = msg;
        if (s == LMOSEM_EDEVICE) c->poisoned = true;
    }
    return s;
}

lmosem_status dev_err(lmosem_ctx *c, const char *what, hipError_t e) {
    return set_err(c, LMOSEM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

lmosem_status alloc_err(lmosem_ctx *c, const char *what, hipError_t e) {
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return set_err(c, LMOSEM_ENOMEM, std::string(what) + ": out of device memory");
    }
    return dev_err(c, what, e);
}

// Closed form of the circle mean of the Klein-Nishina shape
// Psi(c) = t^-3 + t^-1 - (1 - c^2) t^-2, t = 1 + k (1 - c), c = cos(phi):
// with a = 1 + k, b = k, r = sqrt(a^2 - b^2),
//   int t^-1 = 2 pi / r,  int t^-3 = pi (2 a^2 + b^2) / r^5,
//   int sin^2 t^-2 = (a int t^-1 - 2 pi) / b^2.
double psi_bar_closed(double k) {
    double a = 1.0 + k, b = k, r = sqrt(a * a - b * b);
    double j1 = 2.0 * M_PI / r;
    double j3 = M_PI * (2.0 * a * a + b * b) / pow(r, 5.0);
    double s2 = (a * j1 - 2.0 * M_PI) / (b * b);
    return (j3 + j1 - s2) / (2.0 * M_PI);
}

double kn_total_host(double e) {
    double k = e / kMeC2;
    double l = log1p(2.0 * k);
    double k1 = 1.0 + k, k2 = 1.0 + 2.0 * k;
    return 2.0 * M_PI * (k1 / (k * k) * (2.0 * k1 / k2 - l / k) + l / (2.0 * k) - (1.0 + 3.0 * k) / (k2 * k2));
}

bool check_cfg(const lmosem_config *c, std::string &why) {
    if (c->abi_version != LMOSEM_ABI_VERSION) { why = "abi_version mismatch"; return false; }
    if (c->nx <= 0 || c->ny <= 0 || c->nx > 4096 || c->ny > 4096) { why = "bad grid size"; return false; }
    if (!(c->pixel_cm > 0) || !(c->bin_cm > 0)) { why = "pixel_cm and bin_cm must be > 0"; return false; }
    if (c->n_bins <= 0 || c->n_angles <= 0 || c->n_angles > 65535) { why = "bad detector size"; return false; }
    if (!(c->e0_kev > 0) || !(c->fwhm_e_kev > 0) || !(c->fwhm_u_cm > 0)) {
        why = "e0_kev and the FWHMs must be > 0";
        return false;
    }
    if (!(c->win_lo_kev < c->win_hi_kev) || !(c->win_lo_kev > 0)) { why = "need 0 < win_lo < win_hi"; return false; }
    if (c->n_subsets < 1 || c->n_subsets > c->n_angles) { why = "need 1 <= n_subsets <= n_angles"; return false; }
    if (c->scatter_model < 0 || c->scatter_model > 2) {
        why = "scatter_model must be 0 (primary), 1 (first-order scatter) or 2 (learned scatter)";
        return false;
    }
    if (!(c->acq_time > 0)) { why = "acq_time must be > 0"; return false; }
    return true;
}

bool check_events(lmosem_ctx *c, const lmosem_events *ev, lmosem_status &st) {
    if (!ev || ev->n < 0 || ev->n > 0x7fffffffLL ||
        (ev->n > 0 && (!ev->angle || !ev->u_bin || !ev->energy_kev))) {
        st = set_err(c, LMOSEM_EINVAL, "bad event arrays");
        return false;
    }
    int64_t bad = 0;
    hipError_t e = validate_events(c->g, *ev, &bad, c->bad_dev, c->st);
    if (e != hipSuccess) { st = dev_err(c, "validate events", e); return false; }
    if (bad) {
        st = set_err(c, LMOSEM_ERANGE, std::to_string(bad) + " events outside angle/position/energy range");
        return false;
    }
    return true;
}

void drop_graphs(lmosem_evset *s) {
    for (auto &x : s->exec)
        if (x) { hipGraphExecDestroy(x); x = nullptr; }
}

void free_set(lmosem_evset *s) {
    if (!s) return;
    if (s->s.ctx) s->s.ctx->set_bytes -= s->bytes;
    drop_graphs(s);
    hipFree(s->s.u); hipFree(s->s.e); hipFree(s->s.efac); hipFree(s->s.orig); hipFree(s->s.tiles); hipFree(s->s.chunks);
    hipFree(s->s.crange); hipFree(s->s.rrange);
    hipFree(s->H); hipFree(s->Hc); hipFree(s->pmean); hipFree(s->mean); hipFree(s->inv); hipFree(s->pb); hipFree(s->f);
    hipFree(s->ll); hipFree(s->col); hipFree(s->X); hipFree(s->s.ang);
    delete s;
}

// Device bytes a set holds with its current plan and workspace.
int64_t set_device_bytes(const lmosem_ctx *c, const lmosem_evset *s) {
    const Geo g = set_geo(c, s);
    const EvSet &v = s->s;
    const int64_t n = std::max<int64_t>(v.n, 1), rows = std::max(v.max_rows, 1);
    const int64_t chunks = std::max<int64_t>((int64_t)s->pb_chunks, 1);
    const int64_t n_tiles = std::max<int64_t>(v.tile_off.empty() ? 1 : v.tile_off.back(), 1);
    const int64_t n_chunks = std::max<int64_t>(v.chunk_off.empty() ? 1 : v.chunk_off.back(), 1);
    int64_t b = 20 * n + (int64_t)sizeof(Tile) * n_tiles + (int64_t)sizeof(Chunk) * n_chunks +
                8 * (int64_t)g.n_subsets * (v.n_real + 1);
    b += 4 * rows * g.n_qpad + 4 * rows * std::max<int64_t>((int64_t)s->pmean_groups, forward_groups(g)) + 8 * rows + 4 * chunks * g.n_qpad +
         4 * (int64_t)v.n_real * g.n_qpad + 8 * (int64_t)v.n_real;
    if (c->surrogate) b += 24 * rows + 8 * 2 * kPairCap;
    if (s->Hc) b += 4 * n * g.n_qpad;
    return b;
}

// (Re)allocate the per-set workspace for the current tile plan.
lmosem_status alloc_workspace(lmosem_ctx *c, lmosem_evset *s) {
    const Geo g = set_geo(c, s);
    size_t rows = std::max(s->s.max_rows, 1), groups = forward_groups(g);
    size_t chunks = std::max(s->s.max_chunks, 1);
    hipError_t e;
#define AL(p, bytes) do { if (!(p)) { e = hipMalloc(&(p), (bytes)); if (e != hipSuccess) return alloc_err(c, "workspace", e); } } while (0)
    AL(s->H, sizeof(float) * rows * g.n_qpad);
    if (s->pmean && s->pmean_groups < groups) { hipFree(s->pmean); s->pmean = nullptr; }
    if (!s->pmean) s->pmean_groups = groups;
    AL(s->pmean, sizeof(float) * rows * groups);
    AL(s->mean, sizeof(float) * rows);
    AL(s->inv, sizeof(float) * rows);
    if (s->pb && s->pb_chunks < chunks) { hipFree(s->pb); s->pb = nullptr; }
    if (!s->pb) s->pb_chunks = chunks;
    AL(s->pb, sizeof(float) * chunks * g.n_qpad);
    AL(s->f, sizeof(float) * (size_t)s->s.n_real * g.n_qpad);
    AL(s->ll, sizeof(double) * s->s.n_real);
    if (c->surrogate) {
        AL(s->col, 6 * sizeof(float) * (size_t)std::max(s->s.max_rows, 1));
        AL(s->X, sizeof(uint16_t) * 8 * (size_t)kPairCap);
    }
#undef AL
    c->set_bytes -= s->bytes;
    s->bytes = set_device_bytes(c, s);
    c->set_bytes += s->bytes;
    return LMOSEM_OK;
}

bool over_cap(const lmosem_ctx *c, int64_t more) {
    return c->mem_cap > 0 && c->table_bytes + c->set_bytes + more > c->mem_cap;
}

std::string cap_msg(const lmosem_ctx *c, const char *what, int64_t more) {
    return std::string(what) + " would take the context to " + std::to_string(c->table_bytes + c->set_bytes + more) +
           " device bytes, above its cap of " + std::to_string(c->mem_cap) + " (lmosem_set_memory_cap)";
}

lmosem_status load_set(lmosem_ctx *c, const lmosem_events *ev, const lmosem_batch *batch, int force_subset,
                       lmosem_evset **out) {
    lmosem_status st = LMOSEM_OK;
    if (c->surrogate && !c->net) return set_err(c, LMOSEM_ESTATE, "scatter_model 2 needs a network (lmosem_set_surrogate)");
    if (!check_events(c, ev, st)) return st;
    std::vector<int64_t> offs;
    if (batch) {
        if (batch->n_real < 1 || !batch->offsets) return set_err(c, LMOSEM_EINVAL, "bad batch");
        offs.assign(batch->offsets, batch->offsets + batch->n_real + 1);
        if (offs[0] != 0 || offs.back() != ev->n) return set_err(c, LMOSEM_EINVAL, "batch offsets must span the events");
        for (int r = 0; r < batch->n_real; ++r)
            if (offs[r + 1] < offs[r]) return set_err(c, LMOSEM_EINVAL, "batch offsets must not decrease");
    } else {
        offs = {0, ev->n};
    }
    auto *s = new lmosem_evset();
    s->s.ctx = c;
    s->s.ev_tile = c->ev_tile;
    s->s.fwd_waves = c->pixel_waves;
    std::string why;
    hipError_t e = sort_events(c->g, c->t, *ev, offs, force_subset, s->s, c->st, why);
    if (e != hipSuccess) {
        free_set(s);
        return e == hipErrorOutOfMemory ? set_err(c, LMOSEM_ENOMEM, why) : set_err(c, LMOSEM_EDEVICE, why);
    }
    lmosem_status ws = alloc_workspace(c, s);
    if (ws != LMOSEM_OK) { free_set(s); return ws; }
    if (over_cap(c, 0)) {
        const std::string msg = cap_msg(c, "the event set", 0);
        free_set(s);
        return set_err(c, LMOSEM_ENOMEM, msg);
    }
    *out = s;
    return LMOSEM_OK;
}

// Run one launch, bracketed by HIP events on the context stream when timing
// is enabled (kind 0 forward, 1 backprojection, 2 mean/update, 3 the network
// of the learned-scatter rows).
template <class F>
hipError_t timed(lmosem_ctx *c, int kind, F &&launch, hipStream_t st) {
    if (c->inject_failure) { c->inject_failure = false; return hipErrorLaunchFailure; }
    if (!c->timing) return launch();
    lmosem_ctx::Pending p{nullptr, nullptr, kind};
    hipError_t e;
    if ((e = hipEventCreate(&p.a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&p.b)) != hipSuccess) { hipEventDestroy(p.a); return e; }
    if ((e = hipEventRecord(p.a, st)) == hipSuccess && (e = launch()) == hipSuccess)
        e = hipEventRecord(p.b, st);
    if (e != hipSuccess) { hipEventDestroy(p.a); hipEventDestroy(p.b); return e; }
    c->pending.push_back(p);
    return hipSuccess;
}

// As timed, for one kernel launched with its own start and end events
// (launch receives them, or null when timing is off): the interval then
// covers the kernel alone, as a profiler's kernel trace does.
template <class F>
hipError_t timed_kernel(lmosem_ctx *c, int kind, F &&launch) {
    if (c->inject_failure) { c->inject_failure = false; return hipErrorLaunchFailure; }
    if (!c->timing) return launch(nullptr);
    lmosem_ctx::Pending p{nullptr, nullptr, kind};
    hipError_t e;
    if ((e = hipEventCreate(&p.a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&p.b)) != hipSuccess) { hipEventDestroy(p.a); return e; }
    const KernelEvents ke{p.a, p.b};
    if ((e = launch(&ke)) != hipSuccess) { hipEventDestroy(p.a); hipEventDestroy(p.b); return e; }
    c->pending.push_back(p);
    return hipSuccess;
}

hipError_t drain_timing(lmosem_ctx *c) {
    hipError_t e = hipSuccess;
    for (auto &p : c->pending) {
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventSynchronize(p.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
        c->ms[p.kind] += ms;
        c->launches[p.kind] += 1;
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    c->pending.clear();
    return e;
}

// System rows and partial means of subset i: exact forward projection, or
// exact primaries plus the network's scatter term.
hipError_t forward_rows(lmosem_ctx *c, lmosem_evset *s, int i, float *H, hipStream_t st) {
    const Geo g = set_geo(c, s);
    const EvSet &v = s->s;
    const int rows = v.row_off[i + 1] - v.row_off[i];
    if (c->surrogate) {
        // with timing on, each network launch is timed on its own (its pair
        // count is rows x emission pixels, split into batches of kPairCap)
        const int64_t rows_per = std::max<int64_t>(1, kPairCap / g.n_q);
        int64_t row0 = 0;
        const LaunchWrap wrap = [&](const std::function<hipError_t()> &launch) {
            c->net_pairs += std::min<int64_t>(rows_per, rows - row0) * g.n_q;
            row0 += rows_per;
            return timed(c, 3, launch, st);
        };
        return surrogate_rows(g, c->t, c->net, v.ang, v.u, v.e, v.efac, s->f, v.rrange + (size_t)i * (v.n_real + 1),
                              v.n_real, v.row_off[i], rows, H, s->pmean, s->col, s->X, kPairCap, st,
                              c->timing ? &wrap : nullptr);
    }
    return timed_kernel(c, 0, [&](const KernelEvents *ke) {
        return launch_forward(v.ev_tile, g, c->t, v.tiles + v.tile_off[i], v.tile_off[i + 1] - v.tile_off[i], v.u,
                              v.e, v.efac, s->f, H, s->pmean, v.row_off[i], rows, st, ke);
    });
}

int mean_groups(const lmosem_ctx *c, const lmosem_evset *s) { return c->surrogate ? 1 : forward_groups(set_geo(c, s)); }

// One sub-iteration of Eq. 7 on all realisations of a prepared set: the
// system rows are computed (and kept when the set caches them) or, once
// cached, read back for the means.
hipError_t subiteration(lmosem_ctx *c, lmosem_evset *s, int i, bool want_ll, hipStream_t st) {
    const Geo &g = c->g;
    const EvSet &v = s->s;
    const int rows = v.row_off[i + 1] - v.row_off[i];
    const int n_tiles = v.tile_off[i + 1] - v.tile_off[i];
    const int n_chunks = v.chunk_off[i + 1] - v.chunk_off[i];
    const bool cached = s->Hc && s->rows_valid;
    const int groups = cached ? 1 : mean_groups(c, s);
    float *H = s->Hc ? s->Hc + (size_t)v.row_off[i] * g.n_qpad : s->H;
    const float *sens = c->t.sens + (size_t)i * g.n_qpad;
    const int *crange = v.crange + (size_t)i * (v.n_real + 1);
    const int *rrange = v.rrange + (size_t)i * (v.n_real + 1);
    hipError_t e;
    if (cached) {
        // event means and their inverses straight from the stored rows
        if ((e = timed_kernel(c, 0, [&](const KernelEvents *ke) {
                 return launch_row_dot(g, rrange, v.n_real, rows, H, s->f, s->mean, s->inv, c->skipped_dev, st, ke);
             })) != hipSuccess)
            return e;
    } else if (c->surrogate && rows > 0) {
        // many kernels per sub-iteration: bracketed as a whole
        if ((e = timed(c, 0, [&] { return forward_rows(c, s, i, H, st); }, st)) != hipSuccess) return e;
    } else if (n_tiles > 0 && (e = forward_rows(c, s, i, H, st)) != hipSuccess) {
        return e;
    }
    // computed rows: the event means are formed inside the backprojection
    // (from the forward's pixel-group partials); cached rows come with them
    const bool fused_means = !cached && v.chunk_rows <= kMaxChunkRows;
    if (rows > 0 && !cached && !fused_means &&
        (e = timed(c, 2, [&] { return launch_mean(s->pmean, groups, rows, s->mean, s->inv, c->skipped_dev, st); }, st)) !=
            hipSuccess)
        return e;
    if (n_chunks > 0 &&
        (e = timed_kernel(c, 1, [&](const KernelEvents *ke) {
             if (fused_means)
                 return launch_backproject_means(g, v.chunks + v.chunk_off[i], n_chunks, v.chunk_rows, H, s->pmean,
                                                 groups, rows, s->mean, s->inv, c->skipped_dev, s->pb, st, ke);
             return launch_backproject(g, v.chunks + v.chunk_off[i], n_chunks, H, s->inv, s->pb, st, ke);
         })) != hipSuccess)
        return e;
    // the log-likelihood reads the means and the estimate before its update
    if (want_ll && (e = launch_loglik(g, rrange, v.n_real, s->mean, s->f, sens, s->ll, st)) != hipSuccess)
        return e;
    if ((e = timed(c, 2, [&] { return launch_update(g, crange, v.n_real, s->pb, sens, s->f, st); }, st)) != hipSuccess)
        return e;
    return hipSuccess;
}

void count_terms(lmosem_ctx *c, const lmosem_evset *s) {
    for (int i = 0; i < c->g.n_subsets; ++i) {
        c->terms += s->s.terms_sub[i];
        c->useful += s->s.useful_sub[i];
    }
}

// Capture one global iteration (all sub-iterations in order; with want_ll the
// log-likelihood accumulator is cleared by a fill kernel first) as a graph.
hipError_t capture_iteration(lmosem_ctx *c, lmosem_evset *s, bool want_ll) {
    hipError_t e;
    if (!c->gst) {
        if ((e = hipStreamCreateWithFlags(&c->gst, hipStreamNonBlocking)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&c->g_in, hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&c->g_out, hipEventDisableTiming)) != hipSuccess) return e;
    }
    hipGraph_t graph = nullptr;
    if ((e = hipStreamBeginCapture(c->gst, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    hipError_t body = hipSuccess;
    if (want_ll) body = launch_fill_d(s->ll, s->s.n_real, 0.0, c->gst);
    for (int i = 0; i < c->g.n_subsets && body == hipSuccess; ++i) body = subiteration(c, s, i, want_ll, c->gst);
    e = hipStreamEndCapture(c->gst, &graph);
    if (body != hipSuccess) { if (graph) hipGraphDestroy(graph); return body; }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&s->exec[(want_ll ? 1 : 0) + (s->Hc && s->rows_valid ? 2 : 0)], graph, nullptr, nullptr,
                            0);
    hipGraphDestroy(graph);
    return e;
}

// One global iteration: replay the captured graph on the internal stream,
// ordered after and before the caller's stream by events; plain launches on
// the caller's stream while kernel timing is on or graphs are disabled.
hipError_t one_iteration(lmosem_ctx *c, lmosem_evset *s, bool want_ll) {
    hipError_t e;
    const bool cached = s->Hc && s->rows_valid;
    // the surrogate path allocates network workspace lazily: never captured;
    // the iteration that fills the row cache runs once, uncaptured
    const bool graph = (!c->surrogate || cached) && !(s->Hc && !cached) &&
                       (s->use_graph >= 0 ? s->use_graph == 1 : c->graphs);
    if (!graph || c->timing) {
        if (want_ll && (e = launch_fill_d(s->ll, s->s.n_real, 0.0, c->st)) != hipSuccess) return e;
        for (int i = 0; i < c->g.n_subsets; ++i)
            if ((e = subiteration(c, s, i, want_ll, c->st)) != hipSuccess) return e;
    } else {
        const int k = (want_ll ? 1 : 0) + (cached ? 2 : 0);
        if (!s->exec[k] && (e = capture_iteration(c, s, want_ll)) != hipSuccess) return e;
        if ((e = hipEventRecord(c->g_in, c->st)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(c->gst, c->g_in, 0)) != hipSuccess) return e;
        if ((e = hipGraphLaunch(s->exec[k], c->gst)) != hipSuccess) return e;
        if ((e = hipEventRecord(c->g_out, c->gst)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(c->st, c->g_out, 0)) != hipSuccess) return e;
    }
    if (!cached) count_terms(c, s);
    if (s->Hc) s->rows_valid = true;
    return hipSuccess;
}

lmosem_status iterate_set(lmosem_ctx *c, lmosem_evset *s, int n_iters, double *ll_host) {
    std::vector<double> ll;
    if (ll_host) ll.assign((size_t)s->s.n_real * n_iters, 0.0);
    std::vector<double> tmp(s->s.n_real);
    hipError_t e;
    for (int it = 0; it < n_iters; ++it) {
        if ((e = one_iteration(c, s, ll_host != nullptr)) != hipSuccess) return dev_err(c, "iteration", e);
        if (ll_host) {
            if ((e = hipMemcpyAsync(tmp.data(), s->ll, sizeof(double) * s->s.n_real, hipMemcpyDeviceToHost,
                                    c->st)) != hipSuccess ||
                (e = hipStreamSynchronize(c->st)) != hipSuccess)
                return dev_err(c, "loglik", e);
            for (int r = 0; r < s->s.n_real; ++r) ll[(size_t)r * n_iters + it] = tmp[r];
        }
    }
    if (ll_host) std::copy(ll.begin(), ll.end(), ll_host);
    return LMOSEM_OK;
}

#define GUARD(c)                                                              \
    do {                                                                      \
        if (!(c)) return LMOSEM_EINVAL;                                       \
        if ((c)->poisoned) return LMOSEM_ESTATE;                              \
    } while (0)

// build the list-mode tables on first use; a failed build frees what it
// allocated and leaves the context usable (ENOMEM for a table too large)
lmosem_status ensure_paths(lmosem_ctx *c) {
    if (c->paths_ready) return LMOSEM_OK;
    const Geo &g = c->g;
    // the exact path's tables have a known size: refused before any allocation
    const int64_t predicted = (c->surrogate ? 0 : (int64_t)sizeof(float2) * g.n_angles * g.n_rpad * g.n_qpad) +
                              4 * (int64_t)g.n_angles * g.n_p + 4 * (int64_t)(g.n_subsets + 1) * g.n_qpad;
    if (over_cap(c, predicted)) return set_err(c, LMOSEM_ENOMEM, cap_msg(c, "the path tables", predicted));
    const auto t0 = std::chrono::steady_clock::now();
    std::string err;
    int64_t bytes = 0;
    const hipError_t e = build_paths(c->g, c->t, !c->surrogate, c->surrogate, c->st, err, bytes);
    if (e != hipSuccess) {
        hipStreamSynchronize(c->st);
        hipFree(c->t.T); hipFree(c->t.prim); hipFree(c->t.sens); hipFree(c->t.sens_all);
        hipFree(c->t.band); hipFree(c->t.band_lo);
        c->t.T = nullptr; c->t.prim = nullptr; c->t.sens = nullptr; c->t.sens_all = nullptr;
        c->t.band = nullptr; c->t.band_lo = nullptr;
        return alloc_err(c, ("path tables: " + err).c_str(), e);
    }
    if (over_cap(c, bytes)) {   // the near-field band's width is known only once built
        const std::string msg = cap_msg(c, "the path tables", bytes);
        hipStreamSynchronize(c->st);
        hipFree(c->t.T); hipFree(c->t.prim); hipFree(c->t.sens); hipFree(c->t.sens_all);
        hipFree(c->t.band); hipFree(c->t.band_lo);
        c->t.T = nullptr; c->t.prim = nullptr; c->t.sens = nullptr; c->t.sens_all = nullptr;
        c->t.band = nullptr; c->t.band_lo = nullptr;
        return set_err(c, LMOSEM_ENOMEM, msg);
    }
    c->table_bytes += bytes;
    c->table_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    c->paths_ready = true;
    return LMOSEM_OK;
}

#define PATHS(c)                                                              \
    do {                                                                      \
        const lmosem_status ps_ = ensure_paths(c);                            \
        if (ps_ != LMOSEM_OK) return ps_;                                     \
    } while (0)

}  // namespace

extern "C" {

uint32_t lmosem_abi_version(void) { return LMOSEM_ABI_VERSION; }

const char *lmosem_last_error(const lmosem_ctx *c) { return c ? c->err.c_str() : "null context"; }

lmosem_status lmosem_create(const lmosem_config *cfg, const float *mu_dev, void *hip_stream, lmosem_ctx **out) {
    return lmosem_create_emission(cfg, mu_dev, nullptr, hip_stream, out);
}

lmosem_status lmosem_create_emission(const lmosem_config *cfg, const float *mu_dev, const float *emission_dev,
                                     void *hip_stream, lmosem_ctx **out) {
    if (!cfg || !mu_dev || !out) return LMOSEM_EINVAL;
    *out = nullptr;
    std::string why;
    if (!check_cfg(cfg, why)) return LMOSEM_EINVAL;
    auto *c = new lmosem_ctx();
    c->cfg = *cfg;
    c->st = (hipStream_t)hip_stream;
    auto t0 = std::chrono::steady_clock::now();
    const int n_pix = cfg->nx * cfg->ny;
    std::vector<float> mu(n_pix);
    hipError_t e = hipMemcpyAsync(mu.data(), mu_dev, sizeof(float) * n_pix, hipMemcpyDeviceToHost, c->st);
    std::vector<float> em;
    if (e == hipSuccess && emission_dev) {
        em.resize(n_pix);
        e = hipMemcpyAsync(em.data(), emission_dev, sizeof(float) * n_pix, hipMemcpyDeviceToHost, c->st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) { delete c; return LMOSEM_EDEVICE; }
    // the support (mu > 0) with the emission pixels first
    std::vector<int> p_pix, q_of_pix(n_pix, -1);
    for (int p = 0; p < n_pix; ++p)
        if (!(mu[p] >= 0.0f) || !std::isfinite(mu[p])) { delete c; return LMOSEM_ERANGE; }
    for (int pass = 0; pass < 2; ++pass)
        for (int p = 0; p < n_pix; ++p) {
            const bool emits = em.empty() || em[p] > 0.0f;
            if (mu[p] > 0.0f && emits == (pass == 0)) { q_of_pix[p] = (int)p_pix.size(); p_pix.push_back(p); }
        }
    int n_q = 0;
    for (int p = 0; p < n_pix; ++p) n_q += mu[p] > 0.0f && (em.empty() || em[p] > 0.0f);
    if (n_q == 0) { delete c; return LMOSEM_ERANGE; }

    Geo &g = c->g;
    g.nx = cfg->nx; g.ny = cfg->ny; g.n_pix = n_pix;
    g.n_p = (int)p_pix.size();
    g.n_q = n_q;
    g.n_qpad = (g.n_q + 63) / 64 * 64;
    // forward workgroups of 4 waves (fewer for an emission set of up to 192
    // pixels, whose single workgroup would otherwise carry idle waves)
    g.fwd_waves = std::min(4, g.n_qpad / 64);
    g.n_rpad = g.n_p + kRankPad;
    g.n_angles = cfg->n_angles; g.n_bins = cfg->n_bins; g.n_subsets = cfg->n_subsets;
    g.scatter = cfg->scatter_model != 0;
    c->surrogate = cfg->scatter_model == 2;
    g.dx = cfg->pixel_cm; g.bin_cm = cfg->bin_cm; g.half_len = 0.5 * cfg->n_bins * cfg->bin_cm;
    g.e0 = cfg->e0_kev; g.kappa = cfg->e0_kev / kMeC2;
    const double fw = 2.0 * sqrt(2.0 * log(2.0));
    g.sig_e = cfg->fwhm_e_kev / fw;
    g.sig_u = cfg->fwhm_u_cm / fw;
    g.win_lo = cfg->win_lo_kev; g.win_hi = cfg->win_hi_kev;
    g.psi_bar = psi_bar_closed(g.kappa);
    g.sigma_kn_e0 = kn_total_host(g.e0);
    g.zk = g.sig_u * sqrt(2.0 * M_PI) * erf(3.0 / sqrt(2.0)) - 6.0 * g.sig_u * exp(-4.5);
    g.e_c = std::round(0.5 * (g.win_lo + g.win_hi) * 64.0) / 64.0;
    g.c2 = 1.0 / (2.0 * g.sig_e * g.sig_e * log(2.0));
    g.acq_time = cfg->acq_time;

    std::vector<double> cs(2 * g.n_angles);
    for (int a = 0; a < g.n_angles; ++a) {
        double th = cfg->angle0_rad + 2.0 * M_PI * a / g.n_angles;
        cs[2 * a] = cos(th);
        cs[2 * a + 1] = sin(th);
    }
// an allocation failure also clears HIP's last-error state, so that later
// calls of the caller's runtime do not report it again
#define CK(call, what) do { e = (call); if (e != hipSuccess) { lmosem_destroy(c); if (e == hipErrorOutOfMemory) (void)hipGetLastError(); return e == hipErrorOutOfMemory ? LMOSEM_ENOMEM : LMOSEM_EDEVICE; } } while (0)
    CK(hipMalloc(&c->t.p_pix, sizeof(int) * (g.n_p + n_pix)), "alloc");
    CK(hipMalloc(&c->t.mu, sizeof(float) * n_pix), "alloc");
    CK(hipMalloc(&c->t.cs, sizeof(double) * 2 * g.n_angles), "alloc");
    CK(hipMalloc(&c->bad_dev, sizeof(int)), "alloc");
    CK(hipMalloc(&c->skipped_dev, sizeof(unsigned long long)), "alloc");
    CK(hipMemsetAsync(c->skipped_dev, 0, sizeof(unsigned long long), c->st), "clear");
    CK(hipMemcpyAsync(c->t.p_pix, p_pix.data(), sizeof(int) * g.n_p, hipMemcpyHostToDevice, c->st), "upload");
    CK(hipMemcpyAsync(c->t.p_pix + g.n_p, q_of_pix.data(), sizeof(int) * n_pix, hipMemcpyHostToDevice, c->st),
       "upload");
    CK(hipMemcpyAsync(c->t.mu, mu.data(), sizeof(float) * n_pix, hipMemcpyHostToDevice, c->st), "upload");
    CK(hipMemcpyAsync(c->t.cs, cs.data(), sizeof(double) * 2 * g.n_angles, hipMemcpyHostToDevice, c->st), "upload");
#undef CK
    std::string err;
    e = build_base(g, c->t, c->st, err, c->table_bytes);
    if (e != hipSuccess) {
        lmosem_destroy(c);
        if (e == hipErrorOutOfMemory) (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? LMOSEM_ENOMEM : LMOSEM_EDEVICE;
    }
    c->table_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (const char *v = getenv("LMOSEM_EVENT_TILE")) {
        int t = atoi(v);
        if (t == 8 || t == 16 || t == 32) c->ev_tile = t;
    }
    *out = c;
    return LMOSEM_OK;
}

void lmosem_destroy(lmosem_ctx *c) {
    if (!c) return;
    drain_timing(c);
    if (c->gst) hipStreamSynchronize(c->gst);
    if (c->g_in) hipEventDestroy(c->g_in);
    if (c->g_out) hipEventDestroy(c->g_out);
    if (c->gst) hipStreamDestroy(c->gst);
    hipFree(c->t.p_pix); hipFree(c->t.mu); hipFree(c->t.cs); hipFree(c->t.s_sorted); hipFree(c->t.us_sorted); hipFree(c->t.mu_sorted);
    hipFree(c->t.T); hipFree(c->t.sens); hipFree(c->t.sens_all); hipFree(c->t.Ldet); hipFree(c->t.Lback);
    hipFree(c->t.prim); hipFree(c->t.band); hipFree(c->t.band_lo); hipFree(c->t.Ld); hipFree(c->t.Bt);
    hipFree(c->t.D_sorted); hipFree(c->bad_dev); hipFree(c->skipped_dev);
    delete c;
}

lmosem_status lmosem_sensitivity(lmosem_ctx *c, int32_t subset, float *sens_dev) {
    GUARD(c);
    PATHS(c);
    if (!sens_dev || subset < -1 || subset >= c->g.n_subsets) return set_err(c, LMOSEM_EINVAL, "bad subset");
    const float *src = subset < 0 ? c->t.sens_all : c->t.sens + (size_t)subset * c->g.n_qpad;
    hipError_t e = launch_scatter_image(c->g, c->t, src, 1, sens_dev, c->st);
    return e == hipSuccess ? LMOSEM_OK : dev_err(c, "sensitivity", e);
}

lmosem_status lmosem_events_load(lmosem_ctx *c, const lmosem_events *ev, const lmosem_batch *batch,
                                 lmosem_evset **out) {
    GUARD(c);
    PATHS(c);
    if (!out) return set_err(c, LMOSEM_EINVAL, "null output");
    *out = nullptr;
    return load_set(c, ev, batch, -1, out);
}

void lmosem_events_free(lmosem_evset *s) { free_set(s); }

lmosem_status lmosem_iterate(lmosem_ctx *c, lmosem_evset *s, int32_t n_iters, float *images_dev,
                             double *loglik_host) {
    GUARD(c);
    PATHS(c);
    if (!s || s->s.ctx != c || !images_dev || n_iters < 0) return set_err(c, LMOSEM_EINVAL, "bad arguments");
    const Geo &g = c->g;
    hipError_t e = launch_gather_image(g, c->t, images_dev, s->s.n_real, g.n_pix, s->f, 0, c->st);
    if (e != hipSuccess) return dev_err(c, "gather image", e);
    lmosem_status st = iterate_set(c, s, n_iters, loglik_host);
    if (st != LMOSEM_OK) return st;
    e = launch_scatter_image(g, c->t, s->f, s->s.n_real, images_dev, c->st);
    return e == hipSuccess ? LMOSEM_OK : dev_err(c, "scatter image", e);
}

lmosem_status lmosem_reconstruct(lmosem_ctx *c, const lmosem_events *ev, const lmosem_batch *batch,
                                 int32_t n_iters, const float *init_dev, float *images_dev,
                                 double *loglik_host) {
    GUARD(c);
    PATHS(c);
    if (!images_dev || n_iters < 0) return set_err(c, LMOSEM_EINVAL, "bad arguments");
    const Geo &g = c->g;
    hipError_t e;
    if (init_dev) {
        int bad = 0;
        if ((e = hipMemsetAsync(c->bad_dev, 0, sizeof(int), c->st)) != hipSuccess ||
            (e = launch_check_image(g, c->t, init_dev, c->bad_dev, c->st)) != hipSuccess ||
            (e = hipMemcpyAsync(&bad, c->bad_dev, sizeof(int), hipMemcpyDeviceToHost, c->st)) != hipSuccess ||
            (e = hipStreamSynchronize(c->st)) != hipSuccess)
            return dev_err(c, "check init", e);
        if (bad) return set_err(c, LMOSEM_ERANGE, "initial image negative or not finite on the support");
    }
    lmosem_evset *s = nullptr;
    lmosem_status st = load_set(c, ev, batch, -1, &s);
    if (st != LMOSEM_OK) return st;
    e = launch_gather_image(g, c->t, init_dev, s->s.n_real, 0, s->f, 1, c->st);
    if (e != hipSuccess) { free_set(s); return dev_err(c, "init", e); }
    st = iterate_set(c, s, n_iters, loglik_host);
    if (st == LMOSEM_OK) {
        e = launch_scatter_image(g, c->t, s->f, s->s.n_real, images_dev, c->st);
        if (e != hipSuccess) st = dev_err(c, "scatter image", e);
    }
    if (st == LMOSEM_OK && (e = hipStreamSynchronize(c->st)) != hipSuccess) st = dev_err(c, "reconstruct", e);
    free_set(s);
    return st;
}

lmosem_status lmosem_subset_update(lmosem_ctx *c, int32_t subset, const lmosem_events *ev, float *image_dev,
                                   float *event_mean_dev) {
    GUARD(c);
    PATHS(c);
    if (!image_dev || subset < 0 || subset >= c->g.n_subsets) return set_err(c, LMOSEM_EINVAL, "bad arguments");
    const char *val = getenv("LMOSEM_VALIDATE");
    if (val && atoi(val) == 1 && ev && ev->n > 0) {
        std::vector<int32_t> ang(ev->n);
        hipError_t e = hipMemcpyAsync(ang.data(), ev->angle, sizeof(int32_t) * ev->n, hipMemcpyDeviceToHost, c->st);
        if (e == hipSuccess) e = hipStreamSynchronize(c->st);
        if (e != hipSuccess) return dev_err(c, "validate", e);
        int64_t wrong = 0;
        for (int32_t a : ang) wrong += (a >= 0 && a % c->g.n_subsets != subset);
        if (wrong) return set_err(c, LMOSEM_ERANGE, std::to_string(wrong) + " events not in the subset");
    }
    lmosem_evset *s = nullptr;
    lmosem_status st = load_set(c, ev, nullptr, subset, &s);
    if (st != LMOSEM_OK) return st;
    const Geo &g = c->g;
    hipError_t e = launch_gather_image(g, c->t, image_dev, 1, 0, s->f, 0, c->st);
    if (e == hipSuccess) e = subiteration(c, s, subset, false, c->st);
    if (e == hipSuccess) { c->terms += s->s.terms_sub[subset]; c->useful += s->s.useful_sub[subset]; }
    if (e == hipSuccess && event_mean_dev)
        e = launch_scatter_rows(s->mean, s->s.orig + s->s.row_off[subset],
                                s->s.row_off[subset + 1] - s->s.row_off[subset], event_mean_dev, c->st);
    if (e == hipSuccess) e = launch_scatter_image(g, c->t, s->f, 1, image_dev, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    free_set(s);
    return e == hipSuccess ? LMOSEM_OK : dev_err(c, "subset update", e);
}

lmosem_status lmosem_forward(lmosem_ctx *c, const lmosem_events *ev, const float *image_dev, float *mean_dev) {
    GUARD(c);
    PATHS(c);
    if (!image_dev || !mean_dev) return set_err(c, LMOSEM_EINVAL, "bad arguments");
    lmosem_evset *s = nullptr;
    lmosem_status st = load_set(c, ev, nullptr, 0, &s);
    if (st != LMOSEM_OK) return st;
    const Geo &g = c->g;
    const EvSet &v = s->s;
    const int rows = v.row_off[1];
    hipError_t e = launch_gather_image(g, c->t, image_dev, 1, 0, s->f, 0, c->st);
    if (e == hipSuccess) e = forward_rows(c, s, 0, s->H, c->st);
    if (e == hipSuccess) e = launch_mean(s->pmean, mean_groups(c, s), rows, s->mean, s->inv, c->skipped_dev, c->st);
    if (e == hipSuccess) e = launch_scatter_rows(s->mean, v.orig, rows, mean_dev, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e == hipSuccess) { c->terms += v.terms_sub[0]; c->useful += v.useful_sub[0]; }
    free_set(s);
    return e == hipSuccess ? LMOSEM_OK : dev_err(c, "forward", e);
}

lmosem_status lmosem_forward_noalloc(lmosem_ctx *c, const lmosem_events *ev, const float *image_dev,
                                     float *event_mean_dev) {
    GUARD(c);
    if (!c->paths_ready)
        return set_err(c, LMOSEM_EINVAL, "the path tables are not built yet: make one list-mode call on this context "
                                         "first (for example lmosem_sensitivity)");
    if (c->surrogate) return set_err(c, LMOSEM_ENOTSUP, "no allocation-free forward for scatter_model 2");
    if (!ev || ev->n < 0 || ev->n > 0x7fffffffLL || (ev->n > 0 && (!ev->angle || !ev->u_bin || !ev->energy_kev)))
        return set_err(c, LMOSEM_EINVAL, "bad event arrays");
    if (!image_dev || (ev->n > 0 && !event_mean_dev)) return set_err(c, LMOSEM_EINVAL, "bad arguments");
    size_t need = 0;
    hipError_t e = forward_noalloc_bytes(c->g, ev->n, c->ev_tile, need);
    if (e != hipSuccess) return dev_err(c, "forward (no allocation)", e);
    if (need > kScratchBytes)
        return set_err(c, LMOSEM_ENOMEM, std::to_string(ev->n) + " events need " + std::to_string(need) +
                                             " bytes of scratch memory; the library's scratch array holds " +
                                             std::to_string(kScratchBytes));
    lmosem_status st = LMOSEM_OK;
    if (!check_events(c, ev, st)) return st;
    int64_t terms = 0, useful = 0;
    e = forward_noalloc(c->g, c->t, *ev, c->ev_tile, image_dev, event_mean_dev, c->skipped_dev, c->st, terms, useful);
    if (e != hipSuccess) return dev_err(c, "forward (no allocation)", e);
    c->terms += terms;
    c->useful += useful;
    return LMOSEM_OK;
}

lmosem_status lmosem_backproject(lmosem_ctx *c, const lmosem_events *ev, const float *weights_dev,
                                 float *image_dev) {
    GUARD(c);
    PATHS(c);
    if (!image_dev || (!weights_dev && ev && ev->n > 0)) return set_err(c, LMOSEM_EINVAL, "bad arguments");
    lmosem_evset *s = nullptr;
    lmosem_status st = load_set(c, ev, nullptr, 0, &s);
    if (st != LMOSEM_OK) return st;
    const Geo &g = c->g;
    const EvSet &v = s->s;
    const int rows = v.row_off[1];
    hipError_t e = launch_fill(s->f, (size_t)g.n_qpad, 0.0f, c->st);
    if (e == hipSuccess) e = forward_rows(c, s, 0, s->H, c->st);
    if (e == hipSuccess) e = launch_gather_rows(weights_dev, v.orig, rows, s->inv, c->st);
    if (e == hipSuccess) e = launch_backproject(g, v.chunks, v.chunk_off[1], s->H, s->inv, s->pb, c->st);
    if (e == hipSuccess) e = launch_sum_real(g, v.crange, 1, s->pb, s->f, c->st);
    if (e == hipSuccess) e = launch_scatter_image(g, c->t, s->f, 1, image_dev, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e == hipSuccess) { c->terms += v.terms_sub[0]; c->useful += v.useful_sub[0]; }
    free_set(s);
    return e == hipSuccess ? LMOSEM_OK : dev_err(c, "backproject", e);
}

lmosem_status lmosem_set_tuning(lmosem_ctx *c, int32_t event_tile) {
    GUARD(c);
    if (event_tile == 0) event_tile = 8;
    if (event_tile != 8 && event_tile != 16 && event_tile != 32)
        return set_err(c, LMOSEM_EINVAL, "event_tile must be 8, 16 or 32");
    c->ev_tile = event_tile;
    return LMOSEM_OK;
}

lmosem_status lmosem_set_pixel_tile(lmosem_ctx *c, int32_t pixels) {
    GUARD(c);
    if (pixels != 0 && pixels != 64 && pixels != 128 && pixels != 192 && pixels != 256)
        return set_err(c, LMOSEM_EINVAL, "pixel tile must be 64, 128, 192 or 256 (0: the default)");
    c->pixel_waves = pixels / 64;
    return LMOSEM_OK;
}

struct lmosem_net {
    lmo::Net *n = nullptr;
};

lmosem_status lmosem_net_create(const float *params_host, void *hip_stream, lmosem_net **out) {
    if (!params_host || !out) return LMOSEM_EINVAL;
    *out = nullptr;
    lmo::Net *n = nullptr;
    hipError_t e = net_create(params_host, (hipStream_t)hip_stream, &n);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? LMOSEM_ENOMEM : LMOSEM_EDEVICE;
    *out = new lmosem_net{n};
    return LMOSEM_OK;
}

void lmosem_net_destroy(lmosem_net *net) {
    if (!net) return;
    net_destroy(net->n);
    delete net;
}

lmosem_status lmosem_net_get_params(lmosem_net *net, float *params_host) {
    if (!net || !params_host) return LMOSEM_EINVAL;
    return net_get_params(net->n, params_host) == hipSuccess ? LMOSEM_OK : LMOSEM_EDEVICE;
}

lmosem_status lmosem_net_forward(lmosem_net *net, const float *X_dev, int64_t n, float *y_dev) {
    if (!net || n < 0 || (n > 0 && (!X_dev || !y_dev))) return LMOSEM_EINVAL;
    return net_forward(net->n, X_dev, n, y_dev, net_stream(net->n)) == hipSuccess ? LMOSEM_OK : LMOSEM_EDEVICE;
}

lmosem_status lmosem_net_forward_train(lmosem_net *net, const float *X_dev, int32_t n, float *y_dev) {
    if (!net || !X_dev || !y_dev || n <= 0 || n % 16) return LMOSEM_EINVAL;
    return net_forward_train(net->n, X_dev, n, y_dev) == hipSuccess ? LMOSEM_OK : LMOSEM_EDEVICE;
}

lmosem_status lmosem_net_gradient(lmosem_net *net, const float *X_dev, const float *dy_dev, int32_t n,
                                  float *grad_host) {
    if (!net || !X_dev || !dy_dev || !grad_host || n <= 0 || n % 16) return LMOSEM_EINVAL;
    return net_gradient(net->n, X_dev, dy_dev, n, grad_host) == hipSuccess ? LMOSEM_OK : LMOSEM_EDEVICE;
}

lmosem_status lmosem_net_train(lmosem_net *net, const float *X_dev, const float *t_dev, int64_t n, int32_t batch,
                               int32_t epochs, float lr, float lr_decay, double *loss_host) {
    if (!net || !X_dev || !t_dev || batch <= 0 || batch % 16 || n < batch || epochs < 0 || !(lr > 0))
        return LMOSEM_EINVAL;
    return net_train(net->n, X_dev, t_dev, n, batch, epochs, lr, lr_decay, loss_host) == hipSuccess ? LMOSEM_OK
                                                                                                    : LMOSEM_EDEVICE;
}

lmosem_status lmosem_surrogate_samples(lmosem_ctx *c, const int32_t *pixel, const int32_t *angle,
                                       const float *u_bin, const float *energy, int64_t n, float *X_dev,
                                       float *target_dev, float *scatter_dev) {
    GUARD(c);
    if (!c->t.Bt)
        return set_err(c, LMOSEM_ENOTSUP, "training samples need the first-order scatter model (scatter_model 1 or 2)");
    if (n < 0 || (n > 0 && (!pixel || !angle || !u_bin || !energy || !X_dev || !target_dev)))
        return set_err(c, LMOSEM_EINVAL, "bad sample arrays");
    // the samples' angles, positions and energies follow the event rules;
    // their pixels must lie in the emission set
    lmosem_events ev{n, angle, u_bin, energy};
    lmosem_status st = LMOSEM_OK;
    if (!check_events(c, &ev, st)) return st;
    if (n > 0) {
        std::vector<int32_t> px(n);
        hipError_t e = hipMemcpyAsync(px.data(), pixel, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->st);
        if (e == hipSuccess) e = hipStreamSynchronize(c->st);
        if (e != hipSuccess) return dev_err(c, "samples", e);
        std::vector<int> qop(c->g.n_pix);
        e = hipMemcpy(qop.data(), c->t.p_pix + c->g.n_p, sizeof(int) * c->g.n_pix, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return dev_err(c, "samples", e);
        for (int32_t p : px)
            if (p < 0 || p >= c->g.n_pix || qop[p] < 0 || qop[p] >= c->g.n_q)
                return set_err(c, LMOSEM_ERANGE, "sample pixel outside the emission set");
    }
    hipError_t e = surrogate_samples(c->g, c->t, pixel, angle, u_bin, energy, n, X_dev, target_dev, scatter_dev,
                                     c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    return e == hipSuccess ? LMOSEM_OK : dev_err(c, "samples", e);
}

lmosem_status lmosem_set_surrogate(lmosem_ctx *c, lmosem_net *net) {
    GUARD(c);
    if (!c->surrogate) return set_err(c, LMOSEM_EINVAL, "the context was not created with scatter_model 2");
    c->net = net ? net->n : nullptr;
    return LMOSEM_OK;
}

lmosem_status lmosem_set_memory_cap(lmosem_ctx *c, int64_t bytes) {
    GUARD(c);
    if (bytes < 0) return set_err(c, LMOSEM_EINVAL, "the memory cap must be >= 0");
    c->mem_cap = bytes;
    return LMOSEM_OK;
}

lmosem_status lmosem_memory_held(const lmosem_ctx *c, int64_t *bytes) {
    if (!c || !bytes) return LMOSEM_EINVAL;
    *bytes = c->table_bytes + c->set_bytes;
    return LMOSEM_OK;
}

lmosem_status lmosem_inject_failure(lmosem_ctx *c) {
    GUARD(c);
    c->inject_failure = true;
    return LMOSEM_OK;
}

lmosem_status lmosem_set_graphs(lmosem_ctx *c, int32_t enable) {
    GUARD(c);
    c->graphs = enable != 0;
    return LMOSEM_OK;
}

namespace {

// validation of a binning; the energy edges go to the device
lmosem_status binning(lmosem_ctx *c, int32_t n_pos, const double *edges, int32_t n_e, double **edges_dev) {
    if (n_pos < 1 || n_e < 1 || !edges) return set_err(c, LMOSEM_EINVAL, "bad binning");
    for (int k = 0; k < n_e; ++k)
        if (!(edges[k + 1] > edges[k]) || !std::isfinite(edges[k]) || !std::isfinite(edges[k + 1]))
            return set_err(c, LMOSEM_EINVAL, "energy edges must increase");
    if ((int64_t)c->g.n_angles * n_pos * n_e > (1 << 26)) return set_err(c, LMOSEM_ERANGE, "too many bins");
    hipError_t e = hipMalloc(edges_dev, sizeof(double) * (n_e + 1));
    if (e == hipSuccess) e = hipMemcpyAsync(*edges_dev, edges, sizeof(double) * (n_e + 1), hipMemcpyHostToDevice, c->st);
    return e == hipSuccess ? LMOSEM_OK : dev_err(c, "binning", e);
}

}  // namespace

lmosem_status lmosem_bin_events(lmosem_ctx *c, const lmosem_events *ev, int32_t n_pos, const double *e_edges,
                                int32_t n_ebins, float *counts_dev) {
    GUARD(c);
    if (!counts_dev) return set_err(c, LMOSEM_EINVAL, "bad counts");
    // events outside every bin (any angle, position or energy) are dropped
    if (!ev || ev->n < 0 || (ev->n > 0 && (!ev->angle || !ev->u_bin || !ev->energy_kev)))
        return set_err(c, LMOSEM_EINVAL, "bad event arrays");
    lmosem_status st = LMOSEM_OK;
    double *edges = nullptr;
    if ((st = binning(c, n_pos, e_edges, n_ebins, &edges)) != LMOSEM_OK) { hipFree(edges); return st; }
    const size_t n_cnt = (size_t)c->g.n_angles * n_pos * n_ebins;
    hipError_t e = launch_fill(counts_dev, n_cnt, 0.0f, c->st);
    if (e == hipSuccess) e = launch_bin_events(c->g, *ev, n_pos, edges, n_ebins, counts_dev, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    hipFree(edges);
    return e == hipSuccess ? LMOSEM_OK : dev_err(c, "bin events", e);
}

lmosem_status lmosem_emission_mask(lmosem_ctx *c, const float *image_dev, double rel_threshold, int32_t margin_px,
                                   float *mask_dev) {
    GUARD(c);
    if (!image_dev || !mask_dev || !(rel_threshold >= 0.0 && rel_threshold <= 1.0) || margin_px < 0 || margin_px > 32)
        return set_err(c, LMOSEM_EINVAL, "bad arguments");
    float *mx = nullptr, host[2] = {0.0f, 0.0f};
    hipError_t e = hipMalloc(&mx, 2 * sizeof(float));
    if (e == hipSuccess) e = launch_image_max(image_dev, c->g.n_pix, mx, c->st);
    if (e == hipSuccess) e = hipMemcpyAsync(host, mx, sizeof host, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    hipFree(mx);
    if (e != hipSuccess) return dev_err(c, "emission mask", e);
    if (host[1] != 0.0f) return set_err(c, LMOSEM_ERANGE, "image values must be finite and >= 0");
    e = launch_emission_mask(c->g, c->t.mu, image_dev, rel_threshold * (double)host[0], margin_px, mask_dev, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    return e == hipSuccess ? LMOSEM_OK : dev_err(c, "emission mask", e);
}

lmosem_status lmosem_binned_rows(lmosem_ctx *c, int32_t n_pos, const double *e_edges, int32_t n_ebins, int64_t n,
                                 const int32_t *bins_dev, float *rows_dev) {
    GUARD(c);
    if (n < 0 || n > (1 << 24) || (n > 0 && (!bins_dev || !rows_dev))) return set_err(c, LMOSEM_EINVAL, "bad arguments");
    if (n == 0) return LMOSEM_OK;
    const Geo &g = c->g;
    std::vector<int32_t> bins(n);
    hipError_t e = hipMemcpyAsync(bins.data(), bins_dev, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) return dev_err(c, "binned rows", e);
    const int64_t n_all = (int64_t)g.n_angles * n_pos * n_ebins;
    for (int32_t b : bins)
        if (b < 0 || b >= n_all) return set_err(c, LMOSEM_ERANGE, "bin index out of range");
    double *edges = nullptr;
    lmosem_status st = binning(c, n_pos, e_edges, n_ebins, &edges);
    if (st != LMOSEM_OK) { hipFree(edges); return st; }
    float *H = nullptr;
    e = hipMalloc(&H, sizeof(float) * (size_t)n * g.n_qpad);
    if (e == hipSuccess)
        e = launch_binned_rows(g, c->t, n_pos, edges, n_ebins, reinterpret_cast<const int *>(bins_dev), (int)n, H, c->st);
    if (e == hipSuccess) e = launch_scatter_image(g, c->t, H, (int)n, rows_dev, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    hipFree(H);
    hipFree(edges);
    return e == hipSuccess ? LMOSEM_OK : dev_err(c, "binned rows", e);
}

lmosem_status lmosem_binned_reconstruct(lmosem_ctx *c, int32_t n_pos, const double *e_edges, int32_t n_ebins,
                                        const float *counts_dev, int32_t n_iters, const float *init_dev,
                                        float *image_dev) {
    GUARD(c);
    if (!counts_dev || !image_dev || n_iters < 0) return set_err(c, LMOSEM_EINVAL, "bad arguments");
    const Geo &g = c->g;
    double *edges = nullptr;
    lmosem_status st = binning(c, n_pos, e_edges, n_ebins, &edges);
    if (st != LMOSEM_OK) { hipFree(edges); return st; }
    // rows ordered by subset, then angle, position bin and energy bin
    const int per_angle = n_pos * n_ebins;
    std::vector<int> row_bin, sub_off(g.n_subsets + 1, 0), chunk_off(g.n_subsets + 1, 0);
    std::vector<Chunk> chunks;
    std::vector<int> cr;   // per subset {0, n_chunks}
    const int kRows = 256;
    for (int i = 0; i < g.n_subsets; ++i) {
        sub_off[i] = (int)row_bin.size();
        for (int a = i; a < g.n_angles; a += g.n_subsets)
            for (int k = 0; k < per_angle; ++k) row_bin.push_back(a * per_angle + k);
        const int rows = (int)row_bin.size() - sub_off[i];
        chunk_off[i] = (int)chunks.size();
        for (int j0 = 0; j0 < rows; j0 += kRows) chunks.push_back(Chunk{j0, std::min(rows, j0 + kRows), 0, 0});
        cr.push_back(0);
        cr.push_back((int)chunks.size() - chunk_off[i]);
    }
    sub_off[g.n_subsets] = (int)row_bin.size();
    chunk_off[g.n_subsets] = (int)chunks.size();
    const int n_rows = (int)row_bin.size();
    int max_rows = 0, max_chunks = 0;
    for (int i = 0; i < g.n_subsets; ++i) {
        max_rows = std::max(max_rows, sub_off[i + 1] - sub_off[i]);
        max_chunks = std::max(max_chunks, chunk_off[i + 1] - chunk_off[i]);
    }
    std::vector<int> rr;   // per subset {0, rows}
    for (int i = 0; i < g.n_subsets; ++i) { rr.push_back(0); rr.push_back(sub_off[i + 1] - sub_off[i]); }
    std::vector<int> row0(g.n_angles);   // first row of each angle
    for (int a = 0; a < g.n_angles; ++a) row0[a] = sub_off[a % g.n_subsets] + (a / g.n_subsets) * per_angle;

    float *H = nullptr, *y = nullptr, *mean = nullptr, *inv = nullptr, *w = nullptr, *ones = nullptr, *pb = nullptr;
    float *sens = nullptr, *f = nullptr;
    int *d_rows = nullptr, *d_cr = nullptr, *d_rr = nullptr, *d_row0 = nullptr;
    Chunk *d_chunks = nullptr;
    unsigned long long *dead = nullptr;
    hipError_t e = hipSuccess;
    auto al = [&](void **p, size_t bytes) { if (e == hipSuccess) e = hipMalloc(p, bytes); };
    al((void **)&H, sizeof(float) * (size_t)n_rows * g.n_qpad);
    al((void **)&y, sizeof(float) * n_rows);
    al((void **)&mean, sizeof(float) * max_rows);
    al((void **)&inv, sizeof(float) * max_rows);
    al((void **)&w, sizeof(float) * max_rows);
    al((void **)&ones, sizeof(float) * max_rows);
    al((void **)&pb, sizeof(float) * (size_t)std::max(max_chunks, 1) * g.n_qpad);
    al((void **)&sens, sizeof(float) * (size_t)g.n_subsets * g.n_qpad);
    al((void **)&f, sizeof(float) * g.n_qpad);
    al((void **)&d_rows, sizeof(int) * n_rows);
    al((void **)&d_cr, sizeof(int) * cr.size());
    al((void **)&d_rr, sizeof(int) * rr.size());
    al((void **)&d_row0, sizeof(int) * row0.size());
    al((void **)&d_chunks, sizeof(Chunk) * std::max<size_t>(chunks.size(), 1));
    al((void **)&dead, sizeof(unsigned long long));
    auto up = [&](void *dst, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->st);
    };
    up(d_rows, row_bin.data(), sizeof(int) * n_rows);
    up(d_cr, cr.data(), sizeof(int) * cr.size());
    up(d_rr, rr.data(), sizeof(int) * rr.size());
    up(d_row0, row0.data(), sizeof(int) * row0.size());
    up(d_chunks, chunks.data(), sizeof(Chunk) * chunks.size());
    if (e == hipSuccess) e = launch_fill(ones, max_rows, 1.0f, c->st);
    if (e == hipSuccess) {
        e = launch_binned_rows_all(g, c->t, n_pos, edges, n_ebins, d_row0, H, c->st);
        if (e == hipErrorNotSupported) e = launch_binned_rows(g, c->t, n_pos, edges, n_ebins, d_rows, n_rows, H, c->st);
    }
    if (e == hipSuccess) e = launch_gather_counts(counts_dev, d_rows, n_rows, y, c->st);
    // the binned sensitivity of each subset: column sums of its rows
    for (int i = 0; i < g.n_subsets && e == hipSuccess; ++i) {
        const float *Hi = H + (size_t)sub_off[i] * g.n_qpad;
        e = launch_backproject(g, d_chunks + chunk_off[i], chunk_off[i + 1] - chunk_off[i], Hi, ones, pb, c->st);
        if (e == hipSuccess) e = launch_sum_real(g, d_cr + 2 * i, 1, pb, sens + (size_t)i * g.n_qpad, c->st);
    }
    if (e == hipSuccess) e = launch_gather_image(g, c->t, init_dev, 1, 0, f, 0, c->st);
    for (int it = 0; it < n_iters && e == hipSuccess; ++it)
        for (int i = 0; i < g.n_subsets && e == hipSuccess; ++i) {
            const int rows = sub_off[i + 1] - sub_off[i];
            const float *Hi = H + (size_t)sub_off[i] * g.n_qpad;
            e = launch_row_dot(g, d_rr + 2 * i, 1, rows, Hi, f, mean, inv, dead, c->st);
            if (e == hipSuccess) e = launch_count_weights(y + sub_off[i], inv, rows, w, c->st);
            if (e == hipSuccess)
                e = launch_backproject(g, d_chunks + chunk_off[i], chunk_off[i + 1] - chunk_off[i], Hi, w, pb, c->st);
            if (e == hipSuccess) e = launch_update(g, d_cr + 2 * i, 1, pb, sens + (size_t)i * g.n_qpad, f, c->st);
        }
    if (e == hipSuccess) e = launch_scatter_image(g, c->t, f, 1, image_dev, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    for (void *p : {(void *)H, (void *)y, (void *)mean, (void *)inv, (void *)w, (void *)ones, (void *)pb, (void *)sens,
                    (void *)f, (void *)d_rows, (void *)d_cr, (void *)d_rr, (void *)d_row0, (void *)d_chunks, (void *)dead,
                    (void *)edges})
        hipFree(p);
    if (e == hipErrorOutOfMemory) { (void)hipGetLastError(); return set_err(c, LMOSEM_ENOMEM, "binned reconstruction: out of memory"); }
    return e == hipSuccess ? LMOSEM_OK : dev_err(c, "binned reconstruction", e);
}

lmosem_status lmosem_cache_rows(lmosem_ctx *c, lmosem_evset *s, int32_t enable) {
    GUARD(c);
    PATHS(c);
    if (!s || s->s.ctx != c) return set_err(c, LMOSEM_EINVAL, "bad event set");
    drop_graphs(s);
    s->rows_valid = false;
    if (!enable) {
        hipFree(s->Hc);
        s->Hc = nullptr;
        c->set_bytes -= s->bytes;
        s->bytes = set_device_bytes(c, s);
        c->set_bytes += s->bytes;
        return LMOSEM_OK;
    }
    if (s->Hc) return LMOSEM_OK;
    const size_t n = (size_t)std::max<int64_t>(s->s.n, 1) * c->g.n_qpad;
    if (over_cap(c, (int64_t)(sizeof(float) * n)))
        return set_err(c, LMOSEM_ENOMEM, cap_msg(c, "the row cache", (int64_t)(sizeof(float) * n)));
    hipError_t e = hipMalloc(&s->Hc, sizeof(float) * n);
    if (e != hipSuccess) {
        s->Hc = nullptr;
        (void)hipGetLastError();
        return set_err(c, LMOSEM_ENOMEM, "row cache: " + std::to_string(sizeof(float) * n) + " bytes not available");
    }
    c->set_bytes -= s->bytes;
    s->bytes = set_device_bytes(c, s);
    c->set_bytes += s->bytes;
    // zero padding columns (the learned-scatter rows never write them)
    e = launch_fill(s->Hc, n, 0.0f, c->st);
    return e == hipSuccess ? LMOSEM_OK : dev_err(c, "row cache", e);
}

}  // extern "C"

namespace {

std::string tune_key(const lmosem_ctx *c, const lmosem_evset *s) {
    int lg = 0;
    while ((1 << (lg + 1)) <= std::max(1, s->s.max_rows)) ++lg;
    char buf[160];
    snprintf(buf, sizeof buf, "np=%d nq=%d na=%d ns=%d real=%d rows2^%d", c->g.n_p, c->g.n_q, c->g.n_angles,
             c->g.n_subsets,
             s->s.n_real, lg);
    return buf;
}

bool tune_lookup(const std::string &key, int &ev, int &ch, int &graph, int &waves) {
    const char *path = getenv("LMOSEM_TUNE_CACHE");
    if (!path) return false;
    FILE *fp = fopen(path, "r");
    if (!fp) return false;
    char line[256];
    bool found = false;
    while (fgets(line, sizeof line, fp)) {
        std::string l(line);
        size_t bar = l.find('|');
        if (bar == std::string::npos || l.substr(0, bar) != key) continue;
        int w = 0;
        const int got = sscanf(l.c_str() + bar + 1, "%d %d %d %d", &ev, &ch, &graph, &w);
        found = got >= 3;
        waves = got == 4 ? w : 0;   // lines without a pixel tile keep the context's
    }
    fclose(fp);
    return found && (ev == 8 || ev == 16 || ev == 32) && ch >= 32 && (graph == 0 || graph == 1) && waves >= 0 &&
           waves <= 4;
}

void tune_store(const std::string &key, int ev, int ch, int graph, int waves) {
    const char *path = getenv("LMOSEM_TUNE_CACHE");
    if (!path) return;
    if (FILE *fp = fopen(path, "a")) {
        fprintf(fp, "%s|%d %d %d %d\n", key.c_str(), ev, ch, graph, waves);
        fclose(fp);
    }
}

// time one launch sequence on the context stream: one warm-up run, then the
// fastest of up to three timed runs (three while a run takes under 2 ms, so
// that short trials are not decided by one sample; one for longer runs,
// whose spread is small)
template <class F>
hipError_t time_ms(lmosem_ctx *c, F &&run, float &ms) {
    hipEvent_t a, b;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) { hipEventDestroy(a); return e; }
    e = run();   // warm-up
    ms = 3.4e38f;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
        float t = 0.0f;
        if ((e = hipEventRecord(a, c->st)) == hipSuccess && (e = run()) == hipSuccess &&
            (e = hipEventRecord(b, c->st)) == hipSuccess && (e = hipEventSynchronize(b)) == hipSuccess &&
            (e = hipEventElapsedTime(&t, a, b)) == hipSuccess)
            ms = std::min(ms, t);
        if (t >= 2.0f) break;
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    return e;
}

}  // namespace

extern "C" {

lmosem_status lmosem_autotune(lmosem_ctx *c, lmosem_evset *s, int32_t *event_tile, int32_t *chunk_rows,
                              int32_t *use_graphs) {
    GUARD(c);
    PATHS(c);
    if (!s || s->s.ctx != c) return set_err(c, LMOSEM_EINVAL, "bad event set");
    const Geo &g = c->g;
    EvSet &v = s->s;
    std::string why, key = tune_key(c, s);
    // tune the computing path; a row cache is refilled by the next iteration
    float *hc = s->Hc;
    s->Hc = nullptr;
    s->rows_valid = false;
    struct Restore {
        lmosem_evset *s;
        float *hc;
        ~Restore() { s->Hc = hc; s->rows_valid = false; drop_graphs(s); }
    } restore{s, hc};
    int best_ev = v.ev_tile, best_ch = v.chunk_rows, best_graph = -1, best_waves = v.fwd_waves;
    float fwd_ms = 0.0f;   // the fastest forward launch of the largest subset
    hipError_t e = hipSuccess;
    if (tune_lookup(key, best_ev, best_ch, best_graph, best_waves)) {
        v.fwd_waves = best_waves;
    } else {
        best_graph = -1;
        // the largest subset is the one the choice matters for
        int big = 0;
        for (int i = 1; i < g.n_subsets; ++i)
            if (v.row_off[i + 1] - v.row_off[i] > v.row_off[big + 1] - v.row_off[big]) big = i;
        const int rows = v.row_off[big + 1] - v.row_off[big];
        // events per tile x pixel tile (waves of 64 emission pixels per
        // workgroup: 1, 2, 4 and the context's own choice, at most the
        // emission set's waves)
        std::vector<int> waves_opts;
        for (int w : {1, 2, 4, g.fwd_waves})
            if (w >= 1 && w <= std::min(4, g.n_qpad / 64) &&
                std::find(waves_opts.begin(), waves_opts.end(), w) == waves_opts.end())
                waves_opts.push_back(w);
        // every candidate is timed in a sweep; a second sweep follows when the
        // first took under 300 ms, each candidate keeping its faster time, so
        // that clocks still rising during the first sweep do not favour the
        // candidates timed last
        float best = 3.4e38f;
        std::vector<float> cand_ms;
        float sweep_ms = 0.0f;
        for (int sweep = 0; sweep < 2 && !c->surrogate && e == hipSuccess; ++sweep) {
            if (sweep == 1 && sweep_ms >= 300.0f) break;
            size_t ci = 0;
            for (int ev : {8, 16, 32}) {
                if (e != hipSuccess) break;
                if ((e = plan_tiles(g, c->t, v, ev, v.chunk_rows, c->st, why)) != hipSuccess) break;
                for (int w : waves_opts) {
                    v.fwd_waves = w;
                    lmosem_status ws = alloc_workspace(c, s);
                    if (ws != LMOSEM_OK) return ws;
                    const Geo gw = set_geo(c, s);
                    float ms = 0.0f;
                    e = time_ms(c, [&] {
                        return launch_forward(ev, gw, c->t, v.tiles + v.tile_off[big],
                                              v.tile_off[big + 1] - v.tile_off[big], v.u, v.e, v.efac, s->f, s->H,
                                              s->pmean, v.row_off[big], rows, c->st);
                    }, ms);
                    if (e != hipSuccess) break;
                    sweep_ms += 4.0f * ms;   // warm-up and timed runs
                    if (sweep == 0) cand_ms.push_back(ms);
                    else cand_ms[ci] = std::min(cand_ms[ci], ms);
                    if (cand_ms[ci] < best) { best = cand_ms[ci]; best_ev = ev; best_waves = w; }
                    ++ci;
                }
            }
        }
        if (!c->surrogate) v.fwd_waves = best_waves;
        fwd_ms = best < 3.4e38f ? best : 0.0f;
        best = 3.4e38f;
        for (int ch : {64, 128, 256, 512, 1024, 2048, 4096}) {
            if (e != hipSuccess) break;
            if ((e = plan_tiles(g, c->t, v, best_ev, ch, c->st, why)) != hipSuccess) break;
            lmosem_status ws = alloc_workspace(c, s);
            if (ws != LMOSEM_OK) return ws;
            // the backprojection together with the update that adds its chunk
            // partials (more chunks: a faster backprojection, a longer update),
            // five times over (on the set's scratch image)
            float ms = 0.0f;
            e = time_ms(c, [&] {
                hipError_t r = hipSuccess;
                for (int k = 0; k < 5 && r == hipSuccess; ++k) {
                    r = launch_backproject(g, v.chunks + v.chunk_off[big], v.chunk_off[big + 1] - v.chunk_off[big],
                                           s->H, s->inv, s->pb, c->st);
                    if (r == hipSuccess)
                        r = launch_update(g, v.crange + (size_t)big * (v.n_real + 1), v.n_real, s->pb,
                                          c->t.sens + (size_t)big * g.n_qpad, s->f, c->st);
                }
                return r;
            }, ms);
            if (e == hipSuccess && ms < best) { best = ms; best_ch = ch; }
        }
    }
    if (e == hipSuccess) e = plan_tiles(g, c->t, v, best_ev, best_ch, c->st, why);
    if (e != hipSuccess) return dev_err(c, "autotune", e);
    lmosem_status ws = alloc_workspace(c, s);
    if (ws != LMOSEM_OK) return ws;
    drop_graphs(s);
    if (c->surrogate) best_graph = 0;
    // an iteration of more than about 50 ms hides its few dozen launches
    // either way: replay it without timing both (which would cost four
    // iterations)
    if (best_graph < 0 && fwd_ms * g.n_subsets > 50.0f) {
        best_graph = 1;
        tune_store(key, best_ev, best_ch, best_graph, v.fwd_waves);
    }
    if (best_graph < 0) {
        // one full iteration launched directly versus replayed as a graph
        // (on a scratch image: the caller's images are gathered at the next
        // lmosem_iterate)
        float ms_direct = 0.0f, ms_graph = 0.0f;
        e = launch_fill(s->f, (size_t)v.n_real * g.n_qpad, 1.0f, c->st);
        s->use_graph = 0;
        if (e == hipSuccess) e = time_ms(c, [&] { return one_iteration(c, s, false); }, ms_direct);
        s->use_graph = 1;
        if (e == hipSuccess) e = time_ms(c, [&] { return one_iteration(c, s, false); }, ms_graph);
        if (e != hipSuccess) return dev_err(c, "autotune", e);
        best_graph = ms_graph < ms_direct ? 1 : 0;
        tune_store(key, best_ev, best_ch, best_graph, v.fwd_waves);
    }
    s->use_graph = best_graph;
    if (event_tile) *event_tile = best_ev;
    if (chunk_rows) *chunk_rows = best_ch;
    if (use_graphs) *use_graphs = best_graph;
    return LMOSEM_OK;
}

lmosem_status lmosem_evset_plan(const lmosem_evset *s, int32_t *out4) {
    if (!s || !out4) return LMOSEM_EINVAL;
    const lmosem_ctx *c = s->s.ctx;
    out4[0] = s->s.ev_tile;
    out4[1] = s->s.fwd_waves > 0 ? s->s.fwd_waves : c->g.fwd_waves;
    out4[2] = s->s.chunk_rows;
    out4[3] = s->use_graph >= 0 ? s->use_graph : (c->graphs ? 1 : 0);
    return LMOSEM_OK;
}

lmosem_status lmosem_get_stats(const lmosem_ctx *c, lmosem_stats *out) {
    if (!c || !out) return LMOSEM_EINVAL;
    if (c->poisoned) return LMOSEM_ESTATE;
    unsigned long long sk = 0;
    hipError_t e = hipMemcpyAsync(&sk, c->skipped_dev, sizeof sk, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e == hipSuccess) e = drain_timing(const_cast<lmosem_ctx *>(c));
    if (e != hipSuccess) return LMOSEM_EDEVICE;
    out->n_support = c->g.n_p;
    out->n_emission = c->g.n_q;
    out->skipped_events = (int64_t)sk;
    out->inner_terms = c->terms;
    out->useful_terms = c->useful;
    out->table_ms = c->table_ms;
    out->table_bytes = c->table_bytes;
    out->event_tile = c->ev_tile;

    out->forward_launches = c->launches[0];
    out->forward_ms = c->ms[0];
    out->backproject_launches = c->launches[1];
    out->backproject_ms = c->ms[1];
    out->update_launches = c->launches[2];
    out->update_ms = c->ms[2];
    out->network_launches = c->launches[3];
    out->network_ms = c->ms[3];
    out->network_pairs = c->net_pairs;
    return LMOSEM_OK;
}

lmosem_status lmosem_set_timing(lmosem_ctx *c, int32_t enable) {
    GUARD(c);
    hipError_t e = drain_timing(c);
    if (e != hipSuccess) return dev_err(c, "timing", e);
    c->timing = enable != 0;
    if (c->timing) {
        for (int k = 0; k < 4; ++k) { c->launches[k] = 0; c->ms[k] = 0.0; }
        c->net_pairs = 0;
    }
    return LMOSEM_OK;
}

lmosem_status lmosem_measure_alu_rates(void *hip_stream, double *out3) {
    if (!out3) return LMOSEM_EINVAL;
    hipError_t e = measure_alu_rates((hipStream_t)hip_stream, out3);
    return e == hipSuccess ? LMOSEM_OK : LMOSEM_EDEVICE;
}

}  // extern "C"
