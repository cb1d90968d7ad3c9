// Internal declarations of the gfx950 list-mode OSEM library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/lmosem.h"

namespace lmo {

constexpr double kMeC2 = 510.99895;     // electron rest energy, keV
constexpr float kNegHuge = -1.0e30f;     // log2 weight of a path that never contributes
constexpr int kRankPad = 8;              // padding rank rows per angle (never contribute)

// Geometry and physics constants shared by the kernels (host-computed, FP64).
struct Geo {
    int nx, ny, n_pix;
    int n_p;          // support pixels (mu > 0): the path ends and scatter points
    int n_q;          // emission pixels: support indices 0 .. n_q-1 (the support is
                      // ordered with the emission pixels first)
    int n_qpad;       // n_q rounded up to a multiple of 64 (row stride of H and the table)
    int n_rpad;       // rank rows per angle in the path table: n_p + kRankPad
    int fwd_waves;    // waves (64 emission pixels each) per forward-projection workgroup
    int n_angles, n_bins, n_subsets, scatter;
    double dx, bin_cm, half_len;
    double e0, kappa, sig_e, sig_u, win_lo, win_hi;
    double psi_bar;       // circle mean of the Klein-Nishina shape at e0
    double sigma_kn_e0;   // Klein-Nishina total cross-section at e0 (units r_e^2)
    double zk;            // normaliser of the truncated position response
    double e_c;           // energy centre for the table encoding
    double c2;            // log2(e) / (2 sig_e^2)
    double acq_time;
};

// One forward-projection tile: up to EV consecutive events of one
// (subset, realisation, angle) group sorted by detector position, and the
// rank range of path ends (sorted by detector position at that angle) whose
// position response can reach any of them.
struct Tile {
    int e0;      // first event (index into the sorted event arrays)
    int n;       // events in the tile
    int angle;
    int real;    // realisation
    int r0, r1;  // path-end rank range [r0, r1)
};

// Backprojection chunk: rows [j0, j1) of one realisation within a sub-iteration.
struct Chunk {
    int j0, j1;  // rows relative to the sub-iteration's first row
    int real;
    int pad;
};

// Device tables of one context.
struct Tables {
    int *p_pix = nullptr;        // [n_p] support pixel index
    float *mu = nullptr;         // [n_pix]
    double *cs = nullptr;        // [n_angles][2] cos, sin of theta_a
    int *s_sorted = nullptr;     // [n_angles][n_p] path-end support index by rank
    double *us_sorted = nullptr; // [n_angles][n_p] detector position of each rank (cm)
    float *mu_sorted = nullptr;  // [n_angles][n_p] mu at each rank's pixel
    float2 *T = nullptr;         // [n_angles][n_rpad][n_qpad] (alpha, beta) per path
    float *sens = nullptr;       // [n_subsets][n_qpad]
    float *sens_all = nullptr;   // [n_qpad]
    float *Ldet = nullptr;       // [n_angles][n_p] attenuation from the pixel centre to the detector
    float *Lback = nullptr;      // [n_angles][n_p] attenuation from the pixel centre away from it
    float *prim = nullptr;       // [n_angles][n_p] alpha of each pixel's primary path
    // per-angle line integrals (every context) and scatter-point factors
    // (scatter contexts), kept for path weights evaluated on the fly
    // (training targets, binned rows)
    double *Ld = nullptr;        // [n_angles][n_p] L_a(p)
    double *Bt = nullptr;        // [n_p][n_p] B(q, s) at [s][q]
    double *D_sorted = nullptr;  // [n_angles][n_p] detector mass of each rank's position response
    // learned-scatter contexts: exact near-field paths of each emission pixel
    float2 *band = nullptr;      // [n_angles][n_qpad][band_w] (alpha, beta), rank band_lo + k
    int *band_lo = nullptr;      // [n_angles][n_p] first rank of each pixel's band
    int band_w = 0;              // longest band
};

// ---- table build (tables.hip) ----
// build_base at create; build_paths before the first list-mode use
hipError_t build_base(const Geo &g, Tables &t, hipStream_t st, std::string &err, int64_t &bytes);
hipError_t build_paths(const Geo &g, Tables &t, bool store_paths, bool store_band, hipStream_t st,
                       std::string &err, int64_t &bytes);

// ---- event ingest (events.hip) ----
struct EvSet;
hipError_t validate_events(const Geo &g, const lmosem_events &ev, int64_t *bad_host, int *bad_dev,
                           hipStream_t st);
hipError_t sort_events(const Geo &g, const Tables &t, const lmosem_events &ev,
                       const std::vector<int64_t> &offs, int force_subset, EvSet &set,
                       hipStream_t st, std::string &err);
hipError_t plan_tiles(const Geo &g, const Tables &t, EvSet &set, int ev_tile, int chunk_rows,
                      hipStream_t st, std::string &err);
// the steps of the ingest on buffers the caller provides (no allocation)
hipError_t launch_event_keys(const Geo &g, int64_t n, int n_real, const int64_t *offs_dev, const int32_t *angle,
                             const float *u_bin, int force_subset, uint64_t *keys, int *idx, hipStream_t st);
hipError_t launch_gather_events(const Geo &g, int64_t n, const uint64_t *keys, const int *idx, const lmosem_events &ev,
                                int *sa, float *su, float *se, float *efac, int *orig, int *counts, hipStream_t st);
hipError_t launch_tile_ranks(const Geo &g, Tile *tiles, int n_tiles, const double *us_sorted, const float *su,
                             long long *terms, long long *useful, hipStream_t st);
int sort_key_bits(int n_groups);
hipError_t sort_pairs_bytes(int64_t n, int n_groups, size_t &bytes);   // temporary storage of sort_pairs
hipError_t sort_pairs(void *tmp, size_t tmp_bytes, const uint64_t *keys, uint64_t *keys2, const int *idx, int *idx2,
                      int64_t n, int n_groups, hipStream_t st);
// tiles of ev_tile consecutive events per angle of one sorted, single-subset,
// single-realisation event set with counts[a] events at angle a
void host_tiles(const Geo &g, const std::vector<int> &counts, int n_angles_used, int ev_tile, std::vector<Tile> &tiles);

// ---- forward projection without allocation (noalloc.hip) ----
// Bytes of the library's file-scope device scratch array, and its address on
// the current device (looked up once per device).
extern const size_t kScratchBytes;
hipError_t scratch_address(void **ptr);
// bytes of the scratch array that forward_noalloc needs for n events
hipError_t forward_noalloc_bytes(const Geo &g, int64_t n, int ev_tile, size_t &need);
// per-event means of the (validated) events at the image, in the caller's
// event order, every buffer in the scratch array; synchronises st
hipError_t forward_noalloc(const Geo &g, const Tables &t, const lmosem_events &ev, int ev_tile, const float *image,
                           float *mean_out, unsigned long long *skipped, hipStream_t st, int64_t &terms,
                           int64_t &useful);

// ---- binned data (binned.hip) ----
hipError_t launch_binned_rows(const Geo &g, const Tables &t, int n_pos, const double *edges_dev, int n_e,
                              const int *row_bin_dev, int n_rows, float *H, hipStream_t st);
hipError_t launch_image_max(const float *img, int n, float *out, hipStream_t st);
hipError_t launch_emission_mask(const Geo &g, const float *mu, const float *img, double thr, int margin, float *mask,
                                hipStream_t st);
hipError_t launch_binned_rows_all(const Geo &g, const Tables &t, int n_pos, const double *edges_dev, int n_e,
                                  const int *angle_row0_dev, float *H, hipStream_t st);
hipError_t launch_bin_events(const Geo &g, const lmosem_events &ev, int n_pos, const double *edges_dev, int n_e,
                             float *counts, hipStream_t st);
hipError_t launch_gather_counts(const float *counts, const int *row_bin, int n_rows, float *y, hipStream_t st);
hipError_t launch_count_weights(const float *y, const float *inv, int n_rows, float *w, hipStream_t st);

// ---- per sub-iteration kernels (osem.hip) ----
// Events a launch function records at its kernel's start and end (HIP's
// launch with events: the timestamps bracket the kernel itself, not the
// queue work around it); a launch function that launches nothing records
// both at once.
struct KernelEvents {
    hipEvent_t start, stop;
};
__host__ __device__ int forward_groups(const Geo &g);
hipError_t launch_forward(int ev_tile, const Geo &g, const Tables &t, const Tile *tiles, int n_tiles,
                          const float *ev_u, const float *ev_e, const float *efac, const float *f, float *H,
                          float *pmean, int row_base, int n_rows, hipStream_t st, const KernelEvents *ke = nullptr);
hipError_t launch_mean(const float *pmean, int n_groups, int n_rows, float *mean, float *inv,
                       unsigned long long *skipped, hipStream_t st);
hipError_t launch_row_dot(const Geo &g, const int *rrange, int n_real, int n_rows, const float *H, const float *f,
                          float *mean, float *inv, unsigned long long *skipped, hipStream_t st,
                          const KernelEvents *ke = nullptr);
hipError_t launch_backproject(const Geo &g, const Chunk *chunks, int n_chunks, const float *H,
                              const float *inv, float *pb, hipStream_t st, const KernelEvents *ke = nullptr);
// rows per backprojection chunk at most when the means are formed in the
// backprojection (the autotuner's largest chunk)
constexpr int kMaxChunkRows = 1024;
// the event means and their inverses from the forward's pixel-group partials
// (as launch_mean) and the backprojection, in one kernel; chunk_rows is the
// plan's chunk size (at most kMaxChunkRows, else hipErrorInvalidValue)
hipError_t launch_backproject_means(const Geo &g, const Chunk *chunks, int n_chunks, int chunk_rows,
                                    const float *H, const float *pmean, int n_groups, int n_rows, float *mean,
                                    float *inv, unsigned long long *skipped, float *pb, hipStream_t st,
                                    const KernelEvents *ke = nullptr);
hipError_t launch_update(const Geo &g, const int *crange, int n_real, const float *pb,
                         const float *sens, float *f, hipStream_t st);
hipError_t launch_loglik(const Geo &g, const int *rrange, int n_real, const float *mean,
                         const float *f, const float *sens, double *ll, hipStream_t st);
hipError_t launch_sum_real(const Geo &g, const int *crange, int n_real, const float *pb,
                           float *out, hipStream_t st);
hipError_t launch_gather_image(const Geo &g, const Tables &t, const float *img, int n_real,
                               int64_t img_stride, float *f, int ones_if_null, hipStream_t st);
hipError_t launch_scatter_image(const Geo &g, const Tables &t, const float *f, int n_real,
                                float *img, hipStream_t st);
hipError_t launch_scatter_rows(const float *src, const int *orig, int n, float *dst,
                               hipStream_t st);
hipError_t launch_gather_rows(const float *src, const int *orig, int n, float *dst,
                              hipStream_t st);
hipError_t launch_fill(float *p, size_t n, float v, hipStream_t st);
hipError_t launch_fill_d(double *p, size_t n, double v, hipStream_t st);
hipError_t launch_check_image(const Geo &g, const Tables &t, const float *img, int *bad,
                              hipStream_t st);

// ---- surrogate network (mlp.hip) and its use (surrogate.hip) ----
struct Net;
extern const int kNetParams;
hipError_t net_create(const float *params_host, hipStream_t st, Net **out);
void net_destroy(Net *n);
hipStream_t net_stream(const Net *n);   // the stream the network was created on
hipError_t net_get_params(Net *n, float *host);
hipError_t net_forward(Net *n, const float *X, int64_t count, float *y, hipStream_t st);
// the packed weights of the fused inference kernel (mlp_infer.h)
void net_fused_weights(const Net *n, const uint16_t **fw, const float **fb);
hipError_t net_gradient(Net *n, const float *X, const float *dy, int count, float *grad_host);
hipError_t net_forward_train(Net *n, const float *X, int count, float *y);
hipError_t net_train(Net *n, const float *X, const float *t, int64_t count, int batch, int epochs, float lr,
                     float lr_decay, double *loss_host);
hipError_t gemm_nt(const uint16_t *A, int lda, const uint16_t *Bt, int ldb, float *C, int ldc, int M, int N,
                   int K, bool accumulate, hipStream_t st, float *split_ws = nullptr);
hipError_t surrogate_samples(const Geo &g, const Tables &t, const int32_t *pixel, const int32_t *angle,
                             const float *u_bin, const float *energy, int64_t n, float *X, float *target,
                             float *scatter, hipStream_t st);
// wraps one launch (per-kernel timing); the argument enqueues it
using LaunchWrap = std::function<hipError_t(const std::function<hipError_t()> &)>;
hipError_t surrogate_rows(const Geo &g, const Tables &t, Net *net, const int *ev_angle, const float *su,
                          const float *se, const float *efac, const float *f, const int *rrange, int n_real,
                          int row_base, int rows, float *H, float *pmean, float *col, uint16_t *X,
                          int64_t pair_cap, hipStream_t st, const LaunchWrap *wrap_net = nullptr);

// ---- ALU rate probes (probe.hip) ----
hipError_t measure_alu_rates(hipStream_t st, double *out3);

// A prepared, sorted event set.
struct EvSet {
    lmosem_ctx *ctx = nullptr;
    int n_real = 0;
    int64_t n = 0;
    int ev_tile = 8;
    int fwd_waves = 0;      // waves per forward workgroup (the pixel tile, 64 pixels each); 0: the context's
    int chunk_rows = 256;   // rows per backprojection chunk
    std::vector<int> counts;   // events per (subset, realisation, angle) group
    // sorted SoA
    int *ang = nullptr;      // detector angle
    float *u = nullptr;      // detector position, cm
    float *e = nullptr;      // energy minus the encoding centre, keV
    float *efac = nullptr;   // 2^(-c2 e^2) / Z_K per event
    int *orig = nullptr;     // original event index
    // per subset
    std::vector<int> row_off;               // [n_subsets+1] rows of each subset
    std::vector<int> tile_off;              // [n_subsets+1]
    std::vector<int> chunk_off;             // [n_subsets+1]
    Tile *tiles = nullptr;                  // all tiles, subset-major
    Chunk *chunks = nullptr;                // all chunks, subset-major
    int *crange = nullptr;                  // [n_subsets][n_real+1] chunk ranges per realisation
    int *rrange = nullptr;                  // [n_subsets][n_real+1] row ranges per realisation
    std::vector<int64_t> terms_sub;         // per subset: terms evaluated
    std::vector<int64_t> useful_sub;        // per subset: terms with K > 0
    int max_rows = 0, max_chunks = 0;
};

}  // namespace lmo
