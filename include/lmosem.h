/*
 * lmosem.h — C ABI of the MI355X (gfx950) list-mode OSEM reconstruction with
 * attenuation and first-order scatter compensation for 2-D SPECT
 * (Rahman, Laforest, Jha, ISBI 2020).
 *
 * The problem (Sec. 2.1): from list-mode events A_j = (detector angle,
 * position, energy), an attenuation map mu from CT and the acquisition time T,
 * estimate the activity f by maximising the list-mode likelihood (Eq. 1-3),
 * where each event's density is a mixture over photon paths (Eq. 2) weighted
 * by f at the path's start pixel times the path sensitivity s_eff (Eq. 4).
 * The estimate is computed with ordered-subsets list-mode EM (Eq. 7-9):
 * subsets by detector angle, each sub-iteration starting from the previous
 * one's estimate.
 *
 * Paths: the primary path q -> detector and the first-order in-plane scatter
 * paths q -> s -> detector through every pixel s with mu(s) > 0 (Sec. 2.2).
 * Path weights: attenuation by exact line integrals through mu, Compton
 * energy loss and Klein-Nishina angular weight at the scatter point,
 * Compton-only energy scaling of mu after the scatter, an ideal parallel-hole
 * collimator, a truncated Gaussian position response of FWHM fwhm_u_cm and a
 * Gaussian energy response of FWHM fwhm_e_kev evaluated at each event's
 * recorded energy.
 *
 * Conventions
 *   image      float32, row-major [ny][nx], pixel (i, j) centred at
 *              ((i - (nx-1)/2) pixel_cm, (j - (ny-1)/2) pixel_cm).  Activity is
 *              estimated on the emission set: the mu > 0 support, or the part
 *              of it a mask selects (lmosem_create_emission); outputs are 0
 *              elsewhere and inputs are ignored there.
 *   angle      theta_a = angle0_rad + 2 pi a / n_angles, a in [0, n_angles);
 *              photons reach the detector travelling along (cos, sin) theta_a.
 *   position   u_bin in [0, n_bins): u = (u_bin - n_bins/2) bin_cm along
 *              the detector axis (-sin, cos) theta_a.
 *   subsets    subset i = { a : a mod n_subsets == i }, visited i = 0, 1, ...
 *
 * Memory and streams
 *   Every array argument is a device pointer owned by the caller (for
 *   example a torch tensor's data_ptr()), except those named *_host.  The
 *   library keeps no caller pointer beyond a call.  All work is enqueued on
 *   the HIP stream given to lmosem_create; calls return once the work is
 *   enqueued, except those that validate inputs or write host memory, which
 *   synchronise that stream.  A context is not thread-safe; separate
 *   contexts are independent.  The context owns its device tables and frees
 *   them in lmosem_destroy.
 *
 * Errors
 *   Every call returns a status and never throws.  LMOSEM_EINVAL and
 *   LMOSEM_ERANGE leave the context usable.  LMOSEM_EDEVICE (a failed HIP
 *   call) poisons it: later calls return LMOSEM_ESTATE.  lmosem_last_error
 *   returns a message for the last failure.
 */
#ifndef LMOSEM_H
#define LMOSEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LMOSEM_ABI_VERSION 2u

typedef enum {
    LMOSEM_OK = 0,
    LMOSEM_EINVAL = -1,   /* bad argument or configuration */
    LMOSEM_ERANGE = -2,   /* input values outside their valid range */
    LMOSEM_ENOMEM = -3,   /* device allocation failed, or would exceed the context's
                             memory cap (lmosem_set_memory_cap) */
    LMOSEM_EDEVICE = -4,  /* a HIP call failed; the context is poisoned */
    LMOSEM_ESTATE = -5,   /* context poisoned by an earlier device error */
    LMOSEM_ENOTSUP = -6   /* valid but not supported by this library */
} lmosem_status;

typedef struct lmosem_ctx lmosem_ctx;
typedef struct lmosem_evset lmosem_evset;
typedef struct lmosem_net lmosem_net;

/* Geometry and physics of one acquisition (all units explicit). */
typedef struct {
    uint32_t abi_version;     /* must equal LMOSEM_ABI_VERSION */
    int32_t nx, ny;           /* image grid */
    double pixel_cm;          /* pixel pitch */
    int32_t n_bins;           /* detector bins; detector length n_bins * bin_cm */
    double bin_cm;
    int32_t n_angles;         /* detector angles over 360 degrees */
    double angle0_rad;
    double e0_kev;            /* photopeak energy */
    double fwhm_e_kev;        /* energy resolution (constant FWHM) */
    double fwhm_u_cm;         /* intrinsic position resolution (FWHM) */
    double win_lo_kev;        /* accepted energies [win_lo, win_hi]: photopeak */
    double win_hi_kev;        /*   and scatter windows together */
    int32_t n_subsets;        /* 1 .. n_angles */
    int32_t scatter_model;    /* 0: primary paths only; 1: primary + first-order scatter;
                                 2: primary + learned first-order scatter (needs a network,
                                 lmosem_set_surrogate; only the near-field band of the
                                 path table is stored) */
    double acq_time;          /* T (> 0) */
} lmosem_config;

/* List-mode events, structure of arrays, device pointers, n >= 0. */
typedef struct {
    int64_t n;
    const int32_t *angle;     /* [n] detector angle index */
    const float *u_bin;       /* [n] position in detector bins, [0, n_bins) */
    const float *energy_kev;  /* [n] recorded energy, within [win_lo, win_hi] */
} lmosem_events;

/* Several independent realisations concatenated in one event array:
 * realisation r holds events offsets[r] .. offsets[r+1]-1.  Host pointer,
 * offsets[0] == 0, non-decreasing, offsets[n_real] == events.n. */
typedef struct {
    int32_t n_real;
    const int64_t *offsets;
} lmosem_batch;

/* Per-context counters, filled by lmosem_get_stats. */
typedef struct {
    int64_t n_support;          /* pixels with mu > 0 (path ends and scatter points) */
    int64_t skipped_events;     /* events whose model mean was <= 1e-30, since create */
    int64_t inner_terms;        /* (event, emission pixel, path end) terms evaluated by
                                   the forward projection, since create */
    int64_t useful_terms;       /* of those, terms with a non-zero position response */
    double table_ms;            /* time of the table builds so far (lmosem_create, and
                                   the path tables at the first list-mode call) */
    int64_t table_bytes;        /* device bytes held by the tables built so far */
    int32_t event_tile;         /* events per forward-projection tile */
    int32_t n_emission;         /* emission pixels (the estimated image), <= n_support */
    /* kernel times from HIP events on the context's stream, recorded only
       while timing is enabled (lmosem_set_timing) */
    int64_t forward_launches;
    double forward_ms;          /* summed over forward-projection launches */
    int64_t backproject_launches;
    double backproject_ms;
    int64_t update_launches;    /* mean + update kernels of a sub-iteration */
    double update_ms;
    int64_t network_launches;   /* learned-scatter contexts: launches of the fused network */
    double network_ms;          /*   kernel, their summed time, */
    int64_t network_pairs;      /*   and the (event, pixel) pairs they evaluated */
} lmosem_stats;

/* Version of this ABI (LMOSEM_ABI_VERSION of the built library). */
uint32_t lmosem_abi_version(void);

/* Build a context for one attenuation map: validates the configuration and
 * mu (finite, >= 0, at least one pixel > 0; mu is read on the device and
 * copied once to the host) and computes the attenuation line integrals, the
 * scatter-point factors and the ranked path ends (the parts of the model of
 * s_eff in Eq. 4 that every use needs).  The first call that needs them
 * (sensitivity, forward, backprojection, updates, event sets) builds every
 * path's weight and end energy and the per-subset sensitivity images (the
 * denominators of Eq. 6/7); that call returns ENOMEM if they do not fit,
 * and the binned functions never need them.  mu_dev: [ny][nx] float32 in
 * 1/cm at e0_kev.  hip_stream: a hipStream_t, or NULL for the null stream.
 * Errors: EINVAL (config), ERANGE (mu), ENOMEM, EDEVICE. */
lmosem_status lmosem_create(const lmosem_config *cfg, const float *mu_dev, void *hip_stream,
                            lmosem_ctx **out);

/* As lmosem_create, with the estimated image restricted to an emission set
 * (Sec. 2.2: the work of every iteration scales with the number of non-zero
 * pixels, so the initial estimate is confined to a crude object boundary,
 * e.g. from a binned OS-MLEM).  emission_dev: [ny][nx] float32, device,
 * nullable; the emission set is {mu > 0 and emission > 0} (NULL: mu > 0).
 * Scatter points and path ends stay the whole mu > 0 support, so the model
 * of the remaining emission pixels is unchanged.  Images written by the
 * context are 0 outside the emission set; images read by it are read only
 * on it.  Errors: as lmosem_create; ERANGE also for an empty emission set. */
lmosem_status lmosem_create_emission(const lmosem_config *cfg, const float *mu_dev, const float *emission_dev,
                                     void *hip_stream, lmosem_ctx **out);

/* Free the context and everything it owns (NULL is a no-op). */
void lmosem_destroy(lmosem_ctx *ctx);

/* Message describing the last failure on this context ("" if none). */
const char *lmosem_last_error(const lmosem_ctx *ctx);

/* Sensitivity image T * sum_{paths P_q reaching the subset's angles} s_eff(P_q)
 * (denominator of Eq. 7) into sens_dev [ny][nx]; subset -1 sums all angles
 * (denominator of Eq. 6).  Errors: EINVAL (subset out of range). */
lmosem_status lmosem_sensitivity(lmosem_ctx *ctx, int32_t subset, float *sens_dev);

/* Per-event means for a given image: mean_j = sum_q f_q h(q; A_j), the
 * denominator of Eq. 8 (the path mixture of Eq. 2 without the normaliser of
 * Eq. 4, which cancels).  image_dev [ny][nx], event_mean_dev [ev->n], in the
 * caller's event order.  Validates the events (synchronises).
 * Errors: EINVAL, ERANGE (events out of range), ENOMEM. */
lmosem_status lmosem_forward(lmosem_ctx *ctx, const lmosem_events *ev, const float *image_dev,
                             float *event_mean_dev);

/* lmosem_forward for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc): the same per-event means,
 * bit for bit, with every buffer of the call (the estimate on the emission
 * set, the sorted events and their tile plan, the sort's temporary storage,
 * the system rows of one chunk of tiles at a time) carved from one
 * file-scope device array of 64 MiB that the library holds on each GPU it
 * runs on until the process ends.  No hipMalloc or hipFree, no allocating
 * library routine.  Every call on a GPU shares that array (whatever its
 * context), so calls that overlap on one GPU race; each call clears what
 * must start at zero.  Needs the context's path tables (built by its first
 * list-mode call, e.g. lmosem_sensitivity) and the exact path
 * (scatter_model 0 or 1).  Validates the events and synchronises.
 * Errors: EINVAL (arguments, or tables not built yet), ENOMEM (the events
 * need more than the array holds: about 60 bytes per event plus a chunk of
 * at least one tile of rows; roughly 1M events), ENOTSUP (scatter_model 2),
 * ERANGE (events out of range). */
lmosem_status lmosem_forward_noalloc(lmosem_ctx *ctx, const lmosem_events *ev, const float *image_dev,
                                     float *event_mean_dev);

/* Weighted backprojection b_q = sum_j h(q; A_j) w_j into image_dev [ny][nx]
 * (with w_j = 1/mean_j this is the numerator of Eq. 7 divided by f_q).
 * weights_dev [ev->n].  Validates the events (synchronises). */
lmosem_status lmosem_backproject(lmosem_ctx *ctx, const lmosem_events *ev,
                                 const float *weights_dev, float *image_dev);

/* One sub-iteration of Eq. 7 for subset `subset`: every given event is
 * taken as a member of that subset (the caller passes the events detected
 * at the subset's angles).  image_dev [ny][nx] is updated in place:
 * f_q <- f_q * (sum_j h(q; A_j) / mean_j) / sens_q^(subset); pixels with zero
 * sensitivity keep their value and events with mean <= 1e-30 are skipped
 * and counted.  event_mean_dev (nullable, [ev->n]) receives the means at the
 * input image.  Membership is checked only when the environment variable
 * LMOSEM_VALIDATE=1 (then the call synchronises).  Errors: EINVAL, ERANGE. */
lmosem_status lmosem_subset_update(lmosem_ctx *ctx, int32_t subset, const lmosem_events *ev,
                                   float *image_dev, float *event_mean_dev);

/* Full OS-LM-MLEM (Eq. 7-9): n_iters global iterations over all subsets in
 * order, for one realisation (batch NULL) or several independent ones.
 * init_dev (nullable: 1 on the emission set) is [ny][nx], shared by all
 * realisations; images_dev [n_real][ny][nx] receives the estimates.
 * loglik_host (nullable) [n_real][n_iters] receives, per global iteration,
 * sum_i (sum_{j in S_i} log mean_j - sum_q f_q sens_q^(i)) at the estimate
 * each sub-iteration starts from (for one subset: Eq. 3 up to constants at
 * the iteration's starting estimate).  Validates events and init
 * (synchronises).  Errors: EINVAL, ERANGE, ENOMEM. */
lmosem_status lmosem_reconstruct(lmosem_ctx *ctx, const lmosem_events *ev,
                                 const lmosem_batch *batch, int32_t n_iters,
                                 const float *init_dev, float *images_dev, double *loglik_host);

/* Prepared event sets: validate once, sort by (subset, realisation, angle,
 * position) and plan the forward-projection tiles, so that repeated
 * iterations pay nothing for ingest.  The set keeps device copies and is
 * tied to its context; free it before the context. */
lmosem_status lmosem_events_load(lmosem_ctx *ctx, const lmosem_events *ev,
                                 const lmosem_batch *batch, lmosem_evset **out);
void lmosem_events_free(lmosem_evset *set);

/* n_iters global iterations on a prepared set; images_dev [n_real][ny][nx]
 * is the starting estimate on entry and the result on return (values
 * outside the emission set are set to 0).  loglik_host as in lmosem_reconstruct
 * (nullable; if given the call synchronises). */
lmosem_status lmosem_iterate(lmosem_ctx *ctx, lmosem_evset *set, int32_t n_iters,
                             float *images_dev, double *loglik_host);

/* Tuning: events per forward tile (8, 16 or 32; 0 restores the default 8)
 * for event sets loaded afterwards.  A context starts from 8, or from
 * LMOSEM_EVENT_TILE (8, 16 or 32) when that is set in the environment at
 * creation; other values of it are ignored. */
lmosem_status lmosem_set_tuning(lmosem_ctx *ctx, int32_t event_tile);

/* Tuning: emission pixels per forward-projection workgroup (the pixel tile:
 * 64, 128, 192 or 256, one wave of 64 threads per 64 pixels; 0 restores the
 * default, the emission set's width up to 256) for event sets loaded
 * afterwards; lmosem_autotune may replace it.  Results do not depend on it
 * beyond FP32 summation order.  Errors: EINVAL. */
lmosem_status lmosem_set_pixel_tile(lmosem_ctx *ctx, int32_t pixels);

/* Autotuner: times the forward projection of the set's largest subset for
 * 8, 16 and 32 events per tile, each with pixel tiles of 64, 128 and 256
 * emission pixels per workgroup (and the context's own, when the emission
 * set is narrower), the backprojection with the update that
 * adds its chunk partials for 64-4096 rows per chunk (using the set's
 * scratch image), and one whole iteration launched kernel by kernel against one
 * replayed as a HIP graph (iterations estimated above 50 ms are replayed
 * without that comparison); re-plans the set with the fastest choices and
 * returns them (outputs may be NULL).  With LMOSEM_TUNE_CACHE=<file> in the
 * environment the choice is looked up in / appended to that file, keyed by
 * support and emission-set sizes, angles, subsets, realisations and subset size.  Results do
 * not depend on the choice beyond FP32 summation order.  Synchronises. */
lmosem_status lmosem_autotune(lmosem_ctx *ctx, lmosem_evset *set, int32_t *event_tile,
                              int32_t *chunk_rows, int32_t *use_graphs);

/* Cap on the device memory the context holds (0, the default: no cap): its
 * tables plus the workspace, sorted events and row caches of its live event
 * sets.  A call that would take the context past the cap returns
 * LMOSEM_ENOMEM and leaves the context usable: the path tables are refused
 * before they are allocated (for scatter_model 2, whose near-field band's
 * width is known only once built, they are freed again), an event set after
 * its sort is planned, a row cache before it is allocated.  Memory a call
 * uses only while it runs is not counted.  Errors: EINVAL (bytes < 0). */
lmosem_status lmosem_set_memory_cap(lmosem_ctx *ctx, int64_t bytes);
/* The device bytes the context holds as the cap counts them. */
lmosem_status lmosem_memory_held(const lmosem_ctx *ctx, int64_t *bytes);

/* Testing hook for the error path: the context's next kernel launch of a
 * list-mode call (forward projection, backprojection, update) is not made
 * and reports a failed HIP launch instead, as a device failure would; that
 * call returns LMOSEM_EDEVICE and poisons the context (every later call
 * returns LMOSEM_ESTATE; lmosem_destroy still frees it).  Nothing runs on
 * the device for the failing launch. */
lmosem_status lmosem_inject_failure(lmosem_ctx *ctx);

/* The plan a set iterates with: out4[0] events per forward tile, out4[1]
 * waves of 64 emission pixels per forward workgroup (the pixel tile),
 * out4[2] rows per backprojection chunk, out4[3] 1 if iterations replay a
 * graph.  Errors: EINVAL. */
lmosem_status lmosem_evset_plan(const lmosem_evset *set, int32_t *out4);

/* Replay each global iteration of lmosem_iterate / lmosem_reconstruct as one
 * captured HIP graph (1, the default) or launch kernel by kernel (0); an
 * autotuned event set follows its own measured choice instead.  The graph
 * runs on a stream of the context that is ordered after the caller's stream
 * on entry and before it on exit. */
lmosem_status lmosem_set_graphs(lmosem_ctx *ctx, int32_t enable);

/* Keep the system rows of a prepared set across iterations (enable = 1) or
 * stop (0).  The rows h_j(q) do not depend on the estimate (Eq. 8 divides
 * them only by the event means), so after one iteration has computed and
 * stored all of them (n events x padded emission set x 4 bytes, allocated here,
 * owned by the set, zero-filled), every later sub-iteration reads them twice
 * from HBM (the event means, then the backprojection of Eq. 7) instead of
 * recomputing every path term.  Results equal the recomputing path up to
 * FP32 summation order.  Autotuning the set, or enabling again after
 * disabling, recomputes the rows at the next iteration.  Errors: ENOMEM (the
 * set stays usable without the cache), EINVAL. */
lmosem_status lmosem_cache_rows(lmosem_ctx *ctx, lmosem_evset *set, int32_t enable);

/* ---- binned data (the binned alternative of Sec. 2.2) ----------------
 * Bins (a, b, k): detector angle a, position bin b of n_pos equal bins over
 * the detector, energy bin k = [e_edges[k], e_edges[k+1]) (the last bin
 * includes its upper edge); flat index (a * n_pos + b) * n_ebins + k.  e_edges
 * is a host array of n_ebins + 1 increasing energies (keV).  The binned
 * system row of a bin is the integral of the list-mode row h (Eq. 2, 8) over
 * the bin, from closed-form position and energy masses with every path
 * weight in FP64. */

/* counts_dev[n_angles][n_pos][n_ebins] = number of events in each bin (the
 * array is overwritten; events outside every bin are not counted). */
lmosem_status lmosem_bin_events(lmosem_ctx *ctx, const lmosem_events *ev, int32_t n_pos, const double *e_edges,
                                int32_t n_ebins, float *counts_dev);
/* rows_dev[n][ny][nx] = the binned system rows of the n bins listed in
 * bins_dev (flat indices; 0 off the emission set).  Errors: ERANGE for a bin
 * index out of range. */
lmosem_status lmosem_binned_rows(lmosem_ctx *ctx, int32_t n_pos, const double *e_edges, int32_t n_ebins, int64_t n,
                                 const int32_t *bins_dev, float *rows_dev);
/* Binned OS-MLEM (Eq. 7 with counts): subsets by detector angle as in list
 * mode; each sub-iteration f <- f * H_i^T (y_i / H_i f) / H_i^T 1 over the
 * subset's bins (bins with zero mean are left out).  counts_dev as written by
 * lmosem_bin_events; init_dev (nullable: 1 on the emission set) and image_dev are
 * [ny][nx].  Allocates its rows (n_angles * n_pos * n_ebins x padded emission set
 * floats) for the call; ENOMEM if they do not fit. */
lmosem_status lmosem_binned_reconstruct(lmosem_ctx *ctx, int32_t n_pos, const double *e_edges, int32_t n_ebins,
                                        const float *counts_dev, int32_t n_iters, const float *init_dev,
                                        float *image_dev);

/* Emission set from a crude image (Sec. 2.2: a rough object boundary from a
 * quick binned OS-MLEM keeps the number of estimated pixels small):
 *   mask[p] = 1 if mu[p] > 0 and a pixel p' within margin_px pixels of p
 *             ((di^2 + dj^2) <= margin_px^2) has
 *             image[p'] >= rel_threshold * max(image), in FP64;
 *   mask[p] = 0 otherwise.
 * mu is this context's map.  image_dev, mask_dev: [ny][nx] float32, device;
 * the mask is meant for lmosem_create_emission.  rel_threshold in [0, 1],
 * margin_px in [0, 32].  Synchronises.  Errors: EINVAL (arguments), ERANGE
 * (image values negative or not finite). */
lmosem_status lmosem_emission_mask(lmosem_ctx *ctx, const float *image_dev, double rel_threshold, int32_t margin_px,
                                   float *mask_dev);

/* Counters of this context (synchronises the context's stream). */
lmosem_status lmosem_get_stats(const lmosem_ctx *ctx, lmosem_stats *out);

/* Enable (1) or disable (0) per-kernel timing with HIP events around every
 * sub-iteration kernel; enabling also clears the accumulated times. */
lmosem_status lmosem_set_timing(lmosem_ctx *ctx, int32_t enable);

/* Diagnostic: measured vector-ALU rates of this GPU, in lane-operations per
 * second: out[0] FP32 FMA, out[1] FP32 exp2 (v_exp_f32), out[2] the mix of
 * two FMAs and one exp2 that the forward projection issues per term (in
 * terms per second).  Runs short probe kernels on hip_stream (synchronises). */
lmosem_status lmosem_measure_alu_rates(void *hip_stream, double *out3);

/* ---- learned scatter surrogate -------------------------------------
 * Not part of the paper: a network S_net(x) stands in for the first-order
 * scatter part of each system row, S(q; a, u, E) = sum_{s != q} s_eff-weighted
 * K G terms (Sec. 2.2), one evaluation per (event, emission pixel), for the
 * pairs whose event lies outside q's own position response
 * (|u - u_q| >= 3 sigma_u).  Inside it (the near field) the scatter sum is
 * exact, from a table of the path ends within 6 sigma_u of u_q, and the
 * primary term is always exact.  Network: 8 -> 128 -> 128 -> 128 -> 1, GELU
 * (tanh form), bf16 weights and activations with FP32 accumulation on MFMA,
 * FP32 master weights, Adam.  Inputs x (8 floats per pair: offset from q's
 * detector position, energy, where the event's detector line enters and
 * leaves the body relative to q's depth, that line's response-weighted
 * attenuation, attenuation from q toward and away from the detector, mu at
 * q) and the target y = ln(S / S0 + 1e-4), S0 = 1 / (pixel_cm * sigma_E), are
 * produced by lmosem_surrogate_samples.  Parameters are passed flat (34305
 * floats): W1[8][128] b1[128] W2[128][128] b2[128] W3[128][128] b3[128]
 * W4[128] b4, W[in][out].  A context runs the network on its own stream: do
 * not train a network while a context iterates with it. */

/* New network from host parameters; its kernels run on hip_stream (the
 * weights are ready on every stream when this returns). */
lmosem_status lmosem_net_create(const float *params_host, void *hip_stream, lmosem_net **out);
void lmosem_net_destroy(lmosem_net *net);
/* Current FP32 master parameters into params_host[34305] (synchronises). */
lmosem_status lmosem_net_get_params(lmosem_net *net, float *params_host);
/* y_dev[n] = network(X_dev[n][8]), on the network's stream; one fused kernel
 * (all four layers, weights in LDS) with bf16 inputs, weights and
 * activations and FP32 accumulation, as in training; its GELU's sigmoid
 * factor is a polynomial evaluated in fp16 arithmetic (within 2e-3 of the
 * tanh form), the activation rounded to bf16.  The learned-scatter rows use
 * the same kernel. */
lmosem_status lmosem_net_forward(lmosem_net *net, const float *X_dev, int64_t n, float *y_dev);
/* y_dev[n] from the training kernels' forward pass (bf16 inputs, weights and
 * activations, FP32 accumulation): the outputs that lmosem_net_train's loss
 * and lmosem_net_gradient's linearisation use; n a positive multiple of 16,
 * on the network's stream.  Errors: EINVAL, EDEVICE. */
lmosem_status lmosem_net_forward_train(lmosem_net *net, const float *X_dev, int32_t n, float *y_dev);
/* Gradient of sum_i dy_dev[i] y_i over all parameters into grad_host[34305];
 * n a positive multiple of 16 (synchronises). */
lmosem_status lmosem_net_gradient(lmosem_net *net, const float *X_dev, const float *dy_dev, int32_t n,
                                  float *grad_host);
/* Adam (beta 0.9 / 0.999, eps 1e-8) on the mean-squared error over
 * minibatches of `batch` samples taken in order (the caller shuffles);
 * lr is multiplied by lr_decay after each epoch; loss_host (nullable)
 * receives each epoch's mean loss. */
lmosem_status lmosem_net_train(lmosem_net *net, const float *X_dev, const float *t_dev, int64_t n, int32_t batch,
                               int32_t epochs, float lr, float lr_decay, double *loss_host);
/* Training samples on a scatter_model-1 or -2 context: for each (emission
 * pixel, angle, u_bin, energy) the network inputs X_dev[n][8], the target
 * target_dev[n] and (nullable) the exact first-order scatter sum
 * scatter_dev[n] (Sec. 2.2), every path weight evaluated in FP64 from the
 * context's line integrals and scatter-point factors (no full path table is
 * needed; any u is accepted, the network is meant for the far field).
 * Errors: ENOTSUP for scatter_model 0, ERANGE for a pixel off the emission set or
 * an invalid angle, position or energy. */
lmosem_status lmosem_surrogate_samples(lmosem_ctx *ctx, const int32_t *pixel, const int32_t *angle,
                                       const float *u_bin, const float *energy, int64_t n, float *X_dev,
                                       float *target_dev, float *scatter_dev);
/* Use `net` (not owned; keep it alive) for the scatter term of a
 * scatter_model-2 context. */
lmosem_status lmosem_set_surrogate(lmosem_ctx *ctx, lmosem_net *net);

#ifdef __cplusplus
}
#endif

#endif /* LMOSEM_H */
