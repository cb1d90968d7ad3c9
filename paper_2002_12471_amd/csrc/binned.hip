// Binned data: the binned alternative to list mode (Sec. 2.2).  Events are
// counted in bins (a, b, k): angle a, one of n_pos equal position bins over
// the detector, and energy bin [e_k, e_k+1).  The binned system row of a bin
// integrates the list-mode row over it,
//     H[(a,b,k)][q] = sum over paths from q of w * (mass of K over the
//                     position bin) * (mass of G over the energy bin),
// with every path weight in FP64 from the line integrals and scatter-point
// factors (the function the table build uses).  Binned OS-MLEM then runs on
// these rows with the kernels of the cached-row path (row means,
// backprojection of y / mean, update).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "lmosem_int.h"
#include "paths.h"

namespace lmo {

// mass of the truncated position response centred at us over [u0, u1]
__device__ inline double pos_mass(const Geo &g, double us, double u0, double u1) {
    const double s = g.sig_u;
    const double a = fmax(u0 - us, -3.0 * s), b = fmin(u1 - us, 3.0 * s);
    if (b <= a) return 0.0;
    const double gs = s * sqrt(M_PI / 2.0) * (erf(b / (M_SQRT2 * s)) - erf(a / (M_SQRT2 * s)));
    return (gs - exp(-4.5) * (b - a)) / g.zk;
}

// mass of the energy response centred at ep over [e0, e1]
__device__ inline double energy_mass(const Geo &g, double ep, double e0, double e1) {
    const double s2 = M_SQRT2 * g.sig_e;
    return 0.5 * (erf((e1 - ep) / s2) - erf((e0 - ep) / s2));
}

// H[row][q] for the bins listed in row_bin (flat id (a * n_pos + b) * n_e + k);
// one block row per bin, one thread per emission pixel; padding columns are 0.
__global__ __launch_bounds__(256) void k_binned_rows(Geo g, const int *__restrict__ p_pix,
                                                     const double *__restrict__ cs, const double *__restrict__ Ld,
                                                     const double *__restrict__ Bt, const int *__restrict__ s_sorted,
                                                     const double *__restrict__ us_sorted, int n_pos,
                                                     const double *__restrict__ edges, int n_e,
                                                     const int *__restrict__ row_bin, float *__restrict__ H) {
    const int row = blockIdx.y;
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= g.n_qpad) return;
    float *out = H + (size_t)row * g.n_qpad + q;
    if (q >= g.n_q) { *out = 0.0f; return; }
    const int bin = row_bin[row];
    const int a = bin / (n_pos * n_e), b = (bin / n_e) % n_pos, k = bin % n_e;
    const double width = 2.0 * g.half_len / n_pos;
    const double u0 = -g.half_len + b * width, u1 = u0 + width;
    const double e0 = edges[k], e1 = edges[k + 1];
    const double nx = cs[2 * a], ny = cs[2 * a + 1];
    const double *us = us_sorted + (size_t)a * g.n_p;
    const double reach = 3.0 * g.sig_u;
    int lo = 0, hi = g.n_p;   // first rank with us > u0 - reach
    while (lo < hi) { const int m = (lo + hi) >> 1; if (us[m] > u0 - reach) hi = m; else lo = m + 1; }
    double sum = 0.0;
    for (int r = lo; r < g.n_p && us[r] < u1 + reach; ++r) {
        const double pm = pos_mass(g, us[r], u0, u1);
        if (pm <= 0.0) continue;
        const PathW pw = path_weight(g, p_pix, Ld, Bt, nx, ny, a, q, s_sorted[(size_t)a * g.n_p + r]);
        if (pw.w > 0.0) sum += pw.w * pm * energy_mass(g, pw.ep, e0, e1);
    }
    *out = (float)sum;
}

// All bins of every angle at once.  A path end's position response spans at
// most W consecutive position bins, and path ends are ranked by position, so
// one thread per (angle, emission pixel) walks the ranks once, evaluating each
// path weight once (rather than once per bin that the path reaches), with W
// bins of accumulators that slide along the detector.  The position-bin
// masses depend on the rank only and come precomputed (k_rank_bin_masses).
template <int W>
__global__ void k_rank_bin_masses(Geo g, const double *__restrict__ us_sorted, int n_pos, int *__restrict__ rb0,
                                  double *__restrict__ rpm) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x, a = blockIdx.y;
    if (r >= g.n_p) return;
    const size_t o = (size_t)a * g.n_p + r;
    const double us = us_sorted[o];
    const double width = 2.0 * g.half_len / n_pos;
    const int b0 = min(max((int)floor((us - 3.0 * g.sig_u + g.half_len) / width), 0), n_pos - 1);
    rb0[o] = b0;
    for (int i = 0; i < W; ++i) {
        const int b = b0 + i;
        const double u0 = -g.half_len + b * width, u1 = u0 + width;
        rpm[o * W + i] = b < n_pos ? pos_mass(g, us, u0, u1) : 0.0;
    }
}

template <int W, int KMAX>
__global__ __launch_bounds__(64) void k_binned_rows_all(Geo g, const int *__restrict__ p_pix,
                                                        const double *__restrict__ cs, const double *__restrict__ Ld,
                                                        const double *__restrict__ Bt,
                                                        const int *__restrict__ s_sorted, const int *__restrict__ rb0,
                                                        const double *__restrict__ rpm, int n_pos,
                                                        const double *__restrict__ edges, int n_e,
                                                        const int *__restrict__ angle_row0, float *__restrict__ H) {
    const int a = blockIdx.y;
    const int q = blockIdx.x * 64 + threadIdx.x;   // n_qpad is a multiple of 64
    const bool active = q < g.n_q;
    const double nx = cs[2 * a], ny = cs[2 * a + 1];
    const double s2 = M_SQRT2 * g.sig_e;
    float *Hq = H + (size_t)angle_row0[a] * g.n_qpad + q;
    double acc[W][KMAX];
#pragma unroll
    for (int i = 0; i < W; ++i)
#pragma unroll
        for (int k = 0; k < KMAX; ++k) acc[i][k] = 0.0;
    int base = 0;
    // write the lowest bin of the window and slide it up by one bin
    auto shift = [&]() {
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < n_e) Hq[(size_t)(base * n_e + k) * g.n_qpad] = (float)acc[0][k];
#pragma unroll
        for (int i = 0; i + 1 < W; ++i)
#pragma unroll
            for (int k = 0; k < KMAX; ++k) acc[i][k] = acc[i + 1][k];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) acc[W - 1][k] = 0.0;
        ++base;
    };
    for (int r = 0; r < g.n_p; ++r) {
        const size_t o = (size_t)a * g.n_p + r;
        const int b0 = rb0[o];
        while (base < b0) shift();
        if (!active) continue;
        const PathW pw = path_weight(g, p_pix, Ld, Bt, nx, ny, a, q, s_sorted[o]);
        if (!(pw.w > 0.0)) continue;
        double ef[KMAX + 1];
#pragma unroll
        for (int k = 0; k <= KMAX; ++k) ef[k] = k <= n_e ? erf((edges[k] - pw.ep) / s2) : 0.0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const double wp = pw.w * rpm[o * W + i];
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k < n_e) acc[i][k] += wp * (0.5 * (ef[k + 1] - ef[k]));
        }
    }
    while (base < n_pos) shift();
}

// counts[(a * n_pos + b) * n_e + k] += 1 per event inside a bin
__global__ void k_bin_events(Geo g, int64_t n, const int32_t *__restrict__ angle, const float *__restrict__ u_bin,
                             const float *__restrict__ energy, int n_pos, const double *__restrict__ edges, int n_e,
                             float *__restrict__ counts) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int a = angle[j];
    if (a < 0 || a >= g.n_angles) return;
    const float ub = u_bin[j];
    if (!(ub >= 0.0f) || !(ub < (float)g.n_bins)) return;
    const int b = min((int)((double)ub * n_pos / g.n_bins), n_pos - 1);
    const double e = (double)energy[j];
    if (!(e >= edges[0]) || !(e <= edges[n_e])) return;
    int k = 0;
    while (k + 1 < n_e && e >= edges[k + 1]) ++k;
    atomicAdd(counts + ((size_t)a * n_pos + b) * n_e + k, 1.0f);   // integer counts: exact in any order
}

__global__ void k_gather_counts(const float *__restrict__ counts, const int *__restrict__ row_bin, int n_rows,
                                float *__restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_rows) y[i] = counts[row_bin[i]];
}

// weights of the binned backprojection: y_i / mean_i (0 for a dead bin)
__global__ void k_count_weights(const float *__restrict__ y, const float *__restrict__ inv, int n_rows,
                                float *__restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_rows) w[i] = y[i] * inv[i];
}

hipError_t launch_binned_rows(const Geo &g, const Tables &t, int n_pos, const double *edges_dev, int n_e,
                              const int *row_bin_dev, int n_rows, float *H, hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    if (!t.Ld) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((g.n_qpad + 255) / 256), (unsigned)n_rows);
    hipLaunchKernelGGL(k_binned_rows, grid, dim3(256), 0, st, g, t.p_pix, t.cs, t.Ld, t.Bt, t.s_sorted, t.us_sorted,
                       n_pos, edges_dev, n_e, row_bin_dev, H);
    return hipGetLastError();
}

template <int W, int KMAX>
void launch_rows_all(const Geo &g, const Tables &t, int n_pos, const double *edges_dev, int n_e,
                     const int *angle_row0_dev, int *rb0, double *rpm, float *H, hipStream_t st) {
    hipLaunchKernelGGL(k_rank_bin_masses<W>, dim3((unsigned)((g.n_p + 255) / 256), (unsigned)g.n_angles), dim3(256),
                       0, st, g, t.us_sorted, n_pos, rb0, rpm);
    hipLaunchKernelGGL((k_binned_rows_all<W, KMAX>), dim3((unsigned)(g.n_qpad / 64), (unsigned)g.n_angles), dim3(64),
                       0, st, g, t.p_pix, t.cs, t.Ld, t.Bt, t.s_sorted, rb0, rpm, n_pos, edges_dev, n_e,
                       angle_row0_dev, H);
}

// Rows of every bin, angle a's rows starting at angle_row0[a] in (position
// bin, energy bin) order.  hipErrorNotSupported when a position response
// spans more bins, or there are more energy bins, than the instantiated
// windows hold (the caller then lists the bins for k_binned_rows).
hipError_t launch_binned_rows_all(const Geo &g, const Tables &t, int n_pos, const double *edges_dev, int n_e,
                                  const int *angle_row0_dev, float *H, hipStream_t st) {
    if (!t.Ld) return hipErrorInvalidValue;
    const double width = 2.0 * g.half_len / n_pos;
    const int span = (int)ceil(6.0 * g.sig_u / width) + 2;   // bins a response can touch
    const int W = span <= 8 ? 8 : span <= 16 ? 16 : 0;
    if (W == 0 || n_e > (W == 8 ? 4 : 2)) return hipErrorNotSupported;
    int *rb0 = nullptr;
    double *rpm = nullptr;
    const size_t na_np = (size_t)g.n_angles * g.n_p;
    hipError_t e = hipMalloc(&rb0, sizeof(int) * na_np);
    if (e == hipSuccess) e = hipMalloc(&rpm, sizeof(double) * na_np * W);
    if (e == hipSuccess) {
        // the fewest accumulators that hold the energy bins
        if (W == 8 && n_e == 1) launch_rows_all<8, 1>(g, t, n_pos, edges_dev, n_e, angle_row0_dev, rb0, rpm, H, st);
        else if (W == 8 && n_e == 2) launch_rows_all<8, 2>(g, t, n_pos, edges_dev, n_e, angle_row0_dev, rb0, rpm, H, st);
        else if (W == 8) launch_rows_all<8, 4>(g, t, n_pos, edges_dev, n_e, angle_row0_dev, rb0, rpm, H, st);
        else if (n_e == 1) launch_rows_all<16, 1>(g, t, n_pos, edges_dev, n_e, angle_row0_dev, rb0, rpm, H, st);
        else launch_rows_all<16, 2>(g, t, n_pos, edges_dev, n_e, angle_row0_dev, rb0, rpm, H, st);
        e = hipGetLastError();
    }
    // the scratch is released once the kernels are done
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(rb0);
    hipFree(rpm);
    return e;
}

hipError_t launch_bin_events(const Geo &g, const lmosem_events &ev, int n_pos, const double *edges_dev, int n_e,
                             float *counts, hipStream_t st) {
    if (ev.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin_events, dim3((unsigned)((ev.n + 255) / 256)), dim3(256), 0, st, g, ev.n, ev.angle,
                       ev.u_bin, ev.energy_kev, n_pos, edges_dev, n_e, counts);
    return hipGetLastError();
}

hipError_t launch_gather_counts(const float *counts, const int *row_bin, int n_rows, float *y, hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_counts, dim3((n_rows + 255) / 256), dim3(256), 0, st, counts, row_bin, n_rows, y);
    return hipGetLastError();
}

hipError_t launch_count_weights(const float *y, const float *inv, int n_rows, float *w, hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_weights, dim3((n_rows + 255) / 256), dim3(256), 0, st, y, inv, n_rows, w);
    return hipGetLastError();
}

}  // namespace lmo
