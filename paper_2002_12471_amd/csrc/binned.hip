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
