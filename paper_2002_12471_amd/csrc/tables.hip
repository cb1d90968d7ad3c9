// Path tables for one attenuation map (built once per context, FP64 on the GPU).
//
// Every path of the model starts at an emission pixel q and ends at a pixel
// s where it leaves for the detector along n_a: s == q is the primary path,
// s != q the first-order in-plane scatter path through s (Sec. 2.2).  For
// each angle a the path ends are ranked by their detector position
// u_s(a) = c_s . t_a, so that the ends an event's position response can reach
// form one contiguous rank range.  Per (a, rank, q) the table stores the
// path's weight and end energy encoded for the forward kernel:
//     alpha = log2(w / (sqrt(2 pi) sig_e)) - c2 (E' - e_c)^2,  beta = 2 c2 (E' - e_c)
// so that w G(E; E') = 2^(alpha + beta (E - e_c) - c2 (E - e_c)^2).
// The per-subset sensitivity (the denominators of Eq. 6/7) is accumulated
// from the same weights times the detector and window acceptances.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "lmosem_int.h"
#include "paths.h"

namespace lmo {

// Exact radiological path from the centre of pixel (i, j) along (dirx, diry)
// for a length tmax (or until the ray leaves the grid), by stepping from
// boundary to boundary (Amanatides and Woo, Eurographics 1987).
__device__ double traverse(const float *__restrict__ mu, int nx, int ny, double dx, int i, int j,
                           double dirx, double diry, double tmax) {
    const double inf = 1e300;
    int sx = dirx > 0 ? 1 : (dirx < 0 ? -1 : 0);
    int sy = diry > 0 ? 1 : (diry < 0 ? -1 : 0);
    double tdx = sx ? dx / fabs(dirx) : inf;
    double tdy = sy ? dx / fabs(diry) : inf;
    double tmx = sx ? 0.5 * tdx : inf;
    double tmy = sy ? 0.5 * tdy : inf;
    double t = 0.0, sum = 0.0;
    for (;;) {
        double tn = fmin(fmin(tmx, tmy), tmax);
        sum += (double)mu[j * nx + i] * (tn - t);
        t = tn;
        if (t >= tmax) break;
        if (tmx <= tmy) {
            i += sx;
            tmx += tdx;
        } else {
            j += sy;
            tmy += tdy;
        }
        if (i < 0 || i >= nx || j < 0 || j >= ny) break;
    }
    return sum;
}

// L_a(p): attenuation from the centre of support pixel p to the detector.
__global__ void k_line_to_detector(Geo g, const float *__restrict__ mu, const int *__restrict__ p_pix,
                                   const double *__restrict__ cs, double *__restrict__ L) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.n_angles * g.n_p) return;
    int a = idx / g.n_p, p = idx % g.n_p;
    int pix = p_pix[p];
    L[idx] = traverse(mu, g.nx, g.ny, g.dx, pix % g.nx, pix / g.nx, cs[2 * a], cs[2 * a + 1], 1e300);
}

// L^back_a(p): attenuation from the centre of p away from the detector (along -n_a)
__global__ void k_line_away(Geo g, const float *__restrict__ mu, const int *__restrict__ p_pix,
                            const double *__restrict__ cs, const double *__restrict__ L, float *__restrict__ Ldet,
                            float *__restrict__ Lback) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.n_angles * g.n_p) return;
    int a = idx / g.n_p, p = idx % g.n_p;
    int pix = p_pix[p];
    Lback[idx] = (float)traverse(mu, g.nx, g.ny, g.dx, pix % g.nx, pix / g.nx, -cs[2 * a], -cs[2 * a + 1], 1e300);
    Ldet[idx] = (float)L[idx];
}

// Bt[s][q] = B(q, s) = mu(s) dx^2 exp(-l(q,s)) / (2 pi r): the probability that
// a photon emitted at q interacts at the scatter point s (0 for s == q, and
// for a support pixel q outside the emission set, which emits nothing).
__global__ void k_scatter_points(Geo g, const float *__restrict__ mu, const int *__restrict__ p_pix,
                                 double *__restrict__ Bt) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int s = blockIdx.y;
    if (q >= g.n_p) return;
    double b = 0.0;
    if (q != s && q < g.n_q) {
        int pq = p_pix[q], ps = p_pix[s];
        int di = ps % g.nx - pq % g.nx, dj = ps / g.nx - pq / g.nx;
        double r = g.dx * sqrt((double)(di * di + dj * dj));
        double ell = traverse(mu, g.nx, g.ny, g.dx, pq % g.nx, pq / g.nx, g.dx * di / r,
                              g.dx * dj / r, r);
        b = (double)mu[ps] * g.dx * g.dx * exp(-ell) / (2.0 * M_PI * r);
    }
    Bt[(size_t)s * g.n_p + q] = b;
}

__device__ inline double centre_x(const Geo &g, int pix) { return ((pix % g.nx) - 0.5 * (g.nx - 1)) * g.dx; }
__device__ inline double centre_y(const Geo &g, int pix) { return ((pix / g.nx) - 0.5 * (g.ny - 1)) * g.dx; }

// fraction of the truncated position response centred at up on the detector
__device__ double detector_mass(const Geo &g, double up) {
    double s = g.sig_u;
    double a = fmax(-g.half_len - up, -3.0 * s), b = fmin(g.half_len - up, 3.0 * s);
    if (b <= a) return 0.0;
    double gs = s * sqrt(M_PI / 2.0) * (erf(b / (M_SQRT2 * s)) - erf(a / (M_SQRT2 * s)));
    return (gs - exp(-4.5) * (b - a)) / g.zk;
}

// Rank path ends by detector position per angle (ties by index).
__global__ void k_rank(Geo g, const int *__restrict__ p_pix, const double *__restrict__ cs,
                       const float *__restrict__ mu, int *__restrict__ s_sorted, double *__restrict__ us_sorted,
                       float *__restrict__ mu_sorted, double *__restrict__ D_sorted) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    int a = blockIdx.y;
    if (p >= g.n_p) return;
    double tx = -cs[2 * a + 1], ty = cs[2 * a];
    int pix = p_pix[p];
    double u = centre_x(g, pix) * tx + centre_y(g, pix) * ty;
    int rank = 0;
    for (int k = 0; k < g.n_p; ++k) {
        int pk = p_pix[k];
        double uk = centre_x(g, pk) * tx + centre_y(g, pk) * ty;
        rank += (uk < u) || (uk == u && k < p);
    }
    size_t o = (size_t)a * g.n_p + rank;
    s_sorted[o] = p;
    us_sorted[o] = u;
    mu_sorted[o] = mu[pix];
    D_sorted[o] = detector_mass(g, u);
}

// (alpha, beta) code of a path weight; zero weight never contributes
__device__ inline float2 path_code(const Geo &g, PathW p, double log2_gnorm) {
    if (!(p.w > 0.0)) return make_float2(kNegHuge, 0.0f);
    const double ec = p.ep - g.e_c;
    return make_float2((float)(log2(p.w) + log2_gnorm - g.c2 * ec * ec), (float)(2.0 * g.c2 * ec));
}

// Path table and per-angle sensitivities.  One thread per (angle, emission
// pixel q); it walks the path ends in rank order.
__global__ void k_path_table(Geo g, const int *__restrict__ p_pix, const double *__restrict__ cs,
                             const double *__restrict__ L, const double *__restrict__ Bt,
                             const int *__restrict__ s_sorted, const double *__restrict__ D_sorted,
                             float2 *__restrict__ T, double *__restrict__ sens_a, float *__restrict__ prim) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int a = blockIdx.y;
    if (q >= g.n_qpad) return;
    // T is null when only the sensitivity and the primary weights are wanted
    float2 *Ta = T ? T + (size_t)a * g.n_rpad * g.n_qpad + q : nullptr;
    if (Ta)
        for (int r = g.n_p; r < g.n_rpad; ++r) Ta[(size_t)r * g.n_qpad] = make_float2(kNegHuge, 0.0f);
    if (q >= g.n_q) {
        if (Ta)
            for (int r = 0; r < g.n_p; ++r) Ta[(size_t)r * g.n_qpad] = make_float2(kNegHuge, 0.0f);
        sens_a[(size_t)a * g.n_qpad + q] = 0.0;
        return;
    }
    const double nx = cs[2 * a], ny = cs[2 * a + 1];
    const double log2_gnorm = -log2(sqrt(2.0 * M_PI) * g.sig_e);
    const double s2 = M_SQRT2 * g.sig_e;
    double sens = 0.0;
    for (int r = 0; r < g.n_p; ++r) {
        const size_t o = (size_t)a * g.n_p + r;
        const int s = s_sorted[o];
        const PathW pw = path_weight(g, p_pix, L, Bt, nx, ny, a, q, s);
        const float2 code = path_code(g, pw, log2_gnorm);
        if (pw.w > 0.0) {
            const double win = 0.5 * (erf((g.win_hi - pw.ep) / s2) - erf((g.win_lo - pw.ep) / s2));
            sens += pw.w * D_sorted[o] * win;
        }
        if (s == q) prim[(size_t)a * g.n_p + q] = code.x;
        if (Ta) Ta[(size_t)r * g.n_qpad] = code;
    }
    sens_a[(size_t)a * g.n_qpad + q] = sens;
}

// Near-field band of emission pixel q at angle a: the path ends whose detector
// position lies within 6 sig_u of q's own (u_q), i.e. every end that an event
// inside q's primary position response (|u - u_q| < 3 sig_u) can reach.  The
// ends are a contiguous rank range [lo, hi).
__global__ void k_band_range(Geo g, const int *__restrict__ p_pix, const double *__restrict__ cs,
                             const double *__restrict__ us_sorted, int *__restrict__ band_lo,
                             int *__restrict__ band_len) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = blockIdx.y;
    if (q >= g.n_q) return;
    const int pix = p_pix[q];
    const double uq = centre_x(g, pix) * -cs[2 * a + 1] + centre_y(g, pix) * cs[2 * a];
    const double reach = 6.0 * g.sig_u;
    const double *us = us_sorted + (size_t)a * g.n_p;
    int lo = 0, hi = g.n_p;   // first rank with us > uq - reach
    while (lo < hi) { const int m = (lo + hi) >> 1; if (us[m] > uq - reach) hi = m; else lo = m + 1; }
    int lo2 = lo, hi2 = g.n_p;   // first rank with us >= uq + reach
    while (lo2 < hi2) { const int m = (lo2 + hi2) >> 1; if (us[m] >= uq + reach) hi2 = m; else lo2 = m + 1; }
    band_lo[(size_t)a * g.n_p + q] = lo;
    band_len[(size_t)a * g.n_p + q] = lo2 - lo;
}

// Near-field table band[a][q][k] = code of rank band_lo[a][q] + k (the
// primary path s == q and slots past the band never contribute).
__global__ void k_band_table(Geo g, int band_w, const int *__restrict__ p_pix, const double *__restrict__ cs,
                             const double *__restrict__ L, const double *__restrict__ Bt,
                             const int *__restrict__ s_sorted, const int *__restrict__ band_lo,
                             const int *__restrict__ band_len, float2 *__restrict__ band) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = blockIdx.y;
    if (q >= g.n_qpad) return;
    float2 *out = band + ((size_t)a * g.n_qpad + q) * band_w;
    const int lo = q < g.n_q ? band_lo[(size_t)a * g.n_p + q] : 0;
    const int len = q < g.n_q ? band_len[(size_t)a * g.n_p + q] : 0;
    const double nx = cs[2 * a], ny = cs[2 * a + 1];
    const double log2_gnorm = -log2(sqrt(2.0 * M_PI) * g.sig_e);
    for (int k = 0; k < band_w; ++k) {
        float2 code = make_float2(kNegHuge, 0.0f);
        if (k < len) {
            const int s = s_sorted[(size_t)a * g.n_p + lo + k];
            if (s != q) code = path_code(g, path_weight(g, p_pix, L, Bt, nx, ny, a, q, s), log2_gnorm);
        }
        out[k] = code;
    }
}

// sens[i][q] = T sum_{a mod N_s == i} sens_a[a][q]; sens_all = sum over subsets.
__global__ void k_sens_reduce(Geo g, const double *__restrict__ sens_a, float *__restrict__ sens,
                              float *__restrict__ sens_all) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= g.n_qpad) return;
    double tot = 0.0;
    for (int i = 0; i < g.n_subsets; ++i) {
        double s = 0.0;
        for (int a = i; a < g.n_angles; a += g.n_subsets) s += sens_a[(size_t)a * g.n_qpad + q];
        sens[(size_t)i * g.n_qpad + q] = (float)(g.acq_time * s);
        tot += s;
    }
    sens_all[q] = (float)(g.acq_time * tot);
}

// Geometry every context needs at once: line integrals, scatter-point
// factors, path ends ranked per angle and their detector-response masses.
hipError_t build_base(const Geo &g, Tables &t, hipStream_t st, std::string &err, int64_t &bytes) {
    hipError_t e;
    auto fail = [&](const char *what, hipError_t code) {
        char buf[256];
        snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(code));
        err = buf;
        return code;
    };
#define CK(call, what) do { e = (call); if (e != hipSuccess) return fail(what, e); } while (0)
    const size_t na_np = (size_t)g.n_angles * g.n_p;
    CK(hipMalloc(&t.Ld, sizeof(double) * na_np), "alloc L");
    if (g.scatter) CK(hipMalloc(&t.Bt, sizeof(double) * (size_t)g.n_p * g.n_p), "alloc B");
    CK(hipMalloc(&t.D_sorted, sizeof(double) * na_np), "alloc D");
    CK(hipMalloc(&t.s_sorted, sizeof(int) * na_np), "alloc ranks");
    CK(hipMalloc(&t.us_sorted, sizeof(double) * na_np), "alloc positions");
    CK(hipMalloc(&t.mu_sorted, sizeof(float) * na_np), "alloc positions");
    CK(hipMalloc(&t.Ldet, sizeof(float) * na_np), "alloc line integrals");
    CK(hipMalloc(&t.Lback, sizeof(float) * na_np), "alloc line integrals");
    bytes = (int64_t)(na_np * (3 * sizeof(double) + sizeof(int) + 3 * sizeof(float)) +
                      (g.scatter ? sizeof(double) * (size_t)g.n_p * g.n_p : 0));
    hipLaunchKernelGGL(k_line_to_detector, dim3((unsigned)((na_np + 255) / 256)), dim3(256), 0, st, g, t.mu,
                       t.p_pix, t.cs, t.Ld);
    CK(hipGetLastError(), "line integrals");
    hipLaunchKernelGGL(k_line_away, dim3((unsigned)((na_np + 255) / 256)), dim3(256), 0, st, g, t.mu, t.p_pix, t.cs,
                       t.Ld, t.Ldet, t.Lback);
    CK(hipGetLastError(), "line integrals away");
    if (g.scatter) {
        hipLaunchKernelGGL(k_scatter_points, dim3((g.n_p + 255) / 256, g.n_p), dim3(256), 0, st, g,
                           t.mu, t.p_pix, t.Bt);
        CK(hipGetLastError(), "scatter points");
    }
    hipLaunchKernelGGL(k_rank, dim3((g.n_p + 255) / 256, g.n_angles), dim3(256), 0, st, g, t.p_pix,
                       t.cs, t.mu, t.s_sorted, t.us_sorted, t.mu_sorted, t.D_sorted);
    CK(hipGetLastError(), "rank");
    CK(hipStreamSynchronize(st), "table build");
#undef CK
    return hipSuccess;
}

// What list-mode work needs on top of build_base: the per-subset
// sensitivities, the primary weights, and the path table (store_paths) or the
// near-field band (store_band).  Adds its device bytes to `bytes`.
hipError_t build_paths(const Geo &g, Tables &t, bool store_paths, bool store_band, hipStream_t st,
                       std::string &err, int64_t &bytes) {
    hipError_t e;
    double *sens_a = nullptr;
    int *band_len = nullptr;
    size_t nT = (size_t)g.n_angles * g.n_rpad * g.n_qpad;
    auto fail = [&](const char *what, hipError_t code) {
        char buf[256];
        snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(code));
        err = buf;
        hipFree(sens_a); hipFree(band_len);
        return code;
    };
#define CK(call, what) do { e = (call); if (e != hipSuccess) return fail(what, e); } while (0)
    CK(hipMalloc(&sens_a, sizeof(double) * g.n_angles * g.n_qpad), "alloc sens_a");
    if (store_paths) CK(hipMalloc(&t.T, sizeof(float2) * nT), "alloc path table");
    CK(hipMalloc(&t.prim, sizeof(float) * g.n_angles * g.n_p), "alloc primary weights");
    CK(hipMalloc(&t.sens, sizeof(float) * g.n_subsets * g.n_qpad), "alloc sens");
    CK(hipMalloc(&t.sens_all, sizeof(float) * g.n_qpad), "alloc sens_all");
    bytes += (int64_t)((store_paths ? sizeof(float2) * nT : 0) + sizeof(float) * g.n_angles * g.n_p +
                       sizeof(float) * (g.n_subsets + 1) * g.n_qpad);
    hipLaunchKernelGGL(k_path_table, dim3((g.n_qpad + 63) / 64, g.n_angles), dim3(64), 0, st, g,
                       t.p_pix, t.cs, t.Ld, t.Bt, t.s_sorted, t.D_sorted, t.T, sens_a, t.prim);
    CK(hipGetLastError(), "path table");
    if (store_band && g.scatter) {
        CK(hipMalloc(&t.band_lo, sizeof(int) * g.n_angles * g.n_p), "alloc band ranges");
        CK(hipMalloc(&band_len, sizeof(int) * g.n_angles * g.n_p), "alloc band ranges");
        hipLaunchKernelGGL(k_band_range, dim3((g.n_q + 255) / 256, g.n_angles), dim3(256), 0, st, g, t.p_pix, t.cs,
                           t.us_sorted, t.band_lo, band_len);
        CK(hipGetLastError(), "band ranges");
        std::vector<int> len((size_t)g.n_angles * g.n_p);
        CK(hipMemcpyAsync(len.data(), band_len, sizeof(int) * len.size(), hipMemcpyDeviceToHost, st), "band ranges");
        CK(hipStreamSynchronize(st), "band ranges");
        // bands exist for the emission pixels only (q < n_q of every angle)
        t.band_w = 1;
        for (int a = 0; a < g.n_angles; ++a)
            for (int q = 0; q < g.n_q; ++q) t.band_w = std::max(t.band_w, len[(size_t)a * g.n_p + q]);
        const size_t nb = (size_t)g.n_angles * t.band_w * g.n_qpad;
        CK(hipMalloc(&t.band, sizeof(float2) * nb), "alloc near-field table");
        hipLaunchKernelGGL(k_band_table, dim3((g.n_qpad + 63) / 64, g.n_angles), dim3(64), 0, st, g, t.band_w,
                           t.p_pix, t.cs, t.Ld, t.Bt, t.s_sorted, t.band_lo, band_len, t.band);
        CK(hipGetLastError(), "near-field table");
        bytes += (int64_t)(sizeof(float2) * nb + sizeof(int) * g.n_angles * g.n_p);
    }
    hipLaunchKernelGGL(k_sens_reduce, dim3((g.n_qpad + 255) / 256), dim3(256), 0, st, g, sens_a,
                       t.sens, t.sens_all);
    CK(hipGetLastError(), "sensitivity");
    CK(hipStreamSynchronize(st), "table build");
    hipFree(sens_a); hipFree(band_len);
#undef CK
    return hipSuccess;
}

}  // namespace lmo
