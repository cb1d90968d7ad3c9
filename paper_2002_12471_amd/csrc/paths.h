// Per-path weights of the model, shared by the table build and the exact
// training targets of the learned scatter term (device code, FP64).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "lmosem_int.h"

namespace lmo {

// Klein-Nishina total cross-section in units of r_e^2.
__device__ __host__ inline double kn_total(double e) {
    double k = e / kMeC2;
    double l = log1p(2.0 * k);
    double k1 = 1.0 + k, k2 = 1.0 + 2.0 * k;
    return 2.0 * M_PI * (k1 / (k * k) * (2.0 * k1 / k2 - l / k) + l / (2.0 * k) - (1.0 + 3.0 * k) / (k2 * k2));
}

// Weight w and end energy E' of the path from emission pixel q through path
// end s at angle a (s == q: the primary path).
struct PathW {
    double w, ep;
};

__device__ inline PathW path_weight(const Geo &g, const int *__restrict__ p_pix, const double *__restrict__ L,
                                    const double *__restrict__ Bt, double nx, double ny, int a, int q, int s) {
    if (s == q) return {exp(-L[(size_t)a * g.n_p + q]), g.e0};
    if (!g.scatter) return {0.0, g.e0};
    const int pq = p_pix[q], ps = p_pix[s];
    const int di = ps % g.nx - pq % g.nx, dj = ps / g.nx - pq / g.nx;
    const double c = (di * nx + dj * ny) / sqrt((double)(di * di + dj * dj));
    const double t = 1.0 + g.kappa * (1.0 - c);
    const double P = 1.0 / t;
    const double ep = g.e0 * P;
    const double psi = P * P * (P + t - 1.0 + c * c);
    const double rho = kn_total(ep) / g.sigma_kn_e0;
    return {Bt[(size_t)s * g.n_p + q] * psi / g.psi_bar * exp(-rho * L[(size_t)a * g.n_p + s]), ep};
}

}  // namespace lmo
