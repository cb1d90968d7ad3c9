// Emission set from a crude image (Sec. 2.2): the work of every iteration
// grows with the number of pixels the estimate may hold, so the estimate is
// confined to a rough object boundary found by a quick binned OS-MLEM.  The
// boundary is a threshold relative to the image maximum, widened by a margin
// (a disc of margin_px pixels) and kept inside mu > 0:
//     mask[p] = 1  iff  mu[p] > 0 and some p' with |p - p'|^2 <= margin^2
//                       (in pixels) has img[p'] >= rel_threshold * max(img).
#include <hip/hip_runtime.h>
#include <math.h>

#include "lmosem_int.h"

namespace lmo {

// out[0] = max(img), out[1] = number of values that are negative, NaN or
// infinite; one block, fixed reduction order.
__global__ __launch_bounds__(1024) void k_image_max(const float *__restrict__ img, int n, float *__restrict__ out) {
    __shared__ float smax[1024];
    __shared__ int sbad[1024];
    float m = 0.0f;
    int bad = 0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        const float v = img[i];
        if (!(v >= 0.0f) || isinf(v)) ++bad;
        else m = fmaxf(m, v);
    }
    smax[threadIdx.x] = m;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + s]);
            sbad[threadIdx.x] += sbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = smax[0]; out[1] = (float)sbad[0]; }
}

// one thread per pixel; the comparison is in FP64 against thr = t * max
__global__ __launch_bounds__(256) void k_emission_mask(int nx, int ny, const float *__restrict__ mu,
                                                       const float *__restrict__ img, double thr, int margin,
                                                       float *__restrict__ mask) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= nx * ny) return;
    const int i = p % nx, j = p / nx;
    float hit = 0.0f;
    if (mu[p] > 0.0f) {
        const int r2 = margin * margin;
        for (int dj = -margin; dj <= margin && hit == 0.0f; ++dj) {
            const int jj = j + dj;
            if (jj < 0 || jj >= ny) continue;
            for (int di = -margin; di <= margin; ++di) {
                const int ii = i + di;
                if (ii < 0 || ii >= nx || di * di + dj * dj > r2) continue;
                if ((double)img[jj * nx + ii] >= thr) { hit = 1.0f; break; }
            }
        }
    }
    mask[p] = hit;
}

hipError_t launch_image_max(const float *img, int n, float *out, hipStream_t st) {
    hipLaunchKernelGGL(k_image_max, dim3(1), dim3(1024), 0, st, img, n, out);
    return hipGetLastError();
}

hipError_t launch_emission_mask(const Geo &g, const float *mu, const float *img, double thr, int margin, float *mask,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_emission_mask, dim3((unsigned)((g.n_pix + 255) / 256)), dim3(256), 0, st, g.nx, g.ny, mu,
                       img, thr, margin, mask);
    return hipGetLastError();
}

}  // namespace lmo
