// Vector-ALU rate probes: how many FP32 FMAs, exp2s and forward-projection
// terms (FMA, exp2, FMA) the GPU retires per second.  Each thread runs 16
// independent dependency chains so that issue rate, not latency, bounds them.
// The FMA probe keeps its operands in vector registers: an FMA that reads a
// scalar register issues at 64 lanes per CU and clock, one on vector
// registers alone at up to 128 (dual issue), which is what the published
// FP32 rate counts.
#include <hip/hip_runtime.h>

#include "lmosem_int.h"

namespace lmo {

constexpr int kChains = 16;

__global__ __launch_bounds__(256) void k_probe_fma(int iters, float m, float c, float *out) {
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = threadIdx.x * 1e-3f + k;
    __asm__ volatile("" : "+v"(m), "+v"(c));   // the multiplier and addend in vector registers
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) x[k] = fmaf(x[k], m, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    if (s == 12345.678f) out[threadIdx.x] = s;   // keeps the chains alive
}

// x <- -exp2(x) keeps x in [-1, -0.5]: one exp2 and one negation per step
__global__ __launch_bounds__(256) void k_probe_exp(int iters, float m, float c, float *out) {
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = -0.5f - threadIdx.x * 1e-6f - k * 1e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) x[k] = fmaf(__builtin_amdgcn_exp2f(x[k]), m, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    if (s == 12345.678f) out[threadIdx.x] = s;
}

// the forward projection's term: acc += k * exp2(beta * e + alpha), with the
// per-step (alpha, beta) shared by the chains and e, k per chain
__global__ __launch_bounds__(256) void k_probe_term(int iters, float m, float c, float *out) {
    float acc[kChains], e[kChains], kk[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
        acc[k] = 0.0f;
        e[k] = -20.0f + k;
        kk[k] = 1e-3f * (k + 1);
    }
    float alpha = -3.0f - threadIdx.x * 1e-4f, beta = 0.01f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) acc[k] = fmaf(kk[k], __builtin_amdgcn_exp2f(fmaf(beta, e[k], alpha)), acc[k]);
        alpha = fmaf(alpha, m, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += acc[k];
    if (s == 12345.678f) out[threadIdx.x] = s;
}

static double time_kernel(void (*kern)(int, float, float, float *), int iters, float m, float c,
                          float *out, hipStream_t st, hipError_t &err) {
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int blocks = cus * 16;
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, st, 16, m, c, out);   // warm-up
    hipEventRecord(a, st);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, st, iters, m, c, out);
    hipEventRecord(b, st);
    err = hipEventSynchronize(b);
    float ms = 0.0f;
    hipEventElapsedTime(&ms, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    return (double)blocks * 256.0 * iters * kChains / (ms * 1e-3);   // chain steps per second
}

hipError_t measure_alu_rates(hipStream_t st, double *out3) {
    float *scratch = nullptr;
    hipError_t e = hipMalloc(&scratch, 256 * sizeof(float));
    if (e != hipSuccess) return e;
    const int iters = 4096;
    double fma = time_kernel(k_probe_fma, iters, 0.999f, 1e-3f, scratch, st, e);
    if (e == hipSuccess) {
        double expfma = time_kernel(k_probe_exp, iters, -1.0f, 0.0f, scratch, st, e);
        // one exp2 + one FMA per step: exp2 time = step time - FMA time
        double t_exp = 1.0 / expfma - 1.0 / fma;
        out3[0] = fma;
        out3[1] = t_exp > 0 ? 1.0 / t_exp : 0.0;
    }
    if (e == hipSuccess) out3[2] = time_kernel(k_probe_term, iters, 0.9999f, -1e-4f, scratch, st, e);
    hipFree(scratch);
    return e;
}

}  // namespace lmo
