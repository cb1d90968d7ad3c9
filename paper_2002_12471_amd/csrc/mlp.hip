// Scatter-surrogate network on gfx950: 8 -> 128 -> 128 -> 128 -> 1 with GELU
// (tanh form), bf16 weights and activations, FP32 accumulation (MFMA), FP32
// master weights and Adam.
//
// Every matrix product is one kernel, C[m][n] = sum_k A[m][k] Bt[n][k], with
// both operands row-major bf16 and contiguous in k, which is the operand
// layout of v_mfma_f32_16x16x16_bf16 (lane l holds A[l%16][4(l/16)..+3] and
// B[4(l/16)..+3][l%16]; D[4(l/16)+v][l%16] comes back in register v):
//   forward       Z[b][out]  = H[b][in]   . Wt[out][in]
//   data grad     dH[b][in]  = D[b][out]  . W[in][out]
//   weight grad   dW[in][out] = Ht[in][b] . Dt[out][b]
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <vector>

#include "lmosem_int.h"
#include "mlp_infer.h"

namespace lmo {

typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ __host__ inline uint16_t f2bf(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

constexpr float kGeluC = 0.7978845608028654f;   // sqrt(2/pi)
constexpr float kGeluA = 0.044715f;

__device__ inline float gelu(float x) {
    const float u = kGeluC * (x + kGeluA * x * x * x);
    return 0.5f * x * (1.0f + tanhf(u));
}
__device__ inline float gelu_grad(float x) {
    const float u = kGeluC * (x + kGeluA * x * x * x);
    const float t = tanhf(u);
    return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * kGeluC * (1.0f + 3.0f * kGeluA * x * x);
}

// C[M][N] (+)= A[M][K] . Bt[N][K]^T; M, N, K multiples of 16, lda/ldb multiples of 4.
// 64x64 block per workgroup, 32x32 per wave (2x2 MFMA tiles).  With split K,
// blockIdx.z takes k in [z k_slice, (z+1) k_slice) and writes its partial
// product to C + z c_stride.
__global__ __launch_bounds__(256) void k_gemm_nt(const uint16_t *__restrict__ A, int lda,
                                                 const uint16_t *__restrict__ Bt, int ldb,
                                                 float *__restrict__ C, int ldc, int M, int N, int K,
                                                 int accumulate, int k_slice, size_t c_stride) {
    const int kz0 = blockIdx.z * k_slice, kz1 = min(K, kz0 + k_slice);
    C += blockIdx.z * c_stride;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m_base = blockIdx.y * 64 + (wave >> 1) * 32;
    const int n_base = blockIdx.x * 64 + (wave & 1) * 32;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x4 zero = {0, 0, 0, 0};
    for (int k0 = kz0; k0 < kz1; k0 += 16) {
        bf16x4 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int m = m_base + 16 * i + r;
            a[i] = m < M ? *reinterpret_cast<const bf16x4 *>(A + (size_t)m * lda + k0 + kq) : zero;
            const int n = n_base + 16 * i + r;
            b[i] = n < N ? *reinterpret_cast<const bf16x4 *>(Bt + (size_t)n * ldb + k0 + kq) : zero;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m_base + 16 * i + (lane >> 4) * 4 + v;
                const int n = n_base + 16 * j + r;
                if (m < M && n < N) {
                    float *c = C + (size_t)m * ldc + n;
                    *c = accumulate ? *c + acc[i][j][v] : acc[i][j][v];
                }
            }
}

// C[m][n] = sum over the S partial products (fixed order)
__global__ void k_sum_slices(const float *__restrict__ part, int S, int M, int N, float *__restrict__ C, int ldc) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * N) return;
    float s = 0.0f;
    for (int z = 0; z < S; ++z) s += part[(size_t)z * M * N + idx];
    C[(size_t)(idx / N) * ldc + idx % N] = s;
}

constexpr int kSplitMax = 32;   // partial products per split-K product (workspace slices)

// Products with few output blocks and a long K (the weight gradients, K = the
// batch) are split over K into up to kSplitMax slices of at least 256 in
// split_ws ([kSplitMax][M][N]) and summed in a fixed order.
hipError_t gemm_nt(const uint16_t *A, int lda, const uint16_t *Bt, int ldb, float *C, int ldc, int M, int N,
                   int K, bool accumulate, hipStream_t st, float *split_ws) {
    if (M % 16 || N % 16 || K % 16 || lda % 4 || ldb % 4) return hipErrorInvalidValue;
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
    const int blocks_mn = (int)(grid.x * grid.y);
    int S = 1;
    if (split_ws && !accumulate && M * N <= 128 * 128 && K >= 512)
        S = std::min(kSplitMax, std::max(1, std::min(K / 256, 256 / blocks_mn)));
    if (S <= 1) {
        hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, A, lda, Bt, ldb, C, ldc, M, N, K, accumulate ? 1 : 0,
                           K, (size_t)0);
        return hipGetLastError();
    }
    const int k_slice = ((K + S - 1) / S + 15) / 16 * 16;
    S = (K + k_slice - 1) / k_slice;
    grid.z = (unsigned)S;
    hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, A, lda, Bt, ldb, split_ws, N, M, N, K, 0, k_slice,
                       (size_t)M * N);
    hipLaunchKernelGGL(k_sum_slices, dim3((M * N + 255) / 256), dim3(256), 0, st, split_ws, S, M, N, C, ldc);
    return hipGetLastError();
}

// ---------------------------------------------------------------- network state
// Parameter order (flat FP32 master copy): W1[8][128] b1[128] W2[128][128] b2
// W3[128][128] b3 W4[128][1] b4[1]; W[in][out].
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kIn * kHid, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
              kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid * kHid, kOffW4 = kOffB3 + kHid,
              kOffB4 = kOffW4 + kHid, kNParams = kOffB4 + 1;
static_assert(kNParams == 34305, "parameter count");

struct NetBf16 {
    uint16_t *w1t, *w2t, *w3t;   // [out][in] (w1t: [128][16] zero-padded)
    uint16_t *w2, *w3;           // [in][out]
    uint16_t *w4;                // [128]
};

// master FP32 -> bf16 copies in both layouts
__global__ void k_pack(const float *__restrict__ p, NetBf16 nb) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < kHid * kInPad) {   // w1t[out][in]
        const int o = idx / kInPad, i = idx % kInPad;
        nb.w1t[idx] = i < kIn ? f2bf(p[kOffW1 + i * kHid + o]) : 0;
    }
    if (idx < kHid * kHid) {
        const int a = idx / kHid, b = idx % kHid;   // idx = a*128 + b
        nb.w2[idx] = f2bf(p[kOffW2 + idx]);          // [in a][out b]
        nb.w3[idx] = f2bf(p[kOffW3 + idx]);
        nb.w2t[idx] = f2bf(p[kOffW2 + b * kHid + a]);   // [out a][in b]
        nb.w3t[idx] = f2bf(p[kOffW3 + b * kHid + a]);
    }
    if (idx < kHid) nb.w4[idx] = f2bf(p[kOffW4 + idx]);
}

// X [n][8] f32 -> bf16 [n][16] (zero padded) and its transpose [16][n]
__global__ void k_input(const float *__restrict__ X, int n, uint16_t *__restrict__ xb, uint16_t *__restrict__ xt) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
#pragma unroll
    for (int i = 0; i < kInPad; ++i) {
        const uint16_t v = i < kIn ? f2bf(X[(size_t)b * kIn + i]) : 0;
        xb[(size_t)b * kInPad + i] = v;
        if (xt) xt[(size_t)i * n + b] = v;
    }
}

// The elementwise training kernels work on tiles of 16 samples x 128 hidden
// units (256 threads): the row-major [b][k] values are read and written
// along k, and the transposed bf16 copy [k][b] goes through LDS so that it
// is written along b (32 contiguous bytes per hidden unit).
constexpr int kTileB = 16;

template <typename F>
__device__ __forceinline__ void tile_rows_and_transpose(int n, uint16_t *__restrict__ d, uint16_t *__restrict__ dt,
                                                        F value) {
    __shared__ uint16_t tile[kTileB][kHid + 2];
    const int b0 = blockIdx.x * kTileB;
    for (int i = threadIdx.x; i < kTileB * kHid; i += 256) {
        const int bl = i / kHid, k = i % kHid, b = b0 + bl;
        if (b < n) {
            const uint16_t v = value((size_t)b * kHid + k, b, k);
            d[(size_t)b * kHid + k] = v;
            tile[bl][k] = v;
        }
    }
    if (!dt) return;
    __syncthreads();
    for (int i = threadIdx.x; i < kTileB * kHid; i += 256) {
        const int k = i / kTileB, bl = i % kTileB, b = b0 + bl;
        if (b < n) dt[(size_t)k * n + b] = tile[bl][k];
    }
}

// h = gelu(z + bias): z kept (with bias) for the backward pass; h in bf16,
// optionally also transposed
__global__ __launch_bounds__(256) void k_bias_gelu(float *__restrict__ z, const float *__restrict__ bias, int n,
                                                   uint16_t *__restrict__ h, uint16_t *__restrict__ ht) {
    tile_rows_and_transpose(n, h, ht, [&](size_t idx, int, int k) {
        const float v = z[idx] + bias[k];
        z[idx] = v;
        return f2bf(gelu(v));
    });
}

// y[b] = sum_k h[b][k] w4[k] + b4  (one wave per sample group of 64)
__global__ void k_output(const uint16_t *__restrict__ h, const uint16_t *__restrict__ w4,
                         const float *__restrict__ p, int n, float *__restrict__ y) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    float s = 0.0f;
    const uint16_t *hb = h + (size_t)b * kHid;
    for (int k = 0; k < kHid; ++k) s = fmaf(bf2f(hb[k]), bf2f(w4[k]), s);
    y[b] = s + p[kOffB4];
}

// loss partial sums and dy = 2 (y - t) / n_total
__global__ void k_mse(const float *__restrict__ y, const float *__restrict__ t, int n, float inv_total,
                      float *__restrict__ dy, double *__restrict__ loss_part) {
    __shared__ double red[256];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (b < n) {
        const float r = y[b] - t[b];
        dy[b] = 2.0f * r * inv_total;
        l = (double)r * r;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// output layer backward: d3[b][k] = dy[b] w4[k] gelu'(z3[b][k]) (bf16, both layouts)
__global__ __launch_bounds__(256) void k_out_back(const float *__restrict__ dy, const uint16_t *__restrict__ w4,
                                                  const float *__restrict__ z3, int n, uint16_t *__restrict__ d,
                                                  uint16_t *__restrict__ dt) {
    tile_rows_and_transpose(n, d, dt, [&](size_t idx, int b, int k) {
        return f2bf(dy[b] * bf2f(w4[k]) * gelu_grad(z3[idx]));
    });
}

// hidden layer backward: d[b][k] = dh[b][k] gelu'(z[b][k]) (bf16, both layouts)
__global__ __launch_bounds__(256) void k_gelu_back(const float *__restrict__ dh, const float *__restrict__ z, int n,
                                                   uint16_t *__restrict__ d, uint16_t *__restrict__ dt) {
    tile_rows_and_transpose(n, d, dt, [&](size_t idx, int, int) { return f2bf(dh[idx] * gelu_grad(z[idx])); });
}

// bias gradients: column sums of the transposed bf16 deltas dt[k][b]; the
// output layer's from dy and h3t
__global__ void k_bias_grads(const uint16_t *__restrict__ d1t, const uint16_t *__restrict__ d2t,
                             const uint16_t *__restrict__ d3t, const uint16_t *__restrict__ h3t,
                             const float *__restrict__ dy, int n, float *__restrict__ g) {
    __shared__ float red[256];
    const int row = blockIdx.x;   // 0..127 b1, 128..255 b2, 256..383 b3, 384..511 w4, 512 b4
    float s = 0.0f;
    if (row < 3 * kHid) {
        const uint16_t *dt = row < kHid ? d1t : (row < 2 * kHid ? d2t : d3t);
        const int k = row % kHid;
        for (int b = threadIdx.x; b < n; b += 256) s += bf2f(dt[(size_t)k * n + b]);
    } else if (row < 4 * kHid) {
        const int k = row - 3 * kHid;
        for (int b = threadIdx.x; b < n; b += 256) s += bf2f(h3t[(size_t)k * n + b]) * dy[b];
    } else {
        for (int b = threadIdx.x; b < n; b += 256) s += dy[b];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int off;
        if (row < kHid) off = kOffB1 + row;
        else if (row < 2 * kHid) off = kOffB2 + row - kHid;
        else if (row < 3 * kHid) off = kOffB3 + row - 2 * kHid;
        else if (row < 4 * kHid) off = kOffW4 + row - 3 * kHid;
        else off = kOffB4;
        g[off] = red[0];
    }
}

// dW1[i][o] from the padded 16-row product: keep the 8 real input rows
__global__ void k_copy_w1_grad(const float *__restrict__ gw1pad, float *__restrict__ g) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < kIn * kHid) g[kOffW1 + idx] = gw1pad[idx];
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- fused inference
// (the kernel: mlp_infer.h) packed weights: A operands in lane order (W1/4,
// W2 and W3 in bf16), the quartered biases and the output row (bf16-rounded,
// widened)

__global__ void k_pack_fused(const float *__restrict__ p, uint16_t *__restrict__ fw, float *__restrict__ fb) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < kFW1) {
        const int i = idx & 7, lane = (idx >> 3) & 63, ob = idx >> 9;
        const int in = perm_k(lane >> 4, i), out = 16 * ob + (lane & 15);
        fw[idx] = in < kIn ? f2bf(kActScale * p[kOffW1 + in * kHid + out]) : 0;
    }
    if (idx < 2 * kFW2) {
        const int layer = idx / kFW2, r = idx % kFW2;
        const int i = r & 7, lane = (r >> 3) & 63, kb = (r >> 9) & 3, ob = r >> 11;
        const int in = 32 * kb + perm_k(lane >> 4, i), out = 16 * ob + (lane & 15);
        fw[kFW1 + idx] = f2bf(p[(layer ? kOffW3 : kOffW2) + in * kHid + out]);
    }
    if (idx < kFB) {
        float v;
        if (idx < kHid) v = kActScale * p[kOffB1 + idx];
        else if (idx < 2 * kHid) v = kActScale * p[kOffB2 + idx - kHid];
        else if (idx < 3 * kHid) v = kActScale * p[kOffB3 + idx - 2 * kHid];
        else if (idx < 4 * kHid) v = bf2f(f2bf(p[kOffW4 + idx - 3 * kHid]));
        else v = p[kOffB4];
        fb[idx] = v;
    }
}

// samples from an array X[n][8], outputs to y[n]
struct XSource {
    const float *X;
    float *y;
    __device__ uint2 inputs(int64_t p, int g) const {
        const float4 v = *reinterpret_cast<const float4 *>(X + p * kIn + 4 * g);
        return uint2{__builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{v.x, v.y}, bf16x2)),
                     __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{v.z, v.w}, bf16x2))};
    }
    __device__ int64_t out_base(int64_t p0) const { return p0; }
    __device__ void output(int64_t p0, int i, float v) const { y[p0 + i] = v; }
};

// per-epoch loss: fixed-order sum of the minibatch's partial sums
__global__ void k_loss_add(const double *__restrict__ parts, int nparts, double *__restrict__ loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += parts[i];
    *loss += s;
}

// ---------------------------------------------------------------- host side
struct Net {
    hipStream_t st = nullptr;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // [kNParams]
    NetBf16 nb{};
    uint16_t *fw = nullptr;   // fused-inference weights [kFWTotal]
    float *fb = nullptr;      // fused-inference biases and output row [kFB]
    int step = 0;
    // batch workspace
    int cap = 0;
    uint16_t *xb = nullptr, *xt = nullptr, *h1 = nullptr, *h2 = nullptr, *h3 = nullptr;
    uint16_t *h1t = nullptr, *h2t = nullptr, *h3t = nullptr;
    uint16_t *d1 = nullptr, *d2 = nullptr, *d3 = nullptr, *d1t = nullptr, *d2t = nullptr, *d3t = nullptr;
    float *z1 = nullptr, *z2 = nullptr, *z3 = nullptr, *dh = nullptr, *dy = nullptr, *gw1 = nullptr;
    float *split = nullptr;   // split-K partial products [kSplitMax][128][128]
    double *loss_part = nullptr;
};

static void free_ws(Net &n) {
    for (void *q : {(void *)n.xb, (void *)n.xt, (void *)n.h1, (void *)n.h2, (void *)n.h3, (void *)n.h1t,
                    (void *)n.h2t, (void *)n.h3t, (void *)n.d1, (void *)n.d2, (void *)n.d3, (void *)n.d1t,
                    (void *)n.d2t, (void *)n.d3t, (void *)n.z1, (void *)n.z2, (void *)n.z3, (void *)n.dh,
                    (void *)n.dy, (void *)n.gw1, (void *)n.split, (void *)n.loss_part})
        hipFree(q);
    n.xb = n.xt = n.h1 = n.h2 = n.h3 = n.h1t = n.h2t = n.h3t = nullptr;
    n.d1 = n.d2 = n.d3 = n.d1t = n.d2t = n.d3t = nullptr;
    n.z1 = n.z2 = n.z3 = n.dh = n.dy = n.gw1 = n.split = nullptr;
    n.loss_part = nullptr;
    n.cap = 0;
}

static hipError_t ensure_ws(Net &n, int cap) {
    if (cap <= n.cap) return hipSuccess;
    free_ws(n);
    hipError_t e;
    const size_t c = (size_t)cap;
#define A(ptr, bytes) if ((e = hipMalloc(&(ptr), (bytes))) != hipSuccess) { free_ws(n); return e; }
    A(n.xb, c * kInPad * 2) A(n.xt, c * kInPad * 2)
    A(n.h1, c * kHid * 2) A(n.h2, c * kHid * 2) A(n.h3, c * kHid * 2)
    A(n.h1t, c * kHid * 2) A(n.h2t, c * kHid * 2) A(n.h3t, c * kHid * 2)
    A(n.d1, c * kHid * 2) A(n.d2, c * kHid * 2) A(n.d3, c * kHid * 2)
    A(n.d1t, c * kHid * 2) A(n.d2t, c * kHid * 2) A(n.d3t, c * kHid * 2)
    A(n.z1, c * kHid * 4) A(n.z2, c * kHid * 4) A(n.z3, c * kHid * 4) A(n.dh, c * kHid * 4)
    A(n.dy, c * 4) A(n.gw1, kInPad * kHid * 4) A(n.loss_part, (c / 256 + 2) * 8)
    A(n.split, (size_t)kSplitMax * kHid * kHid * 4)
#undef A
    n.cap = cap;
    return hipSuccess;
}

hipError_t net_create(const float *params_host, hipStream_t st, Net **out) {
    Net *n = new Net();
    n->st = st;
    hipError_t e;
    auto bail = [&](hipError_t err) { net_destroy(n); return err; };
    if ((e = hipMalloc(&n->p, kNParams * 4)) != hipSuccess) return bail(e);
    if ((e = hipMalloc(&n->g, kNParams * 4)) != hipSuccess) return bail(e);
    if ((e = hipMalloc(&n->m, kNParams * 4)) != hipSuccess) return bail(e);
    if ((e = hipMalloc(&n->v, kNParams * 4)) != hipSuccess) return bail(e);
    if ((e = hipMalloc(&n->nb.w1t, kHid * kInPad * 2)) != hipSuccess) return bail(e);
    if ((e = hipMalloc(&n->nb.w2t, kHid * kHid * 2)) != hipSuccess) return bail(e);
    if ((e = hipMalloc(&n->nb.w3t, kHid * kHid * 2)) != hipSuccess) return bail(e);
    if ((e = hipMalloc(&n->nb.w2, kHid * kHid * 2)) != hipSuccess) return bail(e);
    if ((e = hipMalloc(&n->nb.w3, kHid * kHid * 2)) != hipSuccess) return bail(e);
    if ((e = hipMalloc(&n->nb.w4, kHid * 2)) != hipSuccess) return bail(e);
    if ((e = hipMalloc(&n->fw, kFWTotal * 2)) != hipSuccess) return bail(e);
    if ((e = hipMalloc(&n->fb, kFB * 4)) != hipSuccess) return bail(e);
    if ((e = hipMemcpyAsync(n->p, params_host, kNParams * 4, hipMemcpyHostToDevice, st)) != hipSuccess) return bail(e);
    if ((e = hipMemsetAsync(n->m, 0, kNParams * 4, st)) != hipSuccess) return bail(e);
    if ((e = hipMemsetAsync(n->v, 0, kNParams * 4, st)) != hipSuccess) return bail(e);
    hipLaunchKernelGGL(k_pack, dim3((kHid * kHid + 255) / 256), dim3(256), 0, st, n->p, n->nb);
    hipLaunchKernelGGL(k_pack_fused, dim3((2 * kFW2 + 255) / 256), dim3(256), 0, st, n->p, n->fw, n->fb);
    if ((e = hipGetLastError()) != hipSuccess) return bail(e);
    // contexts run the network on their own streams: the weights are ready on return
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(e);
    *out = n;
    return hipSuccess;
}

void net_destroy(Net *n) {
    if (!n) return;
    free_ws(*n);
    hipFree(n->p); hipFree(n->g); hipFree(n->m); hipFree(n->v);
    hipFree(n->nb.w1t); hipFree(n->nb.w2t); hipFree(n->nb.w3t); hipFree(n->nb.w2); hipFree(n->nb.w3);
    hipFree(n->nb.w4); hipFree(n->fw); hipFree(n->fb);
    delete n;
}

hipStream_t net_stream(const Net *n) { return n->st; }

hipError_t net_get_params(Net *n, float *host) {
    hipError_t e = hipMemcpyAsync(host, n->p, kNParams * 4, hipMemcpyDeviceToHost, n->st);
    return e == hipSuccess ? hipStreamSynchronize(n->st) : e;
}

static inline unsigned blocks(size_t n) { return (unsigned)((n + 255) / 256); }
static inline unsigned tiles(int nb) { return (unsigned)((nb + kTileB - 1) / kTileB); }

// forward pass of one batch of nb samples (nb a multiple of 16); keeps the
// activations for the backward pass when train is set
static hipError_t forward_batch(Net &n, const float *X, int nb, float *y, bool train) {
    hipError_t e;
    hipStream_t st = n.st;
    hipLaunchKernelGGL(k_input, dim3(blocks(nb)), dim3(256), 0, st, X, nb, n.xb, train ? n.xt : nullptr);
    if ((e = gemm_nt(n.xb, kInPad, n.nb.w1t, kInPad, n.z1, kHid, nb, kHid, kInPad, false, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bias_gelu, dim3(tiles(nb)), dim3(256), 0, st, n.z1, n.p + kOffB1, nb, n.h1,
                       train ? n.h1t : nullptr);
    if ((e = gemm_nt(n.h1, kHid, n.nb.w2t, kHid, n.z2, kHid, nb, kHid, kHid, false, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bias_gelu, dim3(tiles(nb)), dim3(256), 0, st, n.z2, n.p + kOffB2, nb, n.h2,
                       train ? n.h2t : nullptr);
    if ((e = gemm_nt(n.h2, kHid, n.nb.w3t, kHid, n.z3, kHid, nb, kHid, kHid, false, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bias_gelu, dim3(tiles(nb)), dim3(256), 0, st, n.z3, n.p + kOffB3, nb, n.h3,
                       train ? n.h3t : nullptr);
    hipLaunchKernelGGL(k_output, dim3(blocks(nb)), dim3(256), 0, st, n.h3, n.nb.w4, n.p, nb, y);
    return hipGetLastError();
}

// gradients of sum_b dy[b] y[b] into n.g (after forward_batch with train)
static hipError_t backward_batch(Net &n, const float *dy, int nb) {
    hipError_t e;
    hipStream_t st = n.st;
    hipLaunchKernelGGL(k_out_back, dim3(tiles(nb)), dim3(256), 0, st, dy, n.nb.w4, n.z3, nb, n.d3, n.d3t);
    // dW3[in][out] = h2t . d3t ; dh2 = d3 . W3
    if ((e = gemm_nt(n.h2t, nb, n.d3t, nb, n.g + kOffW3, kHid, kHid, kHid, nb, false, st, n.split)) != hipSuccess)
        return e;
    if ((e = gemm_nt(n.d3, kHid, n.nb.w3, kHid, n.dh, kHid, nb, kHid, kHid, false, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gelu_back, dim3(tiles(nb)), dim3(256), 0, st, n.dh, n.z2, nb, n.d2, n.d2t);
    if ((e = gemm_nt(n.h1t, nb, n.d2t, nb, n.g + kOffW2, kHid, kHid, kHid, nb, false, st, n.split)) != hipSuccess)
        return e;
    if ((e = gemm_nt(n.d2, kHid, n.nb.w2, kHid, n.dh, kHid, nb, kHid, kHid, false, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gelu_back, dim3(tiles(nb)), dim3(256), 0, st, n.dh, n.z1, nb, n.d1, n.d1t);
    if ((e = gemm_nt(n.xt, nb, n.d1t, nb, n.gw1, kHid, kInPad, kHid, nb, false, st, n.split)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_copy_w1_grad, dim3(blocks(kIn * kHid)), dim3(256), 0, st, n.gw1, n.g);
    hipLaunchKernelGGL(k_bias_grads, dim3(4 * kHid + 1), dim3(256), 0, st, n.d1t, n.d2t, n.d3t, n.h3t, dy, nb, n.g);
    return hipGetLastError();
}

void net_fused_weights(const Net *n, const uint16_t **fw, const float **fb) {
    *fw = n->fw;
    *fb = n->fb;
}

hipError_t net_forward(Net *n, const float *X, int64_t count, float *y, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t tiles = (count + kFusedTile - 1) / kFusedTile;
    const unsigned grid = (unsigned)std::min<int64_t>(tiles, 256);   // one workgroup per CU
    hipLaunchKernelGGL(k_mlp_infer<XSource>, dim3(grid), dim3(kFusedThreads), 0, st, n->fw, n->fb,
                       XSource{X, y}, count);
    return hipGetLastError();
}

hipError_t net_forward_train(Net *n, const float *X, int count, float *y) {
    if (count <= 0 || count % 16) return hipErrorInvalidValue;
    hipError_t e = ensure_ws(*n, count);
    return e == hipSuccess ? forward_batch(*n, X, count, y, false) : e;
}

hipError_t net_gradient(Net *n, const float *X, const float *dy, int count, float *grad_host) {
    if (count <= 0 || count % 16) return hipErrorInvalidValue;
    hipError_t e = ensure_ws(*n, count);
    if (e == hipSuccess) e = forward_batch(*n, X, count, n->dy, true);
    if (e == hipSuccess) e = backward_batch(*n, dy, count);
    if (e == hipSuccess) e = hipMemcpyAsync(grad_host, n->g, kNParams * 4, hipMemcpyDeviceToHost, n->st);
    if (e == hipSuccess) e = hipStreamSynchronize(n->st);
    return e;
}

// Adam on mean-squared error over minibatches taken in order; the learning
// rate is multiplied by lr_decay after every epoch.  loss_host[epoch] gets
// the epoch's mean loss.
hipError_t net_train(Net *n, const float *X, const float *t, int64_t count, int batch, int epochs, float lr,
                     float lr_decay, double *loss_host) {
    if (batch <= 0 || batch % 16 || count < batch || epochs < 0) return hipErrorInvalidValue;
    hipError_t e = ensure_ws(*n, batch);
    float *y = nullptr;
    double *loss = nullptr;
    if (e == hipSuccess) e = hipMalloc(&y, (size_t)batch * 4);
    if (e == hipSuccess) e = hipMalloc(&loss, sizeof(double) * std::max(epochs, 1));
    if (e == hipSuccess) e = hipMemsetAsync(loss, 0, sizeof(double) * std::max(epochs, 1), n->st);
    const int64_t n_batches = count / batch;
    const int nparts = (batch + 255) / 256;
    for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
        for (int64_t bi = 0; bi < n_batches && e == hipSuccess; ++bi) {
            const float *xb = X + bi * batch * kIn;
            const float *tb = t + bi * batch;
            e = forward_batch(*n, xb, batch, y, true);
            if (e != hipSuccess) break;
            hipLaunchKernelGGL(k_mse, dim3(nparts), dim3(256), 0, n->st, y, tb, batch, 1.0f / batch, n->dy,
                               n->loss_part);
            hipLaunchKernelGGL(k_loss_add, dim3(1), dim3(64), 0, n->st, n->loss_part, nparts, loss + ep);
            if ((e = backward_batch(*n, n->dy, batch)) != hipSuccess) break;
            ++n->step;
            const float c1 = 1.0f - powf(0.9f, (float)n->step), c2 = 1.0f - powf(0.999f, (float)n->step);
            hipLaunchKernelGGL(k_adam, dim3(blocks(kNParams)), dim3(256), 0, n->st, n->p, n->g, n->m, n->v, kNParams,
                               lr, 0.9f, 0.999f, 1e-8f, c1, c2);
            hipLaunchKernelGGL(k_pack, dim3((kHid * kHid + 255) / 256), dim3(256), 0, n->st, n->p, n->nb);
            e = hipGetLastError();
        }
        lr *= lr_decay;
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pack_fused, dim3((2 * kFW2 + 255) / 256), dim3(256), 0, n->st, n->p, n->fw, n->fb);
        e = hipGetLastError();
    }
    std::vector<double> tot(std::max(epochs, 1), 0.0);
    if (e == hipSuccess && epochs > 0)
        e = hipMemcpyAsync(tot.data(), loss, sizeof(double) * epochs, hipMemcpyDeviceToHost, n->st);
    if (e == hipSuccess) e = hipStreamSynchronize(n->st);
    if (e == hipSuccess && loss_host)
        for (int ep = 0; ep < epochs; ++ep) loss_host[ep] = tot[ep] / ((double)n_batches * batch);
    hipFree(y);
    hipFree(loss);
    return e;
}

const int kNetParams = kNParams;

}  // namespace lmo
