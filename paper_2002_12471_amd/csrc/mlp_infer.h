// The fused inference kernel of the scatter-surrogate network (8 -> 128 ->
// 128 -> 128 -> 1, GELU in its tanh form, bf16 MFMA with FP32 accumulation),
// as a template over where its inputs come from and where its outputs go:
// a sample array (lmosem_net_forward) or the (event, pixel) pairs of a
// learned-scatter sub-iteration, whose bf16 inputs a kernel of their own
// formed beforehand.
//
// Src provides  __device__ uint2 inputs(int64_t p, int g) const : inputs
// 4g .. 4g+3 of sample p (g = 0, 1) rounded to bf16, two to a word (the
// lower-numbered input in the low half);  __device__ C out_base(int64_t p0)
// const : for a wave's first sample p0 (the same in every lane), whatever
// locates its output; and  __device__ void output(const C &c, int i, float y)
// const : the network's output for sample p0 + i (0 <= i < 32).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lmo {

constexpr int kIn = 8, kInPad = 16, kHid = 128;
typedef float f32x4 __attribute__((ext_vector_type(4)));

// One kernel for the whole network.  The hidden units are the MFMA rows and
// the samples the columns (Z^T[out][b] = sum_in W^T[out][in] H^T[in][b]), with
// v_mfma_f32_16x16x32_bf16: a 16-row output block comes back with row
// 4 (l/16) + v in register v of lane l (sample l % 16).  A 32-wide k-block over
// inputs h0..h0+31 is permuted so that lane group g = l/16 holds inputs
// {h0 + 4g .. +3} and {h0 + 16 + 4g .. +3} (the same permutation in the A and B
// operands leaves the product unchanged): exactly the rows lane l holds of the
// previous layer's output blocks 2 kb and 2 kb + 1, so activations stay in
// registers from layer to layer.  The output row is one more MFMA product
// whose A operand has W4 in its first row and zeros elsewhere (wasted matrix
// rows are cheaper than 128 widenings and FMAs per sample on the vector ALU,
// which bounds the kernel).  The weights, pre-permuted into A-operand lane
// order, the biases and the output row sit in LDS (80 KB), shared by the
// sixteen waves of one workgroup per CU; each wave takes 32 samples per step
// (118 VGPRs, four waves per SIMD).
//
// Every hidden pre-activation is carried at a quarter of its value, s = z/4
// (layer 1 has W1/4 and b1/4; every layer's biases are quartered), and each
// layer stores g = gelu(4 s)/4, so that the next layer's products with the
// plain weights give the next s; the output is 4 (W4 . g3) + b4.  Powers of
// two scale exactly in bf16, so this is the unscaled network with its
// activations rounded to bf16.  The GELU's sigmoid factor is a polynomial in
// s^2 fitted on |s| <= 1 and evaluated in packed fp16 arithmetic, two
// activations per instruction and no transcendental; beyond |s| = 1 it is
// saturated to 0 or 1 by the clamp modifier of its last step (the tanh form
// is within 7e-5 of that beyond |z| = 4); the product s times that factor is
// formed in FP32 from the two fp16 values and rounded once, to bf16.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
constexpr int kFW1 = 8 * 64 * 8;                 // layer 1 A operands [ob][lane][8]
constexpr int kFW2 = 8 * 4 * 64 * 8;             // hidden layers [ob][kb][lane][8]
constexpr int kFWTotal = kFW1 + 2 * kFW2;        // bf16 elements
constexpr int kFB = 4 * kHid + 1;                // b1 b2 b3, w4 (bf16 values), b4
constexpr int kFusedNB = 2;                      // 16-sample column blocks per wave
constexpr int kFusedWaves = 16;                  // one workgroup per CU: 4 waves per SIMD share one LDS copy
constexpr int kFusedThreads = 64 * kFusedWaves;
constexpr int kFusedTile = kFusedWaves * 16 * kFusedNB;   // samples per workgroup step
constexpr float kActScale = 0.25f;               // s = z / 4

__device__ __host__ inline int perm_k(int g, int i) { return i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4); }

__device__ inline f16x2 clamp01(f16x2 x) {
    return __builtin_elementwise_min(__builtin_elementwise_max(x, f16x2{0, 0}), f16x2{1, 1});
}

// The GELU's sigmoid factor for quarter-scale pre-activations, N pairs side
// by side (independent chains, interleaved step by step): the factor of the
// tanh form, sigma(2 sqrt(2/pi) (z + 0.044715 z^3)) at z = 4 s, is
// 1/2 + s P(s^2 - 1/2), P of degree 6 with fp16 coefficients fitted
// (weighted least squares on |s| times the error, each coefficient rounded
// to fp16 before the lower ones are refitted; gelu_poly_fit.py beside this
// file regenerates them) on |s| <= 1: s times it is within 5e-4 of
// gelu(4 s)/4, fp16 arithmetic included.  t = s^2 - 1/2 is one fused
// multiply-add with no clamp: past |s| = 1, P (positive and increasing there,
// +inf once s^2 leaves fp16's range) makes |s P| exceed 1/2, and the clamp of
// the last step saturates the factor to 0 or 1; the fit script checks this
// in fp16 arithmetic for every fp16 value of s.
template <int N>
__device__ inline void gelu_factor(const f16x2 (&s)[N], f16x2 (&S)[N]) {
    constexpr _Float16 c[7] = {0.7041015625f16, -0.67626953125f16, 0.88525390625f16, -1.1181640625f16,
                               1.5205078125f16, -2.162109375f16,   1.6064453125f16};
    f16x2 t[N], q[N];
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] = __builtin_elementwise_fma(s[i], s[i], f16x2{-0.5f16, -0.5f16});
#pragma unroll
    for (int i = 0; i < N; ++i) q[i] = __builtin_elementwise_fma(f16x2{c[6], c[6]}, t[i], f16x2{c[5], c[5]});
#pragma unroll
    for (int k = 4; k >= 0; --k)
#pragma unroll
        for (int i = 0; i < N; ++i) q[i] = __builtin_elementwise_fma(q[i], t[i], f16x2{c[k], c[k]});
#pragma unroll
    for (int i = 0; i < N; ++i) S[i] = clamp01(__builtin_elementwise_fma(s[i], q[i], f16x2{0.5f16, 0.5f16}));
}

// g = s S(s) in FP32 from fp16 s and S (one mixed-precision FMA each),
// two of them rounded to bf16 together
__device__ inline bf16x2 gelu_out(f16x2 s, f16x2 S) {
    return __builtin_convertvector(f32x2{__builtin_fmaf((float)S[0], (float)s[0], 0.0f),
                                         __builtin_fmaf((float)S[1], (float)s[1], 0.0f)},
                                   bf16x2);
}

// the activations of one 16-row output block of each column block (four
// FP32 accumulators of one sample each) as elements 4h .. 4h+3 of the
// next layer's B operands
__device__ inline void gelu_block(const f32x4 (&acc)[kFusedNB], bf16x8 (&dst)[kFusedNB], int h) {
    f16x2 v[2 * kFusedNB], S[2 * kFusedNB];
#pragma unroll
    for (int nb = 0; nb < kFusedNB; ++nb) {
        v[2 * nb] = __builtin_convertvector(f32x2{acc[nb][0], acc[nb][1]}, f16x2);
        v[2 * nb + 1] = __builtin_convertvector(f32x2{acc[nb][2], acc[nb][3]}, f16x2);
    }
    gelu_factor(v, S);
#pragma unroll
    for (int nb = 0; nb < kFusedNB; ++nb) {
        const bf16x2 lo = gelu_out(v[2 * nb], S[2 * nb]), hi = gelu_out(v[2 * nb + 1], S[2 * nb + 1]);
        dst[nb][4 * h + 0] = lo[0];
        dst[nb][4 * h + 1] = lo[1];
        dst[nb][4 * h + 2] = hi[0];
        dst[nb][4 * h + 3] = hi[1];
    }
}

// bias-initialised accumulators of output block ob for this lane's rows
__device__ inline f32x4 bias4(const float *b, int ob, int g) {
    return *reinterpret_cast<const f32x4 *>(b + 16 * ob + 4 * g);
}

// one 128 -> 128 layer with GELU, activations in and out as B operands
__device__ inline void hidden_layer(const bf16x8 *__restrict__ w, const float *__restrict__ b, int lane, int g,
                                    bf16x8 (&act)[4][kFusedNB]) {
    bf16x8 nxt[4][kFusedNB];
#pragma unroll
    for (int ob = 0; ob < 8; ++ob) {
        f32x4 acc[kFusedNB];
        const f32x4 bv = bias4(b, ob, g);
#pragma unroll
        for (int nb = 0; nb < kFusedNB; ++nb) acc[nb] = bv;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const bf16x8 a = w[(ob * 4 + kb) * 64 + lane];
#pragma unroll
            for (int nb = 0; nb < kFusedNB; ++nb)
                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, act[kb][nb], acc[nb], 0, 0, 0);
        }
        gelu_block(acc, nxt[ob >> 1], ob & 1);
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int nb = 0; nb < kFusedNB; ++nb) act[kb][nb] = nxt[kb][nb];
}

template <class Src>
__global__ __launch_bounds__(kFusedThreads) void k_mlp_infer(const uint16_t *__restrict__ fw,
                                                             const float *__restrict__ fb, Src src, int64_t n) {
    __shared__ __attribute__((aligned(16))) uint16_t s_w[kFWTotal];
    __shared__ __attribute__((aligned(16))) float s_b[kFB + 3];
    __shared__ __attribute__((aligned(16))) __bf16 s_w4[4 * 64 * 8];
    {
        const uint4 *w_src = reinterpret_cast<const uint4 *>(fw);
        uint4 *dst = reinterpret_cast<uint4 *>(s_w);
        for (int i = threadIdx.x; i < kFWTotal / 8; i += kFusedThreads) dst[i] = w_src[i];
        for (int i = threadIdx.x; i < kFB; i += kFusedThreads) s_b[i] = fb[i];
        // the output row as the A operand of an MFMA whose first row is W4
        // (every other row zero), k-blocks permuted as the hidden layers' are;
        // the stored W4 values are bf16 already
        for (int i = threadIdx.x; i < 4 * 64 * 8; i += kFusedThreads) {
            const int kb = i >> 9, l = (i >> 3) & 63, e = i & 7;
            s_w4[i] = (l & 15) == 0 ? (__bf16)fb[3 * kHid + 32 * kb + perm_k(l >> 4, e)] : (__bf16)0.0f;
        }
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int g = lane >> 4, r = lane & 15;
    const bf16x8 *w1 = reinterpret_cast<const bf16x8 *>(s_w);
    const bf16x8 *w2 = reinterpret_cast<const bf16x8 *>(s_w + kFW1);
    const bf16x8 *w3 = reinterpret_cast<const bf16x8 *>(s_w + kFW1 + kFW2);
    const int64_t n_tiles = (n + kFusedTile - 1) / kFusedTile;
    // this lane's inputs of a tile's samples (lane groups 0 and 1 hold
    // features 0..3 and 4..7; every other slot is zero), read one tile ahead
    // so that their latency passes under the current tile's layers
    uint2 in_next[kFusedNB];
    auto read_inputs = [&](int64_t tile) {
        const int64_t base = tile * kFusedTile + wave * 16 * kFusedNB;
#pragma unroll
        for (int nb = 0; nb < kFusedNB; ++nb) {
            const int64_t p = base + 16 * nb + r;
            in_next[nb] = g < 2 && p < n ? src.inputs(p, g) : uint2{0u, 0u};
        }
    };
    if ((int64_t)blockIdx.x < n_tiles) read_inputs(blockIdx.x);
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        // keep the weight reads inside the loop (hoisting them would need
        // 288 registers)
        __asm__ volatile("" ::: "memory");
        const int64_t base = tile * kFusedTile + wave * 16 * kFusedNB;
        // layer 1: the inputs as B operands
        bf16x8 xin[kFusedNB];
#pragma unroll
        for (int nb = 0; nb < kFusedNB; ++nb)
            xin[nb] = __builtin_bit_cast(bf16x8, uint4{in_next[nb].x, in_next[nb].y, 0u, 0u});
        if (tile + gridDim.x < n_tiles) read_inputs(tile + gridDim.x);
        bf16x8 act[4][kFusedNB];
#pragma unroll
        for (int ob = 0; ob < 8; ++ob) {
            const bf16x8 a = w1[ob * 64 + lane];
            const f32x4 bv = bias4(s_b, ob, g);
            f32x4 acc[kFusedNB];
#pragma unroll
            for (int nb = 0; nb < kFusedNB; ++nb) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, xin[nb], bv, 0, 0, 0);
            gelu_block(acc, act[ob >> 1], ob & 1);
        }
        hidden_layer(w2, s_b + kHid, lane, g, act);
        hidden_layer(w3, s_b + 2 * kHid, lane, g, act);
        // output row on the MFMA: row 0 of the product holds y, in register 0
        // of lanes 0-15 (sample r of each 16-sample block)
        const bf16x8 *w4 = reinterpret_cast<const bf16x8 *>(s_w4);
        f32x4 o[kFusedNB];
#pragma unroll
        for (int nb = 0; nb < kFusedNB; ++nb) o[nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const bf16x8 a = w4[kb * 64 + lane];
#pragma unroll
            for (int nb = 0; nb < kFusedNB; ++nb) o[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, act[kb][nb], o[nb], 0, 0, 0);
        }
        const auto oc = src.out_base(base);
#pragma unroll
        for (int nb = 0; nb < kFusedNB; ++nb) {
            const int i = 16 * nb + r;
            if (g == 0 && i < n - base) src.output(oc, i, fmaf(1.0f / kActScale, o[nb][0], s_b[4 * kHid]));
        }
    }
}


}  // namespace lmo
