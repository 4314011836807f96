// mlp.cpp -- the radiance-cache network on gfx950 matrix cores (BF16 operands,
// FP32 accumulation): fused forward, fused forward+backward (weight
// gradients), Adam, and the cache inference used by the renderer.
//
// Network: 64-wide input (42 features, zero padded), five hidden layers of 64
// with ReLU, 3 outputs, no biases.  Weights are stored row-major (out, in):
// W1..W5 (64 x 64) then W6 (3 x 64), 20672 values.
//
// Tiling: one wave owns 32 samples and computes H^T = W X^T with
// v_mfma_f32_32x32x16_bf16 (M = output features, N = samples, K = input
// features).  Operand layouts (lane l, h = l / 32):
//   A (32 x 16): lane holds A[l % 32][8h .. 8h + 7]
//   B (16 x 32): lane holds B[8h .. 8h + 7][l % 32]
//   D (32 x 32): lane holds D[8 (i / 4) + 4 h + i % 4][l % 32], i = 0..15
// A layer's D registers are fed to the next layer as its B operand as they
// are: B k-slot kappa = 16 ks + 8 h + j then holds hidden unit sigma(kappa),
// sigma = swap of bits 2 and 3.  The weights of layers 2..6 are staged into
// LDS with their input columns permuted by sigma, so no activation moves.
#include <hip/hip_runtime.h>
#include <atomic>

#include <string>

#include "mirt_internal.h"

namespace mirt {

#define HIP_TRY_M(x)                                                       \
    do {                                                                   \
        hipError_t err_ = (x);                                             \
        if (err_ != hipSuccess) {                                          \
            set_error(std::string(#x) + ": " + hipGetErrorString(err_));  \
            return RT_ERR_HIP;                                             \
        }                                                                  \
    } while (0)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef short short8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kW = 64;                     // width
constexpr int kLayerElems = kW * kW;
constexpr int kParams = 5 * kLayerElems + 3 * kW;   // 20672

// float -> bf16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ int swap23(int k) { return (k & ~12) | ((k & 4) << 1) | ((k & 8) >> 1); }

__device__ __forceinline__ f32x16 mfma(short8 a, short8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

__device__ __forceinline__ short8 lds8(const uint16_t* p) { return *reinterpret_cast<const short8*>(p); }

__device__ __forceinline__ f32x16 zero16() {
    f32x16 z;
#pragma unroll
    for (int i = 0; i < 16; ++i) z[i] = 0.0f;
    return z;
}

// ----------------------------------------------------------------------------
// weight staging into LDS
// ----------------------------------------------------------------------------
// Forward weights: Wf[layer][out m][k-slot kappa], layers 0..4 (64 rows) and
// the output layer (32 rows, rows >= 3 zero).  Layer 0 takes the input
// features in natural order; later layers read their inputs through sigma.
// Rows are kWp = 72 entries apart: a 16-byte operand read is served eight lanes
// at a time, and 144-byte rows put those eight lanes' rows on distinct banks
// (64-entry rows would put all eight on the same four).
constexpr int kWp = kW + 8;
constexpr int kFwdRows = 5 * kW + 32;
struct MlpLds {
    uint16_t wf[kFwdRows * kWp];
};

__device__ __forceinline__ uint2 ld4(const uint16_t* p) { return *reinterpret_cast<const uint2*>(p); }

// one unit = 8 consecutive k-slots of one row: two 8-byte reads (sigma keeps
// runs of four k-slots together) and one 16-byte LDS store.  w: 8-byte aligned.
__device__ void stage_forward(const uint16_t* __restrict__ w, uint16_t* wf) {
    for (int u = threadIdx.x; u < kFwdRows * 8; u += blockDim.x) {
        const int row = u >> 3, g = u & 7;
        const int layer = row >> 6, m = row & 63;
        const uint16_t* src = w + layer * kLayerElems + m * kW;
        uint2 a = make_uint2(0u, 0u), b = make_uint2(0u, 0u);
        if (layer == 0) {
            a = ld4(src + 8 * g);
            b = ld4(src + 8 * g + 4);
        } else if (layer < 5 || m < 3) {
            a = ld4(src + swap23(8 * g));
            b = ld4(src + swap23(8 * g + 4));
        }
        *reinterpret_cast<uint4*>(wf + row * kWp + 8 * g) = make_uint4(a.x, a.y, b.x, b.y);
    }
}

// ----------------------------------------------------------------------------
// forward through the hidden layers for one wave's 32 samples
// ----------------------------------------------------------------------------
// b[ks] (ks = 0..3) is the B operand (this lane's sample, k-slots 16ks+8h..+7).
// Layer output D (two 32-row tiles) is rounded to BF16 after ReLU and packed
// back into b as bop[ks][j] = D[ks / 2][8 (ks % 2) + j].
// ReLU and round to BF16 of d[base .. base + 7], packed as one B operand:
// rounding (nearest even, the hardware's packed conversion) keeps the sign, so
// the ReLU is applied after it as a signed 16-bit max with 0, which maps every
// negative value and -0 to +0 and leaves the rest unchanged.
__device__ __forceinline__ short8 relu_bf16x8(const f32x16& d, int base) {
    uint32_t u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bf16x2 v = {(__bf16)d[base + 2 * q], (__bf16)d[base + 2 * q + 1]};
        const s16x2 m = __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), (s16x2){0, 0});
        u[q] = __builtin_bit_cast(uint32_t, m);
    }
    return __builtin_bit_cast(short8, make_uint4(u[0], u[1], u[2], u[3]));
}

__device__ __forceinline__ void hidden_layer(const uint16_t* wl, short8 (&b)[4], int l) {
    const int h = l >> 5, r = l & 31;
    f32x16 d0 = zero16(), d1 = zero16();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        d0 = mfma(lds8(wl + r * kWp + 16 * ks + 8 * h), b[ks], d0);
        d1 = mfma(lds8(wl + (32 + r) * kWp + 16 * ks + 8 * h), b[ks], d1);
    }
    b[0] = relu_bf16x8(d0, 0);
    b[1] = relu_bf16x8(d0, 8);
    b[2] = relu_bf16x8(d1, 0);
    b[3] = relu_bf16x8(d1, 8);
}

__device__ __forceinline__ f32x16 output_layer(const uint16_t* w6, const short8 (&b)[4], int l) {
    const int h = l >> 5, r = l & 31;
    f32x16 d = zero16();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) d = mfma(lds8(w6 + r * kWp + 16 * ks + 8 * h), b[ks], d);
    return d;   // lanes 0..31: d[0..2] = y of sample (l % 32)
}

__device__ __forceinline__ void load_input(const uint16_t* __restrict__ x, int64_t sample, bool valid, int l,
                                           short8 (&b)[4]) {
    const int h = l >> 5;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        if (valid) {
            b[ks] = *reinterpret_cast<const short8*>(x + sample * kW + 16 * ks + 8 * h);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) b[ks][j] = 0;
        }
    }
}

constexpr int kFwdWaves = 8;         // waves per block of the inference kernel: two per SIMD
constexpr int kFwdBlocksPerCu = 1;   // ~240 registers per lane (the weights below) leave room for two waves per SIMD

// mode 0: y [n][3]; mode 1: acc[3 pix + c] += w_c * max(y_c, 0) (cache inference)
// Every lane holds its A operands of all six layers in registers (44 x 16 bytes,
// read once from the staged LDS copy), so the tile loop touches no LDS: per
// 32-sample tile it is 44 matrix-core instructions, the ReLU/BF16 conversions
// between them and the input read, whose next tile is fetched before the
// current one is computed.  The second wave on each SIMD overlaps its
// conversions and loads with this wave's matrix work.  In mode 1 the three
// float atomic adds per query (many queries share a pixel) take about as long
// as the network itself.
template <int MODE>
__global__ __launch_bounds__(64 * kFwdWaves) void k_mlp_forward(const uint16_t* __restrict__ w,
                                                                const uint16_t* __restrict__ x, int64_t n,
                                                                float* __restrict__ y, const uint32_t* count_p,
                                                                const uint32_t* __restrict__ pix,
                                                                const float* __restrict__ wt, float* __restrict__ acc) {
    __shared__ __attribute__((aligned(16))) MlpLds S;
    stage_forward(w, S.wf);
    __syncthreads();
    const int l = threadIdx.x & 63, h = l >> 5, r = l & 31;
    short8 wa[5][2][4], wo[4];
#pragma unroll
    for (int layer = 0; layer < 5; ++layer)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                wa[layer][mt][ks] = lds8(S.wf + (layer * kW + 32 * mt + r) * kWp + 16 * ks + 8 * h);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) wo[ks] = lds8(S.wf + (5 * kW + r) * kWp + 16 * ks + 8 * h);
    if (count_p) n = min((int64_t)*count_p, n);
    const int64_t tiles = (n + 31) / 32, stride = (int64_t)gridDim.x * kFwdWaves;
    int64_t t = (int64_t)blockIdx.x * kFwdWaves + (threadIdx.x >> 6);
    short8 b[4];
    if (t < tiles) load_input(x, t * 32 + r, t * 32 + r < n, l, b);
    for (; t < tiles; t += stride) {
        const int64_t s = t * 32 + r;
        const bool valid = s < n;
        short8 bn[4];
        if (t + stride < tiles) load_input(x, s + 32 * stride, s + 32 * stride < n, l, bn);
        // the accumulation target of this lane's sample, read before the matrix work hides its latency
        uint32_t p = 0;
        float w0 = 0.0f, w1 = 0.0f, w2 = 0.0f;
        if (MODE == 1 && l < 32 && valid) {
            p = pix[s];
            w0 = wt[3 * s + 0];
            w1 = wt[3 * s + 1];
            w2 = wt[3 * s + 2];
        }
#pragma unroll
        for (int layer = 0; layer < 5; ++layer) {
            f32x16 d0 = zero16(), d1 = zero16();
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                d0 = mfma(wa[layer][0][ks], b[ks], d0);
                d1 = mfma(wa[layer][1][ks], b[ks], d1);
            }
            b[0] = relu_bf16x8(d0, 0);
            b[1] = relu_bf16x8(d0, 8);
            b[2] = relu_bf16x8(d1, 0);
            b[3] = relu_bf16x8(d1, 8);
        }
        f32x16 d = zero16();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) d = mfma(wo[ks], b[ks], d);
        if (l < 32 && valid) {
            if (MODE == 0) {
                y[s * 3 + 0] = d[0];
                y[s * 3 + 1] = d[1];
                y[s * 3 + 2] = d[2];
            } else {
                atomicAdd(acc + 3 * p + 0, w0 * fmaxf(d[0], 0.0f));
                atomicAdd(acc + 3 * p + 1, w1 * fmaxf(d[1], 0.0f));
                atomicAdd(acc + 3 * p + 2, w2 * fmaxf(d[2], 0.0f));
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) b[q] = bn[q];
    }
}

// ----------------------------------------------------------------------------
// forward + backward: accumulates dW (FP32, natural layout) and the loss sum
// ----------------------------------------------------------------------------
// A training step (16,384 samples) is too small to fill the matrix cores: the
// kernel is bound by the latency of its dependent chain (weight staging, six
// forward and five backward layers, each a few matrix instructions with LDS
// round trips) and by the device atomics of dW.  What shortens the chain: the
// staging issues all of a thread's global reads before its LDS writes, the
// first group's features are read while the weights are staged, and the ReLU
// mask of g_z is a packed integer test on the BF16 activations with the
// hardware's packed conversion (38.9 -> 32.2 us per step).  A variant with
// every wave independent (no block barriers; each product also issued with its
// operands' roles swapped, so that the transposes dW needs come out of the
// matrix cores instead of LDS) ran its chain in 29.5 us but, adding every
// wave's dW separately, doubled the atomics to 57 us.
constexpr int kGradWaves = 2;   // waves per block of the training kernel (LDS budget); one 32-column dW tile each

static_assert(kGradWaves == 2, "each wave of the training kernel reduces one of the two 32-column dW tiles");

struct GradLds {
    uint16_t wf[kFwdRows * kWp];
    uint16_t wb[4 * kW * kWp];
    uint16_t wb6[kW * 16];
    short8 act[kGradWaves][6][4][64];      // per wave, per layer: each lane's packed operand (input, h_1..h_5)
    uint16_t gy[kGradWaves][32 * 32];      // per wave: [channel (32 rows, 3 used)][sample]
    uint16_t gz[kGradWaves][kW * 32];      // per wave: [feature][sample]
    uint16_t ht[kGradWaves][kW * 32];      // per wave: [feature][sample]
};

// g_z = bf16(g_h) where the layer's activation is positive, else +0, for the
// accumulator values g[base .. base + 7] against the packed activation chunk a
// (the same samples and features in the same register order).  A BF16 value is
// positive exactly when its bits, read as a signed 16-bit integer, are; the
// conversion is the hardware's packed one (nearest even).
__device__ __forceinline__ short8 masked_grad(const f32x16& g, int base, const short8& a) {
    uint32_t u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bf16x2 v = {(__bf16)g[base + 2 * q], (__bf16)g[base + 2 * q + 1]};
        const s16x2 act = {a[2 * q], a[2 * q + 1]};
        const s16x2 keep = act > (s16x2){0, 0};   // all ones where positive
        u[q] = __builtin_bit_cast(uint32_t, v) & __builtin_bit_cast(uint32_t, keep);
    }
    return __builtin_bit_cast(short8, make_uint4(u[0], u[1], u[2], u[3]));
}

// Forward weights as in stage_forward, and backward weights Wb[l][in m][k-slot
// kappa] = W_{l+1}[sigma(kappa)][m] for layers 1..4 (the products g_h_{l} =
// W_{l+1}^T g_z_{l+1}), rows kWp apart like the forward copy, plus the output
// layer's transpose Wb6[m][k] = W6[k][m] (k < 3, 16 columns).  One backward
// unit reads 8 consecutive columns m of a row j of W_{l+1} (16 bytes; sigma is
// its own inverse, so that row lands in k-slot sigma(j)).  Every global read
// of a thread is issued before its LDS writes (kStride threads; the trip
// counts are exact multiples), so the reads overlap.
template <int kStride>
__device__ void stage_grad_weights(const uint16_t* __restrict__ w, GradLds& S) {
    constexpr int kFwdUnits = kFwdRows * 8, kBwdUnits = 4 * kW * 8;
    static_assert(kFwdUnits % kStride == 0 && kBwdUnits % kStride == 0 && (kW * 16) % kStride == 0, "stride");
    {
        constexpr int kIt = kFwdUnits / kStride;
        uint2 a[kIt], b[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int u = threadIdx.x + it * kStride;
            const int row = u >> 3, g = u & 7;
            const int layer = row >> 6, m = row & 63;
            const uint16_t* src = w + layer * kLayerElems + m * kW;
            a[it] = make_uint2(0u, 0u);
            b[it] = make_uint2(0u, 0u);
            if (layer == 0) {
                a[it] = ld4(src + 8 * g);
                b[it] = ld4(src + 8 * g + 4);
            } else if (layer < 5 || m < 3) {
                a[it] = ld4(src + swap23(8 * g));
                b[it] = ld4(src + swap23(8 * g + 4));
            }
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int u = threadIdx.x + it * kStride;
            *reinterpret_cast<uint4*>(S.wf + (u >> 3) * kWp + 8 * (u & 7)) =
                make_uint4(a[it].x, a[it].y, b[it].x, b[it].y);
        }
    }
    {
        constexpr int kIt = kBwdUnits / kStride;
        uint4 v[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int u = threadIdx.x + it * kStride;
            const int li = u >> 9, j = (u >> 3) & 63, mg = u & 7;
            v[it] = *reinterpret_cast<const uint4*>(w + (li + 1) * kLayerElems + j * kW + 8 * mg);
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int u = threadIdx.x + it * kStride;
            const int li = u >> 9, j = (u >> 3) & 63, mg = u & 7;
            const uint32_t q[4] = {v[it].x, v[it].y, v[it].z, v[it].w};
            uint16_t* dst = S.wb + (li * kW + 8 * mg) * kWp + swap23(j);
#pragma unroll
            for (int i = 0; i < 8; ++i) dst[i * kWp] = (uint16_t)(q[i >> 1] >> (16 * (i & 1)));
        }
    }
    {
        constexpr int kIt = kW * 16 / kStride;
        uint16_t v[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int e = threadIdx.x + it * kStride, m = e / 16, k = e % 16;
            v[it] = k < 3 ? w[5 * kLayerElems + k * kW + m] : (uint16_t)0;
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) S.wb6[threadIdx.x + it * kStride] = v[it];
    }
}


// write a packed D-layout activation block to LDS as [feature][sample]
__device__ __forceinline__ void store_dlayout(uint16_t* dst, const short8 (&b)[4], int l) {
    const int h = l >> 5, r = l & 31;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int f = 32 * mt + 8 * (i >> 2) + 4 * h + (i & 3);
            dst[f * 32 + r] = (uint16_t)b[2 * mt + (i >> 3)][i & 7];
        }
}

// write the input operand (natural k-slots) to LDS as [feature][sample]
__device__ __forceinline__ void store_input(uint16_t* dst, const short8 (&b)[4], int l) {
    const int h = l >> 5, r = l & 31;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int j = 0; j < 8; ++j) dst[(16 * ks + 8 * h + j) * 32 + r] = (uint16_t)b[ks][j];
}

// dW[m][n] += sum over the block's samples (32 per wave) of A[m][s] B[n][s]
// (A rows m_rows, B rows 64; wave v's operands at a_fs + v a_stride and
// b_fs + v b_stride).  This wave reduces the 32-column tile nt of every row
// tile over all waves' samples, so each dW element takes one atomic add per
// block rather than one per wave.
__device__ __noinline__ void accumulate_dw(const uint16_t* a_fs, int a_stride, int m_rows, const uint16_t* b_fs,
                                           int b_stride, float* dw, int dw_rows, int l, int nt) {
    const int h = l >> 5, r = l & 31;
    for (int mt = 0; mt * 32 < m_rows; ++mt) {
        f32x16 d = zero16();
#pragma unroll
        for (int v = 0; v < kGradWaves; ++v)
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                d = mfma(lds8(a_fs + v * a_stride + (32 * mt + r) * 32 + 16 * ks + 8 * h),
                         lds8(b_fs + v * b_stride + (32 * nt + r) * 32 + 16 * ks + 8 * h), d);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = 32 * mt + 8 * (i >> 2) + 4 * h + (i & 3);
            if (m < dw_rows) atomicAdd(dw + m * kW + 32 * nt + r, d[i]);
        }
    }
}

__device__ __forceinline__ void load_act(const GradLds& S, int wave, int layer, int l, short8 (&b)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) b[q] = S.act[wave][layer][q][l];
}

__global__ __launch_bounds__(64 * kGradWaves) void k_mlp_grad(const uint16_t* __restrict__ w,
                                                              const uint16_t* __restrict__ x,
                                                              const float* __restrict__ target, int64_t n,
                                                              float inv_3n, const uint32_t* count_p,
                                                              int64_t count_base, float* __restrict__ dw,
                                                              float* __restrict__ loss_sum) {
    __shared__ __attribute__((aligned(16))) GradLds S;
    // samples [count_base, count_base + n) of a batch whose valid size is *count_p
    if (count_p) n = min(n, max((int64_t)0, (int64_t)*count_p - count_base));
    const int wave = threadIdx.x >> 6;
    const int l = threadIdx.x & 63, h = l >> 5, r = l & 31;
    const int64_t tiles = (n + 31) / 32;
    const int64_t groups = (tiles + kGradWaves - 1) / kGradWaves;
    // the first group's features are read while the weights are staged
    short8 b[4];
    {
        const int64_t s0 = ((int64_t)blockIdx.x * kGradWaves + wave) * 32 + r;
        load_input(x, s0, (int64_t)blockIdx.x < groups && s0 < n, l, b);
    }
    stage_grad_weights<64 * kGradWaves>(w, S);
    for (int e = threadIdx.x & 63; e < 32 * 32; e += 64) S.gy[wave][e] = 0;
    __syncthreads();
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {   // block-uniform loop
        const int64_t t = g * kGradWaves + wave;
        const int64_t s = t * 32 + r;
        const bool valid = s < n;
        // forward, keeping every layer's operand in this lane's LDS slots
        if (g != blockIdx.x) load_input(x, s, valid, l, b);
#pragma unroll
        for (int q = 0; q < 4; ++q) S.act[wave][0][q][l] = b[q];
        for (int k = 1; k < 6; ++k) {
            hidden_layer(S.wf + (k - 1) * kW * kWp, b, l);
#pragma unroll
            for (int q = 0; q < 4; ++q) S.act[wave][k][q][l] = b[q];
        }
        const f32x16 d = output_layer(S.wf + 5 * kW * kWp, b, l);
        // loss and g_y on lanes 0..31 (this lane's sample); g_y is BF16 like every product operand
        float gyv[3] = {0.0f, 0.0f, 0.0f};
        float lsum = 0.0f;
        if (h == 0 && valid) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float yv = d[c], tv = target[3 * s + c];
                const float den = yv * yv + 0.01f;
                const float e = yv - tv;
                lsum += e * e / den;
                gyv[c] = bf2f(f2bf(2.0f * e / den * inv_3n));
            }
        }
        for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
        if (l == 0 && lsum != 0.0f) atomicAdd(loss_sum, lsum);
        // dW6 = g_y^T h5
        if (h == 0)
            for (int c = 0; c < 3; ++c) S.gy[wave][c * 32 + r] = f2bf(gyv[c]);
        store_dlayout(S.ht[wave], b, l);
        __syncthreads();
        accumulate_dw(S.gy[0], 32 * 32, 32, S.ht[0], kW * 32, dw + 5 * kLayerElems, 3, l, wave);
        // g_h5 = W6^T g_y  (K = channels, padded to 16)
        short8 bgy;
#pragma unroll
        for (int j = 0; j < 8; ++j) bgy[j] = (short)(h == 0 && j < 3 ? f2bf(gyv[j]) : 0);
        f32x16 gh0 = mfma(lds8(S.wb6 + r * 16 + 8 * h), bgy, zero16());
        f32x16 gh1 = mfma(lds8(S.wb6 + (32 + r) * 16 + 8 * h), bgy, zero16());
        for (int L = 5; L >= 1; --L) {
            // g_z_L = bf16(g_h_L * [h_L > 0]), packed like the forward activations
            short8 hl[4], gz[4];
            load_act(S, wave, L, l, hl);
            gz[0] = masked_grad(gh0, 0, hl[0]);
            gz[1] = masked_grad(gh0, 8, hl[1]);
            gz[2] = masked_grad(gh1, 0, hl[2]);
            gz[3] = masked_grad(gh1, 8, hl[3]);
            __syncthreads();
            store_dlayout(S.gz[wave], gz, l);
            short8 hp[4];
            load_act(S, wave, L - 1, l, hp);
            if (L - 1 >= 1) store_dlayout(S.ht[wave], hp, l);
            else store_input(S.ht[wave], hp, l);
            __syncthreads();
            accumulate_dw(S.gz[0], kW * 32, 64, S.ht[0], kW * 32, dw + (L - 1) * kLayerElems, 64, l, wave);
            if (L > 1) {
                const uint16_t* wbl = S.wb + (L - 2) * kW * kWp;
                gh0 = zero16();
                gh1 = zero16();
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    gh0 = mfma(lds8(wbl + r * kWp + 16 * ks + 8 * h), gz[ks], gh0);
                    gh1 = mfma(lds8(wbl + (32 + r) * kWp + 16 * ks + 8 * h), gz[ks], gh1);
                }
            }
        }
        __syncthreads();
    }
}

// Adam with the step count in device memory (*step_p holds the steps already
// taken); k_mlp_step_inc advances it afterwards.  For frames replayed from a
// captured graph.
__global__ void k_mlp_adam_dev(float* __restrict__ w, uint16_t* __restrict__ wb, float* __restrict__ m,
                               float* __restrict__ v, float* __restrict__ g, int n, float lr, float b1, float b2,
                               float eps, const uint32_t* step_p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float t = (float)(*step_p + 1u);
    const float c1 = 1.0f / (1.0f - powf(b1, t)), c2 = 1.0f / (1.0f - powf(b2, t));
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
    g[i] = 0.0f;
}

__global__ void k_mlp_step_inc(uint32_t* step_p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step_p += 1u;
}

// Adam on FP32 master weights; refreshes the BF16 copy and clears the gradient.
__global__ void k_mlp_adam(float* __restrict__ w, uint16_t* __restrict__ wb, float* __restrict__ m,
                           float* __restrict__ v, float* __restrict__ g, int n, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
    g[i] = 0.0f;
}

// Health of the learned form after a frame's training steps: bit 0 of *health
// when one of the steps' loss sums (float bits in loss_bits[0 .. steps)) is
// not finite, bit 1 when a master weight or an Adam moment is not.  Bits are
// only ever added; rt_cache_init clears them.  One thread per parameter.
__global__ __launch_bounds__(256) void k_mlp_health(const float* __restrict__ w, const float* __restrict__ m,
                                                    const float* __restrict__ v, int n,
                                                    const uint32_t* __restrict__ loss_bits, int steps,
                                                    uint32_t* health) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t bad = 0u;
    if (i < n && (!isfinite(w[i]) || !isfinite(m[i]) || !isfinite(v[i]))) bad = 2u;
    if (i < steps && !isfinite(__uint_as_float(loss_bits[i]))) bad |= 1u;
    if (bad) atomicOr(health, bad);
}

// blocks for `tiles` 32-sample tiles at per_block tiles per round, at most per_cu resident blocks per CU
static int grid_for(int64_t tiles, int per_block, int per_cu) {
    static std::atomic<int> cu_count[64];   // per device, 0 = not queried yet
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) {
        cus = cu_count[dev].load(std::memory_order_relaxed);
        if (cus <= 0) {
            int n = 0;
            cus = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0 ? n : 256;
            cu_count[dev].store(cus, std::memory_order_relaxed);
        }
    }
    const int64_t need = (tiles + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)cus * per_cu));
}

// internal launchers used by the renderer's cache frames
rt_status mlp_infer_launch(const uint16_t* w, const uint16_t* x, int64_t cap, const uint32_t* count, const uint32_t* pix,
                           const float* wt, float* acc, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_forward<1>, dim3(grid_for((cap + 31) / 32, kFwdWaves, kFwdBlocksPerCu)),
                       dim3(64 * kFwdWaves), 0, st, w, x, cap, nullptr, count,
                       pix, wt, acc);
    HIP_TRY_M(hipGetLastError());
    return RT_OK;
}

rt_status mlp_grad_launch(const uint16_t* w, const uint16_t* x, const float* target, int64_t n, int64_t n_total,
                          const uint32_t* count, int64_t count_base, float* dw, float* loss, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(grid_for((n + 31) / 32, kGradWaves, 4)), dim3(64 * kGradWaves), 0, st, w, x,
                       target, n, 1.0f / (3.0f * (float)n_total), count, count_base, dw, loss);
    HIP_TRY_M(hipGetLastError());
    return RT_OK;
}

rt_status mlp_health_launch(const float* w, const float* m, const float* v, const uint32_t* loss_bits, int steps,
                           uint32_t* health, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_health, dim3((kParams + 255) / 256), dim3(256), 0, st, w, m, v, kParams, loss_bits,
                       steps, health);
    HIP_TRY_M(hipGetLastError());
    return RT_OK;
}

rt_status mlp_adam_dev_launch(float* w, uint16_t* wb, float* m, float* v, float* g, const uint32_t* step_p, float lr,
                              float b1, float b2, float eps, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_adam_dev, dim3((kParams + 255) / 256), dim3(256), 0, st, w, wb, m, v, g, kParams, lr, b1,
                       b2, eps, step_p);
    hipLaunchKernelGGL(k_mlp_step_inc, dim3(1), dim3(64), 0, st, const_cast<uint32_t*>(step_p));
    HIP_TRY_M(hipGetLastError());
    return RT_OK;
}

rt_status mlp_adam_launch(float* w, uint16_t* wb, float* m, float* v, float* g, int32_t t, float lr, float b1, float b2,
                          float eps, hipStream_t st) {
    const float c1 = 1.0f / (1.0f - powf(b1, (float)t)), c2 = 1.0f / (1.0f - powf(b2, (float)t));
    hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0, st, w, wb, m, v, g, kParams, lr, b1, b2,
                       eps, c1, c2);
    HIP_TRY_M(hipGetLastError());
    return RT_OK;
}

}  // namespace mirt

using namespace mirt;

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

extern "C" {

int32_t rt_mlp_num_params(void) { return kParams; }

rt_status rt_mlp_forward(const uint16_t* w_bf16, const uint16_t* x_bf16, int64_t n, float* y, void* stream) {
    if (n < 0 || (n > 0 && (!w_bf16 || !x_bf16 || !y || !aligned16(w_bf16) || !aligned16(x_bf16)))) {
        set_error("rt_mlp_forward: invalid argument (NULL pointer, n < 0 or w_bf16/x_bf16 not 16-byte aligned)");
        return RT_ERR_INVALID_ARG;
    }
    if (n == 0) return RT_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_mlp_forward<0>, dim3(grid_for((n + 31) / 32, kFwdWaves, kFwdBlocksPerCu)),
                       dim3(64 * kFwdWaves), 0, st, w_bf16, x_bf16, n, y,
                       nullptr, nullptr, nullptr, nullptr);
    HIP_TRY_M(hipGetLastError());
    return RT_OK;
}

rt_status rt_mlp_grad(const uint16_t* w_bf16, const uint16_t* x_bf16, const float* target, int64_t n, int64_t n_total,
                      float* dw, float* loss_sum, void* stream) {
    if (n < 0 || n_total <= 0 ||
        (n > 0 && (!w_bf16 || !x_bf16 || !target || !dw || !loss_sum || !aligned16(w_bf16) || !aligned16(x_bf16)))) {
        set_error("rt_mlp_grad: invalid argument (NULL pointer, n < 0, n_total <= 0 or w_bf16/x_bf16 not 16-byte "
                  "aligned)");
        return RT_ERR_INVALID_ARG;
    }
    if (n == 0) return RT_OK;
    return mlp_grad_launch(w_bf16, x_bf16, target, n, n_total, nullptr, 0, dw, loss_sum,
                           static_cast<hipStream_t>(stream));
}

rt_status rt_mlp_adam(float* w, uint16_t* w_bf16, float* m, float* v, float* grad, int32_t step, float lr, float b1,
                      float b2, float eps, void* stream) {
    if (!w || !w_bf16 || !m || !v || !grad || step < 1) {
        set_error("rt_mlp_adam: invalid argument");
        return RT_ERR_INVALID_ARG;
    }
    return mlp_adam_launch(w, w_bf16, m, v, grad, step, lr, b1, b2, eps, static_cast<hipStream_t>(stream));
}

}  // extern "C"
