// Learned radiance cache on gfx950: parameter initialisation, inference
// operands, MFMA inference (BF16 and FP8 E4M3) and BF16 training (forward,
// backward, ordered gradient reduction, Adam, usability state).
//
// Inference keeps the network in registers and LDS: each wave loads the
// weight fragments once and then streams tiles of 32 samples, the samples
// on the N side of every product, so a layer's accumulators become the next
// layer's B operand without leaving the registers (see the slot permutation
// in gi_mlp.hpp).  BF16 runs on the 32x32x16 instruction, FP8 on the
// 32x32x64 one.
//
// Training (2^14..2^16 samples per step, ~0.6 GFLOP) runs on the matrix cores
// as well: one workgroup per 64 samples computes the forward pass, the loss
// gradient, the backward pass and its partial weight gradient; two more
// kernels sum the partials in a fixed order (groups of 16 workgroups, then
// the groups), so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "gi.h"
#include "gi_device.hpp"
#include "gi_mlp.hpp"

using namespace gi;
using namespace gi::mlp;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kInferBlock = 256;
constexpr float kFltMax = 3.40282347e38f;
constexpr int kStats = 16;             // per-workgroup statistics after the gradient
constexpr int kPartStride = 17792;     // >= kParams + kStats, multiple of 64
constexpr int kHdr = 64;               // workspace header words
constexpr float kFp8Max = 448.0f;

// statistics slots
enum : int { kStLoss = 0, kStErrNum = 1, kStErrDen = 2, kStNonFinite = 3, kStAmax0 = 4 };

gi_status launched_mlp() { return hipGetLastError() == hipSuccess ? GI_OK : GI_ERR_LAUNCH; }
hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

__device__ __forceinline__ float bf16_round(float x) { return (float)(__bf16)x; }

__device__ __forceinline__ float comp(float4 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

// a lane's input point of tile t (zero past the end)
__device__ __forceinline__ float4 tile_input(const float4 *src, uint32_t t, uint32_t ntiles, int s, uint32_t n)
{
    if (t < ntiles) {
        const uint32_t idx = t * 32u + (uint32_t)s;
        if (idx < n) return src[idx];
    }
    return make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// sin and cos of the doubled angle
__device__ __forceinline__ void double_angle(float s, float c, float &s2, float &c2)
{
    s2 = (s + s) * c;
    c2 = __builtin_fmaf(c, c, -(s * s));
}

// The 13 features of one coordinate v: v, then sin and cos of 2^j pi v for
// j = 0..5.  j = 0 and j = 3 come from the hardware sine and cosine (argument
// in revolutions, v 2^(j-1) reduced exactly to [0, 1) by fract), the others
// by one or two angle doublings each, which at most quadruples the sine's
// own error: a few 1e-7, far below a BF16 or FP8 operand's spacing.
__device__ __forceinline__ void encode13(float v, float *f)
{
    float sn[6], cs[6];
    const float x0 = __builtin_amdgcn_fractf(v * 0.5f), x3 = __builtin_amdgcn_fractf(v * 4.0f);
    sn[0] = sin_rev(x0);
    cs[0] = cos_rev(x0);
    sn[3] = sin_rev(x3);
    cs[3] = cos_rev(x3);
    double_angle(sn[0], cs[0], sn[1], cs[1]);
    double_angle(sn[1], cs[1], sn[2], cs[2]);
    double_angle(sn[3], cs[3], sn[4], cs[4]);
    double_angle(sn[4], cs[4], sn[5], cs[5]);
    f[0] = v;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        f[1 + 2 * j] = sn[j];
        f[2 + 2 * j] = cs[j];
    }
}

__device__ __forceinline__ int layer_of_frag(int f)
{
    return f < kFrag0[1] ? 0 : (f < kFrag0[2] ? 1 : (f < kFrag0[3] ? 2 : (f < kFrag0[4] ? 3 : 4)));
}

// weight column feeding operand slot (k-step c, lane half h, operand v) of layer L
__device__ __forceinline__ int frag_column(int L, int c, int h, int v)
{
    return L == 0 ? l0_feature(h, 8 * c + v) : swap23(16 * c + 8 * h + v);
}

// --------------------------------------------------------------------------
// initialisation and inference operands
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mlp_init(gi_mlp m, uint64_t seed)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < (int)kStateWords) m.state[p] = 0u;
    if (p >= kParams) return;
    int L = 0;
    while (L < kLayers - 1 && p >= kOffW[L + 1]) ++L;
    float val = 0.0f;
    if (p < kOffB[L]) {
        const float bound = sqrtf(6.0f / (float)kIn[L]);
        const float u = u01(philox(seed, (uint32_t)p, 0u, 12u, 0u).x);
        val = (2.0f * u - 1.0f) * bound;
    }
    m.params[p] = val;
    m.adam_m[p] = 0.0f;
    m.adam_v[p] = 0.0f;
    if (m.ema) m.ema[p] = 0.0f;
}

// the parameters inference uses: the bias-corrected average when present
struct InferSrc {
    const float *p;
    float scale;
};

__device__ __forceinline__ InferSrc infer_src(const gi_mlp &m)
{
    const uint32_t t = m.state[GI_MLP_STATE_STEPS];
    if (m.ema && t > 0u) return InferSrc{m.ema, 1.0f / (1.0f - powf(m.ema_decay, (float)t))};
    return InferSrc{m.params, 1.0f};
}

// FP32 biases after the fragments (one thread per slot)
__device__ __forceinline__ void write_bias(const gi_mlp &m, const InferSrc &src, int i)
{
    const int L = i < 256 ? i >> 6 : 4, u = i < 256 ? (i & 63) : i - 256;
    const float b = u < kOut[L] ? src.p[kOffB[L] + u] * src.scale : 0.0f;
    reinterpret_cast<float *>(reinterpret_cast<uint8_t *>(m.weights) + kBiasOff)[i] = b;
}

// BF16 fragments: element i = (f * 64 + lane) * 8 + v
__global__ void __launch_bounds__(256) k_mlp_prepare_bf16(gi_mlp m)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const InferSrc src = infer_src(m);
    if (i < kBiasSlots) write_bias(m, src, i);
    if (i >= kFrags * 64 * 8) return;
    const int f = i >> 9, l = (i >> 3) & 63, v = i & 7;
    const int L = layer_of_frag(f), r = f - kFrag0[L];
    const int t = r / kSteps[L], c = r % kSteps[L];
    const int row = 32 * t + (l & 31), k = frag_column(L, c, l >> 5, v);
    float w = 0.0f;
    if (row < kOut[L] && k >= 0 && k < kIn[L]) w = src.p[kOffW[L] + row * kIn[L] + k] * src.scale;
    reinterpret_cast<__bf16 *>(m.weights)[i] = (__bf16)w;
}

// FP8 weight scales: amax|W_L| / 448 (1 for an all-zero matrix)
// FP8 per-layer scale: the smallest power of two s with amax <= 448 s (1 for
// a tensor without range).  The candidate from the quotient's exponent is
// corrected by exact comparisons (448 s is exact), so the rule does not
// depend on how amax / 448 rounds.  Powers of two make the ratio of two
// layers' scales an exponent the scaled matrix instruction applies.
__device__ __forceinline__ float fp8_scale(float amax)
{
    if (!(amax > 0.0f && amax < kInf)) return 1.0f;
    int e;
    frexpf(amax / kFp8Max, &e);
    float s = ldexpf(1.0f, e);
    while (amax > kFp8Max * s) s *= 2.0f;
    while (amax <= 0.5f * kFp8Max * s) s *= 0.5f;
    return s;
}

// the smallest power of two >= x (x > 0 finite), else 1
__device__ __forceinline__ float pow2_at_least(float x)
{
    if (!(x > 0.0f && x < kInf)) return 1.0f;
    int e;
    frexpf(x, &e);
    float s = ldexpf(1.0f, e);
    while (x > s) s *= 2.0f;
    while (x <= 0.5f * s) s *= 0.5f;
    return s;
}

// log2 of a power of two
__device__ __forceinline__ int exp2_of(float pow2)
{
    int e;
    frexpf(pow2, &e);
    return e - 1;
}

__global__ void __launch_bounds__(256) k_mlp_wscale(gi_mlp m)
{
    __shared__ float red[256];
    const int L = blockIdx.x, t = threadIdx.x, cnt = kIn[L] * kOut[L];
    const InferSrc src = infer_src(m);
    float a = 0.0f;
    for (int i = t; i < cnt; i += 256) a = fmaxf(a, fabsf(src.p[kOffW[L] + i] * src.scale));
    red[t] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) red[t] = fmaxf(red[t], red[t + o]);
        __syncthreads();
    }
    if (t == 0) m.scales[L] = fp8_scale(red[0]);
}

__device__ __forceinline__ uint32_t fp8_byte(float x)
{
    x = fminf(fmaxf(x, -kFp8Max), kFp8Max);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xFFu;
}

// FP8 operands for the K = 64 instruction (v_mfma_scale_f32_32x32x64_f8f6f4):
// lane l of a fragment holds row l % 32 of a 32-row output tile and the 32
// consecutive K slots 32 (l / 32) + b, one byte each.  Eleven fragments
// (byte (f * 64 + l) * 32 + b): f = 2 p + t layer 0's tile t, part p (part
// 0: slots b = features 39 h + b of the half-wave h = l / 32; part 1: slots
// b < 7 = features 39 h + 32 + b, the rest zero), f = 4 + 2 (L - 1) + t
// hidden layer L tile t, f = 10 the output layer.  Hidden slot k = 32 h + b
// takes unit 32 (b >> 4) + 8 ((b >> 2) & 3) + 4 h + (b & 3): the previous
// layer's accumulator 4a + b' of tile t sits in lane half h as unit 32 t +
// 8 a + 4 h + b', so byte b of a lane's operand is simply accumulator b of
// the first tile, then of the second.
constexpr int kFp8Frags = 11;
static_assert(kFp8Frags * 64 * 32 <= kBiasOff, "FP8 operands fit the fragment area");

__host__ __device__ constexpr int k64_unit(int h, int b)
{
    return 32 * (b >> 4) + 8 * ((b >> 2) & 3) + 4 * h + (b & 3);
}

__global__ void __launch_bounds__(256) k_mlp_prepare_fp8(gi_mlp m)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const InferSrc src = infer_src(m);
    if (i < kBiasSlots) write_bias(m, src, i);
    if (i >= kFp8Frags * 64 * 32) return;
    const int f = i >> 11, l = (i >> 5) & 63, b = i & 31, h = l >> 5;
    int L, t, k;
    if (f < 4) {
        L = 0;
        t = f & 1;
        k = (f >> 1) == 0 ? 39 * h + b : (b < 7 ? 39 * h + 32 + b : -1);
    } else {
        L = f < 10 ? 1 + ((f - 4) >> 1) : 4;
        t = f < 10 ? (f - 4) & 1 : 0;
        k = k64_unit(h, b);
    }
    const int row = 32 * t + (l & 31);
    float w = 0.0f;
    if (row < kOut[L] && k >= 0 && k < kIn[L]) w = src.p[kOffW[L] + row * kIn[L] + k] * src.scale / m.scales[L];
    reinterpret_cast<uint8_t *>(m.weights)[i] = (uint8_t)fp8_byte(w);
}

// --------------------------------------------------------------------------
// inference
// --------------------------------------------------------------------------
__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma(long a, long b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, b, c, 0, 0, 0);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// two floats -> one register of two BF16 (one v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pk_bf16(float a, float b)
{
    bf16x2 p = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, p);
}

// ReLU on two BF16 bit patterns: as signed 16-bit integers every negative
// value (sign bit set) is below zero, so max(x, 0) clears exactly those;
// rounding and ReLU commute.  Written as the instruction itself (an ALU
// operation, no memory access): expressed as a vector max, the compiler
// splits the preceding pair conversion into two conversions and a permute.
__device__ __forceinline__ uint32_t relu_pk(uint32_t u)
{
    uint32_t r;
    asm("v_pk_max_i16 %0, %1, 0" : "=v"(r) : "v"(u));
    return r;
}

__device__ __forceinline__ bf16x8 to_bf16(f32x8 x)
{
    u32x4 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = pk_bf16(x[2 * i], x[2 * i + 1]);
    return __builtin_bit_cast(bf16x8, r);
}

// accumulators 8*part .. 8*part+7 as a BF16 operand, with ReLU
__device__ __forceinline__ bf16x8 relu_operand(const f32x16 &a, int part)
{
    u32x4 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = relu_pk(pk_bf16(a[8 * part + 2 * i], a[8 * part + 2 * i + 1]));
    return __builtin_bit_cast(bf16x8, r);
}

// accumulators of a 32-row tile initialised with the bias of rows 8a+4h+b
__device__ __forceinline__ f32x16 bias_tile(const float *b, int h)
{
    f32x16 c;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        float4 q = *reinterpret_cast<const float4 *>(b + 8 * a + 4 * h);
        c[4 * a + 0] = q.x;
        c[4 * a + 1] = q.y;
        c[4 * a + 2] = q.z;
        c[4 * a + 3] = q.w;
    }
    return c;
}

__global__ void __launch_bounds__(kInferBlock) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_mlp_infer_bf16(gi_mlp m, uint32_t n, const float4 *pos, const float4 *nrm, float4 *out, int gate)
{
    using FT = bf16x8;
    if (gate && !mlp_selected(m)) return;   // uniform over the grid
    // biases: layers 0-3 at 64 L, layer 4 at 256 padded to 32 rows
    __shared__ __attribute__((aligned(16))) float sb[kBiasSlots];
    const float *bias = reinterpret_cast<const float *>(reinterpret_cast<const uint8_t *>(m.weights) + kBiasOff);
    for (int i = threadIdx.x; i < kBiasSlots; i += kInferBlock) sb[i] = bias[i];
    // the fragments of layers 0 and 1 (18) stay in LDS and are re-read per
    // tile; the other 20 live in registers for the whole kernel (3 waves per
    // SIMD without spills)
    constexpr int kLdsFrags = 18, kRegFrags = kFrags - kLdsFrags;
    __shared__ FT wls[kLdsFrags * 64];
    const FT *wsrc = reinterpret_cast<const FT *>(m.weights);
    for (int i = threadIdx.x; i < kLdsFrags * 64; i += kInferBlock) wls[i] = wsrc[i];
    __syncthreads();
    const int l = threadIdx.x & 63, s = l & 31, h = l >> 5;
    FT wf[kRegFrags];
#pragma unroll
    for (int f = 0; f < kRegFrags; ++f) wf[f] = wsrc[(kLdsFrags + f) * 64 + l];
    auto frag = [&](int f) -> FT { return f < kLdsFrags ? wls[f * 64 + l] : wf[f - kLdsFrags]; };

    // lanes 0-31 encode the normalised position, lanes 32-63 the normal
    float lo[3], rext[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = h ? 0.0f : m.pos_lo[a];
        rext[a] = h ? 1.0f : 1.0f / (m.pos_hi[a] - m.pos_lo[a]);
    }
    const float4 *src = h ? nrm : pos;
    const uint32_t wave = (blockIdx.x * kInferBlock + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * kInferBlock) >> 6;
    const uint32_t ntiles = (n + 31u) / 32u;

    for (uint32_t tile = wave; tile < ntiles; tile += nwaves) {
        const float4 in = tile_input(src, tile, ntiles, s, n);
        // the LDS fragments and biases are re-read every tile: hoisted out of
        // the loop they would take 72 more registers plus the bias tiles,
        // and cost waves (238 registers, 2 waves)
        asm volatile("" ::: "memory");
        const uint32_t idx = tile * 32u + (uint32_t)s;
        const bool ok = idx < n;
        float feat[40];
#pragma unroll
        for (int a = 0; a < 3; ++a) encode13((comp(in, a) - lo[a]) * rext[a], feat + 13 * a);
        feat[39] = 0.0f;

        // layer 0: K = 80 (5 k-steps), two output tiles
        f32x16 acc0 = bias_tile(sb, h), acc1 = bias_tile(sb + 32, h);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            f32x8 x;
#pragma unroll
            for (int v = 0; v < 8; ++v) x[v] = feat[8 * c + v];
            const FT b = to_bf16(x);
            acc0 = mfma(frag(c), b, acc0);
            acc1 = mfma(frag(5 + c), b, acc1);
        }
        // hidden layers 1-3 and the output layer 4
#pragma unroll
        for (int L = 1; L < kLayers; ++L) {
            FT bop[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) bop[c] = relu_operand(c >> 1 ? acc1 : acc0, c & 1);
            const int f0 = kFrag0[L];
            if (L < kLayers - 1) {
                acc0 = bias_tile(sb + 64 * L, h);
                acc1 = bias_tile(sb + 64 * L + 32, h);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    acc0 = mfma(frag(f0 + c), bop[c], acc0);
                    acc1 = mfma(frag(f0 + 4 + c), bop[c], acc1);
                }
            } else {
                acc0 = bias_tile(sb + 256, h);
#pragma unroll
                for (int c = 0; c < 4; ++c) acc0 = mfma(frag(f0 + c), bop[c], acc0);
            }
        }
        // output rows 0..2 sit in accumulators 0..2 of the lower half-wave
        if (ok && h == 0) {
            out[idx] = make_float4(acc0[0], acc0[1], acc0[2], 0.0f);
        }
    }
}

// FP8 inference on the K = 64 instruction (twice the K = 16 instruction's
// rate): per 32-sample tile, layer 0 is two scaled K = 64 products per
// output tile (features 0..31, then 32..38, of each half-wave), every other
// layer one.  Operands are E4M3FN x / s with power-of-two per-layer scales:
// the factor s_w s_a / s_a' that takes a layer's sums to the next layer's
// input scale is then a power of two 2^k, applied by the instruction's E8M0
// operand scales (the bias, pre-divided by s_a', initialises the
// accumulators), so handing an activation on costs a ReLU-and-saturate and
// a conversion.  The fragments stay in LDS.
typedef int i32x8 __attribute__((ext_vector_type(8)));

// The exponent k of 2^k (A B) + C, split over the instruction's two E8M0
// operand scales.  Both are run-time values (a constant scale operand would
// be read as an FP32 constant), passed through an empty asm so that they sit
// in registers the layer's liveness asm can name.
struct E8M0Pair {
    int a, b;
};
__device__ __forceinline__ E8M0Pair e8m0_pair(int k)
{
    int a = 127 + (k >> 1), b = 127 + k - (k >> 1);
    asm volatile("" : "+v"(a), "+v"(b));
    return {a, b};
}
__device__ __forceinline__ f32x16 mfma64(i32x8 a, i32x8 b, f32x16 c, E8M0Pair q)
{
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, q.a, 0, q.b);
}

// four floats (already clamped to [-448, 448]) -> one register of four
// E4M3FN bytes.  Each conversion replaces one half of its third operand; the
// first one's other half is overwritten by the second, so any value serves
// as the first one's (here a's bits: no register has to be zeroed).
__device__ __forceinline__ int pack_fp8x4(float a, float b, float c, float d)
{
    const int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, __builtin_bit_cast(int, a), false);
    return __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
}

// the same for x / scale, scale a power of two (with a, b, c, d clamped to
// [-448 scale, 448 scale]): the conversion applies the scale exactly
typedef short i16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int pack_fp8x4_scaled(float a, float b, float c, float d, float scale)
{
    i16x2 w = __builtin_bit_cast(i16x2, a);
    w = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(w, a, b, scale, false);
    w = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(w, c, d, scale, true);
    return __builtin_bit_cast(int, w);
}

// one half-wave lane's 39 features (its sample's position or normal) -> the
// two layer-0 operands, at input scale sa0 with saturation at 448 sa0 = lim.
// The sines and cosines need the clamp only when lim < 1 (kClampAll).
template <bool kClampAll>
__device__ __forceinline__ void encode_fp8(float4 in, const float *lo, const float *rext, float sa0, float lim,
                                           i32x8 &b0, i32x8 &b1)
{
    float f[40];
#pragma unroll
    for (int a = 0; a < 3; ++a) encode13((comp(in, a) - lo[a]) * rext[a], f + 13 * a);
#pragma unroll
    for (int v = 0; v < 39; ++v)
        if (kClampAll || v % 13 == 0) f[v] = __builtin_amdgcn_fmed3f(f[v], -lim, lim);
    f[39] = 0.0f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        b0[q] = pack_fp8x4_scaled(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3], sa0);
        b1[q] = q < 2 ? pack_fp8x4_scaled(f[32 + 4 * q], f[33 + 4 * q], f[34 + 4 * q], f[35 + 4 * q], sa0) : 0;
    }
}

// accumulators of both tiles (already at the next layer's input scale) ->
// the next layer's K = 64 operand: ReLU and saturation, then conversion
__device__ __forceinline__ i32x8 relu_fp8_operand(const f32x16 &a0, const f32x16 &a1)
{
    i32x8 r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        r[q] = pack_fp8x4(__builtin_amdgcn_fmed3f(a0[4 * q], 0.0f, kFp8Max),
                          __builtin_amdgcn_fmed3f(a0[4 * q + 1], 0.0f, kFp8Max),
                          __builtin_amdgcn_fmed3f(a0[4 * q + 2], 0.0f, kFp8Max),
                          __builtin_amdgcn_fmed3f(a0[4 * q + 3], 0.0f, kFp8Max));
        r[4 + q] = pack_fp8x4(__builtin_amdgcn_fmed3f(a1[4 * q], 0.0f, kFp8Max),
                              __builtin_amdgcn_fmed3f(a1[4 * q + 1], 0.0f, kFp8Max),
                              __builtin_amdgcn_fmed3f(a1[4 * q + 2], 0.0f, kFp8Max),
                              __builtin_amdgcn_fmed3f(a1[4 * q + 3], 0.0f, kFp8Max));
    }
    return r;
}

__global__ void __launch_bounds__(kInferBlock) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_mlp_infer_fp8(gi_mlp m, uint32_t n, const float4 *pos, const float4 *nrm, float4 *out, int gate)
{
    if (gate && !mlp_selected(m)) return;   // uniform over the grid
    // activation scales as stored, rounded up to powers of two; layer L's
    // sums reach the next layer's input scale (the output's for L = 4)
    // through the exponent kx[L]
    float sa[kLayers];
#pragma unroll
    for (int L = 0; L < kLayers; ++L) sa[L] = pow2_at_least(m.scales[5 + L]);
    int kx[kLayers];
#pragma unroll
    for (int L = 0; L < kLayers; ++L)
        kx[L] = __builtin_amdgcn_readfirstlane(
            min(max(exp2_of(m.scales[L]) + exp2_of(sa[L]) - (L + 1 < kLayers ? exp2_of(sa[L + 1]) : 0), -120), 120));
    const float sa0 = sa[0], lim = kFp8Max * sa0;
    const bool clamp_all = lim < 1.0f;   // uniform
    __shared__ __attribute__((aligned(16))) float sb[kBiasSlots];
    const float *bias = reinterpret_cast<const float *>(reinterpret_cast<const uint8_t *>(m.weights) + kBiasOff);
    for (int i = threadIdx.x; i < kBiasSlots; i += kInferBlock) {
        const int L = i < 256 ? i >> 6 : 4;
        sb[i] = L + 1 < kLayers ? bias[i] / sa[L + 1] : bias[i];
    }
    // all eleven fragments in LDS (32 B per lane each), read per tile
    __shared__ i32x8 wl[kFp8Frags * 64];
    const i32x8 *w64 = reinterpret_cast<const i32x8 *>(m.weights);
    for (int i = threadIdx.x; i < kFp8Frags * 64; i += kInferBlock) wl[i] = w64[i];
    __syncthreads();
    const int l = threadIdx.x & 63, s = l & 31, h = l >> 5;

    float lo[3], rext[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = h ? 0.0f : m.pos_lo[a];
        rext[a] = h ? 1.0f : 1.0f / (m.pos_hi[a] - m.pos_lo[a]);
    }
    const float4 *src = h ? nrm : pos;
    const uint32_t wave = (blockIdx.x * kInferBlock + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * kInferBlock) >> 6;
    const uint32_t ntiles = (n + 31u) / 32u;

    // Two adjacent tiles per iteration: the fragments and biases read from
    // LDS serve both, and one tile's activations are converted while the
    // other's products run.  A layer's fragments and biases are read where
    // it runs, through an offset the compiler cannot see through (hoisted
    // to the top of the iteration, all eleven fragments would be spilled to
    // scratch).  The operands of a scaled product (A, B and the two scale
    // registers) stay allocated until its sums have been read: written while
    // the instruction is in flight, A and B reached it corrupted, so each
    // layer's empty asm takes the layer's operands next to the new activation
    // operands.
    for (uint32_t tile = 2 * wave; tile < ntiles; tile += 2 * nwaves) {
        const float4 inA = tile_input(src, tile, ntiles, s, n), inB = tile_input(src, tile + 1, ntiles, s, n);
        const uint32_t idxA = tile * 32u + (uint32_t)s, idxB = idxA + 32u;
        const bool okA = idxA < n, okB = tile + 1 < ntiles && idxB < n;
        i32x8 a0, a1, b0, b1;
        if (clamp_all) {
            encode_fp8<true>(inA, lo, rext, sa0, lim, a0, a1);
            encode_fp8<true>(inB, lo, rext, sa0, lim, b0, b1);
        } else {
            encode_fp8<false>(inA, lo, rext, sa0, lim, a0, a1);
            encode_fp8<false>(inB, lo, rext, sa0, lim, b0, b1);
        }
        uint32_t o = 0;
        asm volatile("" : "+v"(o) : "v"(a0[0]), "v"(b0[0]));
        const i32x8 fa = wl[o + l], fb = wl[o + 64 + l], fc = wl[o + 128 + l], fd = wl[o + 192 + l];
        const f32x16 c0 = bias_tile(sb + o, h), c1 = bias_tile(sb + o + 32, h);
        const E8M0Pair q0 = e8m0_pair(kx[0]);
        f32x16 A0 = mfma64(fa, a0, c0, q0);
        f32x16 A1 = mfma64(fb, a0, c1, q0);
        f32x16 B0 = mfma64(fa, b0, c0, q0);
        f32x16 B1 = mfma64(fb, b0, c1, q0);
        A0 = mfma64(fc, a1, A0, q0);
        A1 = mfma64(fd, a1, A1, q0);
        B0 = mfma64(fc, b1, B0, q0);
        B1 = mfma64(fd, b1, B1, q0);
        i32x8 opA = relu_fp8_operand(A0, A1);
        i32x8 opB = relu_fp8_operand(B0, B1);
        o = 0;
        asm volatile("" : "+v"(o) : "v"(opA), "v"(opB), "v"(a0), "v"(a1), "v"(b0), "v"(b1), "v"(fa), "v"(fb), "v"(fc),
                     "v"(fd), "v"(q0.a), "v"(q0.b));
#pragma unroll
        for (int L = 1; L < kLayers - 1; ++L) {
            const i32x8 f0 = wl[o + (2 + 2 * L) * 64 + l], f1 = wl[o + (3 + 2 * L) * 64 + l];
            const f32x16 d0 = bias_tile(sb + o + 64 * L, h), d1 = bias_tile(sb + o + 64 * L + 32, h);
            const E8M0Pair q = e8m0_pair(kx[L]);
            A0 = mfma64(f0, opA, d0, q);
            A1 = mfma64(f1, opA, d1, q);
            B0 = mfma64(f0, opB, d0, q);
            B1 = mfma64(f1, opB, d1, q);
            const i32x8 nA = relu_fp8_operand(A0, A1);
            const i32x8 nB = relu_fp8_operand(B0, B1);
            o = 0;
            asm volatile("" : "+v"(o) : "v"(nA), "v"(nB), "v"(opA), "v"(opB), "v"(f0), "v"(f1), "v"(q.a), "v"(q.b));
            opA = nA;
            opB = nB;
        }
        const i32x8 f4 = wl[o + 10 * 64 + l];
        const f32x16 d4 = bias_tile(sb + o + 256, h);
        const E8M0Pair q4 = e8m0_pair(kx[kLayers - 1]);
        A0 = mfma64(f4, opA, d4, q4);
        B0 = mfma64(f4, opB, d4, q4);
        const float touched = A0[0] + B0[0];
        asm volatile("" ::"v"(touched), "v"(opA), "v"(opB), "v"(f4), "v"(q4.a), "v"(q4.b));
        // output rows 0..2 sit in accumulators 0..2 of the lower half-wave
        if (h == 0) {
            if (okA) out[idxA] = make_float4(A0[0], A0[1], A0[2], 0.0f);
            if (okB) out[idxB] = make_float4(B0[0], B0[1], B0[2], 0.0f);
        }
    }
}

// --------------------------------------------------------------------------
// training
// --------------------------------------------------------------------------
// number of valid samples (target.w != 0) -> hdr[0]
// sum of a value over a 1024-thread workgroup: wave sums by shuffles, then
// the 16 wave sums in order (integer-valued here, so exact)
__device__ __forceinline__ uint32_t block_sum_1024(uint32_t v, uint32_t *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t r = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) r += red[w];
    return r;
}

__global__ void __launch_bounds__(1024) k_mlp_count(uint32_t n, const float4 *tgt, uint32_t *hdr)
{
    __shared__ uint32_t red[16];
    // 16 independent loads in flight per thread and round
    uint32_t c = 0;
    for (uint32_t i = threadIdx.x; i < n; i += 16384) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t j = i + 1024u * k;
            if (j < n) c += tgt[j].w != 0.0f ? 1u : 0u;
        }
    }
    const uint32_t r = block_sum_1024(c, red);
    if (threadIdx.x == 0) hdr[0] = r;
}

// --------------------------------------------------------------------------
// training on the matrix cores
// --------------------------------------------------------------------------
// One workgroup of two waves takes kMS = 64 samples, each wave a tile of 32
// samples on the N side of the 32x32x16 BF16 product, as in inference:
// forward products W x (weight fragments of the master parameters as the A
// operand), the activations handed from layer to layer in registers, and
// each layer's input also written to LDS unit-major ([unit][sample]); the
// backward products dA = W^T g take the transposed fragments, g handed down
// in registers the same way (the ReLU masks kept as bits from the forward
// pass); the weight gradients dW = g^T a sum over the 64 samples with the
// samples on the K side, both operands read from LDS.  Every operand is
// rounded to BF16 and products accumulate in FP32, as in the VALU form.
constexpr int kMS = 64;                 // samples per workgroup
constexpr int kMBlock = 128;            // two waves
constexpr int kFwdFrags = kFrags;       // 38 forward fragments (inference layout, master parameters)
constexpr int kBwdFrag0[kLayers] = {0, 0, 8, 16, 24};   // backward fragments of layers 1..4 (W^T)
constexpr int kBwdFrags = 26;
constexpr int kTrainFragBytes = (kFwdFrags + kBwdFrags) * 64 * 16;

// backward fragment f of layer L (1..3: 2 row tiles x 4 k-steps; 4: 2 x 1):
// lane l holds rows k = 32 t + l % 32 of W_L^T, K slots 16 c + 8 h + v
// taking output unit swap23(16 c + 8 h + v) (the layout the previous
// backward product leaves in its accumulators); layer 4 takes unit v of
// the lower half-wave (its 3 outputs) and zero elsewhere
__device__ __forceinline__ float bwd_weight(const float *P, int f, int l, int v)
{
    const int L = f < 8 ? 1 : (f < 16 ? 2 : (f < 24 ? 3 : 4));
    const int r = f - kBwdFrag0[L];
    const int t = L < 4 ? r >> 2 : r, c = L < 4 ? r & 3 : 0, h = l >> 5;
    const int k = 32 * t + (l & 31);
    const int u = L < 4 ? swap23(16 * c + 8 * h + v) : (h == 0 && v < 3 ? v : -1);
    if (u < 0 || u >= kOut[L] || k >= kIn[L]) return 0.0f;
    return P[kOffW[L] + u * kIn[L] + k];
}

// forward and backward BF16 fragments of the master parameters, one element per thread
__global__ void __launch_bounds__(256) k_mlp_train_frags(gi_mlp m, __bf16 *frags)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= (kFwdFrags + kBwdFrags) * 64 * 8) return;
    const int f = i >> 9, l = (i >> 3) & 63, v = i & 7;
    float w = 0.0f;
    if (f < kFwdFrags) {
        const int L = layer_of_frag(f), r = f - kFrag0[L];
        const int t = r / kSteps[L], c = r % kSteps[L];
        const int row = 32 * t + (l & 31), k = frag_column(L, c, l >> 5, v);
        if (row < kOut[L] && k >= 0 && k < kIn[L]) w = m.params[kOffW[L] + row * kIn[L] + k];
    } else {
        w = bwd_weight(m.params, f - kFwdFrags, l, v);
    }
    frags[i] = (__bf16)w;
}

// sum over the 32 lanes of each half-wave (fixed butterfly order)
__device__ __forceinline__ float half_sum(float v)
{
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// The same sum by DPP moves (no LDS round trips), in a fixed order: pairs,
// quads, mirrored halves of each row of 16 lanes, mirrored rows, then row 0's
// total broadcast into row 1 and row 2's into row 3.  The half-wave's total
// lands in its upper 16 lanes (16-31 and 48-63).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_add(float v)
{
    return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl, kRowMask,
                                                                     0xF, false));
}
__device__ __forceinline__ float half_sum_dpp(float v)
{
    v = dpp_add<0xB1, 0xF>(v);     // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4E, 0xF>(v);     // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141, 0xF>(v);    // row_half_mirror
    v = dpp_add<0x140, 0xF>(v);    // row_mirror
    return dpp_add<0x142, 0xA>(v); // row_bcast:15 into rows 1 and 3
}
__device__ __forceinline__ float half_max(float v)
{
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// the 16 accumulators of a tile as BF16 operand halves (no ReLU)
__device__ __forceinline__ bf16x8 bf16_operand(const f32x16 &a, int part)
{
    u32x4 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = pk_bf16(a[8 * part + 2 * i], a[8 * part + 2 * i + 1]);
    return __builtin_bit_cast(bf16x8, r);
}

__global__ void __launch_bounds__(kMBlock) k_mlp_fwdbwd_mfma(gi_mlp m, uint32_t n, const float4 *pos,
                                                            const float4 *nrm, const float4 *tgt,
                                                            const float4 *qp, const uint32_t *hdr,
                                                            const bf16x8 *frags, float *part)
{
    __shared__ __attribute__((aligned(16))) __bf16 sX[80 * kMS];       // layer 0 input [feature][sample]
    __shared__ __attribute__((aligned(16))) __bf16 sA[4 * 64 * kMS];   // layer 1..4 inputs [unit][sample]
    __shared__ __attribute__((aligned(16))) __bf16 sG[64 * kMS];       // BF16 gradient [unit][sample]
    __shared__ float sDb[2][64];                                       // bias gradient per wave
    __shared__ float sSt[2][kStats];
    // all 64 forward and backward fragments staged in LDS (64 KB): each
    // layer's operands are then an LDS read away instead of an L2 round trip
    __shared__ bf16x8 sF[(kFwdFrags + kBwdFrags) * 64];
    for (int i = threadIdx.x; i < (kFwdFrags + kBwdFrags) * 64; i += kMBlock) sF[i] = frags[i];
    // the biases too (layer L's at 64 L, the output layer's at 256)
    __shared__ float sBias[kBiasSlots];
    for (int i = threadIdx.x; i < kBiasSlots; i += kMBlock) {
        const int L = i < 256 ? i >> 6 : 4, u = i < 256 ? i & 63 : i - 256;
        sBias[i] = u < kOut[L] ? m.params[kOffB[L] + u] : 0.0f;
    }

    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, s = l & 31, h = l >> 5;
    const int sl = 32 * wv + s;                                        // sample within the workgroup
    const uint32_t idx = blockIdx.x * kMS + sl;
    float *pw = part + (size_t)blockIdx.x * kPartStride;
    const bf16x8 *bfr = sF + kFwdFrags * 64;

    // inputs and encoding: lanes 0-31 the position's 39 features, 32-63 the normal's
    const float4 tg = idx < n ? tgt[idx] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const bool valid = idx < n && tg.w != 0.0f;
    const float4 in = valid ? (h ? nrm[idx] : pos[idx]) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float feat[40];
    float amax[kLayers] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        encode13(h ? comp(in, a) : (comp(in, a) - m.pos_lo[a]) / (m.pos_hi[a] - m.pos_lo[a]), feat + 13 * a);
    feat[39] = 0.0f;
#pragma unroll
    for (int j = 0; j < 39; ++j) {
        if (!valid) feat[j] = 0.0f;
        amax[0] = fmaxf(amax[0], fabsf(feat[j]));
        sX[(39 * h + j) * kMS + sl] = (__bf16)feat[j];
    }
    if (h) {
        sX[78 * kMS + sl] = (__bf16)0.0f;
        sX[79 * kMS + sl] = (__bf16)0.0f;
    }

    __syncthreads();   // sF

    // forward
    uint32_t mask[kLayers - 1];
    f32x16 acc0, acc1;
    {
        acc0 = f32x16{};
        acc1 = f32x16{};
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                acc0[4 * a + b] = sBias[8 * a + 4 * h + b];
                acc1[4 * a + b] = sBias[32 + 8 * a + 4 * h + b];
            }
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            f32x8 x;
#pragma unroll
            for (int v = 0; v < 8; ++v) x[v] = feat[8 * c + v];
            const bf16x8 b = to_bf16(x);
            acc0 = mfma(sF[c * 64 + l], b, acc0);
            acc1 = mfma(sF[(5 + c) * 64 + l], b, acc1);
        }
    }
#pragma unroll
    for (int L = 1; L < kLayers; ++L) {
        // layer L-1's ReLU output: kept as the ReLU mask and written to LDS as layer L's input
        uint32_t mk = 0u;
        float mx = 0.0f;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const float z = t ? acc1[i] : acc0[i];
                const float a = fmaxf(z, 0.0f);
                mk |= (z > 0.0f ? 1u : 0u) << (16 * t + i);
                mx = fmaxf(mx, a);
                const int k = 32 * t + 8 * (i >> 2) + 4 * h + (i & 3);
                sA[((L - 1) * 64 + k) * kMS + sl] = (__bf16)a;
            }
        mask[L - 1] = mk;
        if (valid) amax[L] = mx;
        bf16x8 bop[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) bop[c] = relu_operand(c >> 1 ? acc1 : acc0, c & 1);
        const int f0 = kFrag0[L];
        if (L < kLayers - 1) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    acc0[4 * a + b] = sBias[64 * L + 8 * a + 4 * h + b];
                    acc1[4 * a + b] = sBias[64 * L + 32 + 8 * a + 4 * h + b];
                }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                acc0 = mfma(sF[(f0 + c) * 64 + l], bop[c], acc0);
                acc1 = mfma(sF[(f0 + 4 + c) * 64 + l], bop[c], acc1);
            }
        } else {
            acc0 = f32x16{};
#pragma unroll
            for (int b = 0; b < 3; ++b) acc0[b] = h ? 0.0f : sBias[256 + b];
#pragma unroll
            for (int c = 0; c < 4; ++c) acc0 = mfma(sF[(f0 + c) * 64 + l], bop[c], acc0);
        }
    }
    // loss gradient (lower half-wave: outputs 0..2 in accumulators 0..2)
    const float ntot = (float)max(hdr[0], 1u) * 3.0f;
    float loss = 0.0f, enum_ = 0.0f, eden = 0.0f, nonfinite = 0.0f;
    float g[3] = {0.0f, 0.0f, 0.0f};
    if (h == 0) {
        const float4 q = (valid && qp) ? qp[idx] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float z = acc0[c];
            if (valid) {
                const float den = z * z + 0.01f, d = z - comp(tg, c);
                g[c] = 2.0f * d / den / ntot;
                loss += d * d / den;
                // squared errors of the cache (as the target uses it) and of
                // the probe query against the label (none without probe values)
                if (qp) {
                    const float ec = fmaxf(z, 0.0f) - comp(tg, c), ep = comp(q, c) - comp(tg, c);
                    enum_ += ec * ec;
                    eden += ep * ep;
                }
                nonfinite += __builtin_isfinite(z) ? 0.0f : 1.0f;
            }
        }
    }
    // statistics of the workgroup: per half-wave, then the two waves in order
    {
        float st[4 + kLayers] = {loss, enum_, eden, nonfinite};
#pragma unroll
        for (int j = 0; j < 4; ++j) st[j] = half_sum(st[j]);
#pragma unroll
        for (int L = 0; L < kLayers; ++L) st[4 + L] = half_max(amax[L]);
#pragma unroll
        for (int j = 0; j < 4 + kLayers; ++j) {
            // lane 0 holds the lower half's value, lane 32 the upper half's
            const float o = __shfl(st[j], 32, 64);
            if (l == 0) sSt[wv][j] = j < 4 ? st[j] + o : fmaxf(st[j], o);
        }
    }

    // backward: layer 4 first (3 output units)
    f32x16 g0, g1;     // this lane's gradient of the current layer's pre-activation
    // unrolled: every layer's sizes and offsets are constants
#pragma unroll
    for (int L = kLayers - 1; L >= 0; --L) {
        const int out = kOut[L], in = kIn[L];
        // bias gradient (unrounded FP32 g) and the BF16 gradient in LDS [unit][sample]
        if (L == kLayers - 1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float sum = half_sum_dpp(g[c]);
                if (l == 31) sDb[wv][c] = sum;
            }
            if (h == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) sG[c * kMS + sl] = (__bf16)g[c];
            }
        } else {
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const float v = t ? g1[i] : g0[i];
                    const int u = 32 * t + 8 * (i >> 2) + 4 * h + (i & 3);
                    const float sum = half_sum_dpp(v);
                    if (s == 31) sDb[wv][u] = sum;
                    sG[u * kMS + sl] = (__bf16)v;
                }
        }
        __syncthreads();
        if (threadIdx.x < out) pw[kOffB[L] + threadIdx.x] = sDb[0][threadIdx.x] + sDb[1][threadIdx.x];
        // dW = g^T a over the workgroup's 64 samples: output tiles (unit tile i, input tile j)
        const __bf16 *Ain = L == 0 ? sX : sA + (L - 1) * 64 * kMS;
        const int ti = (out + 31) / 32, tj = (in + 31) / 32;
        for (int tile = wv; tile < ti * tj; tile += 2) {
            const int i0 = 32 * (tile / tj), j0 = 32 * (tile % tj);
            const int ur = i0 + (l & 31), kr = j0 + (l & 31);
            f32x16 d = f32x16{};
#pragma unroll
            for (int c = 0; c < kMS / 16; ++c) {
                const int s0 = 16 * c + 8 * h;
                const bf16x8 a = ur < out ? *reinterpret_cast<const bf16x8 *>(sG + ur * kMS + s0) : bf16x8{};
                const bf16x8 b = kr < (L == 0 ? 80 : in) ? *reinterpret_cast<const bf16x8 *>(Ain + kr * kMS + s0)
                                                         : bf16x8{};
                d = mfma(a, b, d);
            }
            // accumulator 4a + b: row (unit) i0 + 8a + 4h + b, column (input) kr
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int u = i0 + 8 * (i >> 2) + 4 * h + (i & 3);
                if (u < out && kr < in) pw[kOffW[L] + u * in + kr] = d[i];
            }
        }
        if (L == 0) break;
        // dA = W^T g: the BF16 gradient from registers as the B operand
        bf16x8 bop[4];
        int nc;
        if (L == kLayers - 1) {
            f32x8 x = f32x8{};
            if (h == 0) {
                x[0] = g[0];
                x[1] = g[1];
                x[2] = g[2];
            }
            bop[0] = to_bf16(x);
            nc = 1;
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) bop[c] = bf16_operand(c >> 1 ? g1 : g0, c & 1);
            nc = 4;
        }
        f32x16 d0 = f32x16{}, d1 = f32x16{};
        const int fb = kBwdFrag0[L];
        for (int c = 0; c < nc; ++c) {
            const int f0 = L == kLayers - 1 ? fb : fb + c, f1 = L == kLayers - 1 ? fb + 1 : fb + 4 + c;
            d0 = mfma(bfr[f0 * 64 + l], bop[c], d0);
            d1 = mfma(bfr[f1 * 64 + l], bop[c], d1);
        }
        // ReLU mask of layer L-1's output
        const uint32_t mk = mask[L - 1];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            g0[i] = (mk >> i) & 1u ? d0[i] : 0.0f;
            g1[i] = (mk >> (16 + i)) & 1u ? d1[i] : 0.0f;
        }
        __syncthreads();     // sG and sDb are rewritten by the next layer
    }
    __syncthreads();
    if (threadIdx.x < kStats) {
        // slots 0-3 sums (loss, error numerator and denominator, non-finite outputs), 4-8 the
        // activation amax of every layer input, the rest unused (zero)
        const int j = threadIdx.x;
        const float v = j < 4 ? sSt[0][j] + sSt[1][j] : (j < 4 + kLayers ? fmaxf(sSt[0][j], sSt[1][j]) : 0.0f);
        pw[kParams + j] = v;
    }
}

// First level of the ordered reduction: rows g*kGroup .. g*kGroup+kGroup-1
// of the partials are summed in order (max for the amax slots) into row
// g*kGroup; each thread owns one column, so the in-place write is private.
constexpr uint32_t kGroup = 16;

__device__ __forceinline__ bool stat_is_max(int p)
{
    const int j = p - kParams;
    return j >= kStAmax0 && j < kStAmax0 + kLayers;
}

__global__ void __launch_bounds__(256) k_mlp_reduce1(uint32_t nwg, float *part)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kParams + kStats) return;
    const uint32_t w0 = blockIdx.y * kGroup, w1 = min(w0 + kGroup, nwg);
    const bool is_max = stat_is_max(p);
    // the group's loads are all issued before the first add; the order of
    // the adds is the partials' order
    float x[kGroup];
#pragma unroll
    for (uint32_t k = 0; k < kGroup; ++k) x[k] = w0 + k < w1 ? part[(size_t)(w0 + k) * kPartStride + p] : 0.0f;
    float acc = 0.0f;
#pragma unroll
    for (uint32_t k = 0; k < kGroup; ++k) acc = is_max ? fmaxf(acc, x[k]) : acc + x[k];
    part[(size_t)w0 * kPartStride + p] = acc;
}

// second level: the group sums in group order; statistics into state / scales
__global__ void __launch_bounds__(256) k_mlp_reduce(gi_mlp m, uint32_t nwg, const float *part, float *grad,
                                                    const uint32_t *hdr)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kParams + kStats) return;
    const int j = p - kParams;
    const bool is_max = stat_is_max(p);
    // group sums in group order, 16 loads in flight per round
    float acc = 0.0f;
    for (uint32_t w = 0; w < nwg; w += 16 * kGroup) {
        float x[16];
#pragma unroll
        for (uint32_t k = 0; k < 16; ++k) {
            const uint32_t wk = w + k * kGroup;
            x[k] = wk < nwg ? part[(size_t)wk * kPartStride + p] : 0.0f;
        }
#pragma unroll
        for (uint32_t k = 0; k < 16; ++k) acc = is_max ? fmaxf(acc, x[k]) : acc + x[k];
    }
    if (j < 0) {
        grad[p] = acc;
        return;
    }
    const uint32_t valid = hdr[0];
    const float ntot = (float)max(valid, 1u) * 3.0f;
    if (j == kStLoss) {
        m.state[GI_MLP_STATE_LOSS] = __float_as_uint(acc / ntot);
        m.state[GI_MLP_STATE_VALID] = valid;
    } else if (j == kStErrNum) {
        float den = 0.0f;
        for (uint32_t w = 0; w < nwg; w += kGroup) den += part[(size_t)w * kPartStride + kParams + kStErrDen];
        m.state[GI_MLP_STATE_BATCH_ERR] = __float_as_uint(den > 0.0f ? acc / den : (acc > 0.0f ? kFltMax : 0.0f));
    } else if (j == kStNonFinite) {
        m.state[GI_MLP_STATE_NONFINITE] = (uint32_t)acc;
    } else if (is_max) {
        m.scales[5 + (j - kStAmax0)] = fp8_scale(acc);
    }
}

__global__ void __launch_bounds__(256) k_mlp_adam(gi_mlp m, const float *grad, float lr, float c1, float c2)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kParams) return;
    const float g = grad[p];
    const float mm = 0.9f * m.adam_m[p] + 0.1f * g;
    const float vv = 0.99f * m.adam_v[p] + 0.01f * g * g;
    m.adam_m[p] = mm;
    m.adam_v[p] = vv;
    const float np = m.params[p] - lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
    m.params[p] = np;
    if (m.ema) m.ema[p] = m.ema_decay * m.ema[p] + (1.0f - m.ema_decay) * np;
}

// usability after step t (one workgroup of 1024 threads)
__global__ void __launch_bounds__(1024) k_mlp_state(gi_mlp m, uint32_t t)
{
    __shared__ uint32_t red[16];
    // all of a thread's loads in flight at once
    uint32_t bad = 0;
    constexpr int kPer = (kParams + 1023) / 1024;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int p = threadIdx.x + 1024 * k;
        if (p < kParams) bad += __builtin_isfinite(m.params[p]) ? 0u : 1u;
    }
    const uint32_t nonfinite = block_sum_1024(bad, red);
    if (threadIdx.x == 0) {
        const float be = __uint_as_float(m.state[GI_MLP_STATE_BATCH_ERR]);
        const float old = __uint_as_float(m.state[GI_MLP_STATE_EMA_ERR]);
        const float ema = t <= 1u ? be : 0.9f * old + 0.1f * be;
        const bool ok = t >= m.warmup_steps && m.state[GI_MLP_STATE_NONFINITE] == 0u && ema <= m.max_rel_err &&
                        nonfinite == 0u;
        m.state[GI_MLP_STATE_STEPS] = t;
        m.state[GI_MLP_STATE_EMA_ERR] = __float_as_uint(ema);
        m.state[GI_MLP_STATE_USABLE] = ok ? 1u : 0u;
    }
}

constexpr uint32_t train_wgs(uint32_t n) { return (n + kMS - 1) / kMS; }

// workspace: header, gradient, one partial gradient per workgroup, then the
// BF16 fragments of the master parameters the matrix-core kernel reads
constexpr uint64_t train_frag_off(uint32_t n) { return 4ull * (kHdr + (uint64_t)kPartStride * (1ull + train_wgs(n))); }
constexpr uint64_t train_bytes(uint32_t n) { return train_frag_off(n) + kTrainFragBytes; }

// Scratch of the allocation-free training step (gi_mlp_train_step_noalloc):
// the workspace of a GI_MLP_NOALLOC_MAX_BATCH-sample step, one copy per GPU,
// held from the code object's load until the process ends.  Every word the
// step reads is written earlier in the same step (count, partial gradients,
// reductions), so nothing needs clearing between calls; calls that overlap
// on one GPU share it and race.
constexpr uint64_t kNoallocBytes = train_bytes(GI_MLP_NOALLOC_MAX_BATCH);
static_assert(kNoallocBytes == GI_MLP_NOALLOC_SCRATCH_BYTES, "gi.h states the scratch size");
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

// device address of `scratch` on each GPU (the host-side symbol is only a
// stand-in), looked up once per device with that device current
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

gi_status scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GI_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GI_ERR_DEVICE;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return GI_OK;
}

gi_status prepare(const gi_mlp &m, hipStream_t st)
{
    if (m.precision == GI_MLP_BF16) {
        k_mlp_prepare_bf16<<<(kFrags * 64 * 8 + 255) / 256, 256, 0, st>>>(m);
    } else {
        k_mlp_wscale<<<kLayers, 256, 0, st>>>(m);
        k_mlp_prepare_fp8<<<(kFp8Frags * 64 * 32 + 255) / 256, 256, 0, st>>>(m);
    }
    return launched_mlp();
}

gi_status check_batch(uint32_t n, const float *pos4, const float *nrm4, const float *target4)
{
    if (n > GI_MLP_MAX_BATCH) return GI_ERR_SHAPE;
    if (n && (!pos4 || !nrm4 || !target4)) return GI_ERR_NULL;
    return GI_OK;
}

gi_status grad_launch(const gi_mlp &m, uint32_t n, const float *pos4, const float *nrm4, const float *target4,
                      const float *qprobe4, float *grad, void *ws, hipStream_t st)
{
    uint32_t *hdr = reinterpret_cast<uint32_t *>(ws);
    float *part = reinterpret_cast<float *>(ws) + kHdr + kPartStride;
    const uint32_t nwg = train_wgs(n);
    k_mlp_count<<<1, 1024, 0, st>>>(n, reinterpret_cast<const float4 *>(target4), hdr);
    __bf16 *frags = reinterpret_cast<__bf16 *>(reinterpret_cast<uint8_t *>(ws) + train_frag_off(n));
    if (nwg) {
        k_mlp_train_frags<<<((kFwdFrags + kBwdFrags) * 64 * 8 + 255) / 256, 256, 0, st>>>(m, frags);
        k_mlp_fwdbwd_mfma<<<nwg, kMBlock, 0, st>>>(m, n, reinterpret_cast<const float4 *>(pos4),
                                                   reinterpret_cast<const float4 *>(nrm4),
                                                   reinterpret_cast<const float4 *>(target4),
                                                   reinterpret_cast<const float4 *>(qprobe4), hdr,
                                                   reinterpret_cast<const bf16x8 *>(frags), part);
    }
    const uint32_t cols = (kParams + kStats + 255) / 256;
    if (nwg) k_mlp_reduce1<<<dim3(cols, (nwg + kGroup - 1) / kGroup), 256, 0, st>>>(nwg, part);
    k_mlp_reduce<<<cols, 256, 0, st>>>(m, nwg, part, grad, hdr);
    return launched_mlp();
}

gi_status adam_launch(const gi_mlp &m, const float *grad, uint32_t t, float lr, hipStream_t st)
{
    const double c1 = 1.0 / (1.0 - std::pow(0.9, (double)t));
    const double c2 = 1.0 / (1.0 - std::pow(0.99, (double)t));
    k_mlp_adam<<<(kParams + 255) / 256, 256, 0, st>>>(m, grad, lr, (float)c1, (float)c2);
    k_mlp_state<<<1, 1024, 0, st>>>(m, t);
    gi_status s = launched_mlp();
    if (s != GI_OK) return s;
    return prepare(m, st);
}

}  // namespace

namespace gi {

gi_status check_mlp(const gi_mlp *m)
{
    if (!m) return GI_ERR_NULL;
    if (!m->params || !m->adam_m || !m->adam_v || !m->weights || !m->scales || !m->state) return GI_ERR_NULL;
    if (m->precision > GI_MLP_FP8 || m->mode > GI_MLP_NEVER) return GI_ERR_PARAM;
    for (int a = 0; a < 3; ++a)
        if (!(m->pos_hi[a] > m->pos_lo[a])) return GI_ERR_PARAM;
    if (!(m->max_rel_err > 0.0f)) return GI_ERR_PARAM;
    if (!(m->ema_decay >= 0.0f && m->ema_decay < 1.0f)) return GI_ERR_PARAM;
    return GI_OK;
}

gi_status mlp_infer_launch(const gi_mlp &m, uint32_t n, const float4 *pos, const float4 *nrm, float4 *out,
                           bool gate, hipStream_t st)
{
    if (n == 0) return GI_OK;
    const uint32_t tiles = (n + 31u) / 32u;
    const uint32_t blocks = std::min<uint32_t>((tiles + 3u) / 4u, 2048u);
    if (m.precision == GI_MLP_BF16)
        k_mlp_infer_bf16<<<blocks, kInferBlock, 0, st>>>(m, n, pos, nrm, out, gate ? 1 : 0);
    else
        k_mlp_infer_fp8<<<blocks, kInferBlock, 0, st>>>(m, n, pos, nrm, out, gate ? 1 : 0);
    return launched_mlp();
}

}  // namespace gi

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

gi_status gi_mlp_init(const gi_mlp *mlp, uint64_t seed, void *stream)
{
    gi_status s;
    if ((s = check_mlp(mlp)) != GI_OK) return s;
    k_mlp_init<<<(kParams + 255) / 256, 256, 0, S(stream)>>>(*mlp, seed);
    if ((s = launched_mlp()) != GI_OK) return s;
    return prepare(*mlp, S(stream));
}

gi_status gi_mlp_prepare(const gi_mlp *mlp, void *stream)
{
    gi_status s;
    if ((s = check_mlp(mlp)) != GI_OK) return s;
    return prepare(*mlp, S(stream));
}

gi_status gi_mlp_infer(const gi_mlp *mlp, uint32_t n, const float *pos4, const float *nrm4, float *out4,
                       void *stream)
{
    gi_status s;
    if ((s = check_mlp(mlp)) != GI_OK) return s;
    if (n == 0) return GI_OK;
    if (!pos4 || !nrm4 || !out4) return GI_ERR_NULL;
    if (out4 == pos4 || out4 == nrm4) return GI_ERR_ALIAS;
    return mlp_infer_launch(*mlp, n, reinterpret_cast<const float4 *>(pos4), reinterpret_cast<const float4 *>(nrm4),
                            reinterpret_cast<float4 *>(out4), false, S(stream));
}

uint64_t gi_mlp_train_workspace_bytes(uint32_t n) { return train_bytes(n); }

gi_status gi_mlp_grad(const gi_mlp *mlp, uint32_t n, const float *pos4, const float *nrm4, const float *target4,
                      const float *qprobe4, float *grad, void *workspace, uint64_t workspace_bytes, void *stream)
{
    gi_status s;
    if ((s = check_mlp(mlp)) != GI_OK) return s;
    if ((s = check_batch(n, pos4, nrm4, target4)) != GI_OK) return s;
    if (!grad || !workspace) return GI_ERR_NULL;
    if (workspace_bytes < train_bytes(n)) return GI_ERR_SHAPE;
    return grad_launch(*mlp, n, pos4, nrm4, target4, qprobe4, grad, workspace, S(stream));
}

gi_status gi_mlp_adam(const gi_mlp *mlp, const float *grad, uint32_t t, float lr, void *stream)
{
    gi_status s;
    if ((s = check_mlp(mlp)) != GI_OK) return s;
    if (!grad) return GI_ERR_NULL;
    if (t < 1 || !(lr > 0.0f)) return GI_ERR_PARAM;
    return adam_launch(*mlp, grad, t, lr, S(stream));
}

gi_status gi_mlp_train_step(const gi_mlp *mlp, uint32_t n, const float *pos4, const float *nrm4,
                            const float *target4, const float *qprobe4, uint32_t t, float lr, void *workspace,
                            uint64_t workspace_bytes, void *stream)
{
    gi_status s;
    if ((s = check_mlp(mlp)) != GI_OK) return s;
    if ((s = check_batch(n, pos4, nrm4, target4)) != GI_OK) return s;
    if (!workspace) return GI_ERR_NULL;
    if (workspace_bytes < train_bytes(n)) return GI_ERR_SHAPE;
    if (t < 1 || !(lr > 0.0f)) return GI_ERR_PARAM;
    float *grad = reinterpret_cast<float *>(workspace) + kHdr;
    if ((s = grad_launch(*mlp, n, pos4, nrm4, target4, qprobe4, grad, workspace, S(stream))) != GI_OK) return s;
    return adam_launch(*mlp, grad, t, lr, S(stream));
}

gi_status gi_mlp_train_step_noalloc(const gi_mlp *mlp, uint32_t n, const float *pos4, const float *nrm4,
                                    const float *target4, const float *qprobe4, uint32_t t, float lr,
                                    void *stream)
{
    gi_status s;
    if ((s = check_mlp(mlp)) != GI_OK) return s;
    if ((s = check_batch(n, pos4, nrm4, target4)) != GI_OK) return s;
    if (n > GI_MLP_NOALLOC_MAX_BATCH) return GI_ERR_SHAPE;
    if (t < 1 || !(lr > 0.0f)) return GI_ERR_PARAM;
    void *ws = nullptr;
    if ((s = scratch_address(&ws)) != GI_OK) return s;
    float *grad = reinterpret_cast<float *>(ws) + kHdr;
    if ((s = grad_launch(*mlp, n, pos4, nrm4, target4, qprobe4, grad, ws, S(stream))) != GI_OK) return s;
    return adam_launch(*mlp, grad, t, lr, S(stream));
}

}  // extern "C"
