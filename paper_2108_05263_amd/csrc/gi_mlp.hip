// Learned radiance cache on gfx950: parameter initialisation, inference
// operands, MFMA inference (BF16 and FP8 E4M3) and BF16 training (forward,
// backward, ordered gradient reduction, Adam, usability state).
//
// Inference keeps the whole network in registers: each wave loads the 38
// weight fragments of the 32x32x16 MFMA once and then streams tiles of 32
// samples, the samples on the N side of every product, so a layer's
// accumulators become the next layer's B operand without leaving the
// registers (see the slot permutation in gi_mlp.hpp).
//
// Training (2^14..2^16 samples per step, ~0.6 GFLOP) runs on the vector ALUs
// with the operands in LDS: one workgroup per 32 samples computes the
// forward pass, the loss gradient and the backward pass, and writes its
// partial gradient; two more kernels sum the partials in a fixed order
// (groups of 16 workgroups, then the groups), so the result does not depend
// on scheduling.
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
constexpr int kTrainS = 32;            // samples per training workgroup
constexpr int kTrainBlock = 256;
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
    if (t == 0) m.scales[L] = red[0] > 0.0f ? red[0] / kFp8Max : 1.0f;
}

__device__ __forceinline__ uint32_t fp8_byte(float x)
{
    x = fminf(fmaxf(x, -kFp8Max), kFp8Max);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xFFu;
}

// FP8 fragments: byte i = (f * 64 + lane) * 8 + v
__global__ void __launch_bounds__(256) k_mlp_prepare_fp8(gi_mlp m)
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
    if (row < kOut[L] && k >= 0 && k < kIn[L]) w = src.p[kOffW[L] + row * kIn[L] + k] * src.scale / m.scales[L];
    reinterpret_cast<uint8_t *>(m.weights)[i] = (uint8_t)fp8_byte(w);
}

// --------------------------------------------------------------------------
// inference
// --------------------------------------------------------------------------
template <int P>
struct Frag;
template <>
struct Frag<GI_MLP_BF16> {
    using T = bf16x8;
};
template <>
struct Frag<GI_MLP_FP8> {
    using T = long;
};

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

// eight floats already within +-448 -> eight E4M3FN bytes
__device__ __forceinline__ long to_fp8(f32x8 x)
{
    int lo = __builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], 0, false);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(x[2], x[3], lo, true);
    int hi = __builtin_amdgcn_cvt_pk_fp8_f32(x[4], x[5], 0, false);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(x[6], x[7], hi, true);
    return (long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ f32x8 half_of(const f32x16 &a, int part)
{
    return part ? __builtin_shufflevector(a, a, 8, 9, 10, 11, 12, 13, 14, 15)
                : __builtin_shufflevector(a, a, 0, 1, 2, 3, 4, 5, 6, 7);
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

template <int P>
__global__ void __launch_bounds__(kInferBlock) __attribute__((amdgpu_waves_per_eu(P == GI_MLP_BF16 ? 3 : 4, P == GI_MLP_BF16 ? 3 : 4)))
k_mlp_infer(gi_mlp m, uint32_t n, const float4 *pos,
                                                           const float4 *nrm, float4 *out, int gate)
{
    using FT = typename Frag<P>::T;
    if (gate && !mlp_selected(m)) return;   // uniform over the grid
    // FP8 scales (a non-positive or non-finite activation scale counts as 1):
    // layer L's accumulator holds sum a8 w8 = z / (s_w s_a); its bias enters
    // as b / (s_w s_a) and the next layer's operand is acc * (s_w s_a / s_a')
    float kq[kLayers - 1];
    float smul4 = 1.0f, in0 = 1.0f;
    if (P == GI_MLP_FP8) {
        float sa[kLayers];
#pragma unroll
        for (int L = 0; L < kLayers; ++L) {
            sa[L] = m.scales[5 + L];
            if (!(sa[L] > 0.0f && sa[L] < kInf)) sa[L] = 1.0f;
        }
#pragma unroll
        for (int L = 0; L + 1 < kLayers; ++L) kq[L] = m.scales[L] * sa[L] / sa[L + 1];
        in0 = 1.0f / sa[0];
        smul4 = m.scales[4] * sa[4];
    }
    // biases (accumulator units): layers 0-3 at 64 L, layer 4 at 256 padded to 32 rows
    __shared__ __attribute__((aligned(16))) float sb[kBiasSlots];
    const float *bias = reinterpret_cast<const float *>(reinterpret_cast<const uint8_t *>(m.weights) + kBiasOff);
    for (int i = threadIdx.x; i < kBiasSlots; i += kInferBlock) {
        const int L = i < 256 ? i >> 6 : 4;
        float b = bias[i];
        if (P == GI_MLP_FP8) {
            float sa = m.scales[5 + L];
            if (!(sa > 0.0f && sa < kInf)) sa = 1.0f;
            b = b / (m.scales[L] * sa);
        }
        sb[i] = b;
    }
    // the fragments of layers 0 and 1 (18) stay in LDS and are re-read per
    // tile; the other 20 live in registers for the whole kernel (3 waves per
    // SIMD for BF16, 4 for FP8, without spills)
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
    float lo[3], ext[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = h ? 0.0f : m.pos_lo[a];
        ext[a] = h ? 1.0f : m.pos_hi[a] - m.pos_lo[a];
    }
    const float4 *src = h ? nrm : pos;
    const uint32_t wave = (blockIdx.x * kInferBlock + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * kInferBlock) >> 6;
    const uint32_t ntiles = (n + 31u) / 32u;

    for (uint32_t tile = wave; tile < ntiles; tile += nwaves) {
        // the LDS fragments and biases are re-read every tile: hoisted out of
        // the loop they would take 36 (FP8) to 72 (BF16) more registers
        // plus the bias tiles, and cost waves (FP8: 341 registers, 1 wave)
        asm volatile("" ::: "memory");
        const uint32_t idx = tile * 32u + (uint32_t)s;
        const bool ok = idx < n;
        const float4 in = ok ? src[idx] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float feat[40];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v = (comp(in, a) - lo[a]) / ext[a];
            feat[13 * a] = v;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                // sin(2^j pi v) = sin of 2^(j-1) v revolutions, reduced exactly to [0, 1)
                const float x = __builtin_amdgcn_fractf(v * (float)(1 << j) * 0.5f);
                feat[13 * a + 1 + 2 * j] = sin_rev(x);
                feat[13 * a + 2 + 2 * j] = cos_rev(x);
            }
        }
        feat[39] = 0.0f;

        // layer 0: K = 80 (5 k-steps), two output tiles
        f32x16 acc0 = bias_tile(sb, h), acc1 = bias_tile(sb + 32, h);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            f32x8 x;
#pragma unroll
            for (int v = 0; v < 8; ++v) x[v] = feat[8 * c + v];
            FT b;
            if constexpr (P == GI_MLP_BF16) {
                b = to_bf16(x);
            } else {
#pragma unroll
                for (int v = 0; v < 8; ++v) x[v] = __builtin_amdgcn_fmed3f(x[v] * in0, -kFp8Max, kFp8Max);
                b = to_fp8(x);
            }
            acc0 = mfma(frag(c), b, acc0);
            acc1 = mfma(frag(5 + c), b, acc1);
        }
        // hidden layers 1-3 and the output layer 4
#pragma unroll
        for (int L = 1; L < kLayers; ++L) {
            FT bop[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if constexpr (P == GI_MLP_BF16) {
                    bop[c] = relu_operand(c >> 1 ? acc1 : acc0, c & 1);
                } else {
                    f32x8 x = half_of(c >> 1 ? acc1 : acc0, c & 1);
                    // ReLU, rescale to the next layer's input scale, saturate
#pragma unroll
                    for (int v = 0; v < 8; ++v) x[v] = __builtin_amdgcn_fmed3f(x[v] * kq[L - 1], 0.0f, kFp8Max);
                    bop[c] = to_fp8(x);
                }
            }
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
            out[idx] = make_float4(acc0[0] * smul4, acc0[1] * smul4, acc0[2] * smul4, 0.0f);
        }
    }
}

// --------------------------------------------------------------------------
// training
// --------------------------------------------------------------------------
// LDS weights: row-major [u][k] with row stride in+1 (conflict-free both for
// lanes along u and along k); the layer offsets coincide with the flat
// parameter offsets of the weights.
constexpr int kWStride[kLayers] = {79, 65, 65, 65, 65};
// layer inputs: [s][k] with stride 80 (layer 0) or 64
constexpr int kAOff[kLayers] = {0, 32 * 80, 32 * 80 + 2048, 32 * 80 + 4096, 32 * 80 + 6144};
constexpr int kAStride[kLayers] = {80, 64, 64, 64, 64};
constexpr int kASize = 32 * 80 + 4 * 2048;

__device__ __forceinline__ float block_sum(float v, float *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int o = kTrainBlock / 2; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    float r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ float block_max(float v, float *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int o = kTrainBlock / 2; o > 0; o >>= 1) {
        if (t < o) red[t] = fmaxf(red[t], red[t + o]);
        __syncthreads();
    }
    float r = red[0];
    __syncthreads();
    return r;
}

// number of valid samples (target.w != 0) -> hdr[0]
__global__ void __launch_bounds__(1024) k_mlp_count(uint32_t n, const float4 *tgt, uint32_t *hdr)
{
    __shared__ uint32_t red[1024];
    const int t = threadIdx.x;
    uint32_t c = 0;
    for (uint32_t i = t; i < n; i += 1024) c += tgt[i].w != 0.0f ? 1u : 0u;
    red[t] = c;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    if (t == 0) hdr[0] = red[0];
}

__global__ void __launch_bounds__(kTrainBlock) k_mlp_fwdbwd(gi_mlp m, uint32_t n, const float4 *pos,
                                                            const float4 *nrm, const float4 *tgt,
                                                            const float4 *qp, const uint32_t *hdr, float *part)
{
    __shared__ float sW[kParams];
    __shared__ float sA[kASize];
    __shared__ float sG[2][kTrainS * 64];
    __shared__ float sGr[kTrainS * 64];
    __shared__ float sO[kTrainS * 4], sT[kTrainS * 4], sQ[kTrainS * 4];
    __shared__ float sX[kTrainS * 8];
    __shared__ int sValid[kTrainS];
    __shared__ float red[kTrainBlock];

    const int t = threadIdx.x;
    const uint32_t s0 = blockIdx.x * kTrainS;
    float *pw = part + (size_t)blockIdx.x * kPartStride;

    // weights, rounded to BF16
    for (int L = 0; L < kLayers; ++L) {
        const int in = kIn[L], cnt = in * kOut[L];
        for (int r = t; r < cnt; r += kTrainBlock) {
            const int u = r / in, k = r - u * in;
            sW[kOffW[L] + u * kWStride[L] + k] = bf16_round(m.params[kOffW[L] + r]);
        }
    }
    // per-sample inputs
    if (t < kTrainS) {
        const uint32_t i = s0 + t;
        const bool in_range = i < n;
        const float4 tg = in_range ? tgt[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const bool valid = in_range && tg.w != 0.0f;
        sValid[t] = valid ? 1 : 0;
        const float4 p = valid ? pos[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const float4 nn = valid ? nrm[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const float4 q = (valid && qp) ? qp[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        for (int a = 0; a < 3; ++a) {
            sX[8 * t + a] = (comp(p, a) - m.pos_lo[a]) / (m.pos_hi[a] - m.pos_lo[a]);
            sX[8 * t + 3 + a] = comp(nn, a);
            sT[4 * t + a] = comp(tg, a);
            sQ[4 * t + a] = comp(q, a);
        }
    }
    __syncthreads();
    float amax[kLayers] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    // encoding (precise sin(pi x) / cos(pi x), exact range reduction)
    for (int e = t; e < kTrainS * 80; e += kTrainBlock) {
        const int s = e / 80, f = e - s * 80;
        float x = 0.0f;
        if (f < 78 && sValid[s]) {
            const int i = f / 13, ee = f - 13 * i;
            const float v = sX[8 * s + i];
            if (ee == 0) x = v;
            else if (ee & 1) x = sinpif(ldexpf(v, (ee - 1) >> 1));
            else x = cospif(ldexpf(v, (ee - 2) >> 1));
            amax[0] = fmaxf(amax[0], fabsf(x));
        }
        sA[s * 80 + f] = bf16_round(x);
    }
    __syncthreads();

    // forward, hidden layers: thread (unit u, samples sg + 4i)
    const int u = t & 63, sg = t >> 6;
    for (int L = 0; L < kLayers - 1; ++L) {
        const int in = kIn[L];
        const float *A = sA + kAOff[L];
        const float *Wr = sW + kOffW[L] + u * kWStride[L];
        float acc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = 0.0f;
        for (int k = 0; k < in; ++k) {
            const float w = Wr[k];
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] = fmaf(A[(sg + 4 * i) * kAStride[L] + k], w, acc[i]);
        }
        const float b = m.params[kOffB[L] + u];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int s = sg + 4 * i;
            const float a = fmaxf(acc[i] + b, 0.0f);
            if (sValid[s]) amax[L + 1] = fmaxf(amax[L + 1], a);
            sA[kAOff[L + 1] + s * 64 + u] = bf16_round(a);
        }
        __syncthreads();
    }
    // output layer and loss gradient: thread (sample s, channel c)
    const float ntot = (float)max(hdr[0], 1u) * 3.0f;
    float loss = 0.0f, enum_ = 0.0f, eden = 0.0f, nonfinite = 0.0f;
    if (t < kTrainS * 3) {
        const int s = t / 3, c = t - 3 * s;
        const float *A = sA + kAOff[4] + s * 64;
        const float *Wr = sW + kOffW[4] + c * kWStride[4];
        float z = 0.0f;
        for (int k = 0; k < 64; ++k) z = fmaf(A[k], Wr[k], z);
        z += m.params[kOffB[4] + c];
        sO[4 * s + c] = z;
        float g = 0.0f;
        if (sValid[s]) {
            const float den = z * z + 0.01f, d = z - sT[4 * s + c];
            g = 2.0f * d / den / ntot;
            loss = d * d / den;
            const float q = sQ[4 * s + c];
            enum_ = fabsf(fmaxf(z, 0.0f) - q);
            eden = q + 0.01f;
            nonfinite = __builtin_isfinite(z) ? 0.0f : 1.0f;
        }
        sG[0][s * 64 + c] = g;
        sGr[s * 64 + c] = bf16_round(g);
    }
    {
        const float st[4] = {loss, enum_, eden, nonfinite};
        for (int j = 0; j < 4; ++j) {
            const float r = block_sum(st[j], red);
            if (t == 0) pw[kParams + j] = r;
        }
        for (int L = 0; L < kLayers; ++L) {
            const float r = block_max(amax[L], red);
            if (t == 0) pw[kParams + kStAmax0 + L] = r;
        }
    }
    __syncthreads();

    // backward
    int cur = 0;
    for (int L = kLayers - 1; L >= 0; --L) {
        const int in = kIn[L], out = kOut[L];
        const float *A = sA + kAOff[L];
        const int as = kAStride[L];
        if (t < out) {
            float db = 0.0f;
            for (int s = 0; s < kTrainS; ++s) db += sG[cur][s * 64 + t];
            pw[kOffB[L] + t] = db;
        }
        for (int r = t; r < in * out; r += kTrainBlock) {
            const int uu = r / in, k = r - uu * in;
            float dw = 0.0f;
            for (int s = 0; s < kTrainS; ++s) dw = fmaf(sGr[s * 64 + uu], A[s * as + k], dw);
            pw[kOffW[L] + r] = dw;
        }
        if (L == 0) break;
        // gradient w.r.t. this layer's input (64 units), masked by the ReLU of the previous layer
        {
            const int k = t & 63;
            const float *Wc = sW + kOffW[L] + k;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int s = sg + 4 * i;
                float g = 0.0f;
                for (int uu = 0; uu < out; ++uu) g = fmaf(sGr[s * 64 + uu], Wc[uu * kWStride[L]], g);
                sG[cur ^ 1][s * 64 + k] = A[s * 64 + k] > 0.0f ? g : 0.0f;
            }
        }
        __syncthreads();
        for (int e = t; e < kTrainS * 64; e += kTrainBlock) sGr[e] = bf16_round(sG[cur ^ 1][e]);
        __syncthreads();
        cur ^= 1;
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
    float acc = 0.0f;
    for (uint32_t w = w0; w < w1; ++w) {
        const float x = part[(size_t)w * kPartStride + p];
        acc = is_max ? fmaxf(acc, x) : acc + x;
    }
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
    float acc = 0.0f;
    for (uint32_t w = 0; w < nwg; w += kGroup) {
        const float x = part[(size_t)w * kPartStride + p];
        acc = is_max ? fmaxf(acc, x) : acc + x;
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
        m.state[GI_MLP_STATE_BATCH_ERR] = __float_as_uint(den > 0.0f ? acc / den : 0.0f);
    } else if (j == kStNonFinite) {
        m.state[GI_MLP_STATE_NONFINITE] = (uint32_t)acc;
    } else if (is_max) {
        m.scales[5 + (j - kStAmax0)] = acc > 0.0f ? acc / kFp8Max : 1.0f;
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

// usability after step t (one workgroup)
__global__ void __launch_bounds__(256) k_mlp_state(gi_mlp m, uint32_t t)
{
    __shared__ float red[256];
    const int tid = threadIdx.x;
    float bad = 0.0f;
    for (int p = tid; p < kParams; p += 256) bad += __builtin_isfinite(m.params[p]) ? 0.0f : 1.0f;
    red[tid] = bad;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) {
        const float be = __uint_as_float(m.state[GI_MLP_STATE_BATCH_ERR]);
        const float old = __uint_as_float(m.state[GI_MLP_STATE_EMA_ERR]);
        const float ema = t <= 1u ? be : 0.9f * old + 0.1f * be;
        const bool ok = t >= m.warmup_steps && m.state[GI_MLP_STATE_NONFINITE] == 0u && ema <= m.max_rel_err &&
                        red[0] == 0.0f;
        m.state[GI_MLP_STATE_STEPS] = t;
        m.state[GI_MLP_STATE_EMA_ERR] = __float_as_uint(ema);
        m.state[GI_MLP_STATE_USABLE] = ok ? 1u : 0u;
    }
}

constexpr uint32_t train_wgs(uint32_t n) { return (n + kTrainS - 1) / kTrainS; }

constexpr uint64_t train_bytes(uint32_t n) { return 4ull * (kHdr + (uint64_t)kPartStride * (1ull + train_wgs(n))); }

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
    const int blocks = (kFrags * 64 * 8 + 255) / 256;
    if (m.precision == GI_MLP_BF16) {
        k_mlp_prepare_bf16<<<blocks, 256, 0, st>>>(m);
    } else {
        k_mlp_wscale<<<kLayers, 256, 0, st>>>(m);
        k_mlp_prepare_fp8<<<blocks, 256, 0, st>>>(m);
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
    if (nwg)
        k_mlp_fwdbwd<<<nwg, kTrainBlock, 0, st>>>(m, n, reinterpret_cast<const float4 *>(pos4),
                                                  reinterpret_cast<const float4 *>(nrm4),
                                                  reinterpret_cast<const float4 *>(target4),
                                                  reinterpret_cast<const float4 *>(qprobe4), hdr, part);
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
    k_mlp_state<<<1, 256, 0, st>>>(m, t);
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
        k_mlp_infer<GI_MLP_BF16><<<blocks, kInferBlock, 0, st>>>(m, n, pos, nrm, out, gate ? 1 : 0);
    else
        k_mlp_infer<GI_MLP_FP8><<<blocks, kInferBlock, 0, st>>>(m, n, pos, nrm, out, gate ? 1 : 0);
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
