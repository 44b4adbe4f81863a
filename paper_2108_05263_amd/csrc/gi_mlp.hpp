// Layout constants of the learned radiance cache and the launchers the
// resampling kernels share with the MLP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "gi.h"

namespace gi {
namespace mlp {

// layers (in, out): 78-64, 64-64 (x3), 64-3; flat parameter offsets
constexpr int kLayers = 5;
constexpr int kIn[kLayers] = {78, 64, 64, 64, 64};
constexpr int kOut[kLayers] = {64, 64, 64, 64, 3};
constexpr int kOffW[kLayers] = {0, 5056, 9216, 13376, 17536};
constexpr int kOffB[kLayers] = {4992, 9152, 13312, 17472, 17728};
constexpr int kParams = 17731;
static_assert(kOffB[4] + 3 == kParams, "parameter layout");

// MFMA fragments (32x32x16): per layer, output tiles of 32 rows x k-steps
// of 16.  Layer 0 has 2 tiles x 5 steps (K = 78 padded to 80), layers 1-3
// 2 x 4, layer 4 one tile x 4.  Fragment f holds 64 lanes x 8 operands.
constexpr int kTiles[kLayers] = {2, 2, 2, 2, 1};
constexpr int kSteps[kLayers] = {5, 4, 4, 4, 4};
constexpr int kFrag0[kLayers] = {0, 10, 18, 26, 34};
constexpr int kFrags = 38;
// after the fragments: FP32 biases, layers 0-3 at 64 L, layer 4 at 256 (32 rows, 3 used)
constexpr int kBiasOff = kFrags * 64 * 16;
constexpr int kBiasSlots = 4 * 64 + 32;
static_assert(kBiasOff + kBiasSlots * 4 == GI_MLP_WEIGHT_BYTES, "weight buffer bytes");

// The encoded input is split between the two half-waves: lanes 0-31 hold
// the 39 features of the three position values, lanes 32-63 those of the
// three normal components; slot j = 8c + v (k-step c, operand v) of half h
// is feature 39h + j, slot 39 is zero padding.
__host__ __device__ constexpr int l0_feature(int h, int j) { return j < 39 ? 39 * h + j : -1; }

// Hidden layers take their input straight from the previous layer's
// accumulators.  Lane half h holds units 8a + 4h + b of each 32-row tile
// (accumulator 4a + b), while a k-step's operand slots are 16c + 8h + v; the
// weight column feeding slot kappa is therefore pi(kappa) = kappa with bits
// 2 and 3 swapped, and slot v of k-step c is accumulator 8(c & 1) + v of
// tile c >> 1.
__host__ __device__ constexpr int swap23(int k) { return (k & ~12) | ((k & 4) << 1) | ((k & 8) >> 1); }

constexpr uint32_t kStateWords = GI_MLP_STATE_WORDS;

}  // namespace mlp

// Launch the cache on n points (float4 planes pos, nrm; out float4).  With
// gate set, waves return at once unless the mode / device state selects the
// cache (the same decision the resampling kernels take).
gi_status mlp_infer_launch(const gi_mlp &m, uint32_t n, const float4 *pos, const float4 *nrm, float4 *out,
                           bool gate, hipStream_t stream);

gi_status check_mlp(const gi_mlp *m);

// Does this mode / state select the cache?  (device side)
__device__ __forceinline__ bool mlp_selected(const gi_mlp &m)
{
    if (m.mode == GI_MLP_ALWAYS) return true;
    if (m.mode == GI_MLP_NEVER) return false;
    return m.state[GI_MLP_STATE_USABLE] != 0u;
}

}  // namespace gi
