// Learned temperature-step proposer: an MLP 8 -> 64 -> 64 -> 1 with ReLU.
// Parameter vector (FP32 master copy, 4801 floats):
//   W1 [64][8] | b1 [64] | W2 [64][64] | b2 [64] | w3 [64] | b3
// Normalisation (18 floats, not trained): x_mean[8] | x_std[8] | t_mean | t_std.
// The network maps normalised features to its normalised target, the log of
// the temperature step times the energy spread of the population.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {
namespace mlp {

constexpr int kIn = 8;
constexpr int kHid = 64;
constexpr int kW1 = 0;
constexpr int kB1 = kW1 + kHid * kIn;
constexpr int kW2 = kB1 + kHid;
constexpr int kB2 = kW2 + kHid * kHid;
constexpr int kW3 = kB2 + kHid;
constexpr int kB3 = kW3 + kHid;
constexpr int kParams = kB3 + 1;
constexpr int kNorm = 2 * kIn + 2;
static_assert(kParams == 4801, "parameter count");

// Round to bfloat16 (round to nearest even) and back: the inference path keeps
// weights and activations in BF16 and accumulates in FP32.
__device__ __forceinline__ float bf16r(float x) { return __bfloat162float(__float2bfloat16(x)); }

// Forward pass of one sample by the 64 threads t = 0..63 of a block (t is the
// hidden unit).  x: raw features (normalised here); wb: BF16 parameters;
// norm: normalisation constants; h: 64 floats of shared scratch.  Returns the
// de-normalised output in thread 0.
__device__ __forceinline__ float forward_bf16(const float* x, const __hip_bfloat16* wb, const float* norm, float* h,
                                              int t)
{
    float xn[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) xn[k] = bf16r((x[k] - norm[k]) / norm[kIn + k]);
    float a = __bfloat162float(wb[kB1 + t]);
#pragma unroll
    for (int k = 0; k < kIn; ++k) a += __bfloat162float(wb[kW1 + t * kIn + k]) * xn[k];
    const float h1 = bf16r(a > 0.0f ? a : 0.0f);
    h[t] = h1;
    __syncthreads();
    float a2 = __bfloat162float(wb[kB2 + t]);
    for (int v = 0; v < kHid; ++v) a2 += __bfloat162float(wb[kW2 + t * kHid + v]) * h[v];
    const float h2 = bf16r(a2 > 0.0f ? a2 : 0.0f);
    __syncthreads();
    h[t] = __bfloat162float(wb[kW3 + t]) * h2;
    __syncthreads();
    float y = 0.0f;
    if (t == 0) {
        y = __bfloat162float(wb[kB3]);
        for (int v = 0; v < kHid; ++v) y += h[v];  // fixed order
        y = y * norm[2 * kIn + 1] + norm[2 * kIn];
    }
    __syncthreads();
    return y;
}

}  // namespace mlp
}  // namespace pa
