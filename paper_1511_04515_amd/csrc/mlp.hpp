// The learned step controller's network on the device: 8 -> 64 -> 64 -> 2
// with ReLU hidden layers.  Training parameters are one float vector in the
// order
//   W1 (64 x 8, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (2 x 64), b3 (2)
// (4,866 numbers).  Inference keeps the same offsets with W1 and W2 stored
// transposed (W1T[i][j] = W1[j][i], W2T likewise), so that lane j of a wave
// reads unit j's weights with coalesced loads.  Inputs and outputs are
// standardised with norm = {x mean (8), x std (8), t mean (2), t std (2)}.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace expri {

constexpr int kMlpIn = 8, kMlpHid = 64, kMlpOut = 2;
constexpr int kMlpW1 = 0;
constexpr int kMlpB1 = kMlpW1 + kMlpHid * kMlpIn;
constexpr int kMlpW2 = kMlpB1 + kMlpHid;
constexpr int kMlpB2 = kMlpW2 + kMlpHid * kMlpHid;
constexpr int kMlpW3 = kMlpB2 + kMlpHid;
constexpr int kMlpB3 = kMlpW3 + kMlpOut * kMlpHid;
constexpr int kMlpParams = kMlpB3 + kMlpOut;  // 4866
constexpr int kMlpNorm = 2 * (kMlpIn + kMlpOut);

// round a float to bfloat16 (nearest, ties to even), kept as a float
__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

__device__ __forceinline__ float mlp_w(const uint16_t *w, int i) { return __uint_as_float((uint32_t)w[i] << 16); }
__device__ __forceinline__ float mlp_w(const float *w, int i) { return w[i]; }

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wave evaluates the network on one sample f (raw features, the same in
// every lane); lane j owns hidden unit j; every lane returns the
// de-standardised outputs.  With bfloat16 weights (uint16_t storage) the
// standardised inputs and the hidden activations are rounded to bfloat16 as
// well; sums are float32 in a fixed order.
template <class W>
__device__ __forceinline__ void mlp_infer_wave(const W *w, const float *norm, const float *f, float *out) {
  constexpr bool bf16 = sizeof(W) == 2;
  const int j = threadIdx.x & 63;
  float x[kMlpIn];
#pragma unroll
  for (int i = 0; i < kMlpIn; ++i) {
    x[i] = (f[i] - norm[i]) / norm[kMlpIn + i];
    if (bf16) x[i] = bf16_round(x[i]);
  }
  float z = mlp_w(w, kMlpB1 + j);
#pragma unroll
  for (int i = 0; i < kMlpIn; ++i) z = fmaf(mlp_w(w, kMlpW1 + i * kMlpHid + j), x[i], z);
  float a1 = fmaxf(z, 0.0f);
  if (bf16) a1 = bf16_round(a1);
  z = mlp_w(w, kMlpB2 + j);
#pragma unroll 16
  for (int i = 0; i < kMlpHid; ++i) {
    const float ai = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a1), i));
    z = fmaf(mlp_w(w, kMlpW2 + i * kMlpHid + j), ai, z);
  }
  float a2 = fmaxf(z, 0.0f);
  if (bf16) a2 = bf16_round(a2);
#pragma unroll
  for (int o = 0; o < kMlpOut; ++o) {
    const float y = mlp_w(w, kMlpB3 + o) + wave_sum_f(mlp_w(w, kMlpW3 + o * kMlpHid + j) * a2);
    out[o] = y * norm[2 * kMlpIn + kMlpOut + o] + norm[2 * kMlpIn + o];
  }
}

}  // namespace expri
