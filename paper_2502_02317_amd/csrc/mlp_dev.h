// The proposal network's forward pass and float wave reductions, shared by
// the search-time ranking kernel and the training kernels.
//
// Parameters (float32, 8H + 1): W1 [H][F] row-major, b1 [H], w2 [H], b2.
// logit(f) = b2 + sum_h w2[h] * relu(b1[h] + W1[h] . f), F = 6 features.
#pragma once

#include <hip/hip_runtime.h>

namespace spg {

constexpr int kFeat = 6;
constexpr int kMaxHidden = 64;

__host__ __device__ inline int mlp_n_params(int H) { return H * kFeat + 2 * H + 1; }

__device__ __forceinline__ float mlp_logit(const float *prm, int H, const float *f) {
  const float *W1 = prm, *b1 = prm + H * kFeat, *w2 = b1 + H;
  float acc = w2[H];
  for (int h = 0; h < H; ++h) {
    float a = b1[h];
#pragma unroll
    for (int k = 0; k < kFeat; ++k) a = fmaf(W1[h * kFeat + k], f[k], a);
    acc = fmaf(w2[h], fmaxf(a, 0.0f), acc);
  }
  return acc;
}

__device__ __forceinline__ float wave_max_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float wave_sum_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

}  // namespace spg
