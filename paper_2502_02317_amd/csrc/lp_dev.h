// Device helpers of the reduced-precision search (FP32 or BF16 boundary-MPS
// tensors, FP32 environment vectors), shared by the plain steps and the
// proposal's guarded steps, so that both compute a parent's conditionals with
// the same arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp_dev.h"
#include "search_dev.h"
#include "spg_internal.h"

namespace spg {

// round-to-nearest-even FP32 -> BF16 (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

template <class T> __device__ __forceinline__ float ld(const T *p, long i);
template <> __device__ __forceinline__ float ld<float>(const float *p, long i) { return p[i]; }
template <> __device__ __forceinline__ float ld<uint16_t>(const uint16_t *p, long i) {
  return bf2f(p[i]);
}

// vector store with the form's rounding
__device__ __forceinline__ float vround(float v, int bf16) { return bf16 ? bf2f(f2bf(v)) : v; }

// log g^b_c(s): log of the couplings of x_{r,c} = s to the fixed row above
__device__ __forceinline__ double log_field(const SearchTabs &t, int r, int c, const uint8_t *cb,
                                            int s) {
  if (r == 0) return 0.0;
  const int C = t.cols, d = t.d;
  const uint8_t *up = cb + (r - 1) * C;
  const long dd = (long)d * d;
  double g = t.W_v[((long)(r - 1) * C + c) * dd + up[c] * d + s];
  if (c > 0) g *= t.W_d[((long)(r - 1) * (C - 1) + (c - 1)) * dd + up[c - 1] * d + s];
  if (c < C - 1) g *= t.W_a[((long)(r - 1) * (C - 1) + c) * dd + up[c + 1] * d + s];
  return log(g);
}

// log p(s | b) of the reduced-precision search for s = lane + 64 h (h < 4;
// -inf beyond d), one wavefront per parent b: q(b, s) = g^b(s) sum_al L^b[al]
// U^{anc(b)}[al][s] in FP32 (U = the column's A R_{c+1} products), negative q
// (truncation error) = probability 0, normalised over s in FP32.  For d <= 64
// the lanes form 64 / d groups, group j summing the al = j mod (64 / d)
// terms, and lane s adds the groups' sums in group order.  A parent without a
// positive q takes softmax_s(-beta dE) (local_softmax_norm).
__device__ inline void lp_parent_logp(const SearchTabs &t, int r, int c, int b,
                                      const uint8_t *cfg, int N, const float *U, long ldu,
                                      const float *L, const int32_t *anc, int cl, int lane,
                                      double (&lp)[4]) {
  const int chi = t.chi, d = t.d;
  const float *Ua = U + (long)anc[b] * ldu;
  const float *Lb = L + (long)b * chi;
  float q[4] = {0.f, 0.f, 0.f, 0.f};
  if (d <= 64) {
    const int G = 64 / d, s = lane % d, j = lane / d;
    float part = 0.f;
    if (j < G)
      for (int al = j; al < cl; al += G) part = fmaf(Lb[al], Ua[(long)al * d + s], part);
    float tot = 0.f;
    for (int jj = 0; jj < G; ++jj) tot += __shfl(part, s + jj * d, 64);
    q[0] = tot;
  } else {
    for (int h = 0; h < 4; ++h) {
      const int s = lane + 64 * h;
      if (s >= d) continue;
      float acc = 0.f;
      for (int al = 0; al < cl; ++al) acc = fmaf(Lb[al], Ua[(long)al * d + s], acc);
      q[h] = acc;
    }
  }
  const uint8_t *cb = cfg + (long)b * N;
  float lq[4];
  float mx = -INFINITY;
  for (int h = 0; h < 4; ++h) {
    const int s = lane + 64 * h;
    lq[h] = -INFINITY;
    if (s >= d) continue;
    // negative q (truncation error) = probability 0
    lq[h] = (q[h] > 0.f) ? (float)log_field(t, r, c, cb, s) + logf(q[h]) : -INFINITY;
    mx = fmaxf(mx, lq[h]);
  }
  mx = wave_max_f(mx);
  if (!(mx > -INFINITY)) {                 // no child with positive weight
    double emin, lse;
    local_softmax_norm(t, r, c, cb, lane, emin, lse);
    for (int h = 0; h < 4; ++h) {
      const int s = lane + 64 * h;
      lp[h] = (s < d) ? -t.beta * (delta_energy(t, r, c, cb, s) - emin) - lse : -INFINITY;
    }
    return;
  }
  float se = 0.f;
  for (int h = 0; h < 4; ++h)
    if (lane + 64 * h < d && lq[h] > -INFINITY) se += expf(lq[h] - mx);
  se = wave_sum_f(se);
  const float lse = mx + logf(se);
  for (int h = 0; h < 4; ++h) {
    const int s = lane + 64 * h;
    const float l = (s < d && lq[h] > -INFINITY && mx > -INFINITY) ? lq[h] - lse : -INFINITY;
    lp[h] = (double)l;
  }
}

}  // namespace spg
