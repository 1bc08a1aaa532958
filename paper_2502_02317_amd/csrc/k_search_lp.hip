// Search contractions in reduced precision (the precision form): boundary-MPS
// tensors A in FP32, or in BF16 with FP32 accumulation; environment vectors L
// and R are FP32 (rounded to BF16 on store in the BF16 form).  Couplings to
// the fixed row enter in log domain, relative to their maximum over s, so FP32
// cannot underflow on them; log-probabilities are added to FP64 scores.
#include <cfloat>

#include "spg_internal.h"

namespace spg {

namespace {

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ float wave_sum_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_max_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

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

constexpr int kW = 4;

template <class T>
__global__ __launch_bounds__(256) void k_right_env_lp(SearchTabs t, int r, int c, int n_anc,
                                                      const uint8_t *cfg, int N, const T *A,
                                                      const float *Rnext, float *Rout,
                                                      long rstride, int bf16) {
  __shared__ float Rs[kW][kMaxChi];
  __shared__ float gs[kW][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int a0 = blockIdx.x * kW + w;
  const bool valid = a0 < n_anc;
  const int a = valid ? a0 : 0;
  const int chi = t.chi, d = t.d;
  const uint8_t *cb = cfg + (long)a * N;
  double lmax = -INFINITY;
  double lg[4];
  for (int h = 0; h < 4; ++h) {
    const int s = lane + 64 * h;
    lg[h] = (s < d) ? log_field(t, r, c, cb, s) : -INFINITY;
    lmax = fmax(lmax, lg[h]);
  }
  for (int o = 32; o > 0; o >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, o, 64));
  if (valid) {
    for (int i = lane; i < chi; i += 64) Rs[w][i] = Rnext[a * rstride + i];
    for (int h = 0; h < 4; ++h) {
      const int s = lane + 64 * h;
      if (s < d) gs[w][s] = (float)exp(lg[h] - lmax);
    }
  }
  __syncthreads();
  if (!valid) return;
  float v[2] = {0.f, 0.f};
  for (int h = 0; h < 2; ++h) {
    const int al = lane + 64 * h;
    if (al >= chi) continue;
    float acc = 0.f;
    for (int s = 0; s < d; ++s) {
      const long base = ((long)al * d + s) * chi;
      float u = 0.f;
      for (int b = 0; b < chi; ++b) u = fmaf(ld(A, base + b), Rs[w][b], u);
      acc = fmaf(gs[w][s], u, acc);
    }
    v[h] = acc;
  }
  const float m = wave_max_f(fmaxf(fabsf(v[0]), fabsf(v[1])));
  const float inv = (m > 0.f) ? 1.f / m : 1.f;
  for (int h = 0; h < 2; ++h) {
    const int al = lane + 64 * h;
    if (al < chi) Rout[a * rstride + al] = vround(v[h] * inv, bf16);
  }
}

// out[b*d+s] = (add_score ? score[b] : 0) + log p(s | b)
// The same with the site tensor staged in LDS once per workgroup (when its
// cl x d x cr block fits): every lane of an ancestor's wavefront takes
// (al, s) pairs, u[al][s] = sum_b A[al][s][b] R[b] in b order, then lane al
// sums g(s) u[al][s] in s order; rows al >= cl are zero as before.  The same
// order of terms as k_right_env_lp: identical results.
constexpr int kEnvLds = 32 * 16 * 33;      // floats of the staged block, cl * d * (cr + 1)
constexpr int kEnvU = 32 * 16;             // per-wave u[al][s], cl * d

__host__ __device__ constexpr bool env_lds_fits(int cl, int d, int cr) {
  return d <= 64 && cr <= 64 && cl * d <= kEnvU && cl * d * (cr + 1) <= kEnvLds;
}

template <class T>
__global__ __launch_bounds__(256) void k_right_env_lp_lds(SearchTabs t, int r, int c, int n_anc,
                                                          const uint8_t *cfg, int N, const T *A,
                                                          const float *Rnext, float *Rout,
                                                          long rstride, int bf16, int cl, int cr) {
  __shared__ float As[kEnvLds];
  __shared__ float us[kW][kEnvU];
  __shared__ float Rs[kW][kMaxChi];
  __shared__ float gs[kW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int a0 = blockIdx.x * kW + w;
  const bool valid = a0 < n_anc;
  const int a = valid ? a0 : 0;
  const int chi = t.chi, d = t.d;
  const int npair = cl * d, ldr = cr + 1;
  {
    const int rpp = 64 / cr, sub = lane / cr, bb = lane - sub * cr;
    if (sub < rpp) {
      const int step = kW * rpp;
      int p = w * rpp + sub;
      for (; p + 7 * step < npair; p += 8 * step) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = ld(A, (long)(p + k * step) * chi + bb);
#pragma unroll
        for (int k = 0; k < 8; ++k) As[(p + k * step) * ldr + bb] = v[k];
      }
      for (; p < npair; p += step) As[p * ldr + bb] = ld(A, (long)p * chi + bb);
    }
  }
  const uint8_t *cb = cfg + (long)a * N;
  // couplings relative to their largest value over s
  double lg = (lane < d) ? log_field(t, r, c, cb, lane) : -INFINITY;
  double lmax = lg;
  for (int o = 32; o > 0; o >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, o, 64));
  if (valid) {
    for (int i = lane; i < chi; i += 64) Rs[w][i] = Rnext[a * rstride + i];
    if (lane < d) gs[w][lane] = (float)exp(lg - lmax);
  }
  __syncthreads();
  if (valid) {
    for (int p0 = 0; p0 < npair; p0 += 64 * 8) {
      float u[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) u[k] = 0.f;
      const int pl = p0 + lane;
      for (int b = 0; b < cr; ++b) {
        const float rb = Rs[w][b];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (pl + 64 * k < npair) u[k] = fmaf(As[(pl + 64 * k) * ldr + b], rb, u[k]);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (pl + 64 * k < npair) us[w][pl + 64 * k] = u[k];
    }
  }
  __syncthreads();
  if (!valid) return;
  float v[2] = {0.f, 0.f};
  for (int h = 0; h < 2; ++h) {
    const int al = lane + 64 * h;
    if (al >= cl) continue;
    float acc = 0.f;
    for (int s = 0; s < d; ++s) acc = fmaf(gs[w][s], us[w][al * d + s], acc);
    v[h] = acc;
  }
  const float m = wave_max_f(fmaxf(fabsf(v[0]), fabsf(v[1])));
  const float inv = (m > 0.f) ? 1.f / m : 1.f;
  for (int h = 0; h < 2; ++h) {
    const int al = lane + 64 * h;
    if (al < chi) Rout[a * rstride + al] = vround(v[h] * inv, bf16);
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_marginals_lp(SearchTabs t, int r, int c, int n_beam,
                                                      const uint8_t *cfg, int N, const T *A,
                                                      const float *L, const int32_t *anc,
                                                      const float *Rv, long rstride,
                                                      const double *score, double *out,
                                                      int add_score) {
  __shared__ float Ls[kW][kMaxChi];
  __shared__ float Rs[kW][kMaxChi];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b0 = blockIdx.x * kW + w;
  const bool valid = b0 < n_beam;
  const int b = valid ? b0 : 0;
  const int chi = t.chi, d = t.d;
  const float *Rn = Rv + (long)anc[b] * rstride + (long)(c + 1) * chi;
  if (valid)
    for (int i = lane; i < chi; i += 64) {
      Ls[w][i] = L[(long)b * chi + i];
      Rs[w][i] = Rn[i];
    }
  __syncthreads();
  if (!valid) return;
  const uint8_t *cb = cfg + (long)b * N;
  float lq[4];
  float mx = -INFINITY;
  for (int h = 0; h < 4; ++h) {
    const int s = lane + 64 * h;
    lq[h] = -INFINITY;
    if (s >= d) continue;
    float acc = 0.f;
    for (int al = 0; al < chi; ++al) {
      const float la = Ls[w][al];
      if (la == 0.f) continue;
      const long base = ((long)al * d + s) * chi;
      float u = 0.f;
      for (int bb = 0; bb < chi; ++bb) u = fmaf(ld(A, base + bb), Rs[w][bb], u);
      acc = fmaf(la, u, acc);
    }
    // negative q (truncation error) = probability 0
    lq[h] = (acc > 0.f) ? (float)log_field(t, r, c, cb, s) + logf(acc) : -INFINITY;
    mx = fmaxf(mx, lq[h]);
  }
  mx = wave_max_f(mx);
  float se = 0.f;
  for (int h = 0; h < 4; ++h)
    if (lane + 64 * h < d && lq[h] > -INFINITY) se += expf(lq[h] - mx);
  se = wave_sum_f(se);
  const float lse = mx + logf(se);
  const double base = add_score ? score[b] : 0.0;
  for (int h = 0; h < 4; ++h) {
    const int s = lane + 64 * h;
    if (s >= d) continue;
    const float lp = (lq[h] > -INFINITY && mx > -INFINITY) ? lq[h] - lse : -INFINITY;
    out[(long)b * d + s] = base + (double)lp;
  }
}

// The same conditionals with the site tensor staged in LDS once per
// workgroup (when its cl x d x cr block fits): all 64 lanes of a beam's wave
// take (al, s) pairs, u[al][s] = sum_b A[al][s][b] R[b] in b order with eight
// pairs in flight per lane, then lane s sums L[al] u[al][s] in al order.
// Every sum runs in the same order as above, so the results are identical.
constexpr int kMargLds = 32 * 16 * 33;     // floats of the staged block, cl * d * (cr + 1)
constexpr int kMargU = 32 * 16;            // per-wave u[al][s], cl * d

__host__ __device__ constexpr bool marg_lds_fits(int cl, int d, int cr) {
  return d <= 64 && cr <= 64 && cl * d <= kMargU && cl * d * (cr + 1) <= kMargLds;
}

template <class T>
__global__ __launch_bounds__(256) void k_marginals_lp_lds(SearchTabs t, int r, int c, int n_beam,
                                                          const uint8_t *cfg, int N, const T *A,
                                                          const float *L, const int32_t *anc,
                                                          const float *Rv, long rstride,
                                                          const double *score, double *out,
                                                          int add_score, int cl, int cr) {
  __shared__ float As[kMargLds];
  __shared__ float us[kW][kMargU];
  __shared__ float Ls[kW][kMaxChi];
  __shared__ float Rs[kW][kMaxChi];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int b0 = blockIdx.x * kW + w;
  const bool valid = b0 < n_beam;
  const int b = valid ? b0 : 0;
  const int chi = t.chi, d = t.d;
  const int npair = cl * d, ldr = cr + 1;
  // A[al][s][0..cr) -> As[(al*d + s)*ldr + .]: each wave copies whole rows,
  // 64 / cr rows per pass, eight rows' loads in flight
  {
    const int rpp = 64 / cr, sub = lane / cr, bb = lane - sub * cr;
    if (sub < rpp) {
      const int step = kW * rpp;
      int p = w * rpp + sub;
      for (; p + 7 * step < npair; p += 8 * step) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = ld(A, (long)(p + k * step) * chi + bb);
#pragma unroll
        for (int k = 0; k < 8; ++k) As[(p + k * step) * ldr + bb] = v[k];
      }
      for (; p < npair; p += step) As[p * ldr + bb] = ld(A, (long)p * chi + bb);
    }
  }
  if (valid) {
    const float *Rn = Rv + (long)anc[b] * rstride + (long)(c + 1) * chi;
    for (int i = lane; i < chi; i += 64) {
      Ls[w][i] = L[(long)b * chi + i];
      Rs[w][i] = Rn[i];
    }
  }
  __syncthreads();
  if (valid) {
    for (int p0 = 0; p0 < npair; p0 += 64 * 8) {
      float u[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) u[k] = 0.f;
      const int pl = p0 + lane;
      for (int bb = 0; bb < cr; ++bb) {
        const float rb = Rs[w][bb];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (pl + 64 * k < npair) u[k] = fmaf(As[(pl + 64 * k) * ldr + bb], rb, u[k]);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (pl + 64 * k < npair) us[w][pl + 64 * k] = u[k];
    }
  }
  __syncthreads();
  if (!valid) return;
  const uint8_t *cb = cfg + (long)b * N;
  float lq = -INFINITY;
  const int s = lane;
  if (s < d) {
    float acc = 0.f;
    for (int al = 0; al < cl; ++al) {
      const float la = Ls[w][al];
      if (la == 0.f) continue;
      acc = fmaf(la, us[w][al * d + s], acc);
    }
    // negative q (truncation error) = probability 0
    lq = (acc > 0.f) ? (float)log_field(t, r, c, cb, s) + logf(acc) : -INFINITY;
  }
  const float mx = wave_max_f(lq);
  float se = (s < d && lq > -INFINITY) ? expf(lq - mx) : 0.f;
  se = wave_sum_f(se);
  const float lse = mx + logf(se);
  if (s < d) {
    const double base = add_score ? score[b] : 0.0;
    const float lp = (lq > -INFINITY && mx > -INFINITY) ? lq - lse : -INFINITY;
    out[(long)b * d + s] = base + (double)lp;
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_beam_update_lp(SearchTabs t, int r, int c, int n_new,
                                                        const int32_t *sel, int N,
                                                        const uint8_t *cfg, const double *energy,
                                                        const float *L, const int32_t *anc,
                                                        const double *cand, const T *A,
                                                        int update_L, uint8_t *cfg_o,
                                                        double *energy_o, double *score_o,
                                                        float *L_o, int32_t *anc_o, int bf16) {
  __shared__ float Ls[kW][kMaxChi];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j0 = blockIdx.x * kW + w;
  const bool valid = j0 < n_new;
  const int j = valid ? j0 : 0;
  const int d = t.d, chi = t.chi, C = t.cols;
  const int id = sel[j];
  const int b = id / d, s = id % d;
  const uint8_t *cb = cfg + (long)b * N;
  uint8_t *co = cfg_o + (long)j * N;
  const int k = r * C + c;
  if (valid)
    for (int i = lane; i < N; i += 64) co[i] = (i == k) ? (uint8_t)s : cb[i];
  if (valid && lane == 0) {
    // FP64 energy increment: the Eq. (1) terms that close at (r, c)
    const long dd = (long)d * d;
    double e = t.E_loc[((long)r * C + c) * d + s];
    if (c > 0) e += t.E_h[((long)r * (C - 1) + (c - 1)) * dd + cb[r * C + c - 1] * d + s];
    if (r > 0) {
      const uint8_t *up = cb + (r - 1) * C;
      e += t.E_v[((long)(r - 1) * C + c) * dd + up[c] * d + s];
      if (c > 0) e += t.E_d[((long)(r - 1) * (C - 1) + (c - 1)) * dd + up[c - 1] * d + s];
      if (c < C - 1) e += t.E_a[((long)(r - 1) * (C - 1) + c) * dd + up[c + 1] * d + s];
    }
    energy_o[j] = energy[b] + e;
    score_o[j] = cand[id];
    anc_o[j] = anc[b];
  }
  if (!update_L) return;
  if (valid)
    for (int i = lane; i < chi; i += 64) Ls[w][i] = L[(long)b * chi + i];
  __syncthreads();
  if (!valid) return;
  // L^child = g L^b A[:, s, :]; the positive factor g cancels after normalisation
  float v[2] = {0.f, 0.f};
  for (int h = 0; h < 2; ++h) {
    const int bp = lane + 64 * h;
    if (bp >= chi) continue;
    float acc = 0.f;
    for (int al = 0; al < chi; ++al) acc = fmaf(Ls[w][al], ld(A, ((long)al * d + s) * chi + bp), acc);
    v[h] = acc;
  }
  const float m = wave_max_f(fmaxf(fabsf(v[0]), fabsf(v[1])));
  const float inv = (m > 0.f) ? 1.f / m : 1.f;
  for (int h = 0; h < 2; ++h) {
    const int bp = lane + 64 * h;
    if (bp < chi) L_o[(long)j * chi + bp] = vround(v[h] * inv, bf16);
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_advance_L_lp(SearchTabs t, int r, int c, int n,
                                                      const uint8_t *cfg, int N, const T *A,
                                                      float *L, int bf16) {
  __shared__ float Ls[kW][kMaxChi];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b0 = blockIdx.x * kW + w;
  const bool valid = b0 < n;
  const int b = valid ? b0 : 0;
  const int d = t.d, chi = t.chi;
  const int s = cfg[(long)b * N + r * t.cols + c];
  if (valid)
    for (int i = lane; i < chi; i += 64) Ls[w][i] = L[(long)b * chi + i];
  __syncthreads();
  if (!valid) return;
  float v[2] = {0.f, 0.f};
  for (int h = 0; h < 2; ++h) {
    const int bp = lane + 64 * h;
    if (bp >= chi) continue;
    float acc = 0.f;
    for (int al = 0; al < chi; ++al) acc = fmaf(Ls[w][al], ld(A, ((long)al * d + s) * chi + bp), acc);
    v[h] = acc;
  }
  const float m = wave_max_f(fmaxf(fabsf(v[0]), fabsf(v[1])));
  const float inv = (m > 0.f) ? 1.f / m : 1.f;
  for (int h = 0; h < 2; ++h) {
    const int bp = lane + 64 * h;
    if (bp < chi) L[(long)b * chi + bp] = vround(v[h] * inv, bf16);
  }
}

__global__ void k_to_f32(long n, const double *src, float *dst) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < n) dst[e] = (float)src[e];
}
__global__ void k_to_bf16(long n, const double *src, uint16_t *dst) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < n) dst[e] = f2bf((float)src[e]);
}
__global__ void k_set_e0_f(int n, int chi, float *p, long stride) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * chi) return;
  const int j = (int)(e / chi), i = (int)(e % chi);
  p[j * stride + i] = (i == 0) ? 1.f : 0.f;
}

}  // namespace

void lp_convert(long n, const double *src, void *dst, int precision, hipStream_t s) {
  bc_single("lp_convert");
  if (n <= 0) return;
  if (precision == SPG_FP32)
    hipLaunchKernelGGL(k_to_f32, dim3(nblk(n, 256)), dim3(256), 0, s, n, src, (float *)dst);
  else
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n, 256)), dim3(256), 0, s, n, src, (uint16_t *)dst);
  SPG_CHECK_LAUNCH();
}

void lp_set_e0(int n, int chi, float *p, long stride, hipStream_t s) {
  bc_single("lp_set_e0");
  const long tot = (long)n * chi;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_set_e0_f, dim3(nblk(tot, 256)), dim3(256), 0, s, n, chi, p, stride);
  SPG_CHECK_LAUNCH();
}

void lp_right_env_col(const SearchTabs &t, int precision, int r, int c, int n_anc,
                      const uint8_t *cfg, int N, const void *A_rc, const float *Rnext,
                      float *Rout, long rstride, int cl, int cr, hipStream_t s) {
  bc_single("lp_right_env_col");
  if (n_anc <= 0) return;
  KTimer kt_("right_env", s, 2.0 * n_anc * cl * t.d * cr);
  if (cl > 0 && cr > 0 && env_lds_fits(cl, t.d, cr)) {
    if (precision == SPG_FP32)
      hipLaunchKernelGGL(k_right_env_lp_lds<float>, dim3(nblk(n_anc, kW)), dim3(256), 0, s, t, r,
                         c, n_anc, cfg, N, (const float *)A_rc, Rnext, Rout, rstride, 0, cl, cr);
    else
      hipLaunchKernelGGL(k_right_env_lp_lds<uint16_t>, dim3(nblk(n_anc, kW)), dim3(256), 0, s, t,
                         r, c, n_anc, cfg, N, (const uint16_t *)A_rc, Rnext, Rout, rstride, 1, cl,
                         cr);
    SPG_CHECK_LAUNCH();
    return;
  }
  if (precision == SPG_FP32)
    hipLaunchKernelGGL(k_right_env_lp<float>, dim3(nblk(n_anc, kW)), dim3(256), 0, s, t, r, c,
                       n_anc, cfg, N, (const float *)A_rc, Rnext, Rout, rstride, 0);
  else
    hipLaunchKernelGGL(k_right_env_lp<uint16_t>, dim3(nblk(n_anc, kW)), dim3(256), 0, s, t, r, c,
                       n_anc, cfg, N, (const uint16_t *)A_rc, Rnext, Rout, rstride, 1);
  SPG_CHECK_LAUNCH();
}

void lp_marginals(const SearchTabs &t, int precision, int r, int c, int n_beam,
                  const uint8_t *cfg, int N, const void *A_rc, const float *L, const int32_t *anc,
                  const float *Rv, long rstride, const double *score, double *out, int add_score,
                  int cl, int cr, hipStream_t s) {
  bc_single("lp_marginals");
  if (n_beam <= 0) return;
  KTimer kt_("marginals", s, 2.0 * n_beam * t.d * cl * cr);
  if (cl > 0 && cr > 0 && marg_lds_fits(cl, t.d, cr)) {
    if (precision == SPG_FP32)
      hipLaunchKernelGGL(k_marginals_lp_lds<float>, dim3(nblk(n_beam, kW)), dim3(256), 0, s, t, r,
                         c, n_beam, cfg, N, (const float *)A_rc, L, anc, Rv, rstride, score, out,
                         add_score, cl, cr);
    else
      hipLaunchKernelGGL(k_marginals_lp_lds<uint16_t>, dim3(nblk(n_beam, kW)), dim3(256), 0, s, t,
                         r, c, n_beam, cfg, N, (const uint16_t *)A_rc, L, anc, Rv, rstride, score,
                         out, add_score, cl, cr);
    SPG_CHECK_LAUNCH();
    return;
  }
  if (precision == SPG_FP32)
    hipLaunchKernelGGL(k_marginals_lp<float>, dim3(nblk(n_beam, kW)), dim3(256), 0, s, t, r, c,
                       n_beam, cfg, N, (const float *)A_rc, L, anc, Rv, rstride, score, out,
                       add_score);
  else
    hipLaunchKernelGGL(k_marginals_lp<uint16_t>, dim3(nblk(n_beam, kW)), dim3(256), 0, s, t, r,
                       c, n_beam, cfg, N, (const uint16_t *)A_rc, L, anc, Rv, rstride, score, out,
                       add_score);
  SPG_CHECK_LAUNCH();
}

void lp_beam_update(const SearchTabs &t, int precision, int r, int c, int n_new,
                    const int32_t *sel, int N, const uint8_t *cfg, const double *energy,
                    const float *L, const int32_t *anc, const double *cand, const void *A_rc,
                    int update_L, uint8_t *cfg_o, double *energy_o, double *score_o, float *L_o,
                    int32_t *anc_o, int cl, int cr, hipStream_t s) {
  bc_single("lp_beam_update");
  if (n_new <= 0) return;
  KTimer kt_("beam_update", s, 2.0 * n_new * cl * cr);
  if (precision == SPG_FP32)
    hipLaunchKernelGGL(k_beam_update_lp<float>, dim3(nblk(n_new, kW)), dim3(256), 0, s, t, r, c,
                       n_new, sel, N, cfg, energy, L, anc, cand, (const float *)A_rc, update_L,
                       cfg_o, energy_o, score_o, L_o, anc_o, 0);
  else
    hipLaunchKernelGGL(k_beam_update_lp<uint16_t>, dim3(nblk(n_new, kW)), dim3(256), 0, s, t, r,
                       c, n_new, sel, N, cfg, energy, L, anc, cand, (const uint16_t *)A_rc,
                       update_L, cfg_o, energy_o, score_o, L_o, anc_o, 1);
  SPG_CHECK_LAUNCH();
}

void lp_advance_L(const SearchTabs &t, int precision, int r, int c, int n, const uint8_t *cfg,
                  int N, const void *A_rc, float *L, hipStream_t s) {
  bc_single("lp_advance_L");
  if (n <= 0) return;
  if (precision == SPG_FP32)
    hipLaunchKernelGGL(k_advance_L_lp<float>, dim3(nblk(n, kW)), dim3(256), 0, s, t, r, c, n, cfg,
                       N, (const float *)A_rc, L, 0);
  else
    hipLaunchKernelGGL(k_advance_L_lp<uint16_t>, dim3(nblk(n, kW)), dim3(256), 0, s, t, r, c, n,
                       cfg, N, (const uint16_t *)A_rc, L, 1);
  SPG_CHECK_LAUNCH();
}

}  // namespace spg
