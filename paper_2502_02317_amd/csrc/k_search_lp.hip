// Search contractions in reduced precision (the precision form): boundary-MPS
// tensors A in FP32, or in BF16 with FP32 accumulation; environment vectors L
// and R are FP32 (rounded to BF16 on store in the BF16 form).  Couplings to
// the fixed row enter in log domain, relative to their maximum over s, so FP32
// cannot underflow on them; log-probabilities are added to FP64 scores.
#include <cfloat>

#include "lp_dev.h"
#include "mlp_dev.h"
#include "search_dev.h"
#include "spg_internal.h"

namespace spg {

namespace {

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

constexpr int kW = 4;

typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

// U[a][p] = sum_b R^a[b] A[p][b] for every ancestor a and every pair p =
// (al, s) of the site tensor A[al][s][b] (p = al * d + s, row stride chi):
// the product shared by the right environments and the conditionals of a
// column, one GEMM over all ancestors on the matrix cores (M = ancestors,
// N = cl * d, K = cr).  A workgroup computes a 64 x 64 tile of U, wavefront w
// the 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 blocks of 16 x 16, so every
// operand a lane loads feeds two blocks.  Per block: lane l supplies ancestor
// a0 + l % 16 and pair n0 + l % 16, and the four k of its group l / 16 within
// each block of 16 k; FP32 inputs use four v_mfma_f32_16x16x4f32 per k block,
// BF16 inputs one v_mfma_f32_16x16x16bf16 (R is rounded to BF16, as it is
// stored in that form), accumulation in FP32.  Out-of-range rows, pairs and k
// read element 0 and contribute zero.
template <class T>
__global__ __launch_bounds__(256) void k_u_mfma(int n_anc, int npair, int cr, int chi, const T *A,
                                                const float *R, long rstride, float *U,
                                                long ldu) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int a_base = blockIdx.y * 64 + (w >> 1) * 32, n_base = blockIdx.x * 64 + (w & 1) * 32;
  if (a_base >= n_anc || n_base >= npair) return;   // no barrier below
  const int i = lane & 15, g = lane >> 4;
  const float *Rrow[2];
  const T *Arow[2];
  bool oka[2], okp[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    oka[u] = a_base + 16 * u + i < n_anc;
    okp[u] = n_base + 16 * u + i < npair;
    Rrow[u] = R + (oka[u] ? (long)(a_base + 16 * u + i) * rstride : 0L);
    Arow[u] = A + (okp[u] ? (long)(n_base + 16 * u + i) * chi : 0L);
  }
  f4v acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = (f4v){0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < cr; k0 += 16) {
    float rv[2][4];
    T av[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + 4 * g + j;
        const bool ok = k < cr;
        const float x = Rrow[u][(ok && oka[u]) ? k : 0];
        const T y = Arow[u][(ok && okp[u]) ? k : 0];
        rv[u][j] = (ok && oka[u]) ? x : 0.f;
        av[u][j] = (ok && okp[u]) ? y : (T)0;
      }
    if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int v = 0; v < 2; ++v)
            acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(rv[u][j], (float)av[v][j], acc[u][v],
                                                             0, 0, 0);
    } else {
      s4v x[2], y[2];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          x[u][j] = (short)f2bf(rv[u][j]);
          y[u][j] = (short)av[u][j];
        }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
          acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x[u], y[v], acc[u][v], 0, 0, 0);
    }
  }
  // block (u, v): lane l holds U[a0 + 4 (l / 16) + q][n0 + l % 16], q = 0..3,
  // a0 = a_base + 16 u, n0 = n_base + 16 v
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    if (!okp[v]) continue;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = a_base + 16 * u + 4 * g + q;
        if (a < n_anc) U[(long)a * ldu + n_base + 16 * v + i] = acc[u][v][q];
      }
  }
}

// R^a_c[al] = sum_s g^a_c(s) U^a[al][s], normalised by its largest |entry| m,
// which goes to sc[a * sc_stride] when sc is given (one wavefront per
// ancestor; couplings relative to their maximum over s).
__global__ __launch_bounds__(256) void k_env_from_u(SearchTabs t, int r, int c, int n_anc,
                                                    const uint8_t *cfg, int N, const float *U,
                                                    long ldu, float *Rout, long rstride,
                                                    int bf16, int cl, double *sc,
                                                    long sc_stride) {
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
  if (valid)
    for (int h = 0; h < 4; ++h) {
      const int s = lane + 64 * h;
      if (s < d) gs[w][s] = (float)exp(lg[h] - lmax);
    }
  __syncthreads();
  if (!valid) return;
  const float *Ua = U + (long)a * ldu;
  float v[2] = {0.f, 0.f};
  for (int h = 0; h < 2; ++h) {
    const int al = lane + 64 * h;
    if (al >= cl) continue;
    float acc = 0.f;
    for (int s = 0; s < d; ++s) acc = fmaf(gs[w][s], Ua[(long)al * d + s], acc);
    v[h] = acc;
  }
  const float m = wave_max_f(fmaxf(fabsf(v[0]), fabsf(v[1])));
  const float inv = (m > 0.f) ? 1.f / m : 1.f;
  for (int h = 0; h < 2; ++h) {
    const int al = lane + 64 * h;
    if (al < chi) Rout[a * rstride + al] = (al < cl) ? vround(v[h] * inv, bf16) : 0.f;
  }
  if (sc && lane == 0) sc[(long)a * sc_stride] = (double)m;
}

// out[b*d+s] = (add_score ? score[b] : 0) + log p(s | b) (lp_parent_logp, one
// wavefront per beam state).
__global__ __launch_bounds__(256) void k_marg_from_u(SearchTabs t, int r, int c, int n_beam,
                                                     const uint8_t *cfg, int N, const float *U,
                                                     long ldu, const float *L,
                                                     const int32_t *anc, const double *score,
                                                     double *out, int add_score, int cl) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.x * kW + w;
  if (b >= n_beam) return;                    // no barrier below
  double lp[4];
  lp_parent_logp(t, r, c, b, cfg, N, U, ldu, L, anc, cl, lane, lp);
  const double base = add_score ? score[b] : 0.0;
  for (int h = 0; h < 4; ++h) {
    const int s = lane + 64 * h;
    if (s < t.d) out[(long)b * t.d + s] = base + lp[h];
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
                                                        float *L_o, int32_t *anc_o, int bf16,
                                                        const double *sel_score) {
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
    score_o[j] = sel_score ? sel_score[j] : cand[id];
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

void lp_u_col(const SearchTabs &t, int precision, int n_anc, const void *A_rc,
              const float *Rnext, long rstride, float *U, long ldu, int cl, int cr,
              hipStream_t s) {
  bc_single("lp_u_col");
  const int npair = cl * t.d;
  if (n_anc <= 0 || npair <= 0) return;
  if (cr < 1 || cr > t.chi || cl > t.chi || ldu < npair) {
    set_error("lp_u_col: bond dimensions outside the environment's");
    throw Fail{SPG_ERR_INVALID};
  }
  KTimer kt_("u_mfma", s, 2.0 * n_anc * npair * cr);
  dim3 grid(nblk(npair, 64), nblk(n_anc, 64));
  if (precision == SPG_FP32)
    hipLaunchKernelGGL(k_u_mfma<float>, grid, dim3(256), 0, s, n_anc, npair, cr, t.chi,
                       (const float *)A_rc, Rnext, rstride, U, ldu);
  else
    hipLaunchKernelGGL(k_u_mfma<uint16_t>, grid, dim3(256), 0, s, n_anc, npair, cr, t.chi,
                       (const uint16_t *)A_rc, Rnext, rstride, U, ldu);
  SPG_CHECK_LAUNCH();
}

void lp_env_from_u(const SearchTabs &t, int precision, int r, int c, int n_anc,
                   const uint8_t *cfg, int N, const float *U, long ldu, float *Rout, long rstride,
                   int cl, hipStream_t s, double *sc, long sc_stride) {
  bc_single("lp_env_from_u");
  if (n_anc <= 0) return;
  if (t.d > 256 || cl > 128) {
    set_error("lp_env_from_u: d or bond dimension too large");
    throw Fail{SPG_ERR_UNSUPPORTED};
  }
  KTimer kt_("right_env", s, 2.0 * n_anc * cl * t.d);
  hipLaunchKernelGGL(k_env_from_u, dim3(nblk(n_anc, kW)), dim3(256), 0, s, t, r, c, n_anc, cfg,
                     N, U, ldu, Rout, rstride, precision == SPG_BF16 ? 1 : 0, cl, sc, sc_stride);
  SPG_CHECK_LAUNCH();
}

void lp_marginals_u(const SearchTabs &t, int r, int c, int n_beam, const uint8_t *cfg, int N,
                    const float *U, long ldu, const float *L, const int32_t *anc,
                    const double *score, double *out, int add_score, int cl, hipStream_t s) {
  bc_single("lp_marginals_u");
  if (n_beam <= 0) return;
  if (t.d > 256) {
    set_error("lp_marginals_u: d too large");
    throw Fail{SPG_ERR_UNSUPPORTED};
  }
  KTimer kt_("marginals", s, 2.0 * n_beam * t.d * cl);
  hipLaunchKernelGGL(k_marg_from_u, dim3(nblk(n_beam, kW)), dim3(256), 0, s, t, r, c, n_beam, cfg,
                     N, U, ldu, L, anc, score, out, add_score, cl);
  SPG_CHECK_LAUNCH();
}

void lp_beam_update(const SearchTabs &t, int precision, int r, int c, int n_new,
                    const int32_t *sel, int N, const uint8_t *cfg, const double *energy,
                    const float *L, const int32_t *anc, const double *cand, const void *A_rc,
                    int update_L, uint8_t *cfg_o, double *energy_o, double *score_o, float *L_o,
                    int32_t *anc_o, int cl, int cr, hipStream_t s, const double *sel_score) {
  bc_single("lp_beam_update");
  if (n_new <= 0) return;
  KTimer kt_("beam_update", s, 2.0 * n_new * cl * cr);
  if (precision == SPG_FP32)
    hipLaunchKernelGGL(k_beam_update_lp<float>, dim3(nblk(n_new, kW)), dim3(256), 0, s, t, r, c,
                       n_new, sel, N, cfg, energy, L, anc, cand, (const float *)A_rc, update_L,
                       cfg_o, energy_o, score_o, L_o, anc_o, 0, sel_score);
  else
    hipLaunchKernelGGL(k_beam_update_lp<uint16_t>, dim3(nblk(n_new, kW)), dim3(256), 0, s, t, r,
                       c, n_new, sel, N, cfg, energy, L, anc, cand, (const uint16_t *)A_rc,
                       update_L, cfg_o, energy_o, score_o, L_o, anc_o, 1, sel_score);
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
