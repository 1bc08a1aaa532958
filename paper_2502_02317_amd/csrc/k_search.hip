// Branch-and-bound search kernels (FP64 path).
//
// The beam holds, per partial configuration b: its states (uint8 per site),
// accumulated log-probability score, FP64 energy of the fixed variables, the
// left environment vector L^b of its current row (max-normalised) and the
// index of its row-start ancestor, whose right environments R^a_c are shared
// by all its descendants in the row.
//
// Conditional at site (r,c) for parent b and state s:
//   q(b,s) = g^b_c(s) * L^b A_{r,c}[:, s, :] R^{a(b)}_{c+1},
// g^b_c(s) = the Boltzmann weights of the couplings between s and the fixed
// row r-1 (V from (r-1,c), D from (r-1,c-1), A from (r-1,c+1)).
#include <algorithm>
#include <cfloat>
#include <climits>

#include "search_dev.h"
#include "spg_internal.h"
#include "wave.h"

namespace spg {

namespace {

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }


constexpr int kWaves = 4;   // wavefronts (work items) per 256-thread block

// R^a_c[alpha] = sum_s g^a_c(s) sum_alpha' A[alpha][s][alpha'] R^a_{c+1}[alpha'], max-normalised
__global__ __launch_bounds__(256) void k_right_env(SearchTabs t, int r, int c, int n_anc,
                                                   const uint8_t *cfg, int N, const double *A,
                                                   const double *Rnext, double *Rout,
                                                   long rstride, double *scale, int sstride, long ist) {
  SPG_INST(cfg);
  SPG_INST(A);
  SPG_INST(Rnext);
  SPG_INST(Rout);
  SPG_INST(scale);
  shift_tabs(t, ist);
  __shared__ double Rs[kWaves][kMaxChi];
  __shared__ double gs[kWaves][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int a0 = blockIdx.x * kWaves + w;
  const bool valid = a0 < n_anc;
  const int a = valid ? a0 : 0;
  const int chi = t.chi, d = t.d;
  const uint8_t *cb = cfg + (long)a * N;
  if (valid) {
    for (int i = lane; i < chi; i += 64) Rs[w][i] = Rnext[a * rstride + i];
    for (int s = lane; s < d; s += 64) gs[w][s] = field(t, r, c, cb, s);
  }
  __syncthreads();
  if (!valid) return;
  double v[2] = {0.0, 0.0};
  for (int h = 0; h < 2; ++h) {
    const int al = lane + 64 * h;
    if (al >= chi) continue;
    double acc = 0.0;
    for (int s = 0; s < d; ++s) {
      const double *row = A + ((long)al * d + s) * chi;
      double u = 0.0;
      for (int b = 0; b < chi; ++b) u += row[b] * Rs[w][b];
      acc += gs[w][s] * u;
    }
    v[h] = acc;
  }
  const double m = wave_max_nonneg(fmax(fabs(v[0]), fabs(v[1])));
  const double inv = (m > 0.0) ? 1.0 / m : 1.0;
  for (int h = 0; h < 2; ++h) {
    const int al = lane + 64 * h;
    if (al < chi) Rout[a * rstride + al] = v[h] * inv;
  }
  if (scale && lane == 0) scale[(long)a * sstride] = m;
}

// The same right environments with the site tensor staged in LDS once per
// workgroup (when its cl x d x cr block fits, see marg_lds_fits): every lane of
// an ancestor's wavefront takes (al, s) pairs, u[al][s] = sum_b A[al][s][b] R[b]
// in b order, then lane al sums g(s) u[al][s] in s order; rows al >= cl are
// zero as before.  The same order of terms as k_right_env: identical results.
constexpr int kEnvLds = 32 * 16 * 33;      // doubles of the staged block, cl * d * (cr + 1)
constexpr int kEnvU = 32 * 16;             // per-wave u[al][s], cl * d

__host__ __device__ constexpr bool env_lds_fits(int cl, int d, int cr) {
  return d <= 64 && cr <= 64 && cl * d <= kEnvU && cl * d * (cr + 1) <= kEnvLds;
}

__global__ __launch_bounds__(256) void k_right_env_lds(SearchTabs t, int r, int c, int n_anc,
                                                       const uint8_t *cfg, int N, const double *A,
                                                       const double *Rnext, double *Rout,
                                                       long rstride, double *scale, int sstride,
                                                       int cl, int cr, long ist) {
  SPG_INST(cfg);
  SPG_INST(A);
  SPG_INST(Rnext);
  SPG_INST(Rout);
  SPG_INST(scale);
  shift_tabs(t, ist);
  __shared__ double As[kEnvLds];
  __shared__ double us[kWaves][kEnvU];
  __shared__ double Rs[kWaves][kMaxChi];
  __shared__ double gs[kWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int a0 = blockIdx.x * kWaves + w;
  const bool valid = a0 < n_anc;
  const int a = valid ? a0 : 0;
  const int chi = t.chi, d = t.d;
  const int npair = cl * d, ldr = cr + 1;
  {
    const int rpp = 64 / cr, sub = lane / cr, bb = lane - sub * cr;
    if (sub < rpp) {
      const int step = kWaves * rpp;
      int p = w * rpp + sub;
      for (; p + 7 * step < npair; p += 8 * step) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = A[(long)(p + k * step) * chi + bb];
#pragma unroll
        for (int k = 0; k < 8; ++k) As[(p + k * step) * ldr + bb] = v[k];
      }
      for (; p < npair; p += step) As[p * ldr + bb] = A[(long)p * chi + bb];
    }
  }
  const uint8_t *cb = cfg + (long)a * N;
  if (valid) {
    for (int i = lane; i < chi; i += 64) Rs[w][i] = Rnext[a * rstride + i];
    if (lane < d) gs[w][lane] = field(t, r, c, cb, lane);
  }
  __syncthreads();
  if (valid) {
    for (int p0 = 0; p0 < npair; p0 += 64 * 4) {
      double u[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) u[k] = 0.0;
      const int pl = p0 + lane;
      for (int b = 0; b < cr; ++b) {
        const double rb = Rs[w][b];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (pl + 64 * k < npair) u[k] = fma(As[(pl + 64 * k) * ldr + b], rb, u[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (pl + 64 * k < npair) us[w][pl + 64 * k] = u[k];
    }
  }
  __syncthreads();
  if (!valid) return;
  double v[2] = {0.0, 0.0};
  for (int h = 0; h < 2; ++h) {
    const int al = lane + 64 * h;
    if (al >= cl) continue;
    double acc = 0.0;
    for (int s = 0; s < d; ++s) acc = fma(gs[w][s], us[w][al * d + s], acc);
    v[h] = acc;
  }
  const double m = wave_max_nonneg(fmax(fabs(v[0]), fabs(v[1])));
  const double inv = (m > 0.0) ? 1.0 / m : 1.0;
  for (int h = 0; h < 2; ++h) {
    const int al = lane + 64 * h;
    if (al < chi) Rout[a * rstride + al] = v[h] * inv;
  }
  if (scale && lane == 0) scale[(long)a * sstride] = m;
}

// out[b*d + s] = (add_score ? score[b] : 0) + log p(s | b); a parent with no
// positive weight takes softmax_s(-beta dE) (local_softmax_norm)
// ---- the same right environments and conditionals from the column's U
// products: U^a[al*d + s] = sum_b A[al][s][b] R^a_{c+1}[b], one GEMM over all
// row-start ancestors on the FP64 matrix cores (u64_col), so the site tensor
// is read once per output tile instead of once per ancestor or beam state.
// R^a_c[al] = sum_s g^a(s) U^a[al*d + s] (s order), normalised by its largest
// |entry| (to scale[a * sstride] when given); q(b, s) = g^b(s) sum_al L^b[al]
// U^{anc(b)}[al*d + s] (al order); the epilogue is k_marginals'.
__global__ __launch_bounds__(256) void k_env_from_u64(SearchTabs t, int r, int c, int n_anc,
                                                      const uint8_t *cfg, int N, const double *U,
                                                      long ldu, double *Rout, long rstride,
                                                      int cl, double *scale, int sstride,
                                                      long ist) {
  SPG_INST(cfg);
  SPG_INST(U);
  SPG_INST(Rout);
  SPG_INST(scale);
  shift_tabs(t, ist);
  __shared__ double gs[kWaves][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int a0 = blockIdx.x * kWaves + w;
  const bool valid = a0 < n_anc;
  const int a = valid ? a0 : 0;
  const int chi = t.chi, d = t.d;
  const uint8_t *cb = cfg + (long)a * N;
  if (valid)
    for (int s = lane; s < d; s += 64) gs[w][s] = field(t, r, c, cb, s);
  __syncthreads();
  if (!valid) return;
  const double *Ua = U + (long)a * ldu;
  double v[2] = {0.0, 0.0};
  for (int h = 0; h < 2; ++h) {
    const int al = lane + 64 * h;
    if (al >= cl) continue;
    double acc = 0.0;
    for (int s = 0; s < d; ++s) acc += gs[w][s] * Ua[(long)al * d + s];
    v[h] = acc;
  }
  const double m = wave_max_nonneg(fmax(fabs(v[0]), fabs(v[1])));
  const double inv = (m > 0.0) ? 1.0 / m : 1.0;
  for (int h = 0; h < 2; ++h) {
    const int al = lane + 64 * h;
    if (al < chi) Rout[a * rstride + al] = (al < cl) ? v[h] * inv : 0.0;
  }
  if (scale && lane == 0) scale[(long)a * sstride] = m;
}

__global__ __launch_bounds__(256) void k_marg_from_u64(SearchTabs t, int r, int c, int n_beam,
                                                       const uint8_t *cfg, int N, const double *U,
                                                       long ldu, const double *L,
                                                       const int32_t *anc, const double *score,
                                                       double *out, int add_score, int cl,
                                                       long ist) {
  SPG_INST(cfg);
  SPG_INST(U);
  SPG_INST(L);
  SPG_INST(anc);
  SPG_INST(score);
  SPG_INST(out);
  shift_tabs(t, ist);
  __shared__ double Ls[kWaves][kMaxChi];
  __shared__ double qs[kWaves][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b0 = blockIdx.x * kWaves + w;
  const bool valid = b0 < n_beam;
  const int b = valid ? b0 : 0;
  const int chi = t.chi, d = t.d;
  if (valid)
    for (int i = lane; i < chi; i += 64) Ls[w][i] = L[(long)b * chi + i];
  __syncthreads();
  if (!valid) return;
  const double *Ua = U + (long)anc[b] * ldu;
  const uint8_t *cb = cfg + (long)b * N;
  double part = 0.0;
  for (int s = lane; s < d; s += 64) {
    double acc = 0.0;
    for (int al = 0; al < cl; ++al) {
      const double la = Ls[w][al];
      if (la == 0.0) continue;
      acc = fma(la, Ua[(long)al * d + s], acc);
    }
    double q = field(t, r, c, cb, s) * acc;
    q = (q > 0.0) ? q : 0.0;               // negative q (truncation error) = probability 0
    qs[w][s] = q;
    part += q;
  }
  const double tot = wave_sum(part);
  const double base = add_score ? score[b] : 0.0;
  if (!(tot > 0.0)) {                      // no child with positive weight
    double emin, lse;
    local_softmax_norm(t, r, c, cb, lane, emin, lse);
    for (int s = lane; s < d; s += 64)
      out[(long)b * d + s] = base + (-t.beta * (delta_energy(t, r, c, cb, s) - emin) - lse);
    return;
  }
  const double ltot = log(tot);
  for (int s = lane; s < d; s += 64) {
    const double q = qs[w][s];
    double lp = (q > 0.0 && tot > 0.0) ? log(q) - ltot : -INFINITY;
    if (!(lp == lp)) lp = -INFINITY;
    out[(long)b * d + s] = base + lp;
  }
}

__global__ __launch_bounds__(256) void k_marginals(SearchTabs t, int r, int c, int n_beam,
                                                   const uint8_t *cfg, int N, const double *A,
                                                   const double *L, const int32_t *anc,
                                                   const double *Rv, long rstride,
                                                   const double *score, double *out,
                                                   int add_score, long ist) {
  SPG_INST(cfg);
  SPG_INST(A);
  SPG_INST(L);
  SPG_INST(anc);
  SPG_INST(Rv);
  SPG_INST(score);
  SPG_INST(out);
  shift_tabs(t, ist);
  __shared__ double Ls[kWaves][kMaxChi];
  __shared__ double Rs[kWaves][kMaxChi];
  __shared__ double qs[kWaves][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b0 = blockIdx.x * kWaves + w;
  const bool valid = b0 < n_beam;
  const int b = valid ? b0 : 0;
  const int chi = t.chi, d = t.d;
  const double *Rn = Rv + (long)anc[b] * rstride + (long)(c + 1) * chi;
  if (valid)
    for (int i = lane; i < chi; i += 64) {
      Ls[w][i] = L[(long)b * chi + i];
      Rs[w][i] = Rn[i];
    }
  __syncthreads();
  if (!valid) return;
  const uint8_t *cb = cfg + (long)b * N;
  double part = 0.0;
  for (int s = lane; s < d; s += 64) {
    double acc = 0.0;
    for (int al = 0; al < chi; ++al) {
      const double la = Ls[w][al];
      if (la == 0.0) continue;
      const double *row = A + ((long)al * d + s) * chi;
      double u = 0.0;
      for (int bb = 0; bb < chi; ++bb) u += row[bb] * Rs[w][bb];
      acc += la * u;
    }
    double q = field(t, r, c, cb, s) * acc;
    q = (q > 0.0) ? q : 0.0;               // negative q (truncation error) = probability 0
    qs[w][s] = q;
    part += q;
  }
  const double tot = wave_sum(part);
  const double base = add_score ? score[b] : 0.0;
  if (!(tot > 0.0)) {                      // no child with positive weight
    double emin, lse;
    local_softmax_norm(t, r, c, cb, lane, emin, lse);
    for (int s = lane; s < d; s += 64)
      out[(long)b * d + s] = base + (-t.beta * (delta_energy(t, r, c, cb, s) - emin) - lse);
    return;
  }
  const double ltot = log(tot);
  for (int s = lane; s < d; s += 64) {
    const double q = qs[w][s];
    double lp = (q > 0.0 && tot > 0.0) ? log(q) - ltot : -INFINITY;
    if (!(lp == lp)) lp = -INFINITY;
    out[(long)b * d + s] = base + lp;
  }
}

// The same conditionals with the site tensor staged in LDS once per
// workgroup (when its cl x d x cr block fits): every lane of a beam's
// wavefront takes (al, s) pairs, u[al][s] = sum_b A[al][s][b] R[b] in b order,
// four pairs in flight per lane, then lane s sums L[al] u[al][s] in al order.
// Every sum runs in the same order as above, so the results are identical.
constexpr int kMargLds = 32 * 16 * 33;     // doubles of the staged block, cl * d * (cr + 1)
constexpr int kMargU = 32 * 16;            // per-wave u[al][s], cl * d

__host__ __device__ constexpr bool marg_lds_fits(int cl, int d, int cr) {
  return d <= 64 && cr <= 64 && cl * d <= kMargU && cl * d * (cr + 1) <= kMargLds;
}

__global__ __launch_bounds__(256) void k_marginals_lds(SearchTabs t, int r, int c, int n_beam,
                                                       const uint8_t *cfg, int N, const double *A,
                                                       const double *L, const int32_t *anc,
                                                       const double *Rv, long rstride,
                                                       const double *score, double *out,
                                                       int add_score, int cl, int cr, long ist) {
  SPG_INST(cfg);
  SPG_INST(A);
  SPG_INST(L);
  SPG_INST(anc);
  SPG_INST(Rv);
  SPG_INST(score);
  SPG_INST(out);
  shift_tabs(t, ist);
  __shared__ double As[kMargLds];
  __shared__ double us[kWaves][kMargU];
  __shared__ double Ls[kWaves][kMaxChi];
  __shared__ double Rs[kWaves][kMaxChi];
  __shared__ double qs[kWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b0 = blockIdx.x * kWaves + w;
  const bool valid = b0 < n_beam;
  const int b = valid ? b0 : 0;
  const int chi = t.chi, d = t.d;
  const int npair = cl * d, ldr = cr + 1;
  // A[al][s][0..cr) -> As[(al*d + s)*ldr + .]: each wavefront copies whole
  // rows, 64 / cr rows per pass, eight rows' loads in flight
  {
    const int rpp = 64 / cr, sub = lane / cr, bb = lane - sub * cr;
    if (sub < rpp) {
      const int step = kWaves * rpp;
      int p = w * rpp + sub;
      for (; p + 7 * step < npair; p += 8 * step) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = A[(long)(p + k * step) * chi + bb];
#pragma unroll
        for (int k = 0; k < 8; ++k) As[(p + k * step) * ldr + bb] = v[k];
      }
      for (; p < npair; p += step) As[p * ldr + bb] = A[(long)p * chi + bb];
    }
  }
  if (valid) {
    const double *Rn = Rv + (long)anc[b] * rstride + (long)(c + 1) * chi;
    for (int i = lane; i < chi; i += 64) {
      Ls[w][i] = L[(long)b * chi + i];
      Rs[w][i] = Rn[i];
    }
  }
  __syncthreads();
  if (valid) {
    for (int p0 = 0; p0 < npair; p0 += 64 * 4) {
      double u[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) u[k] = 0.0;
      const int pl = p0 + lane;
      for (int bb = 0; bb < cr; ++bb) {
        const double rb = Rs[w][bb];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (pl + 64 * k < npair) u[k] = fma(As[(pl + 64 * k) * ldr + bb], rb, u[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (pl + 64 * k < npair) us[w][pl + 64 * k] = u[k];
    }
  }
  __syncthreads();
  if (!valid) return;
  const uint8_t *cb = cfg + (long)b * N;
  double part = 0.0;
  const int s = lane;
  if (s < d) {
    double acc = 0.0;
    for (int al = 0; al < cl; ++al) {
      const double la = Ls[w][al];
      if (la == 0.0) continue;
      acc = fma(la, us[w][al * d + s], acc);
    }
    double q = field(t, r, c, cb, s) * acc;
    q = (q > 0.0) ? q : 0.0;               // negative q (truncation error) = probability 0
    qs[w][s] = q;
    part = q;
  }
  const double tot = wave_sum(part);
  const double base = add_score ? score[b] : 0.0;
  if (!(tot > 0.0)) {                      // no child with positive weight
    double emin, lse;
    local_softmax_norm(t, r, c, cb, lane, emin, lse);
    if (s < d) out[(long)b * d + s] = base + (-t.beta * (delta_energy(t, r, c, cb, s) - emin) - lse);
    return;
  }
  const double ltot = log(tot);
  if (s < d) {
    const double q = qs[w][s];
    double lp = (q > 0.0 && tot > 0.0) ? log(q) - ltot : -INFINITY;
    if (!(lp == lp)) lp = -INFINITY;
    out[(long)b * d + s] = base + lp;
  }
}

// Top-M of n scores by (score desc, id asc), written to sel[0..min(M,n)-1] in
// that order, with the selected scores in sel_score (may be null).  Candidate
// i has score cand[i] and id cid[i] (cid null: id = i; ids must be unique and
// non-negative); n is *n_dev when n_dev is given.
//
// First a histogram of gap_bin(best score, score) over 4096 bins: the bin b*
// where the running count reaches M bounds the selection, and the m keys in
// bins <= b* are the first M of the (key, id) order and the rest of bin b*.
// When m <= kSelLdsSort they are compacted to LDS and ordered without a sort:
// a second histogram, uniform in the score gap to the best score over the
// survivors' range, places each in its bin's segment (prefix sums), and its
// final position is the segment's start plus its rank among the few keys of
// the same bin.  When a bin still holds more than kSelBucket keys (ties), the
// survivors are sorted instead (bitonic, in LDS).  When m > kSelLdsSort:
// radix select of the M-th key (8-bit digits), then of the id among keys equal
// to it, compaction, then a bitonic sort of the survivors.
// Up to kSelRegKeys * 1024 candidates are held in registers for all passes,
// which then start at the highest digit where the keys differ.
constexpr int kSelRegKeys = 16;
constexpr int kSelLdsSort = 1024 * kSortLdsRegs;     // 8192
constexpr int kSelBucket = 64;

__global__ __launch_bounds__(1024) void k_select(int n_host, const int *n_dev, int M,
                                                const double *cand, const int32_t *cid,
                                                int32_t *sel, double *sel_score, uint64_t *kw,
                                                int32_t *iw, long ist, unsigned *gclear,
                                                int *cclear) {
  SPG_INST(n_dev);
  SPG_INST(cand);
  SPG_INST(cid);
  SPG_INST(sel);
  SPG_INST(sel_score);
  SPG_INST(kw);
  SPG_INST(iw);
  __shared__ unsigned hist[256];
  __shared__ unsigned gh[kGapBins], gs[kGapBins];
  __shared__ uint64_t sh_prefix;
  __shared__ int sh_need, sh_bstar, sh_m;
  __shared__ unsigned sh_maxc;
  __shared__ double sh_gap[16];
  __shared__ int wsum[16];
  __shared__ uint64_t wmin[16], wmax[16];
  __shared__ uint64_t skey[kSelLdsSort];
  __shared__ int32_t sid[kSelLdsSort];
  const int tid = threadIdx.x;
  const int n = n_dev ? *n_dev : n_host;
  if (gclear) {
    // after the multi-workgroup front end: its histogram and survivor count
    // (n_dev) start from zero at its next call
    __syncthreads();                     // every thread has read n
    for (int b = tid; b < kGapBins; b += 1024) gclear[b] = 0u;
    if (tid == 0) *cclear = 0;
  }
  if (n <= 0) return;
  const int Me = (M < n) ? M : n;
  int p2 = 1;
  while (p2 < Me) p2 <<= 1;
  const bool lds_sort = p2 <= kSelLdsSort;
  auto key_at = [&](int i) { return desc_key(cand[i]); };
  auto id_at = [&](int i) { return cid ? cid[i] : i; };
  // from the gap histogram gh: the boundary bin b* and the count m of keys in
  // bins <= b* (uniform on return)
  auto gap_bound = [&](int &bstar, int &m) {
    unsigned hb[4];
    int own = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      hb[j] = gh[4 * tid + j];
      own += (int)hb[j];
    }
    int tot;
    const int ex = block_excl_scan_count(own, wsum, &tot);
    if (ex < Me && ex + own >= Me) {                 // exactly one thread
      int cum = ex, b = 4 * tid;
      for (int j = 0; j < 4; ++j) {
        cum += (int)hb[j];
        b = 4 * tid + j;
        if (cum >= Me) break;
      }
      sh_bstar = b;
      sh_m = cum;
    }
    __syncthreads();
    bstar = sh_bstar;
    m = sh_m;
  };
  // sorts the m survivors in skey/sid and writes the first Me
  auto sort_out = [&](int m) {
    int p2m = 1;
    while (p2m < m) p2m <<= 1;
    for (int i = m + tid; i < p2m; i += 1024) { skey[i] = ~0ull; sid[i] = INT_MAX; }
    __syncthreads();
    bitonic_sort_lds(skey, sid, p2m);
    for (int i = tid; i < Me; i += 1024) {
      sel[i] = sid[i];
      if (sel_score) sel_score[i] = key_value(skey[i]);
    }
  };
  // the m survivors (a prefix of the order, m >= Me) sit unordered in
  // skey/sid (written before a barrier): writes the first Me in order.  Bins uniform in the gap
  // vmax - v over [0, largest gap] (monotone in the score), prefix sums for
  // the segments, then each survivor's rank within its bin.
  auto order_out = [&](int m, uint64_t kbest) {
    const double vmax = key_value(kbest);
    double gm = 0.0;
    for (int p = tid; p < m; p += 1024) gm = fmax(gm, vmax - key_value(skey[p]));
    gm = wave_max_nonneg(gm);
    if ((tid & 63) == 0) sh_gap[tid >> 6] = gm;
    for (int b = tid; b < kGapBins; b += 1024) gh[b] = 0u;
    if (tid == 0) sh_maxc = 0u;
    __syncthreads();
    gm = 0.0;
    for (int w = 0; w < 16; ++w) gm = fmax(gm, sh_gap[w]);
    if (!(gm > 0.0 && gm <= 1.7e308)) {              // a single score, or -inf among them
      sort_out(m);
      return;
    }
    const double scale = (double)kGapBins / gm;
    auto vbin = [&](uint64_t k) {
      return (int)fmin((vmax - key_value(k)) * scale, (double)(kGapBins - 1));
    };
    for (int p = tid; p < m; p += 1024) atomicAdd(&gh[vbin(skey[p])], 1u);
    __syncthreads();
    unsigned hb[4];
    int own = 0;
    unsigned mc = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      hb[j] = gh[4 * tid + j];
      own += (int)hb[j];
      mc = (hb[j] > mc) ? hb[j] : mc;
    }
    mc = (unsigned)wave_max_u64(mc);
    if ((tid & 63) == 0 && mc > 0u) atomicMax(&sh_maxc, mc);
    int tot;
    unsigned run = (unsigned)block_excl_scan_count(own, wsum, &tot);
    if (sh_maxc > (unsigned)kSelBucket) {            // ties: sort instead
      sort_out(m);
      return;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      gs[4 * tid + j] = run;
      gh[4 * tid + j] = run;
      run += hb[j];
    }
    uint64_t kv[kSortLdsRegs];
    int32_t iv[kSortLdsRegs];
#pragma unroll
    for (int r = 0; r < kSortLdsRegs; ++r) {
      const int p = tid + 1024 * r;
      kv[r] = (p < m) ? skey[p] : 0ull;
      iv[r] = (p < m) ? sid[p] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortLdsRegs; ++r) {
      if (tid + 1024 * r < m) {
        const unsigned pos = atomicAdd(&gh[vbin(kv[r])], 1u);
        skey[pos] = kv[r];
        sid[pos] = iv[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortLdsRegs; ++r) {
      if (tid + 1024 * r < m) {
        const uint64_t k = kv[r];
        const int32_t id = iv[r];
        const int b = vbin(k);
        const int s0 = (int)gs[b], e0 = (int)gh[b];
        int rk = s0;
        int f = s0;
        for (; f + 3 < e0; f += 4) {
          const uint64_t k0 = skey[f], k1 = skey[f + 1], k2 = skey[f + 2], k3 = skey[f + 3];
          const int32_t i0 = sid[f], i1 = sid[f + 1], i2 = sid[f + 2], i3 = sid[f + 3];
          rk += (k0 < k || (k0 == k && i0 < id)) + (k1 < k || (k1 == k && i1 < id)) +
                (k2 < k || (k2 == k && i2 < id)) + (k3 < k || (k3 == k && i3 < id));
        }
        for (; f < e0; ++f) {
          const uint64_t kf = skey[f];
          rk += (kf < k || (kf == k && sid[f] < id)) ? 1 : 0;
        }
        if (rk < Me) {
          sel[rk] = id;
          if (sel_score) sel_score[rk] = key_value(k);
        }
      }
    }
  };
  // the m survivors of a selection of more than kSelLdsSort (every one of
  // them selected, m <= kSelRegKeys * 1024) sit unordered in kw/iw (written
  // before a barrier): placed in order in kw/iw by the gap bins of order_out,
  // each one's position its bin's start plus its rank among the bin's keys,
  // and written to sel.  Returns false, having written nothing, when the gaps
  // are not finite or a bin holds more than kSelBucket keys (the caller then
  // sorts).
  auto order_global = [&](int m) -> bool {
    uint64_t kv[kSelRegKeys];
    int32_t iv[kSelRegKeys];
    uint64_t klo = ~0ull, khi = 0;
#pragma unroll
    for (int r = 0; r < kSelRegKeys; ++r) {
      const int p = tid + 1024 * r;
      kv[r] = (p < m) ? kw[p] : 0ull;
      iv[r] = (p < m) ? iw[p] : 0;
      if (p < m) {
        klo = (kv[r] < klo) ? kv[r] : klo;
        khi = (kv[r] > khi) ? kv[r] : khi;
      }
    }
    klo = wave_min_u64(klo);
    khi = wave_max_u64(khi);
    if ((tid & 63) == 0) {
      wmin[tid >> 6] = klo;
      wmax[tid >> 6] = khi;
    }
    for (int b = tid; b < kGapBins; b += 1024) gh[b] = 0u;
    if (tid == 0) sh_maxc = 0u;
    __syncthreads();
    klo = ~0ull;
    khi = 0;
    for (int w = 0; w < 16; ++w) {
      klo = (wmin[w] < klo) ? wmin[w] : klo;
      khi = (wmax[w] > khi) ? wmax[w] : khi;
    }
    const double vmax = key_value(klo);
    const double gm = vmax - key_value(khi);
    if (!(gm > 0.0 && gm <= 1.7e308)) return false;  // one score, or -inf among them
    const double scale = (double)kGapBins / gm;
    auto vbin = [&](uint64_t k) {
      return (int)fmax(0.0, fmin((vmax - key_value(k)) * scale, (double)(kGapBins - 1)));
    };
#pragma unroll
    for (int r = 0; r < kSelRegKeys; ++r)
      if (tid + 1024 * r < m) atomicAdd(&gh[vbin(kv[r])], 1u);
    __syncthreads();
    unsigned hb[4];
    int own = 0;
    unsigned mc = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      hb[j] = gh[4 * tid + j];
      own += (int)hb[j];
      mc = (hb[j] > mc) ? hb[j] : mc;
    }
    mc = (unsigned)wave_max_u64(mc);
    if ((tid & 63) == 0 && mc > 0u) atomicMax(&sh_maxc, mc);
    int tot;
    unsigned run = (unsigned)block_excl_scan_count(own, wsum, &tot);
    if (sh_maxc > (unsigned)kSelBucket) return false;   // ties: sort instead
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      gs[4 * tid + j] = run;
      gh[4 * tid + j] = run;
      run += hb[j];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSelRegKeys; ++r) {
      if (tid + 1024 * r < m) {
        const unsigned pos = atomicAdd(&gh[vbin(kv[r])], 1u);
        kw[pos] = kv[r];
        iw[pos] = iv[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSelRegKeys; ++r) {
      if (tid + 1024 * r < m) {
        const uint64_t k = kv[r];
        const int32_t id = iv[r];
        const int b = vbin(k);
        const int s0 = (int)gs[b], e0 = (int)gh[b];
        int rk = s0;
        for (int f = s0; f < e0; ++f) {
          const uint64_t kf = kw[f];
          rk += (kf < k || (kf == k && iw[f] < id)) ? 1 : 0;
        }
        sel[rk] = id;
        if (sel_score) sel_score[rk] = key_value(k);
      }
    }
    return true;
  };
  uint64_t kthr = ~0ull;         // take keys < kthr, and keys == kthr with id <= ithr
  uint64_t ithr = 0;
  bool all_eq = true;
  if (n <= kSelRegKeys * 1024) {
    // ---- keys held in registers, kSelRegKeys per thread (ids are the index
    // or read back for ties and survivors only)
    uint64_t kr[kSelRegKeys];
    uint64_t lo = ~0ull, hi = 0;
    {
      // all loads issued before the first use (indices clamped into range);
      // the gap histogram is cleared while they are in flight (the barrier
      // after the min/max orders the clearing before its counts)
      double raw[kSelRegKeys];
#pragma unroll
      for (int q = 0; q < kSelRegKeys; ++q) {
        const int i = tid + 1024 * q;
        raw[q] = cand[(i < n) ? i : n - 1];
      }
      if (Me < n)
        for (int b = tid; b < kGapBins; b += 1024) gh[b] = 0u;
#pragma unroll
      for (int q = 0; q < kSelRegKeys; ++q) kr[q] = (tid + 1024 * q < n) ? desc_key(raw[q]) : 0ull;
    }
#pragma unroll
    for (int q = 0; q < kSelRegKeys; ++q) {
      const int i = tid + 1024 * q;
      if (i < n) {
        lo = (kr[q] < lo) ? kr[q] : lo;
        hi = (kr[q] > hi) ? kr[q] : hi;
      }
    }
    if (Me < n) {
      // digits above the highest bit where the keys differ are shared by all
      // of them: the radix passes start below it
      lo = wave_min_u64(lo);
      hi = wave_max_u64(hi);
      if ((tid & 63) == 0) {
        wmin[tid >> 6] = lo;
        wmax[tid >> 6] = hi;
      }
      __syncthreads();
      lo = ~0ull;
      hi = 0;
      for (int w = 0; w < 16; ++w) {
        lo = (wmin[w] < lo) ? wmin[w] : lo;
        hi = (wmax[w] > hi) ? wmax[w] : hi;
      }
      if (lo != hi) {
        // ---- gap histogram: usually settles the selection in one pass (the
        // bins stay in registers; -inf, often the most crowded bin, is
        // counted once per wavefront)
        const double vmax = key_value(lo);
        const int binf = gap_bin(vmax, -INFINITY);
        int kb[kSelRegKeys];
#pragma unroll
        for (int q = 0; q < kSelRegKeys; ++q) {
          const int i = tid + 1024 * q;
          kb[q] = (i < n) ? gap_bin(vmax, key_value(kr[q])) : kGapBins;
          const unsigned long long inf_lanes = __ballot(kb[q] == binf);
          if (kb[q] < kGapBins && kb[q] != binf) atomicAdd(&gh[kb[q]], 1u);
          if ((tid & 63) == 0 && inf_lanes) atomicAdd(&gh[binf], (unsigned)__popcll(inf_lanes));
        }
        __syncthreads();
        int bstar, m;
        gap_bound(bstar, m);
        if (m <= kSelLdsSort) {
          int cnt = 0;
          unsigned fl = 0u;
#pragma unroll
          for (int q = 0; q < kSelRegKeys; ++q) {
            const bool f = kb[q] <= bstar;             // kGapBins beyond n
            fl |= (f ? 1u : 0u) << q;
            cnt += f;
          }
          int tot;
          int pos = block_excl_scan_count(cnt, wsum, &tot);
#pragma unroll
          for (int q = 0; q < kSelRegKeys; ++q) {
            if ((fl >> q) & 1u) {
              skey[pos] = kr[q];
              sid[pos] = id_at(tid + 1024 * q);
              ++pos;
            }
          }
          __syncthreads();                     // every survivor in skey/sid
          order_out(m, lo);
          return;
        }
      }
      int need = Me, n_eq = n;
      uint64_t prefix = lo;
      if (lo != hi) {
        const int top = (63 - __clzll((long long)(lo ^ hi))) & ~7;   // shift of the first digit that differs
        uint64_t pmask = (top == 56) ? 0ull : ~((1ull << (top + 8)) - 1ull);
        prefix = lo & pmask;
        for (int shift = top; shift >= 0; shift -= 8) {
          for (int i = tid; i < 256; i += 1024) hist[i] = 0u;
          __syncthreads();
#pragma unroll
          for (int q = 0; q < kSelRegKeys; ++q) {
            const int i = tid + 1024 * q;
            if (i < n && (kr[q] & pmask) == prefix) atomicAdd(&hist[(kr[q] >> shift) & 255u], 1u);
          }
          __syncthreads();
          radix_find(shift, prefix, need, hist, &sh_prefix, &sh_need);
          pmask |= (255ull << shift);
        }
        n_eq = (int)hist[prefix & 255u];
      }
      kthr = prefix;
      if (need < n_eq) {
        all_eq = false;
        uint64_t ip = 0, im = 0xFFFFFFFF00000000ull;   // ids fit in 32 bits
        int need_id = need;
        for (int shift = 24; shift >= 0; shift -= 8) {
          for (int i = tid; i < 256; i += 1024) hist[i] = 0u;
          __syncthreads();
#pragma unroll
          for (int q = 0; q < kSelRegKeys; ++q) {
            const int i = tid + 1024 * q;
            const uint64_t ik = (i < n && kr[q] == kthr) ? (uint64_t)(uint32_t)id_at(i) : ~0ull;
            if ((ik & im) == ip) atomicAdd(&hist[(ik >> shift) & 255u], 1u);
          }
          __syncthreads();
          radix_find(shift, ip, need_id, hist, &sh_prefix, &sh_need);
          im |= (255ull << shift);
        }
        ithr = ip;
      }
    }
    // ---- compaction: per-thread counts, one block scan
    int cnt = 0;
    unsigned fl = 0u;
#pragma unroll
    for (int q = 0; q < kSelRegKeys; ++q) {
      const int i = tid + 1024 * q;
      bool f = false;
      if (i < n) {
        f = (Me == n) || (kr[q] < kthr) ||
            (kr[q] == kthr && (all_eq || (uint64_t)(uint32_t)id_at(i) <= ithr));
      }
      fl |= (f ? 1u : 0u) << q;
      cnt += f;
    }
    int tot;
    int pos = block_excl_scan_count(cnt, wsum, &tot);
#pragma unroll
    for (int q = 0; q < kSelRegKeys; ++q) {
      if (((fl >> q) & 1u) && pos < Me) {      // exactly Me flags by construction
        const int i = tid + 1024 * q;
        if (lds_sort) { skey[pos] = kr[q]; sid[pos] = id_at(i); }
        else { kw[pos] = kr[q]; iw[pos] = id_at(i); }
        ++pos;
      }
    }
  } else {
    // ---- keys read from memory on every pass
    if (Me < n) {
      // gap histogram first, as above
      uint64_t lo = ~0ull;
      for (int i = tid; i < n; i += 1024) {
        const uint64_t k = key_at(i);
        lo = (k < lo) ? k : lo;
      }
      lo = wave_min_u64(lo);
      if ((tid & 63) == 0) wmin[tid >> 6] = lo;
      for (int b = tid; b < kGapBins; b += 1024) gh[b] = 0u;
      __syncthreads();
      lo = ~0ull;
      for (int w = 0; w < 16; ++w) lo = (wmin[w] < lo) ? wmin[w] : lo;
      const double vmax = key_value(lo);
      for (int i = tid; i < n; i += 1024) atomicAdd(&gh[gap_bin(vmax, key_value(key_at(i)))], 1u);
      __syncthreads();
      int bstar, m;
      gap_bound(bstar, m);
      if (m <= kSelLdsSort) {
        int base = 0;
        for (int c0 = 0; c0 < n; c0 += 1024) {
          const int i = c0 + tid;
          uint64_t k = 0;
          int f = 0;
          if (i < n) {
            k = key_at(i);
            f = gap_bin(vmax, key_value(k)) <= bstar;
          }
          int tot_f;
          const int pos = block_excl_scan(f, wsum, &tot_f);
          if (f) { skey[base + pos] = k; sid[base + pos] = id_at(i); }
          base += tot_f;
          __syncthreads();
        }
        order_out(m, lo);
        return;
      }
      uint64_t prefix = 0, pmask = 0;
      int need = Me;
      for (int shift = 56; shift >= 0; shift -= 8) {
        radix_digit(n, shift, key_at, pmask, prefix, need, hist, &sh_prefix, &sh_need);
        pmask |= (255ull << shift);
      }
      kthr = prefix;
      // need = how many keys equal to kthr are taken; hist still counts them
      const int n_eq = (int)hist[kthr & 255u];
      if (need < n_eq) {
        all_eq = false;
        const uint64_t kk = kthr;
        auto idkey_at = [&](int i) -> uint64_t {
          return (key_at(i) == kk) ? (uint64_t)(uint32_t)id_at(i) : ~0ull;
        };
        uint64_t ip = 0, im = 0xFFFFFFFF00000000ull;   // ids fit in 32 bits
        int need_id = need;
        for (int shift = 24; shift >= 0; shift -= 8) {
          radix_digit(n, shift, idkey_at, im, ip, need_id, hist, &sh_prefix, &sh_need);
          im |= (255ull << shift);
        }
        ithr = ip;
      }
    }
    // compaction of the survivors (any order: they are sorted next)
    int base = 0;
    for (int c0 = 0; c0 < n; c0 += blockDim.x) {
      const int i = c0 + tid;
      uint64_t k = 0;
      int f = 0;
      if (i < n) {
        k = key_at(i);
        f = (k < kthr) || (k == kthr && (all_eq || (uint64_t)(uint32_t)id_at(i) <= ithr));
        if (Me == n) f = 1;
      }
      int tot_f;
      const int pos = block_excl_scan(f, wsum, &tot_f);
      if (f) {
        if (lds_sort) { skey[base + pos] = k; sid[base + pos] = id_at(i); }
        else { kw[base + pos] = k; iw[base + pos] = id_at(i); }
      }
      base += tot_f;
      __syncthreads();
    }
  }
  // ---- sort the Me survivors (padded to a power of two) by (key, id)
  if (lds_sort) {
    for (int i = Me + tid; i < p2; i += blockDim.x) { skey[i] = ~0ull; sid[i] = INT_MAX; }
    __syncthreads();
    bitonic_sort_lds(skey, sid, p2);
    for (int i = tid; i < Me; i += blockDim.x) {
      sel[i] = sid[i];
      if (sel_score) sel_score[i] = key_value(skey[i]);
    }
  } else {
    __syncthreads();                             // every survivor in kw/iw
    if (Me <= kSelRegKeys * 1024 && order_global(Me)) return;
    for (int i = Me + tid; i < p2; i += blockDim.x) { kw[i] = ~0ull; iw[i] = INT_MAX; }
    __syncthreads();
    bitonic_sort(kw, iw, p2);
    for (int i = tid; i < Me; i += blockDim.x) {
      sel[i] = iw[i];
      if (sel_score) sel_score[i] = key_value(kw[i]);
    }
  }
}

// ---- top-M for more candidates than the one-workgroup select holds in
// registers: the gap histogram over many workgroups (integer atomics, whose
// totals do not depend on their order), relative to the best score or to a
// bound above it that the caller knows (the best parent's score: no child
// scores above it), and the last workgroup to finish finds the boundary bin
// b*; then every workgroup appends its scores in bins <= b* to a survivor list
// (in any order, one atomic per workgroup); k_select on the survivors (their
// scores and original indices) orders them and writes sel and sel_score, and
// clears the histogram and the count for the next call.
struct GselState {
  unsigned long long kmin;
  int count, bstar;
  unsigned done;
  int pad;
};

__device__ __forceinline__ double nan_to_ninf(double v) { return (v == v) ? v : -INFINITY; }

__global__ __launch_bounds__(1024) void k_gsel_init(GselState *st, unsigned *gh) {
  for (int b = threadIdx.x; b < kGapBins; b += 1024) gh[b] = 0u;
  if (threadIdx.x == 0) {
    st->kmin = ~0ull;
    st->count = 0;
    st->done = 0u;
  }
}

__global__ __launch_bounds__(256) void k_gsel_min(int n, const double *cand, GselState *st) {
  uint64_t lo = ~0ull;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const uint64_t k = desc_key(cand[i]);
    lo = (k < lo) ? k : lo;
  }
  lo = wave_min_u64(lo);
  if ((threadIdx.x & 63) == 0) atomicMin(&st->kmin, (unsigned long long)lo);
}

__global__ __launch_bounds__(256) void k_gsel_hist(int n, int Me, const double *cand,
                                                   const double *vref, GselState *st,
                                                   unsigned *gh) {
  __shared__ unsigned h[kGapBins];
  __shared__ int wsum[4];
  __shared__ int last;
  const int tid = threadIdx.x;
  for (int b = tid; b < kGapBins; b += 256) h[b] = 0u;
  __syncthreads();
  const double vmax = vref ? *vref : key_value(st->kmin);
  for (int i = blockIdx.x * 256 + tid; i < n; i += gridDim.x * 256)
    atomicAdd(&h[gap_bin(vmax, nan_to_ninf(cand[i]))], 1u);
  __syncthreads();
  for (int b = tid; b < kGapBins; b += 256)
    if (h[b]) atomicAdd(&gh[b], h[b]);
  __threadfence();
  __syncthreads();
  if (tid == 0) last = (atomicAdd(&st->done, 1u) == gridDim.x - 1) ? 1 : 0;
  __syncthreads();
  if (!last) return;
  __threadfence();
  // the last workgroup: the boundary bin from the complete histogram
  unsigned hb[16];
  int own = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    hb[j] = gh[16 * tid + j];
    own += (int)hb[j];
  }
  int tot;
  const int ex = block_excl_scan_count(own, wsum, &tot);
  if (ex < Me && ex + own >= Me) {
    int cum = ex, b = 16 * tid;
    for (int j = 0; j < 16; ++j) {
      cum += (int)hb[j];
      b = 16 * tid + j;
      if (cum >= Me) break;
    }
    st->bstar = b;
  }
  if (tid == 0) st->done = 0u;
}

// per = scores per thread; workgroup x covers [x * 256 * per, (x + 1) * 256 * per)
__global__ __launch_bounds__(256) void k_gsel_compact(int n, int per, const double *cand,
                                                      const double *vref, GselState *st,
                                                      double *cs, int32_t *is) {
  __shared__ int wsum[4];
  __shared__ int sh_base;
  const int tid = threadIdx.x;
  const int bstar = st->bstar;
  const double vmax = vref ? *vref : key_value(st->kmin);
  const int i0 = blockIdx.x * 256 * per + tid;
  int cnt = 0;
  for (int k = 0; k < per; ++k) {
    const int i = i0 + 256 * k;
    if (i < n && gap_bin(vmax, nan_to_ninf(cand[i])) <= bstar) ++cnt;
  }
  int tot;
  int pos = block_excl_scan_count(cnt, wsum, &tot);
  if (tid == 0) sh_base = (tot > 0) ? atomicAdd(&st->count, tot) : 0;
  __syncthreads();
  pos += sh_base;
  for (int k = 0; k < per; ++k) {
    const int i = i0 + 256 * k;
    if (i < n) {
      const double v = cand[i];
      if (gap_bin(vmax, nan_to_ninf(v)) <= bstar) {
        cs[pos] = v;
        is[pos] = i;
        ++pos;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_beam_update(SearchTabs t, int r, int c, int n_new,
                                                     const int32_t *sel, int N,
                                                     const uint8_t *cfg, const double *energy,
                                                     const double *L, const int32_t *anc,
                                                     const double *cand,
                                                     const double *sel_score, const double *A,
                                                     int update_L, uint8_t *cfg_o,
                                                     double *energy_o, double *score_o,
                                                     double *L_o, int32_t *anc_o, long ist) {
  SPG_INST(sel);
  SPG_INST(cfg);
  SPG_INST(energy);
  SPG_INST(L);
  SPG_INST(anc);
  SPG_INST(cand);
  SPG_INST(sel_score);
  SPG_INST(A);
  SPG_INST(cfg_o);
  SPG_INST(energy_o);
  SPG_INST(score_o);
  SPG_INST(L_o);
  SPG_INST(anc_o);
  shift_tabs(t, ist);
  __shared__ double Ls[kWaves][kMaxChi];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j0 = blockIdx.x * kWaves + w;
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
    energy_o[j] = energy[b] + delta_energy(t, r, c, cb, s);
    score_o[j] = sel_score ? sel_score[j] : cand[id];
    anc_o[j] = anc[b];
  }
  if (!update_L) return;
  if (valid)
    for (int i = lane; i < chi; i += 64) Ls[w][i] = L[(long)b * chi + i];
  __syncthreads();
  if (!valid) return;
  const double g = field(t, r, c, cb, s);
  double v[2] = {0.0, 0.0};
  for (int h = 0; h < 2; ++h) {
    const int bp = lane + 64 * h;
    if (bp >= chi) continue;
    double acc = 0.0;
    for (int al = 0; al < chi; ++al) acc += Ls[w][al] * A[((long)al * d + s) * chi + bp];
    v[h] = g * acc;
  }
  const double m = wave_max_nonneg(fmax(fabs(v[0]), fabs(v[1])));
  const double inv = (m > 0.0) ? 1.0 / m : 1.0;
  for (int h = 0; h < 2; ++h) {
    const int bp = lane + 64 * h;
    if (bp < chi) L_o[(long)j * chi + bp] = v[h] * inv;
  }
}

__global__ void k_reset_row(int n, int chi, double *L, int32_t *anc, long ist) {
  SPG_INST(L);
  SPG_INST(anc);
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * chi) return;
  const int j = (int)(e / chi), i = (int)(e % chi);
  L[e] = (i == 0) ? 1.0 : 0.0;
  if (i == 0) anc[j] = j;
}

// Energy of complete configurations by Eq. (1), one wavefront per state.
__global__ __launch_bounds__(256) void k_energy(SearchTabs t, int n, int N, const uint8_t *cfg,
                                                double *E, long ist) {
  SPG_INST(cfg);
  SPG_INST(E);
  shift_tabs(t, ist);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * kWaves + w;
  if (j >= n) return;
  const int R = t.rows, C = t.cols, d = t.d;
  const long dd = (long)d * d;
  const uint8_t *x = cfg + (long)j * N;
  double acc = 0.0;
  for (int k = lane; k < N; k += 64) {
    const int r = k / C, c = k % C;
    acc += t.E_loc[(long)k * d + x[k]];
    if (c + 1 < C) acc += t.E_h[((long)r * (C - 1) + c) * dd + x[k] * d + x[k + 1]];
    if (r + 1 < R) {
      acc += t.E_v[((long)r * C + c) * dd + x[k] * d + x[k + C]];
      if (c + 1 < C) {
        acc += t.E_d[((long)r * (C - 1) + c) * dd + x[k] * d + x[k + C + 1]];
        acc += t.E_a[((long)r * (C - 1) + c) * dd + x[k + 1] * d + x[k + C]];
      }
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) E[j] = acc;
}

__global__ __launch_bounds__(1024) void k_final_sort(int n, const double *E, const double *score,
                                                    uint64_t *kw, int32_t *iw, int32_t *nv, long ist) {
  SPG_INST(E);
  SPG_INST(score);
  SPG_INST(kw);
  SPG_INST(iw);
  SPG_INST(nv);
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int p2 = 1;
  while (p2 < n) p2 <<= 1;
  int local = 0;
  for (int i = threadIdx.x; i < p2; i += blockDim.x) {
    if (i < n) {
      // rows with a finite log-probability first, by energy; the rest (beam
      // slots filled with pruned or merged-away children) after them
      const double sc = score[i];
      const bool live = (sc == sc && sc > -INFINITY);
      kw[i] = live ? asc_key(E[i]) : ~0ull;
      iw[i] = i;
      local += live;
    } else {
      kw[i] = ~0ull;
      iw[i] = INT_MAX;
    }
  }
  atomicAdd(&cnt, local);
  __syncthreads();
  bitonic_sort(kw, iw, p2);
  if (threadIdx.x == 0) *nv = cnt;
}

__global__ void k_gather_out(int n, int N, const int32_t *perm, const uint8_t *cfg,
                             const double *E, const double *score, int32_t *states,
                             double *energies, double *logp, long ist) {
  SPG_INST(perm);
  SPG_INST(cfg);
  SPG_INST(E);
  SPG_INST(score);
  SPG_INST(states);
  SPG_INST(energies);
  SPG_INST(logp);
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * N) return;
  const int t = (int)(e / N), k = (int)(e % N);
  const int j = perm[t];
  states[e] = cfg[(long)j * N + k];
  if (k == 0) {
    energies[t] = E[j];
    logp[t] = score[j];
  }
}

__global__ __launch_bounds__(1024) void k_cutoff(int n_host, const int *n_dev, double log_cut,
                                                double *cand, long ist) {
  SPG_INST(n_dev);
  SPG_INST(cand);
  __shared__ double red[1024];
  const int n = n_dev ? *n_dev : n_host;
  double m = -INFINITY;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, cand[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  const double thr = red[0] + log_cut;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (!(cand[i] >= thr)) cand[i] = -INFINITY;
}

__global__ void k_cfg_from_i32(long n, const int32_t *src, uint8_t *dst, long ist) {
  SPG_INST(src);
  SPG_INST(dst);
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < n) dst[e] = (uint8_t)src[e];
}

// L^b <- g^b_c(x_c) L^b A[:, x_c, :], max-normalised, x_c read from cfg
__global__ __launch_bounds__(256) void k_advance_L(SearchTabs t, int r, int c, int n,
                                                   const uint8_t *cfg, int N, const double *A,
                                                   double *L, long ist) {
  SPG_INST(cfg);
  SPG_INST(A);
  SPG_INST(L);
  shift_tabs(t, ist);
  __shared__ double Ls[kWaves][kMaxChi];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b0 = blockIdx.x * kWaves + w;
  const bool valid = b0 < n;
  const int b = valid ? b0 : 0;
  const int d = t.d, chi = t.chi;
  const uint8_t *cb = cfg + (long)b * N;
  const int s = cb[r * t.cols + c];
  if (valid)
    for (int i = lane; i < chi; i += 64) Ls[w][i] = L[(long)b * chi + i];
  __syncthreads();
  if (!valid) return;
  const double g = field(t, r, c, cb, s);
  double v[2] = {0.0, 0.0};
  for (int h = 0; h < 2; ++h) {
    const int bp = lane + 64 * h;
    if (bp >= chi) continue;
    double acc = 0.0;
    for (int al = 0; al < chi; ++al) acc += Ls[w][al] * A[((long)al * d + s) * chi + bp];
    v[h] = g * acc;
  }
  const double m = wave_max_nonneg(fmax(fabs(v[0]), fabs(v[1])));
  const double inv = (m > 0.0) ? 1.0 / m : 1.0;
  for (int h = 0; h < 2; ++h) {
    const int bp = lane + 64 * h;
    if (bp < chi) L[(long)b * chi + bp] = v[h] * inv;
  }
}

// ---- merging branches ------------------------------------------------------
// Children of one step that share a frontier (the states of the last w sites
// of the order, the child's own included) compete; the one with the lowest
// energy of its fixed part (ties: lowest id b d + s) keeps its score, the
// others get -inf.  The frontier is packed exactly into 63 bits when
// w * bits <= 63 (bits per state), else hashed.  An open-addressing table
// (power-of-two size, at least twice the children) collects per frontier the
// least energy key and then the least id among children with that energy.
constexpr unsigned long long kEmpty = ~0ull;

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_merge_clear(int T, unsigned long long *tkey, unsigned long long *te,
                              int32_t *tid, unsigned long long *te2, int32_t *tid2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T) return;
  tkey[e] = kEmpty;
  te[e] = kEmpty;
  tid[e] = INT_MAX;
  if (te2) {
    te2[e] = kEmpty;
    tid2[e] = INT_MAX;
  }
}

__global__ void k_merge_insert(SearchTabs t, int r, int c, int n_beam, const uint8_t *cfg, int N,
                               const double *energy, const double *cand, int w, int bits,
                               int T, unsigned long long *tkey, unsigned long long *te,
                               int32_t *slot_of, unsigned long long *ekey_of) {
  const int d = t.d;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n_beam * d) return;
  const int b = (int)(e / d), s = (int)(e % d);
  const double sc = cand[e];
  slot_of[e] = -1;
  if (!(sc > -INFINITY)) return;
  const uint8_t *cb = cfg + (long)b * N;
  const int k = r * t.cols + c;
  unsigned long long key;
  if (w * bits <= 63) {
    key = (unsigned long long)s;
    for (int i = 1; i < w; ++i) key |= (unsigned long long)cb[k - i] << (bits * i);
  } else {
    key = mix64(0x9E3779B97F4A7C15ull + (unsigned long long)s);
    for (int i = 1; i < w; ++i) key = mix64(key + cb[k - i] + 0x9E3779B97F4A7C15ull * i);
    key &= 0x7FFFFFFFFFFFFFFFull;
  }
  const unsigned long long ek = asc_key(energy[b] + delta_energy(t, r, c, cb, s));
  unsigned h = (unsigned)mix64(key) & (unsigned)(T - 1);
  for (int probe = 0; probe < T; ++probe) {
    const unsigned long long cur = atomicCAS(&tkey[h], kEmpty, key);
    if (cur == kEmpty || cur == key) {
      atomicMin(&te[h], ek);
      slot_of[e] = (int)h;
      ekey_of[e] = ek;
      return;
    }
    h = (h + 1) & (unsigned)(T - 1);
  }
}

__global__ void k_merge_tie(long n, const int32_t *slot_of, const unsigned long long *ekey_of,
                            const unsigned long long *te, int32_t *tid) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int h = slot_of[e];
  if (h >= 0 && ekey_of[e] == te[h]) atomicMin(&tid[h], (int32_t)e);
}

// Runner-up of each group: least energy key among the members that were not
// kept, then the least id among those at that energy.
__global__ void k_merge_second(long n, const int32_t *slot_of, const unsigned long long *ekey_of,
                               const int32_t *tid, unsigned long long *te2) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int h = slot_of[e];
  if (h >= 0 && tid[h] != (int32_t)e) atomicMin(&te2[h], ekey_of[e]);
}

__global__ void k_merge_second_tie(long n, const int32_t *slot_of,
                                   const unsigned long long *ekey_of, const int32_t *tid,
                                   const unsigned long long *te2, int32_t *tid2) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int h = slot_of[e];
  if (h >= 0 && tid[h] != (int32_t)e && ekey_of[e] == te2[h]) atomicMin(&tid2[h], (int32_t)e);
}

__global__ void k_merge_apply(long n, const int32_t *slot_of, const int32_t *tid, double *cand,
                              const int32_t *tid2, int32_t *run) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int h = slot_of[e];
  if (h >= 0 && tid[h] != (int32_t)e) cand[e] = -INFINITY;
  if (run) run[e] = (h >= 0 && tid[h] == (int32_t)e && tid2[h] != INT_MAX) ? tid2[h] : -1;
}

// One wavefront per survivor j (see droplet_update).  Configurations are
// compared over the sites fixed so far, 0..k.
__global__ __launch_bounds__(256) void k_droplet_update(SearchTabs t, int r, int c, int n_new,
                                                        const int32_t *sel, int N,
                                                        const uint8_t *cfg, const double *energy,
                                                        const int32_t *run, const uint8_t *din,
                                                        const double *dein, const int32_t *dnin,
                                                        uint8_t *dout, double *deout,
                                                        int32_t *dnout, int D, double ecut,
                                                        int hcut) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * kWaves + w;
  if (j >= n_new) return;
  const int d = t.d, k = r * t.cols + c;
  const int id = sel[j], b = id / d, s = id % d;
  const uint8_t *cb = cfg + (long)b * N;
  const int nin = dnin[b];
  // inherited droplets, the new site set to this state's value
  for (long e = lane; e < (long)nin * N; e += 64) {
    const int m = (int)(e / N), i = (int)(e % N);
    dout[((long)j * D + m) * N + i] = (i == k) ? (uint8_t)s : din[((long)b * D + m) * N + i];
  }
  for (int m = lane; m < nin; m += 64) deout[(long)j * D + m] = dein[(long)b * D + m];
  int cnt = nin;
  const int o = run[id];
  if (o >= 0 && cnt < D) {
    const int bo = o / d, so = o % d;
    const uint8_t *co = cfg + (long)bo * N;
    const double ek = energy[b] + delta_energy(t, r, c, cb, s);
    const double eo = energy[bo] + delta_energy(t, r, c, co, so);
    const double de = eo - ek;
    if (de <= ecut) {
      // distance of the runner-up to this state, then to each inherited droplet
      auto dist = [&](int m) {
        int cntd = 0;
        for (int i0 = 0; i0 <= k; i0 += 64) {
          const int i = i0 + lane;
          bool diff = false;
          if (i <= k) {
            const uint8_t x = (i == k) ? (uint8_t)so : co[i];
            const uint8_t y = (i == k) ? (uint8_t)s
                              : (m < 0 ? cb[i] : din[((long)b * D + m) * N + i]);
            diff = x != y;
          }
          cntd += __popcll(__ballot(diff));
        }
        return cntd;
      };
      bool ok = dist(-1) > hcut;
      for (int m = 0; m < nin && ok; ++m) ok = dist(m) > hcut;
      if (ok) {
        for (int i = lane; i < N; i += 64)
          dout[((long)j * D + cnt) * N + i] = (i == k) ? (uint8_t)so : (i < k ? co[i] : (uint8_t)0);
        if (lane == 0) deout[(long)j * D + cnt] = de;
        ++cnt;
      }
    }
  }
  if (lane == 0) dnout[j] = cnt;
}

}  // namespace

void u64_col(int n_anc, const double *A_rc, int chi, const double *Rnext, long rstride,
             double *U, long ldu, int d, int cl, int cr, hipStream_t s) {
  if (n_anc <= 0 || cl <= 0 || cr <= 0) return;
  GemmDesc g{};
  g.M = n_anc; g.N = cl * d; g.K = cr; g.nb1 = 1; g.nb2 = 1;
  g.A = Rnext; g.a_i = rstride; g.a_k = 1;
  g.B = A_rc; g.b_k = 1; g.b_j = chi;
  g.C = U; g.c_i = ldu; g.c_j = 1;
  g.alpha = 1.0; g.beta = 0.0;
  // many output tiles (the 4096 x 1536 products of the 12x12 d = 24
  // workload): 64 x 64 tiles do more products per tile load (30.8 -> 26.3 us
  // per launch there); each 16 x 16 block keeps its order of products over k
  if ((long)((g.M + 31) / 32) * ((g.N + 31) / 32) >= 2048) g.tile = 64;
  gemm_f64(g, s);
}

void env_from_u64(const SearchTabs &t, int r, int c, int n_anc, const uint8_t *cfg, int N,
                  const double *U, long ldu, double *Rout, long rstride, int cl, hipStream_t s,
                  double *scale, int sstride) {
  KTimer kt_("right_env", s, 2.0 * n_anc * cl * t.d);
  if (n_anc <= 0) return;
  SPG_BC(cfg);
  SPG_BC(U);
  SPG_BC(Rout);
  SPG_BC(scale);
  bc_check_tabs(t);
  if (t.d > 256 || cl > 128) {
    set_error("env_from_u64: d or bond dimension too large");
    throw Fail{SPG_ERR_UNSUPPORTED};
  }
  hipLaunchKernelGGL(k_env_from_u64, dim3(nblk(n_anc, kWaves), g_bc.n), dim3(256), 0, s, t, r, c,
                     n_anc, cfg, N, U, ldu, Rout, rstride, cl, scale, sstride, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void marg_from_u64(const SearchTabs &t, int r, int c, int n_beam, const uint8_t *cfg, int N,
                   const double *U, long ldu, const double *L, const int32_t *anc,
                   const double *score, double *out, int add_score, int cl, hipStream_t s) {
  KTimer kt_("marginals", s, 2.0 * n_beam * t.d * cl);
  if (n_beam <= 0) return;
  SPG_BC(cfg);
  SPG_BC(U);
  SPG_BC(L);
  SPG_BC(anc);
  SPG_BC(score);
  SPG_BC(out);
  bc_check_tabs(t);
  if (t.d > 256) {
    set_error("marg_from_u64: d too large");
    throw Fail{SPG_ERR_UNSUPPORTED};
  }
  hipLaunchKernelGGL(k_marg_from_u64, dim3(nblk(n_beam, kWaves), g_bc.n), dim3(256), 0, s, t, r,
                     c, n_beam, cfg, N, U, ldu, L, anc, score, out, add_score, cl, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void right_env_col(const SearchTabs &t, int r, int c, int n_anc, const uint8_t *cfg, int N,
                   const double *A_rc, const double *Rnext, double *Rout, long rstride,
                   int cl, int cr, hipStream_t s, double *scale, int sstride) {
  KTimer kt_("right_env", s, 2.0 * n_anc * cl * t.d * cr);
  if (n_anc <= 0) return;
  SPG_BC(cfg);
  SPG_BC(A_rc);
  SPG_BC(Rnext);
  SPG_BC(Rout);
  SPG_BC(scale);
  bc_check_tabs(t);
  if (cl > 0 && cr > 0 && env_lds_fits(cl, t.d, cr))
    hipLaunchKernelGGL(k_right_env_lds, dim3(nblk(n_anc, kWaves), g_bc.n), dim3(256), 0, s, t, r,
                       c, n_anc, cfg, N, A_rc, Rnext, Rout, rstride, scale, sstride, cl, cr,
                       g_bc.ist);
  else
    hipLaunchKernelGGL(k_right_env, dim3(nblk(n_anc, kWaves), g_bc.n), dim3(256), 0, s, t, r, c, n_anc, cfg, N, A_rc, Rnext, Rout, rstride, scale, sstride, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void marginals(const SearchTabs &t, int r, int c, int n_beam, const uint8_t *cfg, int N,
               const double *A_rc, const double *L, const int32_t *anc, const double *Rv,
               long rstride, const double *score, double *out, int add_score, int cl, int cr,
               hipStream_t s) {
  KTimer kt_("marginals", s, 2.0 * n_beam * t.d * cl * cr);
  if (n_beam <= 0) return;
  SPG_BC(cfg);
  SPG_BC(A_rc);
  SPG_BC(L);
  SPG_BC(anc);
  SPG_BC(Rv);
  SPG_BC(score);
  SPG_BC(out);
  bc_check_tabs(t);
  if (cl > 0 && cr > 0 && marg_lds_fits(cl, t.d, cr))
    hipLaunchKernelGGL(k_marginals_lds, dim3(nblk(n_beam, kWaves), g_bc.n), dim3(256), 0, s, t, r,
                       c, n_beam, cfg, N, A_rc, L, anc, Rv, rstride, score, out, add_score, cl, cr,
                       g_bc.ist);
  else
    hipLaunchKernelGGL(k_marginals, dim3(nblk(n_beam, kWaves), g_bc.n), dim3(256), 0, s, t, r, c, n_beam, cfg, N, A_rc, L, anc, Rv, rstride, score, out, add_score, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

size_t select_ws_bytes(long n_cap) {
  return 256 + sizeof(unsigned) * (size_t)kGapBins + 12 * (size_t)n_cap;
}

void select_topm(int n_cand, int M, const double *cand, int32_t *sel, uint64_t *keys_work,
                 int32_t *ids_work, hipStream_t s, const int *n_dev, const int32_t *cid,
                 double *sel_score, void *big_ws, long ws_cap, const double *vref) {
  KTimer kt_("select_topm", s, (cid ? 12.0 : 8.0) * n_cand + 4.0 * (M < n_cand ? M : n_cand));
  const int Me = (M < n_cand) ? M : n_cand;
  if (big_ws && !n_dev && !cid && g_bc.n == 1 && n_cand > kSelRegKeys * 1024 && Me < n_cand &&
      Me >= 1 && n_cand <= ws_cap) {
    // workspace: state (256 B), histogram, survivors' scores and indices [n_cand];
    // the histogram and the count are zero at entry (zero-filled allocation, then
    // cleared by the last k_select of each call)
    GselState *st = reinterpret_cast<GselState *>(big_ws);
    unsigned *gh = reinterpret_cast<unsigned *>(static_cast<char *>(big_ws) + 256);
    double *cs = reinterpret_cast<double *>(gh + kGapBins);
    int32_t *is = reinterpret_cast<int32_t *>(cs + ws_cap);
    constexpr int kPer = 8;
    const unsigned G = (unsigned)(((long)n_cand + 256 * kPer - 1) / (256 * kPer));
    if (!vref) {
      hipLaunchKernelGGL(k_gsel_init, dim3(1), dim3(1024), 0, s, st, gh);
      SPG_CHECK_LAUNCH();
      hipLaunchKernelGGL(k_gsel_min, dim3(G), dim3(256), 0, s, n_cand, cand, st);
      SPG_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_gsel_hist, dim3(G), dim3(256), 0, s, n_cand, Me, cand, vref, st, gh);
    SPG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_gsel_compact, dim3(G), dim3(256), 0, s, n_cand, kPer, cand, vref, st,
                       cs, is);
    SPG_CHECK_LAUNCH();
    // the survivors (at least Me) ordered by (score, original index)
    hipLaunchKernelGGL(k_select, dim3(1, 1), dim3(1024), 0, s, 0, (const int *)&st->count, Me,
                       (const double *)cs, (const int32_t *)is, sel, sel_score, keys_work,
                       ids_work, 0L, gh, &st->count);
    SPG_CHECK_LAUNCH();
    return;
  }
  SPG_BC(n_dev);
  SPG_BC(cand);
  SPG_BC(cid);
  SPG_BC(sel);
  SPG_BC(sel_score);
  SPG_BC(keys_work);
  SPG_BC(ids_work);
  hipLaunchKernelGGL(k_select, dim3(1, g_bc.n), dim3(1024), 0, s, n_cand, n_dev, M, cand, cid,
                     sel, sel_score, keys_work, ids_work, g_bc.ist, (unsigned *)nullptr,
                     (int *)nullptr);
  SPG_CHECK_LAUNCH();
}

void beam_update(const SearchTabs &t, int r, int c, int n_new, const int32_t *sel, int N,
                 const uint8_t *cfg, const double *energy, const double *L, const int32_t *anc,
                 const double *cand, const double *A_rc, int update_L, uint8_t *cfg_o,
                 double *energy_o, double *score_o, double *L_o, int32_t *anc_o, int cl,
                 int cr, hipStream_t s, const double *sel_score) {
  KTimer kt_("beam_update", s, 2.0 * n_new * cl * cr);
  if (n_new <= 0) return;
  SPG_BC(sel);
  SPG_BC(cfg);
  SPG_BC(energy);
  SPG_BC(L);
  SPG_BC(anc);
  SPG_BC(cand);
  SPG_BC(sel_score);
  SPG_BC(A_rc);
  SPG_BC(cfg_o);
  SPG_BC(energy_o);
  SPG_BC(score_o);
  SPG_BC(L_o);
  SPG_BC(anc_o);
  bc_check_tabs(t);
  hipLaunchKernelGGL(k_beam_update, dim3(nblk(n_new, kWaves), g_bc.n), dim3(256), 0, s, t, r, c, n_new, sel, N, cfg, energy, L, anc, cand, sel_score, A_rc, update_L, cfg_o, energy_o, score_o, L_o, anc_o, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void beam_reset_row(int n, int chi, double *L, int32_t *anc, hipStream_t s) {
  const long tot = (long)n * chi;
  SPG_BC(L);
  SPG_BC(anc);
  hipLaunchKernelGGL(k_reset_row, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, n, chi, L, anc, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void final_sort(const SearchTabs &t, int n, int N, const uint8_t *cfg, const double *score,
                int32_t *states_out, double *energies_out, double *logp_out, double *e_work,
                int32_t *perm_work, int32_t *n_valid, hipStream_t s) {
  KTimer kt_("final_sort", s);
  SPG_BC(cfg);
  SPG_BC(e_work);
  bc_check_tabs(t);
  hipLaunchKernelGGL(k_energy, dim3(nblk(n, kWaves), g_bc.n), dim3(256), 0, s, t, n, N, cfg, e_work, g_bc.ist);
  SPG_CHECK_LAUNCH();
  uint64_t *kw = reinterpret_cast<uint64_t *>(e_work + n);
  SPG_BC(e_work);
  SPG_BC(score);
  SPG_BC(kw);
  SPG_BC(perm_work);
  SPG_BC(n_valid);
  hipLaunchKernelGGL(k_final_sort, dim3(1, g_bc.n), dim3(1024), 0, s, n, e_work, score, kw, perm_work, n_valid, g_bc.ist);
  SPG_CHECK_LAUNCH();
  const long tot = (long)n * N;
  SPG_BC(perm_work);
  SPG_BC(cfg);
  SPG_BC(e_work);
  SPG_BC(score);
  SPG_BC(states_out);
  SPG_BC(energies_out);
  SPG_BC(logp_out);
  hipLaunchKernelGGL(k_gather_out, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, n, N, perm_work, cfg, e_work, score, states_out, energies_out, logp_out, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void apply_cutoff(int n, double log_cut, double *cand, hipStream_t s, const int *n_dev) {
  SPG_BC(n_dev);
  SPG_BC(cand);
  hipLaunchKernelGGL(k_cutoff, dim3(1, g_bc.n), dim3(1024), 0, s, n, n_dev, log_cut, cand, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void cfg_from_i32(int n, int N, const int32_t *src, uint8_t *dst, hipStream_t s) {
  const long tot = (long)n * N;
  SPG_BC(src);
  SPG_BC(dst);
  hipLaunchKernelGGL(k_cfg_from_i32, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, tot, src, dst, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void advance_L(const SearchTabs &t, int r, int c, int n, const uint8_t *cfg, int N,
               const double *A_rc, double *L, double *tmp, hipStream_t s) {
  (void)tmp;
  SPG_BC(cfg);
  SPG_BC(A_rc);
  SPG_BC(L);
  bc_check_tabs(t);
  hipLaunchKernelGGL(k_advance_L, dim3(nblk(n, kWaves), g_bc.n), dim3(256), 0, s, t, r, c, n, cfg, N, A_rc, L, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void merge_branches(const SearchTabs &t, int r, int c, int n_beam, const uint8_t *cfg, int N,
                    const double *energy, double *cand, MergeWork &mw, hipStream_t s) {
  bc_single("merge_branches");
  KTimer kt_("merge_branches", s, 24.0 * n_beam * t.d);
  const long n = (long)n_beam * t.d;
  if (n <= 0) return;
  int T = 1;
  while (T < 2 * n) T <<= 1;
  if (T > mw.capacity) {
    set_error("merge_branches: table too small");
    throw Fail{SPG_ERR_INVALID};
  }
  const int k = r * t.cols + c;
  const int w = std::min(k + 1, t.cols + 1);
  int bits = 1;
  while ((1 << bits) < t.d) ++bits;
  hipLaunchKernelGGL(k_merge_clear, dim3(nblk(T, 256)), dim3(256), 0, s, T, mw.tkey, mw.te, mw.tid,
                     mw.te2, mw.tid2);
  SPG_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_merge_insert, dim3(nblk(n, 256)), dim3(256), 0, s, t, r, c, n_beam, cfg, N,
                     energy, cand, w, bits, T, mw.tkey, mw.te, mw.slot, mw.ekey);
  SPG_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_merge_tie, dim3(nblk(n, 256)), dim3(256), 0, s, n, mw.slot, mw.ekey, mw.te,
                     mw.tid);
  SPG_CHECK_LAUNCH();
  if (mw.run) {
    hipLaunchKernelGGL(k_merge_second, dim3(nblk(n, 256)), dim3(256), 0, s, n, mw.slot, mw.ekey,
                       mw.tid, mw.te2);
    SPG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_merge_second_tie, dim3(nblk(n, 256)), dim3(256), 0, s, n, mw.slot,
                       mw.ekey, mw.tid, mw.te2, mw.tid2);
    SPG_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_merge_apply, dim3(nblk(n, 256)), dim3(256), 0, s, n, mw.slot, mw.tid, cand,
                     mw.tid2, mw.run);
  SPG_CHECK_LAUNCH();
}

void droplet_update(const SearchTabs &t, int r, int c, int n_new, const int32_t *sel, int N,
                    const uint8_t *cfg, const double *energy, const int32_t *run,
                    const uint8_t *din, const double *dein, const int32_t *dnin, uint8_t *dout,
                    double *deout, int32_t *dnout, int D, double ecut, int hcut, hipStream_t s) {
  bc_single("droplet_update");
  KTimer kt_("droplets", s);
  if (n_new <= 0) return;
  hipLaunchKernelGGL(k_droplet_update, dim3(nblk(n_new, kWaves)), dim3(256), 0, s, t, r, c, n_new,
                     sel, N, cfg, energy, run, din, dein, dnin, dout, deout, dnout, D, ecut, hcut);
  SPG_CHECK_LAUNCH();
}

}  // namespace spg
