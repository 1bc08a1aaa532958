// Search steps with the learned proposal and its exactness guard (FP64
// exact weights).  Per site (r, c), parents b sorted by score (b = 0 best):
//   1. k_propose: features and network -> pred(b,s) = score_b + log p^(s|b);
//      the gap score_0 - pred in bins of 1/64 goes into a histogram;
//   2. k_tau_pred: first bin j* at which the running count reaches K =
//      ceil(kappa M); the candidate set E is every child with bin <= j*
//      (all children when j* is the last bin);
//   3. k_eval: per parent, Z_b = L^b R_c (the right environment one column
//      further left, times its stored scale), the exact q(b,s) of the
//      children in E, their scores score_b + log(q / Z_b) appended to a
//      compact list, and the bound score_b + log((max(U_b,0) + eps Z_b) / Z_b)
//      of every unevaluated child, U_b = Z_b - sum of the evaluated q;
//   4. k_tau_bound: tau = a lower bound of the M-th best score of the list
//      (-inf if it is shorter), the lower edge of the gap bin holding it;
//   5. k_fallback: parents whose bound reaches tau - margin (or with Z_b <= 0
//      or a negative evaluated q) get all d children evaluated as in the plain
//      search (normaliser sum_s max(q, 0)); their list entries are rewritten
//      and the other children appended;
//   6. the plain search's cut-off and top-M selection run on the list.
// An unevaluated child of a parent that did not fall back scores below
// tau - margin, below the true M-th score, so the kept beam is the plain
// search's.  On a reduced-precision env (k_eval_lp, k_fallback_lp) the exact
// weights are the plain reduced-precision search's (U products, FP32 L), and
// Z_b goes through R_c stored in that precision: the relative floor eps and
// the margin grow to the precision's resolution of Z_b (kEpsLp).
#include <cfloat>
#include <climits>

#include "lp_dev.h"
#include "mlp_dev.h"
#include "search_dev.h"
#include "spg_internal.h"
#include "wave.h"

namespace spg {

namespace {

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

constexpr int kWaves = 4;
constexpr int kNBins = 2048;
constexpr double kBinScale = 64.0;
constexpr double kEps = 1e-9;      // relative floor of the unevaluated weight
constexpr double kMargin = 1e-9;   // absolute margin of the bound test (log units)
// the same two for FP32 and for BF16 envs (R_c rounded to 2^-9), set at the
// accuracy the reduced-precision search states for its log-marginals
constexpr double kEpsLp32 = 1e-3, kEpsLpBf16 = 3e-2;

// Per-site features that do not depend on the parent: sf[site][s][0] the
// look-ahead over the unexplored neighbours, sf[site][s][1] the log one-site
// weight of the boundary MPS with every other state summed; both relative to
// their maximum over s, clamped at -30 and divided by 10.  One block per row;
// rscr holds the row's summed right vectors [cols+1][chi].
__global__ __launch_bounds__(256) void k_site_feats(SearchTabs t, const double *A, float *sf,
                                                    double *rscr) {
  __shared__ double vec[kMaxChi];
  __shared__ double red[256];
  const int r = blockIdx.x, tid = threadIdx.x;
  const int R = t.rows, C = t.cols, d = t.d, chi = t.chi;
  const size_t site_sz = (size_t)chi * d * chi;
  double *rs = rscr + (size_t)r * (C + 1) * chi;
  auto block_max = [&](double v) {
    red[tid] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] = fmax(red[tid], red[tid + o]);
      __syncthreads();
    }
    const double m = red[0];
    __syncthreads();
    return m;
  };
  // right vectors r_C = e_0, r_c = sum_s A_c[:, s, :] r_{c+1}, max-normalised
  for (int i = tid; i < chi; i += 256) rs[(size_t)C * chi + i] = (i == 0) ? 1.0 : 0.0;
  __syncthreads();
  for (int c = C - 1; c >= 1; --c) {
    const double *Ac = A + ((size_t)r * C + c) * site_sz;
    const double *rn = rs + (size_t)(c + 1) * chi;
    double v = 0.0;
    if (tid < chi)
      for (int s = 0; s < d; ++s) {
        const double *row = Ac + ((size_t)tid * d + s) * chi;
        for (int b = 0; b < chi; ++b) v += row[b] * rn[b];
      }
    const double m = block_max(tid < chi ? fabs(v) : 0.0);
    if (tid < chi) rs[(size_t)c * chi + tid] = (m > 0.0) ? v / m : v;
    __syncthreads();
  }
  // left vector l_0 = e_0; per column the one-site weights, then l_{c+1}
  for (int i = tid; i < chi; i += 256) vec[i] = (i == 0) ? 1.0 : 0.0;
  __syncthreads();
  const long dd = (long)d * d;
  const double beta = t.beta;
  for (int c = 0; c < C; ++c) {
    const double *Ac = A + ((size_t)r * C + c) * site_sz;
    const double *rn = rs + (size_t)(c + 1) * chi;
    const int s = tid;
    double lm = -INFINITY, la = -INFINITY;
    if (s < d) {
      double m = 0.0;
      for (int al = 0; al < chi; ++al) {
        const double l = vec[al];
        if (l == 0.0) continue;
        const double *row = Ac + ((size_t)al * d + s) * chi;
        double u = 0.0;
        for (int b = 0; b < chi; ++b) u += row[b] * rn[b];
        m += l * u;
      }
      lm = log(fmax(m, 1e-300));
      // log sum_y exp(-beta (E_n(y) + E_pair(s, y))) over unexplored neighbours
      auto lse = [&](const double *pair, long ps, long py, const double *En) {
        double mx = -INFINITY;
        for (int y = 0; y < d; ++y) mx = fmax(mx, -beta * (En[y] + pair[s * ps + y * py]));
        double acc = 0.0;
        for (int y = 0; y < d; ++y) acc += exp(-beta * (En[y] + pair[s * ps + y * py]) - mx);
        return mx + log(acc);
      };
      la = 0.0;
      if (c + 1 < C)
        la += lse(t.E_h + ((long)r * (C - 1) + c) * dd, d, 1, t.E_loc + ((long)r * C + c + 1) * d);
      if (r + 1 < R) {
        la += lse(t.E_v + ((long)r * C + c) * dd, d, 1, t.E_loc + ((long)(r + 1) * C + c) * d);
        if (t.kings && c + 1 < C)
          la += lse(t.E_d + ((long)r * (C - 1) + c) * dd, d, 1,
                    t.E_loc + ((long)(r + 1) * C + c + 1) * d);
        if (t.kings && c > 0)
          la += lse(t.E_a + ((long)r * (C - 1) + c - 1) * dd, d, 1,
                    t.E_loc + ((long)(r + 1) * C + c - 1) * d);
      }
    }
    const double mlm = block_max(lm);
    const double mla = block_max(la);
    if (s < d) {
      float *o = sf + (((size_t)r * C + c) * d + s) * 2;
      o[0] = (float)(fmax(la - mla, -30.0) / 10.0);
      o[1] = (float)(fmax(lm - mlm, -30.0) / 10.0);
    }
    // l_{c+1}[b] = sum_al l[al] sum_s A_c[al][s][b]
    double v = 0.0;
    if (tid < chi)
      for (int al = 0; al < chi; ++al) {
        const double l = vec[al];
        if (l == 0.0) continue;
        for (int s2 = 0; s2 < d; ++s2) v += l * Ac[((size_t)al * d + s2) * chi + tid];
      }
    const double m = block_max(tid < chi ? fabs(v) : 0.0);
    if (tid < chi) vec[tid] = (m > 0.0) ? v / m : v;
    __syncthreads();
  }
}

// Features, network and (search mode) candidate bins, one wavefront per parent.
__global__ __launch_bounds__(256) void k_propose(SearchTabs t, int r, int c, int n_beam,
                                                 const uint8_t *cfg, int N, const double *score,
                                                 const double *smax_p, const float *sf,
                                                 const float *prm, int H, float *feat_out,
                                                 uint16_t *bin_out, unsigned *hist) {
  __shared__ float P[kMaxHidden * (kFeat + 2) + 1];
  const int np = mlp_n_params(H);
  for (int i = threadIdx.x; i < np; i += blockDim.x) P[i] = prm ? prm[i] : 0.0f;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.x * kWaves + w;
  if (b >= n_beam) return;                 // no barrier below
  const int d = t.d, C = t.cols, R = t.rows;
  const uint8_t *cb = cfg + (long)b * N;
  const double sb = score[b], smax = *smax_p;
  double x0[4];
  double mx = -INFINITY;
  for (int j = 0; j < 4; ++j) {
    const int s = lane + 64 * j;
    x0[j] = (s < d) ? -t.beta * delta_energy(t, r, c, cb, s) : -INFINITY;
    mx = fmax(mx, x0[j]);
  }
  mx = wave_max_d(mx);
  const float f3 = (float)c / (float)(C - 1);
  const float f4 = (R > 1) ? (float)r / (float)(R - 1) : 0.0f;
  const float f5 = (float)(fmax(sb - smax, -30.0) / 10.0);
  const float *sfs = sf + ((size_t)r * C + c) * d * 2;
  float lg[4];
  float lmx = -INFINITY;
  for (int j = 0; j < 4; ++j) {
    const int s = lane + 64 * j;
    lg[j] = -INFINITY;
    if (s >= d) continue;
    float f[kFeat];
    f[0] = (float)(fmax(x0[j] - mx, -30.0) / 10.0);
    f[1] = sfs[2 * s];
    f[2] = sfs[2 * s + 1];
    f[3] = f3;
    f[4] = f4;
    f[5] = f5;
    if (feat_out)
      for (int k = 0; k < kFeat; ++k) feat_out[((long)b * d + s) * kFeat + k] = f[k];
    lg[j] = mlp_logit(P, H, f);
    lmx = fmaxf(lmx, lg[j]);
  }
  if (!bin_out) return;
  lmx = wave_max_f(lmx);
  float se = 0.0f;
  for (int j = 0; j < 4; ++j)
    if (lane + 64 * j < d) se += expf(lg[j] - lmx);
  const float lse = lmx + logf(wave_sum_f(se));
  for (int j = 0; j < 4; ++j) {
    const int s = lane + 64 * j;
    if (s >= d) continue;
    const double pred = sb + (double)(lg[j] - lse);
    const double gap = (smax - pred) * kBinScale;
    int bin = kNBins - 1;
    if (gap == gap && gap < (double)(kNBins - 1)) bin = (gap > 0.0) ? (int)floor(gap) : 0;
    bin_out[(long)b * d + s] = (uint16_t)bin;
    atomicAdd(&hist[bin], 1u);
  }
}

// j* from the histogram (one wavefront); clears the histogram and the list
// length for the step.
__global__ __launch_bounds__(64) void k_tau_pred(unsigned *hist, int K, int *jstar,
                                                 int *n_list) {
  const int lane = threadIdx.x;
  constexpr int per = kNBins / 64;
  unsigned own = 0u;
  for (int j = 0; j < per; ++j) own += hist[lane * per + j];
  unsigned inc = own;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned v = __shfl_up(inc, o);
    if (lane >= o) inc += v;
  }
  const unsigned long long hit = __ballot(inc >= (unsigned)K);
  const int first = hit ? (__ffsll((long long)hit) - 1) : -1;
  if (first < 0) {
    if (lane == 0) *jstar = kNBins - 1;
  } else if (lane == first) {
    unsigned cum = inc - own;
    int j = 0;
    for (; j < per - 1; ++j) {
      cum += hist[lane * per + j];
      if (cum >= (unsigned)K) break;
    }
    *jstar = lane * per + j;
  }
  for (int j = 0; j < per; ++j) hist[lane * per + j] = 0u;
  if (lane == 0) *n_list = 0;
}

__device__ __forceinline__ bool in_set(const uint16_t *bins, long i, int js) {
  return js >= kNBins - 1 || (int)bins[i] <= js;
}

// Exact q(b,s) on the candidate set, one wavefront per parent.
__global__ __launch_bounds__(256) void k_eval(SearchTabs t, int r, int c, int n_beam,
                                              const uint8_t *cfg, int N, const double *A,
                                              const double *L, const int32_t *anc,
                                              const double *Rv, long rstride, const double *Rsc,
                                              const double *score, const uint16_t *bins,
                                              const int *jstar_p, double *lkey, int32_t *lid,
                                              int *n_list, double *bound, int32_t *off,
                                              int32_t *cnt, unsigned long long *stats) {
  __shared__ double Ls[kWaves][kMaxChi];
  __shared__ double Rn[kWaves][kMaxChi];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b0 = blockIdx.x * kWaves + w;
  const bool valid = b0 < n_beam;
  const int b = valid ? b0 : 0;
  const int chi = t.chi, d = t.d, C = t.cols;
  const int a = anc[b];
  const double *Rnx = Rv + (long)a * rstride + (long)(c + 1) * chi;
  const double *Rcc = Rv + (long)a * rstride + (long)c * chi;
  double zp = 0.0;
  if (valid)
    for (int i = lane; i < chi; i += 64) {
      const double l = L[(long)b * chi + i];
      Ls[w][i] = l;
      Rn[w][i] = Rnx[i];
      zp += l * Rcc[i];
    }
  __syncthreads();
  if (!valid) return;
  const double Z = Rsc[(long)a * (C + 1) + c] * wave_sum(zp);
  const int js = *jstar_p;
  const uint8_t *cb = cfg + (long)b * N;
  // the candidate set of this parent, in increasing s
  unsigned long long mask[4];
  int nb = 0;
  for (int j = 0; j < 4; ++j) {
    const int s = lane + 64 * j;
    mask[j] = __ballot(s < d && in_set(bins, (long)b * d + s, js));
    nb += __popcll(mask[j]);
  }
  int base = 0;
  if (lane == 0 && nb > 0) base = atomicAdd(n_list, nb);
  base = __shfl(base, 0);
  const double sb = score[b];
  double sumq = 0.0;
  bool neg = false;
  double myq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    unsigned long long m = mask[j];
    while (m) {
      const int l = __ffsll((long long)m) - 1;
      m &= m - 1;
      const int s = l + 64 * j;
      double part = 0.0;
      for (int h = 0; h < 2; ++h) {
        const int bp = lane + 64 * h;
        if (bp >= chi) continue;
        double acc = 0.0;
        for (int al = 0; al < chi; ++al) {
          const double la = Ls[w][al];
          if (la == 0.0) continue;
          acc += la * A[((long)al * d + s) * chi + bp];
        }
        part += acc * Rn[w][bp];
      }
      const double q = field(t, r, c, cb, s) * wave_sum(part);
      sumq += q;
      neg = neg || (q < 0.0);
      if (lane == l) myq[j] = q;
    }
  }
  const bool mark = !(Z > 0.0) || !isfinite(Z) || neg;
  const double lz = log(Z);
  int rank = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const unsigned long long m = mask[j];
    if ((m >> lane) & 1ull) {
      const int pos = base + rank + __popcll(m & ((1ull << lane) - 1ull));
      const double q = myq[j];
      lkey[pos] = (!mark && q > 0.0) ? sb + (log(q) - lz) : -INFINITY;
      lid[pos] = b * d + lane + 64 * j;
    }
    rank += __popcll(m);
  }
  if (lane == 0) {
    double bd;
    if (mark) bd = INFINITY;
    else if (nb == d) bd = -INFINITY;
    else bd = sb + log((fmax(Z - sumq, 0.0) + kEps * Z) / Z);
    bound[b] = bd;
    off[b] = base;
    cnt[b] = nb;
    atomicAdd(&stats[0], (unsigned long long)nb);
  }
}

// tau = a lower bound of the M-th best list score (-inf when the list is
// shorter than M): the lower score edge of the gap bin (gap_bin: 64 bins per
// octave of the gap below the best score) that holds it.  A parent whose
// bound reaches it falls back, a superset of those whose bound reaches the
// exact M-th score; one pass over the list.
__global__ __launch_bounds__(1024) void k_tau_bound(const int *n_list, int M, const double *lkey,
                                                    double *tau) {
  __shared__ unsigned gh[kGapBins];
  __shared__ double wm[16];
  __shared__ int wsum[16];
  __shared__ int sh_b;
  const int tid = threadIdx.x;
  const int n = *n_list;
  if (n < M) {
    if (tid == 0) *tau = -INFINITY;
    return;
  }
  double vmax = -INFINITY;
  for (int i = tid; i < n; i += 1024) vmax = fmax(vmax, lkey[i]);
  vmax = wave_max_d(vmax);
  if ((tid & 63) == 0) wm[tid >> 6] = vmax;
  for (int b = tid; b < kGapBins; b += 1024) gh[b] = 0u;
  __syncthreads();
  vmax = -INFINITY;
  for (int w = 0; w < 16; ++w) vmax = fmax(vmax, wm[w]);
  if (!(vmax > -INFINITY)) {
    if (tid == 0) *tau = -INFINITY;
    return;
  }
  for (int i = tid; i < n; i += 1024) atomicAdd(&gh[gap_bin(vmax, lkey[i])], 1u);
  __syncthreads();
  unsigned hb[4];
  int own = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    hb[j] = gh[4 * tid + j];
    own += (int)hb[j];
  }
  int tot;
  const int ex = block_excl_scan_count(own, wsum, &tot);
  if (ex < M && ex + own >= M) {
    int cum = ex, b = 4 * tid;
    for (int j = 0; j < 4; ++j) {
      cum += (int)hb[j];
      b = 4 * tid + j;
      if (cum >= M) break;
    }
    sh_b = b;
  }
  __syncthreads();
  if (tid == 0) {
    const int b = sh_b;
    // every gap in bins <= b is below the double whose leading bits are bin b + 1
    const double g_hi = __hiloint2double((int)((unsigned)(b + 1 + ((1023 - 32) << 6)) << 14), 0);
    *tau = (b >= kGapBins - 1) ? -INFINITY : vmax - g_hi;
  }
}

// List entries of a parent evaluated in full: lp[j] = log p(s | b) for s = lane
// + 64 j; the children of the candidate set overwrite their entries at
// off[b].., the others are appended.
__device__ inline void write_full_parent(const SearchTabs &t, int b, double sb,
                                         const double (&lp)[4], const uint16_t *bins, int js,
                                         const int32_t *off, const int32_t *cnt, double *lkey,
                                         int32_t *lid, int *n_list, unsigned long long *stats,
                                         int lane) {
  const int d = t.d;
  const int nb = cnt[b];
  int extra = 0;
  if (lane == 0 && d - nb > 0) extra = atomicAdd(n_list, d - nb);
  extra = __shfl(extra, 0);
  const int o = off[b];
  int r_in = 0, r_out = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int s = lane + 64 * j;
    const bool ok = s < d;
    const bool ins = ok && in_set(bins, (long)b * d + s, js);
    const unsigned long long mi = __ballot(ins), mo = __ballot(ok && !ins);
    const unsigned long long below = (1ull << lane) - 1ull;
    if (ok) {
      const int pos = ins ? o + r_in + __popcll(mi & below) : extra + r_out + __popcll(mo & below);
      lkey[pos] = sb + lp[j];
      lid[pos] = b * d + s;
    }
    r_in += __popcll(mi);
    r_out += __popcll(mo);
  }
  if (lane == 0) {
    atomicAdd(&stats[0], (unsigned long long)d);
    atomicAdd(&stats[2], 1ull);
  }
}

// Full evaluation of the parents the guard selects, one wavefront per parent.
__global__ __launch_bounds__(256) void k_fallback(SearchTabs t, int r, int c, int n_beam,
                                                  const uint8_t *cfg, int N, const double *A,
                                                  const double *L, const int32_t *anc,
                                                  const double *Rv, long rstride,
                                                  const double *score, const uint16_t *bins,
                                                  const int *jstar_p, const double *tau_p,
                                                  const double *bound, const int32_t *off,
                                                  const int32_t *cnt, double *lkey, int32_t *lid,
                                                  int *n_list, unsigned long long *stats) {
  __shared__ double Ls[kWaves][kMaxChi];
  __shared__ double Rn[kWaves][kMaxChi];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b0 = blockIdx.x * kWaves + w;
  const int chi = t.chi, d = t.d;
  bool go = b0 < n_beam;
  const int b = go ? b0 : 0;
  if (go) {
    const double bd = bound[b];
    go = (bd == INFINITY) || (cnt[b] < d && bd >= *tau_p - kMargin);
  }
  const double *Rnx = Rv + (long)anc[b] * rstride + (long)(c + 1) * chi;
  if (go)
    for (int i = lane; i < chi; i += 64) {
      Ls[w][i] = L[(long)b * chi + i];
      Rn[w][i] = Rnx[i];
    }
  __syncthreads();
  if (!go) return;
  const uint8_t *cb = cfg + (long)b * N;
  double myq[4] = {0.0, 0.0, 0.0, 0.0};
  double part_tot = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    for (int l = 0; l < 64; ++l) {
      const int s = 64 * j + l;
      if (s >= d) break;
      double part = 0.0;
      for (int h = 0; h < 2; ++h) {
        const int bp = lane + 64 * h;
        if (bp >= chi) continue;
        double acc = 0.0;
        for (int al = 0; al < chi; ++al) {
          const double la = Ls[w][al];
          if (la == 0.0) continue;
          acc += la * A[((long)al * d + s) * chi + bp];
        }
        part += acc * Rn[w][bp];
      }
      double q = field(t, r, c, cb, s) * wave_sum(part);
      q = (q > 0.0) ? q : 0.0;             // negative q (truncation error) = probability 0
      if (lane == l) {
        myq[j] = q;
        part_tot += q;
      }
    }
  }
  const double tot = wave_sum(part_tot);
  const double ltot = log(tot);
  const double sb = score[b];
  // no child with positive weight: softmax_s(-beta dE) (local_softmax_norm)
  const bool dead = !(tot > 0.0);
  double emin = 0.0, lse = 0.0;
  if (dead) local_softmax_norm(t, r, c, cb, lane, emin, lse);
  double lpv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int s = lane + 64 * j;
    double lp = -INFINITY;
    if (s < d) {
      const double q = myq[j];
      lp = (q > 0.0 && tot > 0.0) ? log(q) - ltot : -INFINITY;
      if (!(lp == lp)) lp = -INFINITY;
      if (dead) lp = -t.beta * (delta_energy(t, r, c, cb, s) - emin) - lse;
    }
    lpv[j] = lp;
  }
  write_full_parent(t, b, sb, lpv, bins, *jstar_p, off, cnt, lkey, lid, n_list, stats, lane);
}

// Exact q(b,s) on the candidate set of a reduced-precision env, one
// wavefront per parent: q = exp(log g(s) - max_s log g) * (L^b . U^{anc}[:, s])
// (the couplings relative to their maximum, as in R_c) and
// Z_b = Rsc * (L^b . R_c); list entries and bounds as k_eval.
__global__ __launch_bounds__(256) void k_eval_lp(SearchTabs t, int r, int c, int n_beam,
                                                 const uint8_t *cfg, int N, const float *U,
                                                 long ldu, const float *L, const int32_t *anc,
                                                 const float *Rf, long rstride,
                                                 const double *Rsc, const double *score,
                                                 const uint16_t *bins, const int *jstar_p,
                                                 double eps, double *lkey, int32_t *lid,
                                                 int *n_list, double *bound, int32_t *off,
                                                 int32_t *cnt, unsigned long long *stats, int cl) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.x * kWaves + w;
  if (b >= n_beam) return;                 // no barrier below
  const int chi = t.chi, d = t.d, C = t.cols;
  const int a = anc[b];
  const float *Lb = L + (long)b * chi;
  const float *Ua = U + (long)a * ldu;
  const float *Rc = Rf + (long)a * rstride + (long)c * chi;
  float zp = 0.f;
  for (int al = lane; al < cl; al += 64) zp = fmaf(Lb[al], Rc[al], zp);
  const double Z = Rsc[(long)a * (C + 1) + c] * (double)wave_sum_f(zp);
  const uint8_t *cb = cfg + (long)b * N;
  double lmax = -INFINITY;
  for (int s = lane; s < d; s += 64) lmax = fmax(lmax, log_field(t, r, c, cb, s));
  lmax = wave_max_d(lmax);
  const int js = *jstar_p;
  unsigned long long mask[4];
  int nb = 0;
  for (int j = 0; j < 4; ++j) {
    const int s = lane + 64 * j;
    mask[j] = __ballot(s < d && in_set(bins, (long)b * d + s, js));
    nb += __popcll(mask[j]);
  }
  int base = 0;
  if (lane == 0 && nb > 0) base = atomicAdd(n_list, nb);
  base = __shfl(base, 0);
  const double sb = score[b];
  double sumq = 0.0;
  bool neg = false;
  double myq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    unsigned long long m = mask[j];
    while (m) {
      const int l = __ffsll((long long)m) - 1;
      m &= m - 1;
      const int s = l + 64 * j;
      float part = 0.f;
      for (int al = lane; al < cl; al += 64) part = fmaf(Lb[al], Ua[(long)al * d + s], part);
      const double q = exp(log_field(t, r, c, cb, s) - lmax) * (double)wave_sum_f(part);
      sumq += q;
      neg = neg || (q < 0.0);
      if (lane == l) myq[j] = q;
    }
  }
  const bool mark = !(Z > 0.0) || !isfinite(Z) || neg;
  const double lz = log(Z);
  int rank = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const unsigned long long m = mask[j];
    if ((m >> lane) & 1ull) {
      const int pos = base + rank + __popcll(m & ((1ull << lane) - 1ull));
      const double q = myq[j];
      lkey[pos] = (!mark && q > 0.0) ? sb + (log(q) - lz) : -INFINITY;
      lid[pos] = b * d + lane + 64 * j;
    }
    rank += __popcll(m);
  }
  if (lane == 0) {
    double bd;
    if (mark) bd = INFINITY;
    else if (nb == d) bd = -INFINITY;
    else bd = sb + log((fmax(Z - sumq, 0.0) + eps * Z) / Z);
    bound[b] = bd;
    off[b] = base;
    cnt[b] = nb;
    atomicAdd(&stats[0], (unsigned long long)nb);
  }
}

// Full evaluation of the parents the guard selects on a reduced-precision env:
// the plain reduced-precision conditionals (lp_parent_logp).
__global__ __launch_bounds__(256) void k_fallback_lp(SearchTabs t, int r, int c, int n_beam,
                                                     const uint8_t *cfg, int N, const float *U,
                                                     long ldu, const float *L,
                                                     const int32_t *anc, const double *score,
                                                     const uint16_t *bins, const int *jstar_p,
                                                     const double *tau_p, double margin,
                                                     const double *bound, const int32_t *off,
                                                     const int32_t *cnt, double *lkey,
                                                     int32_t *lid, int *n_list,
                                                     unsigned long long *stats, int cl) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.x * kWaves + w;
  if (b >= n_beam) return;                 // no barrier below
  const double bd = bound[b];
  if (!((bd == INFINITY) || (cnt[b] < t.d && bd >= *tau_p - margin))) return;
  double lp[4];
  lp_parent_logp(t, r, c, b, cfg, N, U, ldu, L, anc, cl, lane, lp);
  write_full_parent(t, b, score[b], lp, bins, *jstar_p, off, cnt, lkey, lid, n_list, stats, lane);
}

// Maximum of n doubles (one block) -> *out.
__global__ __launch_bounds__(256) void k_max(int n, const double *v, double *out) {
  __shared__ double red[256];
  double m = -INFINITY;
  for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, v[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

}  // namespace

void site_features(const SearchTabs &t, const double *A, float *sf, double *rscr,
                   hipStream_t s) {
  bc_single("site_features");
  hipLaunchKernelGGL(k_site_feats, dim3(t.rows), dim3(256), 0, s, t, A, sf, rscr);
  SPG_CHECK_LAUNCH();
}

void propose(const SearchTabs &t, int r, int c, int n_beam, const uint8_t *cfg, int N,
             const double *score, const double *smax, const float *sf, const float *prm, int H,
             float *feat_out, uint16_t *bins, unsigned *hist, hipStream_t s) {
  bc_single("propose");
  KTimer kt_("propose", s, 2.0 * n_beam * t.d * (kFeat * H + 2 * H));
  if (n_beam <= 0) return;
  hipLaunchKernelGGL(k_propose, dim3(nblk(n_beam, kWaves)), dim3(256), 0, s, t, r, c, n_beam,
                     cfg, N, score, smax, sf, prm, H, feat_out, bins, hist);
  SPG_CHECK_LAUNCH();
}

void guided_step(const SearchTabs &t, int r, int c, int n_beam, int M, int K, const uint8_t *cfg,
                 int N, const double *A_rc, const double *L, const int32_t *anc, const double *Rv,
                 long rstride, const double *Rsc, const double *score, GuideWork &g, int cl,
                 int cr, hipStream_t s) {
  bc_single("guided_step");
  hipLaunchKernelGGL(k_tau_pred, dim3(1), dim3(64), 0, s, g.hist, K, g.jstar, g.n_list);
  SPG_CHECK_LAUNCH();
  {
    // work: exact weights of the candidate set are counted by the fallback-free
    // share only on the device; the timer records the full per-parent cost bound
    KTimer kt_("guided_eval", s, 2.0 * n_beam * cl * cr);
    hipLaunchKernelGGL(k_eval, dim3(nblk(n_beam, kWaves)), dim3(256), 0, s, t, r, c, n_beam, cfg,
                       N, A_rc, L, anc, Rv, rstride, Rsc, score, g.bins, g.jstar, g.lkey, g.lid,
                       g.n_list, g.bound, g.off, g.cnt, g.stats);
    SPG_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_tau_bound, dim3(1), dim3(1024), 0, s, g.n_list, M, g.lkey, g.tau);
  SPG_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_fallback, dim3(nblk(n_beam, kWaves)), dim3(256), 0, s, t, r, c, n_beam,
                     cfg, N, A_rc, L, anc, Rv, rstride, score, g.bins, g.jstar, g.tau, g.bound,
                     g.off, g.cnt, g.lkey, g.lid, g.n_list, g.stats);
  SPG_CHECK_LAUNCH();
}

void guided_step_lp(const SearchTabs &t, int precision, int r, int c, int n_beam, int M, int K,
                    const uint8_t *cfg, int N, const float *U, long ldu, const float *L,
                    const int32_t *anc, const float *Rf, long rstride, const double *Rsc,
                    const double *score, GuideWork &g, int cl, hipStream_t s) {
  bc_single("guided_step_lp");
  const double eps = (precision == SPG_BF16) ? kEpsLpBf16 : kEpsLp32;
  hipLaunchKernelGGL(k_tau_pred, dim3(1), dim3(64), 0, s, g.hist, K, g.jstar, g.n_list);
  SPG_CHECK_LAUNCH();
  {
    KTimer kt_("guided_eval", s, 2.0 * n_beam * cl * t.d);
    hipLaunchKernelGGL(k_eval_lp, dim3(nblk(n_beam, kWaves)), dim3(256), 0, s, t, r, c, n_beam,
                       cfg, N, U, ldu, L, anc, Rf, rstride, Rsc, score, g.bins, g.jstar, eps,
                       g.lkey, g.lid, g.n_list, g.bound, g.off, g.cnt, g.stats, cl);
    SPG_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_tau_bound, dim3(1), dim3(1024), 0, s, g.n_list, M, g.lkey, g.tau);
  SPG_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_fallback_lp, dim3(nblk(n_beam, kWaves)), dim3(256), 0, s, t, r, c, n_beam,
                     cfg, N, U, ldu, L, anc, score, g.bins, g.jstar, g.tau, eps, g.bound, g.off,
                     g.cnt, g.lkey, g.lid, g.n_list, g.stats, cl);
  SPG_CHECK_LAUNCH();
}

void max_of(int n, const double *v, double *out, hipStream_t s) {
  bc_single("max_of");
  hipLaunchKernelGGL(k_max, dim3(1), dim3(256), 0, s, n, v, out);
  SPG_CHECK_LAUNCH();
}

}  // namespace spg
