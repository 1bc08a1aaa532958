// Internal declarations of the HIP implementation behind include/spg.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/spg.h"

namespace spg {

// ---- error plumbing ------------------------------------------------------
void set_error(const std::string &msg);
struct Fail {
  int code;
};
#define SPG_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::spg::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
      throw ::spg::Fail{SPG_ERR_HIP};                                              \
    }                                                                              \
  } while (0)
#define SPG_CHECK_LAUNCH() SPG_HIP(hipGetLastError())

// ---- opt-in per-launch timing (HIP events on the launch stream) ----------
struct KTimer {
  // `work`: algorithmic flops (or bytes for memory-bound classes) of the launch
  KTimer(const char *name, hipStream_t s, double work = 0.0);
  ~KTimer();
  int slot = -1;
  hipStream_t s = nullptr;
};

// ---- class-batched launches -------------------------------------------------
// Instances of one shape class keep all their device data in equal-sized
// slices of one allocation, `ist` bytes apart.  While a class runs, every
// launch covers all its instances at once: grid y (z for the GEMM) selects
// the instance and each kernel shifts its pointers by instance * ist.  Host
// wrappers check that every pointer they pass lies in the first slice
// [lo, hi) so no shifted access can leave the allocation.
struct BatchCtx {
  int n = 1;            // instances per launch
  long ist = 0;         // bytes between instances
  const char *lo = nullptr, *hi = nullptr;
};
extern thread_local BatchCtx g_bc;
void bc_check(const void *p, const char *what);   // throws when p is outside [lo, hi)
// Device-to-device copy of `bytes` at dst from src, for every instance of the class.
void copy_d2d(void *dst, const void *src, size_t bytes, hipStream_t s);
#define SPG_BC(p) ::spg::bc_check((const void *)(p), #p)

template <class T>
__device__ __forceinline__ T *inst_ptr(T *p, long ist) {
  return p ? (T *)((const char *)p + (long)blockIdx.y * ist) : p;
}
#define SPG_INST(p) p = ::spg::inst_ptr(p, ist)

// ---- device buffers -------------------------------------------------------
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  bool owned = true;      // false: a view into another allocation (never grows)
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void ensure(size_t n);  // grows (contents lost), zero-filled on growth (device-synchronous)
  void release();
  void view(void *q, size_t n) {  // point at memory owned elsewhere
    release();
    p = q;
    bytes = n;
    owned = false;
  }
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// Maximum sketch width of the truncated SVD (chi + oversample).
constexpr int kMaxSketch = 96;
constexpr int kMaxChi = 80;

// ---- linear algebra kernels (k_linalg.hip) --------------------------------
// C[b1,b2](i,j) = alpha * sum_k A[b1,b2](i,k) B[b1,b2](k,j) + beta * C[b1,b2](i,j)
struct GemmDesc {
  int M, N, K, nb1, nb2;
  const double *A; long a_i, a_k, a_b1, a_b2;
  const double *B; long b_k, b_j, b_b1, b_b2;
  double *C; long c_i, c_j, c_b1, c_b2;
  double alpha, beta;
  double *ws = nullptr;   // optional split-K workspace (ws_len doubles)
  size_t ws_len = 0;
  int kmax = 0;           // internal: global K bound of split-K chunks (0 = K)
  long ist = 0;           // internal: class-batched instance stride (bytes)
  // optional epilogue factor (the MPO site weights w(x) V(x, y)), d = sd:
  // smode 1: C(i, j) of batch b1 times w[i % d] V[(i % d) d + b1];
  // smode 2: every C(i, j) of batch (b1, b2) times w[b1] V[b1 d + b2];
  // smode 3: C(i, j) of batch (b1, b2) times V[b2 d + i % d];
  // smode 4: C(i, j) of batch (b1, b2) times V[(i % d) d + b2] (w unused)
  const double *sw = nullptr, *sV = nullptr;
  int sd = 0, smode = 0;
  int tile = 0;           // output tile 32 or 64 for this product (0: the tuning's)
  int b1_base = 0;        // internal: first batch index b1 of a launch (the epilogue's)
  const char *cls = nullptr;   // kernel class of the launch's timer (null: gemm_f64)
};
void gemm_f64(const GemmDesc &g, hipStream_t s);

// Launch-shape choices read when work is enqueued (set per instance by the
// batch driver and its autotuner; process default 32 / split-K on).
struct Tuning {
  int gemm_tile = 32;   // GEMM output tile: 32 or 64
  int splitk = 1;       // deterministic split-K for skinny long-K products
  int mpo_cols = 1;     // column forms of the MPO d-index contractions (d in {8, 16, 24, 32})
  int qform_split = 1;  // Q of one-panel register QRs by k_qform (a compute unit per column)
  int gemm_f32 = 0;     // FP64 GEMMs with FP32 products and accumulation (reduced precision)
};
extern thread_local Tuning g_tune;

// Householder QR of an m x n matrix (m >= n, n <= kMaxSketch), element (i,j) at
// X[i*xr + j*xc].  Writes Q (m x n, orthonormal columns) to Q[i*qr + j*qc]
// unless Q == nullptr and, if R != nullptr, the n x n upper-triangular factor
// to R[i*n + j] (row-major).  Panels of at most 80 columns are factored in
// registers, by TSQR over blocks of 512 rows beyond that (recursing on the
// stacked R factors); wider ones in LDS (one level of TSQR beyond it) or in
// global memory.  `work` holds qr_work_doubles(m, n) doubles.
size_t qr_work_doubles(int m, int n);
void qr_f64(int m, int n, const double *X, long xr, long xc, double *Q, long qr, long qc,
            double *R, double *work, hipStream_t s);

// One-sided Jacobi SVD of an l x l matrix (row-major, l <= kMaxSketch): writes
// the right singular vectors as columns of V (row-major l x l) sorted by
// singular value, descending (ties by index), and the singular values to sig.
// The leading kk columns are orthonormal to 1e-13 (re-orthonormalised with a
// deterministic completion where columns at the rounding floor failed); the
// others are the normalised Jacobi columns and need not be orthonormal.
void jacobi_svd_f64(int l, int kk, const double *Rm, double *V, double *sig, hipStream_t s);

// Sketch matrix of the truncated SVD: Om[i*l + j] = 2 u(SplitMix64(seed, i*ld + j)) - 1.
void fill_sketch(int n, int l, double *Om, hipStream_t s);

// Frobenius norm of a 4-index box (n0,n1,n2,n3 with strides) -> scales the box
// by 1/norm and writes logs[out] = logs[in] + log(norm) (in < 0 means 0).
// `scratch` holds kNormScratch doubles.
constexpr int kNormScratch = 1040;
void normalize_box(double *T, int n0, int n1, int n2, int n3, long s0, long s1, long s2,
                   long s3, double *logs, int out, int in, double *scratch, hipStream_t s);
void fill_zero(double *p, size_t n, hipStream_t s);
void copy_doubles(double *dst, const double *src, size_t n, hipStream_t s);

// ---- boundary-MPS contraction kernels (k_bmps.hip) -------------------------
struct RowFactors {         // device d x d tables (row-major) / d vectors of one column
  const double *w;          // w_c(x)
  const double *V;          // V_c[x][y]
  const double *Hl, *Dl, *Al;  // H_{c-1}[a][x], D_{c-1}[a][y], A_{c-1}[x][e]
  const double *ones;          // d x d ones (an epilogue factor of 1 per row)
};
// Each column's MPO tensor scaled to a largest entry of 1: W_loc[r][c][.] is
// divided in place by that entry (its log to lsc[r * C + c]), and row_lsc[r]
// receives the sum of the row's logs.  Products of tables that are each at
// most 1 fall far below 1 where the tables peak apart; this keeps the blocks
// of the contraction from underflowing.
void site_scales(int R, int C, int d, double *W_loc, const double *W_h, const double *W_v,
                 const double *W_d, const double *W_a, double *lsc, double *row_lsc,
                 hipStream_t s);
// The bottom row's boundary function written exactly (bond d, x_c on the
// bond): all C padded site tensors of the row at A.  w = W_loc of the row,
// H = W_h of the row.
void bottom_row(int C, int d, int chi, const double *w, const double *H, double *A,
                hipStream_t s);
void init_guess(int d, int chi, int bl, int br, const double *psi, const RowFactors &f,
                double *phi, hipStream_t s);
// P[p][x][y][Q] = w(x)V(x,y) sum_{q,a,e} EL[p][a][e][q] Hl(a,x)Dl(a,y)Al(x,e) psi[q][y][Q]
void left_part(int d, int chi, int pl, int ql, int qr, const double *EL, const double *psi,
               const RowFactors &f, double *T1, double *P, hipStream_t s);
void env_left(int d, int chi, int pl, int pr, int qr, const double *phi, const double *P,
              double *ELn, hipStream_t s);
void env_right(int d, int chi, int pl, int pr, int ql, int qr, const double *phi,
               const double *psi, const double *ER, const RowFactors &f, double *G1,
               double *G2, double *ERn, hipStream_t s);
void two_site_block(int d, int chi, int pl, int ql, int qm, int qr, int pr, const double *EL,
                    const double *ER, const double *psi0, const double *psi1,
                    const RowFactors &f0, const RowFactors &f1, double *T1, double *P,
                    double *Qr, double *P2, double *Q2, double *B, hipStream_t s);
// The whole padded site dst[chi][d][chi]: src[k*sk + (z*pr + P)*sj] for k < nk,
// z < d, P < pr, zero elsewhere.
void unpack_right(int d, int chi, int nk, int pr, const double *src, long sk, long sj,
                  double *dst, hipStream_t s);
void lq_fold(int d, int chi, int bl, int k, const double *R, double *phi_prev, double *tmp,
             hipStream_t s);
void add_logs(double *logs, int out, int a, int b, int c, hipStream_t s);
// dst[k*(d*pr) + z*pr + P] = src[(k*d + z)*chi + P]  (padded MPS site -> compact rows)
void pack_right(int d, int chi, int nk, int pr, const double *src, double *dst, hipStream_t s);
void build_weights(int ntab, int tsize, double beta, const double *E, double *W, double *mins,
                   hipStream_t s);
void set_e0(int n, int chi, double *p, long stride, hipStream_t s);
// p[n][n] = identity (row-major, leading dimension n)
void set_identity(int n, double *p, hipStream_t s);

// ---- search kernels (k_search.hip) ----------------------------------------
struct SearchTabs {         // device tables of the instance
  int rows, cols, d, chi, kings;
  double beta;
  const double *E_loc, *E_h, *E_v, *E_d, *E_a;
  const double *W_v, *W_d, *W_a;
};
inline void bc_check_tabs(const SearchTabs &t) {
  SPG_BC(t.E_loc); SPG_BC(t.E_h); SPG_BC(t.E_v); SPG_BC(t.E_d); SPG_BC(t.E_a);
  SPG_BC(t.W_v); SPG_BC(t.W_d); SPG_BC(t.W_a);
}
// Throws when a launch that has no class-batched form runs inside a class.
void bc_single(const char *what);
// cl, cr: actual bond dimensions left / right of column c (work accounting only)
// scale (optional): scale[a * sstride] receives the max-normalisation divisor
void right_env_col(const SearchTabs &t, int r, int c, int n_anc, const uint8_t *cfg, int N,
                   const double *A_rc, const double *Rnext, double *Rout, long rstride,
                   int cl, int cr, hipStream_t s, double *scale = nullptr, int sstride = 0);
void marginals(const SearchTabs &t, int r, int c, int n_beam, const uint8_t *cfg, int N,
               const double *A_rc, const double *L, const int32_t *anc, const double *Rv,
               long rstride, const double *score, double *out, int add_score, int cl, int cr,
               hipStream_t s);
// n_dev (optional): the count is read on the device (n_cand bounds it);
// cid (optional): candidate ids (default: position); sel_score (optional):
// the selected scores in selection order.
void select_topm(int n_cand, int M, const double *cand, int32_t *sel, uint64_t *keys_work,
                 int32_t *ids_work, hipStream_t s, const int *n_dev = nullptr,
                 const int32_t *cid = nullptr, double *sel_score = nullptr,
                 void *big_ws = nullptr, long ws_cap = 0, const double *vref = nullptr);
// big_ws (optional, select_ws_bytes(ws_cap) bytes, ws_cap >= n_cand, zero-filled
// when allocated): more than 16384 candidates of one instance are selected by a
// gap histogram over many workgroups and a one-workgroup ordering of the
// survivors; vref (optional, device): a score no candidate exceeds, which
// replaces the pass that finds the best one.
size_t select_ws_bytes(long n_cap);
void beam_update(const SearchTabs &t, int r, int c, int n_new, const int32_t *sel, int N,
                 const uint8_t *cfg, const double *energy, const double *L, const int32_t *anc,
                 const double *cand, const double *A_rc, int update_L, uint8_t *cfg_o,
                 double *energy_o, double *score_o, double *L_o, int32_t *anc_o, int cl,
                 int cr, hipStream_t s, const double *sel_score = nullptr);
void beam_reset_row(int n, int chi, double *L, int32_t *anc, hipStream_t s);
// Merging of branches with equal frontiers: workspace (table of `capacity`
// slots, capacity a power of two >= 2 n_beam d; per-child slot and energy key).
struct MergeWork {
  int capacity = 0;
  unsigned long long *tkey = nullptr, *te = nullptr, *ekey = nullptr;
  int32_t *tid = nullptr, *slot = nullptr;
  // droplets (all null without): per slot the next member in (energy, id)
  // order, per child the id of its group's runner-up if it is kept, else -1
  unsigned long long *te2 = nullptr;
  int32_t *tid2 = nullptr, *run = nullptr;
};
// Children of equal frontier: all but the lowest-energy one (ties: lowest id)
// get cand = -inf; with mw.run, run[kept id] = id of the group's runner-up.
void merge_branches(const SearchTabs &t, int r, int c, int n_beam, const uint8_t *cfg, int N,
                    const double *energy, double *cand, MergeWork &mw, hipStream_t s);
// Droplet lists of the n_new survivors sel[] of step (r, c): each inherits its
// parent's list (configurations [D][N] bytes, gaps [D], count) with the new
// site set to its own state, then takes its group's runner-up run[sel[j]] if
// the gap is <= ecut, the runner-up differs from the survivor and from every
// droplet it holds in more than hcut sites, and fewer than D are held.
void droplet_update(const SearchTabs &t, int r, int c, int n_new, const int32_t *sel, int N,
                    const uint8_t *cfg, const double *energy, const int32_t *run,
                    const uint8_t *din, const double *dein, const int32_t *dnin, uint8_t *dout,
                    double *deout, int32_t *dnout, int D, double ecut, int hcut, hipStream_t s);
void final_sort(const SearchTabs &t, int n, int N, const uint8_t *cfg, const double *score,
                int32_t *states_out, double *energies_out, double *logp_out, double *e_work,
                int32_t *perm_work, int32_t *n_valid, hipStream_t s);
void apply_cutoff(int n, double log_cut, double *cand, hipStream_t s,
                  const int *n_dev = nullptr);
void cfg_from_i32(int n, int N, const int32_t *src, uint8_t *dst, hipStream_t s);
void advance_L(const SearchTabs &t, int r, int c, int n, const uint8_t *cfg, int N,
               const double *A_rc, double *L, double *tmp, hipStream_t s);

// ---- learned proposal and guarded steps (k_propose.hip, k_mlp.hip) --------
// Device workspace of the guarded search steps.
struct GuideWork {
  uint16_t *bins;           // [n_beam][d] gap bin of each child
  unsigned *hist;           // [2048] bin counts (cleared by each step)
  int *jstar, *n_list;      // last bin of the candidate set; list length
  double *lkey;             // [n_beam * d] list scores
  int32_t *lid;             // [n_beam * d] list ids b * d + s
  double *bound, *tau;      // [n_beam] bound of unevaluated children; M-th list score
  int32_t *off, *cnt;       // [n_beam] list offset and size of each parent's candidates
  unsigned long long *stats;  // [3] exact evaluations, (unused), fallback parents
};
// sf [rows*cols][d][2]: parent-independent features; rscr [rows][cols+1][chi]
void site_features(const SearchTabs &t, const double *A, float *sf, double *rscr,
                   hipStream_t s);
// Features ([n_beam][d][F], optional) and, when bins/hist are given, the gap
// bins of score_b + log p^(s|b) below *smax counted into hist.
void propose(const SearchTabs &t, int r, int c, int n_beam, const uint8_t *cfg, int N,
             const double *score, const double *smax, const float *sf, const float *prm, int H,
             float *feat_out, uint16_t *bins, unsigned *hist, hipStream_t s);
// Candidate threshold, exact weights on the set, guard and fallback; leaves
// the step's list (lkey, lid, *n_list) for the top-M selection.
void guided_step(const SearchTabs &t, int r, int c, int n_beam, int M, int K, const uint8_t *cfg,
                 int N, const double *A_rc, const double *L, const int32_t *anc, const double *Rv,
                 long rstride, const double *Rsc, const double *score, GuideWork &g, int cl,
                 int cr, hipStream_t s);
// The same guarded step on a reduced-precision env: exact weights from the
// column's U products and FP32 L (the plain reduced-precision search's
// arithmetic), Z_b = Rsc * (L^b . R_c) with R_c in the env's precision; the
// guard's relative floor and margin are those of that precision.
void guided_step_lp(const SearchTabs &t, int precision, int r, int c, int n_beam, int M, int K,
                    const uint8_t *cfg, int N, const float *U, long ldu, const float *L,
                    const int32_t *anc, const float *Rf, long rstride, const double *Rsc,
                    const double *score, GuideWork &g, int cl, hipStream_t s);
void max_of(int n, const double *v, double *out, hipStream_t s);
// Network evaluation and training (k_mlp.hip); deterministic reductions.
void mlp_forward(int n_beam, int d, const float *feats, const float *prm, int H, float *logp,
                 hipStream_t s);
// grad [P] and loss [1] of the mean cross-entropy; partial holds
// mlp_partial_floats(H) floats; loss_acc (optional) += loss.
size_t mlp_partial_floats(int H);
void mlp_loss_grad(int n_beam, int d, const float *feats, const float *target, const float *prm,
                   int H, float *partial, float *grad, float *loss, float *loss_acc,
                   hipStream_t s);
void mlp_adam(int P, float *prm, float *m, float *v, const float *grad, float lr, float bc1,
              float bc2, hipStream_t s);
void to_float(long n, const double *src, float *dst, hipStream_t s);

// ---- reduced-precision search contractions (k_search_lp.hip) --------------
// precision: SPG_FP32 (A in FP32) or SPG_BF16 (A in BF16); vectors L, R FP32.
void lp_convert(long n, const double *src, void *dst, int precision, hipStream_t s);
void lp_set_e0(int n, int chi, float *p, long stride, hipStream_t s);
// U[a][al * d + s] = sum_b R^a[b] A_rc[al][s][b] for every ancestor (MFMA GEMM;
// U rows of stride ldu >= cl * d).
void lp_u_col(const SearchTabs &t, int precision, int n_anc, const void *A_rc,
              const float *Rnext, long rstride, float *U, long ldu, int cl, int cr,
              hipStream_t s);
// R^a_c from U and the couplings to the fixed row (normalised per ancestor).
// FP64 search from per-ancestor products (matrix cores): U^a[al*d + s] =
// sum_b A_c[al][s][b] R^a_{c+1}[b] for every row-start ancestor (one GEMM,
// row stride ldu), the right environment R_c and the conditionals from U.
void u64_col(int n_anc, const double *A_rc, int chi, const double *Rnext, long rstride,
             double *U, long ldu, int d, int cl, int cr, hipStream_t s);
void env_from_u64(const SearchTabs &t, int r, int c, int n_anc, const uint8_t *cfg, int N,
                  const double *U, long ldu, double *Rout, long rstride, int cl, hipStream_t s,
                  double *scale = nullptr, int sstride = 0);
void marg_from_u64(const SearchTabs &t, int r, int c, int n_beam, const uint8_t *cfg, int N,
                   const double *U, long ldu, const double *L, const int32_t *anc,
                   const double *score, double *out, int add_score, int cl, hipStream_t s);
// sc (optional): the normalisation m of each ancestor's R_c, at sc[a * sc_stride]
void lp_env_from_u(const SearchTabs &t, int precision, int r, int c, int n_anc,
                   const uint8_t *cfg, int N, const float *U, long ldu, float *Rout, long rstride,
                   int cl, hipStream_t s, double *sc = nullptr, long sc_stride = 0);
// Conditionals of every beam state from U of its ancestor and its L.
void lp_marginals_u(const SearchTabs &t, int r, int c, int n_beam, const uint8_t *cfg, int N,
                    const float *U, long ldu, const float *L, const int32_t *anc,
                    const double *score, double *out, int add_score, int cl, hipStream_t s);
void lp_beam_update(const SearchTabs &t, int precision, int r, int c, int n_new,
                    const int32_t *sel, int N, const uint8_t *cfg, const double *energy,
                    const float *L, const int32_t *anc, const double *cand, const void *A_rc,
                    int update_L, uint8_t *cfg_o, double *energy_o, double *score_o, float *L_o,
                    int32_t *anc_o, int cl, int cr, hipStream_t s,
                    const double *sel_score = nullptr);
void lp_advance_L(const SearchTabs &t, int precision, int r, int c, int n, const uint8_t *cfg,
                  int N, const void *A_rc, float *L, hipStream_t s);

}  // namespace spg

// ---- opaque handles ---------------------------------------------------------
struct spg_peps {
  int rows = 0, cols = 0, d = 0, kings = 0;
  double beta = 0, shift = 0;
  int device = 0;
  spg::DevBuf E_loc, E_h, E_v, E_d, E_a;   // energies (zero tables for absent classes)
  spg::DevBuf W_loc, W_h, W_v, W_d, W_a;   // Boltzmann weights of the min-shifted tables
                                           // (W_loc divided by the site scales below)
  spg::DevBuf row_lsc;                     // [rows] sum of the log site scales of each row
  spg::DevBuf ones, e0row, e0col, e0vec;   // d x d all-ones, first row / column ones; e_0
};

struct spg_env {
  const spg_peps *peps = nullptr;
  int chi = 0, precision = SPG_FP64;
  std::vector<int32_t> dims;     // [rows][cols+1]
  spg::DevBuf A;                 // [rows][cols][chi][d][chi] float64, zero padded
  spg::DevBuf Alp;               // same tensors in the search precision (FP32 or BF16)
  spg::DevBuf lam;               // [rows] float64 log-scales
  // search workspace (grown on demand)
  spg::DevBuf cfg[2], score[2], energy[2], L[2], anc[2], Rv, cand, sel, keys, ids, ework,
      perm, nvalid, tmp, cfg32;
  spg::DevBuf Ulp;               // reduced precision: U_c [cols][M][chi * d] float
  spg::DevBuf U64;               // FP64 search: U_c [cols][M][chi * d] double
  spg::DevBuf selws;             // multi-workgroup top-M workspace (1280 + 12 M bytes)
  // guarded search with a proposal: right-environment scales, per-site
  // features, step workspace and counters
  spg::DevBuf Rsc, sf, rscr, gbins, ghist, gint, glkey, glid, gbound, gtau, goff, gcnt, gstats,
      selscore, smax;
  spg::DevBuf mkey, me, mid, mslot, mekey;   // merging branches
  spg::DevBuf me2, mid2, mrun;               // runner-ups of merged groups
  // droplets [M][D][N] bytes, gaps [M][D], counts [M], double-buffered like
  // the beam; after a search with droplets: the buffer holding them, the
  // number of final beam slots and D
  spg::DevBuf dcfg[2], dde[2], dn[2];
  int drop_buf = -1, drop_slots = 0, drop_cap = 0;
  int64_t last_stats[3] = {0, 0, 0};
};

struct spg_proposal {
  int H = 0;
  int64_t t = 0;                 // Adam steps taken
  spg::DevBuf prm, m, v, grad, partial, loss;
};
