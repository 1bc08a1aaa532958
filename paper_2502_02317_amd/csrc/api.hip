// C ABI of include/spg.h: argument validation, device buffers and the
// sequencing of the kernels on the caller's stream.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>

#include "mlp_dev.h"
#include "spg_internal.h"

namespace spg {

thread_local std::string g_err;
void set_error(const std::string &m) { g_err = m; }

// Per-launch timing: when enabled, every timed launch records a start and a
// stop event on its own stream; queries synchronise on the stop events.
struct TimerRec {
  const char *name;
  hipEvent_t a, b;
  double work;
};
static bool g_prof = false;
static std::vector<TimerRec> g_recs;
static std::vector<hipEvent_t> g_pool;

static hipEvent_t pool_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  SPG_HIP(hipEventCreate(&e));
  return e;
}

KTimer::KTimer(const char *name, hipStream_t st, double work) {
  if (!g_prof) return;
  s = st;
  TimerRec r{name, pool_event(), pool_event(), work * g_bc.n};
  SPG_HIP(hipEventRecord(r.a, s));
  g_recs.push_back(r);
  slot = (int)g_recs.size() - 1;
}

KTimer::~KTimer() {
  if (slot >= 0) (void)hipEventRecord(g_recs[slot].b, s);
}

thread_local BatchCtx g_bc;

void bc_check(const void *p, const char *what) {
  if (g_bc.n <= 1 || p == nullptr) return;
  const char *c = (const char *)p;
  if (c < g_bc.lo || c >= g_bc.hi) {
    set_error(std::string("class-batched launch with a pointer outside the instance slice: ") +
              what);
    throw Fail{SPG_ERR_INVALID};
  }
}

void copy_d2d(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  if (g_bc.n <= 1) {
    SPG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
    return;
  }
  SPG_BC((const char *)dst + bytes - 1);
  SPG_BC((const char *)src + bytes - 1);
  // one copy per instance by a kernel of our own (instance offsets in 64 bits)
  copy_doubles((double *)dst, (const double *)src, bytes / sizeof(double), s);
}

void bc_single(const char *what) {
  if (g_bc.n > 1) {
    set_error(std::string(what) + " has no class-batched form");
    throw Fail{SPG_ERR_UNSUPPORTED};
  }
}

void DevBuf::ensure(size_t n) {
  if (n <= bytes) return;
  if (!owned) {
    set_error("a buffer view cannot grow");
    throw Fail{SPG_ERR_INVALID};
  }
  release();
  if (hipMalloc(&p, n) != hipSuccess) {
    p = nullptr;
    bytes = 0;
    (void)hipGetLastError();
    set_error("device allocation of " + std::to_string(n) + " bytes failed");
    throw Fail{SPG_ERR_OOM};
  }
  bytes = n;
  SPG_HIP(hipMemset(p, 0, n));
  SPG_HIP(hipDeviceSynchronize());
}

void DevBuf::release() {
  if (p && owned) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
  owned = true;
}

static int fail(int code, const std::string &m) {
  set_error(m);
  return code;
}

#define SPG_TRY try {
#define SPG_CATCH                                                  \
  }                                                                \
  catch (const ::spg::Fail &f) { return f.code; }                  \
  catch (const std::bad_alloc &) {                                 \
    ::spg::set_error("host allocation failed");                    \
    return SPG_ERR_OOM;                                            \
  }

// ---------------------------------------------------------------------------
// Boundary MPS workspace: one per call of spg_boundary_mps, one per stream of a
// batch (instances on one stream run in order and share it).
struct BmpsWork {
  int R, C, d, chi, lmax;
  DevBuf EL, ER, T1, P, Qr, P2, Q2, G1, G2, B, Y, Q, Z, Qz, Om, Cm, Qc, Rc, V, sig, U, Rm,
      qrwork, tmp, logs, psi0, nscr, ident, skws;
  size_t env_sz() const { return (size_t)chi * d * d * chi; }
  size_t site_sz() const { return (size_t)chi * d * chi; }
  double *ELc(int c) { return EL.as<double>() + (size_t)c * env_sz(); }
  double *ERc(int c) { return ER.as<double>() + (size_t)c * env_sz(); }
  // every buffer with its size in bytes for the current shape
  template <class F>
  void each(F &&f) {
    const size_t es = env_sz() * sizeof(double);
    f(EL, es * (C + 1));
    f(ER, es * (C + 1));
    f(T1, 2 * es);
    for (DevBuf *b : {&P, &Qr, &P2, &Q2, &G1, &G2}) f(*b, es);
    const size_t mn = (size_t)chi * d;                  // max rows / cols of a two-site block
    f(B, mn * mn * sizeof(double));
    const size_t ml = mn * lmax * sizeof(double);
    for (DevBuf *b : {&Y, &Q, &Z, &Qz, &Om, &Qc, &Cm, &U, &Rm}) f(*b, ml);
    f(Rc, (size_t)lmax * lmax * sizeof(double));
    f(V, (size_t)lmax * lmax * sizeof(double));
    f(sig, (size_t)lmax * sizeof(double));
    f(qrwork, qr_work_doubles((int)mn, lmax) * sizeof(double));
    f(nscr, kNormScratch * sizeof(double));
    f(ident, (size_t)lmax * lmax * sizeof(double));
    f(skws, 16 * mn * lmax * sizeof(double));
    f(tmp, site_sz() * sizeof(double));
    f(logs, (size_t)(2 * C + 8 + 2 * R) * sizeof(double));
    f(psi0, site_sz() * C * sizeof(double));
  }
  void alloc() {
    each([](DevBuf &b, size_t n) { b.ensure(n); });
  }
};

// Rank-kk split of an m x n matrix view B (element (i,j) at B[i*br + j*bc]):
// U (m x kk, orthonormal columns) written at U[i*ur + j*uc].  Randomised range
// finder with q power iterations, sketch width l = min(k+p, m, n), then the
// SVD of the projected l x n matrix (QR of its transpose + one-sided Jacobi).
static int tsvd_left(BmpsWork &w, const double *B, long br, long bc, int m, int n, int k, int p,
                     int q, double *U, long ur, long uc, hipStream_t s) {
  const int l = std::min(std::min(k + p, m), n);
  const int kk = std::min(k, l);
  double *Om = w.Om.as<double>(), *Y = w.Y.as<double>(), *Q = w.Q.as<double>();
  double *Z = w.Z.as<double>(), *Qz = w.Qz.as<double>(), *Cm = w.Cm.as<double>();
  auto mm = [&](int M, int N, int K, const double *A, long ai, long ak, const double *Bp, long bk,
                long bj, double *Cp, long ci, long cj) {
    GemmDesc g{};
    g.M = M; g.N = N; g.K = K; g.nb1 = 1; g.nb2 = 1;
    g.A = A; g.a_i = ai; g.a_k = ak;
    g.B = Bp; g.b_k = bk; g.b_j = bj;
    g.C = Cp; g.c_i = ci; g.c_j = cj;
    g.alpha = 1.0; g.beta = 0.0;
    g.ws = w.skws.as<double>(); g.ws_len = w.skws.bytes / sizeof(double);
    if ((long)M * N >= (1L << 20)) g.tile = 64;   // the large products at many states per site
    gemm_f64(g, s);
  };
  double *qw = w.qrwork.as<double>();
  // the range-finder panels Y, Z, Q, Qz are column-major (the QR reads and
  // writes them straight from registers)
  mm(m, l, n, B, br, bc, Om, w.lmax, 1, Y, 1, m);            // Y = B Om (Om: stride lmax)
  qr_f64(m, l, Y, 1, m, Q, 1, m, nullptr, qw, s);           // Q = orth(Y)
  for (int it = 0; it < q; ++it) {
    mm(n, l, m, B, bc, br, Q, 1, m, Z, 1, n);                // Z = B^T Q
    qr_f64(n, l, Z, 1, n, Qz, 1, n, nullptr, qw, s);
    mm(m, l, n, B, br, bc, Qz, 1, n, Y, 1, m);               // Y = B Qz
    qr_f64(m, l, Y, 1, m, Q, 1, m, nullptr, qw, s);
  }
  if (l == kk) {
    // sketch width = kept rank: U U^T B only depends on span(Q), so U = Q
    mm(m, kk, l, Q, 1, m, w.ident.as<double>(), w.lmax, 1, U, ur, uc);
    return kk;
  }
  mm(l, n, m, Q, m, 1, B, br, bc, Cm, n, 1);                 // Cm = Q^T B   (l x n)
  qr_f64(n, l, Cm, 1, n, nullptr, l, 1, w.Rc.as<double>(), qw, s);  // Cm^T = Qc Rc (R only)
  jacobi_svd_f64(l, kk, w.Rc.as<double>(), w.V.as<double>(), w.sig.as<double>(), s);
  mm(m, kk, l, Q, 1, m, w.V.as<double>(), l, 1, U, ur, uc);  // U = Q V[:, :kk]
  return kk;
}

// ---------------------------------------------------------------------------
static void row_factors(const spg_peps *pp, int r, int c, bool bottom, RowFactors &f) {
  const int C = pp->cols, d = pp->d;
  const size_t dd = (size_t)d * d;
  f.w = pp->W_loc.as<double>() + ((size_t)r * C + c) * d;
  f.V = bottom ? pp->ones.as<double>() : pp->W_v.as<double>() + ((size_t)r * C + c) * dd;
  f.ones = pp->ones.as<double>();
  if (c == 0) {
    f.Hl = pp->e0row.as<double>();
    f.Dl = pp->e0row.as<double>();
    f.Al = pp->e0col.as<double>();
  } else {
    f.Hl = pp->W_h.as<double>() + ((size_t)r * (C - 1) + c - 1) * dd;
    f.Dl = bottom ? pp->ones.as<double>() : pp->W_d.as<double>() + ((size_t)r * (C - 1) + c - 1) * dd;
    f.Al = bottom ? pp->ones.as<double>() : pp->W_a.as<double>() + ((size_t)r * (C - 1) + c - 1) * dd;
  }
}

static int bmps_lmax(int chi, int d, const spg_mps_params *prm) {
  return std::min(chi + std::max(prm->oversample, 0), chi * d);
}

// Enqueues the contraction on s with workspace w (sized beforehand when the
// call is captured into a graph: growing it allocates and synchronises).
static void boundary_mps_fp64(spg_env *env, const spg_mps_params *prm, hipStream_t s,
                              BmpsWork &w) {
  const spg_peps *pp = env->peps;
  const int R = pp->rows, C = pp->cols, d = pp->d, chi = env->chi;
  w.R = R; w.C = C; w.d = d; w.chi = chi;
  w.lmax = bmps_lmax(chi, d, prm);
  w.alloc();
  const size_t site = w.site_sz(), es = w.env_sz();
  set_identity(w.lmax, w.ident.as<double>(), s);
  // the sketch table, Om[i*lmax + j] for every two-site block of this contraction
  fill_sketch(chi * d, w.lmax, w.Om.as<double>(), s);
  double *A = env->A.as<double>();
  double *logs = w.logs.as<double>();
  // log slots: EL[c] at c, ER[c] at C+1+c, centre at 2C+2, lam[r] at 2C+4+r,
  // the rows' site scales at 2C+8+R+r
  const int sEL = 0, sER = C + 1, sCen = 2 * C + 2, sLam = 2 * C + 4, sRsc = 2 * C + 8 + R;
  fill_zero(logs, (size_t)(2 * C + 8 + 2 * R), s);
  copy_d2d(logs + sRsc, pp->row_lsc.as<double>(), sizeof(double) * R, s);
  // E~_rows = 1 through the state y = 0 of a bond-1 product MPS
  fill_zero(w.psi0.as<double>(), site * C, s);
  for (int c = 0; c < C; ++c) set_e0(1, 1, w.psi0.as<double>() + c * site, 1, s);
  // trivial environments: EL[0] and ER[C] (p = q = 0, all (a, e) / (x, y) for ER)
  fill_zero(w.ELc(0), es, s);
  set_e0(1, 1, w.ELc(0), 1, s);
  fill_zero(w.ERc(C), es, s);
  set_e0(d * d, 1, w.ERc(C), chi, s);                        // ER[0][x][y][0] = 1
  std::vector<int> pdims(C + 1, 1), fdims(C + 1, 1);
  for (int r = R - 1; r >= 0; --r) {
    const bool bottom = (r == R - 1);
    const double *psi = bottom ? w.psi0.as<double>() : A + (size_t)(r + 1) * C * site;
    double *phi = A + (size_t)r * C * site;
    if (bottom && chi >= d) {
      // the bottom row is a chain of nearest-neighbour factors: written exactly
      // at bond d (nothing to fit; a fit would keep chi > d directions at its
      // inner cuts, those beyond the exact rank d weightless and completed
      // differently by every implementation); lam = sum of the tensors' log-norms
      bottom_row(C, d, chi, pp->W_loc.as<double>() + (size_t)r * C * d,
                 pp->W_h.as<double>() + (size_t)r * (C - 1) * d * d, phi, s);
      for (int c = 0; c < C; ++c) {
        const int bl = (c == 0) ? 1 : d, br = (c == C - 1) ? 1 : d;
        normalize_box(phi + c * site, bl, d, br, 1, (long)d * chi, chi, 1, 1, logs, sLam + r,
                      c == 0 ? -1 : sLam + r, w.nscr.as<double>(), s);
      }
      add_logs(logs, sLam + r, sLam + r, sRsc + r, -1, s);   // + the site scales
      for (int c = 0; c <= C; ++c) env->dims[r * (C + 1) + c] = (c == 0 || c == C) ? 1 : d;
      continue;
    }
    if (bottom) std::fill(pdims.begin(), pdims.end(), 1);
    else for (int c = 0; c <= C; ++c) pdims[c] = env->dims[(r + 1) * (C + 1) + c];
    std::vector<RowFactors> f(C);
    for (int c = 0; c < C; ++c) row_factors(pp, r, c, bottom, f[c]);
    // initial guess phi_c[x] = w_c(x) sum_y V_c(x,y) psi_c[y], then right-canonical form
    fill_zero(phi, site * C, s);
    for (int c = 0; c < C; ++c) init_guess(d, chi, pdims[c], pdims[c + 1], psi + c * site, f[c], phi + c * site, s);
    fdims = pdims;
    for (int c = C - 1; c >= 1; --c) {
      const int bl = fdims[c], br = fdims[c + 1];
      double *Mc = w.Cm.as<double>();                           // compact bl x (d*br)
      pack_right(d, chi, bl, br, phi + c * site, Mc, s);
      // QR of Mc^T (d*br x bl): Q -> new right isometry, R folded into phi_{c-1}
      qr_f64(d * br, bl, Mc, 1, (long)d * br, w.Qc.as<double>(), 1, (long)d * br,
             w.Rc.as<double>(), w.qrwork.as<double>(), s);                 // Q column-major
      unpack_right(d, chi, bl, br, w.Qc.as<double>(), (long)d * br, 1, phi + c * site, s);
      lq_fold(d, chi, bl, bl, w.Rc.as<double>(), phi + (c - 1) * site, w.tmp.as<double>(), s);
      // the folded factor only carries the guess's scale, which no later step
      // uses (phi_0 and phi_1 are overwritten before they are read): unit norm,
      // so that it cannot overflow over many columns (its log is discarded)
      normalize_box(phi + (c - 1) * site, fdims[c - 1], d, bl, 1, (long)d * chi, chi, 1, 1, logs,
                    sCen, -1, w.nscr.as<double>(), s);
    }
    auto build_ER = [&](int c) {
      env_right(d, chi, fdims[c], fdims[c + 1], pdims[c], pdims[c + 1], phi + c * site,
                psi + c * site, w.ERc(c + 1), f[c], w.G1.as<double>(), w.G2.as<double>(),
                w.ERc(c), s);
      normalize_box(w.ERc(c), fdims[c], d, d, pdims[c], (long)d * d * chi, (long)d * chi, chi, 1,
                    logs, sER + c, sER + c + 1, w.nscr.as<double>(), s);
    };
    auto build_EL = [&](int c) {
      left_part(d, chi, fdims[c], pdims[c], pdims[c + 1], w.ELc(c), psi + c * site, f[c],
                w.T1.as<double>(), w.P.as<double>(), s);
      env_left(d, chi, fdims[c], fdims[c + 1], pdims[c + 1], phi + c * site, w.P.as<double>(),
               w.ELc(c + 1), s);
      normalize_box(w.ELc(c + 1), fdims[c + 1], d, d, pdims[c + 1], (long)d * d * chi,
                    (long)d * chi, chi, 1, logs, sEL + c + 1, sEL + c, w.nscr.as<double>(), s);
    };
    // two-site update at (c, c+1); right = true: centre moves left (phi_c = U S,
    // phi_{c+1} = V^T).  A side with at most chi rows (left split) or columns
    // (right split) needs no truncation and keeps its natural basis (no rotation
    // of the non-negative block); natural_left: the last update of a sweep,
    // which keeps the natural basis on column 0 whenever it has at most chi
    // rows, phi_1 = B becoming the centre.  Returns true when phi_{c+1} is the
    // centre.
    auto copy_strided = [&](int M, int N, const double *src, long si, double *dst, long di) {
      GemmDesc g{};                              // dst = src I: exact copy by the GEMM
      g.nb1 = 1; g.nb2 = 1; g.alpha = 1.0; g.beta = 0.0;
      g.ws = w.skws.as<double>(); g.ws_len = w.skws.bytes / sizeof(double);
      g.M = M; g.N = N; g.K = N;
      g.A = src; g.a_i = si; g.a_k = 1;
      g.B = w.ident.as<double>(); g.b_k = w.lmax; g.b_j = 1;
      g.C = dst; g.c_i = di; g.c_j = 1;
      gemm_f64(g, s);
    };
    auto update = [&](int c, bool right, bool natural_left) -> bool {
      const int pl = fdims[c], pr = fdims[c + 2];
      two_site_block(d, chi, pl, pdims[c], pdims[c + 1], pdims[c + 2], pr, w.ELc(c), w.ERc(c + 2),
                     psi + c * site, psi + (c + 1) * site, f[c], f[c + 1], w.T1.as<double>(),
                     w.P.as<double>(), w.Qr.as<double>(), w.P2.as<double>(), w.Q2.as<double>(),
                     w.B.as<double>(), s);
      const int m = pl * d, n = d * pr;
      const int k = std::min(chi, std::min(m, n));
      double *Bm = w.B.as<double>();
      double *phic = phi + c * site, *phin = phi + (c + 1) * site;
      fill_zero(phic, site, s);                    // phi_{c+1} is written whole by unpack_right
      GemmDesc g{};
      g.nb1 = 1; g.nb2 = 1; g.alpha = 1.0; g.beta = 0.0;
      g.ws = w.skws.as<double>(); g.ws_len = w.skws.bytes / sizeof(double);
      int kk;
      bool centre_next = false;
      if ((!right || natural_left) && m <= chi) {
        // natural basis on the left: phi_c = I (m x m), phi_{c+1} = B
        copy_strided(m, m, w.ident.as<double>(), w.lmax, phic, chi);
        unpack_right(d, chi, m, pr, Bm, n, 1, phin, s);
        kk = m;
        centre_next = right;
      } else if (right && n <= chi) {
        // natural basis on the right: phi_{c+1} = I (n x n), phi_c = B
        copy_strided(m, n, Bm, n, phic, chi);
        unpack_right(d, chi, n, pr, w.ident.as<double>(), w.lmax, 1, phin, s);
        kk = n;
      } else if (!right) {
        kk = tsvd_left(w, Bm, n, 1, m, n, k, prm->oversample, prm->power_iters, phic, chi, 1, s);
        // Rm = U^T B (kk x n) -> phi_{c+1}[k][z][P]
        g.M = kk; g.N = n; g.K = m;
        g.A = phic; g.a_i = 1; g.a_k = chi;
        g.B = Bm; g.b_k = n; g.b_j = 1;
        g.C = w.Rm.as<double>(); g.c_i = n; g.c_j = 1;
        gemm_f64(g, s);
        unpack_right(d, chi, kk, pr, w.Rm.as<double>(), n, 1, phin, s);
      } else {
        // tsvd of B^T (n x m): U' (n x kk) -> phi_{c+1} = U'^T;  phi_c = B U'
        double *Up = w.U.as<double>();
        kk = tsvd_left(w, Bm, 1, n, n, m, k, prm->oversample, prm->power_iters, Up, k, 1, s);
        g.M = m; g.N = kk; g.K = n;
        g.A = Bm; g.a_i = n; g.a_k = 1;
        g.B = Up; g.b_k = k; g.b_j = 1;
        g.C = phic; g.c_i = chi; g.c_j = 1;
        gemm_f64(g, s);
        unpack_right(d, chi, kk, pr, Up, 1, k, phin, s);
      }
      fdims[c + 1] = kk;
      return centre_next;
    };
    int last_pair_lam_slot = sER + 2;
    bool centre1 = false;                          // the centre is phi_1 (else phi_0)
    for (int sw = 0; sw < std::max(prm->num_sweeps, 1); ++sw) {
      for (int c = C - 1; c >= 2; --c) build_ER(c);
      for (int c = 0; c <= C - 2; ++c) {
        if (c < C - 2) {
          update(c, false, false);
          build_EL(c);
        } else {
          centre1 = update(c, true, false);
          if (C > 2) build_ER(c + 1);
        }
      }
      for (int c = C - 3; c >= 0; --c) {
        centre1 = update(c, true, c == 0);
        if (c > 0) build_ER(c + 1);
      }
    }
    (void)last_pair_lam_slot;
    // normalise the centre; lam_r = lam_{r+1} + log-scale of ER[2] + log |centre|
    if (centre1)
      normalize_box(phi + site, fdims[1], d, fdims[2], 1, (long)d * chi, chi, 1, 1, logs, sCen,
                    -1, w.nscr.as<double>(), s);
    else
      normalize_box(phi, 1, d, fdims[1], 1, (long)d * chi, chi, 1, 1, logs, sCen, -1,
                    w.nscr.as<double>(), s);
    add_logs(logs, sLam + r, bottom ? -1 : sLam + r + 1, (C > 2) ? sER + 2 : -1, sCen, s);
    add_logs(logs, sLam + r, sLam + r, sRsc + r, -1, s);     // + the site scales
    for (int c = 0; c <= C; ++c) env->dims[r * (C + 1) + c] = fdims[c];
  }
  copy_d2d(env->lam.as<double>(), logs + sLam, sizeof(double) * R, s);
}

// Search copy of the boundary MPS in the env's precision (no-op for FP64).
static void make_lp_copy(spg_env *env, hipStream_t s) {
  if (env->precision == SPG_FP64) return;
  const spg_peps *pp = env->peps;
  const long n = (long)pp->rows * pp->cols * env->chi * pp->d * env->chi;
  env->Alp.ensure((size_t)n * (env->precision == SPG_FP32 ? 4 : 2));
  lp_convert(n, env->A.as<double>(), env->Alp.p, env->precision, s);
}

static size_t lp_elt(const spg_env *env) { return env->precision == SPG_FP32 ? 4 : 2; }

static SearchTabs tabs_of(const spg_env *env) {
  const spg_peps *pp = env->peps;
  SearchTabs t;
  t.rows = pp->rows; t.cols = pp->cols; t.d = pp->d; t.chi = env->chi; t.beta = pp->beta;
  t.kings = pp->kings;
  t.E_loc = pp->E_loc.as<double>(); t.E_h = pp->E_h.as<double>(); t.E_v = pp->E_v.as<double>();
  t.E_d = pp->E_d.as<double>(); t.E_a = pp->E_a.as<double>();
  t.W_v = pp->W_v.as<double>(); t.W_d = pp->W_d.as<double>(); t.W_a = pp->W_a.as<double>();
  return t;
}

static int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

}  // namespace spg

using namespace spg;

extern "C" {

const char *spg_last_error(void) { return g_err.c_str(); }

void spg_profile_enable(int32_t on) { g_prof = (on != 0); }

void spg_profile_reset(void) {
  for (auto &r : g_recs) {
    (void)hipEventSynchronize(r.b);
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
}

int spg_profile_query(const char *name, int64_t *count, double *total_ms, double *total_work) {
  if (!name || !count || !total_ms) return fail(SPG_ERR_INVALID, "spg_profile_query: null argument");
  int64_t n = 0;
  double t = 0.0, wk = 0.0;
  for (auto &r : g_recs) {
    if (std::strcmp(r.name, name) != 0) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(SPG_ERR_HIP, "spg_profile_query: event");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(SPG_ERR_HIP, "spg_profile_query: elapsed");
    ++n;
    t += ms;
    wk += r.work;
  }
  *count = n;
  *total_ms = t;
  if (total_work) *total_work = wk;
  return SPG_OK;
}

// Bytes of each table of a PEPS of this shape, in the order E_loc, E_h, E_v,
// E_d, E_a, W_loc, W_h, W_v, W_d, W_a, ones, e0row, e0col, e0vec, row_lsc
// (what spg_build_peps allocates; e0vec stays empty).
constexpr int kPepsTables = 15;
extern "C++" {
static std::array<size_t, kPepsTables> peps_table_bytes(int R, int C, int d) {
  const size_t dd = (size_t)d * d;
  const size_t n_loc = (size_t)R * C * d, n_h = (size_t)R * (C - 1) * dd;
  const size_t n_v = (size_t)(R - 1) * C * dd, n_x = (size_t)(R - 1) * (C - 1) * dd;
  auto b = [](size_t n) { return std::max<size_t>(n, 1) * sizeof(double); };
  return {b(n_loc), b(n_h), b(n_v), b(n_x), b(n_x), b(n_loc), b(n_h), b(n_v), b(n_x), b(n_x),
          b(dd), b(dd), b(dd), 0, (size_t)R * sizeof(double)};
}
}  // extern "C++"

int spg_build_peps(const spg_instance_desc *desc, void *stream, spg_peps_t **out) {
  SPG_TRY
  if (!desc || !out) return fail(SPG_ERR_INVALID, "spg_build_peps: null desc or out");
  const int R = desc->rows, C = desc->cols, d = desc->d;
  if (R < 1 || C < 2 || d < 2) return fail(SPG_ERR_UNSUPPORTED, "spg_build_peps: need rows >= 1, cols >= 2, d >= 2");
  if (d > 256) return fail(SPG_ERR_UNSUPPORTED, "spg_build_peps: d > 256");
  if ((long)R * C > 65536) return fail(SPG_ERR_UNSUPPORTED, "spg_build_peps: more than 65536 sites");
  if (!std::isfinite(desc->beta) || desc->beta < 0)
    return fail(SPG_ERR_NONFINITE, "spg_build_peps: beta must be finite and >= 0");
  if (!desc->local_E || !desc->pair_E_h || (R > 1 && !desc->pair_E_v))
    return fail(SPG_ERR_INVALID, "spg_build_peps: null energy table");
  if (desc->kings && R > 1 && (!desc->pair_E_d || !desc->pair_E_a))
    return fail(SPG_ERR_INVALID, "spg_build_peps: kings=1 needs pair_E_d and pair_E_a");
  const size_t dd = (size_t)d * d;
  const size_t n_loc = (size_t)R * C * d, n_h = (size_t)R * (C - 1) * dd;
  const size_t n_v = (size_t)(R - 1) * C * dd, n_x = (size_t)(R - 1) * (C - 1) * dd;
  auto finite = [](const double *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(p[i])) return false;
    return true;
  };
  if (!finite(desc->local_E, n_loc) || !finite(desc->pair_E_h, n_h) ||
      (n_v && !finite(desc->pair_E_v, n_v)) ||
      (desc->kings && n_x && (!finite(desc->pair_E_d, n_x) || !finite(desc->pair_E_a, n_x))))
    return fail(SPG_ERR_NONFINITE, "spg_build_peps: non-finite energy");
  hipStream_t s = (hipStream_t)stream;
  spg_peps *pp = new spg_peps();
  try {
    pp->rows = R; pp->cols = C; pp->d = d; pp->kings = desc->kings ? 1 : 0; pp->beta = desc->beta;
    SPG_HIP(hipGetDevice(&pp->device));
    auto up = [&](DevBuf &b, const double *src, size_t n) {
      b.ensure(std::max<size_t>(n, 1) * sizeof(double));
      if (n && src) SPG_HIP(hipMemcpyAsync(b.p, src, n * sizeof(double), hipMemcpyHostToDevice, s));
    };
    up(pp->E_loc, desc->local_E, n_loc);
    up(pp->E_h, desc->pair_E_h, n_h);
    up(pp->E_v, desc->pair_E_v, n_v);
    up(pp->E_d, desc->kings ? desc->pair_E_d : nullptr, n_x);   // zero tables on a square lattice
    up(pp->E_a, desc->kings ? desc->pair_E_a : nullptr, n_x);
    pp->W_loc.ensure(std::max<size_t>(n_loc, 1) * 8); pp->W_h.ensure(std::max<size_t>(n_h, 1) * 8);
    pp->W_v.ensure(std::max<size_t>(n_v, 1) * 8); pp->W_d.ensure(std::max<size_t>(n_x, 1) * 8);
    pp->W_a.ensure(std::max<size_t>(n_x, 1) * 8);
    const size_t ntab = (size_t)R * C + (size_t)R * (C - 1) + (size_t)(R - 1) * C + 2 * (size_t)(R - 1) * (C - 1);
    DevBuf mins;
    mins.ensure(std::max<size_t>(ntab, 1) * 8);
    double *mn = mins.as<double>();
    size_t off = 0;
    build_weights(R * C, d, pp->beta, pp->E_loc.as<double>(), pp->W_loc.as<double>(), mn + off, s); off += (size_t)R * C;
    build_weights(R * (C - 1), (int)dd, pp->beta, pp->E_h.as<double>(), pp->W_h.as<double>(), mn + off, s); off += (size_t)R * (C - 1);
    build_weights((R - 1) * C, (int)dd, pp->beta, pp->E_v.as<double>(), pp->W_v.as<double>(), mn + off, s); off += (size_t)(R - 1) * C;
    build_weights((R - 1) * (C - 1), (int)dd, pp->beta, pp->E_d.as<double>(), pp->W_d.as<double>(), mn + off, s); off += (size_t)(R - 1) * (C - 1);
    build_weights((R - 1) * (C - 1), (int)dd, pp->beta, pp->E_a.as<double>(), pp->W_a.as<double>(), mn + off, s); off += (size_t)(R - 1) * (C - 1);
    std::vector<double> hm(ntab);
    if (ntab) SPG_HIP(hipMemcpyAsync(hm.data(), mn, ntab * 8, hipMemcpyDeviceToHost, s));
    // each column's MPO tensor scaled to a largest entry of 1 (the row logs go
    // to the boundary MPS's log-scales)
    DevBuf lsc;
    lsc.ensure((size_t)R * C * 8);
    pp->row_lsc.ensure((size_t)R * 8);
    site_scales(R, C, d, pp->W_loc.as<double>(), pp->W_h.as<double>(), pp->W_v.as<double>(),
                pp->W_d.as<double>(), pp->W_a.as<double>(), lsc.as<double>(),
                pp->row_lsc.as<double>(), s);
    // constant helper tables
    std::vector<double> ones(dd, 1.0), e0r(dd, 0.0), e0c(dd, 0.0);
    for (int i = 0; i < d; ++i) { e0r[i] = 1.0; e0c[(size_t)i * d] = 1.0; }
    up(pp->ones, ones.data(), dd);
    up(pp->e0row, e0r.data(), dd);
    up(pp->e0col, e0c.data(), dd);
    SPG_HIP(hipStreamSynchronize(s));
    mins.release();
    lsc.release();
    double sh = 0.0;
    for (double v : hm) sh += v;
    pp->shift = sh;
    // the tables as peps_table_bytes sizes them (what batch plans lay out)
    const auto tb = peps_table_bytes(R, C, d);
    const DevBuf *tabs[] = {&pp->E_loc, &pp->E_h, &pp->E_v, &pp->E_d, &pp->E_a, &pp->W_loc,
                            &pp->W_h, &pp->W_v, &pp->W_d, &pp->W_a, &pp->ones, &pp->e0row,
                            &pp->e0col, &pp->e0vec, &pp->row_lsc};
    for (int t = 0; t < kPepsTables; ++t)
      if (tabs[t]->bytes != tb[t]) {
        set_error("spg_build_peps: table sizes differ from peps_table_bytes");
        throw Fail{SPG_ERR_INVALID};
      }
  } catch (...) {
    spg_free_peps(pp);
    throw;
  }
  *out = pp;
  return SPG_OK;
  SPG_CATCH
}

void spg_free_peps(spg_peps_t *pp) {
  if (!pp) return;
  for (DevBuf *b : {&pp->E_loc, &pp->E_h, &pp->E_v, &pp->E_d, &pp->E_a, &pp->W_loc, &pp->W_h,
                    &pp->W_v, &pp->W_d, &pp->W_a, &pp->ones, &pp->e0row, &pp->e0col, &pp->e0vec,
                    &pp->row_lsc})
    b->release();
  delete pp;
}

void spg_free_env(spg_env_t *env) {
  if (!env) return;
  (void)hipDeviceSynchronize();
  for (DevBuf *b : {&env->A, &env->Alp, &env->lam, &env->cfg[0], &env->cfg[1], &env->score[0],
                    &env->score[1], &env->energy[0], &env->energy[1], &env->L[0], &env->L[1],
                    &env->anc[0], &env->anc[1], &env->Rv, &env->Ulp, &env->U64, &env->selws, &env->cand, &env->sel,
                    &env->keys,
                    &env->ids, &env->ework, &env->perm, &env->nvalid, &env->tmp, &env->cfg32})
    b->release();
  delete env;
}

// log Z = lam_0 + log sum_X A_0[x_0]..A_{C-1}[x_{C-1}] - beta * shift, from the
// top row copied to the host (small); the device work must be complete.
// `off` (bytes) selects an instance of a class-batched env; beta and shift are
// that instance's.
static double host_log_Z(const spg_env *env, size_t off, double beta, double shift) {
  const spg_peps *pp = env->peps;
  const int R = pp->rows, C = pp->cols, d = pp->d, chi = env->chi;
  std::vector<double> A0((size_t)C * chi * d * chi), lam(R);
  SPG_HIP(hipMemcpy(A0.data(), (const char *)env->A.p + off, A0.size() * 8,
                    hipMemcpyDeviceToHost));
  SPG_HIP(hipMemcpy(lam.data(), (const char *)env->lam.p + off, R * 8, hipMemcpyDeviceToHost));
  std::vector<double> v(chi, 0.0), nv(chi);
  v[0] = 1.0;
  for (int c = 0; c < C; ++c) {
    std::fill(nv.begin(), nv.end(), 0.0);
    const double *T = A0.data() + (size_t)c * chi * d * chi;
    for (int a = 0; a < chi; ++a)
      for (int x = 0; x < d; ++x)
        for (int b = 0; b < chi; ++b) nv[b] += v[a] * T[((size_t)a * d + x) * chi + b];
    v = nv;
  }
  return lam[0] + std::log(v[0]) - beta * shift;
}

static double host_log_Z(const spg_env *env) {
  return host_log_Z(env, 0, env->peps->beta, env->peps->shift);
}

static int check_mps_params(const spg_mps_params *p) {
  if (!p) return fail(SPG_ERR_INVALID, "null mps params");
  if (p->chi < 1 || p->chi > kMaxChi) return fail(SPG_ERR_UNSUPPORTED, "chi must be in 1..80");
  if (p->num_sweeps < 1) return fail(SPG_ERR_INVALID, "num_sweeps must be >= 1");
  if (p->oversample < 0 || p->power_iters < 0 || p->power_iters > 8)
    return fail(SPG_ERR_INVALID, "oversample >= 0 and power_iters in 0..8 required");
  if (p->chi + p->oversample > kMaxSketch)
    return fail(SPG_ERR_UNSUPPORTED, "chi + oversample must be <= 96");
  if (p->precision != SPG_FP64 && p->precision != SPG_FP32 && p->precision != SPG_BF16)
    return fail(SPG_ERR_INVALID, "precision must be SPG_FP64, SPG_FP32 or SPG_BF16");
  return SPG_OK;
}

int spg_boundary_mps(const spg_peps_t *peps, const spg_mps_params *params, void *stream,
                     spg_env_t **out, double *log_Z_out) {
  SPG_TRY
  if (!peps || !out) return fail(SPG_ERR_INVALID, "spg_boundary_mps: null peps or out");
  int rc = check_mps_params(params);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  spg_env *env = new spg_env();
  try {
    env->peps = peps;
    env->chi = params->chi;
    env->precision = params->precision;
    const int R = peps->rows, C = peps->cols, d = peps->d, chi = params->chi;
    env->dims.assign((size_t)R * (C + 1), 1);
    env->A.ensure((size_t)R * C * chi * d * chi * sizeof(double));
    env->lam.ensure((size_t)R * sizeof(double));
    {
      BmpsWork w;
      boundary_mps_fp64(env, params, s, w);
      make_lp_copy(env, s);
      // keep the workspace alive until the stream has consumed it
      SPG_HIP(hipStreamSynchronize(s));
    }
    if (log_Z_out) {
      SPG_HIP(hipStreamSynchronize(s));
      const double lz = host_log_Z(env);
      *log_Z_out = lz;
      if (!std::isfinite(lz)) {
        *out = env;
        return fail(SPG_ERR_NONFINITE, "spg_boundary_mps: log Z is not finite");
      }
    }
  } catch (...) {
    spg_free_env(env);
    throw;
  }
  *out = env;
  return SPG_OK;
  SPG_CATCH
}

int spg_env_info(const spg_env_t *env, int32_t *rows, int32_t *cols, int32_t *d, int32_t *chi,
                 int32_t *bond_dims) {
  if (!env) return fail(SPG_ERR_INVALID, "spg_env_info: null env");
  if (rows) *rows = env->peps->rows;
  if (cols) *cols = env->peps->cols;
  if (d) *d = env->peps->d;
  if (chi) *chi = env->chi;
  if (bond_dims) std::memcpy(bond_dims, env->dims.data(), env->dims.size() * sizeof(int32_t));
  return SPG_OK;
}

int spg_env_export(const spg_env_t *env, double *tensors, double *lam) {
  SPG_TRY
  if (!env) return fail(SPG_ERR_INVALID, "spg_env_export: null env");
  const spg_peps *pp = env->peps;
  const size_t n = (size_t)pp->rows * pp->cols * env->chi * pp->d * env->chi;
  if (tensors) SPG_HIP(hipMemcpy(tensors, env->A.p, n * 8, hipMemcpyDeviceToHost));
  if (lam) SPG_HIP(hipMemcpy(lam, env->lam.p, (size_t)pp->rows * 8, hipMemcpyDeviceToHost));
  return SPG_OK;
  SPG_CATCH
}

int spg_env_import(const spg_peps_t *peps, int32_t chi, const int32_t *bond_dims,
                   const double *tensors, const double *lam, int32_t precision, void *stream,
                   spg_env_t **out) {
  SPG_TRY
  if (!peps || !bond_dims || !tensors || !out) return fail(SPG_ERR_INVALID, "spg_env_import: null argument");
  if (chi < 1 || chi > kMaxChi) return fail(SPG_ERR_UNSUPPORTED, "spg_env_import: chi must be in 1..80");
  if (precision != SPG_FP64 && precision != SPG_FP32 && precision != SPG_BF16)
    return fail(SPG_ERR_INVALID, "spg_env_import: precision");
  const int R = peps->rows, C = peps->cols, d = peps->d;
  for (int r = 0; r < R; ++r) {
    if (bond_dims[r * (C + 1)] != 1 || bond_dims[r * (C + 1) + C] != 1)
      return fail(SPG_ERR_INVALID, "spg_env_import: boundary bonds must be 1");
    for (int c = 0; c <= C; ++c)
      if (bond_dims[r * (C + 1) + c] < 1 || bond_dims[r * (C + 1) + c] > chi)
        return fail(SPG_ERR_INVALID, "spg_env_import: bond dimension out of range");
  }
  hipStream_t s = (hipStream_t)stream;
  spg_env *env = new spg_env();
  try {
    env->peps = peps;
    env->chi = chi;
    env->precision = precision;
    env->dims.assign(bond_dims, bond_dims + (size_t)R * (C + 1));
    const size_t n = (size_t)R * C * chi * d * chi;
    env->A.ensure(n * 8);
    env->lam.ensure((size_t)R * 8);
    SPG_HIP(hipMemcpyAsync(env->A.p, tensors, n * 8, hipMemcpyHostToDevice, s));
    if (lam) SPG_HIP(hipMemcpyAsync(env->lam.p, lam, (size_t)R * 8, hipMemcpyHostToDevice, s));
    make_lp_copy(env, s);
    SPG_HIP(hipStreamSynchronize(s));
  } catch (...) {
    spg_free_env(env);
    throw;
  }
  *out = env;
  return SPG_OK;
  SPG_CATCH
}

// Search buffers of an env with beam M, with their sizes in bytes.
extern "C++" template <class F>
static void each_search_buffer(spg_env *env, int M, F &&f) {
  const spg_peps *pp = env->peps;
  const int N = pp->rows * pp->cols, d = pp->d, chi = env->chi, C = pp->cols;
  const int p2 = pow2_at_least(std::max(M, 1));
  for (int i = 0; i < 2; ++i) {
    f(env->cfg[i], (size_t)M * N);
    f(env->score[i], (size_t)M * 8);
    f(env->energy[i], (size_t)M * 8);
    f(env->L[i], (size_t)M * chi * 8);
    f(env->anc[i], (size_t)M * 4);
  }
  f(env->Rv, (size_t)M * (C + 1) * chi * 8);
  // reduced-precision search: U_c of every column for the row's ancestors
  if (env->precision != SPG_FP64) f(env->Ulp, (size_t)C * M * chi * d * 4);
  else f(env->U64, (size_t)C * M * chi * d * 8);
  f(env->cand, (size_t)M * d * 8);
  f(env->selws, select_ws_bytes((long)M * d));
  f(env->sel, (size_t)M * 4);
  f(env->keys, (size_t)p2 * 8);
  f(env->ids, (size_t)p2 * 4);
  f(env->ework, (size_t)(M + p2) * 8);
  f(env->perm, (size_t)p2 * 4);
  f(env->nvalid, 8);
}

static void ensure_search(spg_env *env, int M) {
  each_search_buffer(env, M, [](DevBuf &b, size_t n) { b.ensure(n); });
}

// Work buffers of one teacher-forced marginals call (n_beam states).
struct MargBufs {
  uint8_t *cfg;            // [n][N]
  int32_t *anc;            // [n]
  void *Rv;                // [n][C+1][chi] (double; float in reduced precision)
  void *L;                 // [n][chi] (double; float in reduced precision)
  double *L2;              // [n][chi] double (reduced precision: beam_reset_row's target)
  float *U;                // [n][chi*d] (reduced precision)
};

static int marginals_check(const spg_env_t *cenv, int32_t site, int32_t n_beam,
                           const int32_t *beam_cfg, const double *log_cond_out,
                           const char *who) {
  if (!cenv || !beam_cfg || !log_cond_out)
    return fail(SPG_ERR_INVALID, std::string(who) + ": null argument");
  const spg_peps *pp = cenv->peps;
  if (site < 0 || site >= pp->rows * pp->cols)
    return fail(SPG_ERR_INVALID, std::string(who) + ": site out of range");
  if (n_beam < 1) return fail(SPG_ERR_INVALID, std::string(who) + ": n_beam must be >= 1");
  return SPG_OK;
}

static void marginals_run(spg_env *env, int32_t site, int32_t n_beam, const int32_t *beam_cfg,
                          double *log_cond_out, hipStream_t s, const MargBufs &b) {
  const spg_peps *pp = env->peps;
  const int C = pp->cols, N = pp->rows * C, d = pp->d, chi = env->chi;
  const int r = site / C, c = site % C;
  uint8_t *cfg = b.cfg;
  cfg_from_i32(n_beam, N, beam_cfg, cfg, s);
  const SearchTabs t = tabs_of(env);
  const double *A = env->A.as<double>();
  const size_t site_sz = (size_t)chi * d * chi;
  const long rstride = (long)(C + 1) * chi;
  int32_t *anc = b.anc;
  const int* dm = env->dims.data() + r * (C + 1);
  if (env->precision == SPG_FP64) {
    double *Rv = static_cast<double *>(b.Rv);
    set_e0(n_beam, chi, Rv + (size_t)C * chi, rstride, s);
    for (int cc = C - 1; cc > c; --cc)
      right_env_col(t, r, cc, n_beam, cfg, N, A + ((size_t)r * C + cc) * site_sz,
                    Rv + (size_t)(cc + 1) * chi, Rv + (size_t)cc * chi, rstride, dm[cc],
                    dm[cc + 1], s);
    double *L = static_cast<double *>(b.L);
    beam_reset_row(n_beam, chi, L, anc, s);
    for (int cc = 0; cc < c; ++cc)
      advance_L(t, r, cc, n_beam, cfg, N, A + ((size_t)r * C + cc) * site_sz, L, nullptr, s);
    marginals(t, r, c, n_beam, cfg, N, A + ((size_t)r * C + c) * site_sz, L, anc, Rv, rstride,
              nullptr, log_cond_out, 0, dm[c], dm[c + 1], s);
  } else {
    const int pr = env->precision;
    const char *Al = env->Alp.as<char>();
    const size_t eb = lp_elt(env);
    float *Rv = static_cast<float *>(b.Rv);
    float *U = b.U;
    const long ldu = (long)chi * d;
    lp_set_e0(n_beam, chi, Rv + (size_t)C * chi, rstride, s);
    // the products and environments of the search, each beam state its own ancestor
    for (int cc = C - 1; cc >= c; --cc) {
      lp_u_col(t, pr, n_beam, Al + ((size_t)r * C + cc) * site_sz * eb,
               Rv + (size_t)(cc + 1) * chi, rstride, U, ldu, dm[cc], dm[cc + 1], s);
      if (cc > c)
        lp_env_from_u(t, pr, r, cc, n_beam, cfg, N, U, ldu, Rv + (size_t)cc * chi, rstride,
                      dm[cc], s);
    }
    float *L = static_cast<float *>(b.L);
    beam_reset_row(n_beam, chi, b.L2, anc, s);
    lp_set_e0(n_beam, chi, L, chi, s);
    for (int cc = 0; cc < c; ++cc)
      lp_advance_L(t, pr, r, cc, n_beam, cfg, N, Al + ((size_t)r * C + cc) * site_sz * eb, L, s);
    lp_marginals_u(t, r, c, n_beam, cfg, N, U, ldu, L, anc, nullptr, log_cond_out, 0, dm[c], s);
  }
}

int spg_marginals(const spg_env_t *cenv, int32_t site, int32_t n_beam, const int32_t *beam_cfg,
                  double *log_cond_out, void *stream) {
  SPG_TRY
  const int rc = marginals_check(cenv, site, n_beam, beam_cfg, log_cond_out, "spg_marginals");
  if (rc != SPG_OK) return rc;
  spg_env *env = const_cast<spg_env *>(cenv);
  const int N = env->peps->rows * env->peps->cols;
  ensure_search(env, n_beam);
  env->cfg32.ensure((size_t)n_beam * N);
  MargBufs b{env->cfg32.as<uint8_t>(), env->anc[0].as<int32_t>(), env->Rv.p, env->L[0].p,
             env->L[1].as<double>(), env->Ulp.as<float>()};
  marginals_run(env, site, n_beam, beam_cfg, log_cond_out, (hipStream_t)stream, b);
  return SPG_OK;
  SPG_CATCH
}

int spg_topm(int32_t n, int32_t M, const double *scores, int32_t *sel_out, double *scores_out,
             void *stream) {
  SPG_TRY
  if (n < 0 || M < 1) return fail(SPG_ERR_INVALID, "spg_topm: n >= 0 and M >= 1 required");
  if (n == 0) return SPG_OK;
  if (!scores || !sel_out) return fail(SPG_ERR_INVALID, "spg_topm: null pointer");
  hipStream_t s = (hipStream_t)stream;
  const int Me = std::min(M, (int)n);
  const int p2 = pow2_at_least(Me);
  DevBuf keys, ids, ws;
  keys.ensure((size_t)p2 * 8);
  ids.ensure((size_t)p2 * 4);
  ws.ensure(select_ws_bytes(n));
  select_topm(n, M, scores, sel_out, keys.as<uint64_t>(), ids.as<int32_t>(), s, nullptr, nullptr,
              scores_out, ws.p, (long)n);
  SPG_HIP(hipStreamSynchronize(s));                 // before the work buffers are freed
  return SPG_OK;
  SPG_CATCH
}

// ---- spg_marginals_noalloc: the same conditionals without allocating ------
// All work buffers live in one static device array per GPU (held until the
// process ends).  In host code `scratch` names a host-side stand-in, not a
// device address: the address comes from hipGetSymbolAddress, once per device
// with that device current, and only that address reaches kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kScratchDevices];

static int scratch_address(int dev, unsigned char **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= kScratchDevices)
    return fail(SPG_ERR_UNSUPPORTED, "spg_marginals_noalloc: device index beyond 63");
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(SPG_ERR_HIP, std::string("spg_marginals_noalloc: hipGetSymbolAddress: ") +
                                   hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<unsigned char *>(g_scratch_ptr[dev]);
  return SPG_OK;
}

static size_t up256(size_t n) { return (n + 255) & ~size_t(255); }

int spg_marginals_noalloc(const spg_env_t *cenv, int32_t site, int32_t n_beam,
                          const int32_t *beam_cfg, double *log_cond_out, void *stream) {
  SPG_TRY
  const int rc = marginals_check(cenv, site, n_beam, beam_cfg, log_cond_out,
                                 "spg_marginals_noalloc");
  if (rc != SPG_OK) return rc;
  spg_env *env = const_cast<spg_env *>(cenv);
  const spg_peps *pp = env->peps;
  const int C = pp->cols, N = pp->rows * C, d = pp->d, chi = env->chi;
  const bool lp = env->precision != SPG_FP64;
  const size_t n = (size_t)n_beam, eb = lp ? 4 : 8;
  const size_t o_cfg = 0, o_anc = o_cfg + up256(n * N), o_R = o_anc + up256(n * 4);
  const size_t o_L = o_R + up256(n * (C + 1) * chi * eb), o_L2 = o_L + up256(n * chi * eb);
  const size_t o_U = o_L2 + (lp ? up256(n * chi * 8) : 0);
  const size_t need = o_U + (lp ? up256(n * chi * d * 4) : 0);
  if (need > kScratchBytes)
    return fail(SPG_ERR_INVALID, "spg_marginals_noalloc: n_beam = " + std::to_string(n_beam) +
                                     " needs " + std::to_string(need) +
                                     " bytes of scratch, more than its " +
                                     std::to_string(kScratchBytes));
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pp->device) {
    (void)hipGetLastError();
    return fail(SPG_ERR_INVALID, "spg_marginals_noalloc: the env's device must be current");
  }
  unsigned char *base = nullptr;
  const int rs = scratch_address(dev, &base);
  if (rs != SPG_OK) return rs;
  hipStream_t s = (hipStream_t)stream;
  // the previous call's contents stay in the array: clear the part this call uses
  fill_zero(reinterpret_cast<double *>(base), need / 8, s);
  MargBufs b{base + o_cfg, reinterpret_cast<int32_t *>(base + o_anc), base + o_R, base + o_L,
             lp ? reinterpret_cast<double *>(base + o_L2) : nullptr,
             lp ? reinterpret_cast<float *>(base + o_U) : nullptr};
  marginals_run(env, site, n_beam, beam_cfg, log_cond_out, s, b);
  return SPG_OK;
  SPG_CATCH
}

// Training targets recorded by an exact search: per step k, features
// [B_k][d][F] at feats + off[k] * F and exact log-conditionals [B_k][d] at
// targets + off[k].
struct TrainData {
  DevBuf feats, targets;
  std::vector<long> off;
  std::vector<int> nb;
};

static void ensure_guide(spg_env *env, int M) {
  const spg_peps *pp = env->peps;
  const int R = pp->rows, C = pp->cols, N = R * C, d = pp->d, chi = env->chi;
  env->Rsc.ensure((size_t)M * (C + 1) * 8);
  env->sf.ensure((size_t)N * d * 2 * 4);
  env->rscr.ensure((size_t)R * (C + 1) * chi * 8);
  env->gbins.ensure((size_t)M * d * 2);
  env->ghist.ensure(2048 * 4);
  env->gint.ensure(64);
  env->glkey.ensure((size_t)M * d * 8);
  env->glid.ensure((size_t)M * d * 4);
  env->gbound.ensure((size_t)M * 8);
  env->gtau.ensure(8);
  env->goff.ensure((size_t)M * 4);
  env->gcnt.ensure((size_t)M * 4);
  env->gstats.ensure(3 * 8);
  env->selscore.ensure((size_t)M * 8);
  env->smax.ensure(8);
}

static MergeWork merge_work(spg_env *env, int M, bool runners) {
  const int d = env->peps->d;
  int T = 1;
  while (T < 2 * M * d) T <<= 1;
  env->mkey.ensure((size_t)T * 8);
  env->me.ensure((size_t)T * 8);
  env->mid.ensure((size_t)T * 4);
  env->mslot.ensure((size_t)M * d * 4);
  env->mekey.ensure((size_t)M * d * 8);
  MergeWork mw;
  mw.capacity = T;
  mw.tkey = env->mkey.as<unsigned long long>();
  mw.te = env->me.as<unsigned long long>();
  mw.tid = env->mid.as<int32_t>();
  mw.slot = env->mslot.as<int32_t>();
  mw.ekey = env->mekey.as<unsigned long long>();
  if (runners) {
    env->me2.ensure((size_t)T * 8);
    env->mid2.ensure((size_t)T * 4);
    env->mrun.ensure((size_t)M * d * 4);
    mw.te2 = env->me2.as<unsigned long long>();
    mw.tid2 = env->mid2.as<int32_t>();
    mw.run = env->mrun.as<int32_t>();
  }
  return mw;
}

static GuideWork guide_of(spg_env *env) {
  GuideWork g;
  g.bins = env->gbins.as<uint16_t>();
  g.hist = env->ghist.as<unsigned>();
  g.jstar = env->gint.as<int>();
  g.n_list = env->gint.as<int>() + 1;
  g.lkey = env->glkey.as<double>();
  g.lid = env->glid.as<int32_t>();
  g.bound = env->gbound.as<double>();
  g.tau = env->gtau.as<double>();
  g.off = env->goff.as<int32_t>();
  g.cnt = env->gcnt.as<int32_t>();
  g.stats = env->gstats.as<unsigned long long>();
  return g;
}

// The search of spg_branch_and_bound; with `prop` the guarded steps, with
// `td` (exact path only) the training targets of every step are recorded.
static void run_search(spg_env *env, const spg_search_params *prm, const spg_proposal *prop,
                       TrainData *td, int32_t *states_out, double *energies_out,
                       double *logp_out, int32_t *n_out, hipStream_t s, bool sync_out = true) {
  const spg_peps *pp = env->peps;
  const int R = pp->rows, C = pp->cols, N = R * C, d = pp->d, chi = env->chi;
  const int M = prm->max_states;
  ensure_search(env, M);
  const bool guided = prop != nullptr;
  if (guided || td) {
    ensure_guide(env, M);
    fill_zero(env->gstats.as<double>(), 3, s);
    fill_zero(env->ghist.as<double>(), 1024, s);
  }
  const SearchTabs t = tabs_of(env);
  const double *A = env->A.as<double>();
  const size_t site_sz = (size_t)chi * d * chi;
  const long rstride = (long)(C + 1) * chi;
  double *Rv = env->Rv.as<double>();
  double *Rsc = (guided || td) ? env->Rsc.as<double>() : nullptr;
  GuideWork g{};
  if (guided || td) {
    g = guide_of(env);
    site_features(t, A, env->sf.as<float>(), env->rscr.as<double>(), s);
  }
  const int K = guided ? (int)std::min<double>(std::ceil(prm->kappa * M), 2147483647.0) : 0;
  const int D = prm->merge_branches ? prm->max_droplets : 0;
  MergeWork mw;
  if (prm->merge_branches) mw = merge_work(env, M, D > 0);
  env->drop_buf = -1;
  if (D > 0) {
    for (int i = 0; i < 2; ++i) {
      env->dcfg[i].ensure((size_t)M * D * N);
      env->dde[i].ensure((size_t)M * D * 8);
      env->dn[i].ensure((size_t)std::max(M, 2) * 4);
    }
    fill_zero(env->dn[0].as<double>(), 1, s);       // the root holds no droplet (count 0)
  }
  int cur = 0;
  long B = 1;
  fill_zero(env->score[0].as<double>(), 1, s);
  fill_zero(env->energy[0].as<double>(), 1, s);
  const double log_cut = (prm->cut_off_prob > 0.0) ? std::log(prm->cut_off_prob) : 0.0;
  const bool lp = env->precision != SPG_FP64;
  // FP64 plain search: conditionals from the per-ancestor products U (the
  // guarded and the training searches keep the per-state contraction)
  const bool u64 = !lp && !guided && !td;
  const long ldu = (long)chi * d;                  // U row stride
  const char *Al = env->Alp.as<char>();
  const size_t eb = lp ? lp_elt(env) : 0;
  int64_t n_resolved = 0;
  if (td) {
    td->off.clear();
    td->nb.clear();
    long tot = 0, b = 1;
    for (int k = 0; k < N; ++k) {
      td->off.push_back(tot);
      td->nb.push_back((int)b);
      tot += b * d;
      b = std::min<long>(M, b * d);
    }
    td->feats.ensure((size_t)tot * SPG_PROPOSAL_FEATURES * 4);
    td->targets.ensure((size_t)tot * 4);
    env->tmp.ensure((size_t)M * d * 8);
  }
  for (int r = 0; r < R; ++r) {
    const int n_anc = (int)B;
    const int *dm = env->dims.data() + r * (C + 1);
    beam_reset_row(n_anc, chi, lp ? env->L[cur ^ 1].as<double>() : env->L[cur].as<double>(),
                   env->anc[cur].as<int32_t>(), s);
    if (lp) {
      lp_set_e0(n_anc, chi, env->L[cur].as<float>(), chi, s);
      float *Rf = env->Rv.as<float>();
      lp_set_e0(n_anc, chi, Rf + (size_t)C * chi, rstride, s);
      // U_c = A_c R_{c+1} for every ancestor and column: R_c comes from U_c,
      // and the conditionals of column c read U_c again (the guarded steps
      // also need R_0 and the scales: Z_b = scale * L^b . R_c)
      for (int c = C - 1; c >= 0; --c) {
        float *Uc = env->Ulp.as<float>() + (size_t)c * M * ldu;
        lp_u_col(t, env->precision, n_anc, Al + ((size_t)r * C + c) * site_sz * eb,
                 Rf + (size_t)(c + 1) * chi, rstride, Uc, ldu, dm[c], dm[c + 1], s);
        if (c >= 1 || guided)
          lp_env_from_u(t, env->precision, r, c, n_anc, env->cfg[cur].as<uint8_t>(), N, Uc, ldu,
                        Rf + (size_t)c * chi, rstride, dm[c], s, guided ? Rsc + c : nullptr,
                        C + 1);
      }
    } else if (u64) {
      // U_c = A_c R_{c+1} for every ancestor and column on the matrix cores;
      // R_c comes from U_c, and the conditionals of column c read U_c again
      set_e0(n_anc, chi, Rv + (size_t)C * chi, rstride, s);
      for (int c = C - 1; c >= 0; --c) {
        double *Uc = env->U64.as<double>() + (size_t)c * M * ldu;
        u64_col(n_anc, A + ((size_t)r * C + c) * site_sz, chi, Rv + (size_t)(c + 1) * chi,
                rstride, Uc, ldu, d, dm[c], dm[c + 1], s);
        if (c >= 1)
          env_from_u64(t, r, c, n_anc, env->cfg[cur].as<uint8_t>(), N, Uc, ldu,
                       Rv + (size_t)c * chi, rstride, dm[c], s);
      }
    } else {
      set_e0(n_anc, chi, Rv + (size_t)C * chi, rstride, s);
      // the guarded steps also need R_0 and the scales (Z_b = scale * L^b . R_c)
      const int c_lo = guided ? 0 : 1;
      for (int c = C - 1; c >= c_lo; --c)
        right_env_col(t, r, c, n_anc, env->cfg[cur].as<uint8_t>(), N,
                      A + ((size_t)r * C + c) * site_sz, Rv + (size_t)(c + 1) * chi,
                      Rv + (size_t)c * chi, rstride, dm[c], dm[c + 1], s,
                      guided ? Rsc + c : nullptr, C + 1);
    }
    for (int c = 0; c < C; ++c) {
      const int k = r * C + c;
      const double *Arc = A + ((size_t)r * C + c) * site_sz;
      const void *Alc = lp ? (const void *)(Al + ((size_t)r * C + c) * site_sz * eb) : nullptr;
      const uint8_t *cfg = env->cfg[cur].as<uint8_t>();
      const double *score = env->score[cur].as<double>();
      const long Bn = std::min<long>(M, B * d);
      n_resolved += B * d;
      const double *sel_score = nullptr;
      if (guided) {
        // parents are sorted by score: score[0] is the best
        propose(t, r, c, (int)B, cfg, N, score, score, env->sf.as<float>(),
                prop->prm.as<float>(), prop->H, nullptr, g.bins, g.hist, s);
        if (lp)
          guided_step_lp(t, env->precision, r, c, (int)B, M, K, cfg, N,
                         env->Ulp.as<float>() + (size_t)c * M * ldu, ldu, env->L[cur].as<float>(),
                         env->anc[cur].as<int32_t>(), env->Rv.as<float>(), rstride, Rsc, score,
                         g, dm[c], s);
        else
          guided_step(t, r, c, (int)B, M, K, cfg, N, Arc, env->L[cur].as<double>(),
                      env->anc[cur].as<int32_t>(), Rv, rstride, Rsc, score, g, dm[c], dm[c + 1],
                      s);
        if (prm->cut_off_prob > 0.0)
          apply_cutoff((int)(B * d), log_cut, g.lkey, s, g.n_list);
        select_topm((int)(B * d), M, g.lkey, env->sel.as<int32_t>(), env->keys.as<uint64_t>(),
                    env->ids.as<int32_t>(), s, g.n_list, g.lid, env->selscore.as<double>());
        sel_score = env->selscore.as<double>();
      } else {
        if (lp)
          lp_marginals_u(t, r, c, (int)B, cfg, N, env->Ulp.as<float>() + (size_t)c * M * ldu, ldu,
                         env->L[cur].as<float>(), env->anc[cur].as<int32_t>(), score,
                         env->cand.as<double>(), 1, dm[c], s);
        else if (u64)
          marg_from_u64(t, r, c, (int)B, cfg, N, env->U64.as<double>() + (size_t)c * M * ldu,
                        ldu, env->L[cur].as<double>(), env->anc[cur].as<int32_t>(), score,
                        env->cand.as<double>(), 1, dm[c], s);
        else
          marginals(t, r, c, (int)B, cfg, N, Arc, env->L[cur].as<double>(),
                    env->anc[cur].as<int32_t>(), Rv, rstride, score, env->cand.as<double>(), 1,
                    dm[c], dm[c + 1], s);
        if (td) {
          propose(t, r, c, (int)B, cfg, N, score, score, env->sf.as<float>(), nullptr, 1,
                  td->feats.as<float>() + td->off[k] * SPG_PROPOSAL_FEATURES, nullptr, nullptr,
                  s);
          marginals(t, r, c, (int)B, cfg, N, Arc, env->L[cur].as<double>(),
                    env->anc[cur].as<int32_t>(), Rv, rstride, nullptr, env->tmp.as<double>(), 0,
                    dm[c], dm[c + 1], s);
          to_float(B * d, env->tmp.as<double>(), td->targets.as<float>() + td->off[k], s);
        }
        if (prm->merge_branches)
          merge_branches(t, r, c, (int)B, cfg, N, env->energy[cur].as<double>(),
                         env->cand.as<double>(), mw, s);
        if (prm->cut_off_prob > 0.0)
          apply_cutoff((int)(B * d), log_cut, env->cand.as<double>(), s);
        select_topm((int)(B * d), M, env->cand.as<double>(), env->sel.as<int32_t>(),
                    env->keys.as<uint64_t>(), env->ids.as<int32_t>(), s, nullptr, nullptr,
                    nullptr, env->selws.p, (long)M * d, score);   // no child above score[0]
      }
      const int nx = cur ^ 1;
      if (lp)
        lp_beam_update(t, env->precision, r, c, (int)Bn, env->sel.as<int32_t>(), N, cfg,
                       env->energy[cur].as<double>(), env->L[cur].as<float>(),
                       env->anc[cur].as<int32_t>(), env->cand.as<double>(), Alc, c < C - 1,
                       env->cfg[nx].as<uint8_t>(), env->energy[nx].as<double>(),
                       env->score[nx].as<double>(), env->L[nx].as<float>(),
                       env->anc[nx].as<int32_t>(), dm[c], dm[c + 1], s, sel_score);
      else
        beam_update(t, r, c, (int)Bn, env->sel.as<int32_t>(), N, cfg,
                    env->energy[cur].as<double>(), env->L[cur].as<double>(),
                    env->anc[cur].as<int32_t>(), env->cand.as<double>(), Arc, c < C - 1,
                    env->cfg[nx].as<uint8_t>(), env->energy[nx].as<double>(),
                    env->score[nx].as<double>(), env->L[nx].as<double>(),
                    env->anc[nx].as<int32_t>(), dm[c], dm[c + 1], s, sel_score);
      if (D > 0)
        droplet_update(t, r, c, (int)Bn, env->sel.as<int32_t>(), N, cfg,
                       env->energy[cur].as<double>(), mw.run, env->dcfg[cur].as<uint8_t>(),
                       env->dde[cur].as<double>(), env->dn[cur].as<int32_t>(),
                       env->dcfg[nx].as<uint8_t>(), env->dde[nx].as<double>(),
                       env->dn[nx].as<int32_t>(), D, prm->droplet_energy, prm->droplet_hamming,
                       s);
      cur = nx;
      B = Bn;
    }
  }
  if (states_out) {
    final_sort(t, (int)B, N, env->cfg[cur].as<uint8_t>(), env->score[cur].as<double>(),
               states_out, energies_out, logp_out, env->ework.as<double>(),
               env->perm.as<int32_t>(), env->nvalid.as<int32_t>(), s);
    if (D > 0) {
      env->drop_buf = cur;
      env->drop_slots = (int)B;
      env->drop_cap = D;
    }
  }
  if (!sync_out) return;           // enqueued only (batches read env->nvalid later)
  int32_t nv = 0;
  unsigned long long st[3] = {0, 0, 0};
  if (states_out) SPG_HIP(hipMemcpyAsync(&nv, env->nvalid.p, 4, hipMemcpyDeviceToHost, s));
  if (guided) SPG_HIP(hipMemcpyAsync(st, env->gstats.p, sizeof(st), hipMemcpyDeviceToHost, s));
  SPG_HIP(hipStreamSynchronize(s));
  env->last_stats[0] = guided ? (int64_t)st[0] : n_resolved;
  env->last_stats[1] = n_resolved;
  env->last_stats[2] = guided ? (int64_t)st[2] : 0;
  if (n_out) *n_out = nv;
}

int spg_branch_and_bound(const spg_env_t *cenv, const spg_search_params *prm, int32_t *states_out,
                         double *energies_out, double *logp_out, int32_t *n_out, void *stream) {
  SPG_TRY
  if (!cenv || !prm || !states_out || !energies_out || !logp_out || !n_out)
    return fail(SPG_ERR_INVALID, "spg_branch_and_bound: null argument");
  if (prm->max_states < 1 || prm->max_states > 65536)
    return fail(SPG_ERR_UNSUPPORTED, "spg_branch_and_bound: max_states must be in 1..65536");
  if (!(prm->cut_off_prob >= 0.0) || prm->cut_off_prob >= 1.0)
    return fail(SPG_ERR_INVALID, "spg_branch_and_bound: cut_off_prob must be in [0, 1)");
  spg_env *env = const_cast<spg_env *>(cenv);
  if (prm->proposal && prm->merge_branches)
    return fail(SPG_ERR_UNSUPPORTED, "spg_branch_and_bound: merging with a proposal");
  if (prm->max_droplets < 0 || prm->max_droplets > SPG_MAX_DROPLETS)
    return fail(SPG_ERR_UNSUPPORTED, "spg_branch_and_bound: max_droplets must be in 0..64");
  if (prm->max_droplets > 0) {
    if (!prm->merge_branches)
      return fail(SPG_ERR_INVALID, "spg_branch_and_bound: droplets need merge_branches");
    if (!(prm->droplet_energy >= 0.0) || prm->droplet_hamming < 0)
      return fail(SPG_ERR_INVALID,
                  "spg_branch_and_bound: droplet_energy >= 0 and droplet_hamming >= 0 required");
  }
  if (prm->proposal && !(prm->kappa > 0.0))
    return fail(SPG_ERR_INVALID, "spg_branch_and_bound: kappa must be > 0 with a proposal");
  run_search(env, prm, prm->proposal, nullptr, states_out, energies_out, logp_out, n_out,
             (hipStream_t)stream);
  return SPG_OK;
  SPG_CATCH
}

int spg_droplets(const spg_env_t *cenv, int32_t state, int32_t max_out, int32_t *configs_out,
                 double *energies_out, int32_t *n_out) {
  SPG_TRY
  if (!cenv || !n_out || max_out < 0 || (max_out > 0 && (!configs_out || !energies_out)))
    return fail(SPG_ERR_INVALID, "spg_droplets: null argument or negative max_out");
  const spg_env *env = cenv;
  if (env->drop_buf < 0)
    return fail(SPG_ERR_INVALID, "spg_droplets: the last search on this env collected none");
  const int N = env->peps->rows * env->peps->cols, D = env->drop_cap, buf = env->drop_buf;
  int32_t nv = 0;
  SPG_HIP(hipDeviceSynchronize());
  SPG_HIP(hipMemcpy(&nv, env->nvalid.p, 4, hipMemcpyDeviceToHost));
  if (state < 0 || state >= nv)
    return fail(SPG_ERR_INVALID, "spg_droplets: state outside the returned states");
  int32_t slot = 0, cnt = 0;
  double e = 0.0;
  SPG_HIP(hipMemcpy(&slot, env->perm.as<int32_t>() + state, 4, hipMemcpyDeviceToHost));
  if (slot < 0 || slot >= env->drop_slots)
    return fail(SPG_ERR_INVALID, "spg_droplets: internal slot out of range");
  SPG_HIP(hipMemcpy(&cnt, env->dn[buf].as<int32_t>() + slot, 4, hipMemcpyDeviceToHost));
  SPG_HIP(hipMemcpy(&e, env->ework.as<double>() + slot, 8, hipMemcpyDeviceToHost));
  const int n = std::min(cnt, max_out);
  if (n > 0) {
    std::vector<uint8_t> x((size_t)n * N);
    std::vector<double> de(n);
    SPG_HIP(hipMemcpy(x.data(), env->dcfg[buf].as<uint8_t>() + (size_t)slot * D * N, x.size(),
                      hipMemcpyDeviceToHost));
    SPG_HIP(hipMemcpy(de.data(), env->dde[buf].as<double>() + (size_t)slot * D, (size_t)n * 8,
                      hipMemcpyDeviceToHost));
    for (size_t i = 0; i < x.size(); ++i) configs_out[i] = x[i];
    for (int m = 0; m < n; ++m) energies_out[m] = e + de[m];
  }
  *n_out = cnt;
  return SPG_OK;
  SPG_CATCH
}

// ---------------------------------------------------------------------------
// Ising instance -> Potts tables of a cluster lattice (host only).
int spg_ising_to_potts(int32_t n_spins, int32_t n_terms, const int32_t *term_i,
                       const int32_t *term_j, const double *term_J, int32_t rows, int32_t cols,
                       int32_t t, int32_t kings, const int32_t *cluster_of, double *local_E,
                       double *pair_E_h, double *pair_E_v, double *pair_E_d,
                       double *pair_E_a) {
  SPG_TRY
  if (n_spins < 1 || n_terms < 0 || rows < 1 || cols < 1 || !cluster_of || !local_E ||
      (n_terms > 0 && (!term_i || !term_j || !term_J)))
    return fail(SPG_ERR_INVALID, "spg_ising_to_potts: bad sizes or null argument");
  if (t < 1 || t > 8)
    return fail(SPG_ERR_UNSUPPORTED, "spg_ising_to_potts: spins per cluster must be in 1..8");
  const long ncl = (long)rows * cols;
  if (ncl * t != n_spins)
    return fail(SPG_ERR_INVALID, "spg_ising_to_potts: rows * cols * t must equal n_spins");
  if ((cols > 1 && !pair_E_h) || (rows > 1 && !pair_E_v) ||
      (kings && rows > 1 && cols > 1 && (!pair_E_d || !pair_E_a)))
    return fail(SPG_ERR_INVALID, "spg_ising_to_potts: a needed pair table is null");
  const int d = 1 << t;
  // position of each spin in its cluster (ascending spin index)
  std::vector<int> pos(n_spins), fill(ncl, 0);
  for (int i = 0; i < n_spins; ++i) {
    const int cl = cluster_of[i];
    if (cl < 0 || cl >= ncl)
      return fail(SPG_ERR_INVALID, "spg_ising_to_potts: cluster index out of range");
    if (fill[cl] >= t)
      return fail(SPG_ERR_INVALID, "spg_ising_to_potts: a cluster holds more than t spins");
    pos[i] = fill[cl]++;
  }
  const size_t dd = (size_t)d * d;
  std::fill(local_E, local_E + ncl * d, 0.0);
  if (cols > 1) std::fill(pair_E_h, pair_E_h + (size_t)rows * (cols - 1) * dd, 0.0);
  if (rows > 1) std::fill(pair_E_v, pair_E_v + (size_t)(rows - 1) * cols * dd, 0.0);
  if (kings && rows > 1 && cols > 1) {
    std::fill(pair_E_d, pair_E_d + (size_t)(rows - 1) * (cols - 1) * dd, 0.0);
    std::fill(pair_E_a, pair_E_a + (size_t)(rows - 1) * (cols - 1) * dd, 0.0);
  }
  auto spin = [](int x, int k) { return ((x >> k) & 1) ? 1.0 : -1.0; };
  for (int q = 0; q < n_terms; ++q) {
    int i = term_i[q], j = term_j[q];
    const double J = term_J[q];
    if (i < 0 || i >= n_spins || j < 0 || j >= n_spins)
      return fail(SPG_ERR_INVALID, "spg_ising_to_potts: spin index out of range");
    if (!std::isfinite(J)) return fail(SPG_ERR_NONFINITE, "spg_ising_to_potts: coupling not finite");
    int a = cluster_of[i], b = cluster_of[j];
    if (i == j || a == b) {
      // field h_i s_i, or a coupling inside one cluster
      double *row = local_E + (size_t)a * d;
      for (int x = 0; x < d; ++x)
        row[x] += (i == j) ? J * spin(x, pos[i]) : J * spin(x, pos[i]) * spin(x, pos[j]);
      continue;
    }
    int ra = a / cols, ca = a % cols, rb = b / cols, cb = b % cols;
    // orient the pair as the table stores it: first index the upper (or left) cluster
    if (rb < ra || (rb == ra && cb < ca)) {
      std::swap(i, j);
      std::swap(a, b);
      std::swap(ra, rb);
      std::swap(ca, cb);
    }
    double *tab = nullptr;
    if (rb == ra && cb == ca + 1) tab = pair_E_h + ((size_t)ra * (cols - 1) + ca) * dd;
    else if (rb == ra + 1 && cb == ca) tab = pair_E_v + ((size_t)ra * cols + ca) * dd;
    else if (kings && rb == ra + 1 && cb == ca + 1)
      tab = pair_E_d + ((size_t)ra * (cols - 1) + ca) * dd;
    else if (kings && rb == ra + 1 && cb == ca - 1)
      tab = pair_E_a + ((size_t)ra * (cols - 1) + cb) * dd;    // [x_(r,c+1)][x_(r+1,c)]
    else
      return fail(SPG_ERR_INVALID,
                  "spg_ising_to_potts: a coupling joins clusters that are not lattice neighbours");
    for (int x = 0; x < d; ++x) {
      const double sx = J * spin(x, pos[i]);
      for (int y = 0; y < d; ++y) tab[(size_t)x * d + y] += sx * spin(y, pos[j]);
    }
  }
  return SPG_OK;
  SPG_CATCH
}

int spg_search_stats(const spg_env_t *env, int64_t *counts) {
  if (!env || !counts) return fail(SPG_ERR_INVALID, "spg_search_stats: null argument");
  for (int i = 0; i < 3; ++i) counts[i] = env->last_stats[i];
  return SPG_OK;
}

// ---- learned proposal ------------------------------------------------------

int spg_proposal_create(int32_t hidden, uint64_t seed, spg_proposal_t **out) {
  SPG_TRY
  if (!out) return fail(SPG_ERR_INVALID, "spg_proposal_create: null out");
  if (hidden < 1 || hidden > kMaxHidden)
    return fail(SPG_ERR_INVALID, "spg_proposal_create: hidden must be in 1..64");
  const int H = hidden, P = mlp_n_params(H);
  std::vector<float> w(P, 0.0f);
  // uniform(-1, 1) from SplitMix64 output i (top 53 bits), scaled per layer
  for (int i = 0; i < P; ++i) {
    const bool w1 = i < H * kFeat, w2 = i >= H * kFeat + H && i < H * kFeat + 2 * H;
    if (!w1 && !w2) continue;
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    w[i] = (float)(u * std::sqrt(6.0 / (w1 ? kFeat : H)));
  }
  spg_proposal *p = new spg_proposal();
  try {
    p->H = H;
    p->prm.ensure((size_t)P * 4);
    p->m.ensure((size_t)P * 4);
    p->v.ensure((size_t)P * 4);
    p->grad.ensure((size_t)P * 4);
    p->loss.ensure(64);
    p->partial.ensure(mlp_partial_floats(H) * 4);
    SPG_HIP(hipMemcpy(p->prm.p, w.data(), (size_t)P * 4, hipMemcpyHostToDevice));
  } catch (...) {
    delete p;
    throw;
  }
  *out = p;
  return SPG_OK;
  SPG_CATCH
}

void spg_proposal_free(spg_proposal_t *prop) { delete prop; }

int spg_proposal_params(spg_proposal_t *prop, float *host_out, const float *host_in,
                        int32_t *n_params) {
  SPG_TRY
  if (!prop) return fail(SPG_ERR_INVALID, "spg_proposal_params: null proposal");
  const int P = mlp_n_params(prop->H);
  if (n_params) *n_params = P;
  SPG_HIP(hipDeviceSynchronize());
  if (host_out) SPG_HIP(hipMemcpy(host_out, prop->prm.p, (size_t)P * 4, hipMemcpyDeviceToHost));
  if (host_in) {
    SPG_HIP(hipMemcpy(prop->prm.p, host_in, (size_t)P * 4, hipMemcpyHostToDevice));
    SPG_HIP(hipMemset(prop->m.p, 0, (size_t)P * 4));
    SPG_HIP(hipMemset(prop->v.p, 0, (size_t)P * 4));
    prop->t = 0;
  }
  return SPG_OK;
  SPG_CATCH
}

int spg_proposal_features(const spg_env_t *cenv, int32_t site, int32_t n_beam,
                          const int32_t *beam_cfg, const double *beam_score, float *feats_out,
                          void *stream) {
  SPG_TRY
  if (!cenv || !beam_cfg || !beam_score || !feats_out)
    return fail(SPG_ERR_INVALID, "spg_proposal_features: null argument");
  spg_env *env = const_cast<spg_env *>(cenv);
  const spg_peps *pp = env->peps;
  const int C = pp->cols, N = pp->rows * C;
  if (site < 0 || site >= N) return fail(SPG_ERR_INVALID, "spg_proposal_features: site out of range");
  if (n_beam < 1) return fail(SPG_ERR_INVALID, "spg_proposal_features: n_beam must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  ensure_search(env, n_beam);
  ensure_guide(env, n_beam);
  env->cfg32.ensure((size_t)n_beam * N);
  uint8_t *cfg = env->cfg32.as<uint8_t>();
  cfg_from_i32(n_beam, N, beam_cfg, cfg, s);
  const SearchTabs t = tabs_of(env);
  site_features(t, env->A.as<double>(), env->sf.as<float>(), env->rscr.as<double>(), s);
  max_of(n_beam, beam_score, env->smax.as<double>(), s);
  propose(t, site / C, site % C, n_beam, cfg, N, beam_score, env->smax.as<double>(),
          env->sf.as<float>(), nullptr, 1, feats_out, nullptr, nullptr, s);
  return SPG_OK;
  SPG_CATCH
}

int spg_proposal_forward(const spg_proposal_t *prop, int32_t n_beam, int32_t d,
                         const float *feats, float *logp_out, void *stream) {
  SPG_TRY
  if (!prop || !feats || !logp_out) return fail(SPG_ERR_INVALID, "spg_proposal_forward: null argument");
  if (n_beam < 1 || d < 1 || d > 256)
    return fail(SPG_ERR_INVALID, "spg_proposal_forward: n_beam >= 1 and 1 <= d <= 256");
  mlp_forward(n_beam, d, feats, prop->prm.as<float>(), prop->H, logp_out, (hipStream_t)stream);
  return SPG_OK;
  SPG_CATCH
}

int spg_proposal_loss_grad(const spg_proposal_t *prop, int32_t n_beam, int32_t d,
                           const float *feats, const float *target_logp, float *grad_out,
                           float *loss_out, void *stream) {
  SPG_TRY
  if (!prop || !feats || !target_logp || !grad_out || !loss_out)
    return fail(SPG_ERR_INVALID, "spg_proposal_loss_grad: null argument");
  if (n_beam < 1 || d < 1 || d > 256)
    return fail(SPG_ERR_INVALID, "spg_proposal_loss_grad: n_beam >= 1 and 1 <= d <= 256");
  spg_proposal *p = const_cast<spg_proposal *>(prop);
  mlp_loss_grad(n_beam, d, feats, target_logp, p->prm.as<float>(), p->H, p->partial.as<float>(),
                grad_out, loss_out, nullptr, (hipStream_t)stream);
  return SPG_OK;
  SPG_CATCH
}

int spg_proposal_adam(spg_proposal_t *prop, const float *grad, float learning_rate,
                      void *stream) {
  SPG_TRY
  if (!prop || !grad) return fail(SPG_ERR_INVALID, "spg_proposal_adam: null argument");
  if (!(learning_rate > 0.0f)) return fail(SPG_ERR_INVALID, "spg_proposal_adam: learning_rate must be > 0");
  prop->t += 1;
  const double tt = (double)prop->t;
  mlp_adam(mlp_n_params(prop->H), prop->prm.as<float>(), prop->m.as<float>(),
           prop->v.as<float>(), grad, learning_rate, (float)(1.0 - std::pow(0.9, tt)),
           (float)(1.0 - std::pow(0.999, tt)), (hipStream_t)stream);
  return SPG_OK;
  SPG_CATCH
}

int spg_proposal_train(spg_proposal_t *prop, const spg_env_t *cenv, const spg_train_params *tp,
                       void *stream, float *loss_out) {
  SPG_TRY
  if (!prop || !cenv || !tp) return fail(SPG_ERR_INVALID, "spg_proposal_train: null argument");
  if (tp->epochs < 1 || !(tp->learning_rate > 0.0f))
    return fail(SPG_ERR_INVALID, "spg_proposal_train: epochs >= 1 and learning_rate > 0");
  if (tp->max_states < 1 || tp->max_states > 65536)
    return fail(SPG_ERR_UNSUPPORTED, "spg_proposal_train: max_states must be in 1..65536");
  spg_env *env = const_cast<spg_env *>(cenv);
  if (env->precision != SPG_FP64)
    return fail(SPG_ERR_UNSUPPORTED, "spg_proposal_train: needs an FP64 env");
  hipStream_t s = (hipStream_t)stream;
  const int N = env->peps->rows * env->peps->cols, d = env->peps->d;
  spg_search_params sp{};
  sp.max_states = tp->max_states;
  TrainData td;
  run_search(env, &sp, nullptr, &td, nullptr, nullptr, nullptr, nullptr, s);
  DevBuf eloss;
  eloss.ensure((size_t)tp->epochs * 4);
  for (int e = 0; e < tp->epochs; ++e)
    for (int k = 0; k < N; ++k) {
      mlp_loss_grad(td.nb[k], d, td.feats.as<float>() + td.off[k] * SPG_PROPOSAL_FEATURES,
                    td.targets.as<float>() + td.off[k], prop->prm.as<float>(), prop->H,
                    prop->partial.as<float>(), prop->grad.as<float>(), prop->loss.as<float>(),
                    eloss.as<float>() + e, s);
      prop->t += 1;
      const double tt = (double)prop->t;
      mlp_adam(mlp_n_params(prop->H), prop->prm.as<float>(), prop->m.as<float>(),
               prop->v.as<float>(), prop->grad.as<float>(), tp->learning_rate,
               (float)(1.0 - std::pow(0.9, tt)), (float)(1.0 - std::pow(0.999, tt)), s);
    }
  std::vector<float> h(tp->epochs);
  SPG_HIP(hipMemcpyAsync(h.data(), eloss.p, (size_t)tp->epochs * 4, hipMemcpyDeviceToHost, s));
  SPG_HIP(hipStreamSynchronize(s));
  if (loss_out)
    for (int e = 0; e < tp->epochs; ++e) loss_out[e] = h[e] / (float)N;
  return SPG_OK;
  SPG_CATCH
}


// ---- batches ------------------------------------------------------------------
// A shape class: instances with equal lattice, d, kings, chi, beam, sweeps and
// truncation parameters and an FP64 search.  All their device data sit in
// equal slices of one allocation; the class runs its whole path once with
// every launch covering all members (class-batched launches).
struct BatchClass {
  std::vector<int> members;
  DevBuf arena;
  size_t slice = 0;
  spg_peps peps;                  // tables: views into slice 0
  spg_env env;                    // boundary MPS and search buffers: views into slice 0
  BmpsWork w;                     // contraction workspace: views into slice 0
  DevBuf states, energies, logp;  // outputs: views into slice 0
};

struct spg_batch {
  int n = 0;
  std::vector<spg_batch_item> items;
  std::vector<const spg_peps *> src;
  // unit u: a class (cls[u] >= 0) or one instance on the stream path
  std::vector<int> unit_cls, unit_inst;
  std::vector<Tuning> unit_tune;
  std::vector<int> inst_unit, inst_member;
  std::vector<std::unique_ptr<BatchClass>> classes;
  std::vector<spg_env *> envs;    // stream-path instances (nullptr for class members)
  std::vector<std::unique_ptr<BmpsWork>> slots;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr, ev_in = nullptr, ev_out = nullptr;
  hipStream_t origin = nullptr;   // capture and replay stream (the caller's may be the null stream)
  std::vector<std::unique_ptr<DevBuf>> states, energies, logp;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool warm = false;
  ~spg_batch() {
    (void)hipDeviceSynchronize();
    drop_graph();
    for (auto e : done) (void)hipEventDestroy(e);
    for (auto e : {fork, ev_in, ev_out})
      if (e) (void)hipEventDestroy(e);
    if (origin) (void)hipStreamDestroy(origin);
    for (auto st : streams) (void)hipStreamDestroy(st);
    for (auto e : envs) spg_free_env(e);
  }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
};

static spg_mps_params item_mps(const spg_batch_item &it) {
  spg_mps_params m{};
  m.chi = it.chi; m.num_sweeps = it.num_sweeps; m.precision = it.precision;
  m.oversample = it.oversample; m.power_iters = it.power_iters;
  return m;
}

static bool same_class(const spg_batch_item &a, const spg_peps *pa, const spg_batch_item &b,
                       const spg_peps *pb) {
  return a.precision == SPG_FP64 && b.precision == SPG_FP64 && a.chi == b.chi &&
         a.num_sweeps == b.num_sweeps && a.oversample == b.oversample &&
         a.power_iters == b.power_iters && a.max_states == b.max_states &&
         a.cut_off_prob == b.cut_off_prob && pa->rows == pb->rows && pa->cols == pb->cols &&
         pa->d == pb->d && pa->kings == pb->kings;
}

// Largest allocation of one class: classes whose slices would exceed it are
// split, so every address within a class stays inside a 1 GiB span.
constexpr size_t kClassBytes = (size_t)1 << 30;

// Lay out one slice: every buffer of the class's peps, env, workspace and
// outputs, 256-byte aligned; allocate n slices (unless layout_only) and point
// the views at slice 0.  Returns the slice size.
static size_t build_class(BatchClass &k, const std::vector<const spg_peps *> &src,
                          const spg_batch_item &it, bool layout_only = false,
                          std::vector<std::pair<size_t, size_t>> *layout = nullptr) {
  const spg_peps *p0 = src[k.members[0]];
  const int R = p0->rows, C = p0->cols, d = p0->d, chi = it.chi, M = it.max_states;
  k.peps.rows = R; k.peps.cols = C; k.peps.d = d; k.peps.kings = p0->kings;
  k.peps.beta = p0->beta; k.peps.shift = p0->shift; k.peps.device = p0->device;
  k.env.peps = &k.peps;
  k.env.chi = chi;
  k.env.precision = SPG_FP64;
  k.env.dims.assign((size_t)R * (C + 1), 1);
  const spg_mps_params mp = item_mps(it);
  k.w.R = R; k.w.C = C; k.w.d = d; k.w.chi = chi;
  k.w.lmax = bmps_lmax(chi, d, &mp);
  std::vector<std::pair<DevBuf *, size_t>> list;
  auto add = [&](DevBuf &b, size_t n) { list.emplace_back(&b, std::max<size_t>(n, 8)); };
  spg_peps *pk = &k.peps;
  const DevBuf *srcb[] = {&p0->E_loc, &p0->E_h, &p0->E_v, &p0->E_d, &p0->E_a, &p0->W_loc,
                          &p0->W_h, &p0->W_v, &p0->W_d, &p0->W_a, &p0->ones, &p0->e0row,
                          &p0->e0col, &p0->e0vec, &p0->row_lsc};
  DevBuf *dstb[] = {&pk->E_loc, &pk->E_h, &pk->E_v, &pk->E_d, &pk->E_a, &pk->W_loc, &pk->W_h,
                    &pk->W_v, &pk->W_d, &pk->W_a, &pk->ones, &pk->e0row, &pk->e0col, &pk->e0vec,
                    &pk->row_lsc};
  constexpr int kPepsBufs = kPepsTables;
  for (int t = 0; t < kPepsBufs; ++t) add(*dstb[t], srcb[t]->bytes);
  add(k.env.A, (size_t)R * C * chi * d * chi * sizeof(double));
  add(k.env.lam, (size_t)R * sizeof(double));
  each_search_buffer(&k.env, M, add);
  k.w.each(add);
  add(k.states, (size_t)M * R * C * 4);
  add(k.energies, (size_t)M * 8);
  add(k.logp, (size_t)M * 8);
  std::vector<size_t> off;
  size_t tot = 0;
  for (auto &e : list) {
    off.push_back(tot);
    tot += (e.second + 255) / 256 * 256;
  }
  k.slice = tot;
  if (layout)
    for (size_t q = 0; q < list.size(); ++q) layout->emplace_back(off[q], list[q].second);
  if (layout_only) return tot;
  const int n = (int)k.members.size();
  if (tot * n > kClassBytes) {
    set_error("build_class: class allocation above its cap");
    throw Fail{SPG_ERR_UNSUPPORTED};
  }
  k.arena.ensure(tot * n);
  char *base = k.arena.as<char>();
  for (size_t q = 0; q < list.size(); ++q) list[q].first->view(base + off[q], list[q].second);
  // each member's tables into its slice
  for (int m = 0; m < n; ++m) {
    const spg_peps *pm = src[k.members[m]];
    const DevBuf *sb[] = {&pm->E_loc, &pm->E_h, &pm->E_v, &pm->E_d, &pm->E_a, &pm->W_loc,
                          &pm->W_h, &pm->W_v, &pm->W_d, &pm->W_a, &pm->ones, &pm->e0row,
                          &pm->e0col, &pm->e0vec, &pm->row_lsc};
    for (int t = 0; t < kPepsBufs; ++t)
      if (sb[t]->bytes)
        SPG_HIP(hipMemcpy(base + (size_t)m * tot + off[t], sb[t]->p, sb[t]->bytes,
                          hipMemcpyDeviceToDevice));
  }
  return tot;
}

// Unit u's whole path (contraction, search, output) enqueued on stream st.
static void enqueue_unit(spg_batch *b, int u, hipStream_t st) {
  const Tuning saved_t = g_tune;
  const BatchCtx saved_b = g_bc;
  g_tune = b->unit_tune[u];
  try {
    if (b->unit_cls[u] >= 0) {
      BatchClass &k = *b->classes[b->unit_cls[u]];
      const spg_batch_item &it = b->items[k.members[0]];
      g_bc.n = (int)k.members.size();
      g_bc.ist = (long)k.slice;
      g_bc.lo = k.arena.as<char>();
      g_bc.hi = k.arena.as<char>() + k.slice;
      const spg_mps_params mp = item_mps(it);
      boundary_mps_fp64(&k.env, &mp, st, k.w);
      spg_search_params sp{};
      sp.max_states = it.max_states;
      sp.cut_off_prob = it.cut_off_prob;
      run_search(&k.env, &sp, nullptr, nullptr, k.states.as<int32_t>(), k.energies.as<double>(),
                 k.logp.as<double>(), nullptr, st, false);
    } else {
      const int i = b->unit_inst[u];
      const spg_batch_item &it = b->items[i];
      spg_env *env = b->envs[i];
      const spg_mps_params mp = item_mps(it);
      boundary_mps_fp64(env, &mp, st, *b->slots[u % b->slots.size()]);
      make_lp_copy(env, st);
      spg_search_params sp{};
      sp.max_states = it.max_states;
      sp.cut_off_prob = it.cut_off_prob;
      run_search(env, &sp, nullptr, nullptr, b->states[i]->as<int32_t>(),
                 b->energies[i]->as<double>(), b->logp[i]->as<double>(), nullptr, st, false);
    }
  } catch (...) {
    g_tune = saved_t;
    g_bc = saved_b;
    throw;
  }
  g_tune = saved_t;
  g_bc = saved_b;
}

// Every unit, round-robin over the batch's streams, forked from and joined
// back into s.
static void enqueue_batch(spg_batch *b, hipStream_t s) {
  SPG_HIP(hipEventRecord(b->fork, s));
  for (auto st : b->streams) SPG_HIP(hipStreamWaitEvent(st, b->fork, 0));
  const int S = (int)b->streams.size();
  const int U = (int)b->unit_cls.size();
  for (int u = 0; u < U; ++u) enqueue_unit(b, u, b->streams[u % S]);
  for (int k = 0; k < S; ++k) {
    SPG_HIP(hipEventRecord(b->done[k], b->streams[k]));
    SPG_HIP(hipStreamWaitEvent(s, b->done[k], 0));
  }
}

// Units of a batch, in order: lists of member instances.  With
// SPG_BATCH_CLASSES, FP64 instances of equal shape form classes of as many
// members as fit in kClassBytes; every other instance is a unit of its own.
extern "C++" {
static std::vector<std::vector<int>> batch_units(const std::vector<const spg_peps *> &src,
                                                 const spg_batch_item *items, int n, int flags) {
  std::vector<std::vector<int>> units;
  std::vector<int> placed(n, 0);
  for (int i = 0; i < n; ++i) {
    if (placed[i]) continue;
    std::vector<int> mem{i};
    if ((flags & SPG_BATCH_CLASSES) && items[i].precision == SPG_FP64) {
      BatchClass probe;
      probe.members = mem;
      const size_t slice = build_class(probe, src, items[i], true);
      const size_t cap = std::max<size_t>(1, kClassBytes / slice);
      for (int j = i + 1; j < n && mem.size() < cap; ++j)
        if (!placed[j] && same_class(items[i], src[i], items[j], src[j])) mem.push_back(j);
    }
    for (int m : mem) placed[m] = 1;
    units.push_back(mem);
  }
  return units;
}
}  // extern "C++"

// Argument checks shared by spg_batch_create and spg_batch_plan.
static int check_batch_items(const spg_batch_item *items, int32_t n, int32_t flags,
                             const char *who) {
  if (n < 1) return fail(SPG_ERR_INVALID, std::string(who) + ": n must be >= 1");
  if (flags & ~SPG_BATCH_CLASSES) return fail(SPG_ERR_INVALID, std::string(who) + ": unknown flags");
  for (int i = 0; i < n; ++i) {
    const spg_mps_params mp = item_mps(items[i]);
    int rc = check_mps_params(&mp);
    if (rc) return rc;
    if (items[i].max_states < 1 || items[i].max_states > 65536)
      return fail(SPG_ERR_UNSUPPORTED, std::string(who) + ": max_states must be in 1..65536");
    if (!(items[i].cut_off_prob >= 0.0) || items[i].cut_off_prob >= 1.0)
      return fail(SPG_ERR_INVALID, std::string(who) + ": cut_off_prob must be in [0, 1)");
  }
  return SPG_OK;
}

int spg_batch_create(const spg_peps_t *const *peps, const spg_batch_item *items, int32_t n,
                     int32_t n_streams, int32_t flags, spg_batch_t **out) {
  SPG_TRY
  if (!peps || !items || !out) return fail(SPG_ERR_INVALID, "spg_batch_create: null argument");
  if (n_streams < 1 || n_streams > 64)
    return fail(SPG_ERR_INVALID, "spg_batch_create: n_streams must be in 1..64");
  int rc0 = check_batch_items(items, n, flags, "spg_batch_create");
  if (rc0) return rc0;
  for (int i = 0; i < n; ++i)
    if (!peps[i]) return fail(SPG_ERR_INVALID, "spg_batch_create: null peps");
  spg_batch *b = new spg_batch();
  try {
    b->n = n;
    b->items.assign(items, items + n);
    b->src.assign(peps, peps + n);
    b->inst_unit.assign(n, -1);
    b->inst_member.assign(n, 0);
    b->envs.assign(n, nullptr);
    // units: classes of two or more FP64 instances (with SPG_BATCH_CLASSES), else single
    for (const std::vector<int> &mem : batch_units(b->src, items, n, flags)) {
      const int i = mem[0];
      const int u = (int)b->unit_cls.size();
      if (mem.size() > 1) {
        std::unique_ptr<BatchClass> k(new BatchClass());
        k->members = mem;
        build_class(*k, b->src, items[i]);
        for (size_t m = 0; m < mem.size(); ++m) {
          b->inst_unit[mem[m]] = u;
          b->inst_member[mem[m]] = (int)m;
        }
        b->unit_cls.push_back((int)b->classes.size());
        b->unit_inst.push_back(-1);
        b->classes.push_back(std::move(k));
      } else {
        b->inst_unit[i] = u;
        b->unit_cls.push_back(-1);
        b->unit_inst.push_back(i);
        const spg_peps *pp = peps[i];
        spg_env *env = new spg_env();
        b->envs[i] = env;
        env->peps = pp;
        env->chi = items[i].chi;
        env->precision = items[i].precision;
        const int R = pp->rows, C = pp->cols, d = pp->d, chi = items[i].chi;
        env->dims.assign((size_t)R * (C + 1), 1);
        env->A.ensure((size_t)R * C * chi * d * chi * sizeof(double));
        env->lam.ensure((size_t)R * sizeof(double));
        ensure_search(env, items[i].max_states);
      }
    }
    b->states.resize(n);
    b->energies.resize(n);
    b->logp.resize(n);
    for (int i = 0; i < n; ++i) {
      if (!b->envs[i]) continue;
      const spg_peps *pp = peps[i];
      const int M = items[i].max_states;
      b->states[i].reset(new DevBuf());
      b->energies[i].reset(new DevBuf());
      b->logp[i].reset(new DevBuf());
      b->states[i]->ensure((size_t)M * pp->rows * pp->cols * 4);
      b->energies[i]->ensure((size_t)M * 8);
      b->logp[i]->ensure((size_t)M * 8);
    }
    b->unit_tune.assign(b->unit_cls.size(), g_tune);
    const int S = std::min<int>(n_streams, (int)b->unit_cls.size());
    for (int k = 0; k < S; ++k) {
      hipStream_t st;
      SPG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      b->streams.push_back(st);
      hipEvent_t e;
      SPG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->done.push_back(e);
      b->slots.emplace_back(new BmpsWork());
    }
    SPG_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    SPG_HIP(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    SPG_HIP(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    SPG_HIP(hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking));
  } catch (...) {
    delete b;
    throw;
  }
  *out = b;
  return SPG_OK;
  SPG_CATCH
}

int spg_batch_plan(const int32_t *shapes, const spg_batch_item *items, int32_t n, int32_t flags,
                   int32_t *unit_of, int32_t *n_units, int64_t *unit_bytes, int32_t max_buffers,
                   int64_t *layout, int32_t *n_buffers) {
  SPG_TRY
  if (!shapes || !items || !unit_of || !n_units || !unit_bytes || !n_buffers)
    return fail(SPG_ERR_INVALID, "spg_batch_plan: null argument");
  if (max_buffers < 0 || (max_buffers > 0 && !layout))
    return fail(SPG_ERR_INVALID, "spg_batch_plan: layout needs max_buffers >= 1");
  int rc = check_batch_items(items, n, flags, "spg_batch_plan");
  if (rc) return rc;
  // PEPS of the given shapes that only carry their tables' sizes
  std::vector<std::unique_ptr<spg_peps>> held;
  std::vector<const spg_peps *> src;
  for (int i = 0; i < n; ++i) {
    const int R = shapes[4 * i], C = shapes[4 * i + 1], d = shapes[4 * i + 2];
    const int kings = shapes[4 * i + 3];
    if (R < 1 || C < 2 || d < 2 || d > 256 || (long)R * C > 65536 || (kings != 0 && kings != 1))
      return fail(SPG_ERR_UNSUPPORTED, "spg_batch_plan: shape outside the limits of spg_build_peps");
    std::unique_ptr<spg_peps> pp(new spg_peps());
    pp->rows = R; pp->cols = C; pp->d = d; pp->kings = kings;
    const auto tb = peps_table_bytes(R, C, d);
    DevBuf *tabs[] = {&pp->E_loc, &pp->E_h, &pp->E_v, &pp->E_d, &pp->E_a, &pp->W_loc, &pp->W_h,
                      &pp->W_v, &pp->W_d, &pp->W_a, &pp->ones, &pp->e0row, &pp->e0col,
                      &pp->e0vec, &pp->row_lsc};
    for (int t = 0; t < kPepsTables; ++t) tabs[t]->view(nullptr, tb[t]);
    src.push_back(pp.get());
    held.push_back(std::move(pp));
  }
  const std::vector<std::vector<int>> units = batch_units(src, items, n, flags);
  for (size_t u = 0; u < units.size(); ++u) {
    const std::vector<int> &mem = units[u];
    for (int m : mem) unit_of[m] = (int32_t)u;
    unit_bytes[2 * u] = (int64_t)mem.size();
    unit_bytes[2 * u + 1] = 0;
    n_buffers[u] = 0;
    if (mem.size() < 2) continue;
    BatchClass k;
    k.members = mem;
    std::vector<std::pair<size_t, size_t>> lay;
    unit_bytes[2 * u + 1] = (int64_t)build_class(k, src, items[mem[0]], true, &lay);
    n_buffers[u] = (int32_t)lay.size();
    if ((int)lay.size() > max_buffers) continue;
    for (size_t q = 0; q < lay.size(); ++q) {
      layout[((size_t)u * max_buffers + q) * 2] = (int64_t)lay[q].first;
      layout[((size_t)u * max_buffers + q) * 2 + 1] = (int64_t)lay[q].second;
    }
  }
  *n_units = (int32_t)units.size();
  return SPG_OK;
  SPG_CATCH
}

void spg_batch_free(spg_batch_t *b) { delete b; }

int spg_batch_info(const spg_batch_t *b, int32_t *n_units, int32_t *unit_of) {
  if (!b) return fail(SPG_ERR_INVALID, "spg_batch_info: null batch");
  if (n_units) *n_units = (int32_t)b->unit_cls.size();
  if (unit_of)
    for (int i = 0; i < b->n; ++i) unit_of[i] = b->inst_unit[i];
  return SPG_OK;
}

int spg_batch_run(spg_batch_t *b, int32_t use_graph, void *stream) {
  SPG_TRY
  if (!b) return fail(SPG_ERR_INVALID, "spg_batch_run: null batch");
  hipStream_t s = (hipStream_t)stream;
  if (!use_graph || !b->warm) {
    // eager pass: also sizes every workspace so a later capture allocates nothing
    enqueue_batch(b, s);
    if (!b->warm) SPG_HIP(hipStreamSynchronize(s));
    b->warm = true;
    if (!use_graph) return SPG_OK;
  }
  hipStream_t o = b->origin;
  if (!b->exec) {
    SPG_HIP(hipStreamSynchronize(o));
    const bool prof = g_prof;
    g_prof = false;                    // no timing events inside the graph
    SPG_HIP(hipStreamBeginCapture(o, hipStreamCaptureModeRelaxed));
    try {
      enqueue_batch(b, o);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(o, &g);
      if (g) (void)hipGraphDestroy(g);
      g_prof = prof;
      throw;
    }
    g_prof = prof;
    SPG_HIP(hipStreamEndCapture(o, &b->graph));
    SPG_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  // the replay runs on the batch's own stream, ordered after and before s
  SPG_HIP(hipEventRecord(b->ev_in, s));
  SPG_HIP(hipStreamWaitEvent(o, b->ev_in, 0));
  SPG_HIP(hipGraphLaunch(b->exec, o));
  SPG_HIP(hipEventRecord(b->ev_out, o));
  SPG_HIP(hipStreamWaitEvent(s, b->ev_out, 0));
  return SPG_OK;
  SPG_CATCH
}

int spg_batch_result(const spg_batch_t *b, int32_t i, int32_t *states_out, double *energies_out,
                     double *logp_out, int32_t *n_out, double *log_Z) {
  SPG_TRY
  if (!b || !n_out) return fail(SPG_ERR_INVALID, "spg_batch_result: null argument");
  if (i < 0 || i >= b->n) return fail(SPG_ERR_INVALID, "spg_batch_result: index out of range");
  SPG_HIP(hipDeviceSynchronize());
  const spg_peps *pp = b->src[i];
  const size_t N = (size_t)pp->rows * pp->cols;
  const int u = b->inst_unit[i];
  const spg_env *env;
  size_t off = 0;
  const char *st, *en, *lp;
  if (b->unit_cls[u] >= 0) {
    const BatchClass &k = *b->classes[b->unit_cls[u]];
    off = (size_t)b->inst_member[i] * k.slice;
    env = &k.env;
    st = k.states.as<char>() + off;
    en = k.energies.as<char>() + off;
    lp = k.logp.as<char>() + off;
  } else {
    env = b->envs[i];
    st = b->states[i]->as<char>();
    en = b->energies[i]->as<char>();
    lp = b->logp[i]->as<char>();
  }
  int32_t nv = 0;
  SPG_HIP(hipMemcpy(&nv, (const char *)env->nvalid.p + off, 4, hipMemcpyDeviceToHost));
  *n_out = nv;
  if (nv > 0) {
    if (states_out)
      SPG_HIP(hipMemcpy(states_out, st, (size_t)nv * N * 4, hipMemcpyDeviceToDevice));
    if (energies_out) SPG_HIP(hipMemcpy(energies_out, en, (size_t)nv * 8, hipMemcpyDeviceToDevice));
    if (logp_out) SPG_HIP(hipMemcpy(logp_out, lp, (size_t)nv * 8, hipMemcpyDeviceToDevice));
  }
  if (log_Z) *log_Z = host_log_Z(env, off, pp->beta, pp->shift);
  return SPG_OK;
  SPG_CATCH
}

int spg_batch_set_tuning(spg_batch_t *b, int32_t i, int32_t gemm_tile) {
  if (!b || i < 0 || i >= b->n) return fail(SPG_ERR_INVALID, "spg_batch_set_tuning: bad batch or index");
  if (gemm_tile != 32 && gemm_tile != 64)
    return fail(SPG_ERR_INVALID, "spg_batch_set_tuning: gemm_tile must be 32 or 64");
  b->unit_tune[b->inst_unit[i]].gemm_tile = gemm_tile;
  b->drop_graph();
  return SPG_OK;
}

int spg_batch_tuning(const spg_batch_t *b, int32_t i, int32_t *gemm_tile, int32_t *mpo_columns,
                     int32_t *q_split) {
  if (!b || i < 0 || i >= b->n) return fail(SPG_ERR_INVALID, "spg_batch_tuning: bad batch or index");
  const Tuning &t = b->unit_tune[b->inst_unit[i]];
  if (gemm_tile) *gemm_tile = t.gemm_tile;
  if (mpo_columns) *mpo_columns = t.mpo_cols;
  if (q_split) *q_split = t.qform_split;
  return SPG_OK;
}

int spg_batch_autotune(spg_batch_t *b, void *stream, int32_t *tile_out) {
  SPG_TRY
  if (!b) return fail(SPG_ERR_INVALID, "spg_batch_autotune: null batch");
  hipStream_t s = (hipStream_t)stream;
  if (!b->warm) {
    enqueue_batch(b, s);
    SPG_HIP(hipStreamSynchronize(s));
    b->warm = true;
  }
  // every unit (a class or a single instance) timed twice per candidate (the
  // first run only warms); a greedy search over three knobs, each kept at its
  // fastest value before the next is tried: the GEMM tile (64, 32), then the
  // MPO d-index contraction form and the Q formation of one-panel QRs (each
  // form pair gives bitwise equal results)
  hipEvent_t e0, e1;
  SPG_HIP(hipEventCreate(&e0));
  SPG_HIP(hipEventCreate(&e1));
  try {
    auto time_unit = [&](size_t u) {
      float ms = 0.0f;
      for (int rep = 0; rep < 2; ++rep) {
        SPG_HIP(hipEventRecord(e0, s));
        enqueue_unit(b, (int)u, s);
        SPG_HIP(hipEventRecord(e1, s));
        SPG_HIP(hipEventSynchronize(e1));
        SPG_HIP(hipEventElapsedTime(&ms, e0, e1));
      }
      return ms;
    };
    for (size_t u = 0; u < b->unit_cls.size(); ++u) {
      Tuning &tu = b->unit_tune[u];
      int *knob[3] = {&tu.gemm_tile, &tu.mpo_cols, &tu.qform_split};
      const int cand[3][2] = {{64, 32}, {1, 0}, {1, 0}};
      for (int k = 0; k < 3; ++k) {
        float best = 1e30f;
        int best_v = cand[k][0];
        for (int v : cand[k]) {
          *knob[k] = v;
          const float ms = time_unit(u);
          if (ms < best) {
            best = ms;
            best_v = v;
          }
        }
        *knob[k] = best_v;
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->drop_graph();
  // refresh every instance's results with its chosen tiles
  enqueue_batch(b, s);
  SPG_HIP(hipStreamSynchronize(s));
  if (tile_out)
    for (int i = 0; i < b->n; ++i) tile_out[i] = b->unit_tune[b->inst_unit[i]].gemm_tile;
  return SPG_OK;
  SPG_CATCH
}

int spg_set_tuning(int32_t gemm_tile) {
  if (gemm_tile != 32 && gemm_tile != 64)
    return fail(SPG_ERR_INVALID, "spg_set_tuning: gemm_tile must be 32 or 64");
  g_tune.gemm_tile = gemm_tile;
  return SPG_OK;
}

int spg_set_gemm_precision(int32_t fp32_products) {
  if (fp32_products != 0 && fp32_products != 1)
    return fail(SPG_ERR_INVALID, "spg_set_gemm_precision: fp32_products must be 0 or 1");
  g_tune.gemm_f32 = fp32_products;
  return SPG_OK;
}

int spg_set_kernel_forms(int32_t mpo_columns, int32_t q_split) {
  if ((mpo_columns != 0 && mpo_columns != 1) || (q_split != 0 && q_split != 1))
    return fail(SPG_ERR_INVALID, "spg_set_kernel_forms: each switch must be 0 or 1");
  g_tune.mpo_cols = mpo_columns;
  g_tune.qform_split = q_split;
  return SPG_OK;
}

}  // extern "C"
