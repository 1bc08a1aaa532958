// Dense FP64 linear algebra for the boundary-MPS compression on gfx950:
// strided batched GEMM, Householder QR, one-sided Jacobi SVD of the small
// projected matrix, the SplitMix64 sketch and box normalisation.
#include <algorithm>
#include <cmath>

#include "spg_internal.h"
#include "wave.h"

namespace spg {

namespace {


// Block-wide sum; every thread receives the result.  `red` holds >= 16 doubles.
__device__ double block_sum(double v, double *red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += red[w];
  return t;
}

// Block-wide maximum of non-negative values; every thread receives it.
__device__ double block_max_nonneg(double v, double *red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_max_nonneg(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t = fmax(t, red[w]);
  return t;
}

// Squared tail norms below this lose digits to subnormal squares: the tail is
// then summed again divided by its largest entry (a column's tail shrinks to
// the rounding floor of the panel after a few reflections on graded panels).
constexpr double kTinySq = 1e-280;

// Householder reflector of a column with head al and tail x_i: the tail's
// squared norm is am^2 sg (sg summed from x_i / am; am = 1 on the plain
// path).  H = I - tau v v^T with v = 1 at the head and sc x_i below, R = beta.
__device__ __forceinline__ void householder(double al, double sg, double am, double &tj,
                                            double &sc, double &beta) {
  tj = 0.0; sc = 0.0; beta = al;
  if (sg != 0.0) {
    const double a = (am == 1.0) ? al : al / am;   // am = 1 unless the column was rescaled
    const double nrm = am * sqrt(a * a + sg);
    beta = (al >= 0.0) ? -nrm : nrm;
    const double x = al - beta;                     // |x| = |al| + nrm: no cancellation
    tj = -x / beta;                                 // (beta - al) / beta
    sc = 1.0 / x;                                   // independent of tj: the two overlap
  }
}

// ---------------------------------------------------------------- GEMM
// TILE x TILE output tile per 256-thread workgroup (TILE = 64 or 32), K staged
// through LDS in steps of kGemmKs (all of a step's loads are in flight at
// once: these products are short, so load latency rather than arithmetic
// sets their time); the products run on the matrix cores
// (v_mfma_f64_16x16x4f64).  Wavefront w owns the (TILE/2)^2 quadrant
// (w / 2, w % 2) of the tile as (TILE/32)^2 blocks of 16 x 16; per block and
// k step of 4, lane l supplies A[row l % 16][k + l / 16] and
// B[k + l / 16][col l % 16], and holds D[l / 16 + 4 q][l % 16], q = 0..3.
// The tile is picked per launch by the tuning.
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v_g __attribute__((ext_vector_type(4)));
constexpr int kGemmKs = 32;
// F32: the reduced-precision form, the staged FP64 operands rounded to FP32 at
// the product and accumulated in FP32 (v_mfma_f32_16x16x4f32, same operand
// layout; lane l holds D[4 (l / 16) + q][l % 16]); epilogue and output in FP64
template <int TILE, bool F32>
__device__ __forceinline__ void gemm_body(const GemmDesc &g) {
  constexpr int KS = kGemmKs, NQ = KS * TILE / 256;
  const int nbb = g.nb1 * g.nb2;
  const int inst = blockIdx.z / nbb, bz = blockIdx.z % nbb;   // class-batched instance
  const int b1 = bz / g.nb2, b2 = bz % g.nb2;
  const long io = (long)inst * g.ist;
  const double *A = (const double *)((const char *)g.A + io) + b1 * g.a_b1 + b2 * g.a_b2;
  const double *B = (const double *)((const char *)g.B + io) + b1 * g.b_b1 + b2 * g.b_b2;
  double *C = (double *)((char *)g.C + io) + b1 * g.c_b1 + b2 * g.c_b2;
  __shared__ double As[KS][TILE + 1];
  __shared__ double Bs[KS][TILE + 1];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.y * TILE, j0 = blockIdx.x * TILE;
  // split-K chunks: chunk b1 covers global k in [b1*K, min((b1+1)*K, kmax))
  const int Kend = (g.kmax > 0) ? min(g.K, g.kmax - b1 * g.K) : g.K;
  constexpr int NB = TILE / 32;                 // 16 x 16 blocks per quadrant side
  d4v macc[NB][NB];
  f4v_g macc32[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      macc[i][j] = (d4v){0.0, 0.0, 0.0, 0.0};
      macc32[i][j] = (f4v_g){0.f, 0.f, 0.f, 0.f};
    }
  const int lane = tid & 63, wq = tid >> 6;
  const int qr0 = (wq >> 1) * (TILE / 2), qc0 = (wq & 1) * (TILE / 2);
  // consecutive threads take consecutive addresses of whichever index has
  // unit stride, so tile loads are contiguous for either operand layout
  const bool a_rows = (g.a_i == 1 && g.a_k != 1);      // A column-major: i fastest
  const bool b_cols = (g.b_k == 1 && g.b_j != 1);      // B column-major: k fastest
  // every load of a step is issued before any is used, and the loads of the
  // next step are in flight while this one is multiplied: out-of-range
  // elements read a valid address (the operand's first element) and are
  // replaced by zero, so no branch separates the loads
  double va[NQ], vb[NQ];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tid + 256 * q;
      const int r = a_rows ? (e % TILE) : (e / KS), kk = a_rows ? (e / TILE) : (e % KS);
      const int gi = i0 + r, gk = k0 + kk;
      const bool oka = gi < g.M && gk < Kend;
      const double xa = A[oka ? (long)gi * g.a_i + (long)gk * g.a_k : 0L];
      va[q] = oka ? xa : 0.0;
      const int kb = b_cols ? (e % KS) : (e / TILE), cb = b_cols ? (e / KS) : (e % TILE);
      const int gkb = k0 + kb, gj = j0 + cb;
      const bool okb = gkb < Kend && gj < g.N;
      const double xb = B[okb ? (long)gkb * g.b_k + (long)gj * g.b_j : 0L];
      vb[q] = okb ? xb : 0.0;
    }
  };
  if (Kend > 0) fetch(0);
  for (int k0 = 0; k0 < Kend; k0 += KS) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tid + 256 * q;
      const int r = a_rows ? (e % TILE) : (e / KS), kk = a_rows ? (e / TILE) : (e % KS);
      As[kk][r] = va[q];
      const int kb = b_cols ? (e % KS) : (e / TILE), cb = b_cols ? (e / KS) : (e % TILE);
      Bs[kb][cb] = vb[q];
    }
    __syncthreads();
    if (k0 + KS < Kend) fetch(k0 + KS);
    const int kn = min(KS, Kend - k0);
    // rows kn..KS-1 of the staged step are not this step's: read as zero
    for (int kk = 0; kk < kn; kk += 4) {
      const int k = kk + (lane >> 4);
      const bool ok = k < kn;
      const int kr = ok ? k : 0;
      double a[NB], b[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const double x = As[kr][qr0 + 16 * i + (lane & 15)];
        a[i] = ok ? x : 0.0;
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const double x = Bs[kr][qc0 + 16 * j + (lane & 15)];
        b[j] = ok ? x : 0.0;
      }
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if constexpr (F32)
            macc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a[i], (float)b[j],
                                                                macc32[i][j], 0, 0, 0);
          else
            macc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], macc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  const double *sw = g.sw ? (const double *)((const char *)g.sw + io) : nullptr;
  const double *sV = g.sV ? (const double *)((const char *)g.sV + io) : nullptr;
  const int b1g = b1 + g.b1_base;               // the batch index over all launches
  const double fb = (g.smode == 2) ? sw[b1g] * sV[b1g * g.sd + b2] : 1.0;
  auto put = [&](int gi, int gj, double a) {
    if (gi >= g.M || gj >= g.N) return;
    double f = fb;
    if (g.smode == 1) {
      const int x = gi % g.sd;
      f = sw[x] * sV[x * g.sd + b1g];
    } else if (g.smode == 3) {
      f = sV[b2 * g.sd + gi % g.sd];
    } else if (g.smode == 4) {
      f = sV[(gi % g.sd) * g.sd + b2];
    }
    double *cp = C + gi * g.c_i + gj * g.c_j;
    double v = g.alpha * a;
    if (g.smode) v *= f;
    *cp = (g.beta != 0.0) ? v + g.beta * (*cp) : v;
  };
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if constexpr (F32)
          put(i0 + qr0 + 16 * i + 4 * (lane >> 4) + q, j0 + qc0 + 16 * j + (lane & 15),
              (double)macc32[i][j][q]);
        else
          put(i0 + qr0 + 16 * i + (lane >> 4) + 4 * q, j0 + qc0 + 16 * j + (lane & 15),
              macc[i][j][q]);
      }
}

template <int TILE>
__global__ __launch_bounds__(256) void k_gemm(GemmDesc g) {
  gemm_body<TILE, false>(g);
}
template <int TILE>
__global__ __launch_bounds__(256) void k_gemm_f32p(GemmDesc g) {
  gemm_body<TILE, true>(g);
}

// Deterministic split-K epilogue: C = alpha * sum_s P[s] + beta * C (P: [S][M][N]).
__global__ void k_splitk_reduce(int M, int N, int S, const double *P, double *C, long c_i,
                                long c_j, double alpha, double beta, long ist) {
  SPG_INST(P);
  SPG_INST(C);
  const unsigned e = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned mn = (unsigned)(M * N);
  if (e >= mn) return;
  // chunks summed in order, four loads in flight (clamped to the last chunk)
  double acc = 0.0;
  for (int s0 = 0; s0 < S; s0 += 4) {
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = P[(long)min(s0 + k, S - 1) * mn + e];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (s0 + k < S) acc += v[k];
  }
  const int i = (int)(e / N), j = (int)(e % N);
  double *cp = C + i * c_i + j * c_j;
  const double v = alpha * acc;
  *cp = (beta != 0.0) ? v + beta * (*cp) : v;
}

// ---------------------------------------------------------------- QR
// Householder QR in one workgroup (LAPACK dgeqrf/dorgqr conventions:
// H_j = I - tau_j v_j v_j^T, v_j[j] = 1).  The matrix is copied to a
// column-major workspace; Q is formed by backward accumulation.
__global__ __launch_bounds__(1024) void k_qr(int m, int n, const double *X, long xr, long xc,
                                            double *Qo, long qr, long qc, double *R,
                                            double *work, long ist) {
  SPG_INST(X);
  SPG_INST(Qo);
  SPG_INST(R);
  SPG_INST(work);
  double *W = work;                      // m x n column-major (v below diagonal, R above)
  double *Qw = work + (size_t)m * n;     // m x n column-major
  double *tau = work + 2 * (size_t)m * n;
  __shared__ double red[16];
  __shared__ double sh_tau, sh_scale, sh_beta;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  const size_t mn = (size_t)m * n;
  for (size_t e = tid; e < mn; e += blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    W[e] = X[i * xr + j * xc];
    Qw[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double *col = W + (size_t)j * m;
    double loc = 0.0;
    for (int i = j + 1 + tid; i < m; i += blockDim.x) loc += col[i] * col[i];
    double sig = block_sum(loc, red), am = 1.0;
    if (sig < kTinySq) {                         // uniform: every thread holds sig
      double mx = 0.0;
      for (int i = j + 1 + tid; i < m; i += blockDim.x) mx = fmax(mx, fabs(col[i]));
      am = block_max_nonneg(mx, red);
      loc = 0.0;
      if (am > 0.0)
        for (int i = j + 1 + tid; i < m; i += blockDim.x) {
          const double x = col[i] / am;
          loc += x * x;
        }
      sig = block_sum(loc, red);
      if (am == 0.0) am = 1.0;
    }
    if (tid == 0) {
      double t, sc, b;
      householder(col[j], sig, am, t, sc, b);
      sh_tau = t; sh_scale = sc; sh_beta = b;
    }
    __syncthreads();
    const double tj = sh_tau, sc = sh_scale;
    if (tj != 0.0)
      for (int i = j + 1 + tid; i < m; i += blockDim.x) col[i] *= sc;
    __syncthreads();
    if (tj != 0.0) {
      for (int k = j + 1 + wid; k < n; k += nw) {
        double *ck = W + (size_t)k * m;
        double dot = (lane == 0) ? ck[j] : 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) dot += col[i] * ck[i];
        dot = wave_sum(dot);
        const double f = tj * dot;
        if (lane == 0) ck[j] -= f;
        for (int i = j + 1 + lane; i < m; i += 64) ck[i] -= f * col[i];
      }
    }
    if (tid == 0) {
      col[j] = sh_beta;
      tau[j] = tj;
    }
    __syncthreads();
  }
  if (R != nullptr)
    for (int e = tid; e < n * n; e += blockDim.x) {
      const int i = e / n, j = e % n;
      R[e] = (i <= j) ? W[(size_t)j * m + i] : 0.0;
    }
  // Q = H_0 H_1 ... H_{n-1} [I; 0]
  for (int j = n - 1; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    const double *v = W + (size_t)j * m;
    for (int k = j + wid; k < n; k += nw) {
      double *qk = Qw + (size_t)k * m;
      double dot = (lane == 0) ? qk[j] : 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) dot += v[i] * qk[i];
      dot = wave_sum(dot);
      const double f = tj * dot;
      if (lane == 0) qk[j] -= f;
      for (int i = j + 1 + lane; i < m; i += 64) qk[i] -= f * v[i];
    }
    __syncthreads();
  }
  for (size_t e = tid; e < mn; e += blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    Qo[i * qr + j * qc] = Qw[e];
  }
}

// LDS-resident Householder QR of one row block (in place: factor, write R,
// then form Q over the reflectors as LAPACK dorg2r does).  Block b covers rows
// [b*mb, min(m, (b+1)*mb)); missing rows are zero.  R_b goes to Rs + b*n*n
// (row-major n x n), Q rows to Qo.
//
// Each wavefront owns trailing columns in turn, so one step costs strided
// passes over a few columns with wavefront DPP sums, and one barrier.  Writes that would race with the step's readers are
// deferred by a step: during the factorisation column j keeps its raw entries
// (every group rescales them on the fly) and is finalised (v_j scaled below
// the diagonal, beta_j on it) during step j+1, when nobody reads it; while Q
// is formed, column j is turned into H_j e_j during step j-1 by the group that
// then applies H_{j-1} to it.  Norms of the next pivot column come from the
// group that updates it (lookahead), one slot per column.
constexpr int kQrLds = 18432;   // doubles of LDS for the panel (144 KiB)
__global__ __launch_bounds__(1024) void k_qr_lds(int m, int n, int mb, const double *X, long xr,
                                                long xc, double *Qo, long qr, long qc, double *Rs,
                                                int want_q, long ist) {
  SPG_INST(X);
  SPG_INST(Qo);
  SPG_INST(Rs);
  __shared__ double W[kQrLds];
  __shared__ double tau[kMaxSketch + 32];
  __shared__ double sig2[kMaxSketch + 32];   // |column j below the diagonal|^2 before step j
  __shared__ double sam[kMaxSketch + 32];    // its scale: sig2 sums (x / sam)^2
  __shared__ double red[16];
  const int tid = threadIdx.x;
  const int grp = tid >> 6, l16 = tid & 63, ngrp = blockDim.x >> 6;
  const int r0 = blockIdx.x * mb;
  const int mr = min(mb, m - r0);          // real rows of this block
  const int ld = max(mr, n);               // rows in LDS (zero rows appended if short)
  for (int e = tid; e < ld * n; e += blockDim.x) {
    const int i = e % ld, j = e / ld;
    W[e] = (i < mr) ? X[(long)(r0 + i) * xr + (long)j * xc] : 0.0;
  }
  __syncthreads();
  {
    double loc = 0.0;
    for (int i = 1 + tid; i < ld; i += blockDim.x) loc += W[i] * W[i];
    double t = block_sum(loc, red), am = 1.0;
    if (t < kTinySq) {
      double mx = 0.0;
      for (int i = 1 + tid; i < ld; i += blockDim.x) mx = fmax(mx, fabs(W[i]));
      am = block_max_nonneg(mx, red);
      loc = 0.0;
      if (am > 0.0)
        for (int i = 1 + tid; i < ld; i += blockDim.x) {
          const double x = W[i] / am;
          loc += x * x;
        }
      t = block_sum(loc, red);
      if (am == 0.0) am = 1.0;
    }
    if (tid == 0) {
      sig2[0] = t;
      sam[0] = am;
    }
  }
  __syncthreads();
  // reflector of column j from its raw entries: H_j = I - tau v v^T with
  // v_j = 1, v_i = scale * col[i] (i > j), and R[j][j] = beta
  auto reflector = [&](int j, double &tj, double &sc, double &beta) {
    householder(W[j * ld + j], sig2[j], sam[j], tj, sc, beta);
  };
  for (int j = 0; j < n; ++j) {
    double tj, sc, beta;
    reflector(j, tj, sc, beta);
    const double *col = W + j * ld;
    for (int k = j + 1 + grp; k < n; k += ngrp) {
      double *ck = W + k * ld;
      if (tj != 0.0) {
        double dot = 0.0;
        for (int i = j + 1 + l16; i < ld; i += 64) dot += col[i] * ck[i];
        dot = ck[j] + sc * wave_sum(dot);
        const double f = tj * dot, fs = f * sc;
        if (l16 == 0) ck[j] -= f;
        for (int i = j + 1 + l16; i < ld; i += 64) ck[i] -= fs * col[i];
      }
      if (k == j + 1) {
        double a = 0.0, am = 1.0;
        for (int i = j + 2 + l16; i < ld; i += 64) a += ck[i] * ck[i];
        a = wave_sum(a);
        if (a < kTinySq) {
          double mx = 0.0;
          for (int i = j + 2 + l16; i < ld; i += 64) mx = fmax(mx, fabs(ck[i]));
          am = wave_max_nonneg(mx);
          a = 0.0;
          if (am > 0.0)
            for (int i = j + 2 + l16; i < ld; i += 64) {
              const double x = ck[i] / am;
              a += x * x;
            }
          a = wave_sum(a);
          if (am == 0.0) am = 1.0;
        }
        if (l16 == 0) {
          sig2[j + 1] = a;
          sam[j + 1] = am;
        }
      }
    }
    // finalise column j - 1 (nobody reads it any more)
    if (j > 0 && grp == ngrp - 1) {
      double tp, sp, bp;
      reflector(j - 1, tp, sp, bp);
      double *cp = W + (j - 1) * ld;
      for (int i = j + l16; i < ld; i += 64) cp[i] *= sp;
      if (l16 == 0) {
        tau[j - 1] = tp;
        cp[j - 1] = bp;
      }
    }
    __syncthreads();
  }
  if (tid < 64) {
    double tp, sp, bp;
    reflector(n - 1, tp, sp, bp);
    double *cp = W + (n - 1) * ld;
    for (int i = n + l16; i < ld; i += 64) cp[i] *= sp;
    if (l16 == 0) {
      tau[n - 1] = tp;
      cp[n - 1] = bp;
    }
  }
  __syncthreads();
  double *Rb = Rs + (long)blockIdx.x * n * n;
  for (int e = tid; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    Rb[e] = (i <= j) ? W[j * ld + i] : 0.0;
  }
  if (!want_q) return;
  __syncthreads();
  // Q = H_0 H_1 ... H_{n-1} [I; 0], backward: step j applies H_j to columns
  // j+1..; the group that takes column k = j+1 first turns it into
  // H_{j+1} e_{j+1} (its reflector is no longer read by anyone)
  auto to_unit = [&](int k) {
    double *ck = W + k * ld;
    const double tk = tau[k];
    for (int i = l16; i < ld; i += 64) {
      const double v = ck[i];
      ck[i] = (i < k) ? 0.0 : (i == k) ? 1.0 - tk : -tk * v;
    }
  };
  for (int j = n - 1; j >= 0; --j) {
    const double tj = tau[j];
    const double *v = W + j * ld;
    for (int k = j + 1 + grp; k < n; k += ngrp) {
      if (k == j + 1) to_unit(k);
      if (tj == 0.0) continue;
      double *ck = W + k * ld;
      double dot = 0.0;
      for (int i = j + 1 + l16; i < ld; i += 64) dot += v[i] * ck[i];
      dot = ck[j] + wave_sum(dot);
      const double f = tj * dot;
      if (l16 == 0) ck[j] -= f;
      for (int i = j + 1 + l16; i < ld; i += 64) ck[i] -= f * v[i];
    }
    __syncthreads();
  }
  if (tid < 64) to_unit(0);
  __syncthreads();
  for (int e = tid; e < mr * n; e += blockDim.x) {
    const int i = e % mr, j = e / mr;
    Qo[(long)(r0 + i) * qr + (long)j * qc] = W[j * ld + i];
  }
}

// ---------------------------------------------------------------- QR (registers)
// Householder QR of one panel of at most 64*RPL rows and 16*CPW columns in one
// workgroup of 16 wavefronts, held in registers: wave w owns columns
// [w*CPW, (w+1)*CPW) and lane l rows l + 64 t (t < RPL; zero beyond m).
//
// Factorisation, step j: every wave applies H_j = I - tau_j v_j v_j^T
// (published in an LDS slot) to its own columns k > j, a wave-wide dot product
// per column, then an axpy; the owner of column j+1 does that column first and
// publishes the next reflector before the step's one barrier.  Slot j mod
// kRegSlots is rewritten only after kRegSlots further barriers.
//
// Q = H_0 H_1 ... H_{n-1} [I; 0] is formed in place as LAPACK's dorg2r does
// (backwards; column j turns into H_j e_j once H_j has been applied to the
// columns right of it).  The reflectors never change, so they are published
// kRegSlots at a time and each wave then runs through the chunk on its own
// columns without further barriers.
//
// HBM traffic goes through LDS 64 rows at a time, in whichever order is
// contiguous for the strides given, so loads and stores are coalesced for
// row- and column-major panels alike.  The panel is scaled by a power of two
// (largest entry in [1/2, 1)) before the factorisation and R scaled back, so
// squared norms neither underflow nor overflow; Q does not depend on it.
constexpr int kRegSlots = 16;
constexpr int kStageLd = 65;                 // padded row count of the staging tile

template <int RPL, int CPW>
struct QrRegLds {
  static constexpr int kSlots = kRegSlots * 64 * RPL;
  static constexpr int kStage = 16 * CPW * kStageLd;
  static constexpr int kBuf = kSlots > kStage ? kSlots : kStage;
};

__device__ __forceinline__ double read_lane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Totals over the wave of the CPW per-lane partial sums (uniform results),
// four at a time.
template <int CPW>
__device__ __forceinline__ void wave_sums(const double (&d)[CPW], double (&out)[CPW]) {
  if constexpr (CPW == 1) {
    out[0] = wave_sum(d[0]);
  } else {
#pragma unroll
    for (int g = 0; g < CPW; g += 4) {
      const double r = wave_sum4(d[g], (g + 1 < CPW) ? d[(g + 1) % CPW] : 0.0,
                                 (g + 2 < CPW) ? d[(g + 2) % CPW] : 0.0,
                                 (g + 3 < CPW) ? d[(g + 3) % CPW] : 0.0);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (g + k < CPW) out[(g + k) % CPW] = read_lane(r, 16 * k);
    }
  }
}

template <int RPL, int CPW>
__global__ __launch_bounds__(1024) void k_qr_reg(int m, int n, int mb, const double *X, long xr,
                                                long xc, double *Qo, long qr, long qc, double *Rs,
                                                int want_q, double *Vq, double *Tq, long ist) {
  SPG_INST(X);
  SPG_INST(Qo);
  SPG_INST(Rs);
  SPG_INST(Vq);
  SPG_INST(Tq);
  // workgroup x factorises rows [x mb, min(m, (x+1) mb)) (one TSQR block;
  // mb = m for a single panel): its Q rows and its own n x n R
  {
    const int r0 = blockIdx.x * mb;
    m = min(mb, m - r0);
    X += (long)r0 * xr;
    if (Qo) Qo += (long)r0 * qr;
    if (Rs) Rs += (long)blockIdx.x * n * n;
  }
  __shared__ double buf[QrRegLds<RPL, CPW>::kBuf];
  __shared__ double taus[16 * CPW];
  __shared__ double red[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c0 = w * CPW;
  double a[CPW][RPL];

  // ---- load: column-major panels straight into registers (each wavefront
  // reads contiguous column segments); others 64 rows per pass through the
  // staging tile buf[j*kStageLd + r]
  const bool in_cols = (xc == 1) || (xr != 1 && (xc < 0 ? -xc : xc) < (xr < 0 ? -xr : xr));
  if (xr == 1) {
#pragma unroll
    for (int s = 0; s < CPW; ++s)
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int i = lane + 64 * t;
        a[s][t] = (i < m && c0 + s < n) ? X[(long)i + (long)(c0 + s) * xc] : 0.0;
      }
  } else
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r0 = 64 * t;
    if (r0 < m) {
      for (int e = tid; e < 64 * n; e += 1024) {
        int r, j;
        if (in_cols) { r = e / n; j = e - r * n; }
        else { j = e >> 6; r = e & 63; }
        const int i = r0 + r;
        buf[j * kStageLd + r] = (i < m) ? X[(long)i * xr + (long)j * xc] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < CPW; ++s)
      a[s][t] = (r0 < m && c0 + s < n) ? buf[(c0 + s) * kStageLd + lane] : 0.0;
    __syncthreads();
  }

  // ---- scale by a power of two so that the largest entry lies in [1/2, 1):
  // exact, and squared norms stay clear of underflow and overflow
  {
    double mx = 0.0;
#pragma unroll
    for (int s = 0; s < CPW; ++s)
#pragma unroll
      for (int t = 0; t < RPL; ++t) mx = fmax(mx, fabs(a[s][t]));
    mx = wave_max_nonneg(mx);
    if (lane == 0) red[w] = mx;
  }
  __syncthreads();
  int ex = 0;
  {
    double mx = 0.0;
    for (int v = 0; v < 16; ++v) mx = fmax(mx, red[v]);
    if (mx > 0.0 && mx <= 1.7e308) (void)frexp(mx, &ex);
  }
#pragma unroll
  for (int s = 0; s < CPW; ++s)
#pragma unroll
    for (int t = 0; t < RPL; ++t) a[s][t] = ldexp(a[s][t], -ex);

  // ---- factorisation, with lookahead: during step j the owner of column
  // j+1 applies H_j to that column first, then forms and publishes reflector
  // j+1 before updating its other columns, so the reflector's serial chain
  // overlaps the other wavefronts' updates and one barrier ends the step.
  //
  // Reflector of column jj (held in `col` by its owner): H = I - tau v v^T
  // with v = 1 at row jj, zero above, R[jj][jj] = beta; v goes to the LDS slot
  // of jj and into the column below the diagonal, tau to taus[jj].
  auto reflect = [&](double (&col)[RPL], int jj) {
    double sg = 0.0, at = 0.0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int i = lane + 64 * t;
      const double x = col[t];
      const double xm = (i > jj) ? x : 0.0;        // masked operand: the sum stays one chain
      sg = fma(xm, xm, sg);
      if (t == (jj >> 6)) at = x;
    }
    sg = wave_sum(sg);
    const double al = read_lane(at, jj & 63);
    double am = 1.0;
    if (sg < kTinySq) {                          // uniform over the wavefront
      double mx = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t)
        if (lane + 64 * t > jj) mx = fmax(mx, fabs(col[t]));
      am = wave_max_nonneg(mx);
      sg = 0.0;
      if (am > 0.0) {
#pragma unroll
        for (int t = 0; t < RPL; ++t)
          if (lane + 64 * t > jj) {
            const double x = col[t] / am;
            sg = fma(x, x, sg);
          }
      }
      sg = wave_sum(sg);
      if (am == 0.0) am = 1.0;
    }
    double tj, sc, beta;
    householder(al, sg, am, tj, sc, beta);
    double *vs = buf + (jj % kRegSlots) * (64 * RPL);
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int i = lane + 64 * t;
      const double v = (i < jj) ? 0.0 : (i == jj) ? 1.0 : col[t] * sc;
      vs[i] = v;
      if (i == jj) col[t] = beta;
      else if (i > jj) col[t] = v;
    }
    if (lane == 0) taus[jj] = tj;
  };
  if (w == 0) reflect(a[0], 0);          // column 0 belongs to wavefront 0
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double tj = taus[j];
    const double *vj = buf + (j % kRegSlots) * (64 * RPL);
    const int jn = j + 1;
    const int osn = (jn < n && w == jn / CPW) ? jn - c0 : -1;   // own slot of column j+1
    if (tj != 0.0 && max(c0, j + 1) < min(c0 + CPW, n)) {      // some own column k > j
      double v[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) v[t] = vj[lane + 64 * t];
      if (osn >= 0) {
#pragma unroll
        for (int s = 0; s < CPW; ++s) {
          if (s != osn) continue;
          double dt = 0.0;
#pragma unroll
          for (int t = 0; t < RPL; ++t) dt = fma(v[t], a[s][t], dt);
          const double f = -tj * wave_sum(dt);
#pragma unroll
          for (int t = 0; t < RPL; ++t) a[s][t] = fma(f, v[t], a[s][t]);
          reflect(a[s], jn);
        }
      }
      double dot[CPW];
#pragma unroll
      for (int s = 0; s < CPW; ++s) {
        dot[s] = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) dot[s] = fma(v[t], a[s][t], dot[s]);
      }
      double tot[CPW];
      wave_sums<CPW>(dot, tot);
#pragma unroll
      for (int s = 0; s < CPW; ++s) {
        if (s != osn && c0 + s > j && c0 + s < n) {
          const double f = -tj * tot[s];
#pragma unroll
          for (int t = 0; t < RPL; ++t) a[s][t] = fma(f, v[t], a[s][t]);
        }
      }
    } else if (osn >= 0) {
      // H_j is the identity here: only the next reflector
#pragma unroll
      for (int s = 0; s < CPW; ++s)
        if (s == osn) reflect(a[s], jn);
    }
    __syncthreads();
  }

  // ---- R (row-major n x n), through the staging tile
  if (Rs) {
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      if (64 * t < n) {
        __syncthreads();
#pragma unroll
        for (int s = 0; s < CPW; ++s)
          if (c0 + s < n) buf[(c0 + s) * kStageLd + lane] = a[s][t];
        __syncthreads();
        for (int e = tid; e < 64 * n; e += 1024) {
          const int r = e / n, j = e - r * n, i = 64 * t + r;
          if (i < n) Rs[(long)i * n + j] = (i <= j) ? ldexp(buf[j * kStageLd + r], ex) : 0.0;
        }
      }
    }
  }
  if (!want_q) return;
  if (Vq) {
    // Q formed by k_qform: the reflectors (column-major m x n, rows below the
    // diagonal; the rest is not read) and the taus
#pragma unroll
    for (int s = 0; s < CPW; ++s)
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int i = lane + 64 * t;
        if (i < m && c0 + s < n) Vq[(long)i + (long)(c0 + s) * m] = a[s][t];
      }
    if (tid < n) Tq[tid] = taus[tid];
    return;
  }

  // ---- Q in place, reflectors published kRegSlots at a time
  for (int lo = ((n - 1) / kRegSlots) * kRegSlots; lo >= 0; lo -= kRegSlots) {
    const int hi = min(n, lo + kRegSlots);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < CPW; ++s) {
      const int c = c0 + s;
      if (c >= lo && c < hi) {
        double *vc = buf + (c - lo) * (64 * RPL);
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int i = lane + 64 * t;
          vc[i] = (i < c) ? 0.0 : (i == c) ? 1.0 : a[s][t];
        }
      }
    }
    __syncthreads();
    if (c0 >= n || c0 + CPW - 1 < lo) continue;      // no own column is touched by this chunk
    for (int j = hi - 1; j >= lo; --j) {
      const double tj = taus[j];
      const double *vj = buf + (j - lo) * (64 * RPL);
      if (tj != 0.0 && max(c0, j + 1) < min(c0 + CPW, n)) {
        double v[RPL];
#pragma unroll
        for (int t = 0; t < RPL; ++t) v[t] = vj[lane + 64 * t];
        double dot[CPW];
#pragma unroll
        for (int s = 0; s < CPW; ++s) {
          dot[s] = 0.0;
#pragma unroll
          for (int t = 0; t < RPL; ++t) dot[s] = fma(v[t], a[s][t], dot[s]);
        }
        double tot[CPW];
        wave_sums<CPW>(dot, tot);
#pragma unroll
        for (int s = 0; s < CPW; ++s) {
          if (c0 + s > j && c0 + s < n) {
            const double f = -tj * tot[s];
#pragma unroll
            for (int t = 0; t < RPL; ++t) a[s][t] = fma(f, v[t], a[s][t]);
          }
        }
      }
#pragma unroll
      for (int s = 0; s < CPW; ++s) {
        if (c0 + s == j) {
#pragma unroll
          for (int t = 0; t < RPL; ++t) {
            const int i = lane + 64 * t;
            a[s][t] = (i < j) ? 0.0 : (i == j) ? 1.0 - tj : -tj * a[s][t];
          }
        }
      }
    }
  }

  // ---- store Q: column-major straight from registers, others 64 rows per pass
  const bool out_cols = (qc == 1) || (qr != 1 && (qc < 0 ? -qc : qc) < (qr < 0 ? -qr : qr));
  if (qr == 1) {
#pragma unroll
    for (int s = 0; s < CPW; ++s)
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int i = lane + 64 * t;
        if (i < m && c0 + s < n) Qo[(long)i + (long)(c0 + s) * qc] = a[s][t];
      }
    return;
  }
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r0 = 64 * t;
    if (r0 < m) {
      __syncthreads();
#pragma unroll
      for (int s = 0; s < CPW; ++s)
        if (c0 + s < n) buf[(c0 + s) * kStageLd + lane] = a[s][t];
      __syncthreads();
      for (int e = tid; e < 64 * n; e += 1024) {
        int r, j;
        if (out_cols) { r = e / n; j = e - r * n; }
        else { j = e >> 6; r = e & 63; }
        const int i = r0 + r;
        if (i < m) Qo[(long)i * qr + (long)j * qc] = buf[j * kStageLd + r];
      }
    }
  }
}

// Q of a register-kernel panel from its stored reflectors, one wavefront per
// column and four columns per workgroup (so the columns' chains run on
// kQformCols-wide groups of compute units): column c is H_c e_c, then H_j
// applied for j = c-1 down to 0, each as a dot product with v_j, its total
// over the wavefront and an update, exactly as the panel kernel's own Q
// formation does it.  The total is taken in the slot c % CPW of the panel
// kernel's batched sums (the other slots zero; each slot's total depends on
// that slot alone), so Q is bitwise the panel kernel's.  The reflectors pass
// through LDS kRegSlots at a time, the next chunk's loads in flight while the
// current chunk is applied.  Column-major output, m <= 64 RPL.
constexpr int kQformCols = 4;
template <int RPL, int CPW>
__global__ __launch_bounds__(64 * kQformCols) void k_qform(int m, int n, const double *Vq,
                                                           const double *Tq, double *Qo, long qc,
                                                           long ist) {
  SPG_INST(Vq);
  SPG_INST(Tq);
  SPG_INST(Qo);
  constexpr int kChunk = kRegSlots * 64 * RPL;              // doubles of one chunk
  constexpr int kPer = kChunk / (64 * kQformCols);          // per thread
  __shared__ double vbuf[kChunk];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int cw0 = blockIdx.x * kQformCols;
  const int c = cw0 + w, slot = c % CPW;
  const int ctop = min(n, cw0 + kQformCols) - 1;            // highest column of the group
  // raw loads of chunk [lo, lo + kRegSlots): element e = jj * 64 RPL + i of
  // reflector lo + jj (a valid address where the row is not read)
  auto fetch = [&](int lo, double (&raw)[kPer]) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + 64 * kQformCols * k;
      const int jj = e / (64 * RPL), i = e % (64 * RPL), j = lo + jj;
      raw[k] = Vq[(j <= ctop && i > j && i < m) ? (long)i + (long)j * m : 0L];
    }
  };
  auto publish = [&](int lo, const double (&raw)[kPer]) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + 64 * kQformCols * k;
      const int jj = e / (64 * RPL), i = e % (64 * RPL), j = lo + jj;
      vbuf[e] = (i < j) ? 0.0 : (i == j) ? 1.0 : (i < m ? raw[k] : 0.0);
    }
  };
  double q[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) q[t] = 0.0;
  double raw[kPer];
  int lo = (ctop / kRegSlots) * kRegSlots;
  fetch(lo, raw);
  for (; lo >= 0; lo -= kRegSlots) {
    const int hi = min(ctop + 1, lo + kRegSlots);
    __syncthreads();
    publish(lo, raw);
    __syncthreads();
    if (lo >= kRegSlots) fetch(lo - kRegSlots, raw);        // next chunk, in flight
    if (c > ctop) continue;
    for (int j = hi - 1; j >= lo; --j) {
      if (j > c) continue;
      const double tj = Tq[j];
      const double *vj = vbuf + (j - lo) * (64 * RPL);
      double v[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) v[t] = vj[lane + 64 * t];
      if (j == c) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int i = lane + 64 * t;
          q[t] = (i < j) ? 0.0 : (i == j) ? 1.0 - tj : -tj * v[t];
        }
      } else if (tj != 0.0) {
        double dot[CPW], tot[CPW];
        double dt = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) dt = fma(v[t], q[t], dt);
#pragma unroll
        for (int k = 0; k < CPW; ++k) dot[k] = (k == slot) ? dt : 0.0;
        wave_sums<CPW>(dot, tot);
        double tk = 0.0;
#pragma unroll
        for (int k = 0; k < CPW; ++k)
          if (k == slot) tk = tot[k];
        const double f = -tj * tk;
#pragma unroll
        for (int t = 0; t < RPL; ++t) q[t] = fma(f, v[t], q[t]);
      }
    }
  }
  if (c > ctop) return;
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int i = lane + 64 * t;
    if (i < m) Qo[(long)i + (long)c * qc] = q[t];
  }
}

// ---------------------------------------------------------------- Jacobi SVD
// Right singular vectors of an upper-triangular l x l factor R (row-major):
// one-sided (Hestenes) Jacobi orthogonalises the columns of R^T (faster than
// R's own columns for a triangular factor); R^T J = X Sigma gives the wanted
// vectors as the normalised columns of X, so no rotations are accumulated.
// R is first scaled by a power of two so that its largest entry lies in
// [1/2, 1) (exact, and it keeps squared column norms and their products far
// from underflow at the tiny scales two-site blocks can have).  Round-robin pair ordering, one
// 16-lane DPP row per pair, so a round of up to 48 pairs is one pass and its
// sums need no LDS.
//
// After convergence every pair of columns above the rounding floor passed the
// rotation test, so only the floor columns (never rotated, last in sorted
// order) can fail orthonormality: the first of them is the first failing
// column i0 (without convergence the sorted columns are checked to 1e-13).
// Then columns i0.. are re-orthonormalised by CGS2 in sorted order, with a
// deterministic completion from the unit vectors for columns that lose their
// norm, so the kk returned vectors are always orthonormal.
constexpr int kJacRows = kMaxSketch / 16;     // most rows per lane of a pair group

// NR = rows per lane of a pair group, ceil(l / 16)
template <int NR>
__global__ __launch_bounds__(1024) void k_jacobi(int l, int kk, const double *Rm, double *Vo,
                                                double *sig, long ist) {
  SPG_INST(Rm);
  SPG_INST(Vo);
  SPG_INST(sig);
  __shared__ double W[kMaxSketch * kMaxSketch];
  __shared__ double V[kMaxSketch * kMaxSketch];
  __shared__ double nrm[kMaxSketch];
  __shared__ double snrm[kMaxSketch];
  __shared__ double hbuf[kMaxSketch];
  __shared__ int rotated, bad, first_bad;
  __shared__ double sh_fro, sh_nv;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  // W column-major with column j = row j of R, i.e. W = R^T (same storage as
  // Rm), times 2^-e with max |R_ij| = m 2^e, 1/2 <= m < 1
  double mx = 0.0;
  for (int e = tid; e < l * l; e += blockDim.x) {
    const double x = Rm[e];
    W[e] = x;
    mx = fmax(mx, fabs(x));
  }
  mx = wave_max_nonneg(mx);
  if (lane == 0) hbuf[wid] = mx;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int v = 0; v < nw; ++v) t = fmax(t, hbuf[v]);
    sh_nv = t;
  }
  __syncthreads();
  int ex = 0;
  if (sh_nv > 0.0 && sh_nv <= 1.7e308) (void)frexp(sh_nv, &ex);
  double ss = 0.0;
  for (int e = tid; e < l * l; e += blockDim.x) {
    const double x = ldexp(W[e], -ex);
    W[e] = x;
    ss = fma(x, x, ss);
  }
  const int le = (l + 1) & ~1;
  ss = block_sum(ss, hbuf);
  if (tid == 0) sh_fro = ss;
  __syncthreads();
  // columns below 1e-13 |R|_F sit at the rounding floor of the range finder's
  // projection: rotating them only shuffles noise
  const double tiny = 1e-26 * sh_fro;
  const int grp = tid >> 4, r16 = tid & 15, ngrp = blockDim.x >> 4;
  const int np = le / 2, nc = le - 1;
  bool converged = false;
  for (int sweep = 0; sweep < 30; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int t = 0; t < nc; ++t) {
      for (int k = grp; k < np; k += ngrp) {
        int p, q;
        if (k == 0) { p = t; q = nc; }
        else {
          p = t + k; if (p >= nc) p -= nc;
          q = t - k; if (q < 0) q += nc;
        }
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        if (q >= l) continue;
        double x[NR], y[NR];
        double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
        for (int h = 0; h < NR; ++h) {
          const int r = r16 + 16 * h;
          x[h] = (r < l) ? W[p * l + r] : 0.0;
          y[h] = (r < l) ? W[q * l + r] : 0.0;
          a = fma(x[h], x[h], a);
          b = fma(y[h], y[h], b);
          g = fma(x[h], y[h], g);
        }
        a = row16_sum(a);
        b = row16_sum(b);
        g = row16_sum(g);
        if (a > tiny && b > tiny && g * g > 1e-28 * (a * b)) {
          // tan of the rotation angle is t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2))
          // with zeta = (b - a) / 2g; multiplied through by 2|g| it is
          // t = g2 / den, g2 = sgn(b - a) 2g, den = |b - a| + sqrt((b - a)^2 + 4g^2),
          // so cos = den / sqrt(den^2 + g2^2) and sin = g2 / sqrt(den^2 + g2^2):
          // no division (the prescaling keeps the squares in range)
          const double dd = b - a;
          const double g2 = (dd >= 0.0) ? 2.0 * g : -2.0 * g;
          const double den = fabs(dd) + sqrt(fma(dd, dd, g2 * g2));
          const double hn = rsqrt(fma(den, den, g2 * g2));
          const double cs = den * hn, sn = g2 * hn;
#pragma unroll
          for (int h = 0; h < NR; ++h) {
            const int r = r16 + 16 * h;
            if (r < l) {
              W[p * l + r] = cs * x[h] - sn * y[h];
              W[q * l + r] = sn * x[h] + cs * y[h];
            }
          }
          if (r16 == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (rotated == 0) {
      converged = true;
      break;
    }
    __syncthreads();
  }
  for (int j = wid; j < l; j += nw) {
    double a = 0.0;
    for (int r = lane; r < l; r += 64) a += W[j * l + r] * W[j * l + r];
    a = wave_sum(a);
    if (lane == 0) nrm[j] = sqrt(a);
  }
  __syncthreads();
  // sorted, normalised columns into V (column-major)
  for (int j = wid; j < l; j += nw) {
    const double nj = nrm[j];
    int rank = 0;
    for (int base = 0; base < l; base += 64) {
      const int i = base + lane;
      const bool before = (i < l) && (nrm[i] > nj || (nrm[i] == nj && i < j));
      rank += __popcll(__ballot(before));
    }
    const double inv = (nrm[j] > 0.0) ? 1.0 / nrm[j] : 0.0;
    for (int r = lane; r < l; r += 64) V[rank * l + r] = W[j * l + r] * inv;
    if (lane == 0) {
      sig[rank] = ldexp(nrm[j], ex);
      snrm[rank] = nrm[j];
    }
  }
  if (tid == 0) {
    bad = 0;
    first_bad = kk;
  }
  __syncthreads();
  if (converged) {
    // every pair of columns above the rounding floor passed the rotation test
    // (|cos| <= 1e-14): only columns at the floor, never rotated, can fail the
    // check, and in sorted order they come last.  The first of them (norm^2
    // within twice the floor) starts the tail.
    if (wid == 0) {
      int fb = kk;
      for (int base = 0; base < kk && fb == kk; base += 64) {
        const int j = base + lane;
        const unsigned long long hit = __ballot(j < kk && snrm[j] * snrm[j] <= 2.0 * tiny);
        if (hit) fb = base + __ffsll((long long)hit) - 1;
      }
      if (lane == 0 && fb < kk) {
        bad = 1;
        first_bad = fb;
      }
    }
  } else {
    // only the leading kk columns are used: check those
    for (int e = wid; e < kk * kk; e += nw) {
      const int i = e / kk, j = e % kk;
      if (j > i) continue;
      double g = 0.0;
      for (int r = lane; r < l; r += 64) g += V[i * l + r] * V[j * l + r];
      g = wave_sum(g);
      if (lane == 0 && fabs(g - (i == j ? 1.0 : 0.0)) > 1e-13) {
        bad = 1;
        atomicMin(&first_bad, i);
      }
    }
  }
  __syncthreads();
  if (bad) {
    // CGS2 in sorted order from the first failing column (the ones before it
    // are orthonormal to the rotation test's tolerance and stay as they are);
    // a column that loses its norm is replaced by the first unit vector that
    // survives the projection
    for (int i = first_bad; i < kk; ++i) {
      int cand = -1;
      for (;;) {
        for (int pass = 0; pass < 2; ++pass) {
          for (int j = wid; j < i; j += nw) {
            double g = 0.0;
            for (int r = lane; r < l; r += 64) g += V[j * l + r] * V[i * l + r];
            g = wave_sum(g);
            if (lane == 0) hbuf[j] = g;
          }
          __syncthreads();
          for (int r = tid; r < l; r += blockDim.x) {
            double acc = V[i * l + r];
            for (int j = 0; j < i; ++j) acc -= hbuf[j] * V[j * l + r];
            V[i * l + r] = acc;
          }
          __syncthreads();
        }
        if (wid == 0) {
          double a = 0.0;
          for (int r = lane; r < l; r += 64) a += V[i * l + r] * V[i * l + r];
          a = wave_sum(a);
          if (lane == 0) sh_nv = sqrt(a);
        }
        __syncthreads();
        const double nv = sh_nv;
        // after two Gram-Schmidt passes a remainder of norm 1e-3 is orthogonal
        // to the earlier columns to ~u / 1e-3; below that, try the next unit
        // vector (the columns at the rounding floor are noise whose
        // remainders after ~60 projections are ~0.4: a stricter bound sent
        // most of them to the unit-vector loop)
        if (nv > 1e-3 || cand >= l - 1) {
          const double inv = (nv > 0.0) ? 1.0 / nv : 0.0;
          for (int r = tid; r < l; r += blockDim.x) V[i * l + r] *= inv;
          __syncthreads();
          break;
        }
        ++cand;
        for (int r = tid; r < l; r += blockDim.x) V[i * l + r] = (r == cand) ? 1.0 : 0.0;
        __syncthreads();
      }
    }
  }
  for (int e = tid; e < l * l; e += blockDim.x) {
    const int r = e / l, c = e % l;      // Vo row-major
    Vo[e] = V[c * l + r];
  }
}

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t idx) {
  uint64_t z = seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_sketch(int n, int l, double *Om, long ist) {
  SPG_INST(Om);
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * l) return;
  const long i = e / l, j = e % l;
  const uint64_t z = splitmix64_at(0x5EED5EED12345678ull, (uint64_t)(i * 1024 + j));
  Om[e] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

// Box normalisation in two launches: per-block partial sums of squares (a
// fixed block count and order); the last block to finish (found through a
// release fence and an atomic counter in the scratch) folds them in a fixed
// order and writes the log-scale and 1/norm, then resets the counter; a
// second launch rescales.  Each thread keeps four loads in flight.
constexpr int kNormBlocks = 1024;
constexpr int kNormInv = kNormBlocks, kNormCount = kNormBlocks + 1;   // scratch slots
static_assert(kNormScratch >= kNormBlocks + 2, "normalisation scratch too small");

__device__ __forceinline__ long box_offset(unsigned e, unsigned n1, unsigned n2, unsigned n3,
                                           long s0, long s1, long s2, long s3) {
  const unsigned i3 = e % n3; e /= n3;
  const unsigned i2 = e % n2; e /= n2;
  const unsigned i1 = e % n1; const unsigned i0 = e / n1;
  return (long)i0 * s0 + (long)i1 * s1 + (long)i2 * s2 + (long)i3 * s3;
}

__global__ __launch_bounds__(256) void k_box_sumsq(const double *T, unsigned tot, unsigned n1,
                                                   unsigned n2, unsigned n3, long s0, long s1,
                                                   long s2, long s3, double *scr, double *logs,
                                                   int out, int in, long ist) {
  SPG_INST(T);
  SPG_INST(scr);
  SPG_INST(logs);
  __shared__ double red[16];
  __shared__ int last;
  const unsigned stride = gridDim.x * blockDim.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  unsigned e = blockIdx.x * blockDim.x + threadIdx.x;
  for (; e + 3 * stride < tot; e += 4 * stride) {
    const double v0 = T[box_offset(e, n1, n2, n3, s0, s1, s2, s3)];
    const double v1 = T[box_offset(e + stride, n1, n2, n3, s0, s1, s2, s3)];
    const double v2 = T[box_offset(e + 2 * stride, n1, n2, n3, s0, s1, s2, s3)];
    const double v3 = T[box_offset(e + 3 * stride, n1, n2, n3, s0, s1, s2, s3)];
    a0 = fma(v0, v0, a0);
    a1 = fma(v1, v1, a1);
    a2 = fma(v2, v2, a2);
    a3 = fma(v3, v3, a3);
  }
  for (; e < tot; e += stride) {
    const double v = T[box_offset(e, n1, n2, n3, s0, s1, s2, s3)];
    a0 = fma(v, v, a0);
  }
  const double t = block_sum((a0 + a1) + (a2 + a3), red);
  unsigned *cnt = (unsigned *)(scr + kNormCount);
  if (threadIdx.x == 0) {
    scr[blockIdx.x] = t;
    __threadfence();
    last = (atomicAdd(cnt, 1u) == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double acc = 0.0;
  for (unsigned i = threadIdx.x; i < gridDim.x; i += blockDim.x) acc += scr[i];
  const double ss = block_sum(acc, red);
  if (threadIdx.x == 0) {
    const double nr = sqrt(ss);
    scr[kNormInv] = (nr > 0.0) ? 1.0 / nr : 1.0;
    logs[out] = (in >= 0 ? logs[in] : 0.0) + (nr > 0.0 ? log(nr) : 0.0);
    *cnt = 0u;
  }
}

__global__ __launch_bounds__(256) void k_box_scale(double *T, unsigned tot, unsigned n1,
                                                   unsigned n2, unsigned n3, long s0, long s1,
                                                   long s2, long s3, const double *scr, long ist) {
  SPG_INST(T);
  SPG_INST(scr);
  const double f = scr[kNormInv];
  const unsigned stride = gridDim.x * blockDim.x;
  unsigned e = blockIdx.x * blockDim.x + threadIdx.x;
  for (; e + 3 * stride < tot; e += 4 * stride) {
    const long o0 = box_offset(e, n1, n2, n3, s0, s1, s2, s3);
    const long o1 = box_offset(e + stride, n1, n2, n3, s0, s1, s2, s3);
    const long o2 = box_offset(e + 2 * stride, n1, n2, n3, s0, s1, s2, s3);
    const long o3 = box_offset(e + 3 * stride, n1, n2, n3, s0, s1, s2, s3);
    const double v0 = T[o0], v1 = T[o1], v2 = T[o2], v3 = T[o3];
    T[o0] = v0 * f;
    T[o1] = v1 * f;
    T[o2] = v2 * f;
    T[o3] = v3 * f;
  }
  for (; e < tot; e += stride) {
    const long o = box_offset(e, n1, n2, n3, s0, s1, s2, s3);
    T[o] *= f;
  }
}

__global__ void k_copy(double *dst, const double *src, size_t n, long ist) {
  SPG_INST(dst);
  SPG_INST(src);
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e < n) dst[e] = src[e];
}

__global__ void k_fill_zero(double *p, size_t n, long ist) {
  SPG_INST(p);
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e < n) p[e] = 0.0;
}

}  // namespace

thread_local Tuning g_tune;

template <int TILE, bool F32>
static void gemm_launch(const GemmDesc &g, hipStream_t s) {
  const long tiles = (long)((g.N + TILE - 1) / TILE) * ((g.M + TILE - 1) / TILE) * g.nb1 * g.nb2;
  if (g_tune.splitk && g.ws && tiles < 64 && g.nb1 * g.nb2 == 1 && g.K >= 256) {
    // few output tiles and a long K: split K into chunks of >= 64 written to
    // a workspace, then sum them in a fixed order
    int S = (int)std::min<long>(std::min<long>(g.K / 64, 128 / tiles), 16);
    while (S > 1 && (size_t)S * g.M * g.N > g.ws_len) --S;
    if (S > 1) {
      const int kc = ((g.K + S - 1) / S + 15) / 16 * 16;
      S = (g.K + kc - 1) / kc;
      GemmDesc h = g;
      h.nb1 = S; h.nb2 = 1;
      h.K = kc;
      h.a_b1 = kc * g.a_k; h.b_b1 = kc * g.b_k;
      h.C = g.ws; h.c_i = g.N; h.c_j = 1; h.c_b1 = (long)g.M * g.N;
      h.alpha = 1.0; h.beta = 0.0; h.kmax = g.K;
      dim3 grid((h.N + TILE - 1) / TILE, (h.M + TILE - 1) / TILE, S * g_bc.n);
      if constexpr (F32)
        hipLaunchKernelGGL(k_gemm_f32p<TILE>, grid, dim3(256), 0, s, h);
      else
        hipLaunchKernelGGL(k_gemm<TILE>, grid, dim3(256), 0, s, h);
      SPG_CHECK_LAUNCH();
      const long mn = (long)g.M * g.N;
      hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((mn + 255) / 256), g_bc.n), dim3(256), 0,
                         s, g.M, g.N, S, g.ws, g.C, g.c_i, g.c_j, g.alpha, g.beta, g_bc.ist);
      SPG_CHECK_LAUNCH();
      return;
    }
  }
  dim3 grid((g.N + TILE - 1) / TILE, (g.M + TILE - 1) / TILE, g.nb1 * g.nb2 * g_bc.n);
  if constexpr (F32)
    hipLaunchKernelGGL(k_gemm_f32p<TILE>, grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL(k_gemm<TILE>, grid, dim3(256), 0, s, g);
  SPG_CHECK_LAUNCH();
}

void gemm_f64(const GemmDesc &g, hipStream_t s) {
  KTimer kt_(g.cls ? g.cls : "gemm_f64", s, 2.0 * g.M * g.N * g.K * g.nb1 * g.nb2);
  if (g.M <= 0 || g.N <= 0 || g.nb1 <= 0 || g.nb2 <= 0) return;
  SPG_BC(g.A);
  SPG_BC(g.B);
  SPG_BC(g.C);
  SPG_BC(g.ws);
  SPG_BC(g.sw);
  SPG_BC(g.sV);
  if (g.smode != 0 && (g.sw == nullptr || g.sV == nullptr || g.sd <= 0 || g.ws != nullptr)) {
    set_error("gemm_f64: epilogue factor needs both tables and no split-K workspace");
    throw Fail{SPG_ERR_INVALID};
  }
  GemmDesc h = g;
  h.ist = g_bc.ist;
  const bool t32 = (g.tile ? g.tile : g_tune.gemm_tile) == 32;
  auto launch = [&](const GemmDesc &k) {
    if (g_tune.gemm_f32) {
      if (t32) gemm_launch<32, true>(k, s);
      else gemm_launch<64, true>(k, s);
    } else {
      if (t32) gemm_launch<32, false>(k, s);
      else gemm_launch<64, false>(k, s);
    }
  };
  const long per_b1 = (long)h.nb2 * g_bc.n;      // grid z entries per first batch index
  if ((long)h.nb1 * per_b1 <= 65535) {
    launch(h);
    return;
  }
  // more batches than one launch's grid holds: launches over runs of the first
  // batch index (each batch's tiles are computed as in one launch)
  const long run = 65535 / per_b1;
  if (run < 1 || g.kmax != 0) {
    set_error("gemm_f64: batch too large for one launch");
    throw Fail{SPG_ERR_UNSUPPORTED};
  }
  for (long c0 = 0; c0 < g.nb1; c0 += run) {
    GemmDesc k = h;
    k.nb1 = (int)std::min<long>(run, g.nb1 - c0);
    k.A = g.A + c0 * g.a_b1;
    k.B = g.B + c0 * g.b_b1;
    k.C = g.C + c0 * g.c_b1;
    k.b1_base = (int)c0;
    k.ws = nullptr;                               // no split-K: every batch as in one launch
    k.ws_len = 0;
    launch(k);
  }
}

// Householder QR flops: 2mn^2 - 2n^3/3 for R, the same again to form Q.
static double qr_flops(int m, int n, int want_q) {
  const double r = 2.0 * m * n * n - 2.0 * n * n * n / 3.0;
  return want_q ? 2.0 * r : r;
}

size_t qr_work_doubles(int m, int n) {
  return 3 * (size_t)m * n + 2 * (size_t)kQrLds + 2 * (size_t)n * n + n + 64;
}

// Register-resident panels: up to 512 rows (8 per lane) and 80 columns (5 per
// wavefront).
constexpr int kQrRegRows = 512, kQrRegCols = 80;

template <int RPL>
static void qr_reg_rows(int cpw, int m, int n, int mb, const double *X, long xr, long xc,
                        double *Q, long qr, long qc, double *R, int want_q, dim3 grid, long ist,
                        hipStream_t s, double *Vq = nullptr, double *Tq = nullptr) {
  // with Vq and Tq (one panel, column-major Q): the panel kernel stores the
  // reflectors and k_qform forms Q, a compute unit per column
#define SPG_QR_REG(C)                                                                         \
  case C:                                                                                      \
    {                                                                                          \
      KTimer kt_("qr_f64", s, qr_flops(m, n, want_q && !Vq));                                  \
      hipLaunchKernelGGL((k_qr_reg<RPL, C>), grid, dim3(1024), 0, s, m, n, mb, X, xr, xc, Q,   \
                         qr, qc, R, want_q, Vq, Tq, ist);                                      \
      SPG_CHECK_LAUNCH();                                                                      \
    }                                                                                          \
    if (Vq) {                                                                                  \
      KTimer kt_("qform_f64", s, qr_flops(m, n, 1) - qr_flops(m, n, 0));                        \
      hipLaunchKernelGGL((k_qform<RPL, C>), dim3((n + kQformCols - 1) / kQformCols, grid.y),   \
                         dim3(64 * kQformCols), 0, s, m, n, Vq, Tq, Q, qc, ist);               \
    }                                                                                          \
    break;
  switch (cpw) {
    SPG_QR_REG(1)
    SPG_QR_REG(2)
    SPG_QR_REG(3)
    SPG_QR_REG(4)
    SPG_QR_REG(5)
    default:
      set_error("qr_f64: register panel too wide");
      throw Fail{SPG_ERR_UNSUPPORTED};
  }
#undef SPG_QR_REG
  SPG_CHECK_LAUNCH();
}

// grid.x workgroups, each factorising mb rows of the panel (the last one the
// rest); the rows per lane are set by mb
static void qr_reg(int m, int n, int mb, const double *X, long xr, long xc, double *Q, long qr,
                   long qc, double *R, int want_q, dim3 grid, long ist, hipStream_t s,
                   double *Vq = nullptr, double *Tq = nullptr) {
  const int cpw = (n + 15) / 16;
  if (mb <= 64)
    qr_reg_rows<1>(cpw, m, n, mb, X, xr, xc, Q, qr, qc, R, want_q, grid, ist, s, Vq, Tq);
  else if (mb <= 128)
    qr_reg_rows<2>(cpw, m, n, mb, X, xr, xc, Q, qr, qc, R, want_q, grid, ist, s, Vq, Tq);
  else if (mb <= 256)
    qr_reg_rows<4>(cpw, m, n, mb, X, xr, xc, Q, qr, qc, R, want_q, grid, ist, s, Vq, Tq);
  else
    qr_reg_rows<8>(cpw, m, n, mb, X, xr, xc, Q, qr, qc, R, want_q, grid, ist, s, Vq, Tq);
}

// One LDS panel factorisation launch.
static void qr_panel(dim3 grid, int m, int n, int mb, const double *X, long xr, long xc,
                     double *Q, long qr, long qc, double *R, int want_q, long ist, hipStream_t s) {
  hipLaunchKernelGGL(k_qr_lds, grid, dim3(1024), 0, s, m, n, mb, X, xr, xc, Q, qr, qc, R, want_q,
                     ist);
  SPG_CHECK_LAUNCH();
}

void qr_f64(int m, int n, const double *X, long xr, long xc, double *Q, long qr, long qc,
            double *R, double *work, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  if (m < n) {
    set_error("qr_f64: needs rows >= columns");
    throw Fail{SPG_ERR_INVALID};
  }
  if (n > kMaxSketch) {
    set_error("qr_f64: more columns than supported");
    throw Fail{SPG_ERR_UNSUPPORTED};
  }
  const int want_q = (Q != nullptr);
  SPG_BC(X);
  SPG_BC(Q);
  SPG_BC(R);
  SPG_BC(work);
  const unsigned nI = (unsigned)g_bc.n;
  const long ist = g_bc.ist;
  if (m <= kQrRegRows && n <= kQrRegCols) {
    // (timed inside qr_reg_rows: the panel kernel, and k_qform when it runs)
    // Q of 32 or more columns, column-major: formed by k_qform from the stored
    // reflectors (work: m x n reflectors, then n taus)
    const bool split = g_tune.qform_split && want_q && qr == 1 && n >= 32 && work != nullptr;
    qr_reg(m, n, m, X, xr, xc, Q, qr, qc, R, want_q, dim3(1, nI), ist, s,
           split ? work : nullptr, split ? work + (long)m * n : nullptr);
    return;
  }
  if (n <= kQrRegCols) {
    // TSQR on the register kernel: p blocks of at most 512 rows in one launch
    // (a workgroup each), the QR of their stacked R factors (the register
    // kernel again, or TSQR of the p*n stacked rows when they exceed 512, with
    // the rest of the workspace), and Q = diag(Q_b) Q_s
    const int p = (m + kQrRegRows - 1) / kQrRegRows;
    const int mb = (m + p - 1) / p;
    if (m - (p - 1) * mb >= n) {
      double *Q1 = work;                          // m x n row-major
      double *S = Q1 + (long)m * n;               // p*n x n row-major (stacked R_b)
      double *Qs = S + (long)p * n * n;           // p*n x n row-major
      double *Rt = Qs + (long)p * n * n;          // n x n
      // (each launch timed inside qr_reg_rows)
      qr_reg(m, n, mb, X, xr, xc, want_q ? Q1 : nullptr, (long)n, 1L, S, want_q, dim3(p, nI),
             ist, s);
      if (p * n <= kQrRegRows)
        qr_reg(p * n, n, p * n, S, (long)n, 1L, want_q ? Qs : nullptr, (long)n, 1L, R ? R : Rt,
               want_q, dim3(1, nI), ist, s);
      else
        qr_f64(p * n, n, S, (long)n, 1L, want_q ? Qs : nullptr, (long)n, 1L, R ? R : Rt,
               Rt + (long)n * n, s);
      if (!want_q) return;
      const int full = m / mb, tail = m - full * mb;
      GemmDesc g{};
      g.N = n; g.K = n; g.nb2 = 1; g.alpha = 1.0; g.beta = 0.0;
      g.a_i = n; g.a_k = 1; g.b_k = n; g.b_j = 1; g.c_i = qr; g.c_j = qc;
      if (full > 0) {
        g.M = mb; g.nb1 = full;
        g.A = Q1; g.a_b1 = (long)mb * n;
        g.B = Qs; g.b_b1 = (long)n * n;
        g.C = Q; g.c_b1 = (long)mb * qr;
        gemm_f64(g, s);
      }
      if (tail > 0) {
        g.M = tail; g.nb1 = 1;
        g.A = Q1 + (long)full * mb * n; g.a_b1 = 0;
        g.B = Qs + (long)full * n * n; g.b_b1 = 0;
        g.C = Q + (long)full * mb * qr; g.c_b1 = 0;
        gemm_f64(g, s);
      }
      return;
    }
  }
  if ((long)m * n <= kQrLds) {
    // one LDS-resident block; R straight to the caller (or to scratch)
    double *Rd = R ? R : work;
    KTimer kt_("qr_f64", s, qr_flops(m, n, want_q));
    qr_panel(dim3(1, nI), m, n, m, X, xr, xc, Q, qr, qc, Rd, want_q, ist, s);
    return;
  }
  // fewest blocks that fit in LDS, with rows split evenly between them (the
  // cost of a block grows with its rows)
  const int mb_max = kQrLds / n;                // >= n since n <= kMaxSketch
  const int p = (m + mb_max - 1) / mb_max;
  const int mb = std::max((m + p - 1) / p, n);
  if ((long)p * n * n <= kQrLds) {
    // one level of TSQR: block QRs, QR of the stacked R factors, Q = diag(Q_b) Q_s
    double *Q1 = work;                          // m x n row-major
    double *S = Q1 + (long)m * n;               // p*n x n row-major (stacked R_b)
    double *Qs = S + (long)p * n * n;           // p*n x n row-major
    double *Rt = Qs + (long)p * n * n;          // n x n
    {
      KTimer kt_("qr_f64", s, qr_flops(m, n, want_q));
      qr_panel(dim3(p, nI), m, n, mb, X, xr, xc, Q1, (long)n, 1L, S, want_q, ist, s);
    }
    {
      KTimer kt_("qr_f64", s, qr_flops(p * n, n, want_q));
      qr_panel(dim3(1, nI), p * n, n, p * n, S, (long)n, 1L, Qs, (long)n, 1L, R ? R : Rt, want_q,
               ist, s);
    }
    if (!want_q) return;
    const int full = m / mb, tail = m - full * mb;
    GemmDesc g{};
    g.N = n; g.K = n; g.nb2 = 1; g.alpha = 1.0; g.beta = 0.0;
    g.a_i = n; g.a_k = 1; g.b_k = n; g.b_j = 1; g.c_i = qr; g.c_j = qc;
    if (full > 0) {
      g.M = mb; g.nb1 = full;
      g.A = Q1; g.a_b1 = (long)mb * n;
      g.B = Qs; g.b_b1 = (long)n * n;
      g.C = Q; g.c_b1 = (long)mb * qr;
      gemm_f64(g, s);
    }
    if (tail > 0) {
      g.M = tail; g.nb1 = 1;
      g.A = Q1 + (long)full * mb * n; g.a_b1 = 0;
      g.B = Qs + (long)full * n * n; g.b_b1 = 0;
      g.C = Q + (long)full * mb * qr; g.c_b1 = 0;
      gemm_f64(g, s);
    }
    return;
  }
  // large panels: global-memory Householder in one workgroup
  KTimer kt_("qr_f64", s, qr_flops(m, n, want_q));
  hipLaunchKernelGGL(k_qr, dim3(1, nI), dim3(1024), 0, s, m, n, X, xr, xc,
                     Q ? Q : work + 2L * m * n + n, Q ? qr : (long)n, Q ? qc : 1L, R, work, ist);
  SPG_CHECK_LAUNCH();
}

void jacobi_svd_f64(int l, int kk, const double *Rm, double *V, double *sig, hipStream_t s) {
  KTimer kt_("jacobi_svd_f64", s);
  if (l <= 0) return;
  if (l > kMaxSketch) {
    set_error("jacobi_svd_f64: size above the LDS limit");
    throw Fail{SPG_ERR_UNSUPPORTED};
  }
  SPG_BC(Rm);
  SPG_BC(V);
  SPG_BC(sig);
  if (kk < 1 || kk > l) {
    set_error("jacobi_svd_f64: kk must be in 1..l");
    throw Fail{SPG_ERR_INVALID};
  }
  const dim3 grid(1, g_bc.n);
  switch ((l + 15) / 16) {
    case 1: hipLaunchKernelGGL(k_jacobi<1>, grid, dim3(1024), 0, s, l, kk, Rm, V, sig, g_bc.ist); break;
    case 2: hipLaunchKernelGGL(k_jacobi<2>, grid, dim3(1024), 0, s, l, kk, Rm, V, sig, g_bc.ist); break;
    case 3: hipLaunchKernelGGL(k_jacobi<3>, grid, dim3(1024), 0, s, l, kk, Rm, V, sig, g_bc.ist); break;
    case 4: hipLaunchKernelGGL(k_jacobi<4>, grid, dim3(1024), 0, s, l, kk, Rm, V, sig, g_bc.ist); break;
    case 5: hipLaunchKernelGGL(k_jacobi<5>, grid, dim3(1024), 0, s, l, kk, Rm, V, sig, g_bc.ist); break;
    default: hipLaunchKernelGGL(k_jacobi<kJacRows>, grid, dim3(1024), 0, s, l, kk, Rm, V, sig, g_bc.ist); break;
  }
  SPG_CHECK_LAUNCH();
}

void fill_sketch(int n, int l, double *Om, hipStream_t s) {
  const long tot = (long)n * l;
  if (tot <= 0) return;
  SPG_BC(Om);
  hipLaunchKernelGGL(k_sketch, dim3((unsigned)((tot + 255) / 256), g_bc.n), dim3(256), 0, s, n, l,
                     Om, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void normalize_box(double *T, int n0, int n1, int n2, int n3, long s0, long s1, long s2,
                   long s3, double *logs, int out, int in, double *scratch, hipStream_t s) {
  KTimer kt_("normalize_box", s, 16.0 * n0 * n1 * n2 * n3);
  const long tot = (long)n0 * n1 * n2 * n3;
  if (tot <= 0) return;
  if (tot >= (1L << 31)) {
    set_error("normalize_box: box too large");
    throw Fail{SPG_ERR_UNSUPPORTED};
  }
  // about four elements per thread
  const int nb = (int)std::min<long>(kNormBlocks, (tot + 1023) / 1024);
  SPG_BC(T);
  SPG_BC(logs);
  SPG_BC(scratch);
  const unsigned nI = (unsigned)g_bc.n;
  hipLaunchKernelGGL(k_box_sumsq, dim3(nb, nI), dim3(256), 0, s, T, (unsigned)tot, (unsigned)n1,
                     (unsigned)n2, (unsigned)n3, s0, s1, s2, s3, scratch, logs, out, in,
                     g_bc.ist);
  SPG_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_box_scale, dim3(nb, nI), dim3(256), 0, s, T, (unsigned)tot, (unsigned)n1,
                     (unsigned)n2, (unsigned)n3, s0, s1, s2, s3, scratch, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void copy_doubles(double *dst, const double *src, size_t n, hipStream_t s) {
  if (n == 0) return;
  SPG_BC(dst);
  SPG_BC(src);
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + 255) / 256), g_bc.n), dim3(256), 0, s, dst, src,
                     n, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void fill_zero(double *p, size_t n, hipStream_t s) {
  if (n == 0) return;
  SPG_BC(p);
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256), g_bc.n), dim3(256), 0, s, p, n,
                     g_bc.ist);
  SPG_CHECK_LAUNCH();
}

}  // namespace spg
