// Boundary-MPS contraction kernels (FP64) for one row update of the
// Boltzmann PEPS: the row transfer operator acts on the previous boundary MPS
// psi through the row MPO whose site tensor at column c is
//   W_c[(a,e), x, y] = w_c(x) V_c(x,y) H_{c-1}(a,x) D_{c-1}(a,y) A_{c-1}(x,e),
// with left bond (a, e) = (x_{c-1}, y_{c-1}) and right bond (x_c, y_c).
// Tensor layouts (padded to chi on every bond index, row-major):
//   MPS site      phi[p][x][P]          chi x d x chi
//   environment   E[p][a][e][q]         chi x d x d x chi   (p: new MPS, q: psi)
// The small d-index contractions are plain kernels (one thread per output);
// the bond-index contractions go through the strided batched GEMM.
#include "spg_internal.h"

namespace spg {

namespace {

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

// sum over k < n, in order, of fa(k) * fb(k) as an fma chain (the rounding of
// `acc += fa(k) * fb(k)`), with the loads of four iterations in flight
// before their terms are added.
template <class FA, class FB>
__device__ __forceinline__ double fma_chain(int n, const FA &fa, const FB &fb) {
  double acc = 0.0;
  int k = 0;
  for (; k + 3 < n; k += 4) {
    const double a0 = fa(k), a1 = fa(k + 1), a2 = fa(k + 2), a3 = fa(k + 3);
    const double b0 = fb(k), b1 = fb(k + 1), b2 = fb(k + 2), b3 = fb(k + 3);
    acc = fma(a0, b0, acc);
    acc = fma(a1, b1, acc);
    acc = fma(a2, b2, acc);
    acc = fma(a3, b3, acc);
  }
  for (; k < n; ++k) acc = fma(fa(k), fb(k), acc);
  return acc;
}

// Index of this thread in a flat launch (every box here holds < 2^31 entries).
__device__ __forceinline__ unsigned flat_id() { return blockIdx.x * blockDim.x + threadIdx.x; }

// phi[p][x][P] = w(x) sum_y V(x,y) psi[p][y][P]
__global__ void k_init_guess(int d, int chi, int bl, int br, const double *psi, const double *w,
                             const double *V, double *phi, long ist) {
  SPG_INST(psi);
  SPG_INST(w);
  SPG_INST(V);
  SPG_INST(phi);
  const unsigned e = flat_id();
  if (e >= (unsigned)(bl * d * br)) return;
  const int P = e % br, x = (e / br) % d, p = e / (br * d);
  const double *src = psi + (long)p * d * chi + P;
  const double acc = fma_chain(d, [&](int y) { return V[x * d + y]; },
                               [&](int y) { return src[(long)y * chi]; });
  phi[((long)p * d + x) * chi + P] = w[x] * acc;
}

// The bottom row's boundary function F_{rows-1} written exactly, x_c on the
// bond: A_c[a][x][x'] = H_{c-1}(a, x) w_c(x) delta(x, x') (a < 1 at c = 0;
// the last column closes the bond at x' = 0).  Every entry of the C padded
// chi x d x chi tensors is written.  w: the row's d-vectors [C][d]; H: its
// horizontal tables [C-1][d][d].
__global__ void k_bottom_row(int C, int d, int chi, const double *w, const double *H, double *A,
                             long ist) {
  SPG_INST(w);
  SPG_INST(H);
  SPG_INST(A);
  const long site = (long)chi * d * chi;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= site * C) return;
  const int c = (int)(e / site);
  const long o = e - c * site;
  const int k = (int)(o % chi), x = (int)((o / chi) % d), a = (int)(o / ((long)chi * d));
  const int bl = (c == 0) ? 1 : d;
  const bool on = (a < bl) && (c < C - 1 ? k == x : k == 0);
  double v = 0.0;
  if (on) {
    v = w[(long)c * d + x];
    if (c > 0) v *= H[((long)(c - 1) * d + a) * d + x];
  }
  A[e] = v;
}

// Largest entry of each column's MPO tensor,
//   max over (a, e, x, y) of w(x) V(x, y) H(a, x) D(a, y) A(x, e)
//   = max over (x, y) of w(x) V(x, y) max_a [H(a, x) D(a, y)] max_e A(x, e),
// in logs, one workgroup per site (r, c); the site's w is then divided by it
// (in place) and the log written to lsc.  The tables are the ones the MPO
// kernels read: V, D, A are ones on the bottom row; column 0 has no left
// neighbour (H, D through a = 0 and A through e = 0 only).
__global__ __launch_bounds__(256) void k_site_scale(int R, int C, int d, double *W_loc,
                                                    const double *W_h, const double *W_v,
                                                    const double *W_d, const double *W_a,
                                                    double *lsc, long ist) {
  SPG_INST(W_loc);
  SPG_INST(W_h);
  SPG_INST(W_v);
  SPG_INST(W_d);
  SPG_INST(W_a);
  SPG_INST(lsc);
  __shared__ double part[4];
  const int site = blockIdx.x, r = site / C, c = site % C;
  const bool bottom = (r == R - 1);
  const long dd = (long)d * d;
  double *w = W_loc + (long)site * d;
  const double *V = bottom ? nullptr : W_v + ((long)r * C + c) * dd;
  const double *H = c > 0 ? W_h + ((long)r * (C - 1) + c - 1) * dd : nullptr;
  const double *D = (c > 0 && !bottom) ? W_d + ((long)r * (C - 1) + c - 1) * dd : nullptr;
  const double *A = (c > 0 && !bottom) ? W_a + ((long)r * (C - 1) + c - 1) * dd : nullptr;
  const int na = c > 0 ? d : 1;
  double best = -INFINITY;
  for (int p = threadIdx.x; p < d * d; p += blockDim.x) {
    const int x = p / d, y = p - x * d;
    double m1 = -INFINITY;
    for (int a = 0; a < na; ++a) {
      const double h = H ? log(H[(long)a * d + x]) : 0.0;
      const double g = D ? log(D[(long)a * d + y]) : 0.0;
      m1 = fmax(m1, h + g);
    }
    double m2 = 0.0;
    if (A) {
      m2 = -INFINITY;
      for (int e = 0; e < d; ++e) m2 = fmax(m2, log(A[(long)x * d + e]));
    }
    best = fmax(best, log(w[x]) + (V ? log(V[(long)x * d + y]) : 0.0) + m1 + m2);
  }
  for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o, 64));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = best;
  __syncthreads();
  double ls = fmax(fmax(part[0], part[1]), fmax(part[2], part[3]));
  if (!(ls > -INFINITY) || !(ls < INFINITY)) ls = 0.0;     // an all-zero tensor stays as it is
  for (int x = threadIdx.x; x < d; x += blockDim.x) w[x] *= exp(-ls);
  if (threadIdx.x == 0) lsc[site] = ls;
}

// row_lsc[r] = sum over c of lsc[r * C + c], in column order
__global__ void k_row_lsc(int R, int C, const double *lsc, double *row_lsc, long ist) {
  SPG_INST(lsc);
  SPG_INST(row_lsc);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double t = 0.0;
  for (int c = 0; c < C; ++c) t += lsc[(long)r * C + c];
  row_lsc[r] = t;
}

// T1[p][a][x][q] = sum_e Al[x][e] EL[p][a][e][q]
__global__ void k_T1(int d, int chi, int pl, int ql, const double *EL, const double *Al,
                     double *T1, long ist) {
  SPG_INST(EL);
  SPG_INST(Al);
  SPG_INST(T1);
  const unsigned e = flat_id();
  if (e >= (unsigned)(pl * d * d * ql)) return;
  const int q = e % ql, x = (e / ql) % d, a = (e / (ql * d)) % d;
  const int p = e / (ql * d * d);
  const double *src = EL + (((long)p * d + a) * d) * chi + q;
  const double acc = fma_chain(d, [&](int ee) { return Al[x * d + ee]; },
                               [&](int ee) { return src[(long)ee * chi]; });
  T1[(((long)p * d + a) * d + x) * chi + q] = acc;
}

// T2[p][x][y][q] = sum_a Hl[a][x] Dl[a][y] T1[p][a][x][q]
__global__ void k_T2(int d, int chi, int pl, int ql, const double *T1, const double *Hl,
                     const double *Dl, double *T2, long ist) {
  SPG_INST(T1);
  SPG_INST(Hl);
  SPG_INST(Dl);
  SPG_INST(T2);
  const unsigned e = flat_id();
  if (e >= (unsigned)(pl * d * d * ql)) return;
  const int q = e % ql, y = (e / ql) % d, x = (e / (ql * d)) % d;
  const int p = e / (ql * d * d);
  const double *src = T1 + ((long)p * d * d + x) * chi + q;
  const double acc = fma_chain(d, [&](int a) { return Hl[a * d + x] * Dl[a * d + y]; },
                               [&](int a) { return src[(long)a * d * chi]; });
  T2[(((long)p * d + x) * d + y) * chi + q] = acc;
}

// G3[p][x][a][q] = sum_y G2[p][x][y][q] Dl[a][y]
__global__ void k_G3(int d, int chi, int pl, int ql, const double *G2, const double *Dl,
                     double *G3, long ist) {
  SPG_INST(G2);
  SPG_INST(Dl);
  SPG_INST(G3);
  const unsigned e = flat_id();
  if (e >= (unsigned)(pl * d * d * ql)) return;
  const int q = e % ql, a = (e / ql) % d, x = (e / (ql * d)) % d;
  const int p = e / (ql * d * d);
  const double *src = G2 + (((long)p * d + x) * d) * chi + q;
  const double acc = fma_chain(d, [&](int y) { return Dl[a * d + y]; },
                               [&](int y) { return src[(long)y * chi]; });
  G3[(((long)p * d + x) * d + a) * chi + q] = acc;
}

// ER[p][a][e][q] = sum_x G3[p][x][a][q] Hl[a][x] Al[x][e]
__global__ void k_ERfin(int d, int chi, int pl, int ql, const double *G3, const double *Hl,
                        const double *Al, double *ER, long ist) {
  SPG_INST(G3);
  SPG_INST(Hl);
  SPG_INST(Al);
  SPG_INST(ER);
  const unsigned e = flat_id();
  if (e >= (unsigned)(pl * d * d * ql)) return;
  const int q = e % ql, ee = (e / ql) % d, a = (e / (ql * d)) % d;
  const int p = e / (ql * d * d);
  const double *src = G3 + ((long)p * d * d + a) * chi + q;
  const double acc = fma_chain(d, [&](int x) { return Hl[a * d + x] * Al[x * d + ee]; },
                               [&](int x) { return src[(long)x * d * chi]; });
  ER[(((long)p * d + a) * d + ee) * chi + q] = acc;
}

// P2[p][x][z][Q] = sum_y P[p][x][y][Q] A1[z][y]
__global__ void k_P2(int d, int chi, int pl, int nq, const double *P, const double *A1,
                     double *P2, long ist) {
  SPG_INST(P);
  SPG_INST(A1);
  SPG_INST(P2);
  const unsigned e = flat_id();
  if (e >= (unsigned)(pl * d * d * nq)) return;
  const int Q = e % nq, z = (e / nq) % d, x = (e / (nq * d)) % d;
  const int p = e / (nq * d * d);
  const double *src = P + (((long)p * d + x) * d) * chi + Q;
  const double acc = fma_chain(d, [&](int y) { return A1[z * d + y]; },
                               [&](int y) { return src[(long)y * chi]; });
  P2[(((long)p * d + x) * d + z) * chi + Q] = acc;
}

// Q2[Q][x][z][P] = sum_v Qr[Q][z][v][P] D1[x][v]
__global__ void k_Q2(int d, int chi, int nq, int pr, const double *Qr, const double *D1,
                     double *Q2, long ist) {
  SPG_INST(Qr);
  SPG_INST(D1);
  SPG_INST(Q2);
  const unsigned e = flat_id();
  if (e >= (unsigned)(nq * d * d * pr)) return;
  const int P = e % pr, z = (e / pr) % d, x = (e / (pr * d)) % d;
  const int Q = e / (pr * d * d);
  const double *src = Qr + (((long)Q * d + z) * d) * chi + P;
  const double acc = fma_chain(d, [&](int v) { return D1[x * d + v]; },
                               [&](int v) { return src[(long)v * chi]; });
  Q2[(((long)Q * d + x) * d + z) * chi + P] = acc;
}

// Column forms of the six kernels above for d = D in {8, 16, 24, 32}.  In
// each, the d outputs that differ only in the output's own d index read the
// same d-long column of the source; here one thread loads that column once
// into registers and writes all d outputs, so every source entry is read from
// memory once (the one-thread-per-output forms re-read each column d times,
// from workgroups that the dispatcher spreads over XCDs with separate L2
// caches).  The d x d coefficient table is staged in LDS, laid out so that the
// terms of one output are contiguous, and read at the same address by the
// whole wavefront.  Every output keeps its operands and the order of its
// terms: results are bitwise those of the forms above.
constexpr int kColThreads = 64;

// cf[i * D + k] = tab[i * d + k] (tr = false) or tab[k * d + i] (tr = true)
template <int D>
__device__ __forceinline__ void stage_table(double *cf, const double *tab, bool tr) {
  for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
    const int i = e / D, k = e % D;
    cf[e] = tr ? tab[k * D + i] : tab[e];
  }
  __syncthreads();
}

template <int D>
__device__ __forceinline__ void load_col(double (&v)[D], const double *src, long stride) {
#pragma unroll
  for (int k = 0; k < D; ++k) v[k] = src[k * stride];
}

// sum over k < D, in order, of row[k] * v[k] as an fma chain
template <int D>
__device__ __forceinline__ double dot_row(const double *row, const double (&v)[D]) {
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) acc = fma(row[k], v[k], acc);
  return acc;
}

// the same with row[k] * h[k] as the coefficient
template <int D>
__device__ __forceinline__ double dot_row2(const double *row, const double (&h)[D],
                                           const double (&v)[D]) {
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) acc = fma(h[k] * row[k], v[k], acc);
  return acc;
}

// T1[p][a][x][q] = sum_e Al[x][e] EL[p][a][e][q]; thread (p, a, q)
template <int D>
__global__ __launch_bounds__(kColThreads) void k_T1c(int chi, int pl, int ql, const double *EL,
                                                     const double *Al, double *T1, long ist) {
  SPG_INST(EL);
  SPG_INST(Al);
  SPG_INST(T1);
  __shared__ double cf[D * D];
  stage_table<D>(cf, Al, false);
  const unsigned t = flat_id();
  if (t >= (unsigned)(pl * D * ql)) return;
  const int q = t % ql, a = (t / ql) % D, p = t / (ql * D);
  const long base = (((long)p * D + a) * D) * chi + q;
  double v[D];
  load_col(v, EL + base, chi);
  for (int x = 0; x < D; ++x) T1[base + (long)x * chi] = dot_row(cf + x * D, v);
}

// T2[p][x][y][q] = sum_a Hl[a][x] Dl[a][y] T1[p][a][x][q]; thread (p, x, q)
template <int D>
__global__ __launch_bounds__(kColThreads) void k_T2c(int chi, int pl, int ql, const double *T1,
                                                     const double *Hl, const double *Dl,
                                                     double *T2, long ist) {
  SPG_INST(T1);
  SPG_INST(Hl);
  SPG_INST(Dl);
  SPG_INST(T2);
  __shared__ double cf[D * D];                       // cf[y][a] = Dl[a][y]
  stage_table<D>(cf, Dl, true);
  const unsigned t = flat_id();
  if (t >= (unsigned)(pl * D * ql)) return;
  const int q = t % ql, x = (t / ql) % D, p = t / (ql * D);
  double v[D], h[D];
  load_col(v, T1 + ((long)p * D * D + x) * chi + q, (long)D * chi);
  load_col(h, Hl + x, D);
  double *out = T2 + (((long)p * D + x) * D) * chi + q;
  for (int y = 0; y < D; ++y) out[(long)y * chi] = dot_row2(cf + y * D, h, v);
}

// G3[p][x][a][q] = sum_y Dl[a][y] G2[p][x][y][q]; thread (p, x, q)
template <int D>
__global__ __launch_bounds__(kColThreads) void k_G3c(int chi, int pl, int ql, const double *G2,
                                                     const double *Dl, double *G3, long ist) {
  SPG_INST(G2);
  SPG_INST(Dl);
  SPG_INST(G3);
  __shared__ double cf[D * D];
  stage_table<D>(cf, Dl, false);
  const unsigned t = flat_id();
  if (t >= (unsigned)(pl * D * ql)) return;
  const int q = t % ql, x = (t / ql) % D, p = t / (ql * D);
  const long base = (((long)p * D + x) * D) * chi + q;
  double v[D];
  load_col(v, G2 + base, chi);
  for (int a = 0; a < D; ++a) G3[base + (long)a * chi] = dot_row(cf + a * D, v);
}

// ER[p][a][e][q] = sum_x Hl[a][x] Al[x][e] G3[p][x][a][q]; thread (p, a, q)
template <int D>
__global__ __launch_bounds__(kColThreads) void k_ERfinc(int chi, int pl, int ql, const double *G3,
                                                        const double *Hl, const double *Al,
                                                        double *ER, long ist) {
  SPG_INST(G3);
  SPG_INST(Hl);
  SPG_INST(Al);
  SPG_INST(ER);
  __shared__ double cf[D * D];                       // cf[e][x] = Al[x][e]
  stage_table<D>(cf, Al, true);
  const unsigned t = flat_id();
  if (t >= (unsigned)(pl * D * ql)) return;
  const int q = t % ql, a = (t / ql) % D, p = t / (ql * D);
  double v[D], h[D];
  load_col(v, G3 + ((long)p * D * D + a) * chi + q, (long)D * chi);
  load_col(h, Hl + (long)a * D, 1);
  double *out = ER + (((long)p * D + a) * D) * chi + q;
  for (int ee = 0; ee < D; ++ee) out[(long)ee * chi] = dot_row2(cf + ee * D, h, v);
}

// P2[p][x][z][Q] = sum_y A1[z][y] P[p][x][y][Q]; thread (p, x, Q)
template <int D>
__global__ __launch_bounds__(kColThreads) void k_P2c(int chi, int pl, int nq, const double *P,
                                                     const double *A1, double *P2, long ist) {
  SPG_INST(P);
  SPG_INST(A1);
  SPG_INST(P2);
  __shared__ double cf[D * D];
  stage_table<D>(cf, A1, false);
  const unsigned t = flat_id();
  if (t >= (unsigned)(pl * D * nq)) return;
  const int Q = t % nq, x = (t / nq) % D, p = t / (nq * D);
  const long base = (((long)p * D + x) * D) * chi + Q;
  double v[D];
  load_col(v, P + base, chi);
  for (int z = 0; z < D; ++z) P2[base + (long)z * chi] = dot_row(cf + z * D, v);
}

// Q2[Q][x][z][P] = sum_v D1[x][v] Qr[Q][z][v][P]; thread (Q, z, P)
template <int D>
__global__ __launch_bounds__(kColThreads) void k_Q2c(int chi, int nq, int pr, const double *Qr,
                                                     const double *D1, double *Q2, long ist) {
  SPG_INST(Qr);
  SPG_INST(D1);
  SPG_INST(Q2);
  __shared__ double cf[D * D];
  stage_table<D>(cf, D1, false);
  const unsigned t = flat_id();
  if (t >= (unsigned)(nq * D * pr)) return;
  const int P = t % pr, z = (t / pr) % D, Q = t / (pr * D);
  double v[D];
  load_col(v, Qr + (((long)Q * D + z) * D) * chi + P, chi);
  double *out = Q2 + ((long)Q * D * D + z) * chi + P;
  for (int x = 0; x < D; ++x) out[(long)x * D * chi] = dot_row(cf + x * D, v);
}

// The whole padded site dst[chi][d][chi]: entries k < nk, P < pr from src,
// zero elsewhere.
__global__ void k_unpack_right(int d, int chi, int nk, int pr, const double *src, long sk,
                               long sj, double *dst, long ist) {
  SPG_INST(src);
  SPG_INST(dst);
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long tot = (long)chi * d * chi;
  if (e >= tot) return;
  const int P = e % chi, z = (e / chi) % d, k = (int)(e / ((long)chi * d));
  dst[e] = (k < nk && P < pr) ? src[k * sk + ((long)z * pr + P) * sj] : 0.0;
}

// tmp[p][x][k] = sum_q phi[p][x][q] R[k][q]  (R row-major k x bl), then copy back
__global__ void k_lq_fold(int d, int chi, int pl, int bl, int kk, const double *R,
                          const double *phi, double *tmp, long ist) {
  SPG_INST(R);
  SPG_INST(phi);
  SPG_INST(tmp);
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long tot = (long)pl * d * chi;            // every entry of the padded site
  if (e >= tot) return;
  const int k = e % chi;
  const long px = e / chi;
  double acc = 0.0;
  if (k < kk)
    acc = fma_chain(bl, [&](int q) { return phi[px * chi + q]; },
                    [&](int q) { return R[(long)k * bl + q]; });
  tmp[px * chi + k] = acc;
}

__global__ void k_pack_right(int d, int chi, int nk, int pr, const double *src, double *dst, long ist) {
  SPG_INST(src);
  SPG_INST(dst);
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long tot = (long)nk * d * pr;
  if (e >= tot) return;
  const int P = e % pr, z = (e / pr) % d, k = (int)(e / ((long)pr * d));
  dst[e] = src[((long)k * d + z) * chi + P];
}

// w = exp(-beta (E - min E)) per table of `tsize` entries, one block per table.
__global__ __launch_bounds__(256) void k_weights(int ntab, int tsize, double beta,
                                                 const double *E, double *W, double *mins, long ist) {
  SPG_INST(E);
  SPG_INST(W);
  SPG_INST(mins);
  __shared__ double red[256];
  const int t = blockIdx.x;
  if (t >= ntab) return;
  const double *e = E + (long)t * tsize;
  double m = INFINITY;
  for (int i = threadIdx.x; i < tsize; i += blockDim.x) m = fmin(m, e[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  const double mn = red[0];
  for (int i = threadIdx.x; i < tsize; i += blockDim.x)
    W[(long)t * tsize + i] = exp(-beta * (e[i] - mn));
  if (threadIdx.x == 0) mins[t] = mn;
}

__global__ void k_set_e0(int n, int chi, double *p, long stride, long ist) {
  SPG_INST(p);
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * chi) return;
  const int j = (int)(e / chi), i = (int)(e % chi);
  p[j * stride + i] = (i == 0) ? 1.0 : 0.0;
}

__global__ void k_set_identity(int n, double *p, long ist) {
  SPG_INST(p);
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  p[e] = (e / n == e % n) ? 1.0 : 0.0;
}

__global__ void k_add_logs(double *logs, int out, int a, int b, int c, long ist) {
  SPG_INST(logs);
  logs[out] = (a >= 0 ? logs[a] : 0.0) + (b >= 0 ? logs[b] : 0.0) + (c >= 0 ? logs[c] : 0.0);
}

}  // namespace

void init_guess(int d, int chi, int bl, int br, const double *psi, const RowFactors &f,
                double *phi, hipStream_t s) {
  const long tot = (long)bl * d * br;
  SPG_BC(psi);
  SPG_BC(f.w);
  SPG_BC(f.V);
  SPG_BC(phi);
  hipLaunchKernelGGL(k_init_guess, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, d, chi, bl, br, psi, f.w, f.V, phi, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void bottom_row(int C, int d, int chi, const double *w, const double *H, double *A,
                hipStream_t s) {
  const long tot = (long)C * chi * d * chi;
  SPG_BC(w);
  SPG_BC(H);
  SPG_BC(A);
  hipLaunchKernelGGL(k_bottom_row, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, C, d, chi, w, H, A, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

// The column forms exist for d in {8, 16, 24, 32}; other d up to 32 (and
// calls with the column forms switched off) take the per-output forms.  Above
// d = 32 the d-index contractions are batched GEMMs on the matrix cores (K =
// d, 2d flops per output: above the FP64 ridge from d of about 40), with the
// horizontal table H applied in the producing GEMM's epilogue where its
// factor depends on both indices.
inline bool gemm_form(int d) { return d > 32; }
inline bool col_form(int d) {
  return g_tune.mpo_cols && (d == 8 || d == 16 || d == 24 || d == 32);
}

// Above d = 32 the products of the contraction are large (K and the batch
// counts grow with d): 64 x 64 tiles from d = 64 (the tile does not change
// any output's order of terms).
inline void large_d_tile(GemmDesc &g, int d) {
  if (d >= 64) g.tile = 64;
}

// C[b1][b2](i, j) = sum_k A(i, k) B[b1][b2](k, j) for i < d, j < n, k < d, with
// the d x d coefficient table A shared by all batches (element (i, k) at
// A[i * ai + k * ak]), every batch's B and C rows chi apart and their
// columns adjacent; smode 3 / 4 scale the outputs by the table H (see GemmDesc).
static void mpo_gemm(int d, int nb1, int n, const double *A, long ai, long ak,
                     const double *B, long bk, long bb1, long bb2, double *C, long ci, long cb1,
                     long cb2, int smode, const double *ones, const double *H, hipStream_t s) {
  GemmDesc g{};
  g.M = d; g.N = n; g.K = d; g.nb1 = nb1; g.nb2 = d;
  g.A = A; g.a_i = ai; g.a_k = ak; g.a_b1 = 0; g.a_b2 = 0;
  g.B = B; g.b_k = bk; g.b_j = 1; g.b_b1 = bb1; g.b_b2 = bb2;
  g.C = C; g.c_i = ci; g.c_j = 1; g.c_b1 = cb1; g.c_b2 = cb2;
  g.alpha = 1.0; g.beta = 0.0;
  if (smode) {
    g.sw = ones; g.sV = H; g.sd = d; g.smode = smode;
  }
  large_d_tile(g, d);
  g.cls = "mpo_gemm_f64";
  gemm_f64(g, s);
}

#define SPG_LAUNCH_COL(KN, nthr, ...)                                            \
  do {                                                                           \
    const dim3 g_(nblk((nthr), kColThreads), g_bc.n), b_(kColThreads);           \
    switch (d) {                                                                 \
      case 8: hipLaunchKernelGGL(KN<8>, g_, b_, 0, s, __VA_ARGS__); break;       \
      case 16: hipLaunchKernelGGL(KN<16>, g_, b_, 0, s, __VA_ARGS__); break;     \
      case 24: hipLaunchKernelGGL(KN<24>, g_, b_, 0, s, __VA_ARGS__); break;     \
      default: hipLaunchKernelGGL(KN<32>, g_, b_, 0, s, __VA_ARGS__); break;     \
    }                                                                            \
  } while (0)

void left_part(int d, int chi, int pl, int ql, int qr, const double *EL, const double *psi,
               const RowFactors &f, double *T1, double *P, hipStream_t s) {
  const long tot = (long)pl * d * d * ql;
  double *T2 = T1 + (long)chi * d * d * chi;
  const long dc = (long)d * chi, ddc = (long)d * d * chi;
  if (gemm_form(d)) {
    // T1'[p][a][x][q] = H(a, x) sum_e Al[x][e] EL[p][a][e][q]   (batch (p, a); rows x)
    mpo_gemm(d, pl, ql, f.Al, d, 1, EL, chi, ddc, dc, T1, chi, ddc, dc, 3, f.ones, f.Hl, s);
    // T2[p][x][y][q] = sum_a Dl[a][y] T1'[p][a][x][q]   (batch (p, x); rows y)
    mpo_gemm(d, pl, ql, f.Dl, 1, d, T1, dc, ddc, chi, T2, chi, ddc, dc, 0, nullptr, nullptr,
             s);
  } else {
  SPG_BC(EL);
  SPG_BC(f.Al);
  SPG_BC(T1);
  if (col_form(d))
    SPG_LAUNCH_COL(k_T1c, (long)pl * d * ql, chi, pl, ql, EL, f.Al, T1, g_bc.ist);
  else
    hipLaunchKernelGGL(k_T1, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, d, chi, pl, ql, EL, f.Al, T1, g_bc.ist);
  SPG_CHECK_LAUNCH();
  // T2 written into P (the GEMM below reads T2 and writes P in place would alias),
  // so T2 goes to the second half of T1's buffer.
  SPG_BC(T1);
  SPG_BC(f.Hl);
  SPG_BC(f.Dl);
  SPG_BC(T2);
  if (col_form(d))
    SPG_LAUNCH_COL(k_T2c, (long)pl * d * ql, chi, pl, ql, T1, f.Hl, f.Dl, T2, g_bc.ist);
  else
    hipLaunchKernelGGL(k_T2, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, d, chi, pl, ql, T1, f.Hl, f.Dl, T2, g_bc.ist);
  SPG_CHECK_LAUNCH();
  }
  // P[p][x][y][Q] = sum_q T2[p][x][y][q] psi[q][y][Q]   (batch y; rows (p,x))
  GemmDesc g{};
  g.M = pl * d; g.N = qr; g.K = ql; g.nb1 = d; g.nb2 = 1;
  g.A = T2; g.a_i = (long)d * chi; g.a_k = 1; g.a_b1 = chi; g.a_b2 = 0;
  g.B = psi; g.b_k = (long)d * chi; g.b_j = 1; g.b_b1 = chi; g.b_b2 = 0;
  g.C = P; g.c_i = (long)d * chi; g.c_j = 1; g.c_b1 = chi; g.c_b2 = 0;
  g.alpha = 1.0; g.beta = 0.0;
  g.sw = f.w; g.sV = f.V; g.sd = d; g.smode = 1;        // P[p][x][y][Q] *= w(x) V(x, y)
  large_d_tile(g, d);
  gemm_f64(g, s);
}

void env_left(int d, int chi, int pl, int pr, int qr, const double *phi, const double *P,
              double *ELn, hipStream_t s) {
  // ELn[P][x][y][Q] = sum_p phi[p][x][P] P[p][x][y][Q]   (batch x; cols (y,Q) over d*chi)
  GemmDesc g{};
  g.M = pr; g.N = d * chi; g.K = pl; g.nb1 = d; g.nb2 = 1;
  g.A = phi; g.a_i = 1; g.a_k = (long)d * chi; g.a_b1 = chi; g.a_b2 = 0;
  g.B = P; g.b_k = (long)d * d * chi; g.b_j = 1; g.b_b1 = (long)d * chi; g.b_b2 = 0;
  g.C = ELn; g.c_i = (long)d * d * chi; g.c_j = 1; g.c_b1 = (long)d * chi; g.c_b2 = 0;
  g.alpha = 1.0; g.beta = 0.0;
  (void)qr;
  large_d_tile(g, d);
  gemm_f64(g, s);
}

void env_right(int d, int chi, int pl, int pr, int ql, int qr, const double *phi,
               const double *psi, const double *ER, const RowFactors &f, double *G1,
               double *G2, double *ERn, hipStream_t s) {
  // G1[p][x][y][Q] = sum_P phi[p][x][P] ER[P][x][y][Q]   (batch x; cols (y,Q))
  GemmDesc g{};
  g.M = pl; g.N = d * chi; g.K = pr; g.nb1 = d; g.nb2 = 1;
  g.A = phi; g.a_i = (long)d * chi; g.a_k = 1; g.a_b1 = chi; g.a_b2 = 0;
  g.B = ER; g.b_k = (long)d * d * chi; g.b_j = 1; g.b_b1 = (long)d * chi; g.b_b2 = 0;
  g.C = G1; g.c_i = (long)d * d * chi; g.c_j = 1; g.c_b1 = (long)d * chi; g.c_b2 = 0;
  g.alpha = 1.0; g.beta = 0.0;
  large_d_tile(g, d);
  gemm_f64(g, s);
  (void)qr;
  // G2[p][x][y][q] = sum_Q G1[p][x][y][Q] psi[q][y][Q]   (batch y; rows (p,x))
  GemmDesc h{};
  h.M = pl * d; h.N = ql; h.K = qr; h.nb1 = d; h.nb2 = 1;
  h.A = G1; h.a_i = (long)d * chi; h.a_k = 1; h.a_b1 = chi; h.a_b2 = 0;
  h.B = psi; h.b_k = 1; h.b_j = (long)d * chi; h.b_b1 = chi; h.b_b2 = 0;
  h.C = G2; h.c_i = (long)d * chi; h.c_j = 1; h.c_b1 = chi; h.c_b2 = 0;
  h.alpha = 1.0; h.beta = 0.0;
  h.sw = f.w; h.sV = f.V; h.sd = d; h.smode = 1;        // G2[p][x][y][q] *= w(x) V(x, y)
  large_d_tile(h, d);
  gemm_f64(h, s);
  const long tot = (long)pl * d * d * ql;
  double *G3 = G1;  // G1 no longer needed
  if (gemm_form(d)) {
    const long dc = (long)d * chi, ddc = (long)d * d * chi;
    // G3'[p][x][a][q] = H(a, x) sum_y Dl[a][y] G2[p][x][y][q]   (batch (p, x); rows a)
    mpo_gemm(d, pl, ql, f.Dl, d, 1, G2, chi, ddc, dc, G3, chi, ddc, dc, 4, f.ones, f.Hl, s);
    // ER[p][a][e][q] = sum_x Al[x][e] G3'[p][x][a][q]   (batch (p, a); rows e)
    mpo_gemm(d, pl, ql, f.Al, 1, d, G3, dc, ddc, chi, ERn, chi, ddc, dc, 0, nullptr, nullptr,
             s);
    return;
  }
  SPG_BC(G2);
  SPG_BC(f.Dl);
  SPG_BC(G3);
  if (col_form(d))
    SPG_LAUNCH_COL(k_G3c, (long)pl * d * ql, chi, pl, ql, G2, f.Dl, G3, g_bc.ist);
  else
    hipLaunchKernelGGL(k_G3, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, d, chi, pl, ql, G2, f.Dl, G3, g_bc.ist);
  SPG_CHECK_LAUNCH();
  SPG_BC(G3);
  SPG_BC(f.Hl);
  SPG_BC(f.Al);
  SPG_BC(ERn);
  if (col_form(d))
    SPG_LAUNCH_COL(k_ERfinc, (long)pl * d * ql, chi, pl, ql, G3, f.Hl, f.Al, ERn, g_bc.ist);
  else
    hipLaunchKernelGGL(k_ERfin, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, d, chi, pl, ql, G3, f.Hl, f.Al, ERn, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void two_site_block(int d, int chi, int pl, int ql, int qm, int qr, int pr, const double *EL,
                    const double *ER, const double *psi0, const double *psi1,
                    const RowFactors &f0, const RowFactors &f1, double *T1, double *P,
                    double *Qr, double *P2, double *Q2, double *B, hipStream_t s) {
  // P[p][x][y][Q] : left part through column c (Q = psi bond between c and c+1, qm)
  left_part(d, chi, pl, ql, qm, EL, psi0, f0, T1, P, s);
  // Qr[q][x][y][P] = w1(x)V1(x,y) sum_Q psi1[q][y][Q] ER[P][x][y][Q]   (batch (x,y))
  GemmDesc g{};
  g.M = qm; g.N = pr; g.K = qr; g.nb1 = d; g.nb2 = d;
  g.A = psi1; g.a_i = (long)d * chi; g.a_k = 1; g.a_b1 = 0; g.a_b2 = chi;
  g.B = ER; g.b_k = 1; g.b_j = (long)d * d * chi; g.b_b1 = (long)d * chi; g.b_b2 = chi;
  g.C = Qr; g.c_i = (long)d * d * chi; g.c_j = 1; g.c_b1 = (long)d * chi; g.c_b2 = chi;
  g.alpha = 1.0; g.beta = 0.0;
  g.sw = f1.w; g.sV = f1.V; g.sd = d; g.smode = 2;      // Qr[q][x][y][P] *= w1(x) V1(x, y)
  large_d_tile(g, d);
  gemm_f64(g, s);
  const long totq = (long)qm * d * d * pr;
  const long totp = (long)pl * d * d * qm;
  const long dc = (long)d * chi, ddc = (long)d * d * chi;
  if (gemm_form(d)) {
    // P2[p][x][z][Q] = sum_y A1[z][y] P[p][x][y][Q]   (batch (p, x); rows z)
    mpo_gemm(d, pl, qm, f1.Al, d, 1, P, chi, ddc, dc, P2, chi, ddc, dc, 0, nullptr, nullptr,
             s);
    // Q2[Q][x][z][P] = sum_v D1[x][v] Qr[Q][z][v][P]   (batch (Q, z); rows x)
    mpo_gemm(d, qm, pr, f1.Dl, d, 1, Qr, chi, ddc, dc, Q2, dc, ddc, chi, 0, nullptr, nullptr,
             s);
  } else {
  SPG_BC(P);
  SPG_BC(f1.Al);
  SPG_BC(P2);
  if (col_form(d))
    SPG_LAUNCH_COL(k_P2c, (long)pl * d * qm, chi, pl, qm, P, f1.Al, P2, g_bc.ist);
  else
    hipLaunchKernelGGL(k_P2, dim3(nblk(totp, 256), g_bc.n), dim3(256), 0, s, d, chi, pl, qm, P, f1.Al, P2, g_bc.ist);
  SPG_CHECK_LAUNCH();
  SPG_BC(Qr);
  SPG_BC(f1.Dl);
  SPG_BC(Q2);
  if (col_form(d))
    SPG_LAUNCH_COL(k_Q2c, (long)qm * d * pr, chi, qm, pr, Qr, f1.Dl, Q2, g_bc.ist);
  else
    hipLaunchKernelGGL(k_Q2, dim3(nblk(totq, 256), g_bc.n), dim3(256), 0, s, d, chi, qm, pr, Qr, f1.Dl, Q2, g_bc.ist);
  SPG_CHECK_LAUNCH();
  }
  // B[p][x][z][P] = sum_Q P2[p][x][z][Q] Q2[Q][x][z][P]   (batch (x,z)), compact output
  GemmDesc h{};
  h.M = pl; h.N = pr; h.K = qm; h.nb1 = d; h.nb2 = d;
  h.A = P2; h.a_i = (long)d * d * chi; h.a_k = 1; h.a_b1 = (long)d * chi; h.a_b2 = chi;
  h.B = Q2; h.b_k = (long)d * d * chi; h.b_j = 1; h.b_b1 = (long)d * chi; h.b_b2 = chi;
  h.C = B; h.c_i = (long)d * d * pr; h.c_j = 1; h.c_b1 = (long)d * pr; h.c_b2 = pr;
  h.alpha = 1.0; h.beta = 0.0;
  h.sw = f1.ones; h.sV = f1.Hl; h.sd = d; h.smode = 2;  // B[p][x][z][P] *= 1 * H1(x, z)
  large_d_tile(h, d);
  gemm_f64(h, s);
}

void unpack_right(int d, int chi, int nk, int pr, const double *src, long sk, long sj,
                  double *dst, hipStream_t s) {
  const long tot = (long)chi * d * chi;
  SPG_BC(src);
  SPG_BC(dst);
  hipLaunchKernelGGL(k_unpack_right, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, d, chi, nk, pr, src, sk, sj, dst, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void lq_fold(int d, int chi, int bl, int k, const double *R, double *phi_prev, double *tmp,
             hipStream_t s) {
  // phi_prev has left dim pl = chi rows at most; fold over all padded rows (zeros stay zero)
  const int pl = chi;
  const long tot = (long)pl * d * chi;
  SPG_BC(R);
  SPG_BC(phi_prev);
  SPG_BC(tmp);
  hipLaunchKernelGGL(k_lq_fold, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, d, chi, pl, bl, k, R, phi_prev, tmp, g_bc.ist);
  SPG_CHECK_LAUNCH();
  copy_d2d(phi_prev, tmp, sizeof(double) * chi * d * chi, s);
}

void pack_right(int d, int chi, int nk, int pr, const double *src, double *dst, hipStream_t s) {
  const long tot = (long)nk * d * pr;
  if (tot <= 0) return;
  SPG_BC(src);
  SPG_BC(dst);
  hipLaunchKernelGGL(k_pack_right, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, d, chi, nk, pr, src, dst, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void build_weights(int ntab, int tsize, double beta, const double *E, double *W, double *mins,
                   hipStream_t s) {
  if (ntab <= 0) return;
  SPG_BC(E);
  SPG_BC(W);
  SPG_BC(mins);
  hipLaunchKernelGGL(k_weights, dim3(ntab, g_bc.n), dim3(256), 0, s, ntab, tsize, beta, E, W, mins, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void site_scales(int R, int C, int d, double *W_loc, const double *W_h, const double *W_v,
                 const double *W_d, const double *W_a, double *lsc, double *row_lsc,
                 hipStream_t s) {
  SPG_BC(W_loc);
  SPG_BC(W_h);
  SPG_BC(W_v);
  SPG_BC(W_d);
  SPG_BC(W_a);
  SPG_BC(lsc);
  SPG_BC(row_lsc);
  hipLaunchKernelGGL(k_site_scale, dim3(R * C, g_bc.n), dim3(256), 0, s, R, C, d, W_loc, W_h, W_v, W_d, W_a, lsc, g_bc.ist);
  SPG_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_row_lsc, dim3(nblk(R, 64), g_bc.n), dim3(64), 0, s, R, C, lsc, row_lsc, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void set_e0(int n, int chi, double *p, long stride, hipStream_t s) {
  const long tot = (long)n * chi;
  if (tot <= 0) return;
  SPG_BC(p);
  hipLaunchKernelGGL(k_set_e0, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, n, chi, p, stride, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void set_identity(int n, double *p, hipStream_t s) {
  const long tot = (long)n * n;
  if (tot <= 0) return;
  SPG_BC(p);
  hipLaunchKernelGGL(k_set_identity, dim3(nblk(tot, 256), g_bc.n), dim3(256), 0, s, n, p, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

void add_logs(double *logs, int out, int a, int b, int c, hipStream_t s) {
  SPG_BC(logs);
  hipLaunchKernelGGL(k_add_logs, dim3(1, g_bc.n), dim3(1), 0, s, logs, out, a, b, c, g_bc.ist);
  SPG_CHECK_LAUNCH();
}

}  // namespace spg
