"""Boundary-MPS contraction of the Boltzmann PEPS (oracle; test infrastructure only).

What is computed (Sec. 2 and Fig. 1(c)-(d) of the paper; the paper defers the
mechanics to its references, so the steps below are the adopted reading):

* Row factors.  F_r(X) = prod_c w_{r,c}(x_c) prod_c W^H_{r,c}(x_c, x_{c+1}) and
  G_r(X, Y) = prod_c W^V_{r,c}(x_c, y_c) W^D_{r,c}(x_c, y_{c+1}) W^A_{r,c}(x_{c+1}, y_c),
  with w, W the Boltzmann factors of the min-shifted energy tables of Eq. (1).
* Boundary functions.  E~_{rows} = 1 and E~_r(X) = F_r(X) sum_Y G_r(X, Y) E~_{r+1}(Y)
  (for r = rows-1 the couplings G are absent).  Then Z = exp(-beta*shift) sum_X E~_0(X).
* Boundary MPS.  E~_r(X) ~ exp(lam_r) A_{r,0}[x_0] ... A_{r,cols-1}[x_{cols-1}], each
  A_{r,c} a (chi_c x d x chi_{c+1}) tensor; the centre (A_{r,0}, or A_{r,1} when
  column 0 kept its natural basis) has unit norm.
* Scale.  Each column's local weights w_c are divided by the largest entry of
  its MPO tensor (``scaled_row``; the logs go to the row's log-scale), so that
  products of tables, each at most 1 but far below it where the others peak,
  do not underflow in the blocks (the 12x12 d=24 workload at beta = 4 lost
  every fitted row to zero without it).
* The bottom row.  E~_{rows-1} = F_{rows-1} is a chain of nearest-neighbour
  factors; with chi >= d it is written exactly as an MPS of bond d (x_c on the
  bond, non-negative tensors, ``bottom_row``).  A fit would keep chi > d
  directions at its inner cuts, the ones beyond the exact rank d carrying no
  weight, and later updates project the next row onto whatever completion an
  implementation picked there (measured: 6e-7 in log Z on a well-conditioned
  4x5 lattice).  With chi < d it is fitted like the other rows.
* One row step (the paper's "SVDTruncate" with "num_sweeps" and
  "graduate_truncation", read as two-site variational fitting):
    1. target T = W_r psi, with psi = the normalised previous boundary MPS and W_r
       the row MPO whose site tensor at column c is
       W_c[(a, e), x, y] = w_c(x) V_c(x, y) H_{c-1}(a, x) D_{c-1}(a, y) A_{c-1}(x, e),
       left bond (a, e) = (x_{c-1}, y_{c-1}), right bond (x_c, y_c);
    2. initial guess phi_c[x] = w_c(x) sum_y V_c(x, y) psi_c[y] (previous row's bond
       dimensions), brought to right-canonical form by LQ factorisations;
    3. ``num_sweeps`` sweeps; each is a left-to-right then a right-to-left pass of
       two-site updates.  An update at columns (c, c+1) forms the exact projection of
       T onto the orthonormal left/right environment bases,
       B = <env_L| T |env_R>, and splits it by the truncated SVD of ``linalg``
       (at most chi kept directions; a side with at most chi rows or columns
       keeps its natural basis, so cuts that truncate nothing rotate nothing);
       the last update of a sweep, at columns (0, 1), keeps the natural basis
       on column 0 whenever that side has at most chi rows;
    4. normalise: lam_r = lam_{r+1} + log of the norm of the final centre.

Where no cut truncates (narrow strips at the exact rank) every tensor is then
a product of non-negative factors and the row functions keep full relative
accuracy; rotations of non-negative blocks into signed factors are where FP64
accuracy is lost on low-temperature instances, because the next row's couplings
select entries far below the largest.

Parity status: the exact regime (chi >= every exact Schmidt rank) is pinned
against brute force and the exact row transfer, including king's strips at the
workloads' d and beta (tests/test_oracle_strips.py); the truncated regime is
pinned by invariants (normalisation, error against the exact row transfer
falling with chi) - "parity unpinned" beyond those, as any truncated
contraction is defined by its own protocol.
"""
from __future__ import annotations

import numpy as np

from .energy import Weights
from .linalg import svd_truncate_left, svd_truncate_right


def row_weights(W: Weights, r: int):
    """Per-column factor arrays of row r: w_c, V_c, and the left couplings
    (H_{c-1}, D_{c-1}, A_{c-1}) as (a-dim x d) arrays, ones for c = 0.
    For the bottom row the vertical couplings are all ones."""
    inst = W.inst
    R, C, d = inst.rows, inst.cols, inst.d
    w = [W.loc[r, c] for c in range(C)]
    if r < R - 1:
        V = [W.v[r, c] for c in range(C)]
    else:
        V = [np.ones((d, d)) for _ in range(C)]
    Hl, Dl, Al = [np.ones((1, d))], [np.ones((1, d))], [np.ones((d, 1))]
    for c in range(1, C):
        Hl.append(W.h[r, c - 1])                              # [x_{c-1}][x_c]
        if r < R - 1:
            Dl.append(W.dg[r, c - 1])                         # [x_{c-1}][y_c]
            Al.append(W.an[r, c - 1])                         # [x_c][y_{c-1}]
        else:
            Dl.append(np.ones((d, d)))
            Al.append(np.ones((d, d)))
    return w, V, Hl, Dl, Al


def _left_part(EL, psi, w, V, Hl, Dl, Al):
    """P[p, x, y, Q] = sum_{a, e, q} E^L[p, a, e, q] W_c[(a, e), x, y] psi_c[q, y, Q]
    (the left environment pushed through column c, before phi_c is applied)."""
    T1 = np.einsum("paeq,xe->paxq", EL, Al)              # A_{c-1}(x, e), sum e
    T2 = np.einsum("paxq,ax,ay->pxyq", T1, Hl, Dl)       # H_{c-1}(a, x) D_{c-1}(a, y), sum a
    T3 = np.einsum("pxyq,qyQ->pxyQ", T2, psi)            # psi_c, sum q
    return T3 * (w[:, None] * V)[None, :, :, None]       # w_c(x) V_c(x, y)


def _right_part(ER, psi, w, V):
    """Q[q, x, y, P] = w_c(x) V_c(x, y) sum_{Q} psi_c[q, y, Q] E^R_{c+1}[P, x, y, Q]."""
    T = np.einsum("qyQ,PxyQ->qxyP", psi, ER)
    return T * (w[:, None] * V)[None, :, :, None]


def env_left(EL, phi, psi, w, V, Hl, Dl, Al):
    """E^L_{c+1}[P, x, y, Q] = sum E^L_c[p, a, e, q] phi_c[p, x, P] W_c[(a, e), x, y] psi_c[q, y, Q]."""
    P = _left_part(EL, psi, w, V, Hl, Dl, Al)
    return np.einsum("pxP,pxyQ->PxyQ", phi, P)


def env_right(ER, phi, psi, w, V, Hl, Dl, Al):
    """E^R_c[p, a, e, q] = sum phi_c[p, x, P] W_c[(a, e), x, y] psi_c[q, y, Q] E^R_{c+1}[P, x, y, Q]."""
    G1 = np.einsum("pxP,PxyQ->pxyQ", phi, ER)            # phi_c, sum P
    G2 = np.einsum("pxyQ,qyQ->pxyq", G1, psi)            # psi_c, sum Q
    G2 = G2 * (w[:, None] * V)[None, :, :, None]         # w_c(x) V_c(x, y)
    G3 = np.einsum("pxyq,ay->pxaq", G2, Dl)              # D_{c-1}(a, y), sum y
    return np.einsum("pxaq,ax,xe->paeq", G3, Hl, Al)     # H_{c-1}(a, x) A_{c-1}(x, e), sum x


def two_site_block(EL, ER, psi0, psi1, f0, f1):
    """B[p, x, z, P] = <env_L| W_c psi_c W_{c+1} psi_{c+1} |env_R> at columns (c, c+1),
    x = x_c, z = x_{c+1}."""
    w0, V0, H0, D0, A0 = f0
    w1, V1, H1, D1, A1 = f1
    P = _left_part(EL, psi0, w0, V0, H0, D0, A0)         # [p, x, y, Q]
    Q = _right_part(ER, psi1, w1, V1)                    # [Q, z, v, P]
    P2 = np.einsum("pxyQ,zy->pxzQ", P, A1)               # A_c(x_{c+1}, y_c), sum y
    Q2 = np.einsum("QzvP,xv->QxzP", Q, D1)               # D_c(x_c, y_{c+1}), sum v
    B = np.einsum("pxzQ,QxzP->pxzP", P2, Q2)             # sum Q
    return B * H1[None, :, :, None]                      # H_c(x_c, x_{c+1})


def _norm(T):
    s = float(np.linalg.norm(T))
    return (T / s, np.log(s)) if s > 0 else (T, 0.0)


def right_canonicalize(phi):
    """LQ sweep from the right: phi_c (c >= 1) become right isometries."""
    phi = [t.copy() for t in phi]
    for c in range(len(phi) - 1, 0, -1):
        bl, d, br = phi[c].shape
        Q, Rr = np.linalg.qr(phi[c].reshape(bl, d * br).T, mode="reduced")
        k = Q.shape[1]
        phi[c] = Q.T.reshape(k, d, br)
        # the folded factor only carries the guess's scale, which no later step
        # uses (phi_0 and phi_1 are overwritten before they are read): keep it
        # at unit norm so that it cannot overflow over many columns
        phi[c - 1] = _norm(np.einsum("pxq,kq->pxk", phi[c - 1], Rr))[0]
    return phi


def row_step(psi, fac, chi, num_sweeps):
    """One boundary-MPS row update: returns (phi, log_scale) with T ~
    exp(log_scale) phi, the centre tensor normalised (phi_0, or phi_1 when
    the last update kept the natural basis at column 0) and the tensors to
    its right right-canonical."""
    C = len(psi)
    w, V, Hl, Dl, Al = fac
    f = [(w[c], V[c], Hl[c], Dl[c], Al[c]) for c in range(C)]
    phi = [np.einsum("x,xy,pyP->pxP", w[c], V[c], psi[c]) for c in range(C)]
    phi = right_canonicalize(phi)
    d = psi[0].shape[1]
    EL = [None] * (C + 1)
    ER = [None] * (C + 1)
    EL[0] = (np.ones((1, 1, 1, 1)), 0.0)
    ER[C] = (np.ones((1, d, d, 1)), 0.0)

    def build_ER(c):
        T, s = ER[c + 1]
        T2, s2 = _norm(env_right(T, phi[c], psi[c], *f[c]))
        ER[c] = (T2, s + s2)

    def build_EL(c):
        T, s = EL[c]
        T2, s2 = _norm(env_left(T, phi[c], psi[c], *f[c]))
        EL[c + 1] = (T2, s + s2)

    def block(c):
        B = two_site_block(EL[c][0], ER[c + 2][0], psi[c], psi[c + 1], f[c], f[c + 1])
        pl, _, _, pr = B.shape
        return B.reshape(pl * d, d * pr), pl, pr, EL[c][1] + ER[c + 2][1]

    lam = 0.0
    centre = 0
    for _ in range(num_sweeps):
        for c in range(C - 1, 1, -1):
            build_ER(c)
        # left-to-right pass
        for c in range(C - 1):
            Bm, pl, pr, s = block(c)
            if c < C - 2:
                U, Rm = svd_truncate_left(Bm, chi)
                phi[c] = U.reshape(pl, d, -1)
                phi[c + 1] = Rm.reshape(-1, d, pr)
                build_EL(c)
            else:
                Lm, Vt = svd_truncate_right(Bm, chi)
                phi[c] = Lm.reshape(pl, d, -1)
                phi[c + 1] = Vt.reshape(-1, d, pr)
                lam = s
                centre = 0
                if C > 2:
                    build_ER(c + 1)
        # right-to-left pass
        for c in range(C - 3, -1, -1):
            Bm, pl, pr, s = block(c)
            if c == 0 and Bm.shape[0] <= chi:
                # last update of the sweep with nothing to truncate on the left:
                # natural basis there, the block itself becomes the centre
                phi[0] = np.eye(Bm.shape[0]).reshape(pl, d, -1)
                phi[1] = Bm.reshape(-1, d, pr)
                centre = 1
            else:
                Lm, Vt = svd_truncate_right(Bm, chi)
                phi[c] = Lm.reshape(pl, d, -1)
                phi[c + 1] = Vt.reshape(-1, d, pr)
                centre = 0
            lam = s
            if c > 0:
                build_ER(c + 1)
    phi[centre], s0 = _norm(phi[centre])
    return phi, lam + s0


def site_log_scales(fac):
    """log of the largest entry of each column's MPO tensor,
    max over (a, e, x, y) of w_c(x) V_c(x, y) H_{c-1}(a, x) D_{c-1}(a, y) A_{c-1}(x, e)
    = max over (x, y) of [w V](x, y) max_a [H D](a, x, y) max_e A(x, e), in logs."""
    w, V, Hl, Dl, Al = fac
    out = []
    with np.errstate(divide="ignore"):
        for c in range(len(w)):
            t = (np.log(Hl[c])[:, :, None] + np.log(Dl[c])[:, None, :]).max(axis=0)   # [x][y]
            v = np.log(w[c])[:, None] + np.log(V[c]) + t + np.log(Al[c]).max(axis=1)[:, None]
            out.append(float(v.max()))
    return out


def scaled_row(W: Weights, r: int):
    """The row's factors with each column's w_c divided by the largest entry of
    its MPO tensor, and the sum of the logs of those divisors.  Every table is
    at most 1, but their products over a column fall far below (at beta = 4
    with 8-spin clusters, to 1e-100 and less), so that blocks built from them
    underflow; with this constant per column (returned to the log-scale) each
    MPO tensor's largest entry is 1."""
    w, V, Hl, Dl, Al = row_weights(W, r)
    ls = site_log_scales((w, V, Hl, Dl, Al))
    return ([w[c] * np.exp(-ls[c]) for c in range(len(w))], V, Hl, Dl, Al), float(sum(ls))


def bottom_row(fac):
    """E~_{rows-1} = F_{rows-1} written exactly, x_c carried on the bond:
    A_c[a, x, x'] = H_{c-1}(a, x) w_c(x) delta(x, x') (bond d, non-negative;
    the last column closes the bond).  Each tensor is divided by its norm and
    the logs are summed into the log-scale."""
    w, _, Hl, _, _ = fac
    C, d = len(w), w[0].shape[0]
    out, lam = [], 0.0
    for c in range(C):
        core = Hl[c] * w[c][None, :]                       # [a][x]
        A = core[:, :, None] * np.eye(d)[None] if c < C - 1 else core[:, :, None]
        A, s = _norm(A)
        out.append(A)
        lam += s
    return out, lam


def boundary_mps(inst, chi: int, num_sweeps: int = 1):
    """All boundary MPSs, bottom row first.  Returns dict with
    'A' [rows][cols] tensors, 'lam' [rows] log-scales and 'logZ'."""
    if inst.cols < 2:
        raise ValueError("cols >= 2 required")
    W = Weights(inst)
    R, C, d = inst.rows, inst.cols, inst.d
    A = [None] * R
    lam = [0.0] * R
    e0 = np.zeros((1, d, 1))
    e0[0, 0, 0] = 1.0
    psi = [e0.copy() for _ in range(C)]          # E~_rows = 1 through y = 0 (couplings are ones)
    prev = 0.0
    for r in range(R - 1, -1, -1):
        fac, ls = scaled_row(W, r)
        if r == R - 1 and chi >= d:
            phi, s = bottom_row(fac)             # exact at bond d: nothing to fit
        else:
            phi, s = row_step(psi, fac, chi, num_sweeps)
        s += ls
        A[r] = phi
        lam[r] = prev + s
        prev = lam[r]
        psi = phi
    # log Z = lam_0 + log sum_X A_0[x_0]..A_{C-1}[x_{C-1}] - beta * shift
    v = np.ones(1)
    for c in range(C):
        v = v @ A[0][c].sum(axis=1)
    logZ = lam[0] + float(np.log(v[0])) - inst.beta * W.shift
    return {"A": A, "lam": lam, "logZ": logZ}


def mps_full(A_row) -> np.ndarray:
    """Dense function of a row MPS (small cases only)."""
    T = A_row[0][0]                                     # (d, chi_1)
    for c in range(1, len(A_row)):
        T = np.tensordot(T, A_row[c], axes=([T.ndim - 1], [0]))
    return T[..., 0]
