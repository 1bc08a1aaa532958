"""Counter-based generator and truncated SVD (oracle; test infrastructure only).

SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014; the 64-bit finaliser constants of S. Vigna's public
reference implementation): output number i (i = 1, 2, ...) from seed s is
mix(s + i * 0x9E3779B97F4A7C15).  Pinned by the reference implementation's
published first outputs for seed 0.  Used for the learned proposal's initial
weights.

Truncated SVD ("SVDTruncate"; the paper names it in its MpsParameters example,
Sec. 3.1, without defining it).  The reading adopted here is the plain
definition: keep the k largest singular triplets of the block.  Two points
are fixed beyond that definition:

* the singular value decomposition is computed by LAPACK's preconditioned
  one-sided Jacobi method (dgejsv, through scipy; Drmac and Veselic, SIAM J.
  Matrix Anal. Appl. 29, 2008), which determines small singular values and
  their vectors to high relative accuracy for matrices whose rows or columns
  carry very different scales (Demmel and Veselic, 1992).  The boundary
  functions of the workloads span hundreds of orders of magnitude and the
  next row's couplings select entries far below the largest, so a method
  with only absolute accuracy (bidiagonalisation) loses them;
* a block with at most chi rows (left split) or columns (right split) needs
  no truncation: it keeps its natural basis, B = I B or B I.  The function is
  the one the SVD would return, without rotating a non-negative block into
  signed factors.

Pinned in tests/test_oracle_linalg.py: agreement with numpy's dense SVD on
well-conditioned matrices, singular values of graded matrices known in
closed form, optimality of the rank-k error (Eckart-Young), and the
natural-basis cases.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg.lapack as lapack

GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(seed: int, idx) -> np.ndarray:
    """Output number idx+1 of SplitMix64 started from ``seed`` (vectorised)."""
    with np.errstate(over="ignore"):
        z = (np.uint64(seed) + (np.asarray(idx, dtype=np.uint64) + np.uint64(1))
             * np.uint64(GOLDEN))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def svd(B: np.ndarray):
    """Thin SVD B = U diag(s) Vt, singular values descending, by LAPACK's
    one-sided Jacobi driver (dgejsv needs rows >= columns; a wide matrix is
    handled through its transpose)."""
    m, n = B.shape
    if m < n:
        U, s, Vt = svd(B.T)
        return Vt.T, s, U.T
    if n == 0 or not np.any(B):
        return np.eye(m, n), np.zeros(n), np.eye(n)
    # joba=0 ('C'): high relative accuracy for column-scaled matrices;
    # jobu=0 ('U'): the n left vectors; jobv=0 ('V'): the right vectors;
    # jobp=0 ('N'): no perturbation of tiny entries
    sva, u, v, work, _, info = lapack.dgejsv(np.asfortranarray(B), joba=0, jobu=0, jobv=0,
                                             jobp=0)
    if info != 0:
        raise np.linalg.LinAlgError(f"dgejsv info={info}")
    s = sva[:n] * (work[0] / work[1])      # LAPACK returns scaled singular values
    return u[:, :n], s, v[:n, :n].T


def svd_truncate_left(B: np.ndarray, chi: int):
    """Split B ~ U @ Rm with U^T U = I and at most chi columns.  With at most
    chi rows nothing needs truncating and the natural basis is kept: U = I,
    Rm = B.  Otherwise U = the min(chi, cols) dominant left singular vectors
    and Rm = diag(s) Vt of the same triplets."""
    m, n = B.shape
    if m <= chi:
        return np.eye(m), B.copy()
    kk = min(chi, n)
    U, s, Vt = svd(B)
    return U[:, :kk], s[:kk, None] * Vt[:kk]


def svd_truncate_right(B: np.ndarray, chi: int):
    """Split B ~ Lm @ V with V V^T = I: ``svd_truncate_left`` of B^T,
    transposed (natural basis when B has at most chi columns)."""
    U, Rm = svd_truncate_left(B.T, chi)
    return Rm.T, U.T
