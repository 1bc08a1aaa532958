"""Counter-based generator and truncated SVD protocol (oracle; test infrastructure only).

SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014; the 64-bit finaliser constants of S. Vigna's public
reference implementation): output number i (i = 1, 2, ...) from seed s is
mix(s + i * 0x9E3779B97F4A7C15).  Pinned by the reference implementation's
published first outputs for seed 0.

Truncated SVD ("SVDTruncate", the paper names it but does not define it; the
reading adopted here): a rank-k factorisation B ~ U (U^T B) with U an isometry
spanning the dominant left singular subspace, computed by the randomized range
finder with subspace (power) iteration of Halko, Martinsson and Tropp (SIAM
Review 53, 2011, Alg. 4.4 + 5.1): sketch width l = min(k + p, m, n), a fixed
sketch matrix Omega whose entries are SplitMix64 outputs mapped to [-1, 1), q
power iterations with re-orthonormalisation, then the exact SVD of the small
projected matrix (skipped when l = k: the kept subspace is then span(Q)).
When rank(B) <= l the result is the exact truncated SVD.
Directions of the kept subspace whose weight in B (the norm of their row of
U^T B) is at most NULL_TOL times the largest weight lie at the rounding floor;
any orthonormal completion could stand there, so they are discarded (zeroed)
to keep the result unique.  Pinned against numpy's dense SVD in
tests/test_oracle_linalg.py.
"""
from __future__ import annotations

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1
SKETCH_SEED = 0x5EED5EED12345678
SKETCH_LD = 1024            # row stride of the fixed sketch table
NULL_TOL = 1e-11


def splitmix64(seed: int, idx) -> np.ndarray:
    """Output number idx+1 of SplitMix64 started from ``seed`` (vectorised)."""
    with np.errstate(over="ignore"):
        z = (np.uint64(seed) + (np.asarray(idx, dtype=np.uint64) + np.uint64(1))
             * np.uint64(GOLDEN))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def sketch(n: int, l: int) -> np.ndarray:
    """Omega[i, j] = 2 u(i*SKETCH_LD + j) - 1 with u = top 53 bits / 2^53."""
    i = np.arange(n)[:, None] * SKETCH_LD + np.arange(l)[None, :]
    z = splitmix64(SKETCH_SEED, i)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def orth(Y: np.ndarray) -> np.ndarray:
    """Orthonormal basis with as many columns as Y (Householder QR)."""
    Q, _ = np.linalg.qr(Y, mode="reduced")
    return Q


def tsvd_left(B: np.ndarray, k: int, p: int, q: int):
    """Rank-min(k, m, n) split B ~ U @ Rm with U^T U = I (left isometry) and
    Rm = U^T B; U holds the dominant left singular vectors, ordered by
    decreasing singular value."""
    m, n = B.shape
    l = min(k + p, m, n)
    kk = min(k, l)
    Y = B @ sketch(n, l)
    Q = orth(Y)
    for _ in range(q):
        Qz = orth(B.T @ Q)
        Q = orth(B @ Qz)
    if l == kk:
        # the sketch width is the kept rank: the subspace is span(Q) itself
        U = Q
    else:
        Csm = Q.T @ B                           # l x n
        Us, s, _ = np.linalg.svd(Csm, full_matrices=False)
        U = Q @ Us[:, :kk]
    return drop_null(U, U.T @ B)


def drop_null(U, Rm):
    """Zero the directions (columns of U, rows of Rm) whose weight, the norm of
    their row of Rm, is at most NULL_TOL times the largest."""
    w = np.linalg.norm(Rm, axis=1)
    if w.size and w.max() > 0:
        null = w <= NULL_TOL * w.max()
        U = U.copy()
        Rm = Rm.copy()
        U[:, null] = 0.0
        Rm[null, :] = 0.0
    return U, Rm


def tsvd_right(B: np.ndarray, k: int, p: int, q: int):
    """Rank-k split B ~ Lm @ V with V V^T = I (right isometry): the transpose of
    ``tsvd_left`` applied to B^T."""
    U, Rm = tsvd_left(B.T, k, p, q)
    return Rm.T, U.T
