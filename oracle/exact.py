"""Exact references (oracle; test infrastructure only).

* ``brute_force``: enumerate all d^N configurations (Eq. (1)); partition function
  Z = sum exp(-beta E), ground energy, and every prefix marginal in the
  row-major variable order.  Pinned by closed forms (beta = 0, no couplings,
  open 1-D chains) in tests/test_oracle_exact.py.
* ``row_transfer``: exact contraction of the Boltzmann PEPS (Sec. 2, Fig. 1(c))
  one lattice row at a time, with the whole row state as a dense vector of
  d^cols entries, in the log domain (the workloads' row functions span more
  than the FP64 range).  Pinned against ``brute_force``.
* ``exact_conditionals``: p(x_k | x_<k) from the row-transfer vectors, i.e. the
  conditional marginals the branch-and-bound search consumes (Fig. 1(d)).

Plain definitions used (Sec. 2):  p(x) = exp(-beta E(x)) / Z,
P(x_<=k) = sum over the later variables of p(x), p(x_k | x_<k) = P(x_<=k) / P(x_<k).
"""
from __future__ import annotations

import numpy as np
from scipy.special import logsumexp

from .energy import potts_energy, Weights


def all_configs(N: int, d: int) -> np.ndarray:
    """[d^N][N] in lexicographic (row-major site) order."""
    idx = np.arange(d ** N)
    return (idx[:, None] // (d ** np.arange(N - 1, -1, -1))[None, :]) % d


def brute_force(inst, max_states: int = 1 << 22) -> dict:
    N, d = inst.n_sites, inst.d
    if d ** N > max_states:
        raise ValueError("instance too large for brute force")
    X = all_configs(N, d)
    E = potts_energy(inst, X)
    logw = -inst.beta * E
    logZ = float(logsumexp(logw))
    # prefix log-marginals: log P(x_<=k) for every prefix of length k+1
    prefix = []
    lw = logw.copy()
    for k in range(N, 0, -1):
        prefix.append(lw - logZ)                        # indexed by the first k sites
        lw = logsumexp(lw.reshape(-1, d), axis=1)       # marginalise site k-1
    prefix = prefix[::-1]                               # prefix[k-1] has d^k entries
    order = np.lexsort((np.arange(len(E)), E))
    return {"logZ": logZ, "E": E, "X": X, "E_min": float(E.min()),
            "argmin": X[order[0]], "prefix_logp": prefix}


def prefix_logp(bf: dict, cfg_prefix) -> float:
    """log P(x_<=k) for a given prefix (length k+1) from a brute-force table."""
    k = len(cfg_prefix)
    d = int(round(len(bf["prefix_logp"][0])))
    idx = 0
    for x in cfg_prefix:
        idx = idx * d + int(x)
    return float(bf["prefix_logp"][k - 1][idx])


def log_row_factor(W: Weights, r: int) -> np.ndarray:
    """log F_r(X) = sum_c log w_{r,c}(x_c) + sum_c log W^H_{r,c}(x_c, x_{c+1}) as a
    dense tensor with one axis per column."""
    C, d = W.inst.cols, W.inst.d
    F = W.log_loc[r, 0].copy()
    for c in range(1, C):
        F = F[..., :, None] + W.log_h[r, c - 1][(None,) * (c - 1) + (slice(None), slice(None))]
        F = F + W.log_loc[r, c][(None,) * c + (slice(None),)]
    return F.reshape((d,) * C)


def log_apply_couplings(W: Weights, r: int, LY: np.ndarray) -> np.ndarray:
    """log sum_Y G_r(X, Y) exp(LY(Y)), with G_r the product of the V, D and A
    weights between row r (X) and row r+1 (Y); LY holds log Phi(Y).  The sum
    over Y is done one column at a time (log-sum-exp), each y_c summed once
    all three of its couplings are applied."""
    C, d = W.inst.cols, W.inst.d
    T = LY                                          # axes: y_0..y_{C-1}
    for c in range(C):
        # axes now: x_0..x_{c-1}, [y_{c-1}], y_c..y_{C-1}
        if c > 0:
            # introduce x_c through A(x_c, y_{c-1}) and sum y_{c-1}
            T = np.moveaxis(T, c, -1)                # y_{c-1} last
            T = logsumexp(T[..., None, :] + W.log_an[r, c - 1], axis=-1)   # -> x_c last
            T = np.moveaxis(T, -1, c)                # x_c at position c
        else:
            T = np.repeat(T[None], d, axis=0)        # axis for x_0
        shp = [1] * T.ndim
        shp[c], shp[c + 1] = d, d
        T = T + W.log_v[r, c].reshape(shp)           # V(x_c, y_c)
        if c > 0:
            shp = [1] * T.ndim
            shp[c - 1], shp[c + 1] = d, d
            T = T + W.log_dg[r, c - 1].reshape(shp)     # D(x_{c-1}, y_c)
    return logsumexp(T, axis=C)                      # y_{C-1}: no pending coupling


def row_transfer(inst, max_row_states: int = 1 << 16) -> tuple:
    """Exact boundary functions in the log domain (no under- or overflow at
    any temperature): log E~_{rows-1} = log F_{rows-1} and
    log E~_r = log F_r + log sum_Y G_r(., Y) E~_{r+1}(Y).
    Returns (list of dense log E~_r indexed by r, logZ)."""
    W = Weights(inst)
    R, C, d = inst.rows, inst.cols, inst.d
    if d ** C > max_row_states:
        raise ValueError("row too wide for the exact transfer")
    out = [None] * R
    out[R - 1] = log_row_factor(W, R - 1)
    for r in range(R - 2, -1, -1):
        out[r] = log_row_factor(W, r) + log_apply_couplings(W, r, out[r + 1])
    logZ = float(logsumexp(out[0]) - inst.beta * W.shift)
    return out, logZ


def normalised(L: np.ndarray) -> np.ndarray:
    """A log row function as a dense function with largest entry 1."""
    return np.exp(L - L.max())


def log_fields(W: Weights, r: int, above: np.ndarray) -> np.ndarray:
    """log g_c(x) for c = 0..cols-1: the couplings between x = x_{r,c} and the
    fixed row above (V from (r-1,c), D from (r-1,c-1), A from (r-1,c+1)).
    All zero for r = 0."""
    C, d = W.inst.cols, W.inst.d
    g = np.zeros((C, d))
    if r == 0:
        return g
    for c in range(C):
        g[c] += W.log_v[r - 1, c][above[c], :]
        if c > 0:
            g[c] += W.log_dg[r - 1, c - 1][above[c - 1], :]
        if c < C - 1:
            g[c] += W.log_an[r - 1, c][above[c + 1], :]
    return g


def exact_conditionals(inst, rows_log, cfg_prefix) -> np.ndarray:
    """p(x_k = s | x_<k) for the next site k = len(cfg_prefix), from the exact
    log E~_r of ``row_transfer``.

    Given rows 0..r-1 fixed and x_{r,0..c-1} fixed, the unnormalised weight of
    x_{r,c} = s is sum over x_{r,c+1..} of prod_c' g_c'(x_c') E~_r(X_r)
    (log-sum-exp)."""
    W = Weights(inst)
    C, d = inst.cols, inst.d
    k = len(cfg_prefix)
    r, c = divmod(k, C)
    above = np.asarray(cfg_prefix[(r - 1) * C: r * C]) if r > 0 else None
    g = log_fields(W, r, above)
    v = rows_log[r]
    for cc in range(C):
        shp = [1] * C
        shp[cc] = d
        v = v + g[cc].reshape(shp)
    for cc in range(c):
        v = v[cfg_prefix[r * C + cc]]
    lq = logsumexp(v.reshape(d, -1), axis=1)
    return np.exp(lq - logsumexp(lq))
