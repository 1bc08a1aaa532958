"""Learned branch proposal: candidate features and the 2-layer MLP (oracle;
test infrastructure only).

The proposal network is not in the paper; it ranks the children (b, s) of the
beam before exact marginals are computed, so that the exact contraction runs
only for the most promising ones.  Its predictions carry no parity claim
("parity unpinned": a learned heuristic); what is pinned is the arithmetic:
the features against their definitions, the forward pass, and the analytic
backward pass against central finite differences.

Features of candidate (b, s) at site (r, c), F = 6, each clamped at -30 and
divided by 10 where marked (*):
  0*  -beta dE(b, s) - max_s' (-beta dE(b, s'))       energy the choice adds (Eq. (1))
  1*  la(b, s) - max_s' la(b, s')    look-ahead: la = sum over the unexplored
      neighbours n of log sum_y exp(-beta (E_n(y) + E_(rc),n(s, y)))
  2*  lm(s) - max_s' lm(s')   lm = log of the one-site weight of the boundary MPS,
      l_c A_{r,c}[:, s, :] r_{c+1}, l and r the unconditioned (summed) environments
  3   c / (cols - 1)
  4   r / (rows - 1)
  5*  score(b) - max_b' score(b')
Network: h = relu(W1 f + b1), logit = w2 . h + b2, p^(s | b) = softmax_s(logit).
Loss: cross-entropy -sum_b sum_s p(s|b) log p^(s|b) / n_beams.
"""
from __future__ import annotations

import numpy as np


F = 6


def _rel(x):
    x = x - x.max(axis=-1, keepdims=True)
    return np.maximum(x, -30.0) / 10.0


def one_site_logw(A_row, c):
    """lm(s) = log max(l_c A_c[:, s, :] r_{c+1}, tiny), l/r summed over states."""
    l = np.ones(1)
    for cc in range(c):
        l = l @ A_row[cc].sum(axis=1)
        l = l / np.abs(l).max()
    r = np.ones(1)
    for cc in range(len(A_row) - 1, c, -1):
        r = A_row[cc].sum(axis=1) @ r
        r = r / np.abs(r).max()
    m = np.einsum("a,asz,z->s", l, A_row[c], r)
    return np.log(np.maximum(m, 1e-300))


def lookahead(inst, r, c, cfg):
    """la[b, s] over the unexplored neighbours of (r, c): right (H), below (V),
    below-right (D) and below-left (the A edge of (r, c-1))."""
    b = inst.beta
    R, C, d = inst.rows, inst.cols, inst.d
    la = np.zeros((cfg.shape[0], d))

    def add(table_sy, En):
        # log sum_y exp(-beta (E_n(y) + E(s, y)))
        x = -b * (En[None, :] + table_sy)
        m = x.max(axis=1, keepdims=True)
        return (m + np.log(np.exp(x - m).sum(axis=1, keepdims=True)))[:, 0]

    v = np.zeros(d)
    if c + 1 < C:
        v += add(inst.pair_h[r, c], inst.local_E[r, c + 1])
    if r + 1 < R:
        v += add(inst.pair_v[r, c], inst.local_E[r + 1, c])
        if inst.kings and c + 1 < C:
            v += add(inst.pair_d[r, c], inst.local_E[r + 1, c + 1])
        if inst.kings and c > 0:
            v += add(inst.pair_a[r, c - 1], inst.local_E[r + 1, c - 1])
    la[:] = v[None, :]
    return la


def features(inst, A, r, c, cfg, score):
    """[B][d][F] float64 features of the children of the partial configurations
    ``cfg`` (rows 0..r-1 and columns 0..c-1 of row r fixed) with scores ``score``."""
    from .search import delta_energy
    B, d = cfg.shape[0], inst.d
    f = np.zeros((B, d, F))
    f[:, :, 0] = _rel(-inst.beta * delta_energy(inst, cfg, r, c))
    f[:, :, 1] = _rel(lookahead(inst, r, c, cfg))
    f[:, :, 2] = _rel(np.repeat(one_site_logw(A[r], c)[None, :], B, axis=0))
    f[:, :, 3] = c / max(inst.cols - 1, 1)
    f[:, :, 4] = r / max(inst.rows - 1, 1)
    gap = np.maximum(score - score.max(), -30.0) / 10.0
    f[:, :, 5] = gap[:, None]
    return f


def init_params(H: int, seed: int):
    """Deterministic initial parameters (He-style scale), flat layout
    [W1 (H x F) row-major, b1 (H), w2 (H), b2 (1)]."""
    from .linalg import splitmix64
    n = H * F + H + H + 1
    z = splitmix64(seed, np.arange(n))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0) * 2.0 - 1.0
    p = np.zeros(n)
    p[: H * F] = u[: H * F] * np.sqrt(6.0 / F)
    p[H * F + H: H * F + 2 * H] = u[H * F + H: H * F + 2 * H] * np.sqrt(6.0 / H)
    return p


def unpack(p, H):
    W1 = p[: H * F].reshape(H, F)
    b1 = p[H * F: H * F + H]
    w2 = p[H * F + H: H * F + 2 * H]
    b2 = p[H * F + 2 * H]
    return W1, b1, w2, b2


def forward(p, H, feats):
    """log p^(s | b): feats [B][d][F] -> [B][d]."""
    W1, b1, w2, b2 = unpack(p, H)
    h = np.maximum(feats @ W1.T + b1, 0.0)
    logit = h @ w2 + b2
    m = logit.max(axis=1, keepdims=True)
    return logit - m - np.log(np.exp(logit - m).sum(axis=1, keepdims=True))


def loss_and_grad(p, H, feats, target_logp):
    """Cross-entropy against exact conditionals and its analytic gradient."""
    W1, b1, w2, b2 = unpack(p, H)
    B = feats.shape[0]
    pre = feats @ W1.T + b1                     # [B][d][H]
    h = np.maximum(pre, 0.0)
    logit = h @ w2 + b2                         # [B][d]
    m = logit.max(axis=1, keepdims=True)
    lse = m + np.log(np.exp(logit - m).sum(axis=1, keepdims=True))
    lp_hat = logit - lse
    pt = np.exp(target_logp)                    # exact p(s | b); -inf -> 0
    loss = float(-(np.where(pt > 0, pt * lp_hat, 0.0)).sum() / B)
    dlogit = (np.exp(lp_hat) * pt.sum(axis=1, keepdims=True) - pt) / B
    gw2 = np.einsum("bs,bsh->h", dlogit, h)
    gb2 = dlogit.sum()
    dh = dlogit[:, :, None] * w2[None, None, :]
    dpre = dh * (pre > 0)
    gW1 = np.einsum("bsh,bsf->hf", dpre, feats)
    gb1 = dpre.sum(axis=(0, 1))
    return loss, np.concatenate([gW1.ravel(), gb1, gw2, [gb2]])


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015); t counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
