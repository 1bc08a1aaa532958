"""Beam search with a learned proposal and an exactness guard (oracle; test
infrastructure only).

The proposal is not in the paper (a learned heuristic; its predictions are
"parity unpinned").  What this module pins is the rule that makes its use safe:
with the guard below the finite part of the final beam is the one the plain
search of oracle.search.beam_search keeps (Sec. 2, Fig. 1(d)-(e)), whatever the
network predicts, as long as no exact conditional weight q(b, s) is negative.

Per site, with parents b sorted by score (score_0 the best) and d states:
1. pred(b, s) = score_b + log softmax_s(logit(b, s)) from the network.
2. Candidate set E: bin j(b, s) = floor(64 (score_0 - pred)), clamped to
   [0, NBINS-1] (-inf and NaN go to the last bin); K = ceil(kappa M); j* the
   first bin at which the running count reaches K; E = {j <= j*}, or every
   candidate when j* is the last bin or the count never reaches K.
3. Exact weights for E only.  Z_b = L^b R_c (the right environment one column
   further left, so Z_b = sum over all s of q(b, s) with no extra work);
   U_b = Z_b - sum_{s in E_b} q(b, s) is the weight of b's unevaluated children.
   Score of an evaluated child: score_b + log(q / Z_b).  Upper bound of any
   unevaluated child: bound_b = score_b + log((max(U_b, 0) + EPS Z_b) / Z_b)
   (-inf when E_b holds every state).  A parent with Z_b <= 0, a non-finite Z_b
   or a negative evaluated q is marked for fallback.
4. tau = the M-th best exact score over E (-inf when |E| < M).
5. Fallback parents: marked ones and those with an unevaluated child and
   bound_b >= tau - MARGIN.  Their d children are evaluated exactly as in the
   plain search (normaliser sum_s max(q, 0)).
6. The M best of the evaluated children by (score desc, id asc), id = b d + s,
   after the cut-off rule of the plain search.
A child outside E of a parent that does not fall back scores at most
bound_b < tau - MARGIN <= the true M-th score, so it cannot be kept.
"""
from __future__ import annotations

import math

import numpy as np

from .energy import Weights, potts_energy
from .mlp import features, forward
from .search import _fields, delta_energy, marginals, log_conditionals, select_top

NBINS = 2048
BIN_SCALE = 64.0
EPS = 1e-9
MARGIN = 1e-9


def candidate_set(pred, score0, K):
    """Boolean mask of E (step 2)."""
    with np.errstate(invalid="ignore"):
        gap = (score0 - pred) * BIN_SCALE
    j = np.where(np.isfinite(gap), np.floor(np.clip(gap, 0.0, NBINS - 1)), NBINS - 1)
    j = j.astype(np.int64)
    counts = np.bincount(j.ravel(), minlength=NBINS)
    cum = np.cumsum(counts)
    hit = np.nonzero(cum >= K)[0]
    if hit.size == 0 or hit[0] == NBINS - 1:
        return np.ones(pred.shape, dtype=bool)
    return j <= hit[0]


def guided_beam_search(inst, A, M, params, H, kappa=2.0, cut_off_prob=0.0, stats=None):
    """The search of oracle.search.beam_search with the proposal and guard.
    ``stats`` (optional dict) receives 'exact' (exact child evaluations),
    'candidates' (all children) and 'fallback' (fallback parents)."""
    W = Weights(inst)
    Rr, C, d = inst.rows, inst.cols, inst.d
    N = Rr * C
    K = math.ceil(kappa * M)
    cfg = np.zeros((1, N), dtype=np.int64)
    score = np.zeros(1)
    n_exact = n_cand = n_fb = 0
    for r in range(Rr):
        above = cfg[:, (r - 1) * C: r * C] if r > 0 else None
        g_anc = _fields(W, r, above)
        # right environments without normalisation of the last step, so that
        # Z_b = L^b . Rt[c] is on the scale of q(b, s) = g L^b A_c[s] R[c+1]
        R = [None] * (C + 1)
        Rt = [None] * (C + 1)
        R[C] = np.ones((cfg.shape[0], 1))
        for c in range(C - 1, -1, -1):
            Rt[c] = np.einsum("asz,bz,bs->ba", A[r][c], R[c + 1], g_anc[:, c])
            m = np.abs(Rt[c]).max(axis=1, keepdims=True)
            R[c] = Rt[c] / np.where(m > 0, m, 1.0)
        anc = np.arange(cfg.shape[0])
        L = np.ones((cfg.shape[0], 1))
        for c in range(C):
            B = cfg.shape[0]
            n_cand += B * d
            f = features(inst, A, r, c, cfg, score)
            pred = score[:, None] + forward(params, H, f)
            E = candidate_set(pred, score.max(), K)
            q = marginals(A[r][c], g_anc[anc, c], L, R[c + 1][anc])     # all, used only on E
            Z = np.einsum("ba,ba->b", L, Rt[c][anc])
            n_exact += int(E.sum())
            cand = np.full((B, d), -np.inf)
            have = np.zeros((B, d), dtype=bool)
            bound = np.full(B, -np.inf)
            mark = np.zeros(B, dtype=bool)
            for b in range(B):
                Eb = E[b]
                if not np.isfinite(Z[b]) or Z[b] <= 0 or (q[b, Eb] < 0).any():
                    mark[b] = True
                    continue
                with np.errstate(divide="ignore"):
                    cand[b, Eb] = score[b] + np.log(q[b, Eb]) - np.log(Z[b])
                have[b, Eb] = True
                if not Eb.all():
                    U = Z[b] - q[b, Eb].sum()
                    bound[b] = score[b] + math.log((max(U, 0.0) + EPS * Z[b]) / Z[b])
            ev = cand[have]
            tau = np.sort(ev)[::-1][M - 1] if ev.size >= M else -np.inf
            fb = mark | (~E.all(axis=1) & (bound >= tau - MARGIN))
            dE = delta_energy(inst, cfg, r, c)
            for b in np.nonzero(fb)[0]:
                cand[b] = score[b] + log_conditionals(q[b: b + 1], dE[b: b + 1], inst.beta)[0]
                have[b] = True
                n_exact += d
                n_fb += 1
            if cut_off_prob > 0:
                best = cand[have].max()
                cand = np.where(cand >= best + np.log(cut_off_prob), cand, -np.inf)
            # unevaluated children take no part in the selection
            flat = np.where(have, cand, np.nan).reshape(-1)
            ids = np.nonzero(have.reshape(-1))[0]
            keep = ids[select_top(flat[ids], M)]
            b, s = np.divmod(keep, d)
            cfg = cfg[b].copy()
            cfg[:, r * C + c] = s
            score = cand.reshape(-1)[keep]
            Lb = np.einsum("ba,baz->bz", L[b], np.transpose(A[r][c][:, s, :], (1, 0, 2)))
            Lb = Lb * g_anc[anc[b], c, s][:, None]
            m = np.abs(Lb).max(axis=1, keepdims=True)
            L = Lb / np.where(m > 0, m, 1.0)
            anc = anc[b]
    if stats is not None:
        stats.update(exact=n_exact, candidates=n_cand, fallback=n_fb)
    E = potts_energy(inst, cfg)
    return {"beam_states": cfg, "beam_scores": score, "energies": E,
            "n_valid": int(np.isfinite(score).sum())}
