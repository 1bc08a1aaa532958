"""Branch-and-bound (beam) search over conditional marginals (oracle; test
infrastructure only).

The paper's search (Sec. 2, Fig. 1(d)-(e)) adds one Potts variable at a time in
a fixed order and keeps a fixed number of the most probable partial
configurations.  Adopted reading:

* order: row-major, rows top to bottom, columns left to right;
* each partial configuration b carries score(b) = sum of log p(x_k | x_<k), its
  FP64 energy of the fixed variables, and the left environment vector L^b;
* conditional at site (r, c):  q(b, s) = g^b_c(s) * L^b A_{r,c}[:, s, :] R^{a(b)}_{c+1},
  p(s | b) = q(b, s) / sum_s' q(b, s'), where g^b_c(s) are the couplings of s to the
  fixed row r-1, R^a_{c+1} the right environment of the row-start ancestor a
  (R^a_cols = 1, R^a_c = sum_s g^a_c(s) A_{r,c}[:, s, :] R^a_{c+1}); negative q
  (truncation error) counts as zero probability, and a parent with no
  positive q takes softmax_s(-beta dE(b, s)) instead (``log_conditionals``);
* keep the M best children by (score desc, parent position asc, s asc);
  with ``cut_off_prob`` > 0, children below cut_off_prob times the best child
  of the step get score -inf (they sort last and count as discarded);
* output: the final beam, energies recomputed by Eq. (1), sorted by energy
  ascending (ties keep beam order);
* merging branches (optional; the paper's merge of branches, Sec. 3.1, whose
  exact rule it leaves open): after site k, the sites still coupled to the
  unexplored ones are among the last cols + 1 sites of the order (the
  frontier); two partial configurations with the same frontier have the same
  conditional future, and the one with the lower energy of its fixed part
  completes to the lower total energy, so among the children of a step that
  share a frontier only the one with the lowest energy (ties: lowest id
  b d + s) keeps its score, the others get -inf.  Merging comes before the
  cut-off and the selection.
* droplets (optional, with merging; the paper collects low-energy excitations
  while merging, Sec. 3.1, and names only an energy cut-off and a Hamming
  cut-off): the member of a merged group that comes right after the kept one
  in (energy, id) order differs from it only in sites no longer coupled to
  the unexplored ones, so its energy gap dE to the kept one is final.  A
  state inherits its parent's droplets (stored as whole configurations, the
  new site set to the state's own value) and, if it kept a group with a
  runner-up whose dE <= energy_cutoff, takes that runner-up as a new droplet
  when its Hamming distance (sites with different states) to the state and to
  every droplet the state already holds exceeds hamming_cutoff and fewer than
  max_droplets are held.  A droplet's energy is the state's energy plus dE.

The vectors L and R only need a positive scale (it cancels in p(s | b)), so
they are kept max-normalised without log-scales.

Parity status: with exact boundary functions the scores equal brute-force
log P(x_<=k) and the beam equals a brute-force beam search
(tests/test_oracle_search.py); with truncated boundary MPSs the search is
pinned through the invariants only.
"""
from __future__ import annotations

import numpy as np

from .energy import Weights, potts_energy


def _fields(W: Weights, r: int, above: np.ndarray) -> np.ndarray:
    """g[b, c, s] for a batch of fixed rows r-1 (``above`` is [B][cols])."""
    B = above.shape[0] if above is not None else 1
    C, d = W.inst.cols, W.inst.d
    g = np.ones((B, C, d))
    if r == 0:
        return g
    for c in range(C):
        g[:, c] *= W.v[r - 1, c][above[:, c], :]
        if c > 0:
            g[:, c] *= W.dg[r - 1, c - 1][above[:, c - 1], :]
        if c < C - 1:
            g[:, c] *= W.an[r - 1, c][above[:, c + 1], :]
    return g


def delta_energy(inst, cfg: np.ndarray, r: int, c: int) -> np.ndarray:
    """[B][d] energy added by setting x_{r,c} = s (Eq. (1) terms that close)."""
    C = inst.cols
    dE = np.repeat(inst.local_E[r, c][None, :], cfg.shape[0], axis=0).copy()
    if c > 0:
        dE += inst.pair_h[r, c - 1][cfg[:, r * C + c - 1], :]
    if r > 0:
        up = (r - 1) * C
        dE += inst.pair_v[r - 1, c][cfg[:, up + c], :]
        if inst.kings:
            if c > 0:
                dE += inst.pair_d[r - 1, c - 1][cfg[:, up + c - 1], :]
            if c < C - 1:
                dE += inst.pair_a[r - 1, c][cfg[:, up + c + 1], :]
    return dE


def select_top(scores: np.ndarray, M: int) -> np.ndarray:
    """Flat indices (b*d + s) of the M best candidates, ordered by score
    descending then flat index ascending (= parent position, then s)."""
    flat = scores.reshape(-1)
    order = np.lexsort((np.arange(flat.size), -flat))
    return order[:M]


def marginals(A_rc, g_c, L, R_next):
    """q[b, s] = g_c[b, s] * sum_{alpha, alpha'} L[b, alpha] A[alpha, s, alpha'] R[b, alpha'],
    summed over alpha' first (one matrix product for all b), then over alpha."""
    a, d, z = A_rc.shape
    U = (R_next @ A_rc.reshape(a * d, z).T).reshape(-1, a, d)      # U[b, alpha, s]
    return g_c * np.einsum("ba,bas->bs", L, U)


def left_step(L, A_rc, s):
    """L[b] A[:, s[b], :] for every b (grouped by the state s[b])."""
    out = np.empty((L.shape[0], A_rc.shape[2]))
    for x in np.unique(s):
        sel = s == x
        out[sel] = L[sel] @ A_rc[:, x, :]
    return out


def log_conditionals(q: np.ndarray, dE: np.ndarray, beta: float) -> np.ndarray:
    """log p(s | b) = log q(b, s) - log sum_s' max(q(b, s'), 0).

    A weight q <= 0 (truncation or rounding) counts as probability 0.  A parent
    none of whose children has a positive weight has no conditional from the
    contraction; it takes the conditional of the fixed sites' Boltzmann weight
    alone, softmax_s(-beta dE(b, s)) (the unexplored sites left out), so the
    search never runs out of children."""
    qp = np.where(q > 0, q, 0.0)
    tot = qp.sum(axis=1, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        lp = np.log(qp) - np.log(tot)
    lp = np.where(np.isfinite(lp), lp, -np.inf)
    dead = ~(tot[:, 0] > 0)
    if dead.any():
        x = -beta * (dE[dead] - dE[dead].min(axis=1, keepdims=True))
        lp[dead] = x - np.log(np.exp(x).sum(axis=1, keepdims=True))
    return lp


def right_envs(A_row, g):
    """R[a, c] for c = cols..0 (list index c), max-normalised vectors."""
    B = g.shape[0]
    C = len(A_row)
    R = [None] * (C + 1)
    R[C] = np.ones((B, 1))
    for c in range(C - 1, -1, -1):
        S = np.einsum("asz,bz->bas", A_row[c], R[c + 1])         # [B][chi_c][d]
        v = np.einsum("bas,bs->ba", S, g[:, c])
        m = np.abs(v).max(axis=1, keepdims=True)
        R[c] = v / np.where(m > 0, m, 1.0)
    return R


def frontier_width(inst, k: int) -> int:
    """Sites k - w + 1 .. k form the frontier after site k (row-major order)."""
    return min(k + 1, inst.cols + 1)


def merge_branches(cand, cfg, energy, dE, k, w, runners=None):
    """Keep, per frontier (states of sites k-w+1..k-1 and the child's state),
    only the finite child with the lowest energy (ties: lowest id).  With
    ``runners`` (a dict), runners[kept id] = (id, energy) of the group's member
    that comes next in (energy, id) order, for groups of two or more."""
    B, d = cand.shape
    out = np.full_like(cand, -np.inf)
    groups = {}
    for b in range(B):
        prefix = tuple(cfg[b, k - w + 1: k].tolist())
        for s in range(d):
            if not np.isfinite(cand[b, s]):
                continue
            key = prefix + (s,)
            groups.setdefault(key, []).append((energy[b] + dE[b, s], b * d + s))
    for members in groups.values():
        members.sort()
        e, idx = members[0]
        b, s = divmod(idx, d)
        out[b, s] = cand[b, s]
        if runners is not None and len(members) > 1:
            runners[idx] = (members[1][1], members[1][0])
    return out


def hamming(x, y, upto):
    """Number of sites among 0..upto where x and y hold different states."""
    return int(np.count_nonzero(x[: upto + 1] != y[: upto + 1]))


def update_droplets(drops, cfg_new, kept, b, s, k, runners, cfg, energy_kept, d, droplets):
    """Droplet list of the child kept from parent b with state s at site k
    (cfg_new its configuration): the parent's droplets with site k set to s,
    then the group's runner-up if it qualifies (module docstring)."""
    e_cut, h_cut, cap = droplets
    out = []
    for x, de in drops[b]:
        x = x.copy()
        x[k] = s
        out.append((x, de))
    if kept in runners and len(out) < cap:
        o, e_o = runners[kept]
        de = e_o - energy_kept
        if de <= e_cut:
            bo, so = divmod(o, d)
            x = cfg[bo].copy()
            x[k] = so
            if (hamming(x, cfg_new, k) > h_cut
                    and all(hamming(x, y, k) > h_cut for y, _ in out)):
                out.append((x, de))
    return out


def beam_search(inst, A, M: int, cut_off_prob: float = 0.0, trace=None, merge=False,
                droplets=None):
    """Run the search with boundary MPS tensors A[r][c].  Returns dict with
    'states' [n][N], 'energies', 'scores' (the states of finite score first,
    sorted by energy, then the other beam slots) and 'beam_energies'
    (the final beam in beam order).  ``trace`` (optional list) receives per-site
    dicts with the parents' log-conditionals for teacher-forced comparisons.
    ``droplets`` = (energy_cutoff, hamming_cutoff, max_droplets), with merging:
    'droplets' then holds, for each returned state, its list of
    (configuration, energy) in the order they were taken."""
    if droplets is not None and not merge:
        raise ValueError("droplets are collected while merging branches")
    W = Weights(inst)
    Rr, C, d = inst.rows, inst.cols, inst.d
    N = Rr * C
    cfg = np.zeros((1, N), dtype=np.int64)
    score = np.zeros(1)
    energy = np.zeros(1)
    drops = [[]]
    for r in range(Rr):
        above = cfg[:, (r - 1) * C: r * C] if r > 0 else None
        g_anc = _fields(W, r, above)                                  # [n_anc][C][d]
        R = right_envs(A[r], g_anc)
        anc = np.arange(cfg.shape[0])
        L = np.ones((cfg.shape[0], 1))
        for c in range(C):
            q = marginals(A[r][c], g_anc[anc, c], L, R[c + 1][anc])
            dE = delta_energy(inst, cfg, r, c)
            lp = log_conditionals(q, dE, inst.beta)
            cand = score[:, None] + lp
            runners = {}
            if merge:
                k = r * C + c
                cand = merge_branches(cand, cfg, energy, dE, k, frontier_width(inst, k),
                                      runners if droplets is not None else None)
            if cut_off_prob > 0:
                best = cand.max()
                cand = np.where(cand >= best + np.log(cut_off_prob), cand, -np.inf)
            if trace is not None:
                trace.append({"site": r * C + c, "cfg": cfg.copy(), "logp": lp.copy()})
            keep = select_top(cand, M)
            b, s = np.divmod(keep, d)
            parents = cfg
            cfg = cfg[b].copy()
            cfg[:, r * C + c] = s
            score = cand.reshape(-1)[keep]
            e_par = energy
            energy = energy[b] + dE[b, s]
            if droplets is not None:
                k = r * C + c
                drops = [update_droplets(drops, cfg[j], int(keep[j]), int(b[j]), int(s[j]), k,
                                         runners, parents, float(e_par[b[j]] + dE[b[j], s[j]]),
                                         d, droplets)
                         for j in range(len(keep))]
            # L^child = g^b_c(s) * L^b A_{r,c}[:, s, :]
            Lb = left_step(L[b], A[r][c], s)
            Lb = Lb * g_anc[anc[b], c, s][:, None]
            m = np.abs(Lb).max(axis=1, keepdims=True)
            L = Lb / np.where(m > 0, m, 1.0)
            anc = anc[b]
    E = potts_energy(inst, cfg)
    # finite log-probabilities first, by energy, then index; then the slots
    # that hold pruned or merged-away children
    order = np.lexsort((np.arange(len(E)), E, ~np.isfinite(score)))
    out = {"states": cfg[order], "energies": E[order], "scores": score[order],
           "beam_states": cfg, "beam_scores": score, "beam_energies": energy,
           "n_valid": int(np.isfinite(score).sum())}
    if droplets is not None:
        out["droplets"] = [[(x, float(E[i] + de)) for x, de in drops[i]] for i in order]
    return out


def teacher_forced_logp(inst, A, r: int, c: int, cfg: np.ndarray) -> np.ndarray:
    """log p(s | b) at site (r, c) for given partial configurations ``cfg``
    ([B][N], first r*cols+c entries valid), with the row-start ancestor of b
    taken as b's own rows 0..r-1."""
    W = Weights(inst)
    C = inst.cols
    above = cfg[:, (r - 1) * C: r * C] if r > 0 else None
    g = _fields(W, r, above) if r > 0 else np.ones((cfg.shape[0], C, inst.d))
    R = right_envs(A[r], g)
    L = np.ones((cfg.shape[0], 1))
    for cc in range(c):
        s = cfg[:, r * C + cc]
        Lb = left_step(L, A[r][cc], s)
        Lb = Lb * g[np.arange(cfg.shape[0]), cc, s][:, None]
        m = np.abs(Lb).max(axis=1, keepdims=True)
        L = Lb / np.where(m > 0, m, 1.0)
    q = marginals(A[r][c], g[:, c], L, R[c + 1])
    return log_conditionals(q, delta_energy(inst, cfg, r, c), inst.beta)


def teacher_forced_condition(inst, A, r: int, c: int, cfg: np.ndarray):
    """Running-error condition numbers of the teacher-forced conditionals.

    The same chain as ``teacher_forced_logp`` contracted with absolute values
    (|L|, |A|, |R|, with L and R built from |A| as well) gives q_abs >= |q| term
    by term; a floating-point evaluation of q with n operations along the chain
    has |fl(q) - q| <= n eps q_abs (standard running error bound).  Both chains
    are divided by the same positive factors, so the bound survives scaling.
    Returns (kappa_s, kappa_Z) = (q_abs(s) / |q(s)|, sum_s q_abs / sum_s q+)."""
    W = Weights(inst)
    C = inst.cols
    nb = cfg.shape[0]
    above = cfg[:, (r - 1) * C: r * C] if r > 0 else None
    g = _fields(W, r, above) if r > 0 else np.ones((nb, C, inst.d))
    Rv, Ra = np.ones((nb, 1)), np.ones((nb, 1))
    for cc in range(C - 1, c, -1):
        v = np.einsum("asz,bz,bs->ba", A[r][cc], Rv, g[:, cc])
        va = np.einsum("asz,bz,bs->ba", np.abs(A[r][cc]), Ra, g[:, cc])
        m = np.where(va.max(axis=1, keepdims=True) > 0, va.max(axis=1, keepdims=True), 1.0)
        Rv, Ra = v / m, va / m
    L, La = np.ones((nb, 1)), np.ones((nb, 1))
    for cc in range(c):
        s = cfg[:, r * C + cc]
        gs = g[np.arange(nb), cc, s][:, None]
        L = gs * np.einsum("ba,baz->bz", L, np.transpose(A[r][cc][:, s, :], (1, 0, 2)))
        La = gs * np.einsum("ba,baz->bz", La, np.transpose(np.abs(A[r][cc])[:, s, :], (1, 0, 2)))
        m = np.where(La.max(axis=1, keepdims=True) > 0, La.max(axis=1, keepdims=True), 1.0)
        L, La = L / m, La / m
    q = marginals(A[r][c], g[:, c], L, Rv)
    qa = marginals(np.abs(A[r][c]), g[:, c], La, Ra)
    with np.errstate(divide="ignore", invalid="ignore"):
        ks = qa / np.abs(q)
        kz = qa.sum(axis=1) / np.where(q > 0, q, 0).sum(axis=1)
    return ks, kz
