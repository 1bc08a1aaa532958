"""Pin of the running-error condition numbers the parity tolerances are built
on (``oracle.search.teacher_forced_condition``), with exact rational
arithmetic (CPU only).

The teacher-forced conditional q(s) = g(s) L A R is a chain of products and
sums; with every FP64 input taken as an exact rational, ``fractions`` gives
the exact q, and the same chain over |A| the exact absolute-value contraction
q_abs.  Checked: the oracle's kappa_s = q_abs / |q| and kappa_Z = sum q_abs /
sum q+ equal the exact ratios, and the FP64 log-conditionals lie within
2 n u (kappa_s + kappa_Z) of the exact ones, n being the operation count the
GPU parity tests use (the kappas themselves to the relative accuracy
1e-12 + 2 n u kappa that their own denominators allow).
"""
from fractions import Fraction

import numpy as np
import pytest

from workloads import random_potts
from oracle.bmps import boundary_mps
from oracle.energy import Weights
from oracle.search import _fields, teacher_forced_logp, teacher_forced_condition

U = np.finfo(float).eps


def _exact_q(A_row, g, c, states, absval):
    """Unnormalised q(s) of one partial row (states of columns < c) in exact
    rational arithmetic; ``absval`` contracts |A| instead of A."""
    F = Fraction
    C = len(A_row)
    T = [[[[F(abs(x) if absval else x) for x in col] for col in mid] for mid in a]
         for a in A_row]                                   # T[c][al][s][be]
    gg = [[F(x) for x in row] for row in g]                # gg[c][s]
    R = [F(1)]
    for cc in range(C - 1, c, -1):
        R = [sum(gg[cc][s] * sum(T[cc][al][s][be] * R[be] for be in range(len(R)))
                 for s in range(len(gg[cc])))
             for al in range(len(T[cc]))]
    L = [F(1)]
    for cc in range(c):
        s = states[cc]
        L = [gg[cc][s] * sum(L[al] * T[cc][al][s][be] for al in range(len(L)))
             for be in range(len(T[cc][0][0]))]
    d = len(gg[c])
    return [gg[c][s] * sum(L[al] * sum(T[c][al][s][be] * R[be] for be in range(len(R)))
                           for al in range(len(L))) for s in range(d)]


@pytest.mark.parametrize("beta,chi", [(0.8, 3), (3.0, 2), (6.0, 2)])
def test_condition_numbers_and_bound_exact(beta, chi):
    inst = random_potts(3, 3, 3, True, seed=11, beta=beta)
    A = boundary_mps(inst, chi=chi)["A"]
    W = Weights(inst)
    rng = np.random.default_rng(2)
    cfg = rng.integers(0, inst.d, size=(12, inst.n_sites))
    checked = 0
    for site in range(inst.n_sites):
        r, c = divmod(site, inst.cols)
        g = (_fields(W, r, cfg[:, (r - 1) * inst.cols: r * inst.cols]) if r > 0
             else np.ones((cfg.shape[0], inst.cols, inst.d)))
        lp = teacher_forced_logp(inst, A, r, c, cfg)
        ks, kz = teacher_forced_condition(inst, A, r, c, cfg)
        n_ops = (inst.d * max(a.shape[2] for a in A[r]) * inst.cols
                 + max(a.shape[0] for a in A[r]) ** 2)
        for b in range(cfg.shape[0]):
            q = _exact_q(A[r], g[b], c, cfg[b, r * inst.cols: r * inst.cols + c], False)
            qa = _exact_q(A[r], g[b], c, cfg[b, r * inst.cols: r * inst.cols + c], True)
            qp = [x if x > 0 else Fraction(0) for x in q]
            tot = sum(qp)
            if tot == 0:
                continue                                    # the local fallback applies
            kz_ex = float(sum(qa) / tot)
            assert abs(kz[b] - kz_ex) <= (1e-12 + 2 * n_ops * U * kz_ex) * kz_ex
            for s in range(inst.d):
                if q[s] != 0:
                    ks_ex = float(qa[s] / abs(q[s]))
                    # |q| itself carries the relative error n u kappa_s
                    assert abs(ks[b, s] - ks_ex) <= (1e-12 + 2 * n_ops * U * ks_ex) * ks_ex
                bound = 2 * n_ops * U * (ks[b, s] + kz[b])
                if q[s] > 0 and bound < 1:
                    exact = np.log(float(q[s] / tot))
                    assert abs(lp[b, s] - exact) <= bound + 1e-15, (lp[b, s], exact, bound)
                    checked += 1
    assert checked > 50
