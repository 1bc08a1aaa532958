"""The search's rule for a parent none of whose children has a positive
conditional weight (CPU only).

A truncated contraction can give every child of a parent a weight q <= 0.
The conditional is then not defined by the contraction; the reading adopted
is the conditional of the fixed sites' Boltzmann weight, softmax_s(-beta dE)
with dE the Eq. (1) energy each child adds (the unexplored sites left out).
"""
import numpy as np

from workloads import random_potts
from oracle.bmps import boundary_mps
from oracle.search import log_conditionals, beam_search, delta_energy


def test_dead_parent_takes_local_softmax():
    q = np.array([[0.3, 0.0, -1.0, 0.7],        # live: q+ normalised, q <= 0 -> -inf
                  [-1.0, 0.0, -2.0, -0.5],       # dead: no positive weight
                  [0.0, 0.0, 0.0, 0.0]])         # dead: all zero
    dE = np.array([[1.0, 2.0, 3.0, 4.0],
                   [0.5, -1.0, 2.0, 0.0],
                   [3.0, 3.0, 3.0, 1.0]])
    beta = 1.7
    lp = log_conditionals(q, dE, beta)
    np.testing.assert_allclose(lp[0], [np.log(0.3), -np.inf, -np.inf, np.log(0.7)])
    for b in (1, 2):
        w = np.exp(-beta * dE[b])
        np.testing.assert_allclose(lp[b], np.log(w / w.sum()), rtol=1e-14)
    # extreme energies do not underflow the normalisation
    lp = log_conditionals(np.zeros((1, 3)), np.array([[0.0, 800.0, 1600.0]]), 1.0)
    np.testing.assert_allclose(lp[0], [0.0, -800.0, -1600.0], atol=1e-12)


def test_search_never_runs_out_of_children():
    """An environment whose weights are all negative (the sign of every site
    tensor flipped) still yields M complete states: every step falls back to
    the local conditionals, so the search is the greedy beam on the energy
    added site by site."""
    inst = random_potts(2, 3, 3, True, seed=4, beta=1.0)
    A = boundary_mps(inst, chi=9)["A"]
    A[0] = [a.copy() for a in A[0]]
    A[0][0] = -A[0][0]                           # row 0: every q < 0
    res = beam_search(inst, A, 4)
    assert res["n_valid"] == 4
    # row 0 follows exp(-beta dE): the best first state minimises the local energy
    cfg0 = np.zeros((1, inst.n_sites), dtype=np.int64)
    dE = delta_energy(inst, cfg0, 0, 0)[0]
    assert int(np.argmin(dE)) in set(res["beam_states"][:, 0].tolist())
