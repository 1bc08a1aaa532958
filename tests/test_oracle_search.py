"""Pins of the oracle's branch-and-bound search (CPU only)."""
import numpy as np
import pytest

from workloads import random_potts, config_instance
from oracle.exact import brute_force, prefix_logp
from oracle.bmps import boundary_mps
from oracle.search import beam_search, select_top


def _bf_beam(bf, N, d, M):
    """Independent brute-force beam search: keep the M most probable prefixes
    by exact log P(x_<=k), ties by parent position then state."""
    beam = [()]
    for k in range(N):
        cands = []
        for pos, pre in enumerate(beam):
            for s in range(d):
                cands.append((-prefix_logp(bf, list(pre) + [s]), pos, s, pre + (s,)))
        cands.sort(key=lambda t: (t[0], t[1], t[2]))
        beam = [t[3] for t in cands[:M]]
    return beam


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_config1_beam_equals_bruteforce_beam(seed):
    inst = config_instance("square4x4_d2", seed)
    bf = brute_force(inst)
    mp = boundary_mps(inst, chi=16)
    M = 8
    res = beam_search(inst, mp["A"], M)
    ref = _bf_beam(bf, inst.n_sites, 2, M)
    got = [tuple(x) for x in res["beam_states"]]
    # interchangeable only within rounding of equal scores
    assert got == ref
    for x, sc in zip(res["beam_states"], res["beam_scores"]):
        assert abs(sc - prefix_logp(bf, list(x))) < 1e-10


@pytest.mark.parametrize("shape", [(3, 3, 2, True), (2, 3, 3, True)])
def test_full_beam_finds_ground_state(shape):
    R, C, d, k = shape
    inst = random_potts(R, C, d, k, seed=9, beta=1.0)
    bf = brute_force(inst)
    mp = boundary_mps(inst, chi=d ** (C // 2))
    res = beam_search(inst, mp["A"], d ** (R * C))
    assert abs(res["energies"][0] - bf["E_min"]) < 1e-12
    np.testing.assert_allclose(np.sort(res["energies"]), np.sort(bf["E"]), atol=1e-12)
    # scores are the exact log-probabilities
    np.testing.assert_allclose(
        np.sort(res["scores"]), np.sort(-inst.beta * bf["E"] - bf["logZ"]), atol=1e-9)


def test_accumulated_energy_equals_eq1():
    inst = random_potts(3, 4, 3, True, seed=13, beta=0.8)
    mp = boundary_mps(inst, chi=9)
    res = beam_search(inst, mp["A"], 20)
    from oracle.energy import potts_energy
    np.testing.assert_allclose(res["beam_energies"], potts_energy(inst, res["beam_states"]),
                               atol=1e-12)


def test_select_top_tie_rule():
    s = np.array([[0.0, -1.0], [0.0, 0.0], [-1.0, 0.0]])
    assert list(select_top(s, 4)) == [0, 2, 3, 5]


def test_cutoff_marks_discarded():
    inst = random_potts(2, 3, 3, True, seed=3, beta=2.0)
    mp = boundary_mps(inst, chi=9)
    full = beam_search(inst, mp["A"], 27)
    cut = beam_search(inst, mp["A"], 27, cut_off_prob=1e-2)
    assert cut["n_valid"] <= full["n_valid"]
    fin = np.isfinite(cut["beam_scores"])
    # every surviving state is within the cut of the best at the last step
    assert np.all(cut["beam_scores"][fin] >= cut["beam_scores"][0] + np.log(1e-2) - 1e-12)


# ---- merging branches ---------------------------------------------------------

import itertools

import pytest as _pytest

from oracle.search import beam_search as _beam, frontier_width


@_pytest.mark.parametrize("R,C,d,kings,seed", [(3, 3, 2, True, 1), (3, 4, 2, False, 2),
                                               (2, 4, 3, True, 3), (4, 3, 2, True, 4)])
def test_merged_search_with_a_frontier_sized_beam_is_exact(R, C, d, kings, seed):
    """With merging, at most d^(cols+1) children survive a step (one per
    frontier); a beam that large keeps them all, so the search is exact
    dynamic programming over frontiers and must reach the brute-force ground
    state, with any exact boundary MPS."""
    from workloads import random_potts
    from oracle.exact import brute_force
    from oracle.bmps import boundary_mps
    inst = random_potts(R, C, d, kings, seed=seed, beta=0.9)
    ref = brute_force(inst)
    A = boundary_mps(inst, d ** C)["A"]
    M = d ** (C + 1)
    res = _beam(inst, A, M, merge=True)
    assert abs(res["energies"][0] - ref["E_min"]) < 1e-9
    # one survivor per frontier in the final beam
    fin = res["beam_states"][np.isfinite(res["beam_scores"])]
    w = frontier_width(inst, R * C - 1)
    keys = {tuple(x[-w:]) for x in fin.tolist()}
    assert len(keys) == len(fin)


def test_merge_keeps_the_lowest_energy_child_per_frontier():
    from oracle.search import merge_branches
    cand = np.array([[0.0, -1.0], [-0.5, -np.inf], [-2.0, -0.1]])
    cfg = np.array([[1, 0, 0], [1, 0, 0], [0, 0, 0]])
    energy = np.array([5.0, 4.0, 1.0])
    dE = np.zeros((3, 2))
    out = merge_branches(cand, cfg, energy, dE, k=1, w=2)     # frontier = (cfg[:,0], s)
    # rows 0 and 1 share frontier (1, s): row 1 has the lower energy for s = 0;
    # s = 1 of row 1 is -inf, so row 0 keeps s = 1; row 2 is alone with frontier (0, s)
    assert np.array_equal(np.isfinite(out), [[False, True], [True, False], [True, True]])
    energy[1] = 5.0                                            # tie: lowest id wins
    out = merge_branches(cand, cfg, energy, dE, k=1, w=2)
    assert np.isfinite(out[0, 0]) and not np.isfinite(out[1, 0])


@_pytest.mark.parametrize("R,C,d,kings,seed", [(3, 2, 3, True, 5), (3, 3, 2, False, 6)])
def test_merged_wide_beam_returns_the_least_energy_state_of_every_frontier(R, C, d, kings, seed):
    """A beam three times the number of frontiers: most slots then hold
    merged-away children of score -inf.  The finite states must be exactly the
    brute-force least-energy configuration of each final frontier, and they
    come first in the returned order."""
    from workloads import random_potts
    from oracle.bmps import boundary_mps
    from oracle.energy import potts_energy
    inst = random_potts(R, C, d, kings, seed=seed, beta=0.7)
    N = R * C
    X = np.array(list(itertools.product(range(d), repeat=N)), dtype=np.int64)
    E = potts_energy(inst, X)
    w = frontier_width(inst, N - 1)
    best = {}
    for i in np.argsort(E, kind="stable"):
        best.setdefault(tuple(X[i, N - w:].tolist()), tuple(X[i].tolist()))
    res = _beam(inst, boundary_mps(inst, d ** C)["A"], 3 * d ** (C + 1), merge=True)
    n = res["n_valid"]
    assert n == len(best) and np.all(np.isfinite(res["scores"][:n]))
    assert {tuple(x) for x in res["states"][:n].tolist()} == set(best.values())
    # merged-away children of lower energy than some returned state exist,
    # so the finite-first order is really exercised
    assert res["energies"][n:].min() < res["energies"][:n].max()
