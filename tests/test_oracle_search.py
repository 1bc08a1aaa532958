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
