"""Droplets collected while merging branches (oracle), pinned by Eq. (1).

A droplet is a whole configuration; its reported energy (the state's energy
plus the gap recorded when its group was merged) must equal the Eq. (1)
energy of that configuration, recomputed independently, which holds only if
the merged-away member differed from the kept one in sites that no later site
couples to.  Also checked: gaps within the cut-off, the Hamming constraints,
the capacity, and that collecting droplets leaves the beam unchanged."""
import numpy as np
import pytest

from workloads import random_potts, config_instance
from oracle.bmps import boundary_mps
from oracle.energy import potts_energy
from oracle.search import beam_search


def _check(inst, A, M, cut, hcut, cap):
    ref = beam_search(inst, A, M, merge=True)
    got = beam_search(inst, A, M, merge=True, droplets=(cut, hcut, cap))
    np.testing.assert_array_equal(got["states"], ref["states"])
    np.testing.assert_array_equal(got["scores"], ref["scores"])
    total = 0
    for st, e, drops in zip(got["states"], got["energies"], got["droplets"]):
        assert len(drops) <= cap
        for i, (x, ex) in enumerate(drops):
            assert abs(float(potts_energy(inst, x[None])[0]) - ex) < 1e-9
            assert -1e-9 <= ex - e <= cut + 1e-9
            assert np.count_nonzero(x != st) > hcut
            for y, _ in drops[:i]:
                assert np.count_nonzero(x != y) > hcut
        total += len(drops)
    return total


@pytest.mark.parametrize("R,C,d,kings,M", [(3, 4, 2, False, 24), (3, 3, 3, True, 40),
                                           (4, 4, 2, True, 20), (2, 5, 4, True, 50)])
def test_droplet_energies_follow_eq1(R, C, d, kings, M):
    inst = random_potts(R, C, d, kings, seed=R * 7 + C + d, beta=1.0)
    A = boundary_mps(inst, 16)["A"]
    n = _check(inst, A, M, 3.0, 0, 8)
    assert n > 0


@pytest.mark.parametrize("hcut", [0, 1, 3])
def test_droplet_hamming_cutoff(hcut):
    inst = config_instance("square4x4_d2", 1)
    A = boundary_mps(inst, 16)["A"]
    _check(inst, A, 32, 10.0, hcut, 16)


def test_droplet_energy_cutoff_and_capacity():
    inst = random_potts(3, 4, 3, True, seed=5, beta=1.0)
    A = boundary_mps(inst, 16)["A"]
    wide = _check(inst, A, 40, 100.0, 0, 32)
    narrow = _check(inst, A, 40, 0.5, 0, 32)
    capped = _check(inst, A, 40, 100.0, 0, 2)
    assert narrow < wide and capped <= 2 * 40


def test_droplets_need_merging():
    inst = config_instance("square4x4_d2", 0)
    A = boundary_mps(inst, 16)["A"]
    with pytest.raises(ValueError):
        beam_search(inst, A, 8, droplets=(1.0, 0, 4))
