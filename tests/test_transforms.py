"""The eight lattice symmetries: pure relabellings of an instance (CPU), and
the search run on all eight orientations in one batch (GPU): every
orientation's states map back to states of the original lattice with the
energies reported, and with exact contraction and an exhaustive beam every
orientation finds the brute-force ground state (the paper's agreement check
over all lattice transformations, Sec. 3.1)."""
import numpy as np
import pytest

from workloads import random_potts, config_instance
from workloads.transforms import lattice_transform
from oracle.energy import potts_energy
from oracle.exact import brute_force


@pytest.mark.parametrize("R,C,kings", [(3, 4, True), (2, 5, False), (4, 4, True)])
def test_transforms_relabel_energies_and_compose(R, C, kings):
    inst = random_potts(R, C, 3, kings, seed=R + C, beta=1.0)
    X = np.random.default_rng(1).integers(0, 3, size=(16, R * C))
    E = potts_energy(inst, X)
    seen = set()
    for k in range(8):
        t, back = lattice_transform(inst, k)
        assert sorted(back.tolist()) == list(range(R * C))
        np.testing.assert_allclose(potts_energy(t, X[:, back]), E, atol=1e-12)
        seen.add(tuple(back.tolist()))
        # undoing the relabelling gives the original tables back
        if k == 0:
            assert np.array_equal(t.local_E, inst.local_E)
    assert len(seen) == 8


def test_brute_force_is_invariant():
    inst = random_potts(2, 3, 3, True, seed=3, beta=0.8)
    ref = brute_force(inst)
    for k in range(8):
        t, _ = lattice_transform(inst, k)
        b = brute_force(t)
        assert abs(b["logZ"] - ref["logZ"]) < 1e-10
        assert abs(b["E_min"] - ref["E_min"]) < 1e-10


torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_02317_amd import spg
    return spg


@pytest.mark.gpu
@pytest.mark.parametrize("name,chi,M", [("kings2x3_d3", 27, 729), ("square4x4_d2", 16, 256)])
def test_all_orientations_in_one_batch(name, chi, M):
    spg = _gpu()
    inst = random_potts(2, 3, 3, True, seed=9, beta=0.7) if name == "kings2x3_d3" \
        else config_instance(name, 3)
    ref = brute_force(inst)
    ts = [lattice_transform(inst, k) for k in range(8)]
    peps = [spg.build_peps(t) for t, _ in ts]
    b = spg.Batch(peps, chi=chi, max_states=M, n_streams=2, classes=True)
    b.run(use_graph=False)
    units, _ = b.units()
    assert units == (1 if inst.rows == inst.cols else 2)
    bests = []
    for k, (t, back) in enumerate(ts):
        st, en, lp, _ = b.result(k)
        assert len(st) > 0
        x_old = np.empty_like(st)
        x_old[:, back] = st
        np.testing.assert_allclose(potts_energy(inst, x_old), en, atol=1e-9)
        bests.append(en[0])
    # exact contraction: every orientation reaches the ground state
    assert max(bests) - min(bests) < 1e-9
    assert abs(min(bests) - ref["E_min"]) < 1e-9
