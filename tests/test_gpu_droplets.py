"""Droplets on the GPU (through the C ABI) against the oracle.

Both sides search the same boundary MPS (the oracle's, imported), so the
merged groups, their runner-ups and the droplet lists must agree: per
returned state (matched by its configuration) the same droplets in the same
order, bitwise configurations, energies to 1e-9, and each droplet's energy
equal to the Eq. (1) energy of its configuration.  Collecting droplets leaves
the returned beam unchanged."""
import numpy as np
import pytest

from workloads import random_potts, config_instance
from oracle.bmps import boundary_mps as oracle_bmps
from oracle.search import beam_search
from oracle.energy import potts_energy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_02317_amd import spg  # noqa: E402

DEV = torch.device("cuda:0")


def _env(inst, chi):
    ora = oracle_bmps(inst, chi)
    T, dims = spg.pack_oracle_mps(ora["A"], chi, inst.d)
    peps = spg.build_peps(inst)
    env = spg.env_import(peps, chi, dims, T, np.array(ora["lam"]))
    return ora, peps, env


def _run(env, inst, M, **kw):
    N = inst.rows * inst.cols
    st = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    en = torch.zeros(M, dtype=torch.float64, device=DEV)
    lp = torch.zeros(M, dtype=torch.float64, device=DEV)
    n = spg.branch_and_bound(env, M, st, en, lp, **kw)
    torch.cuda.synchronize()
    return st[:n].cpu().numpy(), en[:n].cpu().numpy()


# the instances, bond dimensions, beams and cut-offs of the merging parity cases
CASES = [("sq3x4_d2", 3, 4, 2, False, 16, 24, 0.0, 0),
         ("k3x3_d3", 3, 3, 3, True, 27, 40, 0.0, 1),
         ("k2x4_d4", 2, 4, 4, True, 16, 50, 1e-3, 2),
         ("k4x4_d2", 4, 4, 2, True, 16, 20, 0.0, 1)]


@pytest.mark.parametrize("name,R,C,d,kings,chi,M,cut,hcut", CASES)
def test_droplets_match_oracle(name, R, C, d, kings, chi, M, cut, hcut):
    ecut, cap = 5.0, 8
    inst = random_potts(R, C, d, kings, seed=R * 10 + C + d, beta=1.0)
    ora, peps, env = _env(inst, chi)
    st0, en0 = _run(env, inst, M, cut_off_prob=cut, merge_branches=True)
    st, en = _run(env, inst, M, cut_off_prob=cut, merge_branches=True,
                  droplets=(ecut, hcut, cap))
    np.testing.assert_array_equal(st, st0)
    np.testing.assert_array_equal(en, en0)
    ref = beam_search(inst, ora["A"], M, cut_off_prob=cut, merge=True,
                      droplets=(ecut, hcut, cap))
    by_state = {tuple(x.tolist()): dl for x, dl, sc in
                zip(ref["states"], ref["droplets"], ref["scores"]) if np.isfinite(sc)}
    assert len(by_state) == len(st)
    total = 0
    for i in range(len(st)):
        cfg, de = spg.droplets(env, i)
        want = by_state[tuple(st[i].tolist())]
        assert len(cfg) == len(want)
        for (x, e), y, g in zip(want, cfg, de):
            np.testing.assert_array_equal(y, x)
            assert abs(g - e) < 1e-9
        if len(cfg):
            np.testing.assert_allclose(de, potts_energy(inst, cfg), atol=1e-9)
            assert np.all(de - en[i] <= ecut + 1e-9)
        total += len(cfg)
    assert total > 0


def test_droplets_need_merging_and_a_search():
    inst = config_instance("square4x4_d2", 0)
    _, _, env = _env(inst, 16)
    with pytest.raises(spg.SpgError) as e:
        _run(env, inst, 8, droplets=(1.0, 0, 4))
    assert e.value.code == -1
    _run(env, inst, 8, merge_branches=True)
    with pytest.raises(spg.SpgError):
        spg.droplets(env, 0)
    with pytest.raises(spg.SpgError) as e:
        _run(env, inst, 8, merge_branches=True, droplets=(1.0, 0, 65))
    assert e.value.code == -5


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_droplets_reduced_precision_search(precision):
    """With FP32 / BF16 search contractions the beam need not equal the
    oracle's; the droplets must still be exact excitations of their states:
    Eq. (1) energies, gaps within the cut-off, the Hamming rule, and the same
    beam as merging without droplets."""
    R, C, d, kings, chi, M = 3, 4, 2, True, 16, 40
    ecut, hcut, cap = 5.0, 1, 8
    inst = random_potts(R, C, d, kings, seed=3, beta=1.0)
    peps = spg.build_peps(inst)
    env, _ = spg.boundary_mps(peps, chi, precision=precision, want_logZ=False)
    st0, en0 = _run(env, inst, M, merge_branches=True)
    st, en = _run(env, inst, M, merge_branches=True, droplets=(ecut, hcut, cap))
    np.testing.assert_array_equal(st, st0)
    np.testing.assert_array_equal(en, en0)
    total = 0
    for i in range(len(st)):
        cfg, de = spg.droplets(env, i)
        assert len(cfg) <= cap
        if len(cfg) == 0:
            continue
        np.testing.assert_allclose(de, potts_energy(inst, cfg), atol=1e-9)
        assert np.all(de - en[i] >= -1e-9) and np.all(de - en[i] <= ecut + 1e-9)
        for a in range(len(cfg)):
            assert np.count_nonzero(cfg[a] != st[i]) > hcut
            for b in range(a):
                assert np.count_nonzero(cfg[a] != cfg[b]) > hcut
        total += len(cfg)
    assert total > 0
