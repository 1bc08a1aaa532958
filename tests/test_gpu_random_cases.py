"""A seeded sweep of small random cases through the C ABI against the oracle:
lattice shape, d, square or king's, beta, bond dimension, beam width (1 to
more than d^N), cut-off and merging are drawn per case.  Both sides search the
oracle's boundary MPS (imported), so the returned beams must agree: the same
number of states, the same states, scores to 1e-8, energies equal to their
Eq. (1) energies, and the best energy to 1e-9."""
import numpy as np
import pytest

from workloads import random_potts
from oracle.bmps import boundary_mps as oracle_bmps
from oracle.energy import potts_energy
from oracle.search import beam_search

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_02317_amd import spg  # noqa: E402

DEV = torch.device("cuda:0")


def _case(k):
    rng = np.random.default_rng(1000 + k)
    R, C = int(rng.integers(2, 5)), int(rng.integers(2, 6))
    d = int(rng.choice([2, 3, 4, 5]))
    kings = bool(rng.integers(0, 2))
    beta = float(rng.uniform(0.3, 1.0))
    chi = int(rng.choice([4, 8, 16]))
    M = int(rng.choice([1, 7, 33, 100]))
    cut = float(rng.choice([0.0, 1e-3]))
    merge = bool(rng.integers(0, 2))
    return R, C, d, kings, beta, chi, M, cut, merge


@pytest.mark.parametrize("k", range(16))
def test_random_case_matches_oracle(k):
    R, C, d, kings, beta, chi, M, cut, merge = _case(k)
    inst = random_potts(R, C, d, kings, seed=2000 + k, beta=beta)
    ora = oracle_bmps(inst, chi)
    T, dims = spg.pack_oracle_mps(ora["A"], chi, d)
    peps = spg.build_peps(inst)
    env = spg.env_import(peps, chi, dims, T, np.array(ora["lam"]))
    N = R * C
    st = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    en = torch.zeros(M, dtype=torch.float64, device=DEV)
    lp = torch.zeros(M, dtype=torch.float64, device=DEV)
    n = spg.branch_and_bound(env, M, st, en, lp, cut_off_prob=cut, merge_branches=merge)
    torch.cuda.synchronize()
    st, en, lp = st.cpu().numpy()[:n], en.cpu().numpy()[:n], lp.cpu().numpy()[:n]
    ref = beam_search(inst, ora["A"], M, cut_off_prob=cut, merge=merge)
    fin = np.isfinite(ref["scores"])
    assert n == ref["n_valid"], (n, ref["n_valid"])
    assert {tuple(x) for x in st.tolist()} == {tuple(x) for x in ref["states"][fin].tolist()}
    np.testing.assert_allclose(np.sort(lp), np.sort(ref["scores"][fin]), atol=1e-8)
    np.testing.assert_allclose(en, potts_energy(inst, st), atol=1e-9)
    if n:
        assert abs(en[0] - ref["energies"][fin].min()) < 1e-9
