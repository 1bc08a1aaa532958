"""Merging of branches on the GPU (through the C ABI) against the oracle.

Both sides read the same boundary MPS (the oracle's, imported), so the
children's scores agree to rounding and their energies bitwise (the same FP64
sums in the same order); the merge keeps per frontier the child of lowest
energy, ties by id, so the kept sets must be identical.  Checked: the final
beam (states bitwise, scores 1e-8, energies 1e-9) on square and king's
lattices with several d and beams, with the cut-off, with FP32 search
contractions (where only the dynamic-programming property is checked), and the
exact dynamic-programming case: a beam of d^(cols+1) or more after merging
must return the brute-force least-energy state of every final frontier."""
import itertools

import numpy as np
import pytest

from workloads import random_potts, config_instance
from oracle.bmps import boundary_mps as oracle_bmps
from oracle.search import beam_search, frontier_width
from oracle.exact import brute_force
from oracle.energy import potts_energy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_02317_amd import spg  # noqa: E402

DEV = torch.device("cuda:0")


def _env(inst, chi, precision="fp64"):
    ora = oracle_bmps(inst, chi)
    T, dims = spg.pack_oracle_mps(ora["A"], chi, inst.d)
    peps = spg.build_peps(inst)
    env = spg.env_import(peps, chi, dims, T, np.array(ora["lam"]), precision=precision)
    return ora, peps, env


def _run(env, inst, M, **kw):
    N = inst.rows * inst.cols
    st = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    en = torch.zeros(M, dtype=torch.float64, device=DEV)
    lp = torch.zeros(M, dtype=torch.float64, device=DEV)
    n = spg.branch_and_bound(env, M, st, en, lp, **kw)
    torch.cuda.synchronize()
    return st[:n].cpu().numpy(), en[:n].cpu().numpy(), lp[:n].cpu().numpy()


CASES = [("sq3x4_d2", 3, 4, 2, False, 16, 24, 0.0), ("k3x3_d3", 3, 3, 3, True, 27, 40, 0.0),
         ("k2x4_d4", 2, 4, 4, True, 16, 50, 1e-3), ("k4x4_d2", 4, 4, 2, True, 16, 20, 0.0)]


@pytest.mark.parametrize("name,R,C,d,kings,chi,M,cut", CASES)
def test_merged_search_matches_oracle(name, R, C, d, kings, chi, M, cut):
    inst = random_potts(R, C, d, kings, seed=R * 10 + C + d, beta=1.0)
    ora, peps, env = _env(inst, chi)
    st, en, lp = _run(env, inst, M, cut_off_prob=cut, merge_branches=True)
    ref = beam_search(inst, ora["A"], M, cut_off_prob=cut, merge=True)
    assert len(st) == ref["n_valid"]
    fin = np.isfinite(ref["scores"])
    assert {tuple(x) for x in st.tolist()} == {tuple(x) for x in ref["states"][fin].tolist()}
    np.testing.assert_allclose(np.sort(lp), np.sort(ref["scores"][fin]), atol=1e-8)
    np.testing.assert_allclose(en, potts_energy(inst, st), atol=1e-9)
    # one state per final frontier
    w = frontier_width(inst, R * C - 1)
    assert len({tuple(x[-w:]) for x in st.tolist()}) == len(st)


def _dp_states(inst):
    """Per final frontier (the last cols + 1 sites), the configuration of least
    Eq. (1) energy over all d^N, ties by lowest enumeration index."""
    N, d = inst.rows * inst.cols, inst.d
    X = np.array(list(itertools.product(range(d), repeat=N)), dtype=np.int64)
    E = potts_energy(inst, X)
    w = frontier_width(inst, N - 1)
    best = {}
    for i in np.lexsort((np.arange(len(E)), E)):
        best.setdefault(tuple(X[i, N - w:].tolist()), tuple(X[i].tolist()))
    return set(best.values())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("wide", [1, 3])
@pytest.mark.parametrize("R,C,d,kings", [(3, 3, 2, True), (2, 4, 3, True), (3, 4, 2, False),
                                         (3, 2, 3, True)])
def test_frontier_sized_beam_is_exact_dynamic_programming(R, C, d, kings, wide, precision):
    # A beam of at least d^(cols+1) never prunes after merging, so it returns
    # exactly one least-energy state per final frontier, whatever the scores.
    # With wide = 3 most beam slots hold merged-away children (score -inf),
    # which must not be returned among the n_out states.
    inst = random_potts(R, C, d, kings, seed=R + C + d + 40, beta=0.9)
    ref = brute_force(inst)
    _, _, env = _env(inst, d ** (C // 2), precision)          # exact bond dimension
    st, en, lp = _run(env, inst, wide * d ** (C + 1), merge_branches=True)
    assert abs(en[0] - ref["E_min"]) < 1e-9
    assert {tuple(x) for x in st.tolist()} == _dp_states(inst)
    assert np.all(np.isfinite(lp)) and np.all(np.diff(en) >= 0)


def test_merging_with_a_proposal_is_refused():
    inst = config_instance("square4x4_d2", 0)
    _, _, env = _env(inst, 16)
    prop = spg.Proposal(hidden=4, seed=1)
    with pytest.raises(spg.SpgError) as e:
        _run(env, inst, 8, proposal=prop, kappa=2.0, merge_branches=True)
    assert e.value.code == -5
