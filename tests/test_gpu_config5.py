"""The search at the full-stack lattice shape on one GPU: 16x16 king's lattice
of 8-spin clusters (d = 256 states each, dense 256 x 256 pair tables), beta =
4, bond cap chi = 64 and a beam of M = 10000 (Sec. 2: conditionals from the
environments, top-M pruning, Fig. 1(d)-(e)).

The boundary MPS at this shape is not built here (its one-shot MPO
environments take 2 GiB per cut), so the search runs on a seeded synthetic
environment with the workload's bond dimensions and positive entries, as at
12x12.  At this size the per-ancestor products take 21 GB, each site has 2.56
million candidates (the multi-workgroup top-M front end), and M > 8192 (the
global-memory ordering of the survivors).

* Conditionals at sampled sites (row starts, interior, the last row) against
  the oracle's teacher-forced ones: every conditional is a sum of positive
  terms (condition number 1), so they agree to rounding.
* The search: the full beam, Eq. (1) energies recomputed by the oracle, sorted
  and distinct states; for the best states, the returned log-probability is
  the sum of the teacher-forced conditionals along the state (spg_marginals
  at every site), so the search and the conditionals' entry point agree.
"""
import numpy as np
import pytest

from workloads import config_instance, synthetic_env
from oracle.energy import potts_energy
from oracle.search import teacher_forced_logp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_02317_amd import spg  # noqa: E402

DEV = torch.device("cuda:0")
CHI, M = 64, 10000


@pytest.fixture(scope="module")
def shared():
    print("config5 shape: instance and synthetic environment", flush=True)
    inst = config_instance("kings16x16_d256", 0)
    A = synthetic_env(inst.rows, inst.cols, inst.d, CHI, 11)
    T, dims = spg.pack_oracle_mps(A, CHI, inst.d)
    env = spg.env_import(spg.build_peps(inst), CHI, dims, T, np.zeros(inst.rows))
    del T
    return inst, A, env


def test_marginals_at_sampled_sites(shared):
    inst, A, env = shared
    print("config5 shape: sampled conditionals", flush=True)
    rng = np.random.default_rng(3)
    cfg = rng.integers(0, inst.d, size=(16, inst.n_sites))
    cfg_t = torch.tensor(cfg, dtype=torch.int32, device=DEV)
    for site in (0, 7, 16, 100, 255):
        out = torch.empty((16, inst.d), dtype=torch.float64, device=DEV)
        spg.marginals(env, site, cfg_t, out)
        torch.cuda.synchronize()
        r, c = divmod(site, inst.cols)
        ref = teacher_forced_logp(inst, A, r, c, cfg)
        np.testing.assert_allclose(out.cpu().numpy(), ref, atol=1e-10, err_msg=str(site))


def test_search_full_beam(shared):
    inst, A, env = shared
    print("config5 shape: search", flush=True)
    N = inst.n_sites
    st = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    en = torch.zeros(M, dtype=torch.float64, device=DEV)
    lp = torch.zeros(M, dtype=torch.float64, device=DEV)
    n = spg.branch_and_bound(env, M, st, en, lp)
    torch.cuda.synchronize()
    assert n == M
    states, E, logp = st.cpu().numpy(), en.cpu().numpy(), lp.cpu().numpy()
    np.testing.assert_allclose(E, potts_energy(inst, states), atol=1e-9)
    assert np.all(np.diff(E) >= -1e-9)
    assert len({tuple(x) for x in states.tolist()}) == M
    assert np.all(np.isfinite(logp)) and np.all(logp <= 1e-12)
    # the best states' log-probabilities from the conditionals' entry point
    best = torch.tensor(states[:4], dtype=torch.int32, device=DEV)
    tot = np.zeros(4)
    out = torch.empty((4, inst.d), dtype=torch.float64, device=DEV)
    for site in range(N):
        spg.marginals(env, site, best, out)
        torch.cuda.synchronize()
        tot += out.cpu().numpy()[np.arange(4), states[:4, site]]
    np.testing.assert_allclose(tot, logp[:4], rtol=1e-10, atol=1e-8)
