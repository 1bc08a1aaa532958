"""Clusters of many states (d > 32) through the GPU boundary MPS (Sec. 2: the
row transfer operator applied to the boundary MPS, then truncated).

Above d = 32 the MPO's d-index contractions run as batched GEMMs on the matrix
cores, and the range finder's panels of chi * d rows (beyond 512 rows and
beyond 512 stacked R rows) take TSQR on the register QR kernel at two or more
levels.

* Exactness: with no couplings between rows every row function has rank <= d
  across each cut (only the row's own horizontal table crosses it), so with
  chi >= d the truncation keeps everything.  The rows are then independent
  chains: log Z is the sum over rows of log sum_x exp(-beta E_r(x)), with
  E_r the row's own local and horizontal energies (enumerated densely), and
  each row's boundary function is proportional to exp(-beta E_r) (the sum over
  the rows below is a constant), so its overlap with the GPU's is 1 (the closed
  form is pinned against brute force in test_decoupled_rows.py).  At
  d = 72 and chi = 80 the panels have 72 * 72 = 5184 rows (11 blocks, then 792
  stacked rows: two TSQR levels).
* d = 256 (8-spin clusters, 4x4 king's, beta = 4, chi = 64, panels of 16384
  rows): properties that hold at any size (right isometries, finite row
  scales, capped bonds), and the search returns the full beam with Eq. (1)
  energies.
"""
import numpy as np
import pytest

from workloads import random_potts, spin_instance, potts_from_spins
from oracle.bmps import mps_full
from oracle.energy import potts_energy
from test_decoupled_rows import decoupled_log_z

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_02317_amd import spg  # noqa: E402

DEV = torch.device("cuda:0")


def _rows(env):
    T, lam = spg.env_export(env)
    return spg.unpack_mps(T, spg.env_info(env).bond_dims), lam


@pytest.mark.parametrize("d,chi", [(40, 48), (72, 80)])
def test_decoupled_rows_exact(d, chi):
    print(f"large d exact: d={d} chi={chi}", flush=True)
    inst = random_potts(2, 3, d, True, seed=200 + d, beta=0.5)
    inst.pair_v[:] = 0.0
    inst.pair_d[:] = 0.0
    inst.pair_a[:] = 0.0
    lz_exact, lw = decoupled_log_z(inst)
    env, lz = spg.boundary_mps(spg.build_peps(inst), chi)
    assert abs(lz - lz_exact) <= 1e-9 * abs(lz_exact), (lz, lz_exact)
    rows, _ = _rows(env)
    for r in range(inst.rows):
        a = mps_full(rows[r]).ravel()
        b = np.exp(lw[r] - lw[r].max())
        ov = abs(a @ b) / (np.linalg.norm(a) * np.linalg.norm(b))
        assert 1.0 - ov < 1e-10, (r, ov)


def test_d256_properties_and_search():
    print("large d: 4x4 king's, d=256, chi=64", flush=True)
    si = spin_instance(4, 4, 8, True, 5, h=("normal", 0.1), j_in=("pm1", 1.0),
                       j_out=("pm1", 1.0))
    inst = potts_from_spins(si, beta=4.0)
    chi, M = 64, 1000
    env, _ = spg.boundary_mps(spg.build_peps(inst), chi, want_logZ=False)
    rows, lam = _rows(env)
    assert np.all(np.isfinite(lam))
    assert spg.env_info(env).bond_dims.max() <= chi
    for r, row in enumerate(rows[:-1]):
        for c in range(1, inst.cols):
            a = row[c]
            G = np.einsum("axb,cxb->ac", a, a)
            np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-10, err_msg=f"{r},{c}")
    N = inst.rows * inst.cols
    st = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    en = torch.zeros(M, dtype=torch.float64, device=DEV)
    lp = torch.zeros(M, dtype=torch.float64, device=DEV)
    n = spg.branch_and_bound(env, M, st, en, lp)
    torch.cuda.synchronize()
    assert n == M
    states, E = st.cpu().numpy(), en.cpu().numpy()
    np.testing.assert_allclose(E, potts_energy(inst, states), atol=1e-9)
    assert np.all(np.diff(E) >= -1e-9)
