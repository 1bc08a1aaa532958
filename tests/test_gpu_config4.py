"""The 12x12 king's workload with d = 24 (8-spin clusters, the 24 lowest
states kept), beta = 4, chi = 64 and a beam of 4096, on the GPU.

At these shapes the site tensors (64 x 24 x 64) no longer fit the LDS-staged
marginal and right-environment kernels, so the global-memory ones run, and the
truncation's panels reach 64 * 24 = 1536 rows (the LDS-resident QR with TSQR
and the global-memory QR beside the register one).

* Search and marginals: against the oracle on one shared environment.  The
  oracle's own boundary MPS at this size takes hours of dense SVDs, so the
  environment is a seeded synthetic one with the workload's bond dimensions
  (min(chi, d^c, d^(cols-c))) and positive entries; every conditional then
  has condition number 1 and the running-error bound is ~1e-13.
* The GPU's own boundary MPS at full size: properties that hold at any size
  (every tensor right of a row's centre is a right isometry, the bottom row
  is the exact non-negative chain, the bond dimensions are capped), and the
  search returns the full beam with Eq. (1) energies.
"""
import numpy as np
import pytest

from workloads import config_instance
from oracle.energy import potts_energy
from oracle.search import beam_search, teacher_forced_logp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_02317_amd import spg  # noqa: E402

DEV = torch.device("cuda:0")
CHI, M = 64, 4096


def _synthetic_env(inst, seed):
    rng = np.random.default_rng(seed)
    C, d = inst.cols, inst.d
    dims = [min(CHI, d ** c, d ** (C - c)) for c in range(C + 1)]
    return [[rng.random((dims[c], d, dims[c + 1])) for c in range(C)] for _ in range(inst.rows)]


def test_search_and_marginals_on_a_shared_environment():
    print("config4 shape: shared synthetic environment", flush=True)
    inst = config_instance("kings12x12_d24", 0)
    A = _synthetic_env(inst, 7)
    T, dims = spg.pack_oracle_mps(A, CHI, inst.d)
    env = spg.env_import(spg.build_peps(inst), CHI, dims, T, np.zeros(inst.rows))
    rng = np.random.default_rng(1)
    cfg = rng.integers(0, inst.d, size=(64, inst.n_sites))
    cfg_t = torch.tensor(cfg, dtype=torch.int32, device=DEV)
    for site in (0, 13, 30, 77, 143):
        out = torch.empty((64, inst.d), dtype=torch.float64, device=DEV)
        spg.marginals(env, site, cfg_t, out)
        torch.cuda.synchronize()
        r, c = divmod(site, inst.cols)
        ref = teacher_forced_logp(inst, A, r, c, cfg)
        np.testing.assert_allclose(out.cpu().numpy(), ref, atol=1e-10)
    N = inst.n_sites
    st = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    en = torch.zeros(M, dtype=torch.float64, device=DEV)
    lp = torch.zeros(M, dtype=torch.float64, device=DEV)
    n = spg.branch_and_bound(env, M, st, en, lp)
    torch.cuda.synchronize()
    ref = beam_search(inst, A, M)
    assert n == ref["n_valid"] == M
    st, en, lp = st.cpu().numpy(), en.cpu().numpy(), lp.cpu().numpy()
    np.testing.assert_allclose(np.sort(lp), np.sort(ref["scores"]), atol=1e-8)
    shared = {tuple(x) for x in st.tolist()} & {tuple(x) for x in ref["states"].tolist()}
    assert len(shared) >= 0.99 * M
    assert abs(en[0] - ref["energies"][0]) < 1e-9
    np.testing.assert_allclose(en, potts_energy(inst, st), atol=1e-9)


def test_gpu_pipeline_full_size_properties():
    print("config4: GPU boundary MPS and search", flush=True)
    inst = config_instance("kings12x12_d24", 0)
    peps = spg.build_peps(inst)
    env, _ = spg.boundary_mps(peps, CHI, want_logZ=False)
    T, lam = spg.env_export(env)
    info = spg.env_info(env)
    rows = spg.unpack_mps(T, info.bond_dims)
    assert np.all(np.isfinite(lam))
    assert info.bond_dims.max() <= CHI
    bottom = rows[-1]
    assert all((a >= 0).all() for a in bottom)
    for r, row in enumerate(rows[:-1]):
        c0 = 1 if (row[0].shape[0] == 1 and row[0].shape[1] == row[0].shape[2]
                   and np.array_equal(row[0][0], np.eye(row[0].shape[1]))) else 0
        assert abs(np.linalg.norm(row[c0]) - 1.0) < 1e-12, r
        for c in range(c0 + 1, inst.cols):
            a = row[c]
            G = np.einsum("axb,cxb->ac", a, a)
            np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-10, err_msg=f"{r},{c}")
    N = inst.n_sites
    st = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    en = torch.zeros(M, dtype=torch.float64, device=DEV)
    lp = torch.zeros(M, dtype=torch.float64, device=DEV)
    n = spg.branch_and_bound(env, M, st, en, lp)
    torch.cuda.synchronize()
    assert n == M
    st, en = st.cpu().numpy(), en.cpu().numpy()
    np.testing.assert_allclose(en, potts_energy(inst, st), atol=1e-9)
    assert np.all(np.diff(en) >= -1e-9)


@pytest.mark.parametrize("shape,p,q", [((6, 4), 32, 3), ((5, 5), 32, 3)])
def test_panels_beyond_512_rows_match_oracle(shape, p, q):
    """Truncated two-site blocks with 24 * 24 = 576 rows: the range finder's
    panels go through the TSQR of the register QR kernel.  On a
    well-conditioned lattice (d = 24, beta = 0.3) with a sketch of 96 columns
    and three power iterations the range finder reaches the truncated SVD's
    subspace, so log Z and every row function equal the oracle's exact
    truncated SVD."""
    from workloads import spin_instance, potts_from_spins
    from oracle.bmps import boundary_mps as oracle_bmps
    print(f"panels beyond 512 rows {shape}", flush=True)
    R, C = shape
    si = spin_instance(R, C, 8, True, 0, h=("normal", 1.0), j_in=("normal", 1.0),
                       j_out=("normal", 1.0))
    inst = potts_from_spins(si, beta=0.3, d_keep=24)
    env, lz = spg.boundary_mps(spg.build_peps(inst), CHI, oversample=p, power_iters=q)
    ora = oracle_bmps(inst, CHI)
    assert abs(lz - ora["logZ"]) <= 1e-9 * abs(ora["logZ"])
    T, lam = spg.env_export(env)
    rows = spg.unpack_mps(T, spg.env_info(env).bond_dims)
    for r in range(R):
        a, b = rows[r], ora["A"][r]
        E = np.ones((1, 1))
        Ea = np.ones((1, 1))
        Eb = np.ones((1, 1))
        for x, y in zip(a, b):
            E = np.einsum("ij,ixk,jxl->kl", E, x, y)
            Ea = np.einsum("ij,ixk,jxl->kl", Ea, x, x)
            Eb = np.einsum("ij,ixk,jxl->kl", Eb, y, y)
        assert 1.0 - E[0, 0] / np.sqrt(Ea[0, 0] * Eb[0, 0]) < 1e-9, r
