"""spg_marginals_noalloc (the entry point for callers that cannot allocate)
against spg_marginals on the same env and inputs: bitwise equal, on two calls
in a row, the second with fewer beam states (the static scratch keeps the
first call's contents)."""
import numpy as np
import pytest

from workloads import random_potts, config_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_02317_amd import spg  # noqa: E402

DEV = torch.device("cuda:0")


def _both(env, site, cfg, d):
    cfg_t = torch.tensor(cfg, dtype=torch.int32, device=DEV)
    ref = torch.full((cfg.shape[0], d), 7.0, dtype=torch.float64, device=DEV)
    got = torch.full((cfg.shape[0], d), 9.0, dtype=torch.float64, device=DEV)
    spg.marginals(env, site, cfg_t, ref)
    spg.marginals_noalloc(env, site, cfg_t, got)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_noalloc_equals_marginals_two_calls(precision):
    print(f"noalloc small lattice {precision}", flush=True)
    inst = random_potts(3, 4, 3, True, seed=5, beta=0.8)
    env, _ = spg.boundary_mps(spg.build_peps(inst), 9, precision=precision)
    rng = np.random.default_rng(3)
    big = rng.integers(0, inst.d, size=(200, inst.n_sites))
    small = rng.integers(0, inst.d, size=(37, inst.n_sites))
    for site in range(inst.n_sites):
        for cfg in (big, small):
            ref, got = _both(env, site, cfg, inst.d)
            assert np.array_equal(ref, got, equal_nan=True), (site, cfg.shape)


def test_noalloc_bench_workload_size():
    """The 8x8 d=16 workload at chi 32 with a beam of 1024, then 100."""
    print("noalloc kings8x8_d16", flush=True)
    inst = config_instance("kings8x8_d16", 0)
    env, _ = spg.boundary_mps(spg.build_peps(inst), 32, want_logZ=False)
    rng = np.random.default_rng(4)
    for n in (1024, 100):
        cfg = rng.integers(0, inst.d, size=(n, inst.n_sites))
        for site in (0, 9, 37, 63):
            ref, got = _both(env, site, cfg, inst.d)
            assert np.array_equal(ref, got, equal_nan=True), (site, n)


def test_noalloc_rejects_a_beam_beyond_the_scratch():
    import ctypes as C
    print("noalloc size check", flush=True)
    inst = config_instance("kings8x8_d16", 0)
    env, _ = spg.boundary_mps(spg.build_peps(inst), 32, want_logZ=False)
    n = 30000                                # ~2.7 kB each: beyond 64 MiB
    cfg = torch.zeros((n, inst.n_sites), dtype=torch.int32, device=DEV)
    out = torch.full((n, inst.d), 5.0, dtype=torch.float64, device=DEV)
    lib = spg.load()
    rc = lib.spg_marginals_noalloc(env.handle, 3, n, C.c_void_p(cfg.data_ptr()),
                                   C.c_void_p(out.data_ptr()), None)
    assert rc == -1
    assert b"scratch" in lib.spg_last_error()
    torch.cuda.synchronize()
    assert bool((out == 5.0).all())
