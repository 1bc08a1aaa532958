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


def _search(env, N, M, **kw):
    st = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    en = torch.zeros(M, dtype=torch.float64, device=DEV)
    lp = torch.zeros(M, dtype=torch.float64, device=DEV)
    n = spg.branch_and_bound(env, M, st, en, lp, **kw)
    torch.cuda.synchronize()
    return st.cpu().numpy()[:n], en.cpu().numpy()[:n], lp.cpu().numpy()[:n]


def _small_shape(rng, max_states=1 << 15, min_sites=1):
    while True:
        R, C, d = int(rng.integers(1, 5)), int(rng.integers(2, 6)), int(rng.choice([2, 3, 4]))
        if d ** (R * C) <= max_states and d ** (C // 2) <= 64 and R * C >= min_sites:
            return R, C, d


@pytest.mark.parametrize("k", range(12))
def test_random_exact_regime_gpu_pipeline_vs_brute_force(k):
    """The whole GPU pipeline (PEPS, boundary MPS at the exact bond dimension,
    search) against brute force: log Z to 1e-9; with a beam of every state
    the returned energies are the sorted spectrum."""
    from oracle.exact import brute_force
    rng = np.random.default_rng(3000 + k)
    R, C, d = _small_shape(rng)
    kings = bool(rng.integers(0, 2))
    inst = random_potts(R, C, d, kings, seed=4000 + k, beta=float(rng.uniform(0.2, 1.2)))
    bf = brute_force(inst)
    peps = spg.build_peps(inst)
    env, lz = spg.boundary_mps(peps, d ** (C // 2))
    assert abs(lz - bf["logZ"]) < 1e-9 * max(1.0, abs(bf["logZ"]))
    N = R * C
    if d ** N <= 2048:
        st, en, lp = _search(env, N, d ** N)
        assert len(st) == d ** N
        np.testing.assert_allclose(en, np.sort(bf["E"]), atol=1e-9)
        np.testing.assert_allclose(en, potts_energy(inst, st), atol=1e-9)
        # the scores are the exact log-probabilities -beta E - log Z
        np.testing.assert_allclose(lp, -inst.beta * en - bf["logZ"], atol=1e-8)
    else:
        st, en, lp = _search(env, N, 64)
        np.testing.assert_allclose(en, potts_energy(inst, st), atol=1e-9)
        assert en[0] >= bf["E_min"] - 1e-9


def _alone(inst, chi, M, prec, cut):
    peps = spg.build_peps(inst)
    try:
        env, lz = spg.boundary_mps(peps, chi, precision=prec)
    except spg.SpgError as e:
        assert e.code == -4            # non-finite log Z: a batch reports NaN
        env, _ = spg.boundary_mps(peps, chi, precision=prec, want_logZ=False)
        lz = float("nan")
    st, en, lp = _search(env, inst.rows * inst.cols, M, cut_off_prob=cut)
    return st, en, lp, lz


@pytest.mark.parametrize("k", range(6))
def test_random_batch_equals_each_instance_alone(k):
    """Random batches (shapes, d, chi, beams, precisions, shared shape classes,
    stream counts, cut-off): eager runs and graph replays give bitwise each
    instance's own run."""
    rng = np.random.default_rng(5000 + k)
    cut = float(rng.choice([0.0, 1e-3]))
    insts = []
    for i in range(int(rng.integers(2, 6))):
        if insts and rng.random() < 0.4:            # a member of the previous shape class
            p = insts[-1]
            inst = random_potts(p[0].rows, p[0].cols, p[0].d, p[4], seed=6000 + 10 * k + i,
                                beta=1.0)
            insts.append((inst, p[1], p[2], p[3], p[4]))
            continue
        R, C = int(rng.integers(2, 6)), int(rng.integers(2, 6))
        d = int(rng.choice([2, 3, 4, 5]))
        kings = bool(rng.integers(0, 2))
        inst = random_potts(R, C, d, kings, seed=6000 + 10 * k + i,
                            beta=float(rng.uniform(0.3, 1.2)))
        insts.append((inst, int(rng.choice([4, 8, 12])), int(rng.choice([1, 9, 40, 100])),
                      str(rng.choice(["fp64", "fp64", "fp32"])), kings))
    peps = [spg.build_peps(x[0]) for x in insts]
    b = spg.Batch(peps, chi=[x[1] for x in insts], max_states=[x[2] for x in insts],
                  precision=[x[3] for x in insts], cut_off_prob=cut,
                  n_streams=int(rng.integers(1, 4)), classes=bool(rng.integers(0, 2)))
    b.run(use_graph=False)
    eager = [b.result(i) for i in range(b.n)]
    for i, (inst, chi, M, prec, _) in enumerate(insts):
        a = _alone(inst, chi, M, prec, cut)
        for u, v in zip(eager[i][:3], a[:3]):
            assert np.array_equal(u, v), f"instance {i}"
        assert eager[i][3] == a[3] or (np.isnan(eager[i][3]) and np.isnan(a[3])), f"instance {i}"
    for rep in range(2):
        b.run(use_graph=True)
        torch.cuda.synchronize()
        for i in range(b.n):
            for u, v in zip(b.result(i)[:3], eager[i][:3]):
                assert np.array_equal(u, v), f"replay {rep} instance {i}"


@pytest.mark.parametrize("k", range(10))
def test_random_droplets_match_oracle(k):
    """Random merged searches with droplets (cut-offs, beams narrower and wider
    than the number of frontiers): per returned state the oracle's droplets in
    its order, bitwise configurations and energies to 1e-9."""
    rng = np.random.default_rng(7000 + k)
    R, C, d = _small_shape(rng, 1 << 20, min_sites=6)
    kings = bool(rng.integers(0, 2))
    inst = random_potts(R, C, d, kings, seed=8000 + k, beta=float(rng.uniform(0.3, 1.0)))
    chi = min(d ** (C // 2), 16)
    ora = oracle_bmps(inst, chi)
    T, dims = spg.pack_oracle_mps(ora["A"], chi, d)
    env = spg.env_import(spg.build_peps(inst), chi, dims, T, np.array(ora["lam"]))
    M = int(rng.choice([3, 20, 60, 3 * d ** min(C + 1, R * C)]))
    cut = float(rng.choice([0.0, 1e-3]))
    drop = (float(rng.choice([0.5, 3.0, 20.0])), int(rng.integers(0, 3)), int(rng.choice([1, 4, 64])))
    N = R * C
    st, en, _ = _search(env, N, M, cut_off_prob=cut, merge_branches=True, droplets=drop)
    ref = beam_search(inst, ora["A"], M, cut_off_prob=cut, merge=True, droplets=drop)
    fin = np.isfinite(ref["scores"])
    assert {tuple(x) for x in st.tolist()} == {tuple(x) for x in ref["states"][fin].tolist()}
    by_state = {tuple(x.tolist()): dl for x, dl, f in zip(ref["states"], ref["droplets"], fin) if f}
    for i in range(len(st)):
        cfg, de = spg.droplets(env, i)
        want = by_state[tuple(st[i].tolist())]
        assert len(cfg) == len(want), i
        for (x, e), y, g in zip(want, cfg, de):
            np.testing.assert_array_equal(y, x)
            assert abs(g - e) < 1e-9


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("k", range(8))
def test_random_reduced_precision_full_beam(k, prec):
    """Whole reduced-precision searches (the matrix-core products at every
    column of every row) at random shapes in the exact regime, with a beam of
    every state, so nothing is pruned.  A state drops out only if one of its
    conditionals rounds to zero (its running-error bound reaches 1), which
    the most probable states cannot: with FP32 inputs the lowest-energy tenth
    of the spectrum comes back complete and in order, with log-probabilities
    within 1e-3 of -beta E - log Z; with BF16 inputs the ground state does.
    Every returned state is distinct, in energy order and carries its Eq. (1)
    energy."""
    from oracle.exact import brute_force
    rng = np.random.default_rng(9000 + k)
    R, C, d = _small_shape(rng, 2048, min_sites=4)
    kings = bool(rng.integers(0, 2))
    inst = random_potts(R, C, d, kings, seed=9100 + k, beta=float(rng.uniform(0.2, 0.8)))
    bf = brute_force(inst)
    env, _ = spg.boundary_mps(spg.build_peps(inst), d ** (C // 2), precision=prec)
    N = R * C
    st, en, lp = _search(env, N, d ** N)
    assert len({tuple(x) for x in st.tolist()}) == len(st)
    np.testing.assert_allclose(en, potts_energy(inst, st), atol=1e-9)
    assert np.all(np.diff(en) >= 0)
    if prec == "fp32":
        top = np.sort(bf["E"])[: max(1, d ** N // 10)]
        assert len(st) >= len(top)
        np.testing.assert_allclose(en[: len(top)], top, atol=1e-9)
        np.testing.assert_allclose(lp[: len(top)], -inst.beta * top - bf["logZ"], atol=1e-3)
    else:
        assert len(st) >= 1 and abs(en[0] - bf["E_min"]) < 1e-9
