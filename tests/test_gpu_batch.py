"""Batches on the GPU (through the C ABI): every instance of a batch, eager or
replayed from the captured graph, gives bitwise the results of running it on
its own (spg_boundary_mps + spg_branch_and_bound with the same GEMM tile):
the same deterministic kernels run on the same data, on other streams or, for
members of a shape class, in launches that cover the whole class.
Graph replays are interleaved with other eager work and synchronisations and
each replay is checked."""
import numpy as np
import pytest

from workloads import random_potts, cfg3_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_02317_amd import spg  # noqa: E402

DEV = torch.device("cuda:0")


def _instances():
    # uneven sizes, d, chi and beams; one FP32-search instance
    spec = [(3, 3, 4, 6, 16, "fp64"), (5, 4, 3, 12, 40, "fp64"), (4, 4, 4, 8, 33, "fp32"),
            (2, 6, 5, 10, 7, "fp64")]
    out = []
    for k, (R, C, d, chi, M, prec) in enumerate(spec):
        out.append((random_potts(R, C, d, True, seed=500 + k, beta=1.0), chi, M, prec))
    out.append((cfg3_instance(0, 6), 16, 512, "fp64"))
    out.append((cfg3_instance(1, 7), 32, 512, "fp64"))
    return out


def _alone(inst, chi, M, prec, tile):
    spg.set_tuning(tile)
    try:
        peps = spg.build_peps(inst)
        try:
            env, lz = spg.boundary_mps(peps, chi, precision=prec)
        except spg.SpgError as e:
            # a non-finite log Z (truncation-error regime) is reported as NaN by batches
            assert e.code == -4
            env, _ = spg.boundary_mps(peps, chi, precision=prec, want_logZ=False)
            lz = float("nan")
        N = inst.rows * inst.cols
        st = torch.zeros((M, N), dtype=torch.int32, device=DEV)
        en = torch.zeros(M, dtype=torch.float64, device=DEV)
        lp = torch.zeros(M, dtype=torch.float64, device=DEV)
        n = spg.branch_and_bound(env, M, st, en, lp)
        torch.cuda.synchronize()
    finally:
        spg.set_tuning(32)                 # the process default
    return st[:n].cpu().numpy(), en[:n].cpu().numpy(), lp[:n].cpu().numpy(), lz


def _same(a, b, label):
    assert a[0].shape == b[0].shape, label
    assert np.array_equal(a[0], b[0]), label
    assert np.array_equal(a[1], b[1]), label
    assert np.array_equal(a[2], b[2]), label
    assert a[3] == b[3] or (np.isnan(a[3]) and np.isnan(b[3])), label


def _class_instances():
    """Several members per shape class (equal lattice, d, chi, beam), plus
    single instances, so both unit kinds run in one batch."""
    out = []
    for k in range(3):
        out.append((random_potts(3, 4, 4, True, seed=600 + k, beta=1.0), 8, 20, "fp64"))
    for k in range(2):
        out.append((random_potts(2, 5, 3, False, seed=610 + k, beta=0.7), 6, 33, "fp64"))
    out.append((random_potts(4, 4, 4, True, seed=620, beta=1.0), 8, 33, "fp32"))
    out.append((random_potts(3, 4, 4, True, seed=621, beta=1.0), 8, 21, "fp64"))
    for k in range(3):
        out.append((cfg3_instance(40 + k, 6), 16, 512, "fp64"))
    return out


@pytest.mark.parametrize("n_streams,classes,which", [(1, False, "mixed"), (3, False, "mixed"),
                                                     (2, True, "classes"), (1, True, "mixed")])
def test_batch_equals_each_instance_alone(n_streams, classes, which):
    insts = _instances() if which == "mixed" else _class_instances()
    peps = [spg.build_peps(i) for i, _, _, _ in insts]
    b = spg.Batch(peps, chi=[c for _, c, _, _ in insts], max_states=[m for _, _, m, _ in insts],
                  precision=[p for _, _, _, p in insts], n_streams=n_streams, classes=classes)
    n_units, _ = b.units()
    if which == "classes":
        assert n_units == 5            # three classes and two single instances
    b.run(use_graph=False)
    eager = [b.result(i) for i in range(b.n)]
    for i, (inst, chi, M, prec) in enumerate(insts):
        _same(eager[i], _alone(inst, chi, M, prec, 32), f"instance {i}")   # the default tile
    # graph replays, with unrelated eager work and synchronisations in between
    for rep in range(3):
        b.run(use_graph=True)
        torch.cuda.synchronize()
        for i in range(b.n):
            _same(b.result(i), eager[i], f"replay {rep} instance {i}")
        x = torch.randn(300, 300, device=DEV)
        (x @ x).sum().item()
        _alone(insts[0][0], insts[0][1], insts[0][2], insts[0][3], 64)


def test_autotuned_batch_equals_each_instance_alone_with_its_tile():
    insts = _class_instances()
    peps = [spg.build_peps(i) for i, _, _, _ in insts]
    b = spg.Batch(peps, chi=[c for _, c, _, _ in insts], max_states=[m for _, _, m, _ in insts],
                  precision=[p for _, _, _, p in insts], n_streams=2)
    tiles = b.autotune()
    assert set(tiles.tolist()) <= {32, 64}
    # the two kernel forms it also chooses give bitwise equal results, so each
    # instance equals its run alone with the default forms and its tile
    for i in range(b.n):
        t = b.tuning(i)
        assert t["gemm_tile"] == tiles[i]
        assert t["mpo_columns"] in (True, False) and t["q_split"] in (True, False)
    for i, (inst, chi, M, prec) in enumerate(insts):
        _same(b.result(i), _alone(inst, chi, M, prec, int(tiles[i])), f"instance {i}")
    b.run(use_graph=True)
    for i, (inst, chi, M, prec) in enumerate(insts):
        _same(b.result(i), _alone(inst, chi, M, prec, int(tiles[i])), f"graph instance {i}")


def test_gemm_tile_choice_keeps_results_close():
    """The 32 and 64 tiles sum every output in the same order; only split-K
    decisions differ, so results agree to rounding."""
    inst = random_potts(4, 6, 8, True, seed=9, beta=0.8)
    a = _alone(inst, 24, 64, "fp64", 64)
    c = _alone(inst, 24, 64, "fp64", 32)
    assert abs(a[3] - c[3]) <= 1e-9 * max(1.0, abs(a[3]))
    assert abs(a[1][0] - c[1][0]) <= 1e-9 * max(1.0, abs(a[1][0]))


def test_batch_argument_errors():
    inst = random_potts(2, 3, 3, True, seed=1, beta=1.0)
    peps = [spg.build_peps(inst)]
    with pytest.raises(spg.SpgError):
        spg.Batch(peps, chi=[0], max_states=[4])
    with pytest.raises(spg.SpgError):
        spg.Batch(peps, chi=[4], max_states=[0])
    with pytest.raises(spg.SpgError):
        spg.Batch(peps, chi=[4], max_states=[4], n_streams=0)
    b = spg.Batch(peps, chi=[4], max_states=[4])
    with pytest.raises(spg.SpgError):
        b.set_tuning(0, 48)
    with pytest.raises(spg.SpgError):
        b.result(1)


def test_host_plan_matches_the_batch():
    # spg_batch_plan (host only) forms the units spg_batch_create forms
    insts = _class_instances()
    peps = [spg.build_peps(i) for i, _, _, _ in insts]
    chis = [c for _, c, _, _ in insts]
    Ms = [m for _, _, m, _ in insts]
    precs = [p for _, _, _, p in insts]
    b = spg.Batch(peps, chi=chis, max_states=Ms, precision=precs, n_streams=3)
    nu, of = b.units()
    shapes = [(i.rows, i.cols, i.d, int(i.kings)) for i, _, _, _ in insts]
    unit_of, units, _ = spg.batch_plan(shapes, chis, Ms, precision=precs)
    assert nu == len(units)
    assert np.array_equal(of, unit_of)
