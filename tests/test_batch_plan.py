"""Host-side plan of the batched workload (256 king's lattices, side L in
6..12, d = 16, chi in {16, 32}, beam M = 512): the units spg_batch_create
forms and the layout of each class's slice, computed without a device by
spg_batch_plan, checked on the CPU.

A class holds its members in equal slices of one allocation, and every
class-batched kernel shifts its pointers by member x slice bytes (64-bit
arithmetic), so its addresses stay inside the class when each buffer of the
slice is inside the slice and the class inside its allocation.  Checked:
members of a class share their shape; classes stay within the 1 GiB cap (so
every byte offset inside a class, and every element index inside a buffer,
fits in 31 bits); buffers are 256-byte aligned, disjoint and inside the slice;
the PEPS tables and the boundary-MPS tensors have the sizes the method's
shapes give (Sec. 2: [rows][cols] sites of d states, chi x d x chi MPS
tensors), computed here independently of the library; classes are filled up
to the cap in instance order."""
import numpy as np
import pytest

from workloads import cfg3_shapes

from paper_2502_02317_amd import spg

CLASS_CAP = 1 << 30
M = 512
D = 16


@pytest.fixture(scope="module")
def plan():
    L, chi = cfg3_shapes(256)
    shapes = [(int(x), int(x), D, 1) for x in L]
    unit_of, units, layouts = spg.batch_plan(shapes, [int(c) for c in chi], M)
    return L, chi, unit_of, units, layouts


def test_every_instance_in_one_unit(plan):
    L, chi, unit_of, units, _ = plan
    assert len(unit_of) == 256
    assert unit_of.min() == 0 and unit_of.max() == len(units) - 1
    counts = np.bincount(unit_of, minlength=len(units))
    assert [m for m, _ in units] == counts.tolist()
    # units appear in order of their first instance
    firsts = [int(np.flatnonzero(unit_of == u)[0]) for u in range(len(units))]
    assert firsts == sorted(firsts)


def test_class_members_share_their_shape(plan):
    L, chi, unit_of, units, _ = plan
    for u, (m, _) in enumerate(units):
        idx = np.flatnonzero(unit_of == u)
        assert len(set(zip(L[idx].tolist(), chi[idx].tolist()))) == 1


def test_classes_within_the_cap(plan):
    _, _, _, units, _ = plan
    for m, slice_bytes in units:
        if m == 1:
            assert slice_bytes == 0
            continue
        assert slice_bytes > 0 and slice_bytes % 256 == 0
        assert m * slice_bytes <= CLASS_CAP < 2 ** 31


def test_classes_fill_up_to_the_cap_in_order(plan):
    L, chi, unit_of, units, _ = plan
    by_shape = {}
    for u, (m, slice_bytes) in enumerate(units):
        idx = np.flatnonzero(unit_of == u)
        key = (int(L[idx[0]]), int(chi[idx[0]]))
        by_shape.setdefault(key, []).append((m, slice_bytes))
    for key, us in by_shape.items():
        n_shape = int(np.sum((L == key[0]) & (chi == key[1])))
        assert sum(m for m, _ in us) == n_shape
        sl = max(s for _, s in us)
        if sl == 0:                       # one instance of this shape: not a class
            assert n_shape == 1
            continue
        cap = CLASS_CAP // sl
        # every unit but the last of a shape is full; the last holds the rest
        assert all(m == cap for m, _ in us[:-1]), key
        assert 1 <= us[-1][0] <= cap


def test_slice_layout_disjoint_aligned_inside(plan):
    _, _, _, units, layouts = plan
    for (m, slice_bytes), lay in zip(units, layouts):
        if m == 1:
            assert len(lay) == 0
            continue
        off, nb = lay[:, 0], lay[:, 1]
        assert np.all(off % 256 == 0)
        assert np.all(nb > 0)
        ends = off + nb
        assert np.all(off[1:] >= ends[:-1])              # disjoint, in order
        assert ends[-1] <= slice_bytes
        assert slice_bytes == off[-1] + (nb[-1] + 255) // 256 * 256
        assert np.all(nb // 8 < 2 ** 31)                  # element indices in 31 bits


def test_table_and_tensor_sizes_follow_the_shapes(plan):
    L, chi, unit_of, units, layouts = plan
    for u, ((m, _), lay) in enumerate(zip(units, layouts)):
        if m == 1:
            continue
        i = int(np.flatnonzero(unit_of == u)[0])
        R = C = int(L[i])
        c = int(chi[i])
        dd = D * D
        expect = [R * C * D, R * (C - 1) * dd, (R - 1) * C * dd, (R - 1) * (C - 1) * dd,
                  (R - 1) * (C - 1) * dd]
        expect = [8 * n for n in expect + expect] + [8 * dd] * 3 + [8, 8 * R]
        # the 15 PEPS tables (energies, weights, helper tables, an empty one
        # padded to 8 bytes, the row log-scales), then the boundary MPS
        # tensors [rows][cols][chi][d][chi] and their log-scales [rows]
        assert lay[:15, 1].tolist() == expect
        assert int(lay[15, 1]) == 8 * R * C * c * D * c
        assert int(lay[16, 1]) == 8 * R


def test_plan_rejects_bad_shapes():
    with pytest.raises(spg.SpgError):
        spg.batch_plan([(4, 1, 16, 1)], 16, M)           # fewer than 2 columns
    with pytest.raises(spg.SpgError):
        spg.batch_plan([(4, 4, 300, 1)], 16, M)          # d above 256
    with pytest.raises(spg.SpgError):
        spg.batch_plan([(4, 4, 16, 2)], 16, M)           # kings must be 0 or 1


def test_plan_without_classes_or_with_reduced_precision():
    shapes = [(6, 6, D, 1)] * 4 + [(7, 7, D, 1)] * 2
    # classes off: every instance its own unit
    unit_of, units, _ = spg.batch_plan(shapes, 16, M, classes=False)
    assert unit_of.tolist() == list(range(6)) and all(m == 1 for m, _ in units)
    # FP32 instances never join a class; the FP64 ones of equal shape do
    precs = ["fp64", "fp32", "fp64", "fp64", "fp32", "fp64"]
    unit_of, units, _ = spg.batch_plan(shapes, 16, M, precision=precs)
    assert unit_of[0] == unit_of[2] == unit_of[3]
    assert len({unit_of[1], unit_of[4], unit_of[0], unit_of[5]}) == 4
    assert [m for m, _ in units] == [3, 1, 1, 1]
    # different chi or beam: different classes
    unit_of, _, _ = spg.batch_plan([(6, 6, D, 1)] * 3, [16, 32, 16], [M, M, M // 2])
    assert len(set(unit_of.tolist())) == 3


def test_kernel_switches_reject_other_values():
    lib = spg.load()
    assert lib.spg_set_kernel_forms(2, 1) != 0
    assert lib.spg_set_kernel_forms(1, -1) != 0
    assert lib.spg_set_gemm_precision(3) != 0
    assert lib.spg_set_kernel_forms(1, 1) == 0           # the defaults
    assert lib.spg_set_gemm_precision(0) == 0
