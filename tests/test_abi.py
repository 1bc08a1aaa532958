"""The C-ABI library loads and exports every symbol include/spg.h declares;
argument checks that return before any device work (CPU only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "spg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spg_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ["spg_build_peps", "spg_boundary_mps", "spg_marginals", "spg_branch_and_bound"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2502_02317_amd import spg
    lib = spg.load()
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(spg.EXPORTS) == _declared()


def _desc(rows=2, cols=2, d=2, beta=1.0, kings=0):
    from paper_2502_02317_amd.spg import InstanceDesc
    le = np.zeros((rows, cols, d))
    ph = np.zeros((rows, cols - 1, d, d))
    pv = np.zeros((rows - 1, cols, d, d))
    keep = (le, ph, pv)
    return InstanceDesc(rows, cols, d, kings, beta, le.ctypes.data, ph.ctypes.data,
                        pv.ctypes.data, None, None), keep


@pytest.mark.parametrize("kw,code", [
    (dict(d=300), -5), (dict(cols=1), -5), (dict(beta=float("nan")), -4), (dict(beta=-1.0), -4),
    (dict(kings=1), -1)])
def test_build_peps_rejects_bad_arguments(kw, code):
    from paper_2502_02317_amd import spg
    lib = spg.load()
    desc, keep = _desc(**kw)
    h = C.c_void_p()
    assert lib.spg_build_peps(C.byref(desc), None, C.byref(h)) == code
    assert lib.spg_last_error().decode()
    assert not h.value


def test_null_arguments():
    from paper_2502_02317_amd import spg
    lib = spg.load()
    h = C.c_void_p()
    assert lib.spg_build_peps(None, None, C.byref(h)) == -1
    assert lib.spg_boundary_mps(None, None, None, C.byref(h), None) == -1
    assert lib.spg_marginals(None, 0, 1, None, None, None) == -1
    n = C.c_int32()
    assert lib.spg_branch_and_bound(None, None, None, None, None, C.byref(n), None) == -1
    lib.spg_free_peps(None)
    lib.spg_free_env(None)


def test_proposal_entry_points_reject_bad_arguments():
    """Checked before any device call, so these run without a GPU."""
    from paper_2502_02317_amd import spg
    lib = spg.load()
    h = C.c_void_p()
    assert lib.spg_proposal_create(0, 1, C.byref(h)) == -1
    assert lib.spg_proposal_create(65, 1, C.byref(h)) == -1
    assert lib.spg_proposal_create(8, 1, None) == -1
    assert not h.value
    n = C.c_int32()
    assert lib.spg_proposal_params(None, None, None, C.byref(n)) == -1
    assert lib.spg_proposal_train(None, None, None, None, None) == -1
    assert lib.spg_proposal_features(None, 0, 1, None, None, None, None) == -1
    assert lib.spg_proposal_forward(None, 1, 2, None, None, None) == -1
    assert lib.spg_proposal_loss_grad(None, 1, 2, None, None, None, None, None) == -1
    assert lib.spg_proposal_adam(None, None, C.c_float(0.1), None) == -1
    assert lib.spg_search_stats(None, None) == -1
    lib.spg_proposal_free(None)
