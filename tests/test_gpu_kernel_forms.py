"""Kernel forms of the boundary MPS that must give bitwise equal results,
through the C ABI (the row transfer operator applied to the boundary MPS and
truncated, Sec. 2):

* the MPO d-index contractions in column form (one thread per source column,
  all d outputs that share it) against the per-output forms, at each d the
  column forms exist for, with ragged bond dimensions;
* Q of the truncation's one-panel QR factorisations formed by a second kernel
  (a compute unit per column) against the panel kernel's own formation, at
  panel widths 32 to 80 and panels of 64 to 512 rows;

and both for the 8x8 king's d = 16 workload at chi = 32.  Each pair are
deterministic FP64 kernels that keep every output's operands and order of
terms, so equality is exact.
"""
import numpy as np
import pytest

from workloads import random_potts, config_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_02317_amd import spg  # noqa: E402


def _contract(inst, chi, column_forms=True, q_split=True):
    spg.set_kernel_forms(mpo_columns=column_forms, q_split=q_split)
    try:
        peps = spg.build_peps(inst)
        try:
            env, lz = spg.boundary_mps(peps, chi)
        except spg.SpgError as e:
            assert e.code == -4                  # non-finite log Z: compare the tensors only
            env, _ = spg.boundary_mps(peps, chi, want_logZ=False)
            lz = float("nan")
        torch.cuda.synchronize()
        T, lam = spg.env_export(env)
        dims = spg.env_info(env).bond_dims.copy()
    finally:
        spg.set_kernel_forms()                   # the process defaults
    return T, lam, dims, lz


CASES = [
    # (rows, cols, d, kings, seed, beta, chi)
    (4, 4, 8, True, 701, 1.0, 12),
    (3, 5, 8, False, 702, 0.8, 7),
    (4, 3, 16, True, 703, 1.0, 20),
    (3, 4, 24, True, 704, 1.0, 30),
    (3, 3, 32, True, 705, 0.7, 24),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}_d{c[2]}_chi{c[6]}" for c in CASES])
def test_column_forms_equal_per_output_forms(case):
    R, C, d, kings, seed, beta, chi = case
    inst = random_potts(R, C, d, kings, seed=seed, beta=beta)
    a = _contract(inst, chi, column_forms=True)
    b = _contract(inst, chi, column_forms=False)
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert a[3] == b[3] or (np.isnan(a[3]) and np.isnan(b[3]))


def test_column_forms_equal_per_output_forms_kings8x8_d16():
    inst = config_instance("kings8x8_d16", 0)
    a = _contract(inst, 32, column_forms=True)
    b = _contract(inst, 32, column_forms=False)
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])


Q_CASES = [
    # (rows, cols, d, kings, seed, beta, chi): sketch widths chi + 16 up to 80
    (3, 4, 8, True, 721, 1.0, 16),       # 32-column panels of 64 rows
    (3, 5, 16, True, 722, 0.8, 20),      # 36 columns, 256 and 320 rows
    (3, 4, 16, True, 723, 0.7, 48),      # 64 columns, 256 to 512 rows
    (2, 5, 16, False, 724, 0.6, 64),     # 80 columns
]


@pytest.mark.parametrize("case", Q_CASES, ids=[f"{c[0]}x{c[1]}_d{c[2]}_chi{c[6]}" for c in Q_CASES])
def test_q_split_equals_in_kernel_q(case):
    R, C, d, kings, seed, beta, chi = case
    inst = random_potts(R, C, d, kings, seed=seed, beta=beta)
    a = _contract(inst, chi, q_split=True)
    b = _contract(inst, chi, q_split=False)
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert a[3] == b[3] or (np.isnan(a[3]) and np.isnan(b[3]))


def test_q_split_equals_in_kernel_q_kings8x8_d16():
    inst = config_instance("kings8x8_d16", 0)
    a = _contract(inst, 32, q_split=True)
    b = _contract(inst, 32, q_split=False)
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
