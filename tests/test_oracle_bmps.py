"""Invariants of the oracle's boundary MPS in the truncated regime (CPU only)."""
import numpy as np

from workloads import spin_instance, potts_from_spins, random_potts
from oracle.exact import row_transfer, normalised
from oracle.bmps import boundary_mps, mps_full


def _centre(row):
    """Index of the centre: the tensor that is not an isometry towards the right
    (phi_0, or phi_1 when column 0 kept its natural basis)."""
    return 1 if (row[0].shape[0] == 1 and row[0].shape[2] == row[0].shape[1]
                 and np.array_equal(row[0].reshape(row[0].shape[1], -1),
                                    np.eye(row[0].shape[1]))) else 0


def test_canonical_form_and_normalised():
    """Fitted rows: the centre has unit norm and the tensors right of it are
    right isometries.  The bottom row is the exact chain (bond d,
    non-negative), equal to the exact row function."""
    inst = random_potts(4, 5, 3, True, seed=5, beta=0.6)
    mp = boundary_mps(inst, chi=4)
    bottom = mp["A"][-1]
    assert [a.shape for a in bottom] == [(1, 3, 3)] + [(3, 3, 3)] * 3 + [(3, 3, 1)]
    assert all((a >= 0).all() for a in bottom)
    rows, _ = row_transfer(inst)
    ex = normalised(rows[-1])
    ap = mps_full(bottom)
    np.testing.assert_allclose(ap / ap.max(), ex / ex.max(), rtol=1e-13)
    for row in mp["A"][:-1]:
        c0 = _centre(row)
        assert abs(np.linalg.norm(row[c0]) - 1) < 1e-12
        for A in row[c0 + 1:]:
            G = np.einsum("axb,cxb->ac", A, A)
            np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-12)
        assert max(A.shape[0] for A in row) <= 4


def test_truncation_error_falls_with_chi():
    """Well-conditioned strip (moderate beta): the error against the exact row
    transfer falls as chi grows and vanishes at the exact rank."""
    si = spin_instance(5, 3, 2, True, seed=2, h=("normal", 1.0), j_in=("normal", 1.0),
                       j_out=("normal", 0.5))
    inst = potts_from_spins(si, beta=0.5)
    rows, lz = row_transfer(inst)
    errs = []
    for chi in (1, 2, 3, 4):
        mp = boundary_mps(inst, chi=chi)
        e = 0.0
        for r in range(inst.rows):
            ex = normalised(rows[r])
            ex = ex / np.linalg.norm(ex)
            ap = mps_full(mp["A"][r])
            e = max(e, np.linalg.norm(ex - ap / np.linalg.norm(ap) * np.sign(ap.sum())))
        errs.append(e)
    assert errs[-1] < 1e-12
    assert all(a >= b - 1e-12 for a, b in zip(errs, errs[1:]))
    assert errs[0] > 1e-6


def test_truncated_low_temperature_strip():
    """Truncation active (a 4-wide strip at the 8x8 d=16 workload's
    distributions, chi = 32 < 256 states on each side of the middle cut): log Z
    against the exact row transfer falls with chi (measured 1.0e-8, 2.5e-10 and
    2.1e-11 relative at chi = 16, 32, 64: the truncation's error plus the
    rounding of the rotated cut)."""
    si = spin_instance(8, 4, 4, True, seed=0, h=("normal", 1.0), j_in=("normal", 1.0),
                       j_out=("pm1", 1.0))
    inst = potts_from_spins(si, beta=2.0)
    _, lz = row_transfer(inst)
    e16, e32, e64 = (abs(boundary_mps(inst, chi=chi)["logZ"] - lz) for chi in (16, 32, 64))
    assert e16 > e32 > e64
    assert e32 <= 1e-9 * abs(lz)
