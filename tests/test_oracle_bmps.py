"""Invariants of the oracle's boundary MPS in the truncated regime (CPU only)."""
import numpy as np

from workloads import spin_instance, potts_from_spins, random_potts
from oracle.exact import row_transfer
from oracle.bmps import boundary_mps, mps_full


def test_right_canonical_and_normalised():
    inst = random_potts(4, 5, 3, True, seed=5, beta=0.6)
    mp = boundary_mps(inst, chi=4)
    for row in mp["A"]:
        assert abs(np.linalg.norm(row[0]) - 1) < 1e-12
        for A in row[1:]:
            k = A.shape[0]
            np.testing.assert_allclose(np.einsum("axb,cxb->ac", A, A), np.eye(k), atol=1e-12)
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
            ex = rows[r][0] / np.linalg.norm(rows[r][0])
            ap = mps_full(mp["A"][r])
            e = max(e, np.linalg.norm(ex - ap / np.linalg.norm(ap) * np.sign(ap.sum())))
        errs.append(e)
    assert errs[-1] < 1e-12
    assert all(a >= b - 1e-12 for a, b in zip(errs, errs[1:]))
    assert errs[0] > 1e-6
