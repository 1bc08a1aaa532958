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
            G = np.einsum("axb,cxb->ac", A, A)
            # a right isometry, or a partial one where null directions were dropped
            np.testing.assert_allclose(G, np.diag(np.round(np.diag(G))), atol=1e-12)
            assert np.round(np.diag(G)).sum() >= 1
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


def test_result_independent_of_orthonormal_completion(monkeypatch):
    """Blocks of numerical rank below chi occur; with the null-direction rule
    the contraction does not depend on how an implementation completes an
    orthonormal basis (here: Householder QR versus Gram-Schmidt with a
    different completion order)."""
    import oracle.linalg as L
    si = spin_instance(4, 5, 2, True, seed=6, h=("normal", 1.0), j_in=("normal", 1.0),
                       j_out=("normal", 0.4))
    inst = potts_from_spins(si, beta=0.5)
    ref = boundary_mps(inst, 5)

    def orth_gs(Y):
        m, n = Y.shape
        Q = np.zeros((m, n))
        spare = list(range(m))[::-1]
        for j in range(n):
            v = Y[:, j].copy()
            for _ in range(2):
                v -= Q[:, :j] @ (Q[:, :j].T @ v)
            while np.linalg.norm(v) < 1e-12 * max(1.0, np.linalg.norm(Y)):
                v = np.zeros(m)
                v[spare.pop(0)] = 1.0
                for _ in range(2):
                    v -= Q[:, :j] @ (Q[:, :j].T @ v)
            Q[:, j] = v / np.linalg.norm(v)
        return Q

    monkeypatch.setattr(L, "orth", orth_gs)
    alt = boundary_mps(inst, 5)
    assert abs(alt["logZ"] - ref["logZ"]) < 1e-10
    for r in range(inst.rows):
        a, b = mps_full(alt["A"][r]), mps_full(ref["A"][r])
        np.testing.assert_allclose(a, b, atol=1e-9 * np.abs(b).max())
