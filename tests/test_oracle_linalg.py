"""Pins of the oracle's generator and truncated SVD (CPU only)."""
import numpy as np
import pytest

from oracle.linalg import splitmix64, svd, svd_truncate_left, svd_truncate_right


def test_splitmix64_reference_outputs():
    """First outputs of the public SplitMix64 reference implementation, seed 0."""
    out = [int(v) for v in splitmix64(0, np.arange(3))]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


@pytest.mark.parametrize("m,n", [(40, 30), (30, 40), (17, 17), (64, 5)])
def test_svd_matches_dense_lapack(m, n):
    """On a well-conditioned matrix the Jacobi SVD and numpy's bidiagonal SVD
    agree: same singular values, same factorisation, orthonormal factors."""
    rng = np.random.default_rng(m * 100 + n)
    B = rng.normal(size=(m, n))
    U, s, Vt = svd(B)
    k = min(m, n)
    assert U.shape == (m, k) and s.shape == (k,) and Vt.shape == (k, n)
    np.testing.assert_allclose(s, np.linalg.svd(B, compute_uv=False), rtol=1e-13)
    assert np.all(np.diff(s) <= 0)
    np.testing.assert_allclose((U * s) @ Vt, B, atol=1e-13 * np.abs(B).max())
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-13)
    np.testing.assert_allclose(Vt @ Vt.T, np.eye(k), atol=1e-13)


def test_svd_graded_relative_accuracy():
    """B = Q diag(D) with Q orthogonal has singular values D exactly, here
    spanning 90 orders of magnitude: the Jacobi SVD returns every one of them
    to a few ulps (a bidiagonal SVD only resolves them to ~1e-16 max(D))."""
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(40, 30)))
    D = 10.0 ** (-3.0 * np.arange(30))
    U, s, Vt = svd(Q * D)
    np.testing.assert_allclose(s, D, rtol=1e-13)


@pytest.mark.parametrize("chi", [3, 8])
def test_truncation_is_eckart_young_optimal(chi):
    """The rank-chi split reaches the optimal error sqrt(sum of the discarded
    sigma^2) and its factors are an isometry and the projection."""
    rng = np.random.default_rng(chi)
    m, n = 30, 20
    Uo, _ = np.linalg.qr(rng.normal(size=(m, n)))
    Vo, _ = np.linalg.qr(rng.normal(size=(n, n)))
    sv = 0.6 ** np.arange(n)
    B = (Uo * sv) @ Vo.T
    U, Rm = svd_truncate_left(B, chi)
    assert U.shape == (m, chi)
    np.testing.assert_allclose(U.T @ U, np.eye(chi), atol=1e-13)
    np.testing.assert_allclose(Rm, U.T @ B, atol=1e-13)
    opt = np.sqrt((sv[chi:] ** 2).sum())
    assert abs(np.linalg.norm(B - U @ Rm) - opt) <= 1e-12
    Lm, V = svd_truncate_right(B, chi)
    np.testing.assert_allclose(V @ V.T, np.eye(chi), atol=1e-13)
    assert abs(np.linalg.norm(B - Lm @ V) - opt) <= 1e-12


def test_natural_basis_when_nothing_is_truncated():
    """A side with at most chi rows (left split) or columns (right split) is
    not rotated: the identity and the block itself, exactly."""
    rng = np.random.default_rng(5)
    B = rng.random((6, 50))
    U, Rm = svd_truncate_left(B, 6)
    assert np.array_equal(U, np.eye(6)) and np.array_equal(Rm, B)
    Lm, V = svd_truncate_right(B.T, 8)
    assert np.array_equal(V, np.eye(6)) and np.array_equal(Lm, B.T)
    # a tall block with few columns still needs a rotation on the left
    U, Rm = svd_truncate_left(B.T, 8)
    assert U.shape == (50, 6)
    np.testing.assert_allclose(U @ Rm, B.T, atol=1e-13)
