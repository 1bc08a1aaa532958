"""Pins of the oracle's generator and truncated-SVD protocol (CPU only)."""
import numpy as np
import pytest

from oracle.linalg import splitmix64, sketch, tsvd_left, tsvd_right


def test_splitmix64_reference_outputs():
    """First outputs of the public SplitMix64 reference implementation, seed 0."""
    out = [int(v) for v in splitmix64(0, np.arange(3))]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_sketch_range():
    S = sketch(64, 16)
    assert S.shape == (64, 16) and S.min() >= -1 and S.max() < 1
    assert abs(S.mean()) < 0.1


@pytest.mark.parametrize("m,n,r,k", [(40, 30, 5, 8), (64, 200, 12, 12), (100, 20, 20, 16)])
def test_tsvd_exact_when_rank_fits(m, n, r, k):
    rng = np.random.default_rng(m + n)
    B = rng.normal(size=(m, r)) @ rng.normal(size=(r, n))
    U, Rm = tsvd_left(B, k, 16, 1)
    # an isometry on the kept directions; directions beyond rank(B) carry no
    # weight and are zeroed (the null-direction rule)
    G = U.T @ U
    np.testing.assert_allclose(G, np.diag(np.round(np.diag(G))), atol=1e-12)
    assert int(round(np.trace(G))) == min(r, k, U.shape[1])
    if r <= k:
        np.testing.assert_allclose(U @ Rm, B, atol=1e-10 * np.abs(B).max())
    s_ref = np.linalg.svd(B, compute_uv=False)[: U.shape[1]]
    s = np.linalg.svd(Rm, compute_uv=False)
    np.testing.assert_allclose(s[: min(r, k)], s_ref[: min(r, k)], rtol=1e-9)


def test_tsvd_near_optimal_for_decaying_spectrum():
    rng = np.random.default_rng(1)
    m, n, k = 120, 90, 10
    Uo, _ = np.linalg.qr(rng.normal(size=(m, n)))
    Vo, _ = np.linalg.qr(rng.normal(size=(n, n)))
    sv = 0.5 ** np.arange(n)
    B = (Uo * sv) @ Vo.T
    U, Rm = tsvd_left(B, k, 16, 1)
    err = np.linalg.norm(B - U @ Rm, 2)
    assert err <= 1.01 * sv[k]
    Lm, V = tsvd_right(B, k, 16, 1)
    np.testing.assert_allclose(V @ V.T, np.eye(k), atol=1e-12)
    assert np.linalg.norm(B - Lm @ V, 2) <= 1.01 * sv[k]
