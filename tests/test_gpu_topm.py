"""The top-M pruning step (spg_topm) against a plain NumPy ordering, bitwise.

The order is score descending, then index ascending, with NaN ranked as -inf
and the float total order (so -0.0 ranks below +0.0).  Sizes cover the
one-workgroup register path (n <= 16384), the multi-workgroup path beyond it,
survivor sets above the LDS sort's 8192 slots (down to M = n - 1, where every
key but one survives and the multi-workgroup front end hands on all of them),
and the degenerate cases where one histogram bin holds most keys (ties, a
single value, -inf)."""
import numpy as np
import pytest
import torch

from paper_2502_02317_amd import spg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _reference(s: np.ndarray, M: int) -> np.ndarray:
    s = np.where(np.isnan(s), -np.inf, s)
    u = s.view(np.uint64)
    sign = np.uint64(1 << 63)
    asc = np.where(u & sign, ~u, u | sign)            # ascending in the score
    order = np.lexsort((np.arange(len(s)), ~asc))     # descending score, then index
    return order[: min(M, len(s))]


def _run(s: np.ndarray, M: int):
    n = len(s)
    Me = min(M, n)
    x = torch.from_numpy(s).to(DEV)
    sel = torch.full((max(Me, 1),), -1, dtype=torch.int32, device=DEV)
    sc = torch.zeros(max(Me, 1), dtype=torch.float64, device=DEV)
    spg.topm(x, M, sel, sc)
    torch.cuda.synchronize()
    return sel.cpu().numpy()[:Me], sc.cpu().numpy()[:Me]


def _scores(kind: str, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.normal(size=n) * 10.0
    if kind == "logp":
        # beam-like: parent scores plus log-probabilities of d = 16 children
        parents = np.sort(rng.normal(size=(n + 15) // 16) * 5.0)[::-1] - 100.0
        lp = np.log(rng.dirichlet(np.full(16, 0.3), size=len(parents)) + 1e-300)
        return (parents[:, None] + lp).ravel()[:n]
    if kind == "ties":
        return rng.integers(-5, 5, size=n).astype(np.float64)
    if kind == "constant":
        return np.full(n, -3.25)
    if kind == "special":
        s = rng.normal(size=n)
        s[rng.random(n) < 0.3] = -np.inf
        s[rng.random(n) < 0.05] = np.nan
        s[rng.random(n) < 0.05] = 0.0
        s[rng.random(n) < 0.05] = -0.0
        return s
    if kind == "tiny_gaps":
        # a dense cluster just below the best score: the boundary bin is crowded
        return -1.0 - rng.random(n) * 1e-12
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["normal", "logp", "ties", "constant", "special", "tiny_gaps"])
@pytest.mark.parametrize("n,M", [(1, 1), (5, 3), (1000, 1000), (1000, 1007), (16384, 1024),
                                 (16384, 1), (16385, 1024), (65536, 4096), (98304, 4096),
                                 (98304, 9000), (200000, 512), (5000, 4999), (16384, 16383),
                                 (16385, 16384), (40000, 39999)])
def test_topm_matches_reference_order(kind, n, M):
    s = _scores(kind, n, seed=n + M)
    sel, sc = _run(s, M)
    ref = _reference(s, M)
    np.testing.assert_array_equal(sel, ref)
    want = np.where(np.isnan(s[ref]), -np.inf, s[ref])
    np.testing.assert_array_equal(sc.view(np.uint64), want.view(np.uint64))


def test_topm_empty_and_errors():
    x = torch.zeros(0, dtype=torch.float64, device=DEV)
    sel = torch.zeros(1, dtype=torch.int32, device=DEV)
    spg.topm(x, 4, sel)                                  # n = 0: nothing to do
    with pytest.raises(spg.SpgError):
        spg.topm(torch.zeros(3, dtype=torch.float64, device=DEV), 0, sel)
