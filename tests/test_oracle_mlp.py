"""Pins of the proposal network's reference arithmetic (CPU only)."""
import numpy as np

from workloads import random_potts
from oracle.bmps import boundary_mps
from oracle.mlp import (F, features, init_params, forward, loss_and_grad, adam_step,
                        lookahead, one_site_logw)
from oracle.search import delta_energy


def _data(seed=0):
    inst = random_potts(3, 4, 3, True, seed=4, beta=0.7)
    mp = boundary_mps(inst, 9)
    rng = np.random.default_rng(seed)
    cfg = rng.integers(0, 3, size=(7, inst.n_sites))
    sc = rng.normal(size=7)
    return inst, mp, cfg, sc


def test_gradient_matches_central_differences():
    inst, mp, cfg, sc = _data()
    f = features(inst, mp["A"], 1, 2, cfg, sc)
    rng = np.random.default_rng(3)
    t = rng.normal(size=(7, 3))
    t = t - np.log(np.exp(t).sum(axis=1, keepdims=True))
    H = 5
    p = init_params(H, 11)
    loss, g = loss_and_grad(p, H, f, t)
    eps = 1e-6
    num = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = eps
        num[i] = (loss_and_grad(p + e, H, f, t)[0] - loss_and_grad(p - e, H, f, t)[0]) / (2 * eps)
    np.testing.assert_allclose(g, num, rtol=1e-5, atol=1e-8)


def test_forward_is_log_softmax_and_loss_is_cross_entropy():
    inst, mp, cfg, sc = _data()
    f = features(inst, mp["A"], 2, 0, cfg, sc)
    H = 4
    p = init_params(H, 2)
    lp = forward(p, H, f)
    np.testing.assert_allclose(np.exp(lp).sum(axis=1), 1.0, atol=1e-12)
    t = lp.copy()                      # target = prediction: loss = its entropy
    loss, g = loss_and_grad(p, H, f, t)
    assert abs(loss - float(-(np.exp(lp) * lp).sum() / lp.shape[0])) < 1e-12
    assert np.abs(g).max() < 1e-12     # cross-entropy is stationary at the target


def test_features_from_definitions():
    inst, mp, cfg, sc = _data()
    r, c = 1, 1
    f = features(inst, mp["A"], r, c, cfg, sc)
    assert f.shape == (7, 3, F)
    e = -inst.beta * delta_energy(inst, cfg, r, c)
    np.testing.assert_allclose(f[:, :, 0], np.maximum(e - e.max(1, keepdims=True), -30) / 10)
    # look-ahead by brute force over each neighbour's states
    b = inst.beta
    la = np.zeros(3)
    for s in range(3):
        la[s] += np.log(sum(np.exp(-b * (inst.local_E[r, c + 1][y] + inst.pair_h[r, c][s, y])) for y in range(3)))
        la[s] += np.log(sum(np.exp(-b * (inst.local_E[r + 1, c][y] + inst.pair_v[r, c][s, y])) for y in range(3)))
        la[s] += np.log(sum(np.exp(-b * (inst.local_E[r + 1, c + 1][y] + inst.pair_d[r, c][s, y])) for y in range(3)))
        la[s] += np.log(sum(np.exp(-b * (inst.local_E[r + 1, c - 1][y] + inst.pair_a[r, c - 1][s, y])) for y in range(3)))
    np.testing.assert_allclose(lookahead(inst, r, c, cfg)[0], la, atol=1e-12)
    # one-site weight: the MPS contracted with x_c = s and every other state summed
    A = mp["A"][r]
    T = np.einsum("axb,bsc,cyd,dze->s", A[0], A[1], A[2], A[3])
    lm = one_site_logw(A, 1)
    np.testing.assert_allclose(lm - lm.max(), np.log(T) - np.log(T).max(), atol=1e-10)


def test_adam_matches_definition_on_quadratic():
    p = np.array([1.0, -2.0])
    m = v = np.zeros(2)
    for t in range(1, 2001):
        p, m, v = adam_step(p, 2 * p, m, v, t, lr=0.05)
    assert np.abs(p).max() < 1e-3


# ---- guided search: the guard keeps the plain search's beam ------------------

import pytest

from oracle.proposal import guided_beam_search, candidate_set
from oracle.search import beam_search, log_conditionals, marginals


def _finite_beam(res):
    s = res["beam_scores"]
    ok = np.isfinite(s)
    return res["beam_states"][ok], s[ok]


def _same_beam(a, b):
    sa, pa = _finite_beam(a)
    sb, pb = _finite_beam(b)
    assert len(sa) == len(sb)
    ka = {tuple(x): v for x, v in zip(map(tuple, sa), pa)}
    kb = {tuple(x): v for x, v in zip(map(tuple, sb), pb)}
    assert ka.keys() == kb.keys()
    for k in ka:
        assert abs(ka[k] - kb[k]) <= 1e-10


@pytest.mark.parametrize("kappa,seed,M,cut", [(2.0, 1, 12, 0.0), (1.0, 2, 20, 0.0),
                                              (0.5, 3, 9, 0.0), (2.0, 4, 16, 1e-3)])
def test_guided_search_keeps_plain_beam_with_any_network(kappa, seed, M, cut):
    """Random (untrained) networks, several kappa: the guard must restore the
    plain search's finite beam."""
    inst = random_potts(3, 4, 3, True, seed=seed, beta=1.3)
    mp = boundary_mps(inst, 6)
    H = 8
    p = init_params(H, seed)
    st = {}
    g = guided_beam_search(inst, mp["A"], M, p, H, kappa=kappa, cut_off_prob=cut, stats=st)
    e = beam_search(inst, mp["A"], M, cut_off_prob=cut)
    _same_beam(g, e)
    assert st["exact"] <= st["candidates"] + st["fallback"] * inst.d


def test_perfect_network_saves_exact_evaluations():
    """A network whose logits are the exact log-conditionals needs few exact
    evaluations; the planted-mistake case (logits reversed) falls back often but
    keeps the beam."""
    import oracle.proposal as P
    inst = random_potts(3, 4, 4, True, seed=7, beta=1.5)
    mp = boundary_mps(inst, 8)
    M = 24
    e = beam_search(inst, mp["A"], M)

    real_forward = P.forward

    def run(sign):
        # stand-in network: rank children by -beta dE (feature 0); sign -1
        # reverses the ranking (the planted mistake)
        P.forward = lambda prm, H, f: sign * f[:, :, 0] * 10.0
        try:
            st = {}
            g = guided_beam_search(inst, mp["A"], M, None, 0, kappa=2.0, stats=st)
        finally:
            P.forward = real_forward
        return g, st

    g1, s1 = run(+1.0)
    g2, s2 = run(-1.0)
    _same_beam(g1, e)
    _same_beam(g2, e)
    assert s1["exact"] < s2["exact"]
    assert s1["exact"] < 0.8 * s1["candidates"]


def test_candidate_set_counts():
    pred = np.array([[0.0, -0.01, -1.0], [-0.5, -np.inf, -40.0]])
    E = candidate_set(pred, 0.0, 2)
    assert E.tolist() == [[True, True, False], [False, False, False]]
    E = candidate_set(pred, 0.0, 5)          # only reachable through the last bin
    assert E.all()
