"""Pins of the oracle's exact parts against closed forms, a hand-computed
fixture and brute force (CPU only)."""
import os

import numpy as np
import pytest
from scipy.special import logsumexp

from workloads import (PottsInstance, random_potts, spin_instance, potts_from_spins,
                       config_instance)
from oracle.energy import potts_energy, ising_energy
from oracle.exact import brute_force, row_transfer, exact_conditionals, prefix_logp
from oracle.bmps import boundary_mps
from oracle.search import teacher_forced_logp
from lattice_util import transform

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    vals = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_golden_chain_1x2():
    """Hand-computed Z of a two-site chain (tests/golden/chain_1x2_d2.txt)."""
    g = _read_golden("chain_1x2_d2.txt")
    inst = PottsInstance(1, 2, 2, False, np.array([[[0.0, 1.0], [0.5, 0.0]]]),
                         np.array([[[[-1.0, 1.0], [1.0, -1.0]]]]), np.zeros((0, 2, 2, 2)),
                         beta=1.0)
    bf = brute_force(inst)
    assert abs(bf["logZ"] - g["logZ"]) < 1e-14
    assert bf["E_min"] == g["E_min"]
    assert abs(np.exp(bf["prefix_logp"][0][0]) - g["p_x0_0"]) < 1e-14
    _, lz = row_transfer(inst)
    assert abs(lz - g["logZ"]) < 1e-14
    assert abs(boundary_mps(inst, chi=4)["logZ"] - g["logZ"]) < 1e-13


@pytest.mark.parametrize("kings,t,keep", [(False, 1, None), (True, 2, None), (True, 3, 5)])
def test_potts_tables_match_ising_energy(kings, t, keep):
    """Eq. (1) from the cluster tables equals Eq. (2) on the spins."""
    si = spin_instance(3, 3, t, kings, seed=7, h=("normal", 1.0), j_in=("normal", 1.0),
                       j_out=("normal", 1.0))
    inst = potts_from_spins(si, beta=1.0, d_keep=keep)
    rng = np.random.default_rng(0)
    X = rng.integers(0, inst.d, size=(50, inst.n_sites))
    kept = inst.meta["keep"]                                  # [R][C][d] full-state ids
    full = kept[np.arange(3)[None, :, None], np.arange(3)[None, None, :], X.reshape(50, 3, 3)]
    S = 2.0 * ((full[..., None] >> np.arange(t)) & 1) - 1.0
    np.testing.assert_allclose(potts_energy(inst, X), ising_energy(si, S), atol=1e-12)


def test_truncated_spectrum_keeps_lowest_states():
    si = spin_instance(2, 2, 3, True, seed=3)
    full = potts_from_spins(si, beta=1.0)
    part = potts_from_spins(si, beta=1.0, d_keep=4)
    for r in range(2):
        for c in range(2):
            np.testing.assert_allclose(part.local_E[r, c], np.sort(full.local_E[r, c])[:4])


def test_beta_zero_uniform():
    """beta = 0: Z = d^N and every conditional is 1/d."""
    inst = random_potts(2, 3, 3, True, seed=1, beta=0.0)
    bf = brute_force(inst)
    assert abs(bf["logZ"] - inst.n_sites * np.log(3)) < 1e-12
    mp = boundary_mps(inst, chi=16)
    assert abs(mp["logZ"] - inst.n_sites * np.log(3)) < 1e-12
    cfg = np.array([[0, 2, 1, 1, 0, 2]])
    lp = teacher_forced_logp(inst, mp["A"], 1, 1, cfg)
    np.testing.assert_allclose(lp, np.log(1 / 3), atol=1e-12)


def test_no_couplings_product_measure():
    """All pair energies zero: Z = prod_n sum_x exp(-beta E_n(x)) and
    p(x_k | x_<k) = softmax(-beta E_k)."""
    inst = random_potts(3, 3, 3, True, seed=2, beta=0.8)
    for T in (inst.pair_h, inst.pair_v, inst.pair_d, inst.pair_a):
        T[...] = 0.0
    expect = float(np.sum(logsumexp(-0.8 * inst.local_E, axis=2)))
    assert abs(brute_force(inst)["logZ"] - expect) < 1e-12
    mp = boundary_mps(inst, chi=8)
    assert abs(mp["logZ"] - expect) < 1e-12
    cfg = np.array([[1, 0, 2, 2, 1, 0, 0, 0, 0]])
    lp = teacher_forced_logp(inst, mp["A"], 1, 2, cfg)[0]
    np.testing.assert_allclose(lp, -0.8 * inst.local_E[1, 2] - logsumexp(-0.8 * inst.local_E[1, 2]),
                               atol=1e-12)


def _chain_logZ(w_list, M_list):
    """Textbook open-chain transfer matrices: Z = w_0^T M_0 diag(w_1) M_1 ... w_last."""
    v = w_list[0]
    for M, w in zip(M_list, w_list[1:]):
        v = (v @ M) * w
    return float(np.log(v.sum()))


def test_single_row_is_1d_chain():
    inst = random_potts(1, 5, 3, False, seed=4, beta=1.3)
    b = inst.beta
    w = [np.exp(-b * inst.local_E[0, c]) for c in range(5)]
    M = [np.exp(-b * inst.pair_h[0, c]) for c in range(4)]
    expect = _chain_logZ(w, M)
    assert abs(brute_force(inst)["logZ"] - expect) < 1e-12
    assert abs(row_transfer(inst)[1] - expect) < 1e-12
    assert abs(boundary_mps(inst, chi=16)["logZ"] - expect) < 1e-12


def test_vertical_edges_only_independent_columns():
    """Only V edges: the lattice is independent vertical chains, exact at chi = 1."""
    inst = random_potts(4, 3, 3, False, seed=5, beta=0.9)
    inst.pair_h[...] = 0.0
    b = inst.beta
    expect = 0.0
    for c in range(3):
        w = [np.exp(-b * inst.local_E[r, c]) for r in range(4)]
        M = [np.exp(-b * inst.pair_v[r, c]) for r in range(3)]
        expect += _chain_logZ(w, M)
    assert abs(brute_force(inst)["logZ"] - expect) < 1e-12
    assert abs(boundary_mps(inst, chi=1)["logZ"] - expect) < 1e-12


SHAPES = [(2, 2, 2, True), (2, 3, 3, False), (3, 3, 2, True), (3, 3, 3, True), (2, 4, 2, True),
          (3, 4, 2, False), (4, 4, 2, True), (3, 3, 4, True)]


@pytest.mark.parametrize("R,C,d,kings", SHAPES)
def test_row_transfer_and_bmps_match_brute_force(R, C, d, kings):
    inst = random_potts(R, C, d, kings, seed=11 + R * 7 + C, beta=0.9)
    bf = brute_force(inst)
    rows, lz = row_transfer(inst)
    assert abs(lz - bf["logZ"]) < 1e-11
    chi = d ** (C // 2)                                          # >= every exact Schmidt rank
    mp = boundary_mps(inst, chi=chi)
    assert abs(mp["logZ"] - bf["logZ"]) < 1e-10
    # conditionals at every prefix of three configurations
    rng = np.random.default_rng(R * 100 + C)
    for x in list(rng.integers(0, d, size=(2, R * C))) + [bf["argmin"]]:
        for k in range(R * C):
            r, c = divmod(k, C)
            lp_mps = teacher_forced_logp(inst, mp["A"], r, c, x[None])[0]
            ex = exact_conditionals(inst, rows, list(x[:k]))
            np.testing.assert_allclose(lp_mps, np.log(ex), atol=1e-9)
            # brute force: p(x_k | x_<k) = P(x_<=k) / P(x_<k)
            for s in range(d):
                pre = list(x[:k]) + [s]
                lp_bf = prefix_logp(bf, pre) - (prefix_logp(bf, list(x[:k])) if k else 0.0)
                assert abs(lp_bf - lp_mps[s]) < 1e-9


@pytest.mark.parametrize("k", range(8))
def test_lattice_transforms_preserve_Z(k):
    """The eight lattice transformations give the same Z and ground energy."""
    inst = random_potts(2, 3, 3, True, seed=21, beta=0.7)
    bf0 = brute_force(inst)
    ti = transform(inst, k)
    bf = brute_force(ti)
    assert abs(bf["logZ"] - bf0["logZ"]) < 1e-11
    assert abs(bf["E_min"] - bf0["E_min"]) < 1e-12
    chi = ti.d ** (ti.cols // 2)
    assert abs(boundary_mps(ti, chi=chi)["logZ"] - bf0["logZ"]) < 1e-10


def test_config1_exact():
    """4x4 square lattice, d=2: chi=16 is exact."""
    inst = config_instance("square4x4_d2", 0)
    bf = brute_force(inst)
    assert abs(boundary_mps(inst, chi=16)["logZ"] - bf["logZ"]) < 1e-11
