"""The closed form that the large-d GPU tests compare with, pinned on the CPU.

With every coupling between rows zero (the V, D and A tables), the Boltzmann
weight of Eq. (1) factorises over rows: Z is the product of the rows' own
partition functions, each a sum over the row's states of exp(-beta E_r) with
E_r the row's local and horizontal energies.  Checked against brute-force
enumeration of every configuration on small lattices (square and king's)."""
import numpy as np
import pytest

from workloads import random_potts
from oracle.exact import brute_force


def row_energy(inst, r):
    """E_r(x_0, ..., x_{C-1}) of row r alone (local and horizontal terms), dense,
    x_0 slowest."""
    C, d = inst.cols, inst.d
    E = np.zeros((d,) * C)
    for c in range(C):
        shp = [1] * C
        shp[c] = d
        E = E + inst.local_E[r, c].reshape(shp)
    for c in range(C - 1):
        shp = [1] * C
        shp[c] = shp[c + 1] = d
        E = E + inst.pair_h[r, c].reshape(shp)
    return E.ravel()


def decoupled_log_z(inst):
    """log Z of an instance whose rows do not interact: the sum over rows of
    log sum_x exp(-beta E_r(x)); and the rows' log weights."""
    lw = [-inst.beta * row_energy(inst, r) for r in range(inst.rows)]
    return sum(v.max() + np.log(np.exp(v - v.max()).sum()) for v in lw), lw


@pytest.mark.parametrize("shape", [(2, 3, 3, True), (3, 2, 4, False), (2, 2, 5, True)])
def test_decoupled_log_z_equals_brute_force(shape):
    R, C, d, kings = shape
    inst = random_potts(R, C, d, kings, seed=31 + d, beta=0.7)
    inst.pair_v[:] = 0.0
    if kings:
        inst.pair_d[:] = 0.0
        inst.pair_a[:] = 0.0
    lz, _ = decoupled_log_z(inst)
    bf = brute_force(inst)
    ref = bf["logZ"] if isinstance(bf, dict) else bf
    assert abs(lz - ref) <= 1e-12 * abs(ref)


def test_decoupled_log_z_sees_a_vertical_coupling():
    # the closed form ignores vertical tables, so it must fail once one is set
    inst = random_potts(2, 2, 3, False, seed=5, beta=0.7)
    inst.pair_v[:] = 0.0
    inst.pair_v[0, 0, 1, 2] = 1.5
    lz, _ = decoupled_log_z(inst)
    bf = brute_force(inst)
    ref = bf["logZ"] if isinstance(bf, dict) else bf
    assert abs(lz - ref) > 1e-6
