"""Ising input clustered into Potts tables (spg_ising_to_potts, host code).

Pinned two ways: the tables equal those of workloads.potts_from_spins for the
same clustered instance, and for random spin configurations the Ising energy
sum_q J_q s_i s_j (fields on the diagonal) equals the Eq. (1) energy of the
cluster states (oracle.energy.potts_energy), which fixes every table entry
and orientation.  Also: the 1-based text reader, and the error cases."""
import numpy as np
import pytest

from workloads import spin_instance, potts_from_spins
from oracle.energy import potts_energy
from paper_2502_02317_amd import spg


def _terms(si):
    """Term list (i, j, J) of a clustered instance, spin k of cluster (r, c)
    numbered (r * cols + c) * t + k."""
    R, C, t = si.rows, si.cols, si.t
    sid = lambda r, c, k: (r * C + c) * t + k
    out = []
    for r in range(R):
        for c in range(C):
            for k in range(t):
                out.append((sid(r, c, k), sid(r, c, k), si.h[r, c, k]))
                for k2 in range(k + 1, t):
                    out.append((sid(r, c, k), sid(r, c, k2), si.J_in[r, c, k, k2]))
    def block(J, a, b):
        for r in range(J.shape[0]):
            for c in range(J.shape[1]):
                (ra, ca), (rb, cb) = a(r, c), b(r, c)
                for k1 in range(t):
                    for k2 in range(t):
                        out.append((sid(ra, ca, k1), sid(rb, cb, k2), J[r, c, k1, k2]))
    block(si.J_h, lambda r, c: (r, c), lambda r, c: (r, c + 1))
    block(si.J_v, lambda r, c: (r, c), lambda r, c: (r + 1, c))
    if si.kings:
        block(si.J_d, lambda r, c: (r, c), lambda r, c: (r + 1, c + 1))
        block(si.J_a, lambda r, c: (r, c + 1), lambda r, c: (r + 1, c))
    i, j, J = (np.array(x) for x in zip(*out))
    return i.astype(np.int32), j.astype(np.int32), J.astype(np.float64)



@pytest.mark.parametrize("R,C,t,kings", [(3, 4, 2, False), (3, 3, 3, True), (2, 3, 4, True)])
def test_tables_match_clustering_and_ising_energy(R, C, t, kings):
    si = spin_instance(R, C, t, kings, seed=R * 5 + C + t, h=("normal", 1.0),
                       j_in=("normal", 1.0), j_out=("normal", 0.7))
    ref = potts_from_spins(si, beta=1.0)
    i, j, J = _terms(si)
    n = R * C * t
    # shuffle and flip some pairs: the order and orientation of terms are free
    rng = np.random.default_rng(1)
    p = rng.permutation(len(i))
    i, j, J = i[p], j[p], J[p]
    flip = rng.random(len(i)) < 0.5
    i, j = np.where(flip, j, i), np.where(flip, i, j)
    got = spg.ising_to_potts(n, i, j, J, R, C, t, kings)
    np.testing.assert_allclose(got.local_E, ref.local_E, atol=1e-12)
    np.testing.assert_allclose(got.pair_h, ref.pair_h, atol=1e-12)
    np.testing.assert_allclose(got.pair_v, ref.pair_v, atol=1e-12)
    if kings:
        np.testing.assert_allclose(got.pair_d, ref.pair_d, atol=1e-12)
        np.testing.assert_allclose(got.pair_a, ref.pair_a, atol=1e-12)
    # Ising energy = Eq. (1) energy of the cluster states
    s = rng.choice([-1.0, 1.0], size=(300, n))
    e_ising = np.where(i == j, J[None, :] * s[:, i], J[None, :] * s[:, i] * s[:, j]).sum(axis=1)
    bits = ((s + 1) / 2).astype(np.int64).reshape(300, R * C, t)
    x = (bits << np.arange(t)[None, None, :]).sum(axis=2)
    np.testing.assert_allclose(potts_energy(got, x), e_ising, atol=1e-10)


def test_text_reader_round_trip(tmp_path):
    si = spin_instance(2, 3, 2, True, seed=4)
    i, j, J = _terms(si)
    f = tmp_path / "inst.txt"
    with open(f, "w") as h:
        h.write("# 12 spins on a 2 x 3 king's lattice of 2-spin clusters\n")
        for a, b, v in zip(i, j, J):
            h.write(f"{a + 1} {b + 1} {float(v)!r}\n")
        h.write(f"{i[0] + 1} {j[0] + 1} 0.0   # repeated term, adds nothing\n")
    n, ri, rj, rJ = spg.read_ising(str(f))
    assert n == 12
    got = spg.ising_to_potts(n, ri, rj, rJ, 2, 3, 2, True)
    ref = spg.ising_to_potts(12, i, j, J, 2, 3, 2, True)
    for a, b in zip(got.tables(), ref.tables()):
        np.testing.assert_array_equal(a, b)


def test_errors():
    n = 2 * 3 * 2
    with pytest.raises(spg.SpgError) as e:      # (0,0)-(1,2) are not neighbours
        spg.ising_to_potts(n, [0], [11], [1.0], 2, 3, 2, True)
    assert e.value.code == -1
    with pytest.raises(spg.SpgError) as e:      # diagonal coupling without kings
        spg.ising_to_potts(n, [0], [8], [1.0], 2, 3, 2, False)
    assert e.value.code == -1
    with pytest.raises(spg.SpgError) as e:
        spg.ising_to_potts(n, [0], [1], [1.0], 2, 3, 3, True)     # 12 != 2*3*3
    assert e.value.code == -1
    with pytest.raises(spg.SpgError) as e:
        spg.ising_to_potts(2 * 2 * 9, [0], [1], [1.0], 2, 2, 9, True)
    assert e.value.code == -5
    with pytest.raises(spg.SpgError) as e:
        spg.ising_to_potts(n, [0], [1], [float("nan")], 2, 3, 2, True)
    assert e.value.code == -4
