"""Exact row transfer against the oracle's boundary MPS on king's strips with
the workloads' local dimension and temperature (CPU only).

On a strip of cols = 3 every boundary cut has at most d states on one side,
so chi >= d is the exact rank (chi = 16 at d = 16, chi = 64 at d = 24); on
cols = 2 a single cut of d states.  The d = 24, beta = 4 strips (8-spin
clusters, the 24 lowest states) are the ones whose blocks underflowed before
each column's MPO tensor was scaled to a largest entry of 1.  There the boundary MPS represents every row function exactly,
and the branch-and-bound conditionals must equal the exact ones
p(x_k | x_<k) = P(x_<=k) / P(x_<k) (the paper's marginals, Sec. 2, computed
from dense row vectors).  Tolerances: log Z to 1e-10 relative, and every
conditional with p >= 1e-4 max_s p of its parent within 1e-10 in log.  The
bound holds because no cut rotates at the exact rank (natural bases), so each
row function is a sum of products of non-negative factors, each entry
carrying a relative rounding error of at most n u with n the few thousand
operations on its chain (measured: 1e-16 in log Z, 3e-14 in log p).
"""
import numpy as np
import pytest

from workloads import spin_instance, potts_from_spins
from oracle.exact import row_transfer, exact_conditionals
from oracle.bmps import boundary_mps
from oracle.search import beam_search, teacher_forced_logp

STRIPS = [
    # rows, cols, spins per cluster, beta, inter-cluster couplings, d kept, chi
    (4, 3, 4, 2.0, ("pm1", 1.0), None, 16),
    (6, 3, 4, 2.0, ("pm1", 1.0), None, 16),
    (8, 3, 4, 2.0, ("pm1", 1.0), None, 16),
    (12, 2, 8, 4.0, ("normal", 1.0), 24, 64),
    (8, 3, 8, 4.0, ("normal", 1.0), 24, 64),
]


def _strip(rows, cols, t, beta, jout, keep, seed):
    si = spin_instance(rows, cols, t, True, seed, h=("normal", 1.0), j_in=("normal", 1.0),
                       j_out=jout)
    return potts_from_spins(si, beta=beta, d_keep=keep)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("shape", STRIPS, ids=lambda s: f"{s[0]}x{s[1]}_t{s[2]}")
def test_strip_logZ_and_beam_conditionals(shape, seed):
    rows, cols, t, beta, jout, keep, chi = shape
    inst = _strip(rows, cols, t, beta, jout, keep, seed)
    vecs, lz = row_transfer(inst)
    mp = boundary_mps(inst, chi=chi)
    assert abs(mp["logZ"] - lz) <= 1e-10 * abs(lz)
    # the conditionals of every parent the oracle's own beam search visits
    trace = []
    beam_search(inst, mp["A"], 16, trace=trace)
    worst = 0.0
    for step in trace:
        k = step["site"]
        r, c = divmod(k, cols)
        for b in range(step["cfg"].shape[0]):
            pe = exact_conditionals(inst, vecs, list(step["cfg"][b, :k]))
            keep_s = pe >= 1e-4 * pe.max()
            lp = step["logp"][b]
            worst = max(worst, float(np.max(np.abs(lp[keep_s] - np.log(pe[keep_s])))))
    assert worst <= 1e-10, worst


def test_strip_teacher_forced_at_every_site():
    """The same along the exact most probable path, through the teacher-forced
    entry (the one the GPU's marginals are compared with)."""
    inst = _strip(8, 3, 4, 2.0, ("pm1", 1.0), None, 0)
    vecs, _ = row_transfer(inst)
    A = boundary_mps(inst, chi=16)["A"]
    cfg = []
    for k in range(inst.n_sites):
        pe = exact_conditionals(inst, vecs, cfg)
        r, c = divmod(k, inst.cols)
        row = np.zeros((1, inst.n_sites), dtype=np.int64)
        row[0, :k] = cfg
        lp = teacher_forced_logp(inst, A, r, c, row)[0]
        ok = pe >= 1e-4 * pe.max()
        assert np.max(np.abs(lp[ok] - np.log(pe[ok]))) <= 1e-10
        cfg.append(int(np.argmax(pe)))
