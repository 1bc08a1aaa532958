"""Test helper: the 8 rotations/reflections of the cluster grid (the paper's
"all_lattice_transformations", Sec. 3.1), applied to a Potts instance.

An instance is turned into a plain edge list, site coordinates are mapped, and
each edge is re-filed under the class its new geometry gives it, with its
table transposed when the endpoints swap order."""
import numpy as np

from workloads import PottsInstance


def _edge_list(inst):
    R, C = inst.rows, inst.cols
    E = {}
    for r in range(R):
        for c in range(C - 1):
            E[((r, c), (r, c + 1))] = inst.pair_h[r, c]
    for r in range(R - 1):
        for c in range(C):
            E[((r, c), (r + 1, c))] = inst.pair_v[r, c]
        if inst.kings:
            for c in range(C - 1):
                E[((r, c), (r + 1, c + 1))] = inst.pair_d[r, c]
                E[((r, c + 1), (r + 1, c))] = inst.pair_a[r, c]
    return E


def transform(inst, k: int):
    """k in 0..7: k % 4 quarter turns, then a transpose if k >= 4."""
    R, C = inst.rows, inst.cols

    def f(p):
        r, c = p
        rr, cc, RR, CC = r, c, R, C
        for _ in range(k % 4):
            rr, cc, RR, CC = cc, RR - 1 - rr, CC, RR
        if k >= 4:
            rr, cc, RR, CC = cc, rr, CC, RR
        return (rr, cc), (RR, CC)

    (_, (NR, NC)) = f((0, 0))
    d = inst.d
    loc = np.zeros((NR, NC, d))
    for r in range(R):
        for c in range(C):
            (rr, cc), _ = f((r, c))
            loc[rr, cc] = inst.local_E[r, c]
    ph = np.zeros((NR, NC - 1, d, d))
    pv = np.zeros((NR - 1, NC, d, d))
    pd = np.zeros((NR - 1, NC - 1, d, d))
    pa = np.zeros((NR - 1, NC - 1, d, d))
    for (p, q), T in _edge_list(inst).items():
        (a, _), (b, _) = f(p), f(q)
        if a > b:                                   # order endpoints top-left first
            a, b, T = b, a, T.T
        (r1, c1), (r2, c2) = a, b
        if r1 == r2:
            ph[r1, c1] = T
        elif c1 == c2:
            pv[r1, c1] = T
        elif c2 == c1 + 1:
            pd[r1, c1] = T
        else:                                       # (r, c+1)-(r+1, c)
            pa[r1, c2] = T
    return PottsInstance(NR, NC, d, inst.kings, loc, ph, pv,
                         pd if inst.kings else None, pa if inst.kings else None,
                         inst.beta, dict(inst.meta))
