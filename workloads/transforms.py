"""The eight symmetries of the cluster grid (quarter turns, then an optional
transpose) applied to an instance's tables, for running the search on every
orientation of one lattice (the paper's all-lattice-transformations driver,
Sec. 3.1).  Pure relabelling of inputs: no arithmetic of the method."""
from __future__ import annotations

import numpy as np

from . import PottsInstance


def _site_map(R: int, C: int, k: int):
    """(new shape, new coordinate of every old site) for symmetry k in 0..7."""
    r, c = np.meshgrid(np.arange(R), np.arange(C), indexing="ij")
    RR, CC = R, C
    for _ in range(k % 4):                      # quarter turn: (r, c) -> (c, RR - 1 - r)
        r, c, RR, CC = c, RR - 1 - r, CC, RR
    if k >= 4:
        r, c, RR, CC = c, r, CC, RR
    return (RR, CC), r, c


def lattice_transform(inst, k: int):
    """Instance on the grid turned by symmetry k, and ``back`` with
    back[new_site] = old_site, so x_old[back] = x_new maps a state back."""
    R, C, d = inst.rows, inst.cols, inst.d
    (NR, NC), nr, nc = _site_map(R, C, k)
    back = np.empty(NR * NC, dtype=np.int64)
    back[(nr * NC + nc).ravel()] = np.arange(R * C)
    loc = np.zeros((NR, NC, d))
    loc[nr, nc] = inst.local_E
    ph = np.zeros((NR, max(NC - 1, 0), d, d))
    pv = np.zeros((max(NR - 1, 0), NC, d, d))
    pd = np.zeros((max(NR - 1, 0), max(NC - 1, 0), d, d))
    pa = np.zeros_like(pd)

    def put(p, q, T):
        (r1, c1), (r2, c2) = p, q
        if (r1, c1) > (r2, c2):                  # top-left endpoint first
            (r1, c1), (r2, c2), T = (r2, c2), (r1, c1), T.T
        if r1 == r2:
            ph[r1, c1] = T
        elif c1 == c2:
            pv[r1, c1] = T
        elif c2 == c1 + 1:
            pd[r1, c1] = T
        else:
            pa[r1, c2] = T

    def new(r, c):
        return int(nr[r, c]), int(nc[r, c])

    for r in range(R):
        for c in range(C - 1):
            put(new(r, c), new(r, c + 1), inst.pair_h[r, c])
    for r in range(R - 1):
        for c in range(C):
            put(new(r, c), new(r + 1, c), inst.pair_v[r, c])
        if inst.kings:
            for c in range(C - 1):
                put(new(r, c), new(r + 1, c + 1), inst.pair_d[r, c])
                put(new(r, c + 1), new(r + 1, c), inst.pair_a[r, c])
    meta = dict(inst.meta)
    meta["transform"] = k
    out = PottsInstance(NR, NC, d, inst.kings, loc, ph, pv, pd if inst.kings else None,
                        pa if inst.kings else None, inst.beta, meta)
    return out, back
