"""Seeded synthetic inputs for the PEPS branch-and-bound hot path.

This module only *generates* problem instances.  It is shared by the oracle,
the tests and the benchmark, and it contains none of the search or contraction
arithmetic.  An instance is a generalized Potts model on a square lattice of
clusters (paper, Sec. 2, Eq. (1)), optionally with both diagonals (the king's
graph, Fig. 1(b)).  When the instance comes from spins, each cluster of ``t``
Ising spins (Eq. (2)) becomes one Potts variable with ``2**t`` states; the
energy tables are the cluster sums of Eq. (2) written in the Potts form of
Eq. (1).

Conventions (fixed here, used by every consumer):

* sites are ``(r, c)`` with ``0 <= r < rows``, ``0 <= c < cols``;
* spin ``i`` of a cluster in state ``x`` is ``s_i(x) = 2*bit_i(x) - 1``;
* edge classes: ``H[r][c]`` joins (r,c)-(r,c+1), ``V[r][c]`` joins (r,c)-(r+1,c),
  ``D[r][c]`` joins (r,c)-(r+1,c+1), ``A[r][c]`` joins (r,c+1)-(r+1,c); a pair table
  is indexed ``[state of the first site][state of the second site]``;
* random draws use ``numpy.random.Generator(PCG64(seed))`` in this order:
  per site row-major the fields ``h_i`` then the intra-cluster ``J_ij`` (i<j),
  then per edge class H, V, D, A (each row-major) the ``t x t`` inter-cluster
  couplings, row-major over the spin pairs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

__all__ = [
    "PottsInstance", "SpinInstance", "spin_instance", "potts_from_spins",
    "random_potts", "config_instance", "CONFIGS", "ConfigSpec", "synthetic_env",
]


@dataclass
class PottsInstance:
    """Energy tables of Eq. (1) on a rows x cols cluster lattice (float64)."""
    rows: int
    cols: int
    d: int
    kings: bool
    local_E: np.ndarray                  # [rows][cols][d]
    pair_h: np.ndarray                   # [rows][cols-1][d][d]
    pair_v: np.ndarray                   # [rows-1][cols][d][d]
    pair_d: Optional[np.ndarray] = None  # [rows-1][cols-1][d][d] (kings only)
    pair_a: Optional[np.ndarray] = None  # [rows-1][cols-1][d][d] (kings only)
    beta: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def n_sites(self) -> int:
        return self.rows * self.cols

    def tables(self):
        """The five tables, with zero-size arrays where an edge class is absent."""
        R, C, d = self.rows, self.cols, self.d
        z = np.zeros((max(R - 1, 0), max(C - 1, 0), d, d))
        return (self.local_E, self.pair_h, self.pair_v,
                self.pair_d if self.kings else z, self.pair_a if self.kings else z)


@dataclass
class SpinInstance:
    """Ising couplings of Eq. (2) grouped into t-spin clusters."""
    rows: int
    cols: int
    t: int
    kings: bool
    h: np.ndarray        # [rows][cols][t]
    J_in: np.ndarray     # [rows][cols][t][t], upper triangle used
    J_h: np.ndarray      # [rows][cols-1][t][t]  J between spin i of (r,c), spin j of (r,c+1)
    J_v: np.ndarray      # [rows-1][cols][t][t]
    J_d: Optional[np.ndarray]
    J_a: Optional[np.ndarray]  # spin i of (r,c+1), spin j of (r+1,c)


def _draw(rng, kind: str, scale: float, size):
    if kind == "normal":
        return rng.normal(0.0, scale, size=size)
    if kind == "pm1":
        return rng.choice(np.array([-1.0, 1.0]), size=size) * scale
    if kind == "zero":
        return np.zeros(size)
    raise ValueError(kind)


def spin_instance(rows: int, cols: int, t: int, kings: bool, seed: int,
                  h: tuple = ("normal", 1.0), j_in: tuple = ("normal", 1.0),
                  j_out: tuple = ("pm1", 1.0)) -> SpinInstance:
    """Draw a clustered Ising instance in the documented order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H = np.zeros((rows, cols, t))
    Jin = np.zeros((rows, cols, t, t))
    iu = np.triu_indices(t, 1)
    for r in range(rows):
        for c in range(cols):
            H[r, c] = _draw(rng, h[0], h[1], t)
            if t > 1:
                Jin[r, c][iu] = _draw(rng, j_in[0], j_in[1], len(iu[0]))

    def block(nr, nc):
        out = np.zeros((max(nr, 0), max(nc, 0), t, t))
        for r in range(nr):
            for c in range(nc):
                out[r, c] = _draw(rng, j_out[0], j_out[1], t * t).reshape(t, t)
        return out

    Jh = block(rows, cols - 1)
    Jv = block(rows - 1, cols)
    Jd = block(rows - 1, cols - 1) if kings else None
    Ja = block(rows - 1, cols - 1) if kings else None
    return SpinInstance(rows, cols, t, kings, H, Jin, Jh, Jv, Jd, Ja)


def _spins(t: int) -> np.ndarray:
    """[2**t][t] matrix of s_i(x) = 2*bit_i(x) - 1."""
    x = np.arange(2 ** t)[:, None]
    return 2.0 * ((x >> np.arange(t)[None, :]) & 1) - 1.0


def potts_from_spins(si: SpinInstance, beta: float, d_keep: Optional[int] = None,
                     meta: Optional[dict] = None) -> PottsInstance:
    """Cluster energy tables: E_n(x) = sum_{i<j} J s_i s_j + sum h s_i and
    E_mn(x, y) = s(x)^T J s(y).  With ``d_keep`` only the ``d_keep`` lowest local
    states of every cluster are kept (stable in the state index) and the pair
    tables are restricted to them; ``meta['keep']`` records the kept states."""
    t = si.t
    S = _spins(t)                                   # [2^t][t]
    R, C = si.rows, si.cols
    full = 2 ** t
    loc = np.einsum("xi,rci->rcx", S, si.h)
    Jin = np.triu(si.J_in, 1)
    loc = loc + np.einsum("xi,rcij,xj->rcx", S, Jin, S)
    keep = np.tile(np.arange(full), (R, C, 1))
    if d_keep is not None and d_keep < full:
        keep = np.argsort(loc, axis=2, kind="stable")[:, :, :d_keep]
    d = keep.shape[2]
    local_E = np.take_along_axis(loc, keep, axis=2)

    def pair(J, k1, k2):
        out = np.zeros(J.shape[:2] + (d, d))
        for r in range(J.shape[0]):
            for c in range(J.shape[1]):
                full_t = S @ J[r, c] @ S.T
                a, b = k1(r, c), k2(r, c)
                out[r, c] = full_t[np.ix_(keep[a], keep[b])]
        return out

    ph = pair(si.J_h, lambda r, c: (r, c), lambda r, c: (r, c + 1))
    pv = pair(si.J_v, lambda r, c: (r, c), lambda r, c: (r + 1, c))
    pd = pa = None
    if si.kings:
        pd = pair(si.J_d, lambda r, c: (r, c), lambda r, c: (r + 1, c + 1))
        pa = pair(si.J_a, lambda r, c: (r, c + 1), lambda r, c: (r + 1, c))
    m = dict(meta or {})
    m["keep"] = keep
    m["t"] = t
    return PottsInstance(R, C, d, si.kings, local_E, ph, pv, pd, pa, beta, m)


def random_potts(rows: int, cols: int, d: int, kings: bool, seed: int,
                 beta: float = 1.0, scale: float = 1.0,
                 local_scale: Optional[float] = None) -> PottsInstance:
    """Potts instance with i.i.d. Gaussian table entries (no spin structure);
    used for small brute-force cases with d not a power of two."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ls = scale if local_scale is None else local_scale
    loc = rng.normal(0, ls, (rows, cols, d))
    ph = rng.normal(0, scale, (rows, cols - 1, d, d))
    pv = rng.normal(0, scale, (rows - 1, cols, d, d))
    pd = pa = None
    if kings:
        pd = rng.normal(0, scale, (rows - 1, cols - 1, d, d))
        pa = rng.normal(0, scale, (rows - 1, cols - 1, d, d))
    return PottsInstance(rows, cols, d, kings, loc, ph, pv, pd, pa, beta,
                         {"kind": "gaussian", "seed": seed})


@dataclass
class ConfigSpec:
    name: str
    make: Callable[[int], PottsInstance]
    chi: int
    max_states: int
    num_sweeps: int = 1


def _cfg1(seed: int) -> PottsInstance:
    si = spin_instance(4, 4, 1, False, seed, h=("normal", 0.1), j_in=("zero", 0),
                       j_out=("pm1", 1.0))
    return potts_from_spins(si, beta=1.0, meta={"config": "square4x4_d2"})


def _cfg2(seed: int) -> PottsInstance:
    si = spin_instance(8, 8, 4, True, seed, h=("normal", 1.0), j_in=("normal", 1.0),
                       j_out=("pm1", 1.0))
    return potts_from_spins(si, beta=2.0, meta={"config": "kings8x8_d16"})


def cfg3_shapes(n: int = 256, seed: int = 999):
    """Lattice sides and bond dimensions of the batched workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = rng.integers(6, 13, size=n)
    chi = rng.choice(np.array([16, 32]), size=n)
    return L, chi


def cfg3_instance(i: int, L: int) -> PottsInstance:
    si = spin_instance(L, L, 4, True, 1000 + i, h=("normal", 1.0),
                       j_in=("normal", 1.0), j_out=("normal", 1.0))
    return potts_from_spins(si, beta=2.0, meta={"config": f"kings{L}x{L}_d16"})


def _cfg4(seed: int) -> PottsInstance:
    si = spin_instance(12, 12, 8, True, seed, h=("normal", 1.0), j_in=("normal", 1.0),
                       j_out=("normal", 1.0))
    return potts_from_spins(si, beta=4.0, d_keep=24, meta={"config": "kings12x12_d24"})


def _cfg5(seed: int) -> PottsInstance:
    si = spin_instance(16, 16, 8, True, seed, h=("normal", 0.1), j_in=("pm1", 1.0),
                       j_out=("pm1", 1.0))
    return potts_from_spins(si, beta=4.0, meta={"config": "kings16x16_d256"})


CONFIGS = {
    "square4x4_d2": ConfigSpec("square4x4_d2", _cfg1, chi=16, max_states=64),
    "kings8x8_d16": ConfigSpec("kings8x8_d16", _cfg2, chi=32, max_states=1024),
    "kings12x12_d24": ConfigSpec("kings12x12_d24", _cfg4, chi=64, max_states=4096),
    "kings16x16_d256": ConfigSpec("kings16x16_d256", _cfg5, chi=64, max_states=10000),
}


def config_instance(name: str, seed: int) -> PottsInstance:
    return CONFIGS[name].make(seed)


def synthetic_env(rows: int, cols: int, d: int, chi: int, seed: int):
    """A seeded stand-in for a boundary-MPS environment: for each row, ``cols``
    tensors [D_c][d][D_{c+1}] with entries uniform in [0, 1) and the bond
    dimensions a contraction at bond cap ``chi`` has, D_c = min(chi, d**c,
    d**(cols-c)).  Positive entries make every conditional a sum of positive
    terms.  Drawn row by row, column by column, from PCG64(seed)."""
    rng = np.random.default_rng(seed)
    dims = [min(chi, d ** c, d ** (cols - c)) for c in range(cols + 1)]
    return [[rng.random((dims[c], d, dims[c + 1])) for c in range(cols)] for _ in range(rows)]
