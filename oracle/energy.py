"""Energies and Boltzmann weights (oracle; test infrastructure only).

Pinned by: Eq. (1) evaluated from the cluster tables equals Eq. (2) evaluated
directly on the spins (tests/test_oracle_exact.py), and by the closed forms of
``exact``.
"""
from __future__ import annotations

import numpy as np


def potts_energy(inst, X: np.ndarray) -> np.ndarray:
    """Eq. (1): E(x) = sum over edges E_mn(x_m, x_n) + sum over sites E_n(x_n).

    ``X`` is [n_cfg][rows*cols] (row-major sites); returns [n_cfg] float64."""
    X = np.asarray(X)
    R, C = inst.rows, inst.cols
    G = X.reshape(-1, R, C)
    rr, cc = np.meshgrid(np.arange(R), np.arange(C), indexing="ij")
    E = inst.local_E[rr[None], cc[None], G].sum(axis=(1, 2))
    if C > 1:
        r, c = np.meshgrid(np.arange(R), np.arange(C - 1), indexing="ij")
        E = E + inst.pair_h[r[None], c[None], G[:, :, :-1], G[:, :, 1:]].sum(axis=(1, 2))
    if R > 1:
        r, c = np.meshgrid(np.arange(R - 1), np.arange(C), indexing="ij")
        E = E + inst.pair_v[r[None], c[None], G[:, :-1, :], G[:, 1:, :]].sum(axis=(1, 2))
        if inst.kings and C > 1:
            r, c = np.meshgrid(np.arange(R - 1), np.arange(C - 1), indexing="ij")
            E = E + inst.pair_d[r[None], c[None], G[:, :-1, :-1], G[:, 1:, 1:]].sum(axis=(1, 2))
            E = E + inst.pair_a[r[None], c[None], G[:, :-1, 1:], G[:, 1:, :-1]].sum(axis=(1, 2))
    return E


def ising_energy(si, S: np.ndarray) -> np.ndarray:
    """Eq. (2) on the raw spins: E(s) = sum J_ij s_i s_j + sum h_i s_i.

    ``S`` is [n_cfg][rows][cols][t] with entries +-1."""
    S = np.asarray(S, dtype=np.float64)
    E = np.einsum("nrci,rci->n", S, si.h)
    E = E + np.einsum("nrci,rcij,nrcj->n", S, np.triu(si.J_in, 1), S)
    E = E + np.einsum("nrci,rcij,nrcj->n", S[:, :, :-1], si.J_h, S[:, :, 1:])
    E = E + np.einsum("nrci,rcij,nrcj->n", S[:, :-1, :], si.J_v, S[:, 1:, :])
    if si.kings:
        E = E + np.einsum("nrci,rcij,nrcj->n", S[:, :-1, :-1], si.J_d, S[:, 1:, 1:])
        E = E + np.einsum("nrci,rcij,nrcj->n", S[:, :-1, 1:], si.J_a, S[:, 1:, :-1])
    return E


class Weights:
    """Boltzmann factors of the min-shifted tables: w = exp(-beta (E - eps)),
    eps = table minimum, and their exact logs (log_loc, log_h, ...), which stay
    finite where the weights underflow.  The shift only rescales Z:  log Z = log Z~ - beta*shift.

    Absent edge classes (square lattice) and absent neighbours are all-ones
    tables, which is the same as a zero energy."""

    def __init__(self, inst):
        self.inst = inst
        b = inst.beta
        R, C, d = inst.rows, inst.cols, inst.d
        le, ph, pv, pd, pa = inst.tables()
        self.shift = 0.0

        def lw(T):
            """-beta (E - eps): the exact logs of the weights."""
            if T.size == 0:
                return np.zeros(T.shape)
            eps = T.reshape(T.shape[: T.ndim - (1 if T is le else 2)] + (-1,)).min(axis=-1)
            self.shift += float(eps.sum())
            if T is le:
                return -b * (T - eps[..., None])
            return -b * (T - eps[..., None, None])

        self.log_loc = lw(le)                               # [R][C][d]
        self.log_h = lw(ph)                                 # [R][C-1][d][d]
        self.log_v = lw(pv)                                 # [R-1][C][d][d]
        if inst.kings:
            self.log_dg = lw(pd)
            self.log_an = lw(pa)
        else:
            self.log_dg = np.zeros((max(R - 1, 0), max(C - 1, 0), d, d))
            self.log_an = np.zeros((max(R - 1, 0), max(C - 1, 0), d, d))
        self.loc = np.exp(self.log_loc)
        self.h = np.exp(self.log_h)
        self.v = np.exp(self.log_v)
        self.dg = np.exp(self.log_dg)
        self.an = np.exp(self.log_an)
