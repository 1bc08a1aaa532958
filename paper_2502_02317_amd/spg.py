"""Thin ctypes binding of libspg.so (include/spg.h), same entry-point names.

Only argument marshalling happens here: every step of the hot path runs in
the library's HIP kernels.  Device buffers are torch ROCm tensors passed by
``data_ptr()``; streams are ``torch.cuda.Stream`` objects (or None for the
current stream).  If the library is missing the import fails loudly - there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspg.so")

SPG_FP64, SPG_FP32, SPG_BF16 = 0, 1, 2
SPG_MAX_DROPLETS = 64         # include/spg.h
PRECISION = {"fp64": SPG_FP64, "fp32": SPG_FP32, "bf16": SPG_BF16}
ERRORS = {-1: "SPG_ERR_INVALID", -2: "SPG_ERR_OOM", -3: "SPG_ERR_HIP",
          -4: "SPG_ERR_NONFINITE", -5: "SPG_ERR_UNSUPPORTED"}


class SpgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class InstanceDesc(C.Structure):
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32), ("d", C.c_int32), ("kings", C.c_int32),
                ("beta", C.c_double), ("local_E", C.c_void_p), ("pair_E_h", C.c_void_p),
                ("pair_E_v", C.c_void_p), ("pair_E_d", C.c_void_p), ("pair_E_a", C.c_void_p)]


class MpsParams(C.Structure):
    _fields_ = [("chi", C.c_int32), ("num_sweeps", C.c_int32), ("precision", C.c_int32),
                ("oversample", C.c_int32), ("power_iters", C.c_int32)]


class SearchParams(C.Structure):
    _fields_ = [("max_states", C.c_int32), ("cut_off_prob", C.c_double),
                ("proposal", C.c_void_p), ("kappa", C.c_double),
                ("merge_branches", C.c_int32), ("droplet_energy", C.c_double),
                ("droplet_hamming", C.c_int32), ("max_droplets", C.c_int32)]


class TrainParams(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("learning_rate", C.c_float), ("max_states", C.c_int32)]


N_FEATURES = 6
BATCH_CLASSES = 1


class BatchItem(C.Structure):
    _fields_ = [("chi", C.c_int32), ("num_sweeps", C.c_int32), ("precision", C.c_int32),
                ("oversample", C.c_int32), ("power_iters", C.c_int32),
                ("max_states", C.c_int32), ("cut_off_prob", C.c_double)]


EXPORTS = ["spg_build_peps", "spg_boundary_mps", "spg_marginals", "spg_marginals_noalloc",
           "spg_branch_and_bound", "spg_topm",
           "spg_free_peps", "spg_free_env", "spg_last_error", "spg_env_info", "spg_env_export",
           "spg_env_import", "spg_profile_enable", "spg_profile_reset", "spg_profile_query",
           "spg_proposal_create", "spg_proposal_free", "spg_proposal_params",
           "spg_proposal_train", "spg_proposal_features", "spg_proposal_forward",
           "spg_proposal_loss_grad", "spg_proposal_adam", "spg_search_stats",
           "spg_batch_create", "spg_batch_free", "spg_batch_run", "spg_batch_result",
           "spg_batch_set_tuning", "spg_batch_autotune", "spg_set_tuning", "spg_set_kernel_forms",
           "spg_set_gemm_precision", "spg_batch_info", "spg_batch_plan", "spg_batch_tuning",
           "spg_droplets", "spg_ising_to_potts"]
KERNEL_CLASSES = ["gemm_f64", "qr_f64", "qform_f64", "jacobi_svd_f64", "normalize_box", "right_env",
                  "marginals", "select_topm", "beam_update", "final_sort", "propose",
                  "guided_eval", "mlp_grad", "merge_branches", "droplets", "u_mfma",
                  "mpo_gemm_f64"]

_lib = None


def load() -> C.CDLL:
    """Load libspg.so (built in-tree); raises if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2502_02317_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    vp, i32, f64p, i32p = C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)
    lib.spg_build_peps.argtypes = [C.POINTER(InstanceDesc), vp, C.POINTER(vp)]
    lib.spg_boundary_mps.argtypes = [vp, C.POINTER(MpsParams), vp, C.POINTER(vp), f64p]
    lib.spg_marginals.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.spg_marginals_noalloc.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.spg_topm.argtypes = [i32, i32, vp, vp, vp, vp]
    lib.spg_branch_and_bound.argtypes = [vp, C.POINTER(SearchParams), vp, vp, vp, i32p, vp]
    lib.spg_free_peps.argtypes = [vp]
    lib.spg_free_env.argtypes = [vp]
    lib.spg_last_error.restype = C.c_char_p
    lib.spg_env_info.argtypes = [vp, i32p, i32p, i32p, i32p, vp]
    lib.spg_env_export.argtypes = [vp, vp, vp]
    lib.spg_env_import.argtypes = [vp, i32, vp, vp, vp, i32, vp, C.POINTER(vp)]
    lib.spg_profile_enable.argtypes = [i32]
    lib.spg_profile_enable.restype = None
    lib.spg_profile_reset.argtypes = []
    lib.spg_profile_reset.restype = None
    lib.spg_profile_query.argtypes = [C.c_char_p, C.POINTER(C.c_int64), f64p, f64p]
    f32p = C.POINTER(C.c_float)
    lib.spg_proposal_create.argtypes = [i32, C.c_uint64, C.POINTER(vp)]
    lib.spg_proposal_free.argtypes = [vp]
    lib.spg_proposal_free.restype = None
    lib.spg_proposal_params.argtypes = [vp, vp, vp, i32p]
    lib.spg_proposal_train.argtypes = [vp, vp, C.POINTER(TrainParams), vp, f32p]
    lib.spg_proposal_features.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    lib.spg_proposal_forward.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.spg_proposal_loss_grad.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
    lib.spg_proposal_adam.argtypes = [vp, vp, C.c_float, vp]
    lib.spg_search_stats.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.spg_droplets.argtypes = [vp, i32, i32, vp, vp, i32p]
    lib.spg_ising_to_potts.argtypes = [i32, i32, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp,
                                       vp, vp, vp]
    lib.spg_batch_create.argtypes = [C.POINTER(vp), C.POINTER(BatchItem), i32, i32, i32,
                                     C.POINTER(vp)]
    lib.spg_batch_info.argtypes = [vp, i32p, vp]
    lib.spg_batch_free.argtypes = [vp]
    lib.spg_batch_free.restype = None
    lib.spg_batch_run.argtypes = [vp, i32, vp]
    lib.spg_batch_result.argtypes = [vp, i32, vp, vp, vp, i32p, f64p]
    lib.spg_batch_set_tuning.argtypes = [vp, i32, i32]
    lib.spg_batch_autotune.argtypes = [vp, vp, vp]
    lib.spg_batch_tuning.argtypes = [vp, i32, i32p, i32p, i32p]
    lib.spg_set_tuning.argtypes = [i32]
    lib.spg_set_kernel_forms.argtypes = [i32, i32]
    lib.spg_set_gemm_precision.argtypes = [i32]
    lib.spg_batch_plan.argtypes = [vp, vp, i32, i32, vp, i32p, vp, i32, vp, vp]
    for name in ["spg_build_peps", "spg_boundary_mps", "spg_marginals", "spg_marginals_noalloc",
                 "spg_branch_and_bound", "spg_topm",
                 "spg_env_info", "spg_env_export", "spg_env_import", "spg_profile_query",
                 "spg_proposal_create", "spg_proposal_params", "spg_proposal_train",
                 "spg_proposal_features", "spg_proposal_forward", "spg_proposal_loss_grad",
                 "spg_proposal_adam", "spg_search_stats", "spg_batch_create", "spg_batch_run",
                 "spg_batch_result", "spg_batch_set_tuning", "spg_batch_autotune",
                 "spg_set_tuning", "spg_set_kernel_forms", "spg_set_gemm_precision",
                 "spg_batch_info", "spg_batch_plan",
                 "spg_batch_tuning",
                 "spg_droplets",
                 "spg_ising_to_potts"]:
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise SpgError(rc, load().spg_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Peps:
    """Owner of an spg_peps_t handle."""

    def __init__(self, handle, inst):
        self.handle = handle
        self.inst = inst

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.spg_free_peps(self.handle)
            self.handle = None


class Env:
    """Owner of an spg_env_t handle (keeps its Peps alive)."""

    def __init__(self, handle, peps: Peps):
        self.handle = handle
        self.peps = peps

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.spg_free_env(self.handle)
            self.handle = None


def build_peps(inst, stream=None) -> Peps:
    """spg_build_peps on a workloads.PottsInstance-like object (host float64 tables)."""
    lib = load()
    le, ph, pv, pd, pa = (np.ascontiguousarray(t, dtype=np.float64) for t in inst.tables())
    keep = (le, ph, pv, pd, pa)
    desc = InstanceDesc(inst.rows, inst.cols, inst.d, 1 if inst.kings else 0, float(inst.beta),
                        le.ctypes.data, ph.ctypes.data, pv.ctypes.data,
                        pd.ctypes.data if inst.kings else None,
                        pa.ctypes.data if inst.kings else None)
    h = C.c_void_p()
    _check(lib.spg_build_peps(C.byref(desc), _stream(stream), C.byref(h)))
    del keep
    return Peps(h, inst)


def boundary_mps(peps: Peps, chi: int, num_sweeps: int = 1, precision: str = "fp64",
                 oversample: int = 16, power_iters: int = 1, stream=None, want_logZ=True,
                 nonfinite_ok=False):
    """spg_boundary_mps; returns (Env, log Z or None).  With nonfinite_ok a
    non-finite log Z (SPG_ERR_NONFINITE, the env is still returned) comes back
    as the value instead of raising."""
    lib = load()
    prm = MpsParams(chi, num_sweeps, PRECISION[precision], oversample, power_iters)
    h = C.c_void_p()
    lz = C.c_double(0.0)
    rc = lib.spg_boundary_mps(peps.handle, C.byref(prm), _stream(stream), C.byref(h),
                              C.byref(lz) if want_logZ else None)
    env = Env(h, peps) if h.value else None
    if not (nonfinite_ok and want_logZ and rc == -4 and env is not None):
        _check(rc)
    return env, (lz.value if want_logZ else None)


def marginals(env: Env, site: int, beam_cfg, out, stream=None):
    """spg_marginals: beam_cfg int32 [n][N] and out float64 [n][d], torch device tensors."""
    _check(load().spg_marginals(env.handle, int(site), int(beam_cfg.shape[0]), _ptr(beam_cfg),
                                _ptr(out), _stream(stream)))
    return out


def marginals_noalloc(env: Env, site: int, beam_cfg, out, stream=None):
    """spg_marginals_noalloc: as marginals(), with the library's static scratch."""
    _check(load().spg_marginals_noalloc(env.handle, int(site), int(beam_cfg.shape[0]),
                                        _ptr(beam_cfg), _ptr(out), _stream(stream)))
    return out


def topm(scores, M: int, sel_out, scores_out=None, stream=None):
    """spg_topm: scores float64 [n], sel_out int32 [min(M, n)], scores_out
    float64 [min(M, n)] or None; torch device tensors."""
    _check(load().spg_topm(int(scores.shape[0]), int(M), _ptr(scores), _ptr(sel_out),
                           _ptr(scores_out) if scores_out is not None else None, _stream(stream)))
    return sel_out


def branch_and_bound(env: Env, max_states: int, states_out, energies_out, logp_out,
                     cut_off_prob: float = 0.0, stream=None, proposal=None,
                     kappa: float = 2.0, merge_branches: bool = False,
                     droplets=None) -> int:
    """spg_branch_and_bound into device tensors; returns n_out.  With a
    Proposal the guarded steps run (kappa * max_states exact children per step
    before the guard).  ``droplets`` = (energy_cutoff, hamming_cutoff,
    max_droplets) collects droplets while merging (read them with droplets())."""
    de, dh, dm = droplets if droplets is not None else (0.0, 0, 0)
    prm = SearchParams(int(max_states), float(cut_off_prob),
                       proposal.handle if proposal is not None else None, float(kappa),
                       1 if merge_branches else 0, float(de), int(dh), int(dm))
    n = C.c_int32(0)
    _check(load().spg_branch_and_bound(env.handle, C.byref(prm), _ptr(states_out),
                                       _ptr(energies_out), _ptr(logp_out), C.byref(n),
                                       _stream(stream)))
    return n.value


def droplets(env: Env, state: int, max_out: int = SPG_MAX_DROPLETS):
    """spg_droplets: (configurations [n][rows*cols] int32, energies [n]) of the
    state returned at position ``state`` by the last search on ``env``."""
    info = env_info(env)
    N = info.rows * info.cols
    cfg = np.zeros((max_out, N), dtype=np.int32)
    en = np.zeros(max_out)
    n = C.c_int32(0)
    _check(load().spg_droplets(env.handle, int(state), int(max_out), cfg.ctypes.data,
                               en.ctypes.data, C.byref(n)))
    k = min(n.value, max_out)
    return cfg[:k], en[:k]


# ---- Ising input -------------------------------------------------------------

def read_ising(path: str):
    """Ising instance from text: one term per line, ``i j J`` with 1-based spin
    indices (i == j: a field), ``#`` starts a comment.  Returns (n_spins, i, j, J)
    with 0-based int32 indices; n_spins is the largest index seen."""
    ii, jj, JJ = [], [], []
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            if len(line) != 3:
                raise ValueError(f"{path}: expected 'i j J', got {' '.join(line)!r}")
            ii.append(int(line[0]) - 1)
            jj.append(int(line[1]) - 1)
            JJ.append(float(line[2]))
    i = np.asarray(ii, dtype=np.int32)
    j = np.asarray(jj, dtype=np.int32)
    if i.size and min(i.min(), j.min()) < 0:
        raise ValueError(f"{path}: spin indices start at 1")
    n = int(max(i.max(), j.max()) + 1) if i.size else 0
    return n, i, j, np.asarray(JJ, dtype=np.float64)


def lattice_clusters(rows: int, cols: int, t: int) -> np.ndarray:
    """Cluster of every spin when the spins come in consecutive runs of t per
    cluster, clusters row-major: spin i -> cluster i // t."""
    return (np.arange(rows * cols * t) // t).astype(np.int32)


@dataclass
class IsingPotts:
    """Potts tables made from an Ising instance (accepted by build_peps)."""
    rows: int
    cols: int
    d: int
    kings: bool
    local_E: np.ndarray
    pair_h: np.ndarray
    pair_v: np.ndarray
    pair_d: np.ndarray
    pair_a: np.ndarray
    beta: float = 1.0

    @property
    def n_sites(self) -> int:
        return self.rows * self.cols

    def tables(self):
        return self.local_E, self.pair_h, self.pair_v, self.pair_d, self.pair_a


def ising_to_potts(n_spins: int, i, j, J, rows: int, cols: int, t: int, kings: bool,
                   cluster_of=None, beta: float = 1.0) -> IsingPotts:
    """spg_ising_to_potts: the Potts tables of an Ising instance on a rows x cols
    lattice of t-spin clusters (cluster_of defaults to lattice_clusters)."""
    d = 1 << t
    ti = np.ascontiguousarray(i, dtype=np.int32)
    tj = np.ascontiguousarray(j, dtype=np.int32)
    tJ = np.ascontiguousarray(J, dtype=np.float64)
    cl = np.ascontiguousarray(lattice_clusters(rows, cols, t) if cluster_of is None
                              else cluster_of, dtype=np.int32)
    le = np.zeros((rows, cols, d))
    ph = np.zeros((rows, max(cols - 1, 0), d, d))
    pv = np.zeros((max(rows - 1, 0), cols, d, d))
    pd = np.zeros((max(rows - 1, 0), max(cols - 1, 0), d, d))
    pa = np.zeros_like(pd)
    _check(load().spg_ising_to_potts(int(n_spins), int(ti.size), ti.ctypes.data, tj.ctypes.data,
                                     tJ.ctypes.data, int(rows), int(cols), int(t),
                                     1 if kings else 0, cl.ctypes.data, le.ctypes.data,
                                     ph.ctypes.data, pv.ctypes.data, pd.ctypes.data,
                                     pa.ctypes.data))
    return IsingPotts(rows, cols, d, bool(kings), le, ph, pv, pd, pa, float(beta))


@dataclass
class EnvInfo:
    rows: int
    cols: int
    d: int
    chi: int
    bond_dims: np.ndarray


def env_info(env: Env) -> EnvInfo:
    lib = load()
    r, c, d, chi = (C.c_int32() for _ in range(4))
    _check(lib.spg_env_info(env.handle, C.byref(r), C.byref(c), C.byref(d), C.byref(chi), None))
    dims = np.zeros((r.value, c.value + 1), dtype=np.int32)
    _check(lib.spg_env_info(env.handle, None, None, None, None, dims.ctypes.data))
    return EnvInfo(r.value, c.value, d.value, chi.value, dims)


def env_export(env: Env):
    """(tensors [rows][cols][chi][d][chi], lam [rows]) as host float64 arrays."""
    info = env_info(env)
    T = np.zeros((info.rows, info.cols, info.chi, info.d, info.chi))
    lam = np.zeros(info.rows)
    _check(load().spg_env_export(env.handle, T.ctypes.data, lam.ctypes.data))
    return T, lam


def env_import(peps: Peps, chi: int, bond_dims, tensors, lam=None, precision: str = "fp64",
               stream=None) -> Env:
    lib = load()
    dims = np.ascontiguousarray(bond_dims, dtype=np.int32)
    T = np.ascontiguousarray(tensors, dtype=np.float64)
    lm = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
    h = C.c_void_p()
    _check(lib.spg_env_import(peps.handle, int(chi), dims.ctypes.data, T.ctypes.data,
                              None if lm is None else lm.ctypes.data, PRECISION[precision],
                              _stream(stream), C.byref(h)))
    return Env(h, peps)


def profile_enable(on: bool = True):
    load().spg_profile_enable(1 if on else 0)


def profile_reset():
    load().spg_profile_reset()


def profile_query(name: str):
    """(launch count, summed milliseconds, summed algorithmic work) of a timed
    kernel class since the last reset."""
    n, t, w = C.c_int64(0), C.c_double(0.0), C.c_double(0.0)
    _check(load().spg_profile_query(name.encode(), C.byref(n), C.byref(t), C.byref(w)))
    return n.value, t.value, w.value


def pack_oracle_mps(A_rows, chi: int, d: int):
    """Pad an oracle boundary MPS (list of rows of (chi_c, d, chi_c+1) arrays) into the
    library layout; returns (tensors, bond_dims)."""
    R, Cc = len(A_rows), len(A_rows[0])
    T = np.zeros((R, Cc, chi, d, chi))
    dims = np.ones((R, Cc + 1), dtype=np.int32)
    for r in range(R):
        for c in range(Cc):
            a, _, b = A_rows[r][c].shape
            T[r, c, :a, :, :b] = A_rows[r][c]
            dims[r, c], dims[r, c + 1] = a, b
    return T, dims


def unpack_mps(T, dims):
    """Inverse of pack_oracle_mps: list of rows of (chi_c, d, chi_c+1) arrays."""
    R, Cc = T.shape[0], T.shape[1]
    return [[T[r, c, :dims[r, c], :, :dims[r, c + 1]].copy() for c in range(Cc)] for r in range(R)]


# ---- learned proposal ---------------------------------------------------------

class Proposal:
    """Owner of an spg_proposal_t handle (2-layer FP32 network, hidden units H)."""

    def __init__(self, hidden: int = 32, seed: int = 1):
        h = C.c_void_p()
        _check(load().spg_proposal_create(int(hidden), int(seed), C.byref(h)))
        self.handle = h
        self.hidden = int(hidden)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.spg_proposal_free(self.handle)
            self.handle = None

    @property
    def n_params(self) -> int:
        n = C.c_int32(0)
        _check(load().spg_proposal_params(self.handle, None, None, C.byref(n)))
        return n.value

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        n = C.c_int32(0)
        _check(load().spg_proposal_params(self.handle, out.ctypes.data, None, C.byref(n)))
        return out

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        n = C.c_int32(0)
        _check(load().spg_proposal_params(self.handle, None, p.ctypes.data, C.byref(n)))

    def train(self, env: Env, epochs: int = 10, learning_rate: float = 1e-2,
              max_states: int = 64, stream=None) -> np.ndarray:
        tp = TrainParams(int(epochs), float(learning_rate), int(max_states))
        loss = np.zeros(int(epochs), dtype=np.float32)
        _check(load().spg_proposal_train(self.handle, env.handle, C.byref(tp), _stream(stream),
                                         loss.ctypes.data_as(C.POINTER(C.c_float))))
        return loss

    def forward(self, feats, logp_out, stream=None):
        n, d = int(feats.shape[0]), int(feats.shape[1])
        _check(load().spg_proposal_forward(self.handle, n, d, _ptr(feats), _ptr(logp_out),
                                           _stream(stream)))
        return logp_out

    def loss_grad(self, feats, target, grad_out, loss_out, stream=None):
        n, d = int(feats.shape[0]), int(feats.shape[1])
        _check(load().spg_proposal_loss_grad(self.handle, n, d, _ptr(feats), _ptr(target),
                                             _ptr(grad_out), _ptr(loss_out), _stream(stream)))

    def adam(self, grad, learning_rate: float, stream=None):
        _check(load().spg_proposal_adam(self.handle, _ptr(grad), float(learning_rate),
                                        _stream(stream)))


def proposal_features(env: Env, site: int, beam_cfg, beam_score, feats_out, stream=None):
    """spg_proposal_features: beam_cfg int32 [n][N], beam_score float64 [n] ->
    feats_out float32 [n][d][6] (device tensors)."""
    _check(load().spg_proposal_features(env.handle, int(site), int(beam_cfg.shape[0]),
                                        _ptr(beam_cfg), _ptr(beam_score), _ptr(feats_out),
                                        _stream(stream)))
    return feats_out


def search_stats(env: Env):
    """(children evaluated exactly, children resolved, fallback parents) of the
    env's last search."""
    out = (C.c_int64 * 3)()
    _check(load().spg_search_stats(env.handle, out))
    return int(out[0]), int(out[1]), int(out[2])


# ---- batches --------------------------------------------------------------------

def set_tuning(gemm_tile: int) -> None:
    """Default GEMM tile (32 or 64) of calls outside batches on this thread."""
    _check(load().spg_set_tuning(int(gemm_tile)))


def set_gemm_precision(fp32_products: bool) -> None:
    """Reduced-precision FP64 GEMMs on this thread: FP32 operands and FP32
    accumulation on the matrix cores, FP64 results (QR, SVD and the MPO
    contractions stay FP64).  False (default) restores FP64 products."""
    _check(load().spg_set_gemm_precision(1 if fp32_products else 0))


def set_kernel_forms(mpo_columns: bool = True, q_split: bool = True) -> None:
    """Kernel forms of the boundary MPS on this thread (each pair gives bitwise
    equal results): mpo_columns, the column forms of the MPO d-index
    contractions (d in {8, 16, 24, 32}) rather than one thread per output;
    q_split, Q of one-panel QR factorisations formed by a second kernel with a
    compute unit per column rather than by the panel kernel."""
    _check(load().spg_set_kernel_forms(1 if mpo_columns else 0, 1 if q_split else 0))


def batch_plan(shapes, chi, max_states, num_sweeps=1, precision="fp64", oversample=16,
               power_iters=1, cut_off_prob=0.0, classes=True, max_buffers=128):
    """The units spg_batch_create would form for instances of these shapes
    ((rows, cols, d, kings) each), computed on the host without a device.
    Returns (unit_of [n], units: list of (members, slice_bytes), layouts: per
    unit an int64 array [buffers][2] of (offset, bytes) in the slice, empty
    for single instances)."""
    n = len(shapes)
    sh = np.ascontiguousarray(np.asarray(shapes, dtype=np.int32).reshape(n, 4))
    chis = list(chi) if hasattr(chi, "__len__") else [chi] * n
    Ms = list(max_states) if hasattr(max_states, "__len__") else [max_states] * n
    precs = [precision] * n if isinstance(precision, str) else list(precision)
    items = (BatchItem * n)(*[BatchItem(int(chis[i]), int(num_sweeps), PRECISION[precs[i]],
                                        int(oversample), int(power_iters), int(Ms[i]),
                                        float(cut_off_prob)) for i in range(n)])
    unit_of = np.zeros(n, dtype=np.int32)
    nu = C.c_int32(0)
    ub = np.zeros((n, 2), dtype=np.int64)
    lay = np.zeros((n, max_buffers, 2), dtype=np.int64)
    nb = np.zeros(n, dtype=np.int32)
    _check(load().spg_batch_plan(sh.ctypes.data, items, n, BATCH_CLASSES if classes else 0,
                                 unit_of.ctypes.data, C.byref(nu), ub.ctypes.data,
                                 int(max_buffers), lay.ctypes.data, nb.ctypes.data))
    U = nu.value
    if np.any(nb[:U] > max_buffers):
        raise ValueError("batch_plan: a class has more buffers than max_buffers")
    units = [(int(ub[u, 0]), int(ub[u, 1])) for u in range(U)]
    layouts = [lay[u, :nb[u]].copy() for u in range(U)]
    return unit_of, units, layouts


class Batch:
    """Owner of an spg_batch_t: many instances run as one unit (optionally one
    captured graph).  Keeps its Peps objects alive."""

    def __init__(self, peps_list, chi, max_states, num_sweeps=1, precision="fp64",
                 oversample=16, power_iters=1, cut_off_prob=0.0, n_streams=8, classes=True):
        n = len(peps_list)
        chis = list(chi) if hasattr(chi, "__len__") else [chi] * n
        Ms = list(max_states) if hasattr(max_states, "__len__") else [max_states] * n
        precs = [precision] * n if isinstance(precision, str) else list(precision)
        items = (BatchItem * n)(*[BatchItem(int(chis[i]), int(num_sweeps), PRECISION[precs[i]],
                                            int(oversample), int(power_iters), int(Ms[i]),
                                            float(cut_off_prob)) for i in range(n)])
        handles = (C.c_void_p * n)(*[p.handle.value for p in peps_list])
        h = C.c_void_p()
        _check(load().spg_batch_create(handles, items, n, int(n_streams),
                                       BATCH_CLASSES if classes else 0, C.byref(h)))
        self.handle = h
        self.peps = list(peps_list)
        self.n = n
        self.max_states = Ms

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.spg_batch_free(self.handle)
            self.handle = None

    def run(self, use_graph: bool = True, stream=None) -> None:
        _check(load().spg_batch_run(self.handle, 1 if use_graph else 0, _stream(stream)))

    def result(self, i: int):
        """(states int32 [n][N], energies, logp, log Z) of instance i as host arrays."""
        import torch
        if not 0 <= i < self.n:
            n = C.c_int32(0)
            _check(load().spg_batch_result(self.handle, int(i), None, None, None, C.byref(n),
                                           None))
        inst = self.peps[i].inst
        N, M = inst.rows * inst.cols, self.max_states[i]
        st = torch.zeros((M, N), dtype=torch.int32, device="cuda")
        en = torch.zeros(M, dtype=torch.float64, device="cuda")
        lp = torch.zeros(M, dtype=torch.float64, device="cuda")
        n = C.c_int32(0)
        lz = C.c_double(0.0)
        _check(load().spg_batch_result(self.handle, int(i), _ptr(st), _ptr(en), _ptr(lp),
                                       C.byref(n), C.byref(lz)))
        k = n.value
        return st[:k].cpu().numpy(), en[:k].cpu().numpy(), lp[:k].cpu().numpy(), lz.value

    def set_tuning(self, i: int, gemm_tile: int) -> None:
        _check(load().spg_batch_set_tuning(self.handle, int(i), int(gemm_tile)))

    def units(self):
        """(number of units, unit of each instance): a unit is a class of
        same-shape instances sharing every launch, or one instance."""
        nu = C.c_int32(0)
        of = np.zeros(self.n, dtype=np.int32)
        _check(load().spg_batch_info(self.handle, C.byref(nu), of.ctypes.data))
        return nu.value, of

    def tuning(self, i: int) -> dict:
        """The launch choices of instance i's unit: GEMM tile, MPO contraction
        form and Q formation (True = the column / split forms)."""
        t, m, q = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        _check(load().spg_batch_tuning(self.handle, int(i), C.byref(t), C.byref(m), C.byref(q)))
        return {"gemm_tile": t.value, "mpo_columns": bool(m.value), "q_split": bool(q.value)}

    def autotune(self, stream=None) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.int32)
        _check(load().spg_batch_autotune(self.handle, _stream(stream), out.ctypes.data))
        return out

