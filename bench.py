"""Benchmark of the PEPS branch-and-bound hot path on one MI355X.

Workload: 8x8 king's-graph lattice of 4-spin clusters (d = 16), intra-cluster
couplings and fields ~ N(0,1), inter-cluster +-1 spin couplings, beta = 2,
boundary-MPS bond chi = 32 (one sweep), beam M = 1024; synthetic, seed 0.
One step = the whole hot path on that instance: build the PEPS weights,
contract the boundary MPSs, run the branch-and-bound search.

Metric: conditional-marginal evaluations per second, one evaluation being one
resolved candidate (beam state b, local state s) at one site, so a step does
sum_k min(M, d^k) * d of them.  ``value`` is evaluations / wall time of the
whole step (inputs already on the host; the PEPS build copies them over) for
the plain path, every contraction in FP64; the mixed path (search contractions
in FP32 or with BF16 inputs, boundary MPS in FP64) is timed on the same
workload and reported beside it, together with dlogP, the largest
|log p_mixed - log p_fp64| teacher-forced on the FP64 path's beam over states
with p >= 1e-4 of the best at their parent.

The JSON line also carries the roofline of the dominant kernel class (HIP
events on its launch stream over the timed region, algorithmic work counted by
the library from the actual sizes) and the CPU oracle timed on one step of the
same workload on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# truncated SVD: randomized range finder, oversampling 16, one power iteration
WORKLOAD = dict(name="kings8x8_d16", seed=0, chi=32, max_states=1024, num_sweeps=1,
                oversample=16, power_iters=1)
# MI355X published peaks
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "hbm_GBs": 8000.0}
FLOP_CLASSES = {"gemm_f64", "qr_f64", "qform_f64", "right_env", "marginals", "beam_update",
                "u_mfma"}
BYTE_CLASSES = {"normalize_box", "select_topm"}


CLASS_KERNEL = {"gemm_f64": "k_gemm<32>", "qr_f64": "k_qr_reg<8, 3>", "qform_f64": "k_qform<8, 3>",
                "jacobi_svd_f64": "k_jacobi<3>",
                "normalize_box": "k_box_scale", "right_env": "k_right_env",
                "marginals": "k_marginals", "select_topm": "k_select",
                "beam_update": "k_beam_update", "final_sort": "k_final_sort",
                "u_mfma": "k_u_mfma<float>"}
KERNEL_SOURCES = ["k_linalg.hip", "k_bmps.hip", "k_search.hip", "k_search_lp.hip",
                  "k_propose.hip", "k_mlp.hip"]
# batching form: the first BATCH_N instances of the batched workload (lattice
# side 6..12, chi 16/32, d = 16, beta = 2, M = 512), class-batched launches
BATCH_N = 48
BATCH_M = 512


def kernel_source_sha(name):
    """(file, sha256 of the kernel's own source text) for a __global__ function."""
    import hashlib
    import re
    name = name.split("<")[0]            # a template's instances share its source
    for f in KERNEL_SOURCES:
        path = os.path.join(ROOT, "paper_2502_02317_amd", "csrc", f)
        src = open(path).read()
        m = re.search(r"__global__[^{;]*?\b" + re.escape(name) + r"\(", src)
        if not m:
            continue
        end = src.find("\n}\n", m.start())
        body = src[m.start(): end + 3]
        # with the device functions of the same file that the kernel calls
        # (one level: a kernel that is a thin wrapper of a templated body)
        for callee in sorted(set(re.findall(r"\b(\w+)\s*(?:<[^<>;{}]*>)?\s*\(", body))):
            d = re.search(r"__device__[^{;]*?\b" + re.escape(callee) + r"\(", src)
            if d and callee != name:
                body += src[d.start(): src.find("\n}\n", d.start()) + 3]
        return "paper_2502_02317_amd/csrc/" + f, hashlib.sha256(body.encode()).hexdigest()
    return None, None


def committed_traffic(kernel, workload_tag):
    """HBM bytes per dispatch from the committed counter summary, or None when
    the kernel's source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload_tag}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get("kernels", {}).get(kernel)
    if rec is None or kernel_source_sha(kernel)[1] != rec["kernel_sha256"]:
        return None
    return rec["bytes_per_dispatch"]


def evals_per_step(R, C, d, M):
    tot, B = 0, 1
    for _ in range(R * C):
        tot += B * d
        B = min(M, B * d)
    return tot


def search_formula_flops(dims, R, C, d, M):
    """Algorithmic flops of the search contractions by formula, with the
    actual bond dimensions chi_c = dims[r][c]: 2 chi_c chi_{c+1} per resolved
    child (conditionals), 2 chi_c chi_{c+1} d per row-start ancestor per
    column c >= 1 (right environments), 2 chi_c chi_{c+1} per survivor that
    carries its left vector on (c < cols - 1)."""
    tot, B = 0.0, 1
    for r in range(R):
        n_anc = B
        for c in range(1, C):
            tot += 2.0 * dims[r][c] * dims[r][c + 1] * d * n_anc
        for c in range(C):
            cc = 2.0 * dims[r][c] * dims[r][c + 1]
            tot += cc * B * d
            B = min(M, B * d)
            if c < C - 1:
                tot += cc * B
    return tot


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def row_sums(rows):
    """sum_X of each row's boundary function (normalised MPS, without its
    log-scale): the exact functions are positive, so a non-positive sum marks a
    row whose approximation has lost its mass."""
    import numpy as np
    out = []
    for row in rows:
        v = np.ones(1)
        for A in row:
            v = v @ A.sum(axis=1)
        out.append(float(v[0]))
    return out


def finite_or_none(x):
    import math
    return x if (x is not None and math.isfinite(x)) else None


def cpu_baseline(inst, wl):
    """The oracle, as it stands, on one step of the same workload; its own
    result (log Z, best energy) is returned beside its time."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle.bmps import boundary_mps
    from oracle.search import beam_search
    cores = len(os.sched_getaffinity(0))
    with threadpool_limits(limits=cores):
        info = threadpool_info()
        used = max([i.get("num_threads", 1) for i in info] or [1])
        t0 = time.perf_counter()
        mp = boundary_mps(inst, wl["chi"], num_sweeps=wl["num_sweeps"])
        t1 = time.perf_counter()
        res = beam_search(inst, mp["A"], wl["max_states"])
        t2 = time.perf_counter()
    ev = evals_per_step(inst.rows, inst.cols, inst.d, wl["max_states"])
    sums = row_sums(mp["A"])
    return {"value": ev / (t2 - t0), "unit": "evals/s", "cores": used, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"one full step of the same instance (boundary MPS {t1 - t0:.1f} s + "
                      f"search {t2 - t1:.1f} s)",
            "bmps_s": t1 - t0, "search_s": t2 - t1,
            "oracle_logZ": finite_or_none(mp["logZ"]),
            "oracle_rows_with_nonpositive_sum": [r for r, v in enumerate(sums) if not v > 0],
            "oracle_best_energy": float(res["energies"][0]) if res["n_valid"] > 0 else None,
            "oracle_n_states": res["n_valid"],
            "_oracle_A": mp["A"]}


def j1_leg(spg, torch, name, chi, M, train_M, epochs, reps, stream):
    """The mixed-precision + learned-proposal search: FP32 search contractions
    with the network (trained on the method's own FP64 marginals of two other
    instances of the workload, seeds 1 and 2) pre-ranking the children and
    the guard evaluating the rest, against the plain FP64 search and the plain
    FP32 search on the same boundary MPS.  Search-only times (the boundary MPS
    is shared); every conditional marginal the search resolves counts as an
    eval, evaluated exactly or bounded by the guard.  Returns (record, network)."""
    import numpy as np
    from workloads import config_instance
    inst = config_instance(name, 0)
    R, C, d = inst.rows, inst.cols, inst.d
    N = R * C
    dev = torch.device("cuda:0")
    st = torch.zeros((M, N), dtype=torch.int32, device=dev)
    en = torch.zeros(M, dtype=torch.float64, device=dev)
    lp = torch.zeros(M, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prop = spg.Proposal(hidden=32, seed=1)
    for sd in (1, 2):
        po = spg.build_peps(config_instance(name, sd), stream)
        eo, _ = spg.boundary_mps(po, chi, stream=stream, want_logZ=False)
        prop.train(eo, epochs=epochs, learning_rate=5e-3, max_states=train_M, stream=stream)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    peps = spg.build_peps(inst, stream)
    env64, _ = spg.boundary_mps(peps, chi, stream=stream, want_logZ=False)
    T, _ = spg.env_export(env64)
    env32 = spg.env_import(peps, chi, spg.env_info(env64).bond_dims, T, np.zeros(R),
                           precision="fp32", stream=stream)

    def run(env, **kw):
        spg.branch_and_bound(env, M, st, en, lp, stream=stream, **kw)      # warm
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            n = spg.branch_and_bound(env, M, st, en, lp, stream=stream, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - a) * 1e3 / reps
        states = {tuple(x): l for x, l in zip(st[:n].cpu().numpy().tolist(),
                                              lp[:n].cpu().numpy().tolist())}
        return {"ms": ms, "states": states, "E": float(en[0]) if n > 0 else None,
                "stats": spg.search_stats(env)}

    p64, p32 = run(env64), run(env32)
    g32 = run(env32, proposal=prop, kappa=2.0)
    g64 = run(env64, proposal=prop, kappa=2.0)
    resolved = p64["stats"][1]
    rate = {k: resolved / (v["ms"] * 1e-3) for k, v in
            (("plain_fp64", p64), ("plain_fp32", p32), ("guided_fp32", g32), ("guided_fp64", g64))}
    common = p64["states"].keys() & g32["states"].keys()
    dl = [abs(p64["states"][k] - g32["states"][k]) for k in common]
    exact, _, fb = g32["stats"]
    rec = {"workload": f"{name} chi={chi} M={M} (seed 0)",
           "trained_on": "FP64 marginals of seeds 1 and 2 of the workload",
           "train_max_states": train_M, "epochs": epochs, "train_s": train_s,
           "kappa": 2.0, "hidden": 32, "search_ms": {k: v["ms"] for k, v in
                                                    (("plain_fp64", p64), ("plain_fp32", p32),
                                                     ("guided_fp32", g32), ("guided_fp64", g64))},
           "evals_per_s": rate, "resolved_evals": resolved,
           "speedup_guided_fp32_vs_plain_fp64": rate["guided_fp32"] / rate["plain_fp64"],
           "speedup_plain_fp32_vs_plain_fp64": rate["plain_fp32"] / rate["plain_fp64"],
           "guided_fp32_exact_evals": exact, "guided_fp32_exact_fraction": exact / resolved,
           "guided_fp32_fallback_parents": fb,
           "guided_fp64_exact_fraction": g64["stats"][0] / resolved,
           "best_energy": {"plain_fp64": p64["E"], "plain_fp32": p32["E"],
                           "guided_fp32": g32["E"], "guided_fp64": g64["E"]},
           "states_shared_guided_fp32_with_plain_fp64": len(common) / max(len(p64["states"]), 1),
           "states_shared_guided_fp32_with_plain_fp32":
               len(p32["states"].keys() & g32["states"].keys()) / max(len(p32["states"]), 1),
           "logp_shared_states_max_abs_diff_vs_fp64": max(dl) if dl else None,
           "logp_shared_states_median_abs_diff_vs_fp64": float(np.median(dl)) if dl else None}
    return rec, prop


def batching_leg(spg, torch, stream):
    """Batching: the same instances run one by one (boundary MPS + search,
    FP64) and as one batch with class-batched launches."""
    from workloads import cfg3_shapes, cfg3_instance
    L, chi = cfg3_shapes()
    n = BATCH_N
    insts = [cfg3_instance(i, int(L[i])) for i in range(n)]
    peps = [spg.build_peps(x, stream) for x in insts]
    chis = [int(c) for c in chi[:n]]
    ev = sum(evals_per_step(x.rows, x.cols, x.d, BATCH_M) for x in insts)
    dev = torch.device("cuda:0")
    torch.cuda.synchronize()
    a = time.perf_counter()
    for i in range(n):
        env, _ = spg.boundary_mps(peps[i], chis[i], precision="fp64", stream=stream,
                                  want_logZ=False)
        N = insts[i].rows * insts[i].cols
        s_ = torch.zeros((BATCH_M, N), dtype=torch.int32, device=dev)
        e_ = torch.zeros(BATCH_M, dtype=torch.float64, device=dev)
        l_ = torch.zeros(BATCH_M, dtype=torch.float64, device=dev)
        spg.branch_and_bound(env, BATCH_M, s_, e_, l_, stream=stream)
        del env
    torch.cuda.synchronize()
    t_one = time.perf_counter() - a
    b = spg.Batch(peps, chi=chis, max_states=BATCH_M, n_streams=8, classes=True)
    units = b.units()[0]
    b.run(use_graph=False, stream=stream)          # first run sizes and warms
    torch.cuda.synchronize()
    a = time.perf_counter()
    b.run(use_graph=False, stream=stream)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - a
    # the autotuner's choices (GEMM tile, MPO contraction form, Q formation;
    # tuning itself untimed), then the batch timed again with them
    b.autotune(stream=stream)
    b.run(use_graph=False, stream=stream)
    torch.cuda.synchronize()
    a = time.perf_counter()
    b.run(use_graph=False, stream=stream)
    torch.cuda.synchronize()
    t_tuned = time.perf_counter() - a
    choices = [b.tuning(i) for i in range(n)]
    # one more batched run with per-launch events: the FP64 kernel classes'
    # rates when a launch covers every member of a shape class (one
    # workgroup per member for the QR and the Jacobi SVD); work over the
    # summed launch durations, on eight overlapping streams
    spg.profile_reset()
    spg.profile_enable(True)
    b.run(use_graph=False, stream=stream)
    torch.cuda.synchronize()
    spg.profile_enable(False)
    rates = {}
    for k in ("qr_f64", "qform_f64", "gemm_f64"):
        cnt, ms, work = spg.profile_query(k)
        if ms > 0.0:
            ach = work / (ms * 1e-3) / 1e12
            rates[k] = {"launches": cnt, "avg_launch_us": ms * 1e3 / max(cnt, 1),
                        "achieved": ach, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                        "frac": ach / PEAK["fp64"]}
    spg.profile_reset()
    return {"workload": f"first {n} instances of the batched workload (L 6..12, chi 16/32, "
                        f"d 16, beta 2, M {BATCH_M})",
            "instances": n, "units": units, "evals": ev,
            "one_by_one_s": t_one, "batched_s": t_batch, "speedup": t_one / t_batch,
            "evals_per_s_one_by_one": ev / t_one, "evals_per_s_batched": ev / t_batch,
            "batched_autotuned_s": t_tuned, "speedup_autotuned": t_one / t_tuned,
            "autotuned_choices": {
                "gemm_tile_64": sum(c["gemm_tile"] == 64 for c in choices),
                "mpo_columns": sum(c["mpo_columns"] for c in choices),
                "q_split": sum(c["q_split"] for c in choices), "of_instances": n},
            "kernel_rates_batched": rates}


def transforms_leg(spg, torch, inst, wl, M, stream):
    """The bench instance on all eight orientations of its grid: one batch
    (a single shape class) against eight single runs; best of eight and the
    spread of the eight best energies on the original lattice."""
    import numpy as np
    from workloads.transforms import lattice_transform
    from oracle.energy import potts_energy
    ts = [lattice_transform(inst, k) for k in range(8)]
    peps = [spg.build_peps(t, stream) for t, _ in ts]
    dev = torch.device("cuda:0")
    N = inst.rows * inst.cols
    s_ = torch.zeros((M, N), dtype=torch.int32, device=dev)
    e_ = torch.zeros(M, dtype=torch.float64, device=dev)
    l_ = torch.zeros(M, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for p in peps:
        env, _ = spg.boundary_mps(p, wl["chi"], num_sweeps=wl["num_sweeps"], precision="fp64",
                                  oversample=wl["oversample"], power_iters=wl["power_iters"],
                                  stream=stream, want_logZ=False)
        spg.branch_and_bound(env, M, s_, e_, l_, stream=stream)
        del env
    torch.cuda.synchronize()
    t_one = time.perf_counter() - a
    b = spg.Batch(peps, chi=wl["chi"], max_states=M, num_sweeps=wl["num_sweeps"],
                  oversample=wl["oversample"], power_iters=wl["power_iters"], n_streams=2,
                  classes=True)
    b.run(use_graph=False, stream=stream)
    torch.cuda.synchronize()
    a = time.perf_counter()
    b.run(use_graph=False, stream=stream)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - a
    bests = []
    for k, (t, back) in enumerate(ts):
        st, en, _, _ = b.result(k)
        if st.shape[0] == 0:
            # every child of some step had a non-positive weight: no finite state
            bests.append(None)
            continue
        x_old = np.empty_like(st)
        x_old[:, back] = st
        # energies recomputed on the original lattice
        bests.append(float(potts_energy(inst, x_old[:1])[0]))
    found = [e for e in bests if e is not None]
    return {"orientations": 8, "units": b.units()[0], "one_by_one_s": t_one,
            "batched_s": t_batch, "speedup": t_one / t_batch,
            "best_of_8": min(found) if found else None, "best_energies": bests,
            "orientations_without_states": len(bests) - len(found),
            "spread": (max(found) - min(found)) if found else None}


def kings12_leg(spg, torch, stream):
    """The 12x12 king's workload with d = 24 (8-spin clusters, the 24 lowest
    states), beta = 4, chi = 64, beam 4096: boundary MPS in FP64, then the search
    in FP64 and with FP32 / BF16-input contractions on that boundary MPS;
    search-only times, best energies, and the contraction's validity."""
    import numpy as np
    from workloads import config_instance
    inst = config_instance("kings12x12_d24", 0)
    chi, M = 64, 4096
    R, C, d = inst.rows, inst.cols, inst.d
    N = R * C
    ev = evals_per_step(R, C, d, M)
    dev = torch.device("cuda:0")
    st = torch.zeros((M, N), dtype=torch.int32, device=dev)
    en = torch.zeros(M, dtype=torch.float64, device=dev)
    lp = torch.zeros(M, dtype=torch.float64, device=dev)
    peps = spg.build_peps(inst, stream)
    torch.cuda.synchronize()
    a = time.perf_counter()
    env, _ = spg.boundary_mps(peps, chi, stream=stream, want_logZ=False)
    torch.cuda.synchronize()
    bmps_s = time.perf_counter() - a
    try:
        _, lz = spg.boundary_mps(peps, chi, stream=stream)
    except spg.SpgError:
        lz = None
    T, _ = spg.env_export(env)
    sums = row_sums(spg.unpack_mps(T, spg.env_info(env).bond_dims))
    out = {"workload": "kings12x12_d24 beta=4 chi=64 M=4096 (seed 0)", "evals_per_search": ev,
           "boundary_mps_s": bmps_s, "logZ": finite_or_none(lz),
           "rows_with_nonpositive_sum": [r for r, v in enumerate(sums) if not v > 0]}
    for prec in ("fp64", "fp32", "bf16"):
        e = env if prec == "fp64" else spg.env_import(
            peps, chi, spg.env_info(env).bond_dims, T, np.zeros(R), precision=prec,
            stream=stream)
        spg.branch_and_bound(e, M, st, en, lp, stream=stream)      # warm
        torch.cuda.synchronize()
        a = time.perf_counter()
        n = spg.branch_and_bound(e, M, st, en, lp, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - a) * 1e3
        out[f"search_ms_{prec}"] = ms
        out[f"search_evals_per_s_{prec}"] = ev / (ms * 1e-3)
        out[f"n_states_{prec}"] = n
        out[f"best_energy_{prec}"] = float(en[0]) if n > 0 else None
    out["search_speedup_fp32_vs_fp64"] = out["search_ms_fp64"] / out["search_ms_fp32"]
    return out


def kings16_leg(spg, torch, stream):
    """The full-stack lattice shape, one instance: 16x16 king's, d = 256 (8-spin
    clusters with dense 256 x 256 pair tables), beta = 4, chi = 64, beam 10000.
    The FP64 boundary MPS (MPO contractions as matrix-core GEMMs at this d),
    its validity (log Z, the sign of every row function's sum), then the FP64
    and FP32-input searches on it: search-only times, states, best energies; and
    the contraction with FP32 products in its GEMMs, with the FP64 search on it."""
    import numpy as np
    from workloads import config_instance
    inst = config_instance("kings16x16_d256", 0)
    chi, M = 64, 10000
    R, C, d = inst.rows, inst.cols, inst.d
    N = R * C
    ev = evals_per_step(R, C, d, M)
    dev = torch.device("cuda:0")
    st = torch.zeros((M, N), dtype=torch.int32, device=dev)
    en = torch.zeros(M, dtype=torch.float64, device=dev)
    lp = torch.zeros(M, dtype=torch.float64, device=dev)
    peps = spg.build_peps(inst, stream)
    torch.cuda.synchronize()
    spg.profile_reset()
    spg.profile_enable(True)                  # per-launch events on the MPO GEMMs' class
    a = time.perf_counter()
    env, lz = spg.boundary_mps(peps, chi, stream=stream, nonfinite_ok=True)
    torch.cuda.synchronize()
    bmps_s = time.perf_counter() - a
    spg.profile_enable(False)
    g_n, g_ms, g_work = spg.profile_query("mpo_gemm_f64")
    spg.profile_reset()
    T, _ = spg.env_export(env)
    dims = spg.env_info(env).bond_dims
    sums = row_sums(spg.unpack_mps(T, dims))
    out = {"workload": "kings16x16_d256 beta=4 chi=64 M=10000 (seed 0), one instance",
           "evals_per_search": ev, "boundary_mps_s": bmps_s, "logZ": finite_or_none(lz),
           "rows_with_nonpositive_sum": [r for r, v in enumerate(sums) if not v > 0],
           # the MPO d-index contractions as FP64 GEMMs on the matrix cores: flops by
           # formula (2 M N K per batch) over the summed launch durations
           "mpo_gemm_matrix_cores": {
               "instruction": "v_mfma_f64_16x16x4f64", "launches": g_n, "ms": g_ms,
               "achieved": g_work / (g_ms * 1e-3) / 1e12 if g_ms > 0 else None,
               "peak": PEAK["fp64"], "unit": "TFLOP/s",
               "frac": g_work / (g_ms * 1e-3) / 1e12 / PEAK["fp64"] if g_ms > 0 else None}}
    for prec in ("fp64", "fp32"):
        e = env if prec == "fp64" else spg.env_import(peps, chi, dims, T, np.zeros(R),
                                                      precision=prec, stream=stream)
        spg.branch_and_bound(e, M, st, en, lp, stream=stream)      # warm (allocates)
        torch.cuda.synchronize()
        a = time.perf_counter()
        n = spg.branch_and_bound(e, M, st, en, lp, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - a) * 1e3
        out[f"search_ms_{prec}"] = ms
        out[f"search_evals_per_s_{prec}"] = ev / (ms * 1e-3)
        out[f"n_states_{prec}"] = n
        out[f"best_energy_{prec}"] = float(en[0]) if n > 0 else None
        del e
    del env
    out["search_speedup_fp32_vs_fp64"] = out["search_ms_fp64"] / out["search_ms_fp32"]
    # the precision form of the contraction: every GEMM with FP32 products and
    # accumulation on the matrix cores (QR and SVD FP64), then the FP64 search on it
    spg.set_gemm_precision(True)
    try:
        torch.cuda.synchronize()
        a = time.perf_counter()
        env32, lz32 = spg.boundary_mps(peps, chi, stream=stream, nonfinite_ok=True)
        torch.cuda.synchronize()
        t32 = time.perf_counter() - a
    finally:
        spg.set_gemm_precision(False)
    T32, _ = spg.env_export(env32)
    sums32 = row_sums(spg.unpack_mps(T32, spg.env_info(env32).bond_dims))
    n = spg.branch_and_bound(env32, M, st, en, lp, stream=stream)
    torch.cuda.synchronize()
    out["boundary_mps_fp32_products"] = {
        "boundary_mps_s": t32, "speedup_vs_fp64": bmps_s / t32, "logZ": finite_or_none(lz32),
        "rows_with_nonpositive_sum": [r for r, v in enumerate(sums32) if not v > 0],
        "n_states_fp64_search": n, "best_energy_fp64_search": float(en[0]) if n > 0 else None}
    del env32
    return out


def gemm_fp32_leg(spg, torch, stream):
    """The precision form of the boundary MPS's contractions: every GEMM of the
    contraction with FP32 operands and FP32 accumulation on the matrix cores
    (QR, SVD and the MPO d-index contractions FP64), against the FP64 GEMMs on
    the same instance: time, log Z, the row sums' signs, and the FP64 search
    on each result (its best energy)."""
    from workloads import config_instance
    out = {}
    for name, chi, M in (("kings8x8_d16", 32, 1024), ("kings12x12_d24", 64, 4096)):
        inst = config_instance(name, 0)
        N = inst.rows * inst.cols
        dev = torch.device("cuda:0")
        st = torch.zeros((M, N), dtype=torch.int32, device=dev)
        en = torch.zeros(M, dtype=torch.float64, device=dev)
        lp = torch.zeros(M, dtype=torch.float64, device=dev)
        peps = spg.build_peps(inst, stream)
        rec = {"workload": f"{name} chi={chi} M={M} (seed 0)"}
        for tag, f32 in (("fp64", False), ("fp32_products", True)):
            spg.set_gemm_precision(f32)
            try:
                spg.boundary_mps(peps, chi, stream=stream, want_logZ=False)     # warm
                torch.cuda.synchronize()
                a = time.perf_counter()
                env, _ = spg.boundary_mps(peps, chi, stream=stream, want_logZ=False)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - a) * 1e3
                try:
                    _, lz = spg.boundary_mps(peps, chi, stream=stream)
                except spg.SpgError:
                    lz = None
            finally:
                spg.set_gemm_precision(False)
            T, _ = spg.env_export(env)
            sums = row_sums(spg.unpack_mps(T, spg.env_info(env).bond_dims))
            n = spg.branch_and_bound(env, M, st, en, lp, stream=stream)
            torch.cuda.synchronize()
            rec[tag] = {"boundary_mps_ms": ms, "logZ": finite_or_none(lz),
                        "rows_with_nonpositive_sum": [r for r, v in enumerate(sums)
                                                      if not v > 0],
                        "best_energy_fp64_search": float(en[0]) if n > 0 else None}
        a64, a32 = rec["fp64"]["logZ"], rec["fp32_products"]["logZ"]
        rec["dlogZ"] = abs(a32 - a64) if (a64 is not None and a32 is not None) else None
        rec["speedup"] = rec["fp64"]["boundary_mps_ms"] / rec["fp32_products"]["boundary_mps_ms"]
        out[name] = rec
    return out


def merge_leg(spg, torch, inst, wl, M, st, en, lp, stream):
    """Merging branches with equal frontiers: the FP64 search on the same
    boundary MPS with and without it, and with droplets collected while
    merging (search-only time, best energy, droplets of the best states)."""
    peps = spg.build_peps(inst, stream)
    env, _ = spg.boundary_mps(peps, wl["chi"], num_sweeps=wl["num_sweeps"], precision="fp64",
                              oversample=wl["oversample"], power_iters=wl["power_iters"],
                              stream=stream, want_logZ=False)
    res = {}
    # droplets: the paper's example cut-offs (energy 10, Hamming 5), 16 per state
    drop = (10.0, 5, 16)
    for label, merge, dl in (("plain", False, None), ("merged", True, None),
                             ("droplets", True, drop)):
        spg.branch_and_bound(env, M, st, en, lp, stream=stream, merge_branches=merge, droplets=dl)
        torch.cuda.synchronize()
        a = time.perf_counter()
        n = spg.branch_and_bound(env, M, st, en, lp, stream=stream, merge_branches=merge,
                                 droplets=dl)
        torch.cuda.synchronize()
        res[f"search_ms_{label}"] = (time.perf_counter() - a) * 1e3
        res[f"best_energy_{label}"] = float(en[0]) if n > 0 else None
        res[f"n_states_{label}"] = n
    if n > 0:
        counts, gaps = [], []
        for i in range(min(n, 64)):
            _, de = spg.droplets(env, i)
            counts.append(len(de))
            gaps.extend((de - float(en[i])).tolist())
        res["droplet_cutoffs"] = {"energy": drop[0], "hamming": drop[1], "max_per_state": drop[2]}
        res["droplets_of_best_state"] = counts[0]
        res["droplets_best_64_states"] = int(sum(counts))
        res["droplet_gap_range"] = [min(gaps), max(gaps)] if gaps else None
        _, de0 = spg.droplets(env, 0)
        res["best_state_droplet_energies"] = [round(float(x), 6) for x in de0]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32",
                    help="search-contraction precision of the timed (mixed) path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--verbose", action="store_true", help="progress lines on stderr")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="skip the pass with per-launch HIP events (no roofline; for counter runs)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batching and learned-proposal legs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 256 MiB device-to-device (a known-size kernel for "
                         "scaling hardware byte counters)")
    ap.add_argument("--leg", choices=["kings12x12_d24", "kings16x16_d256"], default=None,
                    help="run only this workload leg and print its record (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the hot path of one instance per GPU); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2502_02317_amd import spg
    from workloads import config_instance

    def say(msg):
        if args.verbose:
            print(f"bench: {msg}", file=sys.stderr, flush=True)

    if args.leg is not None:
        stream = torch.cuda.current_stream()
        leg = kings12_leg if args.leg == "kings12x12_d24" else kings16_leg
        print(json.dumps({"leg": args.leg, args.leg: leg(spg, torch, stream)}), flush=True)
        return

    wl = WORKLOAD
    inst = config_instance(wl["name"], wl["seed"])
    R, C, d, M = inst.rows, inst.cols, inst.d, wl["max_states"]
    N = R * C
    dev = torch.device("cuda:0")
    st = torch.zeros((M, N), dtype=torch.int32, device=dev)
    en = torch.zeros(M, dtype=torch.float64, device=dev)
    lp = torch.zeros(M, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(prec):
        peps = spg.build_peps(inst, stream)
        env, _ = spg.boundary_mps(peps, wl["chi"], num_sweeps=wl["num_sweeps"], precision=prec,
                                  oversample=wl["oversample"], power_iters=wl["power_iters"],
                                  stream=stream, want_logZ=False)
        n = spg.branch_and_bound(env, M, st, en, lp, stream=stream)
        return env, n

    def timed(prec, profile):
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        spg.profile_reset()
        spg.profile_enable(profile)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            step(prec)
            if args.verbose:
                torch.cuda.synchronize()
                say(f"{prec} step {i + 1}/{args.steps}")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        spg.profile_enable(False)
        prof = {k: spg.profile_query(k) for k in spg.KERNEL_CLASSES}
        spg.profile_reset()
        return (t1 - t0) * 1e3 / args.steps, prof

    ev = evals_per_step(R, C, d, M)
    # the FP64 plain path (the value) and the mixed path (the precision form:
    # FP32 or BF16-input search contractions), same workload, timed without
    # per-kernel events; then the kernel classes of each from a separate
    # profiled pass (events on each launch's stream) over the same number of steps
    mixed = args.precision != "fp64"
    ms = timed("fp64", False)[0]
    say(f"timed fp64: {ms:.1f} ms/step")
    msmix = timed(args.precision, False)[0] if mixed else ms
    if args.no_kernel_timing:
        prof = {k: (0, 0.0, 0.0) for k in spg.KERNEL_CLASSES}
        prof_mix = prof
    else:
        _, prof = timed("fp64", True)
        prof_mix = timed(args.precision, True)[1] if mixed else prof
        say("profiled passes done")
    env_last, n_last = step("fp64")
    dims_last = spg.env_info(env_last).bond_dims.reshape(R, C + 1)
    best_E = float(en[0]) if n_last > 0 else None     # None: the beam ended with no finite state
    _, n_mix = step(args.precision)
    best_E_mix = float(en[0]) if n_mix > 0 else None

    # search-only and boundary-MPS-only split of the FP64 path (untimed, same work)
    peps = spg.build_peps(inst, stream)
    torch.cuda.synchronize()
    a = time.perf_counter()
    env64, _ = spg.boundary_mps(peps, wl["chi"], num_sweeps=wl["num_sweeps"], precision="fp64",
                                oversample=wl["oversample"], power_iters=wl["power_iters"],
                                stream=stream, want_logZ=False)
    torch.cuda.synchronize()
    b = time.perf_counter()
    spg.branch_and_bound(env64, M, st, en, lp, stream=stream)
    torch.cuda.synchronize()
    c = time.perf_counter()
    env = env64
    search_ms_mix = None
    if mixed:
        env, _ = spg.boundary_mps(peps, wl["chi"], num_sweeps=wl["num_sweeps"],
                                  precision=args.precision, oversample=wl["oversample"],
                                  power_iters=wl["power_iters"], stream=stream, want_logZ=False)
        spg.branch_and_bound(env, M, st, en, lp, stream=stream)
        torch.cuda.synchronize()
        a2 = time.perf_counter()
        spg.branch_and_bound(env, M, st, en, lp, stream=stream)
        torch.cuda.synchronize()
        search_ms_mix = (time.perf_counter() - a2) * 1e3

    # dlogP: teacher-forced on the FP64 path's beam (the oracle's search on the
    # GPU's FP64 boundary MPS gives that beam), states with p64 >= 1e-4 max
    say("split done")
    dlogp = None
    dlogp_info = None
    if mixed:
        from oracle.search import beam_search, teacher_forced_condition
        T, _lam = spg.env_export(env64)
        rows = spg.unpack_mps(T, spg.env_info(env64).bond_dims)
        trace = []
        beam_search(inst, rows, M, trace=trace)
        dlogp, n_keep, n_unres, n_unres64 = 0.0, 0, 0, 0
        u_in = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -9}[args.precision]
        for k in range(N):
            cfg_np = trace[k]["cfg"]
            cfg = torch.tensor(cfg_np, dtype=torch.int32, device=dev)
            o64 = torch.empty((cfg.shape[0], d), dtype=torch.float64, device=dev)
            olo = torch.empty_like(o64)
            spg.marginals(env64, k, cfg, o64)
            spg.marginals(env, k, cfg, olo)
            r64, rlo = o64.cpu().numpy(), olo.cpu().numpy()
            keep = r64 >= r64.max(axis=1, keepdims=True) + np.log(1e-4)
            # entries whose value the reduced precision determines (running-error
            # bound on q below 1); the rest are counted as unresolved
            rr, cc = divmod(k, C)
            ks, _kz = teacher_forced_condition(inst, rows, rr, cc, cfg_np)
            n_ops = wl["chi"] ** 2 + d * wl["chi"] * C
            g = 2 * ((C + 2) * u_in + n_ops * 2.0 ** -24)
            tol = g * (ks + _kz[:, None])
            g64 = 2 * n_ops * 2.0 ** -53
            fine = keep & np.isfinite(tol) & (tol <= 1e-3)
            n_keep += int(keep.sum())
            n_unres += int((keep & ~fine).sum())
            n_unres64 += int((keep & ~(g64 * (ks + _kz[:, None]) <= 1e-3)).sum())
            if fine.any():
                dlogp = max(dlogp, float(np.abs(rlo[fine] - r64[fine]).max()))
        if n_keep == n_unres:
            dlogp = None                  # no entry resolved: nothing measured
        dlogp_info = {"entries": n_keep, "not_resolved_to_1e-3_at_this_precision": n_unres,
                      "not_resolved_to_1e-3_even_in_fp64": n_unres64,
                      "floor": "p64 >= 1e-4 max at the parent"}

    dom = max(prof, key=lambda k: prof[k][1])
    if prof[dom][1] == 0.0:
        dom = "qr_f64"
    cnt, tms, work = prof[dom]
    if tms <= 0.0:
        roof = {"bound": None, "achieved": None, "peak": None, "unit": None}
    elif dom in FLOP_CLASSES:
        achieved = work / (tms * 1e-3) / 1e12
        # the QR kernels run on the FP64 vector ALU, the GEMMs on the FP64
        # matrix cores (the two share one peak on this chip)
        bound = "alu" if dom in ("qr_f64", "qform_f64") else "mfma"
        roof = {"bound": bound, "achieved": achieved, "peak": PEAK["fp64"], "unit": "TFLOP/s"}
    elif dom in BYTE_CLASSES:
        achieved = work / (tms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_GBs"], "unit": "GB/s"}
    else:
        roof = {"bound": "latency", "achieved": None, "peak": None, "unit": None}
    roof["frac"] = roof["achieved"] / roof["peak"] if roof["achieved"] is not None else None
    roof["traffic"] = committed_traffic(CLASS_KERNEL[dom], "kings8x8_d16")
    roof["kernel"] = CLASS_KERNEL[dom]
    roof["kernel_class"] = dom
    roof["launches_per_step"] = cnt / args.steps
    roof["avg_launch_us"] = tms * 1e3 / max(cnt, 1)
    if dom == "qr_f64" and prof.get("qform_f64", (0, 0.0, 0.0))[1] > 0.0:
        # the factorisation and the Q formation of the same QRs together (the
        # accounting of a QR with Q in one kernel)
        qc_, qt_, qw_ = prof["qform_f64"]
        both = (work + qw_) / ((tms + qt_) * 1e-3) / 1e12
        roof["qr_with_q_formation"] = {"achieved": both, "frac": both / PEAK["fp64"],
                                       "kernels": ["k_qr_reg", "k_qform"]}
    if dom in ("qr_f64", "qform_f64", "jacobi_svd_f64") and roof["frac"] is not None:
        # one workgroup per launch at these panel sizes: the rate against the
        # peak of the one compute unit it occupies (256 on the chip)
        roof["workgroups_per_launch"] = 1
        roof["frac_of_one_cu"] = roof["frac"] * 256

    # the matrix-core product of the reduced-precision search (U = R A^T over
    # all ancestors of a row), against the dense MFMA peak of its input type
    mfma = None
    if mixed and prof_mix.get("u_mfma", (0, 0.0, 0.0))[1] > 0.0:
        mc, mt, mw = prof_mix["u_mfma"]
        ach = mw / (mt * 1e-3) / 1e12
        mfma = {"kernel": "k_u_mfma<float>" if args.precision == "fp32"
                else "k_u_mfma<unsigned short>",
                "instruction": "v_mfma_f32_16x16x4_f32" if args.precision == "fp32"
                else "v_mfma_f32_16x16x16_bf16",
                "achieved": ach, "peak": PEAK[args.precision], "unit": "TFLOP/s",
                "frac": ach / PEAK[args.precision], "launches_per_step": mc / args.steps,
                "avg_launch_us": mt * 1e3 / max(mc, 1)}

    # the metric's contraction TFLOP/s: formula flops over summed kernel time
    # (profiled passes), for the search contractions (FP64 path and mixed
    # path) and for the boundary MPS
    search_cls = ("right_env", "marginals", "beam_update", "u_mfma")
    bmps_cls = ("gemm_f64", "qr_f64", "qform_f64", "jacobi_svd_f64", "normalize_box")
    s_fl = search_formula_flops(dims_last, R, C, d, M)
    b_ms = sum(prof[k][1] for k in bmps_cls if k in prof) / args.steps
    b_fl = (prof["gemm_f64"][2] + prof["qr_f64"][2] + prof["qform_f64"][2]) / args.steps

    def search_rate(pr, precision):
        sm = sum(pr[k][1] for k in search_cls if k in pr) / args.steps
        return {"formula_flops": s_fl, "kernel_ms": sm,
                "tflops": s_fl / (sm * 1e-3) / 1e12 if sm > 0 else None, "precision": precision}

    contraction = {
        "search": search_rate(prof, "fp64"),
        "search_mixed": search_rate(prof_mix, args.precision) if mixed else None,
        "boundary_mps": {"gemm_qr_flops": b_fl, "kernel_ms": b_ms,
                         "tflops": b_fl / (b_ms * 1e-3) / 1e12 if b_ms > 0 else None,
                         "precision": "fp64"}}

    out = {
        "metric": "conditional-marginal evals/s", "value": ev / (ms * 1e-3), "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "kings8x8_d16 beta=2 chi=32 M=1024 (seed 0)", "rows": R, "cols": C,
                   "d": d, "chi": wl["chi"], "max_states": M, "num_sweeps": wl["num_sweeps"],
                   "evals_per_step": ev, "search_precision": "fp64",
                   "boundary_mps_precision": "fp64"},
        "mixed": {"value": ev / (msmix * 1e-3), "ms_per_step": msmix,
                  "dtype": {"fp64": "f64", "fp32": "f64+f32", "bf16": "f64+bf16"}[args.precision],
                  "search_precision": args.precision, "search_ms": search_ms_mix,
                  "search_speedup_vs_fp64": ((c - b) * 1e3 / search_ms_mix
                                             if search_ms_mix else None),
                  "dlogP": dlogp, "dlogP_coverage": dlogp_info, "best_energy": best_E_mix,
                  "matrix_cores": mfma},
        "best_energy": best_E,
        "split": {"boundary_mps_ms": (b - a) * 1e3, "search_ms": (c - b) * 1e3,
                  "search_evals_per_s": ev / (c - b)},
        "kernels": {k: {"launches": v[0], "ms": v[1], "work": v[2]} for k, v in prof.items()},
        "roofline": roof,
        "contraction_tflops": contraction,
    }
    prop8 = None
    if not args.no_forms:
        say("mixed precision + learned proposal")
        j8, prop8 = j1_leg(spg, torch, "kings8x8_d16", wl["chi"], M, M, 4, 3, stream)
        j12, _ = j1_leg(spg, torch, "kings12x12_d24", 64, 4096, 1024, 2, 1, stream)
        out["forms"] = {"mixed_learned_proposal": {"kings8x8_d16": j8, "kings12x12_d24": j12},
                        "batching": batching_leg(spg, torch, stream)}
        say("kings12x12_d24")
        out["kings12x12_d24"] = kings12_leg(spg, torch, stream)
        say("boundary MPS with FP32 products")
        out["forms"]["boundary_mps_fp32_products"] = gemm_fp32_leg(spg, torch, stream)
        out["extensions"] = {"lattice_transforms": transforms_leg(spg, torch, inst, wl, M,
                                                                  stream),
                             "merge_branches": merge_leg(spg, torch, inst, wl, M, st, en, lp,
                                                         stream)}
        say("kings16x16_d256")
        try:
            out["kings16x16_d256"] = kings16_leg(spg, torch, stream)
        except (spg.SpgError, RuntimeError) as e:       # reported, not fatal to the line
            out["kings16x16_d256"] = {"error": str(e)}
    # validity of the contraction and of the search on this workload: the
    # GPU's log Z, the sign of every row function's sum, and (with the CPU
    # leg) the oracle's own result beside the GPU's, plus the GPU search run
    # on the oracle's boundary MPS (search parity at full size)
    say("validity")
    peps_v = spg.build_peps(inst, stream)
    try:
        env_v, lz_gpu = spg.boundary_mps(peps_v, wl["chi"], num_sweeps=wl["num_sweeps"],
                                         precision="fp64", oversample=wl["oversample"],
                                         power_iters=wl["power_iters"], stream=stream)
    except spg.SpgError:
        lz_gpu = None                     # the row-0 function's sum is not positive
        env_v, _ = spg.boundary_mps(peps_v, wl["chi"], num_sweeps=wl["num_sweeps"],
                                    precision="fp64", oversample=wl["oversample"],
                                    power_iters=wl["power_iters"], stream=stream,
                                    want_logZ=False)
    Tv, _ = spg.env_export(env_v)
    sums_gpu = row_sums(spg.unpack_mps(Tv, spg.env_info(env_v).bond_dims))
    n_v = spg.branch_and_bound(env_v, M, st, en, lp, stream=stream)
    validity = {"gpu_logZ": finite_or_none(lz_gpu),
                "gpu_rows_with_nonpositive_sum": [r for r, v in enumerate(sums_gpu) if not v > 0],
                "gpu_n_states": n_v,
                "gpu_best_energy": float(en[0]) if n_v > 0 else None}
    if not args.no_cpu:
        say("cpu baseline")
        cb = cpu_baseline(inst, wl)
        A_ora = cb.pop("_oracle_A")
        out["cpu_baseline"] = cb
        T_o, dims_o = spg.pack_oracle_mps(A_ora, wl["chi"], d)
        env_o = spg.env_import(spg.build_peps(inst, stream), wl["chi"], dims_o, T_o,
                               np.zeros(R))
        n_o = spg.branch_and_bound(env_o, M, st, en, lp, stream=stream)
        validity.update({
            "oracle_logZ": cb["oracle_logZ"],
            "oracle_rows_with_nonpositive_sum": cb["oracle_rows_with_nonpositive_sum"],
            "oracle_best_energy": cb["oracle_best_energy"],
            "gpu_search_on_oracle_bmps_best_energy": float(en[0]) if n_o > 0 else None,
            "gpu_search_on_oracle_bmps_n_states": n_o})
        if prop8 is not None:
            # the mixed + learned-proposal search on the oracle's boundary MPS
            env_o32 = spg.env_import(spg.build_peps(inst, stream), wl["chi"], dims_o, T_o,
                                     np.zeros(R), precision="fp32")
            n_j = spg.branch_and_bound(env_o32, M, st, en, lp, stream=stream, proposal=prop8,
                                       kappa=2.0)
            validity["mixed_proposal_search_on_oracle_bmps_best_energy"] = (
                float(en[0]) if n_j > 0 else None)
    out["validity"] = validity
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
