"""Benchmark of the PEPS branch-and-bound hot path on one MI355X.

Workload: 8x8 king's-graph lattice of 4-spin clusters (d = 16), intra-cluster
couplings and fields ~ N(0,1), inter-cluster +-1 spin couplings, beta = 2,
boundary-MPS bond chi = 32 (one sweep), beam M = 1024; synthetic, seed 0.
One step = the whole hot path on that instance: build the PEPS weights,
contract the boundary MPSs, run the branch-and-bound search.

Metric: conditional-marginal evaluations per second, one evaluation being one
resolved candidate (beam state b, local state s) at one site, so a step does
sum_k min(M, d^k) * d of them.  ``value`` is evaluations / wall time of the
whole step (inputs already on the host; the PEPS build copies them over).

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
FLOP_CLASSES = {"gemm_f64", "qr_f64", "right_env", "marginals", "beam_update"}
BYTE_CLASSES = {"normalize_box", "select_topm"}


def evals_per_step(R, C, d, M):
    tot, B = 0, 1
    for _ in range(R * C):
        tot += B * d
        B = min(M, B * d)
    return tot


def cpu_baseline(inst, wl):
    """The oracle, as it stands, on one step of the same workload."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle.bmps import boundary_mps
    from oracle.search import beam_search
    cores = len(os.sched_getaffinity(0))
    with threadpool_limits(limits=cores):
        info = threadpool_info()
        used = max([i.get("num_threads", 1) for i in info] or [1])
        t0 = time.perf_counter()
        mp = boundary_mps(inst, wl["chi"], num_sweeps=wl["num_sweeps"], p=wl["oversample"],
                          q=wl["power_iters"])
        t1 = time.perf_counter()
        beam_search(inst, mp["A"], wl["max_states"])
        t2 = time.perf_counter()
    ev = evals_per_step(inst.rows, inst.cols, inst.d, wl["max_states"])
    return {"value": ev / (t2 - t0), "unit": "evals/s", "cores": used, "kind": "oracle",
            "sample": f"one full step of the same instance (boundary MPS {t1 - t0:.1f} s + "
                      f"search {t2 - t1:.1f} s)",
            "bmps_s": t1 - t0, "search_s": t2 - t1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the hot path of one instance per GPU); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2502_02317_amd import spg
    from workloads import config_instance

    wl = WORKLOAD
    inst = config_instance(wl["name"], wl["seed"])
    R, C, d, M = inst.rows, inst.cols, inst.d, wl["max_states"]
    N = R * C
    dev = torch.device("cuda:0")
    st = torch.zeros((M, N), dtype=torch.int32, device=dev)
    en = torch.zeros(M, dtype=torch.float64, device=dev)
    lp = torch.zeros(M, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        peps = spg.build_peps(inst, stream)
        env, _ = spg.boundary_mps(peps, wl["chi"], num_sweeps=wl["num_sweeps"],
                                  precision=args.precision, oversample=wl["oversample"],
                                  power_iters=wl["power_iters"], stream=stream, want_logZ=False)
        n = spg.branch_and_bound(env, M, st, en, lp, stream=stream)
        return env, n

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region (kernel classes timed with HIP events on the launch stream)
    spg.profile_reset()
    spg.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        env, n = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    spg.profile_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    ev = evals_per_step(R, C, d, M)
    prof = {k: spg.profile_query(k) for k in spg.KERNEL_CLASSES}
    spg.profile_reset()

    # search-only and boundary-MPS-only split (untimed region, same work)
    peps = spg.build_peps(inst, stream)
    torch.cuda.synchronize()
    a = time.perf_counter()
    env, _ = spg.boundary_mps(peps, wl["chi"], num_sweeps=wl["num_sweeps"], precision=args.precision,
                              oversample=wl["oversample"], power_iters=wl["power_iters"],
                              stream=stream, want_logZ=False)
    torch.cuda.synchronize()
    b = time.perf_counter()
    spg.branch_and_bound(env, M, st, en, lp, stream=stream)
    torch.cuda.synchronize()
    c = time.perf_counter()

    dom = max(prof, key=lambda k: prof[k][1])
    cnt, tms, work = prof[dom]
    if dom in FLOP_CLASSES:
        achieved = work / (tms * 1e-3) / 1e12
        peak = PEAK[args.precision]
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s"}
    elif dom in BYTE_CLASSES:
        achieved = work / (tms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_GBs"], "unit": "GB/s"}
    else:
        roof = {"bound": "latency", "achieved": None, "peak": None, "unit": None}
    if roof["achieved"] is not None:
        roof["frac"] = roof["achieved"] / roof["peak"]
    else:
        roof["frac"] = None
    roof["traffic"] = None
    roof["kernel"] = dom
    roof["launches_per_step"] = cnt / args.steps
    roof["avg_launch_us"] = tms * 1e3 / max(cnt, 1)

    out = {
        "metric": "conditional-marginal evals/s", "value": ev / (ms * 1e-3), "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "kings8x8_d16 beta=2 chi=32 M=1024 (seed 0)", "rows": R, "cols": C,
                   "d": d, "chi": wl["chi"], "max_states": M, "num_sweeps": wl["num_sweeps"],
                   "evals_per_step": ev},
        "split": {"boundary_mps_ms": (b - a) * 1e3, "search_ms": (c - b) * 1e3,
                  "search_evals_per_s": ev / (c - b)},
        "kernels": {k: {"launches": v[0], "ms": v[1], "work": v[2]} for k, v in prof.items()},
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
