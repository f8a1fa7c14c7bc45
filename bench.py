"""Benchmark: factor-to-variable message updates per second and query latency of belief
propagation on one MI355X, FP32 log-domain messages vs plain FP64.

A step is one query: cold-start messages, clamp the query's evidence, run the schedule until the
residual falls below tol (or max_iters), read back the marginals. The default workload is the
SmartFL-shaped graph: 200,000 binary variables in 500 layers, one deterministic AND/OR/NOT factor per
variable over 1-4 predecessors, Beta(9,1) priors, 2% observed variables, forward-backward (TOPO)
ranked schedule split into levels by the dependency analysis, tol 1e-6, up to 500 iterations.

Prints one JSON line. `value` is FP32 message updates per second over the timed steps; the FP64
figures, p50/p99 latencies, the roofline of the dominant kernel and the CPU oracle baseline are
extra fields.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def make_workload(name: str, seed: int):
    from paper_2509_22337_amd import workloads as W
    if name == "smartfl":
        return W.smartfl(seed), "smartfl_200k_vars_500_levels_fwd_bwd"
    if name == "datalog":
        return W.datalog(seed), "datalog_2k_tuples_1500_rules_flooding"
    if name == "bingo":
        return W.bingo(seed), "bingo_2M_tuples_4M_rules_flooding"
    raise SystemExit(f"unknown workload {name}")


def run_queries(F, w, precision, steps, warmup, executor="auto"):
    import torch
    g = F.Graph.from_workload(w, precision=precision, executor=executor)
    lat, dev_ms, updates, iters, bytes_it = [], [], 0, [], 0.0
    stats = None
    for i in range(warmup + steps):
        if i == warmup:
            torch.cuda.synchronize()
            t_start = time.perf_counter()
        t0 = time.perf_counter()
        g.messages_reset()
        g.evidence_array(w.evidence)
        st = g.run(w.max_iters, w.tol, w.damping)
        m = g.marginals()
        t1 = time.perf_counter()
        if i >= warmup:
            lat.append((t1 - t0) * 1e3)
            dev_ms.append(st["device_ms"])
            updates += st["message_updates"]
            iters.append(st["iterations"])
            stats = st
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    g.close()
    return dict(wall_s=wall, lat_ms=lat, device_ms=dev_ms, updates=updates, iters=iters, stats=stats, marg=m)


def cpu_baseline(w, budget_s: float):
    """The oracle (single thread) on a bounded sample: as many full iterations of the same
    workload and schedule as fit in about `budget_s` seconds (at least one)."""
    import oracle
    t0 = time.perf_counter()
    _, _, st = oracle.bp(w, max_iters=1, tol=0.0)
    one = time.perf_counter() - t0
    n = max(1, int(budget_s / max(one, 1e-6)))
    t0 = time.perf_counter()
    _, _, st = oracle.bp(w, max_iters=n, tol=0.0)
    dt = time.perf_counter() - t0
    return dict(value=st["message_updates"] / dt, unit="message updates/s", cores=1, kind="oracle",
                sample=f"{n} full iterations of the same graph, schedule and evidence (cold start, tol 0), "
                       f"{dt:.1f} s, single thread")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="smartfl", choices=["smartfl", "datalog", "bingo"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-only", action="store_true", help="skip the FP64 leg (profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        raise SystemExit(2)

    import torch
    import paper_2509_22337_amd as F
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    F.load()
    w, wname = make_workload(args.workload, args.seed)
    print(f"# workload {wname}: V={w.num_vars} F={w.num_factors} E={w.num_edges} "
          f"(non-prior {w.nonprior_edges()})", file=sys.stderr, flush=True)

    r32 = run_queries(F, w, "fp32", args.steps, args.warmup)
    print(f"# fp32: {r32['wall_s']*1e3/args.steps:.2f} ms/query, iters {r32['iters']}", file=sys.stderr, flush=True)
    r64 = None
    if not args.fp32_only:
        r64 = run_queries(F, w, "fp64", args.steps, args.warmup)
        print(f"# fp64: {r64['wall_s']*1e3/args.steps:.2f} ms/query, iters {r64['iters']}", file=sys.stderr,
              flush=True)

    st = r32["stats"]
    mups32 = r32["updates"] / r32["wall_s"]
    # roofline of the dominant kernel (the run's only long kernel): algorithmic bytes of the run's
    # iterations over the device time of the run, HIP events on the library's stream
    bytes_run = st["algorithmic_bytes_per_iter"] * st["iterations"]
    dev_s = float(np.mean(r32["device_ms"])) / 1e3
    achieved = bytes_run / dev_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
            "kernel": "k_persistent" if st["executor"] == F.EXEC_PERSISTENT else "k_fac_thread",
            "bytes_per_launch": bytes_run, "launch_ms": round(dev_s * 1e3, 3)}
    out = {
        "metric": "message updates/sec (f->v), FP32 vs plain FP64; p50/p99 query latency",
        "value": round(mups32, 1),
        "unit": "message updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["wall_s"] * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wname, "seed": args.seed, "num_vars": w.num_vars, "num_edges": w.num_edges,
                   "levels": st["levels"], "max_iters": w.max_iters, "tol": w.tol, "damping": w.damping,
                   "executor": "persistent" if st["executor"] == F.EXEC_PERSISTENT else "levels"},
        "fp32": {"mups": round(mups32, 1), "p50_ms": round(float(np.percentile(r32["lat_ms"], 50)), 3),
                 "p99_ms": round(float(np.percentile(r32["lat_ms"], 99)), 3), "iterations": r32["iters"]},
        "roofline": roof,
    }
    if r64 is not None:
        out["fp64"] = {"mups": round(r64["updates"] / r64["wall_s"], 1),
                       "p50_ms": round(float(np.percentile(r64["lat_ms"], 50)), 3),
                       "p99_ms": round(float(np.percentile(r64["lat_ms"], 99)), 3), "iterations": r64["iters"]}
        out["fp32_vs_fp64_max_abs_marginal_diff"] = float(np.abs(r32["marg"] - r64["marg"]).max())
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
