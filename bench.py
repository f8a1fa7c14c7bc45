"""Benchmark: factor-to-variable message updates per second and query latency of belief
propagation on one MI355X, batched FP32 vs plain FP64.

Workload: the SmartFL-shaped graph. It has 200,000 binary variables in 500 layers, one
deterministic AND/OR/NOT factor per variable over 1-4 predecessors (Zipf), Beta(9,1) priors and a
forward-backward (TOPO) ranked schedule. The dependency analysis splits it into 998 levels. It runs
with tol 1e-6 and up to 500 iterations.

A query clamps 2% of the variables to a consistent world (a different seeded set per query),
starts from uniform messages and runs until the residual falls below tol or max_iters is reached.
It then reads back the marginals. Most evidence sets keep the forward-backward schedule
oscillating, so those queries run to max_iters.

* step (timed): a batch of --batch queries submitted together to the FP32 continuous-batching
  server (one workgroup per running query, --step-iters iterations per launch, queries retire as
  they finish). `value` is the FP32 message updates per second over the timed steps.
* plain FP64: --fp64-queries of the same queries, one after another, each a single-graph FP64 run.
* solo FP32: the first query alone (unbatched FP32), for the latency of one query.
* roofline: the persistent kernel of the batched steps. Its algorithmic bytes (the library's exact
  per-iteration count times iterations, summed over queries) are divided by the summed kernel time,
  measured with HIP events on the server's stream.
* cpu_baseline: the FP64 oracle on one host thread, a bounded number of full iterations of the same
  graph and schedule.

Prints one JSON line on stdout; progress goes to stderr.
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

# Measured HBM traffic of one k_persistent launch in the default configuration (512 queries, 8
# iterations per launch), from rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a plain copy's readings
# (profiles/k_persistent_smartfl_200k_batch512.md). Valid only for the kernel sources it was taken
# with: any change to them makes the reported traffic null until it is measured again.
TRAFFIC_DEFAULT = {"sources_sha256": "31b4714cb3264526fd0ef41714495d8f5ea68d711170594680c817201346c7b0",
                   "bytes_per_launch": 206388724709.6, "raw_bytes_per_launch": 126011867136.0,
                   "queries": 512, "step_iters": 8}


def kernel_sources_sha256() -> str:
    import hashlib
    import glob
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2509_22337_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(*a):
    print("#", *a, file=sys.stderr, flush=True)


def query_evidence(w, q):
    """Evidence of query q: the workload's own clamps for q = 0, another seeded 2% set otherwise."""
    from paper_2509_22337_amd import workloads as W
    ev = w.evidence if q == 0 else W.smartfl_evidence(w, seed=1000 + q)
    v = np.flatnonzero(ev >= 0).astype(np.int32)
    return v, ev[v].astype(np.int8)


def batched_steps(F, w, queries, steps, warmup, step_iters):
    """Continuous-batching FP32 server, all queries of a step submitted at once."""
    import torch
    base = F.Graph.from_workload(w, precision="fp32", executor="persistent")
    handles = [base] + [base.clone() for _ in range(len(queries) - 1)]
    srv = F.Server(precision="fp32", max_active=len(queries), step_iters=step_iters)
    lat, updates, iters, alg_bytes = [], 0, [], 0.0
    k0 = None
    for s in range(warmup + steps):
        if s == warmup:
            torch.cuda.synchronize()
            st0 = srv.stats()
            t_start = time.perf_counter()
        for h in handles:
            h.messages_reset()
            h.evidence_clear()
        tickets = [srv.submit(h, v, x, w.max_iters, w.tol, w.damping) for h, (v, x) in zip(handles, queries)]
        res = [srv.wait(t) for t in tickets]
        if s >= warmup:
            for _, st, l in res:
                lat.append(l)
                updates += st["message_updates"]
                iters.append(st["iterations"])
                alg_bytes += st["algorithmic_bytes_per_iter"] * st["iterations"]
        log(f"batched step {s}: {max(r[2] for r in res):.1f} ms, iterations {sorted(r[1]['iterations'] for r in res)[::8]}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    st1 = srv.stats()
    srv.close()
    for h in handles:
        h.close()
    kernel_ms = st1["kernel_ms"] - st0["kernel_ms"]
    launches = st1["steps"] - st0["steps"]
    return dict(wall_s=wall, lat_ms=lat, updates=updates, iters=iters, alg_bytes=alg_bytes, kernel_ms=kernel_ms,
                launches=launches)


def sequential_queries(F, w, queries, precision):
    import torch
    g = F.Graph.from_workload(w, precision=precision)
    lat, updates, iters, dev_ms = [], 0, [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for v, x in queries:
        t0 = time.perf_counter()
        g.messages_reset()
        g.evidence_clear()
        g.evidence_set(v, x)
        st = g.run(w.max_iters, w.tol, w.damping)
        g.marginals()
        lat.append((time.perf_counter() - t0) * 1e3)
        updates += st["message_updates"]
        iters.append(st["iterations"])
        dev_ms.append(st["device_ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    g.close()
    return dict(wall_s=wall, lat_ms=lat, updates=updates, iters=iters, device_ms=dev_ms)


def serving_mix(F, W, args):
    """The serving mix: graphs of log-uniform size (half Datalog-, half SmartFL-shaped) arriving as
    a Poisson process; when a query completes, it is re-submitted warm with 1-10 new clamps. The
    batched FP32 server takes the arrivals as they come; the plain FP64 side runs a prefix of the same
    query list one run at a time (cold then warm re-query), without arrivals."""
    import torch
    qs = W.serving_mix(args.seed, num_queries=args.queries)
    log(f"serving mix: {len(qs)} graphs, {sum(q.graph.num_vars for q in qs)} variables, "
        f"{sum(q.graph.num_edges for q in qs)} edges, last arrival {qs[-1].arrival_s:.2f} s")
    t0 = time.perf_counter()
    hs = [F.Graph.from_workload(q.graph, precision="fp32") for q in qs]
    log(f"created {len(hs)} fp32 handles in {time.perf_counter() - t0:.1f} s")
    for h in hs:
        h.evidence_clear()
    srv = F.Server(precision="fp32", max_active=args.batch, step_iters=args.step_iters)
    torch.cuda.synchronize()
    st0 = srv.stats()
    pending = {}
    res = []
    nq = len(qs)
    nxt = 0
    t_start = time.perf_counter()
    while len(res) < 2 * nq:
        now = time.perf_counter() - t_start
        while nxt < nq and qs[nxt].arrival_s <= now:
            q = qs[nxt]
            pending[srv.submit(hs[nxt], q.ev_vars, q.ev_vals, q.graph.max_iters, q.graph.tol, q.graph.damping)] = (nxt, 0)
            nxt += 1
        for t in list(pending):
            r = srv.poll(t)
            if r is None:
                continue
            qi, warm = pending.pop(t)
            p1, st, lat = r
            res.append((qi, warm, st, lat))
            if not warm:
                q = qs[qi]
                v, x = W.requery_clamps(q.graph, p1, seed=10_000 + qi)
                pending[srv.submit(hs[qi], v, x, q.graph.max_iters, q.graph.tol, q.graph.damping)] = (qi, 1)
        time.sleep(0.0002)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    st1 = srv.stats()
    srv.close()
    for h in hs:
        h.close()
    upd = sum(r[2]["message_updates"] for r in res)
    alg = sum(r[2]["algorithmic_bytes_per_iter"] * r[2]["iterations"] for r in res)
    cold = [r[3] for r in res if r[1] == 0]
    warm = [r[3] for r in res if r[1] == 1]
    out = dict(mups=round(upd / wall, 1), wall_s=round(wall, 3), runs=len(res), queries_per_s=round(len(res) / wall, 2),
               p50_ms=pct([r[3] for r in res], 50), p99_ms=pct([r[3] for r in res], 99),
               cold_p50_ms=pct(cold, 50), cold_p99_ms=pct(cold, 99), warm_p50_ms=pct(warm, 50),
               warm_p99_ms=pct(warm, 99),
               iterations_p50=int(np.median([r[2]["iterations"] for r in res])),
               levels_executor_runs=int(sum(r[2]["executor"] == F.EXEC_LEVELS for r in res)),
               kernel_ms=st1["kernel_ms"] - st0["kernel_ms"], steps=st1["steps"] - st0["steps"],
               algorithmic_bytes=alg, updates=upd)
    log(f"serving fp32: {out['runs']} runs in {wall:.2f} s, {upd / wall / 1e6:.1f} M updates/s, "
        f"p50 {out['p50_ms']} ms p99 {out['p99_ms']} ms")
    # plain FP64: the first fp64_queries graphs, each a cold run then its warm re-query, one at a time
    lat64, upd64, t64 = [], 0, 0.0
    for qi in range(min(args.fp64_queries, nq)):
        q = qs[qi]
        g = F.Graph.from_workload(q.graph, precision="fp64")
        g.evidence_clear()
        for warm in (0, 1):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            if warm:
                v, x = W.requery_clamps(q.graph, p1, seed=10_000 + qi)
            else:
                v, x = q.ev_vars, q.ev_vals
            g.evidence_set(v, x)
            st = g.run(q.graph.max_iters, q.graph.tol, q.graph.damping)
            p1 = g.marginals()
            dt = time.perf_counter() - ta
            lat64.append(dt * 1e3)
            upd64 += st["message_updates"]
            t64 += dt
        g.close()
    out["plain_fp64"] = dict(mups=round(upd64 / t64, 1), runs=len(lat64), p50_ms=pct(lat64, 50),
                             p99_ms=pct(lat64, 99), note="service time of each run alone, no queueing")
    return out


def flooding_runs(F, w, prec, steps, warmup, iters, label):
    """`steps` timed cold runs of `iters` flooding iterations on the LEVELS executor."""
    import torch
    g = F.Graph.from_workload(w, precision=prec, executor="levels")
    for s in range(warmup + steps):
        if s == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dev_ms, upd, alg = 0.0, 0, 0.0
        g.messages_reset()
        st = g.run(iters, 0.0, 0.0)
        if s >= warmup:
            dev_ms += st["device_ms"]
            upd += st["message_updates"]
            alg += st["algorithmic_bytes_per_iter"] * st["iterations"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.close()
    r = dict(wall_s=wall, dev_ms=dev_ms, updates=upd, alg=alg, iters=st["iterations"], steps=steps,
             mups=round(upd / wall, 1), us_per_iteration=round(dev_ms * 1e3 / (steps * st["iterations"]), 2))
    log(f"{label} {prec}: {wall * 1e3 / steps:.1f} ms/run, {upd / wall / 1e9:.2f} G updates/s, "
        f"{r['us_per_iteration']:.1f} us/iteration")
    return r


def bingo_flooding(F, W, args, terms=False):
    """One BINGO-shaped graph (2M tuples, 4M rules, 19M edges), flooding, FP32 messages, on the
    LEVELS executor: per iteration one launch per degree bucket and phase. A step is one run of
    --max-iters (default 100) iterations; FP64 runs the same graph for the plain comparison.
    terms: the 4M rule factors given as weighted terms (Eq.(4)) instead of AND factors; the typed
    graph's FP32 time is reported beside it."""
    w = W.config("C3", seed=args.seed)
    iters = args.max_iters or 100
    typed = None
    if terms:
        typed = flooding_runs(F, w, "fp32", args.steps, args.warmup, iters, "bingo typed")
        w = W.as_terms(w)
    log(f"workload bingo{'-terms' if terms else ''}: V={w.num_vars} F={w.num_factors} E={w.num_edges} "
        f"(non-prior {w.nonprior_edges()})")
    res = {prec: flooding_runs(F, w, prec, args.steps if prec == "fp32" else 1, args.warmup, iters, "bingo")
           for prec in ("fp32", "fp64")}
    r = res["fp32"]
    achieved = r["alg"] / (r["dev_ms"] / 1e3) / 1e9
    name = "bingo_2M_tuples_4M_rules_19M_edges_flooding" + ("_rules_as_weighted_terms" if terms else "")
    out = {
        "metric": "message updates/sec (f->v) + p50/p99 query latency, batched FP32 vs plain FP64 BP",
        "value": round(r["updates"] / r["wall_s"], 1), "unit": "message updates/s", "n_gpus": 1,
        "steps": r["steps"], "warmup": args.warmup, "ms_per_step": round(r["wall_s"] * 1e3 / r["steps"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "seed": args.seed, "num_vars": w.num_vars, "num_edges": w.num_edges,
                   "iterations": iters, "executor": "levels"},
        "us_per_iteration": r["us_per_iteration"],
        "plain_fp64": {"mups": res["fp64"]["mups"], "us_per_iteration": res["fp64"]["us_per_iteration"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                     "kernel": "one iteration of the LEVELS executor (all kernels)"},
    }
    if typed:
        out["typed_fp32"] = {"mups": typed["mups"], "us_per_iteration": typed["us_per_iteration"]}
        out["terms"] = int(len(w.term_weight))
    return out


def bingo_large(F, W, args):
    """One BINGO-shaped graph ten times the size of the flooding one (20M tuples, 40M rules, 190M
    edges) under an ordered-group schedule of 64 classes by head position, FP32 messages, tol 1e-6,
    up to 200 iterations (--max-iters overrides), on the LEVELS executor. A step is one cold run."""
    import torch
    t0 = time.perf_counter()
    w = W.config("C5", seed=args.seed)
    iters = args.max_iters or w.max_iters
    log(f"workload bingo-large: V={w.num_vars} F={w.num_factors} E={w.num_edges}, generated in "
        f"{time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    g = F.Graph.from_workload(w, precision="fp32", executor="levels")
    log(f"created in {time.perf_counter() - t0:.1f} s")
    del w
    dev_ms, upd, alg, its = 0.0, 0, 0.0, []
    for s in range(args.warmup + args.steps):
        if s == args.warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        g.messages_reset()
        st = g.run(iters, 1e-6, 0.0)
        log(f"run {s}: {st['iterations']} iterations, converged {st['converged']}, residual {st['residual']:.3g}, "
            f"{st['device_ms']:.1f} ms")
        if s >= args.warmup:
            dev_ms += st["device_ms"]
            upd += st["message_updates"]
            alg += st["algorithmic_bytes_per_iter"] * st["iterations"]
            its.append(st["iterations"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    levels = st["levels"]
    g.close()
    achieved = alg / (dev_ms / 1e3) / 1e9
    return {
        "metric": "message updates/sec (f->v) + p50/p99 query latency, batched FP32 vs plain FP64 BP",
        "value": round(upd / wall, 1), "unit": "message updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "bingo_20M_tuples_40M_rules_190M_edges_64_ordered_groups", "seed": args.seed,
                   "levels": levels, "max_iters": iters, "tol": 1e-6, "executor": "levels"},
        "iterations": its, "us_per_iteration": round(dev_ms * 1e3 / sum(its), 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                     "kernel": "one iteration of the LEVELS executor (all kernels)"},
    }


def alarm_ranking(F, W, args):
    """BINGO's alarm-ranking loop (fastlbp_alarm_loop) on a BINGO-shaped derivation graph (68K
    variables, 188K edges, args.alarms alarms) with a sampled ground truth. A step is one whole loop
    (until every true alarm is inspected), cold, under BINGO's round-robin asynchronous order (SEQFIX,
    FP32 messages); each round runs at most 500 iterations, tol 1e-6. The same loop also runs once
    under flooding (synchronous) in FP32 and under SEQFIX in FP64, for the ranking metrics of
    Section 5.3 (inversions, Rank-100%-T, Rank-90%-T)."""
    import torch
    w = W.alarm_graph(args.seed, num_alarms=args.alarms)
    iters = args.max_iters or 500
    total_true = int(w.labels.sum())
    log(f"workload alarms: V={w.num_vars} F={w.num_factors} E={w.num_edges}, {len(w.alarms)} alarms, "
        f"{total_true} true")
    seq = W.seqfix_ranks(w)
    res = {}
    for name, prec, sched, steps in (("seqfix_fp32", "fp32", "seqfix", args.steps),
                                      ("flooding_fp32", "fp32", "flooding", 1), ("seqfix_fp64", "fp64", "seqfix", 1)):
        g = F.Graph.from_workload(w, precision=prec)
        if sched == "seqfix":
            g.schedule_set(F.SCHED_RANKED, seq)
        for s in range(args.warmup + steps):
            if s == args.warmup:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                dev_ms, upd, rounds, alg = 0.0, 0, 0, 0.0
            g.evidence_clear()
            g.messages_reset()
            order, _, st = g.alarm_loop(w.alarms, w.labels, max_rounds=None if s >= args.warmup else 2,
                                        max_iters=iters, tol=1e-6, damping=0.0)
            if s >= args.warmup:
                dev_ms += st["device_ms"]
                upd += st["message_updates"]
                rounds += st["rounds"]
                alg += st["algorithmic_bytes"]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lv = g.schedule_levels().max() + 1 if sched == "seqfix" else 1
        g.close()
        lab = w.labels[order]
        res[name] = dict(rounds=int(st["rounds"]), iterations=int(st["iterations"]),
                         inversions=F.inversion_count(lab), rank_100=F.rank_of_fraction(lab, 1.0, total_true),
                         rank_90=F.rank_of_fraction(lab, 0.9, total_true), mups=round(upd / wall, 1),
                         ms_per_round=round(wall * 1e3 / max(1, rounds), 3), levels=int(lv),
                         wall_s=wall, dev_ms=dev_ms, steps=steps, updates=upd, alg=alg)
        log(f"{name}: {res[name]['rounds']} rounds, inversions {res[name]['inversions']}, Rank-100%-T "
            f"{res[name]['rank_100']}, Rank-90%-T {res[name]['rank_90']}, {res[name]['ms_per_round']:.2f} ms/round, "
            f"{upd / wall / 1e9:.3f} G updates/s")
    r = res["seqfix_fp32"]
    return w, {
        "metric": "message updates/sec (f->v) + p50/p99 query latency, batched FP32 vs plain FP64 BP",
        "value": r["mups"], "unit": "message updates/s", "n_gpus": 1, "steps": r["steps"], "warmup": args.warmup,
        "ms_per_step": round(r["wall_s"] * 1e3 / r["steps"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"alarm_ranking_68k_vars_188k_edges_{len(w.alarms)}_alarms_seqfix", "seed": args.seed,
                   "alarms": len(w.alarms), "true_alarms": total_true, "max_iters": iters, "tol": 1e-6,
                   "levels": r["levels"]},
        "ranking": {k: {f: v[f] for f in ("rounds", "iterations", "inversions", "rank_100", "rank_90", "mups",
                                          "ms_per_round", "levels")} for k, v in res.items()},
        "plain_fp64": {"mups": res["seqfix_fp64"]["mups"], "ms_per_round": res["seqfix_fp64"]["ms_per_round"]},
        "roofline": {"bound": "hbm", "achieved": round(r["alg"] / (r["dev_ms"] / 1e3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(r["alg"] / (r["dev_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS, 6),
                     "traffic": None, "kernel": "k_persistent (one workgroup, SEQFIX levels) and the alarm picks"},
    }


def alarm_cpu_baseline(w, budget_s: float):
    """The oracle's alarm loop under SEQFIX (single thread) for as many rounds as fit in about
    `budget_s` seconds."""
    import oracle
    seq = np.arange(w.num_edges, dtype=np.int32)
    t0 = time.perf_counter()
    _, _, st = oracle.bp(w, max_iters=1, tol=0.0, ranks=seq)
    one = time.perf_counter() - t0
    it_budget = max(1, int(budget_s / max(one, 1e-6)))
    t0 = time.perf_counter()
    marg, m0, m1, st = oracle.bp_pairs(w, np.full(w.num_edges, 0.5), np.full(w.num_edges, 0.5),
                                       min(500, it_budget), 1e-6, 0.0, ranks=seq)
    dt = time.perf_counter() - t0
    return dict(value=round(st["message_updates"] / dt, 1), unit="message updates/s", cores=1, kind="oracle",
                sample=f"the first round of the loop (SEQFIX, tol 1e-6, at most {min(500, it_budget)} iterations): "
                       f"{st['iterations']} iterations, {st['message_updates']} updates in {dt:.1f} s")


def cpu_baseline(w, budget_s: float):
    """The oracle (single thread) on a bounded sample: as many full iterations of the same graph,
    schedule and evidence as fit in about `budget_s` seconds."""
    import oracle
    t0 = time.perf_counter()
    _, _, st = oracle.bp(w, max_iters=1, tol=0.0)
    one = time.perf_counter() - t0
    n = max(1, int(budget_s / max(one, 1e-6)))
    t0 = time.perf_counter()
    _, _, st = oracle.bp(w, max_iters=n, tol=0.0)
    dt = time.perf_counter() - t0
    return dict(value=round(st["message_updates"] / dt, 1), unit="message updates/s", cores=1, kind="oracle",
                sample=f"{n} full iterations (cold start, tol 0) of the same 200k-variable graph, forward-backward "
                       f"schedule and evidence as query 0: {st['message_updates']} updates in {dt:.1f} s")


def pct(a, q):
    return round(float(np.percentile(a, q)), 3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=512, help="queries per batched step (512: two per compute unit)")
    ap.add_argument("--step-iters", type=int, default=8, help="iterations per server launch")
    ap.add_argument("--fp64-queries", type=int, default=3)
    ap.add_argument("--max-iters", type=int, default=None, help="override the workload's 500")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-only", action="store_true", help="only the batched FP32 steps (profiling)")
    ap.add_argument("--alarms", type=int, default=300, help="alarms of the alarm-ranking workload")
    ap.add_argument("--workload", choices=["smartfl", "serving", "bingo", "bingo-terms", "bingo-large", "alarms"],
                    default="smartfl",
                    help="smartfl: batched queries of the 200k-variable SmartFL-shaped graph; serving: the "
                         "512-graph Poisson serving mix with warm re-queries; bingo: one 19M-edge "
                         "BINGO-shaped graph, flooding, 100 iterations (wide-level kernels); bingo-terms: the "
                         "same with its rule factors given as weighted terms; alarms: BINGO's alarm-ranking "
                         "loop on a 68K-variable derivation graph (SEQFIX vs flooding); bingo-large: "
                         "one 190M-edge BINGO-shaped graph, 64 ordered groups, tol 1e-6, up to 200 iterations")
    ap.add_argument("--queries", type=int, default=512, help="graphs in the serving mix")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 5 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU (got --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        raise SystemExit(2)

    import torch
    if args.copy_calibration:
        n = args.copy_calibration << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n, "copy_calibration_bytes_written": n, "launches": 5}))
        return
    import paper_2509_22337_amd as F
    from paper_2509_22337_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    F.load()
    if args.workload == "alarms":
        w, out = alarm_ranking(F, W, args)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = alarm_cpu_baseline(w, args.cpu_budget)
        print(json.dumps(out), flush=True)
        return
    if args.workload in ("bingo", "bingo-terms"):
        print(json.dumps(bingo_flooding(F, W, args, terms=args.workload == "bingo-terms")), flush=True)
        return
    if args.workload == "bingo-large":
        print(json.dumps(bingo_large(F, W, args)), flush=True)
        return
    if args.workload == "serving":
        rs = serving_mix(F, W, args)
        kernel_s = rs["kernel_ms"] / 1e3
        achieved = rs["algorithmic_bytes"] / kernel_s / 1e9
        out = {
            "metric": "message updates/sec (f->v) + p50/p99 query latency, batched FP32 vs plain FP64 BP",
            "value": rs["mups"], "unit": "message updates/s", "n_gpus": 1, "steps": rs["runs"], "warmup": 0,
            "ms_per_step": round(rs["wall_s"] * 1e3 / max(1, rs["runs"]), 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"serving_mix_{args.queries}_graphs_1k_500k_vars_poisson_200qps_warm_requery",
                       "seed": args.seed, "queries": args.queries, "runs": rs["runs"], "max_active": args.batch,
                       "step_iters": args.step_iters, "max_iters": 100, "tol": 1e-6},
            "serving_fp32": {k: v for k, v in rs.items() if k not in ("plain_fp64",)},
            "plain_fp64": rs["plain_fp64"],
            "batched_fp32_vs_plain_fp64": round(rs["mups"] / rs["plain_fp64"]["mups"], 2),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                         "kernel": "server steps (k_persistent + LEVELS kernels, concurrent)"},
        }
        print(json.dumps(out), flush=True)
        return
    w = W.smartfl(args.seed)
    if args.max_iters:
        w.max_iters = args.max_iters
    queries = [query_evidence(w, q) for q in range(args.batch)]
    log(f"workload smartfl: V={w.num_vars} F={w.num_factors} E={w.num_edges} (non-prior {w.nonprior_edges()}), "
        f"{args.batch} queries per step")

    rb = batched_steps(F, w, queries, args.steps, args.warmup, args.step_iters)
    mups_b = rb["updates"] / rb["wall_s"]
    log(f"batched fp32: {rb['wall_s'] * 1e3 / args.steps:.1f} ms/step, {mups_b / 1e6:.1f} M updates/s")
    out = {
        "metric": "message updates/sec (f->v) + p50/p99 query latency, batched FP32 vs plain FP64 BP",
        "value": round(mups_b, 1),
        "unit": "message updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(rb["wall_s"] * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "smartfl_200k_vars_500_layers_fwd_bwd_ranked", "seed": args.seed,
                   "num_vars": w.num_vars, "num_edges": w.num_edges, "levels": 998, "max_iters": w.max_iters,
                   "tol": w.tol, "queries_per_step": args.batch, "step_iters": args.step_iters,
                   "executor": "persistent, one workgroup per query"},
        "batched_fp32": {"mups": round(mups_b, 1), "device_mups": round(rb["updates"] / (rb["kernel_ms"] / 1e3), 1),
                         "p50_ms": pct(rb["lat_ms"], 50), "p99_ms": pct(rb["lat_ms"], 99),
                         "queries": len(rb["lat_ms"]), "iterations_p50": int(np.median(rb["iters"])),
                         "iterations_max": int(max(rb["iters"]))},
    }
    kernel_s = rb["kernel_ms"] / 1e3
    achieved = rb["alg_bytes"] / kernel_s / 1e9
    T = TRAFFIC_DEFAULT
    traffic = None
    if (args.batch == T["queries"] and args.step_iters == T["step_iters"] and args.seed == 0 and not args.max_iters
            and kernel_sources_sha256() == T["sources_sha256"]):
        traffic = T["bytes_per_launch"]
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                       "traffic_note": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-"
                                       "calibrated); null when the kernel sources or launch shape differ from "
                                       "the profiled ones", "kernel": "k_persistent<PolLog32>",
                       "launches": rb["launches"], "avg_launch_ms": round(rb["kernel_ms"] / max(1, rb["launches"]), 4),
                       "algorithmic_bytes": rb["alg_bytes"]}
    if not args.batched_only:
        r64 = sequential_queries(F, w, queries[:args.fp64_queries], "fp64")
        mups64 = r64["updates"] / r64["wall_s"]
        log(f"plain fp64: {mups64 / 1e6:.2f} M updates/s, iterations {r64['iters']}")
        out["plain_fp64"] = {"mups": round(mups64, 1), "p50_ms": pct(r64["lat_ms"], 50),
                             "p99_ms": pct(r64["lat_ms"], 99), "queries": len(r64["lat_ms"]),
                             "iterations": r64["iters"]}
        r32 = sequential_queries(F, w, queries[:1], "fp32")
        out["solo_fp32"] = {"mups": round(r32["updates"] / r32["wall_s"], 1), "latency_ms": round(r32["lat_ms"][0], 3),
                            "iterations": r32["iters"][0], "device_ms": round(r32["device_ms"][0], 3)}
        out["batched_fp32_vs_plain_fp64"] = round(mups_b / mups64, 2)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
