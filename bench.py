"""Benchmark: factor-to-variable message updates per second and query latency of belief
propagation on one MI355X, batched FP32 vs plain FP64.

Default workload (--workload serving): 512 graphs of 1k-500k variables (log-uniform), half
Datalog-shaped (flooding, damping 0.5) and half SmartFL-shaped (forward-backward ranked schedule,
2% clamps), arriving as a Poisson process at 200 queries/s; each query is re-submitted warm with
1-10 new clamps when it completes (1,024 runs), tol 1e-6, at most 100 iterations.

* step (timed): one run of the stream on the FP32 continuous-batching server. `value` is the FP32
  message updates of all runs over the wall time of the whole stream (inputs resident; clamps in
  and marginals out cross PCIe inside the timed region).
* plain FP64: a FIFO server running one FP64 graph at a time on the same arrival stream (a prefix
  of the stream), latency including queueing; the FP32 server's latencies on the same prefix.
* fp32_error: FP32 marginals against the FP64 ones of the same runs.
* roofline: the persistent kernel of the server's steps: method bytes of the runs it advanced over
  its launch time (HIP events on the server's stream).
* cpu_baseline: the FP64 oracle on one host thread, cold runs of the prefix's smallest graphs.
* extra: the saturated narrow-level kernel (512 batched queries of the 200k-variable SmartFL-shaped
  graph) and the wide-level kernels (the 19M-edge BINGO-shaped graph, flooding), each with its own
  roofline.

Other workloads: smartfl (batched queries of one graph), bingo, bingo-terms, bingo-large, alarms.
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

# Measured HBM traffic of one k_persistent launch of the batched SmartFL-shaped queries (512 queries,
# 2 to 8 iterations per launch), from rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a plain copy's readings
# (profiles/k_persistent_smartfl_200k_batch512.md). Valid only for the kernel sources it was taken
# with: any change to them makes the reported traffic null until it is measured again.
TRAFFIC_DEFAULT = {"sources_sha256": "098c65e4dd32525c03fb8cb86ef94d48dae4b6352ded41a05be0ec1bb39a436d",
                   "bytes_per_launch": 119237182021.0, "raw_bytes_per_launch": 83470086135.5,
                   "queries": 512, "step_iters": 8}


# The same for the serving configuration (512 graphs, up to 512 active runs): the average k_persistent
# launch of the server (profiles/k_persistent_serving_mix_512_graphs.md; FETCH_SIZE x2.0, WRITE_SIZE
# x1.0, KiB per dispatch averaged over the profiled command's launches). A serving launch holds
# whatever runs are in flight, so the profiled launches carried their own method bytes
# (`method_bytes_per_launch`), listed for comparison with the traffic.
TRAFFIC_SERVING = {"sources_sha256": "098c65e4dd32525c03fb8cb86ef94d48dae4b6352ded41a05be0ec1bb39a436d",
                   "bytes_per_launch": 9051213802, "fetch_bytes_per_launch": 7395182754,
                   "write_bytes_per_launch": 1656031049, "method_bytes_per_launch": 3811734660,
                   "queries": 512, "max_active": 512, "step_iters": 8}


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


def batched_steps(F, w, queries, steps, warmup, step_iters, keep=0):
    """Continuous-batching FP32 server, all queries of a step submitted at once."""
    import torch
    base = F.Graph.from_workload(w, precision="fp32", executor="persistent")
    handles = [base] + [base.clone() for _ in range(len(queries) - 1)]
    srv = F.Server(precision="fp32", max_active=len(queries), step_iters=step_iters)
    lat, updates, iters, alg_bytes, kept = [], 0, [], 0.0, {}
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
        kept = {q: (res[q][0], res[q][1]) for q in range(min(keep, len(res)))}
        if s >= warmup:
            for _, st, l in res:
                lat.append(l)
                updates += st["message_updates"]
                iters.append(st["iterations"])
                alg_bytes += st["method_bytes_per_iter"] * st["iterations"]
        log(f"batched step {s}: {max(r[2] for r in res):.1f} ms, iterations {sorted(r[1]['iterations'] for r in res)[::8]}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    st1 = srv.stats()
    srv.close()
    for h in handles:
        h.close()
    kernel_ms = st1["kernel_ms"] - st0["kernel_ms"]
    launches = st1["steps"] - st0["steps"]
    return dict(wall_s=wall, lat_ms=lat, updates=updates, iters=iters, alg_bytes=alg_bytes, kept=kept, kernel_ms=kernel_ms,
                launches=launches)


def sequential_queries(F, w, queries, precision):
    import torch
    g = F.Graph.from_workload(w, precision=precision)
    lat, updates, iters, dev_ms, margs, conv = [], 0, [], [], [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for v, x in queries:
        t0 = time.perf_counter()
        g.messages_reset()
        g.evidence_clear()
        g.evidence_set(v, x)
        st = g.run(w.max_iters, w.tol, w.damping)
        margs.append(g.marginals())
        conv.append(bool(st["converged"]))
        lat.append((time.perf_counter() - t0) * 1e3)
        updates += st["message_updates"]
        iters.append(st["iterations"])
        dev_ms.append(st["device_ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    g.close()
    return dict(wall_s=wall, lat_ms=lat, updates=updates, iters=iters, device_ms=dev_ms, marginals=margs, converged=conv)


def _replay_fp32(F, W, qs, hs, args, clamps):
    """The batched FP32 server on a stream: each graph's first query is submitted at its arrival
    time; when it completes, its warm re-query (1-10 new clamps, recorded in `clamps` for the plain
    FP64 side) is submitted at once. Returns per-run results and the server's statistics."""
    import torch
    srv = F.Server(precision="fp32", max_active=args.batch, step_iters=args.step_iters)
    torch.cuda.synchronize()
    st0 = srv.stats()
    pending, res, nxt, nq = {}, [], 0, len(qs)
    t_start = time.perf_counter()
    while len(res) < 2 * nq:
        now = time.perf_counter() - t_start
        while nxt < nq and qs[nxt].arrival_s <= now:
            q = qs[nxt]
            t = srv.submit(hs[nxt], q.ev_vars, q.ev_vals, q.graph.max_iters, q.graph.tol, q.graph.damping)
            pending[t] = (nxt, 0)
            nxt += 1
        for t in list(pending):
            r = srv.poll(t)
            if r is None:
                continue
            qi, warm = pending.pop(t)
            p1, st, lat = r
            res.append(dict(q=qi, warm=warm, stats=st, lat_ms=lat, p1=p1 if qi < args.fp64_graphs else None))
            if not warm:
                q = qs[qi]
                v, x = W.requery_clamps(q.graph, p1, seed=10_000 + qi)
                clamps[qi] = (v, x)
                t2 = srv.submit(hs[qi], v, x, q.graph.max_iters, q.graph.tol, q.graph.damping)
                pending[t2] = (qi, 1)
        time.sleep(0.0002)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    st1 = srv.stats()
    srv.close()
    d = {k: st1[k] - st0[k] for k in ("kernel_ms", "steps", "persistent_launches", "persistent_ms",
                                       "persistent_method_bytes", "method_bytes")}
    d.update(evictions=st1["evictions"], restores=st1["restores"], peak_resident_bytes=st1["peak_resident_bytes"])
    return res, wall, d


def _fifo_fp64(F, qs, clamps, n_graphs):
    """Plain FP64 single-graph BP as a FIFO server on the same stream: one run at a time on the GPU
    (fastlbp_run, the executor the library picks for the graph), in arrival order; a graph's warm
    re-query arrives when its first run completes and joins the queue's tail. Latency = completion
    - arrival, queueing included."""
    import torch
    hs = [F.Graph.from_workload(q.graph, precision="fp64") for q in qs[:n_graphs]]
    for h in hs:
        h.evidence_clear()
    torch.cuda.synchronize()
    queue = [(qs[i].arrival_s, i, 0) for i in range(n_graphs)]
    res, upd, busy = [], 0, 0.0
    t_start = time.perf_counter()
    while queue:
        queue.sort()
        arr, qi, warm = queue.pop(0)
        now = time.perf_counter() - t_start
        if arr > now:
            time.sleep(arr - now)
        q = qs[qi]
        v, x = clamps[qi] if warm else (q.ev_vars, q.ev_vals)
        t0 = time.perf_counter()
        hs[qi].evidence_set(v, x)
        st = hs[qi].run(q.graph.max_iters, q.graph.tol, q.graph.damping)
        p1 = hs[qi].marginals()
        t1 = time.perf_counter()
        busy += t1 - t0
        upd += st["message_updates"]
        done = t1 - t_start
        res.append(dict(q=qi, warm=warm, stats=st, lat_ms=(done - arr) * 1e3, service_ms=(t1 - t0) * 1e3, p1=p1))
        if not warm:
            queue.append((done, qi, 1))
    wall = time.perf_counter() - t_start
    for h in hs:
        h.close()
    return res, wall, upd, busy


def _lat(rs, warm=None):
    a = [r["lat_ms"] for r in rs if warm is None or r["warm"] == warm]
    return dict(p50_ms=pct(a, 50), p99_ms=pct(a, 99)) if a else {}


def serving_mix(F, W, args):
    """The serving configuration: 512 graphs with sizes log-uniform in [1k, 500k] variables, half
    Datalog-shaped (flooding, damping 0.5), half SmartFL-shaped (forward-backward ranks, 2%
    clamps), arriving as a Poisson process at 200 queries/s; when a query completes it is
    re-submitted warm with 1-10 new clamps (1,024 runs); tol 1e-6, at most 100 iterations each.

    * batched FP32 (the value): the continuous-batching server on the whole stream.
    * plain FP64: a FIFO server running one FP64 graph at a time with fastlbp_run, on the same
      arrival stream and the same re-query clamps, over the stream's first --fp64-graphs graphs (a
      bounded prefix: the FIFO queue falls behind the arrivals, so running all of it would take
      minutes); the batched FP32 server's latencies on the same prefix are reported beside it.
    * the FP32 error: FP32 marginals against the FP64 ones of the same runs on the prefix (the FP64
      path matches the oracle to 1e-9 in the tests)."""
    qs = W.serving_mix(args.seed, num_queries=args.queries)
    log(f"serving mix: {len(qs)} graphs, {sum(q.graph.num_vars for q in qs)} variables, "
        f"{sum(q.graph.num_edges for q in qs)} edges, last arrival {qs[-1].arrival_s:.2f} s")
    t0 = time.perf_counter()
    hs = [F.Graph.from_workload(q.graph, precision="fp32") for q in qs]
    for h in hs:
        h.evidence_clear()
    log(f"created {len(hs)} fp32 handles in {time.perf_counter() - t0:.1f} s")
    clamps = {}
    res, wall, sd = _replay_fp32(F, W, qs, hs, args, clamps)
    for h in hs:
        h.close()
    upd = sum(r["stats"]["message_updates"] for r in res)
    log(f"batched fp32: {len(res)} runs in {wall:.2f} s, {upd / wall / 1e9:.3f} G updates/s, "
        f"p50 {_lat(res)['p50_ms']} ms p99 {_lat(res)['p99_ms']} ms")
    n64 = min(args.fp64_graphs, len(qs))
    if n64 == 0:  # profiling runs: the batched FP32 server only
        return qs, res, dict(runs=len(res), wall_s=round(wall, 3), mups=round(upd / wall, 1), latency=dict(all=_lat(res)),
                             server=sd, prefix=dict(latency={}), plain_fp64=dict(latency={}), fp32_error={})
    r64, wall64, upd64, busy64 = _fifo_fp64(F, qs, clamps, n64)
    log(f"plain fp64 FIFO on the first {n64} graphs: {len(r64)} runs in {wall64:.2f} s, "
        f"{upd64 / busy64 / 1e6:.1f} M updates/s busy, p50 {_lat(r64)['p50_ms']} ms p99 {_lat(r64)['p99_ms']} ms")
    pre = [r for r in res if r["q"] < n64]
    upd_pre = sum(r["stats"]["message_updates"] for r in pre)
    # FP32 error against FP64 on the same runs (same graph, clamps and warm start)
    e64 = {(r["q"], r["warm"]): r for r in r64}
    errs, errs_conv = [], []
    for r in pre:
        o = e64[(r["q"], r["warm"])]
        e = float(np.abs(r["p1"] - o["p1"]).max())
        errs.append(e)
        if r["stats"]["converged"] and o["stats"]["converged"]:
            errs_conv.append(e)
    out = dict(
        runs=len(res), wall_s=round(wall, 3), mups=round(upd / wall, 1), queries_per_s=round(len(res) / wall, 2),
        latency=dict(all=_lat(res), cold=_lat(res, 0), warm=_lat(res, 1)),
        iterations_p50=int(np.median([r["stats"]["iterations"] for r in res])),
        converged=int(sum(r["stats"]["converged"] for r in res)),
        executors={n: int(sum(r["stats"]["executor"] == e for r in res))
                   for n, e in (("persistent", F.EXEC_PERSISTENT), ("levels", F.EXEC_LEVELS), ("hybrid", F.EXEC_HYBRID))},
        server=sd, updates=upd,
        prefix=dict(graphs=n64, runs=len(pre), latency=dict(all=_lat(pre), cold=_lat(pre, 0), warm=_lat(pre, 1))),
        plain_fp64=dict(graphs=n64, runs=len(r64), wall_s=round(wall64, 3), busy_s=round(busy64, 3),
                        mups_busy=round(upd64 / busy64, 1),
                        latency=dict(all=_lat(r64), cold=_lat(r64, 0), warm=_lat(r64, 1)),
                        service_p50_ms=pct([r["service_ms"] for r in r64], 50),
                        note="FIFO single-graph FP64 server (fastlbp_run one graph at a time) on the stream's "
                             "first graphs, same arrival times and re-query clamps; latency includes queueing"),
        fp32_error=dict(vs="FP64 marginals of the same runs (plain FP64 leg), runs where both converged",
                        runs=len(errs_conv), max_abs=max(errs_conv) if errs_conv else None,
                        runs_not_both_converged=len(errs) - len(errs_conv),
                        max_abs_not_both_converged=max((e for e in errs if e not in errs_conv), default=None),
                        note="a run that stops at max_iters without converging may end at another point of an "
                             "oscillation in each precision; those runs are listed apart"),
        prefix_updates=upd_pre)
    return qs, res, out


def flooding_runs(F, w, prec, steps, warmup, iters, label, tol=0.0):
    """`steps` timed cold runs of at most `iters` iterations on the LEVELS executor; the marginals of
    the last run are returned for the FP32-vs-FP64 comparison."""
    import torch
    t0 = time.perf_counter()
    kw = {}
    if getattr(w, "term_off", None) is not None:
        kw = dict(term_off=w.term_off, term_weight=w.term_weight, term_ind=w.term_ind)
    g = F.Graph(w.num_vars, w.fac_off, w.edge_var, w.fac_type, w.fac_param, w.edge_param, precision=prec,
                executor="levels", **kw)
    log(f"{label} {prec}: graph created in {time.perf_counter() - t0:.1f} s")
    if w.edge_rank is not None:
        t0 = time.perf_counter()
        g.schedule_set(F.SCHED_RANKED, w.edge_rank)
        log(f"{label} {prec}: schedule set in {time.perf_counter() - t0:.1f} s")
    if w.evidence is not None:
        g.evidence_array(w.evidence)
    for s in range(warmup + steps):
        if s == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dev_ms, upd, mb, ib, its = 0.0, 0, 0.0, 0.0, 0
        g.messages_reset()
        st = g.run(iters, tol, 0.0)
        if s >= warmup:
            dev_ms += st["device_ms"]
            upd += st["message_updates"]
            mb += st["method_bytes_per_iter"] * st["iterations"]
            ib += st["impl_bytes_per_iter"] * st["iterations"]
            its += st["iterations"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m = g.marginals()
    g.close()
    r = dict(wall_s=wall, dev_ms=dev_ms, updates=upd, method_bytes=mb, impl_bytes=ib, iters=st["iterations"],
             steps=steps, converged=st["converged"], residual=st["residual"], levels=st["levels"],
             mups=round(upd / wall, 1), us_per_iteration=round(dev_ms * 1e3 / max(1, its), 2), marginals=m)
    log(f"{label} {prec}: {wall * 1e3 / steps:.1f} ms/run, {upd / wall / 1e9:.2f} G updates/s, "
        f"{r['us_per_iteration']:.1f} us/iteration, {st['iterations']} iterations")
    return r


def _roofline_levels(r, kernel):
    achieved = r["method_bytes"] / (r["dev_ms"] / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None, "kernel": kernel,
            "impl_bytes_achieved_gbs": round(r["impl_bytes"] / (r["dev_ms"] / 1e3) / 1e9, 2),
            "bytes_note": "method bytes per iteration (4 + 5s per edge under flooding, s = 4, + s per NOISY_OR "
                          "activation; ranked: exact from the levels) over the runs' device time (HIP events)"}


def bingo_flooding(F, W, args, terms=False):
    """One BINGO-shaped graph (2M tuples, 4M rules, 19M edges), flooding, FP32 messages, on the
    LEVELS executor: per iteration one launch per degree bucket and phase. A step is one run of
    --max-iters (default 100) iterations; FP64 runs the same graph for the plain comparison and the
    FP32 error (FP32 marginals against FP64 after the same iterations from uniform messages).
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
        "fp32_error": {"vs": f"FP64 marginals after the same {iters} iterations from uniform messages",
                       "max_abs": float(np.abs(r["marginals"] - res["fp64"]["marginals"]).max())},
        "roofline": _roofline_levels(r, "one iteration of the LEVELS executor (all kernels)"),
    }
    if typed:
        out["typed_fp32"] = {"mups": typed["mups"], "us_per_iteration": typed["us_per_iteration"]}
        out["terms"] = int(len(w.term_weight))
    return out


def bingo_large(F, W, args):
    """One BINGO-shaped graph ten times the size of the flooding one (20M tuples, 40M rules, 190M
    edges) under an ordered-group schedule of 64 classes by head position, FP32 messages, tol 1e-6,
    up to 200 iterations (--max-iters overrides), on the LEVELS executor. A step is one cold run.
    One FP64 run of the same graph gives the plain comparison and the FP32 error at convergence."""
    t0 = time.perf_counter()
    w = W.config("C5", seed=args.seed)
    iters = args.max_iters or w.max_iters
    log(f"workload bingo-large: V={w.num_vars} F={w.num_factors} E={w.num_edges}, generated in "
        f"{time.perf_counter() - t0:.1f} s")
    res = {prec: flooding_runs(F, w, prec, args.steps if prec == "fp32" else 1, args.warmup if prec == "fp32" else 0,
                               iters, "bingo-large", tol=1e-6) for prec in ("fp32", "fp64")}
    r = res["fp32"]
    return {
        "metric": "message updates/sec (f->v) + p50/p99 query latency, batched FP32 vs plain FP64 BP",
        "value": round(r["updates"] / r["wall_s"], 1), "unit": "message updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r["wall_s"] * 1e3 / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "bingo_20M_tuples_40M_rules_190M_edges_64_ordered_groups", "seed": args.seed,
                   "levels": r["levels"], "max_iters": iters, "tol": 1e-6, "executor": "levels"},
        "iterations": r["iters"], "converged": r["converged"], "us_per_iteration": r["us_per_iteration"],
        "plain_fp64": {"mups": res["fp64"]["mups"], "us_per_iteration": res["fp64"]["us_per_iteration"],
                       "iterations": res["fp64"]["iters"], "converged": res["fp64"]["converged"]},
        "fp32_error": {"vs": "FP64 marginals of the same graph and schedule (tol 1e-6)",
                       "max_abs": float(np.abs(r["marginals"] - res["fp64"]["marginals"]).max())},
        "roofline": _roofline_levels(r, "one iteration of the LEVELS executor (all kernels)"),
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
                alg += st["method_bytes"]
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
    return dict(value=round(st["message_updates"] / dt, 1), unit="message updates/s", cores=1, kind="oracle", **host_cpu(),
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
    return dict(value=round(st["message_updates"] / dt, 1), unit="message updates/s", cores=1, kind="oracle", **host_cpu(),
                sample=f"{n} full iterations (cold start, tol 0) of the same 200k-variable graph, forward-backward "
                       f"schedule and evidence as query 0: {st['message_updates']} updates in {dt:.1f} s")


def host_cpu() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def serving_cpu_baseline(qs, runs, budget_s: float, n_prefix: int):
    """The oracle (single thread) on a bounded sample of the serving stream: the cold runs of the
    smallest graphs of the stream's first n_prefix graphs, same clamps, tol and iteration bound,
    until about budget_s seconds are spent. Also the largest |FP32 marginal - oracle| over those runs
    (the FP32 results of the batched server)."""
    import oracle
    order = sorted(range(min(n_prefix, len(qs))), key=lambda i: qs[i].graph.num_edges)
    cold = {r["q"]: r for r in runs if r["warm"] == 0 and r["p1"] is not None}
    t_all, upd, errs, errs_conv, names = 0.0, 0, [], [], []
    for i in order:
        if t_all >= budget_s:
            break
        q = qs[i]
        ev = np.full(q.graph.num_vars, -1, dtype=np.int8)
        ev[q.ev_vars] = q.ev_vals
        t0 = time.perf_counter()
        om, _, st = oracle.bp(q.graph, q.graph.max_iters, q.graph.tol, q.graph.damping, evidence=ev)
        t_all += time.perf_counter() - t0
        upd += st["message_updates"]
        names.append(f"{q.graph.name}:{q.graph.num_vars}")
        if i in cold:
            e = float(np.abs(cold[i]["p1"] - om).max())
            errs.append(e)
            if st["converged"] and cold[i]["stats"]["converged"]:
                errs_conv.append(e)
    return dict(value=round(upd / t_all, 1), unit="message updates/s", cores=1, kind="oracle", **host_cpu(),
                sample=f"cold runs of the {len(names)} smallest of the stream's first {n_prefix} graphs "
                       f"({', '.join(names)}): {upd} updates in {t_all:.1f} s, single thread",
                fp32_vs_oracle_max_abs=max(errs) if errs else None,
                fp32_vs_oracle_max_abs_converged=max(errs_conv) if errs_conv else None,
                runs_compared=len(errs))


def extra_workloads(F, W, args):
    """Two more lines of the default run, beside the serving stream: the saturated narrow-level
    kernel (512 batched queries of the 200k-variable SmartFL-shaped graph, one warm-up and one
    timed step) and the wide-level kernels (the 19M-edge BINGO-shaped graph, flooding, 100
    iterations, FP32 and FP64)."""
    import torch
    out = {}
    w = W.smartfl(args.seed)
    queries = [query_evidence(w, q) for q in range(512)]
    log(f"extra: smartfl batched, {len(queries)} queries per step")
    rb = batched_steps(F, w, queries, 1, 1, 8)
    launches = max(1, rb["launches"])
    avg_ms = rb["kernel_ms"] / launches
    per_launch = rb["alg_bytes"] / launches
    ach = per_launch / (avg_ms / 1e3) / 1e9
    T = TRAFFIC_DEFAULT
    traffic = T["bytes_per_launch"] if kernel_sources_sha256() == T["sources_sha256"] else None
    out["smartfl_batched"] = {
        "workload": "smartfl_200k_vars_500_layers_fwd_bwd_ranked, 512 queries per step (2% clamps each), fp32",
        "mups": round(rb["updates"] / rb["wall_s"], 1), "device_mups": round(rb["updates"] / (rb["kernel_ms"] / 1e3), 1),
        "ms_per_step": round(rb["wall_s"] * 1e3, 3), "p50_ms": pct(rb["lat_ms"], 50), "p99_ms": pct(rb["lat_ms"], 99),
        "iterations_p50": int(np.median(rb["iters"])),
        "roofline": {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": traffic,
                     "kernel": "k_persistent<PolLog32> (512 threads, 2 queries per CU)",
                     "launches": rb["launches"], "avg_launch_ms": round(avg_ms, 4), "method_bytes_per_launch": per_launch}}
    del rb
    torch.cuda.empty_cache()
    wb = W.config("C3", seed=args.seed)
    log(f"extra: bingo flooding V={wb.num_vars} E={wb.num_edges}")
    res = {prec: flooding_runs(F, wb, prec, 1, 1 if prec == "fp32" else 0, 100, "bingo") for prec in ("fp32", "fp64")}
    r = res["fp32"]
    out["bingo_flooding"] = {
        "workload": "bingo_2M_tuples_4M_rules_19M_edges_flooding, 100 iterations, fp32 (fp64 for the error)",
        "mups": round(r["updates"] / r["wall_s"], 1), "us_per_iteration": r["us_per_iteration"],
        "plain_fp64_us_per_iteration": res["fp64"]["us_per_iteration"],
        "fp32_error_max_abs": float(np.abs(r["marginals"] - res["fp64"]["marginals"]).max()),
        "roofline": _roofline_levels(r, "one iteration of the LEVELS executor (all kernels)")}
    return out


def pct(a, q):
    return round(float(np.percentile(a, q)), 3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=512, help="queries per batched step (512: two per compute unit)")
    ap.add_argument("--step-iters", type=int, default=8, help="iterations per server launch")
    ap.add_argument("--fp64-queries", type=int, default=3, help="smartfl: plain FP64 queries run one by one")
    ap.add_argument("--fp64-graphs", type=int, default=48,
                    help="serving: graphs of the stream's prefix served by the FIFO plain FP64 server")
    ap.add_argument("--max-iters", type=int, default=None, help="override the workload's 500")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-only", action="store_true", help="only the batched FP32 steps (profiling)")
    ap.add_argument("--serving-only", action="store_true",
                    help="serving: skip the extra lines (batched SmartFL-shaped queries, BINGO-shaped flooding)")
    ap.add_argument("--alarms", type=int, default=300, help="alarms of the alarm-ranking workload")
    ap.add_argument("--workload", choices=["smartfl", "serving", "bingo", "bingo-terms", "bingo-large", "alarms"],
                    default="serving",
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
        qs, runs, rs = serving_mix(F, W, args)
        sd = rs["server"]
        launches = max(1, sd["persistent_launches"])
        avg_ms = sd["persistent_ms"] / launches
        per_launch = sd["persistent_method_bytes"] / launches
        achieved = per_launch / (avg_ms / 1e3) / 1e9 if avg_ms > 0 else 0.0
        T = TRAFFIC_SERVING
        traffic, traffic_detail = None, None
        if (args.queries == T["queries"] and args.batch == T["max_active"] and args.step_iters == T["step_iters"]
                and args.seed == 0 and kernel_sources_sha256() == T["sources_sha256"]):
            traffic = T["bytes_per_launch"]
            traffic_detail = {k: T[k] for k in ("fetch_bytes_per_launch", "write_bytes_per_launch",
                                                "method_bytes_per_launch")}
        p64 = rs["plain_fp64"]
        out = {
            "metric": "message updates/sec (f->v) + p50/p99 query latency, batched FP32 vs plain FP64 BP",
            "value": rs["mups"], "unit": "message updates/s", "n_gpus": 1, "steps": rs["runs"], "warmup": 0,
            "ms_per_step": round(rs["wall_s"] * 1e3 / max(1, rs["runs"]), 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"serving_mix_{args.queries}_graphs_1k_500k_vars_poisson_200qps_warm_requery",
                       "seed": args.seed, "queries": args.queries, "runs": rs["runs"], "max_active": args.batch,
                       "step_iters": args.step_iters, "max_iters": 100, "tol": 1e-6,
                       "note": "a step is one query run (cold or warm re-query); value = f->v updates of all "
                               "runs / wall time of the whole stream"},
            "latency_ms": rs["latency"],
            "serving_fp32": {k: v for k, v in rs.items() if k not in ("plain_fp64", "latency")},
            "plain_fp64": p64,
            "latency_fp32_vs_fp64_same_prefix": {"fp32": rs["prefix"]["latency"], "fp64": p64["latency"]},
            "fp32_error": rs["fp32_error"],
            "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                         "kernel": "k_persistent<PolLog32> (the narrow runs' launch of each server step)",
                         "launches": sd["persistent_launches"], "avg_launch_ms": round(avg_ms, 4),
                         "method_bytes_per_launch": per_launch, "traffic_profiled_launches": traffic_detail,
                         "kernel_share_of_device_ms": round(sd["persistent_ms"] / max(1e-9, sd["kernel_ms"]), 3),
                         "bytes_note": "method bytes: per touched factor edge 4 + 3s, per written edge 2s (tol > 0), "
                                       "s per NOISY_OR activation, s = 4 (FP32); times each run's iterations in the "
                                       "launch; traffic: rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, copy-"
                                       "calibrated, null unless the kernel sources match the profiled ones"},
        }
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = serving_cpu_baseline(qs, runs, args.cpu_budget, args.fp64_graphs)
        if not args.serving_only:
            out["extra"] = extra_workloads(F, W, args)
        print(json.dumps(out), flush=True)
        return
    w = W.smartfl(args.seed)
    if args.max_iters:
        w.max_iters = args.max_iters
    queries = [query_evidence(w, q) for q in range(args.batch)]
    log(f"workload smartfl: V={w.num_vars} F={w.num_factors} E={w.num_edges} (non-prior {w.nonprior_edges()}), "
        f"{args.batch} queries per step")

    rb = batched_steps(F, w, queries, args.steps, args.warmup, args.step_iters, keep=args.fp64_queries)
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
                       "traffic_note": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-"
                                       "calibrated); null when the kernel sources or launch shape differ from "
                                       "the profiled ones", "kernel": "k_persistent<PolLog32>",
                       "launches": rb["launches"], "avg_launch_ms": round(rb["kernel_ms"] / max(1, rb["launches"]), 4),
                       "method_bytes_per_launch": rb["alg_bytes"] / max(1, rb["launches"]),
                       "bytes_note": "method bytes: per touched factor edge 4 + 3s, per written edge 2s (tol > 0), "
                                     "s = 4; each query's iterations; divided by the launches' device time"}
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
        errs = [float(np.abs(rb["kept"][q][0] - r64["marginals"][q]).max()) for q in range(len(r64["marginals"]))
                if q in rb["kept"]]
        conv = [e for q, e in enumerate(errs) if rb["kept"][q][1]["converged"] and r64["converged"][q]]
        out["fp32_error"] = {"vs": "FP64 marginals of the same queries (plain FP64 runs)", "queries": len(errs),
                             "max_abs": max(errs) if errs else None, "both_converged": len(conv),
                             "max_abs_both_converged": max(conv) if conv else None}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
