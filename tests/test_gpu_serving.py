"""Serving: continuous batching. Requests of different graphs and sizes, including warm re-queries
after new evidence, are submitted while others run; every result must equal the same request
sequence run alone on its own handle (within rounding) and match the oracle."""
import sys
import time

import numpy as np
import pytest

import oracle
import paper_2509_22337_amd as F
from paper_2509_22337_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-9, "fp32": 1e-4}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.load()


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def _graphs():
    # convergent, non-chaotic instances of both generators at a few sizes; the last one has a
    # flooding level of ~20k edges, too wide for one workgroup, so the server steps it with the
    # LEVELS executor beside the persistent launch of the others
    return [W.smartfl(4, levels=30, width=60, max_iters=100), W.smartfl(11, levels=30, width=60, max_iters=100),
            W.datalog(1, num_tuples=600, num_rules=450), W.datalog(2, num_tuples=2000, num_rules=1500),
            W.smartfl(13, levels=30, width=60, max_iters=100), W.datalog(3, num_tuples=8000, num_rules=6000)]


def _requests(ws, rng):
    """Two queries per graph: the original clamps, then 1-10 extra clamps (warm re-query)."""
    reqs = []
    for gi, w in enumerate(ws):
        ev = w.evidence
        reqs.append((gi, np.flatnonzero(ev >= 0).astype(np.int32), ev[ev >= 0].astype(np.int8)))
    for gi, w in enumerate(ws):
        k = int(rng.integers(1, 11))
        if "world" in w.meta:
            v = rng.choice(w.num_vars, size=k, replace=False).astype(np.int32)
            x = w.meta["world"][v].astype(np.int8)
        else:  # datalog: clamp tuples without priors to random values (soft factors only)
            v = rng.choice(w.meta["num_tuples"], size=k, replace=False).astype(np.int32)
            x = rng.integers(0, 2, k).astype(np.int8)
        reqs.append((gi, v, x))
    return reqs


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_server_mixed_stream_matches_alone_and_oracle(precision):
    ws = _graphs()
    rng = np.random.default_rng(0)
    reqs = _requests(ws, rng)
    params = [(w.max_iters, w.tol, w.damping) for w in ws]
    # alone: each graph's requests in order on its own handle, one at a time (same executor
    # choice as the server's)
    alone = []
    solo_h = [F.Graph.from_workload(w, precision=precision) for w in ws]
    for h in solo_h:
        h.evidence_clear()
    for gi, v, x in reqs:
        h = solo_h[gi]
        h.evidence_set(v, x)
        st = h.run(*params[gi])
        alone.append((h.marginals(), st))
    # served: all handles fresh, requests submitted in a staggered stream
    srv = F.Server(precision=precision, max_active=3, step_iters=3)
    hs = [F.Graph.from_workload(w, precision=precision) for w in ws]
    for h in hs:
        h.evidence_clear()
    tickets = []
    for i, (gi, v, x) in enumerate(reqs):
        tickets.append(srv.submit(hs[gi], v, x, *params[gi]))
        if i % 3 == 2:
            time.sleep(0.002)  # later requests arrive while earlier ones run
    results = [srv.wait(t) for t in tickets]
    sstats = srv.stats()
    srv.close()
    assert sstats["completed"] == len(reqs)
    # oracle: same evidence sequence, warm start from the oracle's own previous state
    ev_cur = [np.full(w.num_vars, -1, np.int8) for w in ws]
    state = [None] * len(ws)
    for i, (gi, v, x) in enumerate(reqs):
        w = ws[gi]
        ev_cur[gi][v] = x
        m_srv, st_srv, lat = results[i]
        m_alone, st_alone = alone[i]
        E = w.num_edges
        m0, m1 = state[gi] if state[gi] is not None else (np.full(E, 0.5), np.full(E, 0.5))
        om, om0, om1, ost = oracle.bp_pairs(w, m0, m1, w.max_iters, w.tol, w.damping, ranks=w.edge_rank,
                                            evidence=ev_cur[gi])
        state[gi] = (om0, om1)
        d_alone = np.abs(m_srv - m_alone).max()
        d_or = np.abs(m_srv - om).max()
        _say(precision, i, w.name, "iters", st_srv["iterations"], st_alone["iterations"], ost["iterations"],
             "alone", d_alone, "oracle", d_or, "lat ms %.1f" % lat)
        assert st_srv["iterations"] == st_alone["iterations"]
        assert st_srv["executor"] == st_alone["executor"] == (F.EXEC_LEVELS if gi == len(ws) - 1 else F.EXEC_PERSISTENT)
        assert d_alone <= (1e-12 if precision == "fp64" else 1e-6)
        assert d_or <= TOL[precision]
    for h in hs + solo_h:
        h.close()


def test_server_errors():
    w = W.random_tree(2)
    g = F.Graph.from_workload(w, precision="fp64")
    srv = F.Server(precision="fp32", max_active=4)
    with pytest.raises(F.FastLBPError):
        srv.submit(g)  # precision mismatch
    with pytest.raises(F.FastLBPError):
        srv.poll(12345)
    srv.close()
    srv = F.Server(precision="fp64", max_active=1, memory_budget=64)
    with pytest.raises(F.FastLBPError) as ei:
        srv.submit(g)
    assert ei.value.code == F.E_TOO_LARGE
    srv.close()
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_server_steps_hybrid_runs(precision):
    # an alarm graph under the round-robin order (one wide level, ~180 narrow ones: AUTO picks the
    # HYBRID executor) served beside narrow graphs, with warm re-queries that clamp alarms: equal
    # to the same requests run alone, and to the oracle
    wa = W.alarm_graph(0, num_inputs=1500, num_derived=3000, num_alarms=40)
    wa.edge_rank = W.seqfix_ranks(wa)
    wa.max_iters, wa.tol, wa.damping = 20, 0.0, 0.0
    ws = [wa, W.smartfl(4, levels=30, width=60, max_iters=100)]
    reqs = [(0, np.zeros(0, np.int32), np.zeros(0, np.int8)), (1, np.zeros(0, np.int32), np.zeros(0, np.int8))]
    for k in range(3):
        reqs.append((0, wa.alarms[k:k + 1].astype(np.int32), wa.labels[k:k + 1].astype(np.int8)))
    params = [(w.max_iters, w.tol, w.damping) for w in ws]
    solo = [F.Graph.from_workload(w, precision=precision) for w in ws]
    alone = []
    for gi, v, x in reqs:
        solo[gi].evidence_set(v, x)
        st = solo[gi].run(*params[gi])
        alone.append((solo[gi].marginals(), st))
    srv = F.Server(precision=precision, max_active=2, step_iters=4)
    hs = [F.Graph.from_workload(w, precision=precision) for w in ws]
    tickets = [srv.submit(hs[gi], v, x, *params[gi]) for gi, v, x in reqs]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    ev_cur = [np.array(w.evidence, dtype=np.int8, copy=True) for w in ws]
    state = [None, None]
    for i, (gi, v, x) in enumerate(reqs):
        w = ws[gi]
        ev_cur[gi][v] = x
        m_srv, st_srv, _ = results[i]
        m_alone, st_alone = alone[i]
        E = w.num_edges
        m0, m1 = state[gi] if state[gi] is not None else (np.full(E, 0.5), np.full(E, 0.5))
        om, om0, om1, _ = oracle.bp_pairs(w, m0, m1, w.max_iters, w.tol, w.damping, ranks=w.edge_rank,
                                          evidence=ev_cur[gi])
        state[gi] = (om0, om1)
        _say("hybrid serving", precision, i, w.name, st_srv["executor"], np.abs(m_srv - m_alone).max(),
             np.abs(m_srv - om).max())
        assert st_srv["executor"] == st_alone["executor"] == (F.EXEC_HYBRID if gi == 0 else F.EXEC_PERSISTENT)
        assert st_srv["iterations"] == st_alone["iterations"]
        assert np.abs(m_srv - m_alone).max() <= (1e-12 if precision == "fp64" else 1e-6)
        assert np.abs(m_srv - om).max() <= TOL[precision]
    for h in hs + solo:
        h.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_server_serving_mix_generator(precision):
    # the serving-mix generator (log-uniform sizes, half Datalog-shaped with flooding and damping,
    # half SmartFL-shaped with forward-backward ranks, tol 1e-6, at most 100 iterations), scaled
    # down: every query runs cold, then warm with the re-query clamps drawn from its own result.
    # Served in one stream, every run equals the same run alone (same iterations, same marginals
    # within rounding); runs the oracle brings to convergence also match the oracle
    qs = W.serving_mix(3, num_queries=10, min_vars=1000, max_vars=12_000)
    solo = [F.Graph.from_workload(q.graph, precision=precision) for q in qs]
    for h in solo:
        h.evidence_clear()
    alone, clamps = [], []
    for i, q in enumerate(qs):
        h = solo[i]
        h.evidence_set(q.ev_vars, q.ev_vals)
        st = h.run(q.graph.max_iters, q.graph.tol, q.graph.damping)
        m = h.marginals()
        v, x = W.requery_clamps(q.graph, m, seed=500 + i)
        clamps.append((v, x))
        h.evidence_set(v, x)
        st2 = h.run(q.graph.max_iters, q.graph.tol, q.graph.damping)
        alone.append(((m, st), (h.marginals(), st2)))
    srv = F.Server(precision=precision, max_active=6, step_iters=4)
    hs = [F.Graph.from_workload(q.graph, precision=precision) for q in qs]
    for h in hs:
        h.evidence_clear()
    cold = [srv.submit(hs[i], q.ev_vars, q.ev_vals, q.graph.max_iters, q.graph.tol, q.graph.damping)
            for i, q in enumerate(qs)]
    served = []
    for i, q in enumerate(qs):  # a graph's warm re-query is submitted when its cold run completes
        r1 = srv.wait(cold[i])
        t2 = srv.submit(hs[i], clamps[i][0], clamps[i][1], q.graph.max_iters, q.graph.tol, q.graph.damping)
        served.append((r1, t2))
    served = [(r1, srv.wait(t2)) for r1, t2 in served]
    srv.close()
    n_oracle = 0
    for i, q in enumerate(qs):
        w = q.graph
        ev = np.full(w.num_vars, -1, np.int8)
        ev[q.ev_vars] = q.ev_vals
        m0 = m1 = np.full(w.num_edges, 0.5)
        for k in range(2):
            if k == 1:
                ev[clamps[i][0]] = clamps[i][1]
            m_srv, st_srv, _ = served[i][k]
            m_al, st_al = alone[i][k]
            d_al = float(np.abs(m_srv - m_al).max())
            om, m0, m1, ost = oracle.bp_pairs(w, m0, m1, w.max_iters, w.tol, w.damping, ranks=w.edge_rank,
                                              evidence=ev)
            d_or = float(np.abs(m_srv - om).max())
            _say(precision, i, w.name, w.num_vars, "run", k, "iters", st_srv["iterations"], st_al["iterations"],
                 ost["iterations"], "alone", d_al, "oracle", d_or, "converged", ost["converged"])
            assert st_srv["iterations"] == st_al["iterations"]
            assert d_al <= (1e-12 if precision == "fp64" else 1e-6)
            if ost["converged"] and st_srv["converged"] and (k == 0 or alone[i][0][1]["converged"]):
                assert d_or <= TOL[precision]
                n_oracle += 1
    assert n_oracle >= 4
    for h in hs + solo:
        h.close()
