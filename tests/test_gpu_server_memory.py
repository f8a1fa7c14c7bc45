"""Admission by device memory: a server whose budget holds only a few of its graphs' states still
completes every request, evicting idle graphs' state to host memory and restoring it when they are
admitted again; warm re-queries start from the exact messages they left. Results equal those of a
server that never evicts (bit for bit) and the oracle's; the resident state stays within the
budget; an evicted handle used directly afterwards is restored transparently."""
import sys

import numpy as np
import pytest

import oracle
import paper_2509_22337_amd as F
from paper_2509_22337_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.load()


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def _graphs():
    out = []
    for i in range(8):
        if i % 2:
            out.append(W.datalog_scaled(100 + i, 3000 + 500 * i, max_iters=40, tol=1e-6))
        else:
            out.append(W.smartfl(100 + i, levels=12 + i, width=50, max_iters=40, tol=1e-6))
    return out


def _requests(ws):
    reqs = []
    for i, w in enumerate(ws):
        ev = w.evidence
        v = np.flatnonzero(ev >= 0).astype(np.int32)
        reqs.append((i, v, ev[v].astype(np.int8)))
    for i, w in enumerate(ws):  # warm re-queries: a few more clamps
        rng = np.random.default_rng(500 + i)
        v = np.sort(rng.choice(w.num_vars, size=5, replace=False)).astype(np.int32)
        reqs.append((i, v, (rng.random(5) < 0.5).astype(np.int8)))
    return reqs


def _serve(ws, budget, precision):
    hs = [F.Graph.from_workload(w, precision=precision) for w in ws]
    for h in hs:
        h.evidence_clear()
    srv = F.Server(precision=precision, max_active=8, step_iters=4, memory_budget=budget)
    out = {}
    for k, (i, v, x) in enumerate(_requests(ws)):
        t = srv.submit(hs[i], v, x, ws[i].max_iters, ws[i].tol, ws[i].damping)
        out[k] = t
    res = {k: srv.wait(t) for k, t in out.items()}
    st = srv.stats()
    srv.close()
    return hs, res, st


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_budget_smaller_than_graphs(precision):
    ws = _graphs()
    hs_a, big, st_a = _serve(ws, 0, precision)  # default budget: nothing evicted
    one = max(h.info()["state_bytes"] for h in hs_a)
    budget = 3 * one
    hs_b, small, st_b = _serve(ws, budget, precision)
    _say(precision, "budget", budget, "evictions", st_b["evictions"], "restores", st_b["restores"],
         "peak resident", st_b["peak_resident_bytes"], "unlimited peak", st_a["peak_resident_bytes"])
    assert st_a["evictions"] == 0
    assert st_b["evictions"] > 0 and st_b["restores"] > 0
    assert st_b["peak_resident_bytes"] <= budget
    for k in big:
        assert np.array_equal(big[k][0], small[k][0]), f"request {k} differs under the small budget"
        assert big[k][1]["iterations"] == small[k][1]["iterations"]
    # the oracle: cold run of each graph, then its warm re-query from the cold run's messages
    reqs = _requests(ws)
    n = len(ws)
    for i, w in enumerate(ws[:4]):
        ev = np.full(w.num_vars, -1, dtype=np.int8)
        ev[reqs[i][1]] = reqs[i][2]
        _, m0, m1, ost = oracle.bp_pairs(w, np.full(w.num_edges, .5), np.full(w.num_edges, .5), w.max_iters, w.tol,
                                         w.damping, ranks=w.edge_rank, evidence=ev)
        ev2 = ev.copy()
        ev2[reqs[n + i][1]] = reqs[n + i][2]
        om, _, _, ost2 = oracle.bp_pairs(w, m0, m1, w.max_iters, w.tol, w.damping, ranks=w.edge_rank, evidence=ev2)
        if ost["converged"] and ost2["converged"]:
            err = float(np.abs(small[n + i][0] - om).max())
            _say(precision, "graph", i, "warm re-query vs oracle", err)
            assert err <= (1e-9 if precision == "fp64" else 1e-4)
    # handles left evicted by the server: direct use restores them
    for h, k in zip(hs_b, range(n)):
        m = h.marginals()
        assert np.array_equal(m, small[n + k][0])
    for h in hs_a + hs_b:
        h.close()
