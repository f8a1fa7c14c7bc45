"""Batching: many handles (queries of one graph, or different graphs) advanced side by side in one
persistent launch. Each result must be the same as the handle's run alone, and match the oracle."""
import sys

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


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_queries_of_one_graph(precision):
    # the interactive setting: one graph, several evidence sets, run side by side
    w = W.smartfl(4, levels=30, width=60, max_iters=100)
    evs = [w.evidence] + [W.smartfl_evidence(w, seed=s) for s in (9, 4, 11)]
    base = F.Graph.from_workload(w, precision=precision, executor="persistent")
    hs = [base] + [base.clone() for _ in evs[1:]]
    for h, ev in zip(hs, evs):
        h.evidence_array(ev)
    st = F.run_batch(hs, w.max_iters, w.tol, 0.0)
    ms = [h.marginals() for h in hs]
    for i, ev in enumerate(evs):
        # alone: same graph and evidence on a fresh handle
        solo = F.Graph.from_workload(w, precision=precision, executor="persistent")
        solo.evidence_array(ev)
        s1 = solo.run(w.max_iters, w.tol, 0.0)
        m1 = solo.marginals()
        solo.close()
        om, _, ost = oracle.bp(w, evidence=ev)
        _say(precision, i, "iters", st[i]["iterations"], s1["iterations"], ost["iterations"],
             "err", np.abs(ms[i] - om).max())
        assert np.array_equal(ms[i], m1), "batched result differs from the run alone"
        assert st[i]["iterations"] == s1["iterations"]
        if ost["converged"]:
            assert np.abs(ms[i] - om).max() <= TOL[precision]
    for h in hs:
        h.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mixed_graphs(precision):
    # different graphs, sizes and schedules in one launch: flooding + ranked + a tree
    ws = [W.datalog(3, num_tuples=400, num_rules=300), W.smartfl(4, levels=20, width=50, max_iters=60),
          W.random_tree(5, num_vars=16), W.random_loopy(6)]
    hs = [F.Graph.from_workload(w, precision=precision, executor="persistent") for w in ws]
    its = 30
    st = F.run_batch(hs, its, 0.0, 0.25)
    for w, h, s in zip(ws, hs, st):
        m = h.marginals()
        om, _, ost = oracle.bp(w, max_iters=its, tol=0.0, damping=0.25)
        err = np.abs(m - om).max()
        _say(precision, w.name, "err", err)
        assert s["iterations"] == its
        assert err <= TOL[precision]
        h.close()


def test_batch_argument_errors():
    w = W.random_tree(1)
    a = F.Graph.from_workload(w, precision="fp64")
    b = F.Graph.from_workload(w, precision="fp32")
    with pytest.raises(F.FastLBPError):
        F.run_batch([a, b], 5)
    with pytest.raises(F.FastLBPError):
        F.run_batch([a, a], 5)
    a.close()
    b.close()
