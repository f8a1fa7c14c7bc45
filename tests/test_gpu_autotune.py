"""fastlbp_autotune on the GPU: the tuned launch choices compute the same marginals as the default
ones (and the oracle's) within the precision's bound, the choice is reported in the run stats, and
a second handle of the same shape takes the cached choice without timing (deterministic)."""
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


CASES = {
    "datalog_flooding": lambda: W.datalog(0),
    "smartfl_ranked": lambda: W.smartfl(4, levels=30, width=60, max_iters=100),
    "bingo_groups": lambda: W.bingo(1, num_tuples=20000, num_rules=40000, max_fanin=500, max_iters=60,
                                    ranked_classes=16),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_tuned_equals_default_and_oracle(case, precision, tmp_path):
    w = CASES[case]()
    cache = str(tmp_path / "tune.txt")
    om, _, ost = oracle.bp(w)
    d = F.Graph.from_workload(w, precision=precision)
    sd = d.run(w.max_iters, w.tol, w.damping)
    md = d.marginals()
    d.close()
    t = F.Graph.from_workload(w, precision=precision)
    r = t.autotune(probe_iters=3, damping=w.damping, cache_path=cache)
    assert r["from_cache"] == 0 and r["candidates"] >= 2
    st = t.run(w.max_iters, w.tol, w.damping)
    m = t.marginals()
    t.close()
    _say(case, precision, "choice", {k: r[k] for k in ("executor", "thread_max_degree", "wave_max_degree",
                                                          "var_thread_max_degree", "graph_iters", "persistent_threads")},
         "ms/iter best", round(r["best_ms_per_iter"], 4), "default", round(r["default_ms_per_iter"], 4),
         "err vs default", float(np.abs(m - md).max()), "vs oracle", float(np.abs(m - om).max()))
    assert st["tuned"] == 1 and sd["tuned"] == 0
    assert st["executor"] == r["executor"]
    assert st["thread_max_degree"] == r["thread_max_degree"] and st["wave_max_degree"] == r["wave_max_degree"]
    assert r["best_ms_per_iter"] <= r["default_ms_per_iter"] * 1.0001
    if ost["converged"]:
        assert np.abs(m - om).max() <= TOL[precision]
        assert np.abs(md - om).max() <= TOL[precision]
    else:
        assert np.abs(m - md).max() <= TOL[precision]
    # a second handle of the same shape: the cached choice, no timing
    u = F.Graph.from_workload(w, precision=precision)
    r2 = u.autotune(probe_iters=3, damping=w.damping, cache_path=cache)
    assert r2["from_cache"] == 1 and r2["candidates"] == 0 and r2["key"] == r["key"]
    for k in ("executor", "thread_max_degree", "wave_max_degree", "var_thread_max_degree", "graph_iters",
              "persistent_threads"):
        assert r2[k] == r[k]
    s2 = u.run(w.max_iters, w.tol, w.damping)
    m2 = u.marginals()
    u.close()
    assert np.array_equal(m2, m) and s2["iterations"] == st["iterations"]
