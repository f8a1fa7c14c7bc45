"""The HYBRID executor (wide levels as multi-workgroup launches, runs of narrow levels fused into one
single-workgroup launch per iteration) against the oracle and the other executors, on schedules
that mix one wide level with hundreds of narrow ones: the BINGO round-robin order (SEQFIX) on an
alarm graph, and ordered groups of 64 consecutive edges on a BINGO-shaped graph whose narrow levels
also hold wavefront-bucket factors and whose wide level holds a workgroup-bucket factor. Bounds: 1e-9 (FP64), 1e-4 (FP32)."""
import sys

import numpy as np
import pytest

import oracle
import paper_2509_22337_amd as F
from oracle import reference as R
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


def _run(w, ranks, precision, executor, iters, damping):
    g = F.Graph.from_workload(w, precision=precision, executor=executor)
    g.schedule_set(F.SCHED_RANKED, ranks)
    st = g.run(iters, 0.0, damping)
    out = g.marginals(), g.messages_get(), st, g.schedule_levels()
    g.close()
    return out


def _blocks_of(w, n):
    """Ordered groups of n consecutive edges (the oracle's cost stays linear in hub fan-in)."""
    return (np.arange(w.num_edges) // n).astype(np.int32)


CASES = {
    "alarms_seqfix": lambda: (W.alarm_graph(0, num_inputs=1500, num_derived=3000, num_alarms=40), W.seqfix_ranks,
                              20, 0.0),
    "bingo_groups64": lambda: (W.bingo(3, num_tuples=3000, num_rules=6000), lambda w: _blocks_of(w, 64), 12, 0.3),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_hybrid_matches_oracle_and_executors(case, precision):
    w, rank_fn, iters, damping = CASES[case]()
    ranks = rank_fn(w)
    om, omsg, ost = oracle.bp(w, iters, 0.0, damping, ranks=ranks)
    res = {}
    for executor in ("auto", "hybrid", "levels", "persistent"):
        _say(case, precision, executor)
        res[executor] = _run(w, ranks, precision, executor, iters, damping)
        m, msgs, st, lv = res[executor]
        err = max(np.abs(m - om).max(), np.abs(msgs - omsg).max())
        _say("  err", err, "executor", st["executor"], "levels", st["levels"], "ms", st["device_ms"])
        assert err <= TOL[precision], executor
        assert st["iterations"] == iters
    assert res["auto"][2]["executor"] == F.EXEC_HYBRID
    assert res["hybrid"][2]["executor"] == F.EXEC_HYBRID
    assert np.array_equal(res["hybrid"][3], R.alg2_class_atomic(w, ranks).astype(np.int32))
    # the fused levels run the persistent executor's level code: same arithmetic, same results
    if precision == "fp64":
        assert np.abs(res["hybrid"][1] - res["persistent"][1]).max() <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_hybrid_all_levels_fused(precision):
    # every level narrow: one fused launch per iteration; weighted-term factors included
    for seed in range(3):
        w = W.random_terms(seed, max_arity=12)
        ranks = np.random.default_rng(seed).permutation(w.num_edges).astype(np.int32)
        om, omsg, _ = oracle.bp(w, 8, 0.0, 0.2, ranks=ranks)
        m, msgs, st, _ = _run(w, ranks, precision, "hybrid", 8, 0.2)
        assert st["executor"] == F.EXEC_HYBRID
        assert np.abs(msgs - omsg).max() <= TOL[precision], seed
        assert np.abs(m - om).max() <= TOL[precision], seed
