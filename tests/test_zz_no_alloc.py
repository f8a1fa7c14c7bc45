"""fastlbp_run_noalloc (the entry point for callers that cannot allocate) against fastlbp_run:
two calls in a row through the C ABI, the second on a smaller graph, on every executor and both
precisions. Each call's marginals, iteration count and contradiction count must equal those of
fastlbp_run on an identical handle (same kernels, same launch order: bit-equal)."""
import sys

import numpy as np
import pytest

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


CASES = [
    # (executor, first workload, second smaller workload)
    ("persistent", lambda: W.smartfl(1, levels=40, width=80, max_iters=30), lambda: W.smartfl(2, levels=12, width=30, max_iters=30)),
    ("levels", lambda: W.datalog(0), lambda: W.datalog(1, num_tuples=300, num_rules=220)),
    ("hybrid", lambda: W.smartfl(3, levels=30, width=60, max_iters=20), lambda: W.smartfl(4, levels=10, width=20, max_iters=20)),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_equals_run(case, precision):
    executor, big, small = CASES[case]
    for k, make in enumerate((big, small)):
        w = make()
        a = F.Graph.from_workload(w, precision=precision, executor=executor)
        b = F.Graph.from_workload(w, precision=precision, executor=executor, use_graph=False)
        sa = a.run(w.max_iters, w.tol, w.damping)
        sb = b.run_noalloc(w.max_iters, w.tol, w.damping)
        ma, mb = a.marginals(), b.marginals()
        _say(executor, precision, "call", k, "V", w.num_vars, "iterations", sa["iterations"], sb["iterations"],
             "executor", sa["executor"], sb["executor"], "max diff", float(np.abs(ma - mb).max()))
        assert sb["executor"] == sa["executor"]
        assert sb["iterations"] == sa["iterations"]
        assert sb["contradictions"] == sa["contradictions"]
        assert np.array_equal(ma, mb)
        # the handle's own run state is untouched: a later ordinary run continues normally
        sc = b.run(2, 0.0, w.damping)
        assert sc["iterations"] == 2
        a.close()
        b.close()
