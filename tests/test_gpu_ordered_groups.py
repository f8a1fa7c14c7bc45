"""Ordered-group schedules on BINGO-shaped derivation graphs (the shape of the 190M-edge workload:
power-law fan-in of the NOISY_OR heads, 64 rank classes by head position) on the LEVELS executor,
whose wide levels take every degree bucket (thread, wavefront and workgroup per factor).

* A 1/1000-scale instance with fan-in truncated at 500 runs to convergence (tol 1e-6) against the
  oracle: marginals 1e-9 (FP64) / 1e-4 (FP32), equal FP64 iteration counts, levels bit-exact
  against the class-atomic analysis.
* The 190M-edge configuration's own generator at 1/500 scale (fan-in up to 8,883) takes one
  iteration from a random message state: one-step parity against one oracle iteration (1e-9 FP64 /
  1e-5 FP32 absolute on the messages). The FP64 check starts from a state with exact 0/1 entries
  and must reproduce the oracle's contradictions exactly. The FP32 check starts from a state
  without exact 0/1 entries: with an exact 0/1 head message, the linear float64 products of a
  NOISY_OR factor with thousands of inputs underflow to 0 in both entries of some messages. The
  oracle and the FP64 path then count a contradiction, while the log-domain FP32 path keeps the
  exact tiny values.
"""
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


@pytest.fixture(scope="module")
def small():
    w = W.bingo(0, num_tuples=20000, num_rules=40000, max_fanin=500, max_iters=200, ranked_classes=64)
    om, _, ost = oracle.bp(w)
    return w, om, ost, R.alg2_class_atomic(w, w.edge_rank).astype(np.int32)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ordered_groups_to_convergence(small, precision):
    w, om, ost, lv_ref = small
    assert ost["converged"]
    g = F.Graph.from_workload(w, precision=precision, executor="levels")
    st = g.run(w.max_iters, w.tol, w.damping)
    m = g.marginals()
    lv = g.schedule_levels()
    g.close()
    err = float(np.abs(m - om).max())
    _say("ordered groups", precision, "V", w.num_vars, "E", w.num_edges, "levels", st["levels"], "iterations",
         st["iterations"], ost["iterations"], "err", err)
    assert np.array_equal(lv, lv_ref)
    assert st["converged"]
    assert err <= TOL[precision]
    if precision == "fp64":
        assert st["iterations"] == ost["iterations"]


@pytest.fixture(scope="module")
def c5_small():
    w = W.config("C5", scale=0.002)
    rng = np.random.default_rng(3)
    pri = np.repeat(w.fac_type, np.diff(w.fac_off)) == W.PRIOR
    states = {}
    for precision in ("fp64", "fp32"):
        p1 = rng.uniform(0.001, 0.999, w.num_edges)
        if precision == "fp64":
            p1[rng.random(w.num_edges) < 0.05] = 1.0
            p1[rng.random(w.num_edges) < 0.05] = 0.0
        p1[pri] = np.repeat(w.fac_param, np.diff(w.fac_off))[pri]
        _, _, om1, ost = oracle.bp_pairs(w, 1 - p1, p1, 1, 0.0, 0.0, ranks=w.edge_rank)
        states[precision] = (p1, om1, ost)
    return w, states


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ordered_groups_c5_generator_one_step(c5_small, precision):
    w, states = c5_small
    p1, om1, ost = states[precision]
    g = F.Graph.from_workload(w, precision=precision, executor="levels")
    g.messages_set(p1)
    st = g.run(1, 0.0, 0.0)
    got = g.messages_get()
    g.close()
    err = float(np.abs(got - om1).max())
    _say("C5 generator 1/500", precision, "E", w.num_edges, "max degree", int(np.diff(w.fac_off).max()),
         "levels", st["levels"], "one-step err", err, "contradictions", st["contradictions"], ost["contradictions"])
    assert err <= (1e-9 if precision == "fp64" else 1e-5)
    assert st["contradictions"] == ost["contradictions"]
