"""Parity at the full size of the 190M-edge BINGO-shaped graph (20M tuples, 40M rules, power-law
fan-in up to ~10,000) under its 64-group ordered schedule, in the launch configuration its benchmark
times: LEVELS executor, every degree bucket, the incremental variable phase. Within an iteration a
factor's new messages depend on the levels before it, which the oracle cannot reproduce factor by
factor at this size, so two checks stand in:

* First level: one iteration from a seeded start state. The factors of the first level read only
  beliefs built from the start state, so their new messages are one flooding update of those
  factors, which the oracle computes one factor at a time (random factors, the widest, and
  wavefront- and workgroup-bucket ones). Tolerances 1e-9 (FP64) and 1e-4 (FP32) on P(x=1).
* Fixed point: the FP64 run to convergence (tol 1e-6) must end at a fixed point of BP, which any
  update order leaves in place: one oracle update of sampled factors from every level, taken from
  the converged messages, gives those messages back. The bound 2e-5 is 20 times the convergence
  tolerance. On the same generator at 1/1000 and 1/2000 scale the oracle's own converged states
  deviate by 1.5e-7 and 6.7e-7 under this check, and shifting the messages of one level by 1e-3
  makes it deviate by 3e-3. The FP32 path, started from the same converged messages, must stay
  within 1e-4 of them after one iteration over all 64 levels.

At 1/2000 scale the first-level argument was checked on the CPU: the oracle's ordered iteration and
its flooding update of the first level's factors agree to 2e-16.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2509_22337_amd as F
from paper_2509_22337_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32": 1e-4}
FIXED_POINT_TOL = 2e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.load()


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def c5():
    w = W.config("C5", seed=0)
    rng = np.random.default_rng(17)
    p1 = rng.uniform(0.02, 0.98, w.num_edges)
    pri = np.repeat(w.fac_type, np.diff(w.fac_off)) == W.PRIOR
    p1[pri] = np.repeat(w.fac_param, np.diff(w.fac_off))[pri]
    return w, p1


def _graph(w, precision):
    assert w.edge_rank is not None and (w.evidence is None or (w.evidence < 0).all())
    return F.Graph.from_workload(w, precision=precision, executor="levels")


def _factor_level(w, lv):
    """Level of each non-PRIOR factor (the analysis keeps a factor's edges in one level)."""
    deg = np.diff(w.fac_off)
    nonprior = np.flatnonzero(w.fac_type != W.PRIOR)
    first = lv[w.fac_off[nonprior]]
    mn = np.minimum.reduceat(lv, w.fac_off[:-1])[nonprior]
    mx = np.maximum.reduceat(lv, w.fac_off[:-1])[nonprior]
    assert np.array_equal(mn, first) and np.array_equal(mx, first)
    return nonprior, first, deg[nonprior]


def _sample(rng, fac, deg, n):
    widest = fac[np.argsort(deg)[-4:]]
    wave = fac[(deg > 8) & (deg <= 257)]
    block = fac[deg > 257]
    pick = [rng.choice(fac, min(n, len(fac)), replace=False), widest,
            rng.choice(wave, min(200, len(wave)), replace=False), rng.choice(block, min(8, len(block)), replace=False)]
    return np.unique(np.concatenate(pick)).astype(np.int32)


@pytest.fixture(scope="module")
def fp64_state(c5):
    """FP64: the first iteration from the start state, the levels, and the converged messages."""
    w, p1 = c5
    _say("C5 full size fp64: E", w.num_edges)
    g = _graph(w, "fp64")
    lv = g.schedule_levels()
    g.messages_set(p1)
    st1 = g.run(1, 0.0, 0.0)
    first = g.messages_get()
    g.messages_reset()
    st = g.run(w.max_iters, 1e-6, 0.0)
    fixed = g.messages_get()
    g.close()
    _say("  levels", st1["levels"], "converged", st["converged"], "iterations", st["iterations"],
         "residual", st["residual"])
    return lv, st1, first, st, fixed


def _check_first_level(w, p1, lv, got, precision, rng):
    fac, flv, deg = _factor_level(w, lv)
    sel = flv == 0
    sample = _sample(rng, fac[sel], deg[sel], 3000)
    edges, out1, contra = oracle.factor_sample(w, p1, sample)
    err = np.abs(got[edges] - out1)
    _say("  first level", precision, "factors", int(sel.sum()), "sampled", len(sample), "max degree",
         int(deg[sel].max()), "max err", err.max())
    assert len(sample) > 1000 and (deg[np.isin(fac, sample)] > 257).any()
    assert err.max() <= TOL[precision]
    assert not contra.any()


def test_c5_full_size_fp64_first_level(c5, fp64_state):
    w, p1 = c5
    lv, st1, first, _, _ = fp64_state
    assert st1["iterations"] == 1 and st1["executor"] == F.EXEC_LEVELS and st1["levels"] == 64
    _check_first_level(w, p1, lv, first, "fp64", np.random.default_rng(5))


def test_c5_full_size_fp64_fixed_point(c5, fp64_state):
    w, _ = c5
    lv, _, _, st, fixed = fp64_state
    assert st["converged"] and st["executor"] == F.EXEC_LEVELS
    fac, flv, deg = _factor_level(w, lv)
    rng = np.random.default_rng(6)
    sample = _sample(rng, fac, deg, 4000)
    assert len(np.unique(flv[np.isin(fac, sample)])) == 64  # every level is sampled
    edges, out1, contra = oracle.factor_sample(w, fixed, sample)
    dev = np.abs(out1 - fixed[edges])
    _say("  fixed point: sampled", len(sample), "max deviation", dev.max())
    assert not contra.any()
    assert dev.max() <= FIXED_POINT_TOL


def test_c5_full_size_fp32(c5, fp64_state):
    w, p1 = c5
    lv, _, _, _, fixed = fp64_state
    _say("C5 full size fp32: E", w.num_edges)
    g = _graph(w, "fp32")
    assert np.array_equal(g.schedule_levels(), lv)
    g.messages_set(p1)
    st1 = g.run(1, 0.0, 0.0)
    first = g.messages_get()
    assert st1["iterations"] == 1 and st1["executor"] == F.EXEC_LEVELS
    _check_first_level(w, p1, lv, first, "fp32", np.random.default_rng(7))
    g.messages_set(fixed)
    st = g.run(1, 0.0, 0.0)
    again = g.messages_get()
    g.close()
    drift = float(np.abs(again - fixed).max())
    _say("  fp32 one iteration from the fp64 fixed point: max change", drift, "contradictions", st["contradictions"])
    assert drift <= TOL["fp32"]
