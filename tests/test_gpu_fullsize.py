"""Parity at the full size of the 19M-edge BINGO-shaped graph, typed and with its rule factors given
as weighted terms, in the launch configuration the flooding benchmark times (LEVELS executor): one
undamped flooding iteration from a seeded start state, checked on a sample of factors (random ones,
the widest ones, and wavefront- and workgroup-bucket ones) whose new messages the oracle computes
one factor at a time. Tolerances: 1e-9 in FP64 and 1e-4 in FP32 on P(x=1)."""
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


@pytest.fixture(scope="module")
def bingo():
    return W.config("C3", seed=0)


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def _sample(w, rng):
    deg = np.diff(w.fac_off)
    nonprior = np.flatnonzero(w.fac_type != W.PRIOR)
    widest = nonprior[np.argsort(deg[nonprior])[-4:]]
    wave = nonprior[(deg[nonprior] > 8) & (deg[nonprior] <= 257)]
    block = nonprior[deg[nonprior] > 257]
    pick = [rng.choice(nonprior, 2000, replace=False), widest,
            rng.choice(wave, min(200, len(wave)), replace=False), rng.choice(block, min(4, len(block)), replace=False)]
    return np.unique(np.concatenate(pick)).astype(np.int32)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("form", ["typed", "terms"])
def test_bingo_full_size_sampled(bingo, form, precision):
    w = W.as_terms(bingo) if form == "terms" else bingo
    rng = np.random.default_rng(11)
    p1 = rng.uniform(0.02, 0.98, w.num_edges)
    p1[rng.random(w.num_edges) < 2e-4] = 1.0
    p1[rng.random(w.num_edges) < 2e-4] = 0.0
    pri = np.repeat(w.fac_type, np.diff(w.fac_off)) == W.PRIOR
    p1[pri] = np.repeat(w.fac_param, np.diff(w.fac_off))[pri]
    _say("bingo full size", form, precision, "E", w.num_edges)
    g = F.Graph.from_workload(w, precision=precision, executor="levels")
    g.messages_set(p1)
    st = g.run(1, 0.0, 0.0)
    msgs = g.messages_get()
    g.close()
    assert st["iterations"] == 1 and st["executor"] == F.EXEC_LEVELS
    sample = _sample(w, rng)
    if form == "terms":
        assert (w.fac_type[sample] == W.TERMS).sum() > 1000
    edges, out1, contra = oracle.factor_sample(w, p1, sample)
    err = np.abs(msgs[edges] - out1)
    _say("  sampled factors", len(sample), "edges", len(edges), "max err", err.max(), "contradictions", contra.sum())
    assert err.max() <= TOL[precision]
    assert np.all(msgs[edges][contra] == 0.5)
