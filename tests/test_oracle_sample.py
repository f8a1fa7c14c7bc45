"""The oracle's sampled factor update (one flooding update of chosen factors, factor by factor)
against a whole undamped flooding iteration of the oracle on the same state: the sampled outputs
must be the iteration's messages of those edges, PRIOR edges keep their prior, evidence clamps
act through the unary potential, and contradictions are flagged where the iteration counts them."""
import numpy as np
import pytest

import oracle
from paper_2509_22337_amd import workloads as W


def _state(w, seed):
    rng = np.random.default_rng(seed)
    p1 = rng.uniform(0, 1, w.num_edges)
    p1[rng.random(w.num_edges) < 0.1] = 1.0
    p1[rng.random(w.num_edges) < 0.1] = 0.0
    return p1


@pytest.mark.parametrize("make", [lambda s: W.random_loopy(s, max_arity=7), lambda s: W.random_terms(s),
                                  lambda s: W.as_terms(W.random_loopy(s)), lambda s: W.datalog(s, 300, 200)])
def test_sample_equals_one_iteration(make):
    for seed in range(4):
        w = make(seed)
        p1 = _state(w, seed + 7)
        pri = np.repeat(w.fac_type, np.diff(w.fac_off)) == W.PRIOR
        p1[pri] = np.repeat(w.fac_param, np.diff(w.fac_off))[pri]
        _, _, it1, st = oracle.bp_pairs(w, 1 - p1, p1, 1, 0.0, 0.0, ranks=None)
        nonprior = np.flatnonzero(w.fac_type != W.PRIOR).astype(np.int32)
        edges, out1, contra = oracle.factor_sample(w, p1, nonprior)
        assert np.abs(out1 - it1[edges]).max() <= 1e-15
        assert int(contra.sum()) == st["contradictions"]
        # a sample in any order, with repeats, gives the same values
        rng = np.random.default_rng(seed)
        sub = rng.choice(nonprior, size=min(15, len(nonprior)), replace=True)
        e2, o2, _ = oracle.factor_sample(w, p1, sub)
        assert np.abs(o2 - it1[e2]).max() <= 1e-15


def test_sample_ignores_prior_entries_and_rejects_priors():
    w = W.random_loopy(3)
    p1 = _state(w, 1)
    pri = np.repeat(w.fac_type, np.diff(w.fac_off)) == W.PRIOR
    a = np.flatnonzero(w.fac_type != W.PRIOR).astype(np.int32)
    _, o_any, _ = oracle.factor_sample(w, p1, a)
    p2 = p1.copy()
    p2[pri] = 0.5  # whatever the state says on PRIOR edges, the prior is used
    _, o_half, _ = oracle.factor_sample(w, p2, a)
    assert np.array_equal(o_any, o_half)
    with pytest.raises(RuntimeError):
        oracle.factor_sample(w, p1, np.flatnonzero(w.fac_type == W.PRIOR)[:1])
