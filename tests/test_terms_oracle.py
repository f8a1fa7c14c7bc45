"""Weighted-term factors (Section 3.3, Eq.(4)): the C oracle's term messages against truth-table
enumeration of the factor the terms define, against Algorithm 1, and whole BP runs of typed graphs
against the same graphs with their factors rewritten as terms."""
import numpy as np
import pytest

import oracle
from oracle import reference as R
from paper_2509_22337_amd import workloads as W


def _rand_factor(rng, d, l):
    ind = rng.integers(-1, 2, (l, d)).astype(np.int8)
    wts = rng.uniform(0.0, 1.0, l)
    wts[rng.random(l) < 0.2] = 0.0
    return wts, ind


def _rand_msgs(rng, d, exact=False):
    m1 = rng.uniform(0, 1, d)
    if exact:
        m1[rng.random(d) < 0.3] = 0.0
        m1[rng.random(d) < 0.3] = 1.0
    return 1.0 - m1, m1


@pytest.mark.parametrize("seed", range(40))
def test_terms_messages_match_truth_table(seed):
    rng = np.random.default_rng(seed)
    d = int(rng.integers(1, 9))
    l = int(rng.integers(1, 10))
    wts, ind = _rand_factor(rng, d, l)
    m0, m1 = _rand_msgs(rng, d, exact=seed % 2 == 1)
    o0, o1 = oracle.terms_messages(wts, ind, m0, m1)
    e0, e1 = R.eq2_messages_terms(wts, ind, m0, m1)
    scale = max(1e-300, np.abs(np.concatenate([e0, e1])).max())
    assert np.abs(o0 - e0).max() <= 1e-13 * scale
    assert np.abs(o1 - e1).max() <= 1e-13 * scale


@pytest.mark.parametrize("seed", range(10))
def test_terms_messages_match_algorithm1(seed):
    rng = np.random.default_rng(100 + seed)
    d = int(rng.integers(2, 8))
    l = int(rng.integers(1, 8))
    wts, ind = _rand_factor(rng, d, l)
    m0, m1 = _rand_msgs(rng, d)
    o0, o1 = oracle.terms_messages(wts, ind, m0, m1)
    mu = np.stack([m0, m1], axis=1)
    for v in range(d):
        for xv, o in ((0, o0), (1, o1)):
            assert abs(R.alg1_message(v, xv, wts, ind.T, mu) - o[v]) <= 1e-13 * max(1.0, abs(o[v]))


@pytest.mark.parametrize("ftype", [W.AND, W.OR, W.NOT, W.IMPLIES, W.PRIOR])
def test_type_encodings_equal_factor_functions(ftype):
    # the input encodings of the typed factors as terms define the same factor function
    import itertools
    for d in ([2] if ftype == W.NOT else [1] if ftype == W.PRIOR else [2, 3, 5]):
        p = 0.7
        wts, ind = W.terms_of_type(ftype, d, p)
        for x in itertools.product((0, 1), repeat=d):
            assert abs(R.terms_value(wts, ind, x) - R.factor_value(ftype, x, p)) <= 1e-15


@pytest.mark.parametrize("seed", range(6))
def test_typed_graph_equals_its_term_form(seed):
    w = W.random_loopy(seed, num_vars=40, num_factors=50, max_arity=5)
    wt = W.as_terms(w)
    assert (wt.fac_type == W.TERMS).any()
    for ranks in (None, "auto"):
        a = oracle.bp(w, 10, 0.0, 0.2, ranks=ranks)
        b = oracle.bp(wt, 10, 0.0, 0.2, ranks=ranks)
        assert np.abs(a[0] - b[0]).max() <= 1e-12
        assert np.abs(a[1] - b[1]).max() <= 1e-12
        assert a[2]["contradictions"] == b[2]["contradictions"]


def test_random_terms_tree_exact():
    # BP on a factor tree of term factors is exact (Section 3.2): compare with enumeration
    rng = np.random.default_rng(5)
    # a chain of pairwise/ternary term factors over 8 variables is a tree
    b = W._Builder(8)
    wts, inds, nterm = [], [], []
    for i in range(0, 7, 2):
        vs = [i, i + 1, i + 2] if i + 2 < 8 else [i, i + 1]
        tw, ti = _rand_factor(rng, len(vs), 4)
        tw[0] = max(tw[0], 0.2)
        b.add(W.TERMS, vs, 0.0)
        wts.append(tw)
        inds.append(ti.reshape(-1))
        nterm.append(4)
    w = b.build(name="terms_chain", max_iters=20, tol=0.0, damping=0.0)
    w.edge_rank = None
    w.term_off = W._csr(np.array(nterm, dtype=np.int64))
    w.term_weight = np.concatenate(wts)
    w.term_ind = np.concatenate(inds).astype(np.int8)
    w.evidence = np.full(8, -1, np.int8)
    # exact marginals by enumeration of the product of the term factors
    import itertools
    Z, P1 = 0.0, np.zeros(8)
    for x in itertools.product((0, 1), repeat=8):
        f = 1.0
        for a in range(len(nterm)):
            vs = w.edge_var[w.fac_off[a]:w.fac_off[a + 1]]
            ti = inds[a].reshape(4, len(vs))
            f *= R.terms_value(wts[a], ti, [x[v] for v in vs])
        Z += f
        P1 += f * np.array(x)
    if Z <= 0:
        pytest.skip("factor product identically zero")
    m, _, _ = oracle.bp(w, 20, 0.0, 0.0)
    assert np.abs(m - P1 / Z).max() <= 1e-12
