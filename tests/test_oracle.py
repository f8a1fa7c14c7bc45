"""Pins for the CPU oracle (no GPU needed).

The oracle is checked against things other than itself:
  * Eq.(2) by brute-force enumeration of each factor's assignments (factor definitions written out
    independently in ``oracle.reference.factor_value``), and Algorithm 1 on each type's term list;
  * the textbook noisy-OR closed form with independent parents;
  * exact marginals by enumerating the joint distribution on random factor trees, where BP is exact
    (Section 3.2);
  * invariants: normalisation, fixed points, damping-independence of the fixed point on trees,
    and level-by-level execution reproducing class-by-class execution bit for bit (Theorem 2).
"""
import numpy as np
import pytest

from oracle import reference as R
from paper_2509_22337_amd import workloads as W

TYPES = [R.AND, R.OR, R.NOT, R.IMPLIES, R.NOISY_OR]


def _rand_msgs(rng, d, hard_frac=0.2):
    m1 = rng.uniform(0.0, 1.0, d)
    hard = rng.random(d) < hard_frac
    m1[hard] = rng.integers(0, 2, hard.sum())
    scale = rng.uniform(0.2, 2.0, d)  # unnormalised inputs are allowed by Eq.(2)
    return (1.0 - m1) * scale, m1 * scale


def _params(rng, t, d):
    fp, ep = 0.0, np.zeros(d)
    if t == R.NOISY_OR:
        fp = float(rng.choice([0.0, rng.uniform(0, 0.4)]))
        ep[:-1] = rng.uniform(0, 1, d - 1)
        ep[:-1][rng.random(d - 1) < 0.15] = 1.0
    elif t == R.IMPLIES:
        fp = float(rng.choice([1.0, rng.uniform(0, 1)]))
    return fp, ep


@pytest.mark.parametrize("t", TYPES)
def test_factor_messages_match_truth_table(oracle_mod, t):
    rng = np.random.default_rng(100 + t)
    degs = [2] if t == R.NOT else list(range(2, 12))
    for d in degs:
        for _ in range(6):
            m0, m1 = _rand_msgs(rng, d)
            fp, ep = _params(rng, t, d)
            o0, o1 = oracle_mod.factor_messages(t, m0, m1, fp, ep)
            r0, r1 = R.eq2_messages(t, m0, m1, fp, ep)
            scale = max(1e-300, np.abs(np.concatenate([r0, r1])).max())
            assert np.abs(o0 - r0).max() <= 1e-13 * scale, (t, d)
            assert np.abs(o1 - r1).max() <= 1e-13 * scale, (t, d)


@pytest.mark.parametrize("t", TYPES + [R.PRIOR])
def test_algorithm1_on_term_lists_matches_truth_table(t):
    rng = np.random.default_rng(200 + t)
    degs = [1] if t == R.PRIOR else [2] if t == R.NOT else range(2, 7 if t == R.NOISY_OR else 9)
    for d in degs:
        for _ in range(4):
            m0, m1 = _rand_msgs(rng, d)
            fp, ep = _params(rng, t, d)
            if t == R.PRIOR:
                fp = float(rng.uniform())
            p, ind = R.type_terms(t, d, fp, ep)
            mu = np.stack([m0, m1], axis=1)
            # the terms are disjoint cubes that add up to the factor function
            for x in np.ndindex(*([2] * d)):
                tot = sum(p[k] for k in range(len(p)) if all(ind[j][k] in (-1, x[j]) for j in range(d)))
                assert abs(tot - R.factor_value(t, x, fp, ep)) < 1e-14
            if t == R.PRIOR:
                continue
            r0, r1 = R.eq2_messages(t, m0, m1, fp, ep)
            for v in range(d):
                a0 = R.alg1_message(v, 0, p, ind, mu)
                a1 = R.alg1_message(v, 1, p, ind, mu)
                sc = max(abs(r0[v]), abs(r1[v]), 1e-300)
                assert abs(a0 - r0[v]) <= 1e-13 * sc and abs(a1 - r1[v]) <= 1e-13 * sc


def test_noisy_or_textbook_closed_form(oracle_mod):
    # With independent parents q_j = P(x_j = 1): P(y = 1) = 1 - (1 - leak) prod_j (1 - p_j q_j).
    rng = np.random.default_rng(7)
    for d in (2, 5, 40, 300):
        q = rng.uniform(0, 1, d - 1)
        p = np.append(rng.uniform(0, 1, d - 1), 0.0)
        leak = float(rng.uniform(0, 0.3))
        m1 = np.append(q, 0.5)
        o0, o1 = oracle_mod.factor_messages(R.NOISY_OR, 1 - m1, m1, leak, p)
        expect = 1.0 - (1.0 - leak) * np.prod(1.0 - p[:-1] * q)
        assert abs(o1[-1] / (o0[-1] + o1[-1]) - expect) < 1e-13


def test_deterministic_closed_forms(oracle_mod):
    # OR head with independent parents: P(y=0) = prod (1-q_j); AND head: P(y=1) = prod q_j;
    # NOT swaps; IMPLIES to head with p = 1: P(y=0) proportional to 1 - prod q_j.
    rng = np.random.default_rng(8)
    q = rng.uniform(0, 1, 6)
    m1 = np.append(q, 0.5)
    o0, o1 = oracle_mod.factor_messages(R.OR, 1 - m1, m1)
    assert abs(o0[-1] - np.prod(1 - q)) < 1e-15 and abs(o0[-1] + o1[-1] - 1) < 1e-14
    o0, o1 = oracle_mod.factor_messages(R.AND, 1 - m1, m1)
    assert abs(o1[-1] - np.prod(q)) < 1e-15
    o0, o1 = oracle_mod.factor_messages(R.NOT, [0.3, 0.5], [0.7, 0.5])
    assert (o0[1], o1[1]) == (0.7, 0.3)
    o0, o1 = oracle_mod.factor_messages(R.IMPLIES, 1 - m1, m1, 1.0)
    assert abs(o0[-1] - (1 - np.prod(q))) < 1e-15 and abs(o1[-1] - 1.0) < 1e-14


def _tree_iters(w):
    return 2 * int(w.num_vars) + 4


@pytest.mark.parametrize("seed", range(40))
def test_bp_exact_on_trees_flooding(oracle_mod, seed):
    w = W.random_tree(seed, num_vars=int(8 + seed % 9))
    exact, Z = R.exact_marginals(w)
    marg, _, st = oracle_mod.bp(w, max_iters=_tree_iters(w), tol=0.0, damping=0.0, ranks=None)
    if Z <= 0:
        # evidence of probability zero: on a tree the messages reach the exact (zero) partition
        # function, so some message becomes the null pair and the run reports it
        assert st["contradictions"] > 0
        return
    assert np.abs(marg - exact).max() < 1e-12
    assert st["contradictions"] == 0


@pytest.mark.parametrize("seed", range(20))
def test_bp_exact_on_trees_any_schedule_and_damping(oracle_mod, seed):
    w = W.random_tree(1000 + seed, num_vars=14)
    exact, Z = R.exact_marginals(w)
    rng = np.random.default_rng(seed)
    E = w.num_edges
    for ranks in (rng.permutation(E).astype(np.int32), rng.integers(0, 4, E).astype(np.int32)):
        marg, _, st = oracle_mod.bp(w, max_iters=_tree_iters(w), tol=0.0, damping=0.0, ranks=ranks)
        if Z <= 0:
            assert st["contradictions"] > 0  # evidence of probability zero, under any schedule
        else:
            assert np.abs(marg - exact).max() < 1e-12
    if Z <= 0:
        return
    marg, _, st = oracle_mod.bp(w, max_iters=400, tol=1e-15, damping=0.4, ranks=None)
    assert np.abs(marg - exact).max() < 1e-11


def test_tree_with_large_noisy_or(oracle_mod):
    # A star: one NOISY_OR with many parents, each parent with a prior. Exact: independent parents.
    d = 200
    rng = np.random.default_rng(3)
    q = rng.uniform(0.01, 0.5, d)
    p = rng.uniform(0.1, 0.9, d)
    b = W._Builder(d + 1)
    b.add(W.NOISY_OR, list(range(d + 1)), 0.05, np.append(p, 0.0))
    for j in range(d):
        b.add(W.PRIOR, [j], q[j])
    w = b.build(evidence=np.full(d + 1, -1, dtype=np.int8))
    marg, _, _ = oracle_mod.bp(w, max_iters=4, tol=0.0, damping=0.0, ranks=None)
    assert abs(marg[d] - (1 - 0.95 * np.prod(1 - p * q))) < 1e-13
    assert np.abs(marg[:d] - q).max() < 1e-14


@pytest.mark.parametrize("seed", range(10))
def test_invariants_on_loopy_graphs(oracle_mod, seed):
    w = W.random_loopy(seed)
    marg, m1, st = oracle_mod.bp(w, max_iters=200, tol=1e-12, damping=0.3, ranks=None)
    assert np.all((marg >= 0) & (marg <= 1)) and np.all((m1 >= 0) & (m1 <= 1))
    marg0, m0_, m1_, _ = oracle_mod.bp_pairs(w, 1 - m1, m1, 0)
    if st["converged"]:
        # fixed point: one more iteration moves every message by at most tol (plus rounding)
        _, m1b, st2 = oracle_mod.bp(w, max_iters=1, tol=0.0, damping=0.3, ranks=None, msg1=m1)
        assert np.abs(m1b - m1).max() <= 1e-12 + 1e-14


def test_normalisation_of_stored_messages(oracle_mod):
    w = W.random_loopy(3)
    _, m0, m1, _ = oracle_mod.bp_pairs(w, np.full(w.num_edges, 0.5), np.full(w.num_edges, 0.5), 7, damping=0.2)
    assert np.abs(m0 + m1 - 1.0).max() < 1e-15


@pytest.mark.parametrize("seed", range(12))
def test_levels_reproduce_class_semantics_bit_exact(oracle_mod, seed):
    # Theorem 2: executing the batches of the (class-atomic) dependency analysis one after another
    # gives the same messages as executing the rank classes one after another.
    w = W.random_loopy(50 + seed, num_vars=25, num_factors=30)
    rng = np.random.default_rng(seed)
    E = w.num_edges
    for ranks in (rng.integers(0, 6, E).astype(np.int32), rng.permutation(E).astype(np.int32)):
        lv = R.alg2_class_atomic(w, ranks).astype(np.int32)
        a = oracle_mod.bp(w, max_iters=5, tol=0.0, damping=0.25, ranks=ranks)
        b = oracle_mod.bp(w, max_iters=5, tol=0.0, damping=0.25, ranks=ranks, groups=lv)
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[0], b[0])


def test_planted_mistake_is_caught(oracle_mod):
    # The truth-table pin detects a wrong head convention: feeding the inputs in reversed order
    # to a NOISY_OR with unequal parameters must not match.
    rng = np.random.default_rng(11)
    m0, m1 = _rand_msgs(rng, 5, 0.0)
    ep = np.array([0.9, 0.2, 0.5, 0.7, 0.0])
    o0, o1 = oracle_mod.factor_messages(R.NOISY_OR, m0[::-1], m1[::-1], 0.1, ep)
    r0, r1 = R.eq2_messages(R.NOISY_OR, m0, m1, 0.1, ep)
    assert np.abs(o1 - r1).max() > 1e-6
