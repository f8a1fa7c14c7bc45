"""The alarm-ranking loop (Section 5.2.2, Section 5.3) on the CPU: the ranking metrics against brute
force and closed forms, the synthetic ground truth against the model, and the oracle's loop against
picks taken from exact marginals (enumeration) on tree-shaped derivation graphs, where BP is exact."""
import itertools

import numpy as np
import pytest

import oracle
import paper_2509_22337_amd as F
from oracle import reference as R
from paper_2509_22337_amd import workloads as W


def _inversions_brute(l):
    return sum(1 for i, j in itertools.combinations(range(len(l)), 2) if l[i] == 0 and l[j] == 1)


def test_inversion_count():
    rng = np.random.default_rng(0)
    for n in range(0, 30):
        l = rng.integers(0, 2, n)
        assert F.inversion_count(l) == _inversions_brute(l)
    assert F.inversion_count([1, 1, 1, 0, 0]) == 0
    assert F.inversion_count([0, 0, 1, 1, 1]) == 6  # every false before every true: 2 x 3
    assert F.inversion_count([0, 1, 0, 1]) == 3


def test_rank_of_fraction():
    l = [0, 1, 1, 0, 1, 0, 0, 1, 1, 1]  # 6 true
    assert F.rank_of_fraction(l, 1.0) == 10
    assert F.rank_of_fraction(l, 0.9) == 10  # ceil(5.4) = 6 true needed
    assert F.rank_of_fraction(l, 0.5) == 5   # 3 true
    assert F.rank_of_fraction([1] * 10, 0.9) == 9
    assert F.rank_of_fraction([0, 0], 1.0) == 0  # no true alarm: nothing to find
    assert F.rank_of_fraction([0, 1], 1.0, total_true=2) == -1


def test_ground_truth_is_a_world_of_the_model():
    # every factor gives the sampled world a positive value, so the world has positive probability
    for seed in range(5):
        w = W.alarm_graph(seed, num_inputs=30, num_derived=60, num_alarms=20)
        for a in range(w.num_factors):
            e0, e1 = w.fac_off[a], w.fac_off[a + 1]
            x = tuple(int(v) for v in w.world[w.edge_var[e0:e1]])
            assert R.factor_value(int(w.fac_type[a]), x, float(w.fac_param[a]), w.edge_param[e0:e1]) > 0, a
        assert np.array_equal(w.labels, w.world[w.alarms])


def test_seqfix_is_a_total_order():
    w = W.alarm_graph(1, num_inputs=30, num_derived=60, num_alarms=20)
    r = W.seqfix_ranks(w)
    assert len(np.unique(r)) == w.num_edges


@pytest.mark.parametrize("seed", range(6))
def test_oracle_loop_follows_exact_marginals_on_trees(seed):
    # one rule per tuple with a one-tuple body: a forest, so BP (enough iterations) is exact
    w = W.alarm_graph(seed, num_inputs=4, num_derived=7, max_rules=1, body=(1, 1), num_alarms=5)
    assert w.num_vars <= 18
    order, probs, seen = oracle.alarm_loop(w, w.alarms, w.labels, max_iters=60, tol=0.0, damping=0.0)
    ev = np.full(w.num_vars, -1, np.int8)
    inspected = np.zeros(len(w.alarms), bool)
    for r, pick in enumerate(order):
        exact, Z = R.exact_marginals(w, evidence=ev)
        assert Z > 0
        pa = exact[w.alarms]
        assert np.abs(seen[r] - pa).max() <= 1e-10
        cand = np.where(inspected, -1.0, pa)
        best = cand.max()
        assert pa[pick] >= best - 1e-10 and not inspected[pick]
        if (cand >= best - 1e-9).sum() == 1:
            assert pick == int(np.argmax(cand))
        inspected[pick] = True
        ev[w.alarms[pick]] = w.labels[pick]
    # the loop stops exactly when every true alarm has been inspected
    assert w.labels[order].sum() == w.labels.sum()
    assert len(order) == 0 or w.labels[order[-1]] == 1


def test_oracle_loop_follow_replays_the_given_order():
    w = W.alarm_graph(2, num_inputs=20, num_derived=40, num_alarms=15)
    order, _, _ = oracle.alarm_loop(w, w.alarms, w.labels, max_iters=30, tol=1e-9, damping=0.3)
    rev = order[::-1].copy()
    o2, _, _ = oracle.alarm_loop(w, w.alarms, w.labels, max_rounds=len(rev), max_iters=30, tol=1e-9, damping=0.3,
                                 follow=rev)
    assert np.array_equal(o2[:len(rev)], rev[:len(o2)])
