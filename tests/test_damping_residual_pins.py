"""Pins for the two conventions the paper leaves open and the oracle fixes: damping of stored
factor-to-variable messages, and the residual that decides convergence.

The paper never mentions damping and only says that BP iterates "until convergence" (Section 3.2,
Section 4.1). The readings the oracle implements are: a stored message is lambda * old + (1 - lambda)
* new, on normalised messages; the residual of an iteration is the largest |change of P(x = 1)| over
the messages written in it, measured after damping; a run stops after the first iteration whose
residual is below tol. These tests check the oracle against closed forms derived by hand for a graph
where every quantity is known, so that a swapped lambda, a residual taken before damping, or a sum
instead of a maximum, each fails:

    chain c (c = 0, 1):  PRIOR(p_c) on x_c,  NOT(x_c, y_c) with y_c the head.

y_c has no other factor, so the message y_c -> NOT is uniform and the NOT -> x_c message stays
uniform forever. x_c -> NOT is its prior (1 - p_c, p_c), so the new NOT -> y_c message is
(p_c, 1 - p_c) in every iteration. From the uniform start, the stored P(y_c = 1) after k
iterations is  s_k = (1 - p_c) + lambda^k (1/2 - (1 - p_c)),  its change in iteration k is
(1 - lambda) lambda^(k-1) |p_c - 1/2|, and the residual is the larger of the two chains' changes.
The marginal of y_c is s_k (no other factor), that of x_c is p_c (Eq.(3)).
"""
import numpy as np
import pytest

from paper_2509_22337_amd import workloads as W


def _chains(p, q, ranked=False):
    b = W._Builder(4)
    b.add(W.PRIOR, [0], p)
    b.add(W.NOT, [0, 1], ranks=[1, 0] if ranked else None)
    b.add(W.PRIOR, [2], q)
    b.add(W.NOT, [2, 3], ranks=[1, 0] if ranked else None)
    w = b.build(evidence=np.full(4, -1, dtype=np.int8))
    if not ranked:
        w.edge_rank = None
    return w


HEAD_EDGES = (2, 5)   # NOT -> y_0, NOT -> y_1
INPUT_EDGES = (1, 4)  # NOT -> x_0, NOT -> x_1


def _closed_form(p, lam, k):
    new = 1.0 - p
    return new + lam ** k * (0.5 - new)


@pytest.mark.parametrize("ranked", [False, True])
@pytest.mark.parametrize("lam", [0.0, 0.25, 0.6])
def test_damped_messages_and_residual_closed_form(oracle_mod, ranked, lam):
    p, q = 0.9, 0.3
    w = _chains(p, q, ranked)
    for k in range(1, 7):
        marg, m1, st = oracle_mod.bp(w, max_iters=k, tol=0.0, damping=lam)
        sy0, sy1 = _closed_form(p, lam, k), _closed_form(q, lam, k)
        assert abs(m1[HEAD_EDGES[0]] - sy0) < 1e-15 and abs(m1[HEAD_EDGES[1]] - sy1) < 1e-15
        assert m1[INPUT_EDGES[0]] == 0.5 and m1[INPUT_EDGES[1]] == 0.5
        res = (1.0 - lam) * lam ** (k - 1) * max(abs(p - 0.5), abs(q - 0.5))
        assert abs(st["residual"] - res) < 1e-15, (k, st["residual"], res)
        assert st["iterations"] == k and st["message_updates"] == 4 * k
        assert abs(marg[1] - sy0) < 1e-15 and abs(marg[3] - sy1) < 1e-15
        assert abs(marg[0] - p) < 1e-15 and abs(marg[2] - q) < 1e-15


def test_the_pins_discriminate_plausible_mistakes(oracle_mod):
    # the closed forms above are not met by a swapped lambda, a residual taken before damping, or a
    # residual summed over messages: each would give a different number in iteration 1 and 2
    p, q, lam = 0.9, 0.3, 0.25
    w = _chains(p, q)
    _, m1, st = oracle_mod.bp(w, max_iters=1, tol=0.0, damping=lam)
    swapped = _closed_form(p, 1.0 - lam, 1)
    assert abs(m1[HEAD_EDGES[0]] - swapped) > 0.1
    before_damping = max(abs(p - 0.5), abs(q - 0.5))
    summed = (1.0 - lam) * (abs(p - 0.5) + abs(q - 0.5))
    assert abs(st["residual"] - before_damping) > 0.05 and abs(st["residual"] - summed) > 0.05
    _, _, st2 = oracle_mod.bp(w, max_iters=2, tol=0.0, damping=lam)
    # change in iteration 2 alone, not the total change since the start
    assert abs(st2["residual"] - (1 - lam) * lam * 0.4) < 1e-15
    assert abs(st2["residual"] - (1 - lam ** 2) * 0.4) > 0.05


@pytest.mark.parametrize("tol", [1e-2, 1e-3, 1e-6])
def test_stopping_iteration_closed_form(oracle_mod, tol):
    # stop after the first iteration whose residual is below tol:
    # smallest k with (1 - lambda) lambda^(k-1) * 0.4 < tol
    p, q, lam = 0.9, 0.3, 0.25
    w = _chains(p, q)
    k = 1
    while (1 - lam) * lam ** (k - 1) * 0.4 >= tol:
        k += 1
    _, _, st = oracle_mod.bp(w, max_iters=100, tol=tol, damping=lam)
    assert st["iterations"] == k and st["converged"] == 1
    _, _, st = oracle_mod.bp(w, max_iters=k - 1, tol=tol, damping=lam)
    assert st["iterations"] == k - 1 and st["converged"] == 0


def test_fixed_point_start_converges_in_one_iteration(oracle_mod):
    # started at the fixed point, nothing moves whatever lambda is: residual exactly 0
    p, q = 0.9, 0.3
    w = _chains(p, q)
    start = np.full(w.num_edges, 0.5)
    start[HEAD_EDGES[0]], start[HEAD_EDGES[1]] = 1 - p, 1 - q
    start[0], start[3] = p, q  # PRIOR edges (ignored: constant)
    _, m1, st = oracle_mod.bp(w, max_iters=50, tol=1e-12, damping=0.7, msg1=start)
    assert st["iterations"] == 1 and st["converged"] == 1 and st["residual"] == 0.0
    assert np.array_equal(m1[list(HEAD_EDGES)], start[list(HEAD_EDGES)])
