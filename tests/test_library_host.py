"""Host-side tests of libfastlbp (no GPU): exported symbols, validation errors, and the library's
dependency analysis against the oracle's plain implementation of Algorithm 2."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2509_22337_amd as F
from oracle import reference as R
from paper_2509_22337_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = F.load()
    hdr = open(os.path.join(ROOT, "include", "fastlbp.h")).read()
    declared = set(re.findall(r"^[a-z].*?\b(fastlbp_[a-z_]+)\s*\(", hdr, re.M))
    assert declared, "no declarations found"
    assert declared == set(F.EXPORTS), declared ^ set(F.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.fastlbp_version()


def _tiny():
    return W.random_loopy(0, num_vars=10, num_factors=8, evidence_frac=0.0)


def _codes(w, **over):
    a = dict(num_vars=w.num_vars, fac_off=w.fac_off.copy(), edge_var=w.edge_var.copy(), fac_type=w.fac_type.copy(),
             fac_param=w.fac_param.copy(), edge_param=w.edge_param.copy())
    a.update(over)
    try:
        F.validate(**a)
        return F.OK
    except F.FastLBPError as e:
        return e.code


def test_validation_accepts_generators():
    for w in (W.datalog(0), W.smartfl(0, levels=10), _tiny(), W.random_tree(3)):
        assert _codes(w) == F.OK


def test_validation_errors():
    w = _tiny()
    ev = w.edge_var.copy()
    ev[0] = w.num_vars
    assert _codes(w, edge_var=ev) == F.E_BAD_GRAPH
    fo = w.fac_off.copy()
    fo[1], fo[2] = fo[2], fo[1]
    assert _codes(w, fac_off=fo) == F.E_BAD_GRAPH
    fo = w.fac_off.copy()
    fo[0] = 1
    assert _codes(w, fac_off=fo) == F.E_BAD_GRAPH
    ft = w.fac_type.copy()
    ft[0] = 9
    assert _codes(w, fac_type=ft) == F.E_BAD_GRAPH
    # duplicate variable in one factor
    a = int(np.flatnonzero(np.diff(w.fac_off) >= 2)[0])
    ev = w.edge_var.copy()
    ev[w.fac_off[a] + 1] = ev[w.fac_off[a]]
    assert _codes(w, edge_var=ev) == F.E_BAD_GRAPH
    # arity: NOT with 3 edges, PRIOR with 2
    b = W._Builder(4)
    b.add(W.NOT, [0, 1, 2])
    x = b.build()
    assert _codes(x, num_vars=4) == F.E_BAD_GRAPH
    b = W._Builder(4)
    b.add(W.PRIOR, [0, 1], 0.3)
    assert _codes(b.build(), num_vars=4) == F.E_BAD_GRAPH
    b = W._Builder(4)
    b.add(W.AND, [0])
    assert _codes(b.build(), num_vars=4) == F.E_BAD_GRAPH
    # parameters
    fp = w.fac_param.copy()
    pri = np.flatnonzero(w.fac_type == W.PRIOR)[0]
    fp[pri] = 1.5
    assert _codes(w, fac_param=fp) == F.E_BAD_GRAPH
    fp[pri] = np.nan
    assert _codes(w, fac_param=fp) == F.E_BAD_GRAPH
    b = W._Builder(3)
    b.add(W.NOISY_OR, [0, 1, 2], 1.0, [0.5, 0.5, 0])
    assert _codes(b.build(), num_vars=3) == F.E_BAD_GRAPH
    b = W._Builder(3)
    b.add(W.NOISY_OR, [0, 1, 2], 0.0, [0.5, -0.1, 0])
    assert _codes(b.build(), num_vars=3) == F.E_BAD_GRAPH
    # too large a degree
    n = F.MAX_DEGREE + 1
    b = W._Builder(n)
    b.add(W.OR, list(range(n)))
    assert _codes(b.build(), num_vars=n) == F.E_TOO_LARGE
    assert _codes(w, num_vars=-1) == F.E_INVALID_ARG


def test_empty_graph_validates_and_analyzes():
    lv, n = F.analyze_levels(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert n == 0 and len(lv) == 0
    F.validate(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint8))


def test_paper_example_levels():
    w = W.paper_example()
    lv, n = F.analyze_levels(w.num_vars, w.fac_off, w.edge_var, w.edge_rank)
    assert n == 3
    assert lv.tolist() == [0, 0, 0, 1, 1, 1, 1, 2, 2, 2]


@pytest.mark.parametrize("seed", range(40))
def test_levels_bit_exact_vs_oracle(seed):
    w = W.random_loopy(seed, num_vars=int(10 + seed % 25), num_factors=int(8 + seed % 30), evidence_frac=0.0)
    rng = np.random.default_rng(seed)
    E = w.num_edges
    NE = R.edge_neighbourhood(w)
    for ranks in (rng.integers(0, 4, E), rng.permutation(E), np.zeros(E, int), rng.integers(-3, 40, E)):
        ranks = ranks.astype(np.int32)
        lv, n = F.analyze_levels(w.num_vars, w.fac_off, w.edge_var, ranks)
        ref = R.alg2_class_atomic(w, ranks, NE)
        assert np.array_equal(lv, ref.astype(np.int32))
        assert n == int(ref.max()) + 1


def test_levels_flooding_and_smartfl_shape():
    w = W.smartfl(0, levels=12, width=30)
    lv, n = F.analyze_levels(w.num_vars, w.fac_off, w.edge_var, None)
    assert n == 1 and not lv.any()
    lv, n = F.analyze_levels(w.num_vars, w.fac_off, w.edge_var, w.edge_rank)
    ref = R.alg2_class_atomic(w, w.edge_rank)
    assert np.array_equal(lv, ref.astype(np.int32))
    # forward-backward: the PRIOR class, 11 forward classes and 11 backward classes, where the
    # first backward class (inputs of the top level) has no neighbour among the top level's head
    # edges and joins their level
    assert n == 1 + 11 + 11 - 1


def test_graph_create_reports_missing_device():
    pytest.importorskip("torch")
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    w = _tiny()
    with pytest.raises(F.FastLBPError) as ei:
        F.Graph.from_workload(w)
    assert ei.value.code == F.E_DEVICE


@pytest.mark.parametrize("scale", [1 / 500, 1 / 2000, 1 / 5000])
def test_bingo_generator_at_small_scales(scale):
    # the power-law fan-in draw must cover the rule count even when a short draw falls below it;
    # every head's noisy-OR factor then has its rules plus the head, and the graph validates
    w = W.config("C5", seed=0, scale=scale)
    nt, nr = w.meta["num_tuples"], w.meta["num_rules"]
    deg = np.diff(w.fac_off)
    no = w.fac_type == W.NOISY_OR
    assert int((deg[no] - 1).sum()) == nr
    assert int((w.fac_type == W.AND).sum()) == nr
    assert deg[no].max() - 1 <= 10_000
    assert w.num_vars == nt + nr
    assert _codes(w) == F.OK
