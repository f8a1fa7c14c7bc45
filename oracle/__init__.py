"""CPU oracle for the FastLBP hot path (arXiv 2509.22337).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg are the
only code allowed to import this package. The product path (the HIP library and its Python
binding) never imports it, and this package imports nothing from the product.

Contents
  * ``bp``                  plain FP64 loopy BP (C, single thread) - Eq.(1)-(3), schedule by Eq.(5)
                            and Definition 2, executed class by class without dependency analysis.
  * ``factor_messages``     Eq.(2) per factor type by disjoint-cube sums (C).
  * ``terms_messages``      Eq.(4) for a factor given as weighted terms (C, plain sums).
  * ``alarm_loop``          BINGO's interactive alarm-ranking loop (Section 5.2.2, Section 5.3) with a
                            simulated user, one ``bp_pairs`` run per round.
  * ``factor_sample``       one flooding update of a sample of factors from a given state, factor by
                            factor (C): the arithmetic of one ``bp`` iteration, for graphs too large
                            for whole iterations.
  * ``reference``           pure-Python definitions used to pin the above: factor tables, Eq.(2) by
                            truth-table enumeration, Algorithm 1 on each type's term list, exact
                            marginals by enumeration, the edge dependency neighbourhood
                            (Definition 1), Algorithm 2 as printed and its class-atomic variant.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import reference  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_oracle() -> str:
    """Compile the C oracle with gcc (no FMA contraction, so results are reproducible)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("residual", ctypes.c_double),
                ("contradictions", ctypes.c_int64), ("marginal_contradictions", ctypes.c_int64),
                ("message_updates", ctypes.c_int64)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_factor_messages.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, P, P, P, P, P]
        lib.oracle_factor_messages.restype = None
        lib.oracle_bp.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P, P, P, ctypes.c_int32,
                                  ctypes.c_double, ctypes.c_double, P, P, P, ctypes.POINTER(_Stats), P, P, P]
        lib.oracle_bp.restype = ctypes.c_int
        lib.oracle_terms_messages.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P]
        lib.oracle_terms_messages.restype = None
        lib.oracle_factor_sample.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P, P, P, P, P, P,
                                             ctypes.c_int32, P, P, P, P]
        lib.oracle_factor_sample.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def factor_messages(ftype: int, m0, m1, fparam: float = 0.0, eparam=None):
    """Unnormalised Eq.(2) messages of one factor to each of its edges (head last)."""
    lib = _load()
    m0 = np.ascontiguousarray(m0, dtype=np.float64)
    m1 = np.ascontiguousarray(m1, dtype=np.float64)
    d = len(m0)
    ep = np.zeros(d) if eparam is None else np.ascontiguousarray(eparam, dtype=np.float64)
    o0 = np.zeros(d)
    o1 = np.zeros(d)
    lib.oracle_factor_messages(int(ftype), d, float(fparam), _ptr(ep), _ptr(m0), _ptr(m1), _ptr(o0), _ptr(o1))
    return o0, o1


def terms_messages(weights, ind, m0, m1):
    """Unnormalised Eq.(4) messages of a weighted-term factor (ind [l][d], -1 = wildcard)."""
    lib = _load()
    w = np.ascontiguousarray(weights, dtype=np.float64)
    ti = np.ascontiguousarray(ind, dtype=np.int8)
    m0 = np.ascontiguousarray(m0, dtype=np.float64)
    m1 = np.ascontiguousarray(m1, dtype=np.float64)
    d = len(m0)
    o0 = np.zeros(d)
    o1 = np.zeros(d)
    lib.oracle_terms_messages(d, len(w), _ptr(w), _ptr(ti), _ptr(m0), _ptr(m1), _ptr(o0), _ptr(o1))
    return o0, o1


def _terms(w):
    to = getattr(w, "term_off", None)
    if to is None:
        return None, None, None
    return (np.ascontiguousarray(to, dtype=np.int64), np.ascontiguousarray(w.term_weight, dtype=np.float64),
            np.ascontiguousarray(w.term_ind, dtype=np.int8))


def bp(w, max_iters=None, tol=None, damping=None, ranks="auto", groups=None, evidence="auto", msg1=None):
    """Run the oracle on a workload-like object (attributes num_vars, fac_off, edge_var, fac_type,
    fac_param, edge_param, edge_rank, evidence, max_iters, tol, damping).

    ranks: "auto" uses w.edge_rank (None = flooding); an array overrides; None forces flooding.
    groups: optional per-edge group index replacing the rank classes (level-by-level execution).
    msg1: optional start state P(x=1) per edge (default uniform).
    Returns (marginals P(x=1) [V], messages P(x=1) [E], stats dict)."""
    lib = _load()
    max_iters = w.max_iters if max_iters is None else max_iters
    tol = w.tol if tol is None else tol
    damping = w.damping if damping is None else damping
    if isinstance(ranks, str):
        ranks = w.edge_rank
    if isinstance(evidence, str):
        evidence = w.evidence
    E = len(w.edge_var)
    fac_off = np.ascontiguousarray(w.fac_off, dtype=np.int64)
    ev = np.ascontiguousarray(w.edge_var, dtype=np.int32)
    ft = np.ascontiguousarray(w.fac_type, dtype=np.uint8)
    fp = np.ascontiguousarray(w.fac_param, dtype=np.float64)
    epar = np.ascontiguousarray(w.edge_param, dtype=np.float64)
    rk = None if ranks is None else np.ascontiguousarray(ranks, dtype=np.int32)
    gr = None if groups is None else np.ascontiguousarray(groups, dtype=np.int32)
    evd = None if evidence is None else np.ascontiguousarray(evidence, dtype=np.int8)
    if msg1 is None:
        m1 = np.full(E, 0.5)
    else:
        m1 = np.array(msg1, dtype=np.float64, copy=True)
    m0 = 1.0 - m1
    marg = np.zeros(w.num_vars)
    st = _Stats()
    to, tw, ti = _terms(w)
    rc = lib.oracle_bp(int(w.num_vars), len(ft), _ptr(fac_off), _ptr(ev), _ptr(ft), _ptr(fp), _ptr(epar),
                       _ptr(rk), _ptr(gr), _ptr(evd), int(max_iters), float(tol), float(damping),
                       _ptr(m0), _ptr(m1), _ptr(marg), ctypes.byref(st), _ptr(to), _ptr(tw), _ptr(ti))
    if rc != 0:
        raise RuntimeError(f"oracle_bp failed: {rc}")
    stats = {f: getattr(st, f) for f, _ in _Stats._fields_}
    return marg, m1, stats


def bp_pairs(w, msg0, msg1, max_iters, tol=0.0, damping=0.0, ranks=None, groups=None, evidence="auto"):
    """Like ``bp`` but takes and returns the full message pairs (P(x=0), P(x=1)), so a start state
    whose entries are exactly 0 or 1 is represented without rounding."""
    lib = _load()
    if isinstance(evidence, str):
        evidence = w.evidence
    fac_off = np.ascontiguousarray(w.fac_off, dtype=np.int64)
    ev = np.ascontiguousarray(w.edge_var, dtype=np.int32)
    ft = np.ascontiguousarray(w.fac_type, dtype=np.uint8)
    fp = np.ascontiguousarray(w.fac_param, dtype=np.float64)
    epar = np.ascontiguousarray(w.edge_param, dtype=np.float64)
    rk = None if ranks is None else np.ascontiguousarray(ranks, dtype=np.int32)
    gr = None if groups is None else np.ascontiguousarray(groups, dtype=np.int32)
    evd = None if evidence is None else np.ascontiguousarray(evidence, dtype=np.int8)
    m0 = np.array(msg0, dtype=np.float64, copy=True)
    m1 = np.array(msg1, dtype=np.float64, copy=True)
    marg = np.zeros(w.num_vars)
    st = _Stats()
    to, tw, ti = _terms(w)
    lib.oracle_bp(int(w.num_vars), len(ft), _ptr(fac_off), _ptr(ev), _ptr(ft), _ptr(fp), _ptr(epar), _ptr(rk),
                  _ptr(gr), _ptr(evd), int(max_iters), float(tol), float(damping), _ptr(m0), _ptr(m1), _ptr(marg),
                  ctypes.byref(st), _ptr(to), _ptr(tw), _ptr(ti))
    return marg, m0, m1, {f: getattr(st, f) for f, _ in _Stats._fields_}


def factor_sample(w, msg1, factors, evidence="auto"):
    """New messages P(x=1) of the edges of `factors` after one undamped flooding update from the
    state msg1 (P(x=1) per edge; PRIOR edges hold their prior whatever msg1 says).
    Returns (edges [n], P(x=1) [n], contradiction flags [n]) with the factors' edges in order."""
    lib = _load()
    if isinstance(evidence, str):
        evidence = w.evidence
    factors = np.ascontiguousarray(factors, dtype=np.int32)
    fac_off = np.ascontiguousarray(w.fac_off, dtype=np.int64)
    deg = fac_off[factors + 1] - fac_off[factors]
    out_off = np.zeros(len(factors) + 1, dtype=np.int64)
    np.cumsum(deg, out=out_off[1:])
    edges = np.concatenate([np.arange(fac_off[a], fac_off[a + 1]) for a in factors]) if len(factors) else \
        np.zeros(0, np.int64)
    m1 = np.ascontiguousarray(msg1, dtype=np.float64)
    m0 = 1.0 - m1
    out1 = np.zeros(int(out_off[-1]))
    contra = np.zeros(int(out_off[-1]), dtype=np.int8)
    evd = None if evidence is None else np.ascontiguousarray(evidence, dtype=np.int8)
    to, tw, ti = _terms(w)
    rc = lib.oracle_factor_sample(int(w.num_vars), len(w.fac_type), _ptr(fac_off),
                                  _ptr(np.ascontiguousarray(w.edge_var, dtype=np.int32)),
                                  _ptr(np.ascontiguousarray(w.fac_type, dtype=np.uint8)),
                                  _ptr(np.ascontiguousarray(w.fac_param, dtype=np.float64)),
                                  _ptr(np.ascontiguousarray(w.edge_param, dtype=np.float64)), _ptr(evd), _ptr(m0),
                                  _ptr(m1), _ptr(to), _ptr(tw), _ptr(ti), len(factors), _ptr(factors),
                                  _ptr(out_off), _ptr(out1), _ptr(contra))
    if rc != 0:
        raise RuntimeError("oracle_factor_sample: a sampled factor is out of range or a PRIOR")
    return edges, out1, contra.astype(bool)


def alarm_loop(w, alarm_vars, labels, max_rounds=None, max_iters=500, tol=1e-6, damping=0.0, ranks=None,
               follow=None):
    """BINGO's interactive loop with a simulated user (Section 5.2.2): each round runs ``bp_pairs``
    from the messages the previous round left (uniform at first) with the clamps so far, picks the
    uninspected alarm with the highest marginal (the lowest position on ties), or follow[r] when
    `follow` is given, and clamps its variable to its label. Stops once every true alarm has been
    inspected, or after max_rounds rounds.
    Returns (order [rounds], each pick's marginal [rounds], alarm marginals of every round [rounds][A])."""
    alarm_vars = np.asarray(alarm_vars, dtype=np.int64)
    labels = np.asarray(labels, dtype=np.int64)
    A = len(alarm_vars)
    ev = np.full(w.num_vars, -1, np.int8) if w.evidence is None else np.array(w.evidence, dtype=np.int8, copy=True)
    m1 = np.full(w.num_edges, 0.5)
    m0 = 1.0 - m1
    inspected = np.zeros(A, dtype=bool)
    total, found = int(labels.sum()), 0
    order, probs, seen = [], [], []
    n = A if max_rounds is None else int(max_rounds)
    for r in range(n):
        if found >= total or inspected.all():
            break
        marg, m0, m1, _ = bp_pairs(w, m0, m1, max_iters, tol, damping, ranks=ranks, evidence=ev)
        pa = marg[alarm_vars]
        seen.append(pa.copy())
        pick = int(np.argmax(np.where(inspected, -1.0, pa))) if follow is None else int(follow[r])
        order.append(pick)
        probs.append(pa[pick])
        inspected[pick] = True
        ev[alarm_vars[pick]] = labels[pick]
        found += int(labels[pick])
    return np.array(order, dtype=np.int32), np.array(probs), np.array(seen).reshape(len(seen), A)
