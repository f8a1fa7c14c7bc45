"""Seeded synthetic factor-graph generators.

This module builds inputs only: graph structure, factor tags and parameters, update-strategy
ranks and evidence clamps. It holds none of the belief-propagation arithmetic, so both the GPU
path and the CPU oracle can be fed from it without sharing any of the method's code.

Graph format (all numpy arrays, factor-major CSR over edges, head = last edge of a factor):
    num_vars     int
    fac_off      int64[F+1]  edge range of each factor
    edge_var     int32[E]    variable of each edge
    fac_type     uint8[F]    PRIOR=0 AND=1 OR=2 NOT=3 IMPLIES=4 NOISY_OR=5
    fac_param    float64[F]  PRIOR: p(x=1); NOISY_OR: leak; IMPLIES: rule weight p (1 = hard Horn)
    edge_param   float64[E]  NOISY_OR: per-parent activation probability; 0 elsewhere
    edge_rank    int32[E]    update-strategy rank per edge (None = flooding)
    evidence     int8[V]     -1 unobserved, 0 or 1 clamped
  TERMS factors (a sum of weighted terms, Section 3.3) additionally use
    term_off     int64[F+1]  term range of each factor (empty range for the other types)
    term_weight  float64[T]  weight of each term (>= 0)
    term_ind     int8[...]   per term, one indicator per edge of its factor (term-major): the value
                             the edge's variable is fixed to in the term, or -1 for a wildcard

The factor catalogue is the reading of the paper's probabilistic Horn constraints (Section 2.2,
Section 3.3) used throughout this project; the workload shapes stand in for the SmartFL and BINGO
factor graphs of the evaluation (Section 5.1), which are not available.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

PRIOR, AND, OR, NOT, IMPLIES, NOISY_OR, TERMS = 0, 1, 2, 3, 4, 5, 6
TYPE_NAMES = {PRIOR: "PRIOR", AND: "AND", OR: "OR", NOT: "NOT", IMPLIES: "IMPLIES", NOISY_OR: "NOISY_OR",
              TERMS: "TERMS"}


@dataclass
class Workload:
    num_vars: int
    fac_off: np.ndarray
    edge_var: np.ndarray
    fac_type: np.ndarray
    fac_param: np.ndarray
    edge_param: np.ndarray
    edge_rank: Optional[np.ndarray] = None
    evidence: Optional[np.ndarray] = None
    max_iters: int = 50
    tol: float = 0.0
    damping: float = 0.0
    name: str = ""
    meta: dict = field(default_factory=dict)
    term_off: Optional[np.ndarray] = None
    term_weight: Optional[np.ndarray] = None
    term_ind: Optional[np.ndarray] = None

    @property
    def num_factors(self) -> int:
        return int(self.fac_type.shape[0])

    @property
    def num_edges(self) -> int:
        return int(self.edge_var.shape[0])

    def nonprior_edges(self) -> int:
        deg = np.diff(self.fac_off)
        return int(deg[self.fac_type != PRIOR].sum())


class _Builder:
    """Accumulates factors in insertion order."""

    def __init__(self, num_vars: int):
        self.num_vars = num_vars
        self.types: list = []
        self.fparams: list = []
        self.vars: list = []
        self.eparams: list = []
        self.ranks: list = []

    def add(self, ftype, vars_, fparam=0.0, eparams=None, ranks=None):
        vars_ = np.asarray(vars_, dtype=np.int32)
        self.types.append(ftype)
        self.fparams.append(float(fparam))
        self.vars.append(vars_)
        self.eparams.append(np.zeros(len(vars_)) if eparams is None else np.asarray(eparams, dtype=np.float64))
        self.ranks.append(np.zeros(len(vars_), dtype=np.int32) if ranks is None else np.asarray(ranks, dtype=np.int32))

    def build(self, **kw) -> Workload:
        deg = np.array([len(v) for v in self.vars], dtype=np.int64)
        fac_off = np.zeros(len(deg) + 1, dtype=np.int64)
        np.cumsum(deg, out=fac_off[1:])
        cat = (lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
        return Workload(
            num_vars=self.num_vars,
            fac_off=fac_off,
            edge_var=cat(self.vars, np.int32),
            fac_type=np.array(self.types, dtype=np.uint8),
            fac_param=np.array(self.fparams, dtype=np.float64),
            edge_param=cat(self.eparams, np.float64),
            edge_rank=cat(self.ranks, np.int32),
            **kw,
        )


def _csr(deg: np.ndarray) -> np.ndarray:
    off = np.zeros(len(deg) + 1, dtype=np.int64)
    np.cumsum(deg, out=off[1:])
    return off


# ----------------------------------------------------------------------------------------------
# Tiny graphs for pins and parity
# ----------------------------------------------------------------------------------------------

def random_tree(seed: int, num_vars: int = 12, max_arity: int = 4, prior_frac: float = 0.5,
                evidence_frac: float = 0.15, types=(AND, OR, NOT, IMPLIES, NOISY_OR),
                soft_implies: bool = True) -> Workload:
    """A random factor tree (bipartite graph without cycles) over at most ``num_vars`` variables.

    Each new factor attaches to exactly one existing variable and introduces fresh variables for
    its other edges, so the factor graph stays a tree. The existing variable is placed at a random
    position of the factor (sometimes the head, sometimes an input)."""
    rng = np.random.default_rng(seed)
    b = _Builder(num_vars)
    nv = 1
    while nv < num_vars:
        t = int(rng.choice(types))
        if t == NOT:
            arity = 2
        else:
            arity = int(rng.integers(2, max_arity + 1))
        arity = min(arity, num_vars - nv + 1)
        if arity < 2:
            break
        if t == NOT and arity != 2:
            t = OR
        anchor = int(rng.integers(0, nv))
        fresh = list(range(nv, nv + arity - 1))
        nv += arity - 1
        vs = fresh[:]
        vs.insert(int(rng.integers(0, arity)), anchor)
        fparam, eparam = 0.0, None
        if t == NOISY_OR:
            fparam = float(rng.choice([0.0, rng.uniform(0.0, 0.3)]))
            eparam = np.zeros(arity)
            eparam[:-1] = rng.uniform(0.05, 1.0, arity - 1)
        elif t == IMPLIES:
            fparam = float(rng.uniform(0.5, 1.0)) if (soft_implies and rng.random() < 0.5) else 1.0
        b.add(t, vs, fparam, eparam)
    for v in range(nv):
        if rng.random() < prior_frac:
            b.add(PRIOR, [v], float(rng.uniform(0.05, 0.95)))
    w = b.build(name=f"tree{seed}")
    w.num_vars = nv
    ev = np.full(nv, -1, dtype=np.int8)
    for v in range(nv):
        if rng.random() < evidence_frac:
            ev[v] = int(rng.integers(0, 2))
    w.evidence = ev
    w.edge_rank = None
    return w


def random_loopy(seed: int, num_vars: int = 40, num_factors: int = 50, max_arity: int = 5,
                 prior_frac: float = 0.6, evidence_frac: float = 0.05,
                 types=(AND, OR, NOT, IMPLIES, NOISY_OR), hard_evidence_consistent: bool = True) -> Workload:
    """A random loopy factor graph with mixed factor types, priors and (optionally) evidence
    taken from one sampled world, so that hard constraints never contradict the clamps."""
    rng = np.random.default_rng(seed)
    b = _Builder(num_vars)
    world = rng.integers(0, 2, num_vars)
    for _ in range(num_factors):
        t = int(rng.choice(types))
        arity = 2 if t == NOT else int(rng.integers(2, max_arity + 1))
        vs = rng.choice(num_vars, size=arity, replace=False)
        fparam, eparam = 0.0, None
        if t == NOISY_OR:
            fparam = float(rng.choice([0.0, rng.uniform(0.0, 0.2)]))
            eparam = np.zeros(arity)
            eparam[:-1] = rng.uniform(0.3, 0.99, arity - 1)
        elif t == IMPLIES:
            fparam = float(rng.choice([1.0, rng.uniform(0.6, 0.99)]))
        b.add(t, vs, fparam, eparam)
    for v in range(num_vars):
        if rng.random() < prior_frac:
            b.add(PRIOR, [v], float(rng.uniform(0.1, 0.9)))
    w = b.build(name=f"loopy{seed}")
    ev = np.full(num_vars, -1, dtype=np.int8)
    if evidence_frac > 0:
        if hard_evidence_consistent:
            # Only clamp variables that no deterministic factor constrains, so no contradiction arises.
            det = np.zeros(num_vars, bool)
            for a in range(w.num_factors):
                if w.fac_type[a] in (AND, OR, NOT) or (w.fac_type[a] == IMPLIES and w.fac_param[a] >= 1.0):
                    det[w.edge_var[w.fac_off[a]:w.fac_off[a + 1]]] = True
            cand = np.flatnonzero(~det)
        else:
            cand = np.arange(num_vars)
        k = int(round(evidence_frac * num_vars))
        if k and len(cand):
            pick = rng.choice(cand, size=min(k, len(cand)), replace=False)
            ev[pick] = world[pick]
    w.evidence = ev
    w.edge_rank = None
    return w


def paper_example() -> Workload:
    """The 5-variable, 5-factor graph of the motivating example (Section 2, Figure 1), with the
    edge order of the round-robin schedule listed in Section 2.1 as a total order of ranks.

    Edge ids follow that order: (a1,v1) (a2,v2) (a3,v1) (a3,v3) (a4,v1) (a4,v2) (a4,v4)
    (a5,v3) (a5,v4) (a5,v5). Factor types are not given by the paper; OR is used as a
    placeholder because the dependency analysis looks at structure only."""
    b = _Builder(5)
    b.add(PRIOR, [0], 0.5, ranks=[0])          # a1 - v1 (unary in the figure)
    b.add(PRIOR, [1], 0.5, ranks=[1])          # a2 - v2
    b.add(OR, [0, 2], ranks=[2, 3])            # a3 - v1, v3
    b.add(OR, [0, 1, 3], ranks=[4, 5, 6])      # a4 - v1, v2, v4
    b.add(OR, [2, 3, 4], ranks=[7, 8, 9])      # a5 - v3, v4, v5
    w = b.build(name="paper_example")
    w.evidence = np.full(5, -1, dtype=np.int8)
    return w


# ----------------------------------------------------------------------------------------------
# Benchmark-shaped generators
# ----------------------------------------------------------------------------------------------

def datalog(seed: int = 0, num_tuples: int = 2000, num_rules: int = 1500, body=(2, 3),
            rule_p=(0.8, 0.99), prior_frac: float = 0.05, prior_p=(0.1, 0.9)) -> Workload:
    """Random Datalog-style derivation graph (BINGO-like, small).

    Tuples are numbered in a random topological order. Each rule picks a head among tuples with
    index >= 3 and a body of distinct tuples of lower index. A rule r gets a clause variable g_r
    with an AND factor (body..., g_r); each distinct head gets a NOISY_OR over the clause variables
    of its rules, with per-rule probabilities drawn from ``rule_p`` and leak 0. A fraction of the
    tuples receives a PRIOR. Flooding, 50 iterations, damping 0.5."""
    rng = np.random.default_rng(seed)
    lo_head = max(3, body[1])
    heads = rng.integers(lo_head, num_tuples, num_rules)
    order = np.argsort(heads, kind="stable")
    heads = heads[order]
    bsize = rng.integers(body[0], body[1] + 1, num_rules)
    nv = num_tuples + num_rules
    b = _Builder(nv)
    for r in range(num_rules):
        h = int(heads[r])
        bd = rng.choice(h, size=int(bsize[r]), replace=False)
        b.add(AND, list(bd) + [num_tuples + r])
    p = rng.uniform(rule_p[0], rule_p[1], num_rules)
    uniq, start = np.unique(heads, return_index=True)
    ends = list(start[1:]) + [num_rules]
    for h, s, e in zip(uniq, start, ends):
        clause = list(range(num_tuples + s, num_tuples + e))
        ep = np.zeros(len(clause) + 1)
        ep[:-1] = p[s:e]
        b.add(NOISY_OR, clause + [int(h)], 0.0, ep)
    npri = int(round(prior_frac * num_tuples))
    for v in rng.choice(num_tuples, size=npri, replace=False):
        b.add(PRIOR, [int(v)], float(rng.uniform(prior_p[0], prior_p[1])))
    w = b.build(name="datalog", max_iters=50, tol=0.0, damping=0.5)
    w.edge_rank = None
    w.evidence = np.full(nv, -1, dtype=np.int8)
    w.meta = dict(seed=seed, num_tuples=num_tuples, num_rules=num_rules, num_heads=len(uniq))
    return w


def smartfl(seed: int = 0, levels: int = 500, width: int = 400, window: int = 4,
            observed_frac: float = 0.02, max_iters: int = 500, tol: float = 1e-6) -> Workload:
    """SmartFL-shaped layered graph with a forward-backward (TOPO) ranked schedule.

    ``levels`` x ``width`` binary statement variables. Every variable above level 0 gets one
    deterministic factor over k predecessors drawn from the previous ``window`` levels, with
    k ~ Zipf(s=1) on {1..4}; k = 1 gives NOT or a one-input AND (copy), k >= 2 gives AND or OR.
    Every variable has a correctness PRIOR ~ Beta(9,1). A fraction of variables is clamped to a
    forward-sampled world that satisfies every deterministic factor, so evidence is consistent.
    Ranks: the head edge of a level-l factor gets rank l, its input edges rank 2*levels - l,
    PRIOR edges rank 0."""
    rng = np.random.default_rng(seed)
    nv = levels * width
    kvals = np.arange(1, 5)
    kp = (1.0 / kvals) / (1.0 / kvals).sum()
    world = np.zeros(nv, dtype=np.int8)
    prior = rng.beta(9.0, 1.0, nv)
    world[:width] = (rng.random(width) < prior[:width]).astype(np.int8)
    nf = (levels - 1) * width
    k_all = rng.choice(kvals, size=nf, p=kp)
    coin_all = rng.random(nf) < 0.5
    ins_all = np.full((nf, 4), -1, dtype=np.int64)
    ftype = np.where(k_all == 1, np.where(coin_all, NOT, AND), np.where(coin_all, AND, OR)).astype(np.uint8)
    for lvl in range(1, levels):
        lo = max(0, lvl - window) * width
        hi = lvl * width
        sl = slice((lvl - 1) * width, lvl * width)
        k = k_all[sl]
        cand = rng.integers(lo, hi, (width, 4))
        active = np.arange(4)[None, :] < k[:, None]
        for _ in range(100):
            srt = np.sort(np.where(active, cand, -1 - np.arange(4)[None, :]), axis=1)
            bad = np.flatnonzero(((srt[:, 1:] == srt[:, :-1]) & (srt[:, 1:] >= 0)).any(axis=1))
            if len(bad) == 0:
                break
            cand[bad] = rng.integers(lo, hi, (len(bad), 4))
        cand = np.where(active, cand, -1)
        ins_all[sl] = cand
        xin = np.where(active, world[np.maximum(cand, 0)], -1)
        t = ftype[sl]
        any1 = (xin == 1).any(axis=1)
        all1 = ((xin == 1) | ~active).all(axis=1)
        y = np.where(t == NOT, 1 - xin[:, 0], np.where(t == AND, all1, any1)).astype(np.int8)
        world[lvl * width:(lvl + 1) * width] = y
    heads = np.arange(width, nv, dtype=np.int64)
    fdeg = k_all + 1
    foff = _csr(fdeg)
    E1 = int(fdeg.sum())
    evar = np.empty(E1, dtype=np.int64)
    erank = np.empty(E1, dtype=np.int32)
    flevel = heads // width
    for j in range(4):
        sel = k_all > j
        evar[foff[:-1][sel] + j] = ins_all[sel, j]
        erank[foff[:-1][sel] + j] = (2 * levels - flevel[sel]).astype(np.int32)
    evar[foff[1:] - 1] = heads
    erank[foff[1:] - 1] = flevel.astype(np.int32)
    fac_type = np.concatenate([ftype, np.full(nv, PRIOR, dtype=np.uint8)])
    fac_param = np.concatenate([np.zeros(nf), prior])
    deg = np.concatenate([fdeg, np.ones(nv, dtype=np.int64)])
    w = Workload(num_vars=nv, fac_off=_csr(deg), edge_var=np.concatenate([evar, np.arange(nv)]).astype(np.int32),
                 fac_type=fac_type, fac_param=fac_param, edge_param=np.zeros(E1 + nv),
                 edge_rank=np.concatenate([erank, np.zeros(nv, dtype=np.int32)]),
                 max_iters=max_iters, tol=tol, damping=0.0, name="smartfl")
    ev = np.full(nv, -1, dtype=np.int8)
    nobs = int(round(observed_frac * nv))
    pick = rng.choice(nv, size=nobs, replace=False)
    ev[pick] = world[pick]
    w.evidence = ev
    w.meta = dict(seed=seed, levels=levels, width=width, world=world)
    return w


def smartfl_evidence(w: Workload, seed: int, observed_frac: float = 0.02) -> np.ndarray:
    """Another consistent evidence set for a SmartFL-shaped graph (a re-query with new clamps)."""
    rng = np.random.default_rng(seed)
    world = w.meta["world"]
    nv = w.num_vars
    ev = np.full(nv, -1, dtype=np.int8)
    pick = rng.choice(nv, size=int(round(observed_frac * nv)), replace=False)
    ev[pick] = world[pick]
    return ev


def _power_law_counts(rng, total: int, alpha: float, kmax: int) -> np.ndarray:
    k = np.arange(1, kmax + 1, dtype=np.float64)
    pk = k ** (-alpha)
    pk /= pk.sum()
    mean = float((k * pk).sum())
    counts = rng.choice(np.arange(1, kmax + 1), size=int(total / mean * 1.1) + 16, p=pk)
    while counts.sum() < total:  # (rare at small totals: a short draw) draw more
        counts = np.concatenate([counts, rng.choice(np.arange(1, kmax + 1), size=int(total / mean * 0.5) + 16, p=pk)])
    cs = np.cumsum(counts)
    n = int(np.searchsorted(cs, total)) + 1
    counts = counts[:n].copy()
    counts[-1] -= int(cs[n - 1] - total)
    if counts[-1] <= 0:
        counts = counts[:-1]
    return counts.astype(np.int64)


def bingo(seed: int = 0, num_tuples: int = 2_000_000, num_rules: int = 4_000_000, body=(1, 4),
          alpha: float = 2.1, max_fanin: int = 10_000, rule_p=(0.9, 0.99), prior_frac: float = 0.05,
          prior_p=(0.1, 0.9), max_iters: int = 100, ranked_classes: int = 0) -> Workload:
    """BINGO-shaped derivation graph (vectorised; sizes up to tens of millions of edges).

    Rules per head follow a discrete power law (exponent ``alpha``) truncated at ``max_fanin``.
    Heads are distinct tuples; each rule's body has U{body} distinct tuples of lower index, so the
    derivation graph is acyclic. Encoding as in ``datalog``: clause variable + AND per rule,
    NOISY_OR per head over its rules' clause variables. Flooding by default; with
    ``ranked_classes`` = C > 0 every edge of a factor gets rank floor(C * head_tuple / num_tuples)
    (an ordered-group schedule with C classes)."""
    rng = np.random.default_rng(seed)
    counts = _power_law_counts(rng, num_rules, alpha, max_fanin)
    nheads = len(counts)
    lo = body[1] + 1
    heads = np.sort(rng.choice(np.arange(lo, num_tuples), size=nheads, replace=False)).astype(np.int64)
    rule_head = np.repeat(heads, counts)
    nr = len(rule_head)
    bsize = rng.integers(body[0], body[1] + 1, nr)
    # body tuples: distinct, lower index than the head
    bodies = np.full((nr, body[1]), -1, dtype=np.int64)
    bodies[:, :] = (rng.random((nr, body[1])) * rule_head[:, None]).astype(np.int64)
    mask = np.arange(body[1])[None, :] < bsize[:, None]
    for _ in range(64):
        srt = np.sort(np.where(mask, bodies, -1 - np.arange(body[1])[None, :]), axis=1)
        dup = (srt[:, 1:] == srt[:, :-1]) & (srt[:, 1:] >= 0)
        bad = np.flatnonzero(dup.any(axis=1))
        if len(bad) == 0:
            break
        bodies[bad] = (rng.random((len(bad), body[1])) * rule_head[bad, None]).astype(np.int64)
    nv = num_tuples + nr
    # AND factors: body..., clause var
    and_deg = bsize + 1
    and_vars = np.empty(int(and_deg.sum()), dtype=np.int64)
    and_off = _csr(and_deg)
    pos = and_off[:-1]
    for j in range(body[1]):
        sel = bsize > j
        and_vars[pos[sel] + j] = bodies[sel, j]
    and_vars[and_off[1:] - 1] = num_tuples + np.arange(nr)
    # NOISY_OR factors: clause vars of the head's rules..., head
    no_deg = counts + 1
    no_off = _csr(no_deg)
    no_vars = np.empty(int(no_deg.sum()), dtype=np.int64)
    no_eparam = np.zeros(int(no_deg.sum()))
    p = rng.uniform(rule_p[0], rule_p[1], nr)
    rstart = _csr(counts)
    # position of rule r inside its head's factor
    head_idx = np.repeat(np.arange(nheads), counts)
    within = np.arange(nr) - rstart[head_idx]
    dst = no_off[head_idx] + within
    no_vars[dst] = num_tuples + np.arange(nr)
    no_eparam[dst] = p
    no_vars[no_off[1:] - 1] = heads
    # priors
    npri = int(round(prior_frac * num_tuples))
    pv = np.sort(rng.choice(num_tuples, size=npri, replace=False))
    pp = rng.uniform(prior_p[0], prior_p[1], npri)
    F = nr + nheads + npri
    fac_type = np.concatenate([np.full(nr, AND), np.full(nheads, NOISY_OR), np.full(npri, PRIOR)]).astype(np.uint8)
    fac_param = np.concatenate([np.zeros(nr), np.zeros(nheads), pp])
    deg = np.concatenate([and_deg, no_deg, np.ones(npri, dtype=np.int64)])
    fac_off = _csr(deg)
    edge_var = np.concatenate([and_vars, no_vars, pv]).astype(np.int32)
    edge_param = np.concatenate([np.zeros(len(and_vars)), no_eparam, np.zeros(npri)])
    edge_rank = None
    if ranked_classes > 0:
        fac_head_tuple = np.concatenate([rule_head, heads, pv])
        fr = (ranked_classes * fac_head_tuple // num_tuples).astype(np.int32)
        edge_rank = np.repeat(fr, deg).astype(np.int32)
    w = Workload(num_vars=nv, fac_off=fac_off, edge_var=edge_var, fac_type=fac_type, fac_param=fac_param,
                 edge_param=edge_param, edge_rank=edge_rank, evidence=np.full(nv, -1, dtype=np.int8),
                 max_iters=max_iters, tol=0.0 if ranked_classes == 0 else 1e-6, damping=0.0, name="bingo")
    w.meta = dict(seed=seed, num_tuples=num_tuples, num_rules=nr, num_heads=nheads, max_fanin=int(counts.max()),
                  F=F)
    return w


def datalog_scaled(seed: int, num_vars: int, body=(2, 3), rule_p=(0.8, 0.99), prior_frac: float = 0.05,
                   prior_p=(0.1, 0.9), max_iters: int = 50, tol: float = 0.0, damping: float = 0.5) -> Workload:
    """The ``datalog`` generator's distributions at any size, vectorised (a different random stream
    from ``datalog``). About num_vars variables: T tuples and 0.75 T rules, each rule with a clause
    variable and an AND over 2-3 distinct lower-index body tuples; a NOISY_OR per distinct head."""
    rng = np.random.default_rng(seed)
    num_tuples = max(8, int(round(num_vars / 1.75)))
    num_rules = max(1, num_vars - num_tuples)
    lo_head = max(3, body[1])
    heads = np.sort(rng.integers(lo_head, num_tuples, num_rules)).astype(np.int64)
    bsize = rng.integers(body[0], body[1] + 1, num_rules)
    nb = body[1]
    bodies = (rng.random((num_rules, nb)) * heads[:, None]).astype(np.int64)
    mask = np.arange(nb)[None, :] < bsize[:, None]
    for _ in range(200):
        srt = np.sort(np.where(mask, bodies, -1 - np.arange(nb)[None, :]), axis=1)
        bad = np.flatnonzero(((srt[:, 1:] == srt[:, :-1]) & (srt[:, 1:] >= 0)).any(axis=1))
        if len(bad) == 0:
            break
        bodies[bad] = (rng.random((len(bad), nb)) * heads[bad, None]).astype(np.int64)
    nv = num_tuples + num_rules
    and_deg = bsize + 1
    and_off = _csr(and_deg)
    and_vars = np.empty(int(and_deg.sum()), dtype=np.int64)
    for j in range(nb):
        sel = bsize > j
        and_vars[and_off[:-1][sel] + j] = bodies[sel, j]
    and_vars[and_off[1:] - 1] = num_tuples + np.arange(num_rules)
    p = rng.uniform(rule_p[0], rule_p[1], num_rules)
    uniq, start, counts = np.unique(heads, return_index=True, return_counts=True)
    no_deg = counts + 1
    no_off = _csr(no_deg)
    no_vars = np.empty(int(no_deg.sum()), dtype=np.int64)
    no_ep = np.zeros(int(no_deg.sum()))
    hidx = np.repeat(np.arange(len(uniq)), counts)
    dst = no_off[hidx] + (np.arange(num_rules) - start[hidx])
    no_vars[dst] = num_tuples + np.arange(num_rules)
    no_ep[dst] = p
    no_vars[no_off[1:] - 1] = uniq
    npri = int(round(prior_frac * num_tuples))
    pv = np.sort(rng.choice(num_tuples, size=npri, replace=False))
    pp = rng.uniform(prior_p[0], prior_p[1], npri)
    fac_type = np.concatenate([np.full(num_rules, AND), np.full(len(uniq), NOISY_OR),
                               np.full(npri, PRIOR)]).astype(np.uint8)
    deg = np.concatenate([and_deg, no_deg, np.ones(npri, dtype=np.int64)])
    w = Workload(num_vars=nv, fac_off=_csr(deg), edge_var=np.concatenate([and_vars, no_vars, pv]).astype(np.int32),
                 fac_type=fac_type, fac_param=np.concatenate([np.zeros(num_rules + len(uniq)), pp]),
                 edge_param=np.concatenate([np.zeros(len(and_vars)), no_ep, np.zeros(npri)]), edge_rank=None,
                 evidence=np.full(nv, -1, dtype=np.int8), max_iters=max_iters, tol=tol, damping=damping,
                 name="datalog")
    w.meta = dict(seed=seed, num_tuples=num_tuples, num_rules=num_rules, num_heads=len(uniq))
    return w


@dataclass
class Query:
    """One request of the serving mix: a graph, its arrival time and its first evidence clamps."""
    graph: Workload
    arrival_s: float
    ev_vars: np.ndarray
    ev_vals: np.ndarray


def serving_mix(seed: int = 0, num_queries: int = 512, min_vars: int = 1000, max_vars: int = 500_000,
                rate_qps: float = 200.0, max_iters: int = 100, tol: float = 1e-6) -> list:
    """Serving workload: ``num_queries`` graphs with sizes log-uniform in [min_vars, max_vars], half
    Datalog-shaped (flooding, damping 0.5) and half SmartFL-shaped (width 400, ceil(V/400) layers,
    forward-backward ranks, 2% consistent clamps), arriving as a Poisson process at ``rate_qps``.
    Every run uses ``tol`` and at most ``max_iters`` iterations."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(min_vars), np.log(max_vars), num_queries)).astype(np.int64)
    kinds = rng.random(num_queries) < 0.5
    arrivals = np.cumsum(rng.exponential(1.0 / rate_qps, num_queries))
    out = []
    for q in range(num_queries):
        gseed = int(rng.integers(0, 2**31))
        if kinds[q]:
            w = datalog_scaled(gseed, int(sizes[q]), max_iters=max_iters, tol=tol)
        else:
            w = smartfl(gseed, levels=max(2, int(-(-sizes[q] // 400))), width=400, max_iters=max_iters, tol=tol)
        ev = w.evidence
        v = np.flatnonzero(ev >= 0).astype(np.int32)
        out.append(Query(w, float(arrivals[q]), v, ev[v].astype(np.int8)))
    return out


def requery_clamps(w: Workload, marginals: np.ndarray, seed: int) -> tuple:
    """1-10 new clamps for a warm re-query: random variables set to a value of the consistent world
    (SmartFL-shaped graphs) or drawn from the current marginal (Datalog-shaped graphs)."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 11))
    v = np.sort(rng.choice(w.num_vars, size=min(k, w.num_vars), replace=False)).astype(np.int32)
    if "world" in w.meta:
        x = w.meta["world"][v].astype(np.int8)
    else:
        x = (rng.random(len(v)) < marginals[v]).astype(np.int8)
    return v, x


# ----------------------------------------------------------------------------------------------
# Weighted-term factors
# ----------------------------------------------------------------------------------------------

def terms_of_type(ftype: int, d: int, fparam: float = 1.0):
    """A deterministic or Horn factor of degree d (head last) written as disjoint weighted terms:
    (weights [l], indicators [l][d], -1 = wildcard). NOISY_OR has no short disjoint form."""
    n = d - 1
    rows, wts = [], []
    if ftype == NOT:
        return np.array([1.0, 1.0]), np.array([[0, 1], [1, 0]], dtype=np.int8)
    if ftype == PRIOR:
        return np.array([1.0 - fparam, fparam]), np.array([[0], [1]], dtype=np.int8)
    if ftype in (OR, AND):
        idle, fire = (0, 1) if ftype == OR else (1, 0)
        # no input fires: head = idle output; input k is the first to fire: head = fired output
        rows.append([idle] * n + [idle if ftype == OR else 1])
        wts.append(1.0)
        for k in range(n):
            rows.append([idle] * k + [fire] + [-1] * (n - k - 1) + [1 if ftype == OR else 0])
            wts.append(1.0)
        return np.array(wts), np.array(rows, dtype=np.int8)
    if ftype == IMPLIES:
        # body false (input k is the first 0): any head; body true: head 1 with p, head 0 with 1-p
        for k in range(n):
            rows.append([1] * k + [0] + [-1] * (n - k - 1) + [-1])
            wts.append(1.0)
        rows.append([1] * n + [1])
        wts.append(fparam)
        rows.append([1] * n + [0])
        wts.append(1.0 - fparam)
        return np.array(wts), np.array(rows, dtype=np.int8)
    raise ValueError(f"no term form for type {ftype}")


def as_terms(w: Workload) -> Workload:
    """The same graph with every AND / OR / NOT / IMPLIES factor given as a TERMS factor (PRIOR and
    NOISY_OR factors unchanged): both must produce the same messages. Factors of one type and
    degree share one term pattern (IMPLIES differs only in its last two weights), so the rewrite is
    done per (type, degree) group."""
    F = w.num_factors
    deg = np.diff(w.fac_off).astype(np.int64)
    ft0 = np.asarray(w.fac_type)
    conv = np.isin(ft0, (AND, OR, NOT, IMPLIES))
    nterm = np.zeros(F, dtype=np.int64)
    nterm[conv & (ft0 == NOT)] = 2
    nterm[conv & ((ft0 == OR) | (ft0 == AND))] = deg[conv & ((ft0 == OR) | (ft0 == AND))]
    nterm[conv & (ft0 == IMPLIES)] = deg[conv & (ft0 == IMPLIES)] + 1
    toff = _csr(nterm)
    ioff = _csr(nterm * deg)
    weights = np.zeros(int(toff[-1]))
    inds = np.zeros(int(ioff[-1]), dtype=np.int8)
    keys = np.unique(np.stack([ft0[conv].astype(np.int64), deg[conv]], axis=1), axis=0) if conv.any() else []
    for t, d in keys:
        sel = np.flatnonzero(conv & (ft0 == t) & (deg == d))
        tw, ti = terms_of_type(int(t), int(d), 1.0)
        l = len(tw)
        assert l == nterm[sel[0]]
        wmat = np.tile(tw, (len(sel), 1))
        if t == IMPLIES:
            wmat[:, -2] = w.fac_param[sel]
            wmat[:, -1] = 1.0 - w.fac_param[sel]
        weights[toff[sel][:, None] + np.arange(l)[None, :]] = wmat
        inds[ioff[sel][:, None] + np.arange(l * int(d))[None, :]] = ti.reshape(-1)[None, :]
    ft = np.where(conv, TERMS, ft0).astype(np.uint8)
    out = Workload(num_vars=w.num_vars, fac_off=w.fac_off, edge_var=w.edge_var, fac_type=ft,
                   fac_param=np.where(conv, 0.0, w.fac_param), edge_param=w.edge_param,
                   edge_rank=w.edge_rank, evidence=w.evidence, max_iters=w.max_iters, tol=w.tol, damping=w.damping,
                   name=w.name + "_terms", meta=dict(w.meta))
    out.term_off = toff
    out.term_weight = weights
    out.term_ind = inds
    return out


def random_terms(seed: int, num_vars: int = 40, num_factors: int = 50, max_arity: int = 6, max_terms: int = 8,
                 prior_frac: float = 0.5, evidence_frac: float = 0.1, zero_weight_frac: float = 0.1) -> Workload:
    """Random loopy graph of TERMS factors: arity 1..max_arity, 1..max_terms terms with random
    indicators in {-1, 0, 1} and weights U(0, 1) (some exactly 0), plus PRIORs and a few clamps."""
    rng = np.random.default_rng(seed)
    b = _Builder(num_vars)
    wts, inds = [], []
    for _ in range(num_factors):
        d = int(rng.integers(1, max_arity + 1))
        vs = rng.choice(num_vars, size=d, replace=False)
        l = int(rng.integers(1, max_terms + 1))
        ti = rng.integers(-1, 2, (l, d)).astype(np.int8)
        tw = rng.uniform(0.0, 1.0, l)
        tw[rng.random(l) < zero_weight_frac] = 0.0
        tw[int(rng.integers(0, l))] = max(tw.max(), 0.1)  # not all zero
        b.add(TERMS, vs, 0.0)
        wts.append(tw)
        inds.append(ti.reshape(-1))
    nterm = [len(x) for x in wts]
    for v in rng.choice(num_vars, size=int(prior_frac * num_vars), replace=False):
        b.add(PRIOR, [int(v)], float(rng.uniform(0.1, 0.9)))
        nterm.append(0)
    w = b.build(name="random_terms", max_iters=20, tol=0.0, damping=0.0)
    w.edge_rank = None
    w.term_off = _csr(np.array(nterm, dtype=np.int64))
    w.term_weight = np.concatenate(wts)
    w.term_ind = np.concatenate(inds).astype(np.int8)
    ev = np.full(num_vars, -1, np.int8)
    pick = rng.choice(num_vars, size=int(evidence_frac * num_vars), replace=False)
    ev[pick] = rng.integers(0, 2, len(pick))
    w.evidence = ev
    w.meta = dict(seed=seed)
    return w


def alarm_graph(seed: int = 0, num_inputs: int = 8000, num_derived: int = 20000, max_rules: int = 3,
                body=(1, 3), rule_p=(0.5, 0.95), input_p=(0.8, 0.99), num_alarms: int = 1000,
                max_iters: int = 500, tol: float = 1e-6, damping: float = 0.0) -> Workload:
    """A BINGO-style derivation graph with a ground truth for the alarm-ranking loop (Section
    5.2.2). Tuples 0 .. num_inputs-1 are input facts, each with a PRIOR; every later tuple gets
    1..max_rules rules whose bodies are 1-3 distinct lower tuples. A rule is a clause variable
    AND(body, clause), and a tuple's rules meet in NOISY_OR(clauses..., tuple) with one
    activation probability per rule (leak 0). The alarms are the last num_alarms tuples.

    The ground truth is one world drawn from the same generative story, in topological order:
    an input fact holds with its prior, a clause holds exactly when its body holds, and a tuple
    holds when one of its holding clauses fires (each with its activation probability). An alarm
    is true when its tuple holds in that world. Attributes added: ``alarms`` (variable ids),
    ``labels`` (int8, 1 = true alarm) and ``world`` (int8 per variable)."""
    rng = np.random.default_rng(seed)
    T = num_inputs + num_derived
    k = rng.integers(1, max_rules + 1, num_derived)
    heads = np.repeat(np.arange(num_inputs, T, dtype=np.int64), k)
    R = len(heads)
    nb = body[1]
    bsize = rng.integers(body[0], body[1] + 1, R)
    bodies = (rng.random((R, nb)) * heads[:, None]).astype(np.int64)
    mask = np.arange(nb)[None, :] < bsize[:, None]
    for _ in range(200):
        srt = np.sort(np.where(mask, bodies, -1 - np.arange(nb)[None, :]), axis=1)
        bad = np.flatnonzero(((srt[:, 1:] == srt[:, :-1]) & (srt[:, 1:] >= 0)).any(axis=1))
        if len(bad) == 0:
            break
        bodies[bad] = (rng.random((len(bad), nb)) * heads[bad, None]).astype(np.int64)
    p = rng.uniform(rule_p[0], rule_p[1], R)
    pin = rng.uniform(input_p[0], input_p[1], num_inputs)
    # ground truth, in topological order (bodies precede heads; rules are sorted by head)
    fires = rng.random(R) < p
    world = np.zeros(T + R, dtype=np.int8)
    world[:num_inputs] = rng.random(num_inputs) < pin
    for r in range(R):
        c = bool(world[bodies[r, :bsize[r]]].all())
        world[T + r] = c
        if c and fires[r]:
            world[heads[r]] = 1
    nv = T + R
    and_deg = bsize + 1
    and_off = _csr(and_deg)
    and_vars = np.empty(int(and_deg.sum()), dtype=np.int64)
    for j in range(nb):
        sel = bsize > j
        and_vars[and_off[:-1][sel] + j] = bodies[sel, j]
    and_vars[and_off[1:] - 1] = T + np.arange(R)
    no_deg = k + 1
    no_off = _csr(no_deg)
    no_vars = np.empty(int(no_deg.sum()), dtype=np.int64)
    no_ep = np.zeros(int(no_deg.sum()))
    start = _csr(k)[:-1]
    hidx = np.repeat(np.arange(num_derived), k)
    dst = no_off[hidx] + (np.arange(R) - start[hidx])
    no_vars[dst] = T + np.arange(R)
    no_ep[dst] = p
    no_vars[no_off[1:] - 1] = np.arange(num_inputs, T)
    fac_type = np.concatenate([np.full(R, AND), np.full(num_derived, NOISY_OR),
                               np.full(num_inputs, PRIOR)]).astype(np.uint8)
    deg = np.concatenate([and_deg, no_deg, np.ones(num_inputs, dtype=np.int64)])
    w = Workload(num_vars=nv, fac_off=_csr(deg),
                 edge_var=np.concatenate([and_vars, no_vars, np.arange(num_inputs)]).astype(np.int32),
                 fac_type=fac_type, fac_param=np.concatenate([np.zeros(R + num_derived), pin]),
                 edge_param=np.concatenate([np.zeros(len(and_vars)), no_ep, np.zeros(num_inputs)]), edge_rank=None,
                 evidence=np.full(nv, -1, dtype=np.int8), max_iters=max_iters, tol=tol, damping=damping,
                 name="alarms")
    w.alarms = np.arange(T - num_alarms, T, dtype=np.int32)
    w.labels = world[w.alarms].astype(np.int8)
    w.world = world
    w.meta = dict(seed=seed, num_inputs=num_inputs, num_derived=num_derived, num_rules=R)
    return w


def seqfix_ranks(w: Workload) -> np.ndarray:
    """The round-robin asynchronous strategy (SEQFIX, Section 4.2): every edge in its own class, in
    edge order."""
    return np.arange(w.num_edges, dtype=np.int32)


def config(name: str, seed: int = 0, scale: float = 1.0) -> Workload:
    """The five benchmark configurations by short name (C1..C5); ``scale`` shrinks C2/C3/C5 for
    tests that must finish quickly."""
    if name == "C1":
        return datalog(seed)
    if name == "C2":
        lv = max(8, int(500 * scale)) if scale < 1 else 500
        return smartfl(seed, levels=lv)
    if name == "C3":
        return bingo(seed, num_tuples=max(1000, int(2_000_000 * scale)), num_rules=max(2000, int(4_000_000 * scale)))
    if name == "C5":
        return bingo(seed, num_tuples=max(1000, int(20_000_000 * scale)), num_rules=max(2000, int(40_000_000 * scale)),
                     max_iters=200, ranked_classes=64)
    raise ValueError(name)
