"""Pure-Python definitions that pin the C oracle (test infrastructure only).

Everything here is written for clarity on tiny inputs, not for speed:
  * ``factor_value``        the factor function f_a(x_a) of each catalogue type (definition form);
  * ``eq2_messages``        Eq.(2) (Section 3.2) by enumerating every assignment of the factor;
  * ``type_terms`` and ``alg1_message``  the local-structure representation of Eq.(4) (Section 3.3)
                            and Algorithm 1 evaluated on it;
  * ``exact_marginals``     P(X_v = 1) by enumerating the joint distribution (Section 3.1);
  * ``edge_neighbourhood``  N_E of Definition 1 (Section 4.2);
  * ``alg2_as_printed`` and ``alg2_class_atomic``  Algorithm 2 (Section 4.2.3) and the variant
                            that cuts only between rank classes;
  * ``check_theorem2``      the two properties of Theorem 2 for a given grouping.
"""
from __future__ import annotations

import itertools

import numpy as np

PRIOR, AND, OR, NOT, IMPLIES, NOISY_OR = 0, 1, 2, 3, 4, 5


# ------------------------------------------------------------------------------------------------
# Factor functions
# ------------------------------------------------------------------------------------------------

def factor_value(ftype: int, x, fparam: float = 0.0, eparam=None) -> float:
    """f_a(x) for one assignment x (tuple of 0/1 over the factor's edges, head last)."""
    x = tuple(int(v) for v in x)
    if ftype == PRIOR:
        return fparam if x[0] == 1 else 1.0 - fparam
    xs, y = x[:-1], x[-1]
    if ftype == AND:
        return 1.0 if y == int(all(xs)) else 0.0
    if ftype == OR:
        return 1.0 if y == int(any(xs)) else 0.0
    if ftype == NOT:
        return 1.0 if y == 1 - xs[0] else 0.0
    if ftype == IMPLIES:
        if all(xs):
            return fparam if y == 1 else 1.0 - fparam
        return 1.0
    if ftype == NOISY_OR:
        p0 = 1.0 - fparam
        for j, xj in enumerate(xs):
            if xj:
                p0 *= 1.0 - eparam[j]
        return p0 if y == 0 else 1.0 - p0
    raise ValueError(ftype)


def eq2_messages(ftype: int, m0, m1, fparam: float = 0.0, eparam=None):
    """Eq.(2): mu_{a->v}(x_v) = sum over x_a \\ x_v of f_a(x_a) * prod_{v* != v} mu_{v*->a}(x_v*),
    by enumerating all 2^d assignments. Returns unnormalised (out0, out1) per edge."""
    d = len(m0)
    m = np.stack([np.asarray(m0, float), np.asarray(m1, float)], axis=1)
    out = np.zeros((d, 2))
    for x in itertools.product((0, 1), repeat=d):
        f = factor_value(ftype, x, fparam, eparam)
        if f == 0.0:
            continue
        for v in range(d):
            prod = f
            for j in range(d):
                if j != v:
                    prod *= m[j, x[j]]
            out[v, x[v]] += prod
    return out[:, 0], out[:, 1]


def terms_value(weights, ind, x) -> float:
    """A weighted-term factor at assignment x: sum over terms of the weight times the indicator that
    x agrees with every fixed value of the term (ind [l][d], -1 = wildcard)."""
    tot = 0.0
    for t in range(len(weights)):
        if all(c == -1 or c == xi for c, xi in zip(ind[t], x)):
            tot += float(weights[t])
    return tot


def eq2_messages_terms(weights, ind, m0, m1):
    """Eq.(2) for a weighted-term factor by enumerating all 2^d assignments."""
    d = len(m0)
    m = np.stack([np.asarray(m0, float), np.asarray(m1, float)], axis=1)
    out = np.zeros((d, 2))
    for x in itertools.product((0, 1), repeat=d):
        f = terms_value(weights, ind, x)
        if f == 0.0:
            continue
        for v in range(d):
            prod = f
            for j in range(d):
                if j != v:
                    prod *= m[j, x[j]]
            out[v, x[v]] += prod
    return out[:, 0], out[:, 1]


# ------------------------------------------------------------------------------------------------
# Local-structure terms (Eq.(4)) and Algorithm 1
# ------------------------------------------------------------------------------------------------

def type_terms(ftype: int, d: int, fparam: float = 0.0, eparam=None):
    """Weights p[l] and indicator[d][l] (value 0/1, or -1 = wildcard) of disjoint cubes whose
    weighted sum is the factor function. Deterministic types and the Horn rule need O(d) terms;
    NOISY_OR has no compact cube form (its weight depends on which inputs are 1), so every input
    assignment becomes its own term (exponential, tiny d only)."""
    W, IND = [], []
    n = d - 1

    def term(w, ind):
        W.append(w)
        IND.append(list(ind))

    if ftype == PRIOR:
        term(1.0 - fparam, [0])
        term(fparam, [1])
    elif ftype == NOT:
        term(1.0, [0, 1])
        term(1.0, [1, 0])
    elif ftype in (OR, AND, IMPLIES):
        nofire = 0 if ftype == OR else 1
        fire = 1 - nofire
        # every input at its "no-fire" value
        if ftype == OR:
            term(1.0, [0] * n + [0])
        elif ftype == AND:
            term(1.0, [1] * n + [1])
        else:
            term(fparam, [1] * n + [1])
            term(1.0 - fparam, [1] * n + [0])
        # input k is the first one at its "fire" value
        for k in range(n):
            ind = [nofire] * k + [fire] + [-1] * (n - k - 1)
            if ftype == OR:
                ind.append(1)
            elif ftype == AND:
                ind.append(0)
            else:
                ind.append(-1)
            term(1.0, ind)
    elif ftype == NOISY_OR:
        for xs in itertools.product((0, 1), repeat=n):
            p0 = factor_value(NOISY_OR, tuple(xs) + (0,), fparam, eparam)
            term(p0, list(xs) + [0])
            term(1.0 - p0, list(xs) + [1])
    else:
        raise ValueError(ftype)
    return np.array(W), np.array(IND, dtype=np.int64).T  # indicator[d][l]


def alg1_message(v: int, xv: int, p, indicator, mu):
    """Algorithm 1 (Section 3.3): one entry mu_{a->v}(x_v) as the sum of sub-messages.
    p[l] weights, indicator[b][l] values, mu[b][r] incoming messages."""
    b, l = indicator.shape
    r = mu.shape[1]
    message = 0.0
    for t in range(l):
        if indicator[v][t] != xv and indicator[v][t] != -1:
            continue
        sm = p[t]
        for j in range(b):
            if j == v:
                continue
            c = indicator[j][t]
            if c == -1:
                sm *= sum(mu[j][k] for k in range(r))
            else:
                sm *= mu[j][c]
        message += sm
    return message


# ------------------------------------------------------------------------------------------------
# Exact marginals by enumeration
# ------------------------------------------------------------------------------------------------

def exact_marginals(w, evidence="auto"):
    """P(X_v = 1 | evidence) from P(X) = 1/Z prod_a f_a(X_a) by enumerating all 2^V assignments."""
    V = int(w.num_vars)
    assert V <= 22, "enumeration only for tiny graphs"
    if isinstance(evidence, str):
        evidence = w.evidence
    S = 1 << V
    states = np.arange(S, dtype=np.int64)
    bits = ((states[None, :] >> np.arange(V)[:, None]) & 1).astype(np.int8)  # [V, S]
    weight = np.ones(S)
    if evidence is not None:
        for v in range(V):
            if evidence[v] >= 0:
                weight *= (bits[v] == evidence[v])
    for a in range(len(w.fac_type)):
        vs = w.edge_var[w.fac_off[a]:w.fac_off[a + 1]]
        ep = w.edge_param[w.fac_off[a]:w.fac_off[a + 1]]
        d = len(vs)
        table = np.zeros(1 << d)
        for x in itertools.product((0, 1), repeat=d):
            idx = sum(bit << j for j, bit in enumerate(x))
            table[idx] = factor_value(int(w.fac_type[a]), x, float(w.fac_param[a]), ep)
        idx = np.zeros(S, dtype=np.int64)
        for j, v in enumerate(vs):
            idx |= bits[v].astype(np.int64) << j
        weight *= table[idx]
    Z = weight.sum()
    if Z <= 0:
        return np.full(V, np.nan), Z
    return (bits * weight[None, :]).sum(axis=1) / Z, Z


# ------------------------------------------------------------------------------------------------
# Dependency analysis (Section 4.2)
# ------------------------------------------------------------------------------------------------

def edge_lists(w):
    E = len(w.edge_var)
    edge_fac = np.repeat(np.arange(len(w.fac_type)), np.diff(w.fac_off))
    fac_vars = [list(w.edge_var[w.fac_off[a]:w.fac_off[a + 1]]) for a in range(len(w.fac_type))]
    var_facs = [[] for _ in range(int(w.num_vars))]
    for e in range(E):
        var_facs[int(w.edge_var[e])].append(int(edge_fac[e]))
    edge_of = {(int(edge_fac[e]), int(w.edge_var[e])): e for e in range(E)}
    return edge_fac, fac_vars, var_facs, edge_of


def edge_neighbourhood(w):
    """N_E of Definition 1 for every edge e = (a, v):
    { (a*, v*) : v* in N_A(a) \\ {v}, a* in N_V(v*) \\ {a} }, as sets of edge ids."""
    edge_fac, fac_vars, var_facs, edge_of = edge_lists(w)
    NE = []
    for e in range(len(w.edge_var)):
        a, v = int(edge_fac[e]), int(w.edge_var[e])
        s = set()
        for vs in fac_vars[a]:
            if vs == v:
                continue
            for a2 in var_facs[vs]:
                if a2 == a:
                    continue
                s.add(edge_of[(a2, vs)])
        NE.append(s)
    return NE


def _topological_order(ranks):
    """Edges sorted by (rank, edge id): a topological order of the rank classes, ties inside a
    class broken by edge id."""
    return sorted(range(len(ranks)), key=lambda e: (int(ranks[e]), e))


def alg2_as_printed(w, ranks, NE=None):
    """Algorithm 2 as printed: scan edges in topological order; start a new batch when the next
    edge has an N_E-neighbour in the current batch that strictly precedes it. Returns the batch
    index of every edge."""
    NE = edge_neighbourhood(w) if NE is None else NE
    order = _topological_order(ranks)
    level = np.full(len(ranks), -1, dtype=np.int64)
    cur, nxt = 0, []
    for ei in order:
        for e in nxt:
            if e in NE[ei] and ranks[e] < ranks[ei]:
                cur += 1
                nxt = []
                break
        nxt.append(ei)
        level[ei] = cur
    return level


def alg2_class_atomic(w, ranks, NE=None):
    """Algorithm 2 with cuts only between rank classes: a whole class joins the current batch
    unless one of its edges has an N_E-neighbour in the batch (which then precedes it strictly),
    in which case the class starts a new batch."""
    NE = edge_neighbourhood(w) if NE is None else NE
    order = _topological_order(ranks)
    level = np.full(len(ranks), -1, dtype=np.int64)
    cur, batch = 0, set()
    i = 0
    while i < len(order):
        j = i
        while j < len(order) and ranks[order[j]] == ranks[order[i]]:
            j += 1
        cls = order[i:j]
        if any(NE[ei] & batch for ei in cls):
            cur += 1
            batch = set()
        for ei in cls:
            batch.add(ei)
            level[ei] = cur
        i = j
    return level


def check_theorem2(w, ranks, level, NE=None):
    """Theorem 2: for e in batch j and e' in N_E(e): e' < e strictly => batch(e') < j;
    e <= e' => batch(e') >= j. Returns the list of violating (e, e') pairs."""
    NE = edge_neighbourhood(w) if NE is None else NE
    bad = []
    for e in range(len(ranks)):
        for e2 in NE[e]:
            if ranks[e2] < ranks[e] and not level[e2] < level[e]:
                bad.append((e, e2))
            if ranks[e] <= ranks[e2] and not level[e2] >= level[e]:
                bad.append((e, e2))
    return bad


# ----------------------------------------------------------------------------------------------
# General preorders (Definition 2): classes of edges and strict arcs between classes
# ----------------------------------------------------------------------------------------------

def class_reach(num_classes, arcs):
    """reach[x] = set of classes strictly after x (transitive closure of the arcs, by search)."""
    succ = [[] for _ in range(num_classes)]
    for x, y in arcs:
        succ[int(x)].append(int(y))
    reach = []
    for x in range(num_classes):
        seen, stack = set(), list(succ[x])
        while stack:
            y = stack.pop()
            if y not in seen:
                seen.add(y)
                stack.extend(succ[y])
        reach.append(seen)
    return reach


def preorder_is_acyclic(num_classes, arcs):
    reach = class_reach(num_classes, arcs)
    return all(x not in reach[x] for x in range(num_classes))


def preorder_legal(w, edge_class, num_classes, arcs, NE=None):
    """Definition 2: every edge e1 and every e2 in N_E(e1) lie in comparable classes. Pairs with a
    PRIOR edge are skipped (a PRIOR message is constant, so its position cannot matter)."""
    NE = edge_neighbourhood(w) if NE is None else NE
    reach = class_reach(num_classes, arcs)
    edge_fac = np.repeat(np.arange(len(w.fac_type)), np.diff(w.fac_off))
    prior = w.fac_type[edge_fac] == 0
    for e1 in range(len(edge_class)):
        if prior[e1]:
            continue
        for e2 in NE[e1]:
            if prior[e2]:
                continue
            x, y = int(edge_class[e1]), int(edge_class[e2])
            if not (x == y or y in reach[x] or x in reach[y]):
                return False
    return True


def linear_extension(num_classes, arcs, rng=None):
    """Position of each class in a topological order of the arcs: smallest ready class first, or a
    random ready class when rng is given."""
    succ = [[] for _ in range(num_classes)]
    indeg = [0] * num_classes
    for x, y in arcs:
        succ[int(x)].append(int(y))
        indeg[int(y)] += 1
    ready = [c for c in range(num_classes) if indeg[c] == 0]
    pos = [-1] * num_classes
    k = 0
    while ready:
        if rng is None:
            c = min(ready)
        else:
            c = ready[int(rng.integers(0, len(ready)))]
        ready.remove(c)
        pos[c] = k
        k += 1
        for y in succ[c]:
            indeg[y] -= 1
            if indeg[y] == 0:
                ready.append(y)
    return np.array(pos, dtype=np.int64)
