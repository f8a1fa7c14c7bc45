"""Adaptive update strategies for the oracle (test infrastructure): the two rank generators and a
run that re-ranks the edges before every block of iterations, written from their definitions.

* SplitMix64 (Steele, Lea and Flood, 2014): the output for counter c of the stream with seed s
  mixes z = s + (c + 1) * 0x9E3779B97F4A7C15 (mod 2^64) through two xor-shift-multiply rounds and a
  final xor-shift.
* Random ordered groups: all edges of factor a in block b get rank SplitMix64(seed, b * 2^32 + a)
  mod groups.
* Residual-driven ranks: r_e = |P_after(e) - P_before(e)| over the previous block (0 for PRIOR
  edges, whose message is constant); with m = max r,
  rank_e = groups - 1 - min(groups - 1, floor(groups * (r_e / m))), all 0 when m = 0.
* bp_adaptive: blocks of `every` iterations (the last one shorter), each on the schedule of the
  ranks drawn before it, from the previous block's messages; the first residual block is flooding
  (rank 0 everywhere); stop after a block that converged or after max_iters iterations.
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, counter: int) -> int:
    z = (seed + (counter + 1) * GAMMA) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def random_group_ranks(fac_off, groups: int, seed: int, block: int) -> np.ndarray:
    fac_off = np.asarray(fac_off)
    nf = len(fac_off) - 1
    per_factor = [splitmix64(seed, (block << 32) + a) % groups for a in range(nf)]
    return np.repeat(np.array(per_factor, dtype=np.int64), np.diff(fac_off)).astype(np.int32)


def residual_ranks(p_before, p_after, groups: int, constant=None) -> np.ndarray:
    """constant: optional mask of edges whose message cannot change (PRIOR edges): r = 0 there."""
    r = np.abs(np.asarray(p_after, dtype=np.float64) - np.asarray(p_before, dtype=np.float64))
    if constant is not None:
        r[np.asarray(constant, dtype=bool)] = 0.0
    m = r.max() if len(r) else 0.0
    if not m > 0.0:
        return np.zeros(len(r), dtype=np.int32)
    bucket = np.minimum(groups - 1, np.floor(groups * (r / m))).astype(np.int64)
    return (groups - 1 - bucket).astype(np.int32)


def bp_adaptive(w, generator: str, groups: int, every: int, seed: int, max_iters: int, tol: float, damping: float,
                evidence="auto"):
    """The oracle's adaptive run; returns (marginals, messages P(x=1), stats, rank arrays per block)."""
    from . import bp_pairs
    E = len(w.edge_var)
    prior = np.repeat(np.asarray(w.fac_type) == 0, np.diff(w.fac_off))
    m0, m1 = np.full(E, 0.5), np.full(E, 0.5)
    before = after = None
    done, block, its, upd, contra = 0, 0, 0, 0, 0
    used = []
    marg, st = None, None
    while done < max_iters:
        if generator == "random":
            ranks = random_group_ranks(w.fac_off, groups, seed, block)
        elif block == 0:
            ranks = np.zeros(E, dtype=np.int32)
        else:
            ranks = residual_ranks(before, after, groups, constant=prior)
        used.append(ranks)
        before = m1.copy()
        marg, m0, m1, st = bp_pairs(w, m0, m1, min(every, max_iters - done), tol, damping, ranks=ranks,
                                    evidence=evidence)
        after = m1.copy()
        its += st["iterations"]
        upd += st["message_updates"]
        contra += st["contradictions"]
        done += st["iterations"]
        block += 1
        if st["converged"]:
            break
    stats = dict(st or {}, iterations=its, message_updates=upd, contradictions=contra)
    return marg, m1, stats, used
