"""Rank generators of the adaptive update strategies, on the CPU: the oracle's SplitMix64 against
the generator's published output sequence, the library's host generators (fastlbp_ranks_random,
fastlbp_ranks_residual) against the oracle's independent ones bit for bit, uniformity of the random
groups, and hand-derived residual ranks."""
import numpy as np
import pytest

import paper_2509_22337_amd as F
from oracle import adaptive as A
from paper_2509_22337_amd import workloads as W


def test_splitmix64_published_sequence():
    # SplitMix64 with state 0: the first three outputs of the reference generator
    assert A.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert A.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert A.splitmix64(0, 2) == 0x06C45D188009454F


def test_random_ranks_library_equals_oracle():
    for seed, groups, block in ((0, 4, 0), (12345, 64, 3), (2**63 + 11, 7, 17)):
        w = W.random_loopy(seed % 1000, num_vars=50, num_factors=80)
        lib = F.ranks_random(w.fac_off, groups, seed, block)
        ora = A.random_group_ranks(w.fac_off, groups, seed, block)
        assert np.array_equal(lib, ora)
        assert lib.min() >= 0 and lib.max() < groups
        # every edge of a factor shares its factor's rank
        for a in range(w.num_factors):
            assert len(set(lib[w.fac_off[a]:w.fac_off[a + 1]])) <= 1


def test_random_ranks_are_uniform_and_vary_by_block():
    nf, groups = 40000, 16
    off = np.arange(nf + 1, dtype=np.int64)
    r0 = F.ranks_random(off, groups, 99, 0)
    counts = np.bincount(r0, minlength=groups)
    chi2 = float(((counts - nf / groups) ** 2 / (nf / groups)).sum())
    assert chi2 < 45.0  # 15 degrees of freedom: P(chi2 > 45) < 1e-4
    r1 = F.ranks_random(off, groups, 99, 1)
    assert (r0 == r1).mean() < 0.1  # blocks draw independent ranks (1/16 agree by chance)


def test_residual_ranks_hand_derived():
    before = np.array([0.5, 0.5, 0.5, 0.25])
    after = np.array([0.625, 0.5, 1.0, 0.25])
    # changes 1/8, 0, 1/2, 0; max 1/2; 4 * (r / max) = 1, 0, 4, 0 -> buckets 1, 0, 3, 0
    expect = np.array([2, 3, 0, 3], dtype=np.int32)
    assert np.array_equal(F.ranks_residual(before, after, 4), expect)
    assert np.array_equal(A.residual_ranks(before, after, 4), expect)
    assert np.array_equal(F.ranks_residual(before, before, 4), np.zeros(4, dtype=np.int32))
    # a constant (PRIOR) edge with a spurious change counts as unchanged in the oracle's form
    assert np.array_equal(A.residual_ranks(before, after, 4, constant=[False, False, True, False]),
                          np.array([0, 3, 3, 3], dtype=np.int32))


def test_residual_ranks_library_equals_oracle():
    rng = np.random.default_rng(4)
    for groups in (1, 2, 8, 64):
        b = rng.random(5000)
        a = np.clip(b + rng.normal(0, 0.05, 5000), 0, 1)
        same = rng.random(5000) < 0.1
        a[same] = b[same]  # some unchanged
        assert np.array_equal(F.ranks_residual(b, a, groups), A.residual_ranks(b, a, groups))


def test_host_generator_errors():
    with pytest.raises(F.FastLBPError):
        F.ranks_random(np.array([0, 2, 1], dtype=np.int64), 4, 0, 0)
    with pytest.raises(F.FastLBPError):
        F.ranks_residual(np.array([0.5]), np.array([1.5]), 4)
    with pytest.raises(F.FastLBPError):
        F.ranks_residual(np.array([0.5]), np.array([0.5]), 0)
