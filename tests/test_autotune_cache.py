"""The autotuner's cache file (host-only part of fastlbp_autotune): a choice is stored under a shape
key, the last valid line for a key wins, malformed or invalid lines are skipped, and a missing
file or key reads as "not cached". The timing itself needs a GPU (tests/test_gpu_autotune.py)."""
import ctypes

import pytest

import paper_2509_22337_amd as F


@pytest.fixture(scope="module")
def lib():
    return F.load()


def _res(executor, tmax, wmax, vmax, iters=0, threads=0, best=1.0, default=2.0, key=0):
    r = F.TuneResult()
    r.executor, r.thread_max_degree, r.wave_max_degree, r.var_thread_max_degree = executor, tmax, wmax, vmax
    r.graph_iters, r.persistent_threads, r.best_ms_per_iter, r.default_ms_per_iter, r.key = (
        iters, threads, best, default, key)
    return r


def test_put_get_roundtrip_and_last_line_wins(tmp_path):
    path = str(tmp_path / "tune.txt")
    assert F.autotune_cache_get(path, 0x1234) is None  # no file yet
    F.autotune_cache_put(path, _res(F.EXEC_LEVELS, 8, 257, 64, iters=4, key=0x1234))
    F.autotune_cache_put(path, _res(F.EXEC_PERSISTENT, 4, 65, 16, threads=1024, key=0xabc))
    got = F.autotune_cache_get(path, 0x1234)
    assert got["executor"] == F.EXEC_LEVELS and got["graph_iters"] == 4 and got["from_cache"] == 1
    assert got["candidates"] == 0
    # a later line for the same key replaces the earlier one
    F.autotune_cache_put(path, _res(F.EXEC_HYBRID, 4, 257, 64, key=0x1234))
    got = F.autotune_cache_get(path, 0x1234)
    assert got["executor"] == F.EXEC_HYBRID and got["thread_max_degree"] == 4
    other = F.autotune_cache_get(path, 0xabc)
    assert other["executor"] == F.EXEC_PERSISTENT and other["persistent_threads"] == 1024
    assert other["wave_max_degree"] == 65 and other["var_thread_max_degree"] == 16
    assert F.autotune_cache_get(path, 0x999) is None


def test_malformed_and_invalid_lines_are_skipped(tmp_path):
    path = tmp_path / "tune.txt"
    key = 0x00000000deadbeef
    path.write_text(
        "garbage line\n"
        f"{key:016x} 1 8 257 64 0 0 1.0 2.0\n"        # valid
        f"{key:016x} 9 8 257 64 0 0 1.0 2.0\n"        # unknown executor
        f"{key:016x} 1 12 257 64 0 0 1.0 2.0\n"       # thread bucket beyond 8
        f"{key:016x} 1 8 300 64 0 0 1.0 2.0\n"        # wavefront bucket beyond 257
        f"{key:016x} 2 8 257 64 0 768 1.0 2.0\n"      # workgroup size not 512 / 1024
        f"{key:016x}z 1 4 257 64 0 0 1.0 2.0\n"       # bad key
        f"{key:016x} 1 4\n")                          # truncated
    got = F.autotune_cache_get(str(path), key)
    assert got["executor"] == F.EXEC_LEVELS and got["thread_max_degree"] == 8


def test_invalid_result_rejected_and_env_path(tmp_path, monkeypatch):
    path = str(tmp_path / "env.txt")
    with pytest.raises(F.FastLBPError):
        F.autotune_cache_put(path, _res(F.EXEC_LEVELS, 9, 257, 64))
    with pytest.raises(F.FastLBPError):
        F.autotune_cache_put(path, _res(F.EXEC_LEVELS, 8, 8, 64))  # wave cut-off must exceed the thread one
    monkeypatch.setenv("FASTLBP_AUTOTUNE_CACHE", path)
    F.autotune_cache_put(None, _res(F.EXEC_LEVELS, 8, 129, 64, key=7))
    assert F.autotune_cache_get(None, 7)["wave_max_degree"] == 129
    monkeypatch.delenv("FASTLBP_AUTOTUNE_CACHE")
    with pytest.raises(F.FastLBPError):
        F.autotune_cache_get(None, 7)
