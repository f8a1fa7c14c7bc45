"""MI355X-native loopy belief propagation with local-structure factors (FastLBP, arXiv 2509.22337).

The compute path is libfastlbp.so (hand-written HIP for gfx950 behind a C ABI declared in
include/fastlbp.h). This module only marshals arguments: numpy arrays in, numpy arrays out, with
PyTorch supplying the HIP stream and (optionally) the device caching allocator. There is no CPU
fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional

import numpy as np

from .workloads import AND, IMPLIES, NOISY_OR, NOT, OR, PRIOR, TERMS  # noqa: F401  (factor tags)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastlbp.so")

OK, E_INVALID_ARG, E_BAD_GRAPH, E_BAD_SCHEDULE, E_OOM, E_DEVICE, E_TOO_LARGE, E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32 = 0, 1
SCHED_FLOODING, SCHED_RANKED = 0, 1
EXEC_AUTO, EXEC_LEVELS, EXEC_PERSISTENT, EXEC_HYBRID = 0, 1, 2, 3
MAX_DEGREE = 16385

_ERR_NAMES = {E_INVALID_ARG: "E_INVALID_ARG", E_BAD_GRAPH: "E_BAD_GRAPH", E_BAD_SCHEDULE: "E_BAD_SCHEDULE",
              E_OOM: "E_OOM", E_DEVICE: "E_DEVICE", E_TOO_LARGE: "E_TOO_LARGE", E_STATE: "E_STATE"}


class FastLBPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("executor", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("alloc", _ALLOC_FN),
                ("free", _FREE_FN), ("alloc_ctx", ctypes.c_void_p)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("precision", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("step_iters", ctypes.c_int32), ("memory_budget", ctypes.c_size_t), ("step_levels", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("message_updates", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("busy_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("method_bytes", ctypes.c_double), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("pending", ctypes.c_int32), ("active", ctypes.c_int32), ("evictions", ctypes.c_int64),
                ("restores", ctypes.c_int64), ("resident_bytes", ctypes.c_size_t),
                ("peak_resident_bytes", ctypes.c_size_t), ("persistent_launches", ctypes.c_int64),
                ("persistent_ms", ctypes.c_double), ("persistent_method_bytes", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class RunStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("residual", ctypes.c_double),
                ("contradictions", ctypes.c_int64), ("levels", ctypes.c_int32), ("executor", ctypes.c_int32),
                ("method_bytes_per_iter", ctypes.c_double), ("impl_bytes_per_iter", ctypes.c_double),
                ("device_ms", ctypes.c_double),
                ("message_updates", ctypes.c_int64), ("thread_max_degree", ctypes.c_int32),
                ("wave_max_degree", ctypes.c_int32), ("var_thread_max_degree", ctypes.c_int32),
                ("graph_iters", ctypes.c_int32), ("persistent_threads", ctypes.c_int32), ("tuned", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class GraphInfo(ctypes.Structure):
    _fields_ = [("num_vars", ctypes.c_int32), ("num_factors", ctypes.c_int32), ("num_edges", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("resident", ctypes.c_int32), ("state_bytes", ctypes.c_size_t),
                ("structure_bytes", ctypes.c_size_t), ("plan_bytes", ctypes.c_size_t), ("levels", ctypes.c_int32),
                ("executed_levels", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [("executor", ctypes.c_int32), ("thread_max_degree", ctypes.c_int32),
                ("wave_max_degree", ctypes.c_int32), ("var_thread_max_degree", ctypes.c_int32),
                ("graph_iters", ctypes.c_int32), ("persistent_threads", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("best_ms_per_iter", ctypes.c_double), ("default_ms_per_iter", ctypes.c_double),
                ("key", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class AlarmStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("true_found", ctypes.c_int32), ("iterations", ctypes.c_int64),
                ("message_updates", ctypes.c_int64), ("device_ms", ctypes.c_double), ("wall_ms", ctypes.c_double),
                ("method_bytes", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


EXPORTS = [
    "fastlbp_options_default", "fastlbp_graph_create", "fastlbp_graph_create_terms", "fastlbp_graph_clone",
    "fastlbp_graph_destroy",
    "fastlbp_run_batch", "fastlbp_schedule_set", "fastlbp_schedule_set_classes", "fastlbp_classes_to_ranks",
    "fastlbp_schedule_levels", "fastlbp_analyze_levels", "fastlbp_graph_validate", "fastlbp_evidence_set",
    "fastlbp_evidence_clear", "fastlbp_run", "fastlbp_marginals", "fastlbp_messages_get", "fastlbp_messages_set",
    "fastlbp_messages_reset", "fastlbp_last_error", "fastlbp_version", "fastlbp_server_options_default",
    "fastlbp_server_create", "fastlbp_server_submit", "fastlbp_server_poll", "fastlbp_server_wait",
    "fastlbp_server_get_stats", "fastlbp_server_destroy", "fastlbp_alarm_loop", "fastlbp_autotune",
    "fastlbp_autotune_cache_get", "fastlbp_autotune_cache_put", "fastlbp_graph_get_info", "fastlbp_run_adaptive",
    "fastlbp_ranks_random", "fastlbp_ranks_residual", "fastlbp_run_noalloc",
]

_lib = None


def load() -> ctypes.CDLL:
    """Loads libfastlbp.so (built by ``paper_2509_22337_amd.build``). Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FastLBPError(E_DEVICE, f"{LIB_PATH} is not built; run paper_2509_22337_amd.build.build()")
    # PyTorch ships its own HIP runtime with the same soname (libamdhip64.so.7) as the system one
    # the library links against. Loading PyTorch first makes the dynamic loader bind the library to
    # that already-loaded runtime, so streams and allocations are shared by one runtime instead of
    # two runtimes living side by side in the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.fastlbp_options_default.argtypes = [ctypes.POINTER(Options)]
    lib.fastlbp_options_default.restype = None
    lib.fastlbp_graph_create.argtypes = [i32, i32, P, P, P, P, P, ctypes.POINTER(Options), ctypes.POINTER(P)]
    lib.fastlbp_graph_create_terms.argtypes = [i32, i32, P, P, P, P, P, P, P, P, ctypes.POINTER(Options),
                                               ctypes.POINTER(P)]
    lib.fastlbp_graph_clone.argtypes = [P, ctypes.POINTER(P)]
    lib.fastlbp_run_batch.argtypes = [i32, P, i32, f64, f64, P]
    lib.fastlbp_graph_destroy.argtypes = [P]
    lib.fastlbp_graph_destroy.restype = None
    lib.fastlbp_schedule_set.argtypes = [P, i32, P, ctypes.POINTER(i32)]
    lib.fastlbp_schedule_levels.argtypes = [P, P]
    lib.fastlbp_analyze_levels.argtypes = [i32, i32, P, P, P, P, ctypes.POINTER(i32)]
    lib.fastlbp_graph_validate.argtypes = [i32, i32, P, P, P, P, P]
    lib.fastlbp_evidence_set.argtypes = [P, i32, P, P]
    lib.fastlbp_evidence_clear.argtypes = [P]
    lib.fastlbp_run.argtypes = [P, i32, f64, f64, ctypes.POINTER(RunStats)]
    lib.fastlbp_run_noalloc.argtypes = [P, i32, f64, f64, ctypes.POINTER(RunStats)]
    lib.fastlbp_marginals.argtypes = [P, P]
    lib.fastlbp_graph_get_info.argtypes = [P, ctypes.POINTER(GraphInfo)]
    lib.fastlbp_run_adaptive.argtypes = [P, i32, i32, i32, ctypes.c_uint64, i32, f64, f64, ctypes.POINTER(RunStats)]
    lib.fastlbp_ranks_random.argtypes = [i32, P, i32, ctypes.c_uint64, i32, P]
    lib.fastlbp_ranks_residual.argtypes = [i64, P, P, i32, P]
    lib.fastlbp_autotune.argtypes = [P, i32, f64, ctypes.c_char_p, ctypes.POINTER(TuneResult)]
    lib.fastlbp_autotune_cache_get.argtypes = [ctypes.c_char_p, ctypes.c_uint64, ctypes.POINTER(TuneResult)]
    lib.fastlbp_autotune_cache_put.argtypes = [ctypes.c_char_p, ctypes.POINTER(TuneResult)]
    lib.fastlbp_alarm_loop.argtypes = [P, i32, P, P, i32, i32, f64, f64, P, P, ctypes.POINTER(AlarmStats)]
    lib.fastlbp_messages_get.argtypes = [P, P]
    lib.fastlbp_messages_set.argtypes = [P, P]
    lib.fastlbp_messages_reset.argtypes = [P]
    lib.fastlbp_last_error.argtypes = []
    lib.fastlbp_last_error.restype = ctypes.c_char_p
    lib.fastlbp_version.argtypes = []
    lib.fastlbp_version.restype = ctypes.c_char_p
    lib.fastlbp_server_options_default.argtypes = [ctypes.POINTER(ServerOptions)]
    lib.fastlbp_server_options_default.restype = None
    lib.fastlbp_server_create.argtypes = [ctypes.POINTER(ServerOptions), ctypes.POINTER(P)]
    lib.fastlbp_server_submit.argtypes = [P, P, i32, P, P, i32, f64, f64, ctypes.POINTER(ctypes.c_uint64)]
    lib.fastlbp_server_poll.argtypes = [P, ctypes.c_uint64, P, ctypes.POINTER(RunStats), ctypes.POINTER(f64)]
    lib.fastlbp_server_wait.argtypes = [P, ctypes.c_uint64, P, ctypes.POINTER(RunStats), ctypes.POINTER(f64)]
    lib.fastlbp_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    lib.fastlbp_server_destroy.argtypes = [P]
    lib.fastlbp_server_destroy.restype = None
    no_rc = ("fastlbp_options_default", "fastlbp_graph_destroy", "fastlbp_last_error", "fastlbp_version",
             "fastlbp_server_options_default", "fastlbp_server_destroy")
    for name in EXPORTS:
        if name not in no_rc:
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        raise FastLBPError(rc, load().fastlbp_last_error().decode())


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _arrays(fac_off, edge_var, fac_type, fac_param=None, edge_param=None):
    fac_off = np.ascontiguousarray(fac_off, dtype=np.int64)
    edge_var = np.ascontiguousarray(edge_var, dtype=np.int32)
    fac_type = np.ascontiguousarray(fac_type, dtype=np.uint8)
    fac_param = None if fac_param is None else np.ascontiguousarray(fac_param, dtype=np.float64)
    edge_param = None if edge_param is None else np.ascontiguousarray(edge_param, dtype=np.float64)
    return fac_off, edge_var, fac_type, fac_param, edge_param


def validate(num_vars, fac_off, edge_var, fac_type, fac_param=None, edge_param=None) -> None:
    """Host-only graph validation (raises FastLBPError)."""
    fo, ev, ft, fp, ep = _arrays(fac_off, edge_var, fac_type, fac_param, edge_param)
    _check(load().fastlbp_graph_validate(int(num_vars), len(ft), _p(fo), _p(ev), _p(ft), _p(fp), _p(ep)))


def analyze_levels(num_vars, fac_off, edge_var, edge_rank) -> tuple[np.ndarray, int]:
    """Host-only dependency analysis: level of every edge and the number of levels."""
    fo = np.ascontiguousarray(fac_off, dtype=np.int64)
    ev = np.ascontiguousarray(edge_var, dtype=np.int32)
    rk = None if edge_rank is None else np.ascontiguousarray(edge_rank, dtype=np.int32)
    out = np.zeros(len(ev), dtype=np.int32)
    n = ctypes.c_int32(0)
    _check(load().fastlbp_analyze_levels(int(num_vars), len(fo) - 1, _p(fo), _p(ev), _p(rk), _p(out), ctypes.byref(n)))
    return out, int(n.value)


def classes_to_ranks(num_vars, fac_off, edge_var, fac_type, edge_class, num_classes: int, arcs=()) -> np.ndarray:
    """Ranks [E] induced by a class preorder (see fastlbp_classes_to_ranks); raises FastLBPError with
    code E_BAD_SCHEDULE for an illegal or cyclic preorder."""
    fo = np.ascontiguousarray(fac_off, dtype=np.int64)
    ev = np.ascontiguousarray(edge_var, dtype=np.int32)
    ft = None if fac_type is None else np.ascontiguousarray(fac_type, dtype=np.uint8)
    ec = np.ascontiguousarray(edge_class, dtype=np.int32)
    if len(ec) != len(ev):
        raise FastLBPError(E_INVALID_ARG, "edge_class must have one entry per edge")
    ar = np.ascontiguousarray(np.asarray(arcs, dtype=np.int32).reshape(-1, 2))
    out = np.zeros(len(ev), dtype=np.int32)
    _check(load().fastlbp_classes_to_ranks(int(num_vars), len(fo) - 1, _p(fo), _p(ev), _p(ft), int(num_classes),
                                           _p(ec), len(ar), _p(ar) if len(ar) else None, _p(out)))
    return out


def _path(p):
    return None if p is None else str(p).encode()


def autotune_cache_get(path, key: int):
    """The cached launch choice for a shape key (dict), or None."""
    r = TuneResult()
    rc = load().fastlbp_autotune_cache_get(_path(path), ctypes.c_uint64(key), ctypes.byref(r))
    if rc == 1:
        return None
    _check(rc)
    return r.as_dict()


def autotune_cache_put(path, result: "TuneResult") -> None:
    _check(load().fastlbp_autotune_cache_put(_path(path), ctypes.byref(result)))


RANKS_RANDOM, RANKS_RESIDUAL = 0, 1


def ranks_random(fac_off, groups: int, seed: int, block: int) -> np.ndarray:
    """Random ordered groups for one block (fastlbp_ranks_random): every factor's edges share a rank
    in [0, groups) from SplitMix64 of the seed, block and factor."""
    fo = np.ascontiguousarray(fac_off, dtype=np.int64)
    out = np.zeros(int(fo[-1]), dtype=np.int32)
    _check(load().fastlbp_ranks_random(len(fo) - 1, _p(fo), int(groups), ctypes.c_uint64(int(seed) & (2**64 - 1)),
                                       int(block), _p(out)))
    return out


def ranks_residual(p_before, p_after, groups: int) -> np.ndarray:
    """Residual-driven ranks (fastlbp_ranks_residual): the edges whose P(x=1) changed most go first."""
    b = np.ascontiguousarray(p_before, dtype=np.float64)
    a = np.ascontiguousarray(p_after, dtype=np.float64)
    if len(a) != len(b):
        raise FastLBPError(E_INVALID_ARG, "two message states of one length")
    out = np.zeros(len(a), dtype=np.int32)
    _check(load().fastlbp_ranks_residual(len(a), _p(b), _p(a), int(groups), _p(out)))
    return out


def run_batch(graphs, max_iters: int, tol: float = 0.0, damping: float = 0.0) -> list:
    """Runs several handles side by side in one persistent launch (one workgroup each)."""
    arr = (ctypes.c_void_p * len(graphs))(*[g._h.value for g in graphs])
    st = (RunStats * len(graphs))()
    _check(load().fastlbp_run_batch(len(graphs), ctypes.cast(arr, ctypes.c_void_p), int(max_iters), float(tol),
                                    float(damping), ctypes.cast(st, ctypes.c_void_p)))
    return [s.as_dict() for s in st]


class _TorchAllocator:
    """Routes the library's device allocations through PyTorch's caching allocator."""

    def __init__(self, device: int, stream):
        import torch
        self.torch = torch
        self.device = device
        self.stream = stream
        self.alloc_cb = _ALLOC_FN(self._alloc)
        self.free_cb = _FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            return int(self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream))
        except Exception:
            return None

    def _free(self, ptr, ctx):
        if ptr:
            self.torch.cuda.caching_allocator_delete(int(ptr))


_LIVE: "weakref.WeakSet[Graph]" = weakref.WeakSet()


@atexit.register
def _close_all():
    # release device memory while PyTorch (which may own the allocator) is still alive
    for g in list(_LIVE):
        try:
            g.close()
        except Exception:
            pass


class Graph:
    """A factor graph resident on one GPU (see include/fastlbp.h for the semantics of every call)."""

    def __init__(self, num_vars, fac_off, edge_var, fac_type, fac_param=None, edge_param=None, precision="fp64",
                 executor="auto", device: int = 0, use_graph: bool = True, allocator: str = "torch", stream=None,
                 term_off=None, term_weight=None, term_ind=None):
        """term_off / term_weight / term_ind describe the TERMS factors (Eq.(4)): factor a owns terms
        term_off[a] .. term_off[a+1], and term t of it fixes its edges to the row of term_ind that
        follows the previous terms' rows (one int8 per edge, -1 = any value)."""
        lib = load()
        self._h = None
        fo, ev, ft, fp, ep = _arrays(fac_off, edge_var, fac_type, fac_param, edge_param)
        self.num_vars = int(num_vars)
        self.num_edges = len(ev)
        self.fac_type = ft
        self.fac_off = fo
        o = Options()
        lib.fastlbp_options_default(ctypes.byref(o))
        o.precision = {"fp64": FP64, "fp32": FP32}[precision]
        o.executor = {"auto": EXEC_AUTO, "levels": EXEC_LEVELS, "persistent": EXEC_PERSISTENT,
                      "hybrid": EXEC_HYBRID}[executor]
        o.device = int(device)
        o.use_graph = 1 if use_graph else 0
        self._keep = []
        self.stream = None
        try:
            import torch
            if torch.cuda.is_available():
                self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
                o.stream = ctypes.c_void_p(self.stream.cuda_stream)
                if allocator == "torch":
                    ta = _TorchAllocator(device, self.stream)
                    self._keep.append(ta)
                    o.alloc = ta.alloc_cb
                    o.free = ta.free_cb
        except ImportError:
            pass
        h = ctypes.c_void_p()
        if term_off is None:
            _check(lib.fastlbp_graph_create(self.num_vars, len(ft), _p(fo), _p(ev), _p(ft), _p(fp), _p(ep),
                                            ctypes.byref(o), ctypes.byref(h)))
        else:
            to = np.ascontiguousarray(term_off, dtype=np.int64)
            tw = np.ascontiguousarray(term_weight, dtype=np.float64)
            ti = np.ascontiguousarray(term_ind, dtype=np.int8)
            if len(to) != len(ft) + 1:
                raise FastLBPError(E_INVALID_ARG, "term_off needs num_factors + 1 entries")
            _check(lib.fastlbp_graph_create_terms(self.num_vars, len(ft), _p(fo), _p(ev), _p(ft), _p(fp), _p(ep),
                                                  _p(to), _p(tw), _p(ti), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.precision = precision
        _LIVE.add(self)

    def clone(self) -> "Graph":
        """Another handle on the same graph (shared structure and schedule, own messages, no
        evidence, own stream)."""
        h = ctypes.c_void_p()
        _check(load().fastlbp_graph_clone(self._h, ctypes.byref(h)))
        g = Graph.__new__(Graph)
        g._h = h
        g._keep = self._keep
        g.stream = self.stream
        g.num_vars, g.num_edges, g.fac_type, g.fac_off = self.num_vars, self.num_edges, self.fac_type, self.fac_off
        g.precision = self.precision
        _LIVE.add(g)
        return g

    @classmethod
    def from_workload(cls, w, **kw) -> "Graph":
        if getattr(w, "term_off", None) is not None:
            kw = dict(kw, term_off=w.term_off, term_weight=w.term_weight, term_ind=w.term_ind)
        g = cls(w.num_vars, w.fac_off, w.edge_var, w.fac_type, w.fac_param, w.edge_param, **kw)
        if w.edge_rank is not None:
            g.schedule_set(SCHED_RANKED, w.edge_rank)
        if w.evidence is not None:
            g.evidence_array(w.evidence)
        return g

    def close(self):
        if self._h is not None:
            load().fastlbp_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def schedule_set(self, kind: int, edge_rank=None) -> int:
        rk = None if edge_rank is None else np.ascontiguousarray(edge_rank, dtype=np.int32)
        if rk is not None and len(rk) != self.num_edges:
            raise FastLBPError(E_INVALID_ARG, "edge_rank must have one entry per edge")
        n = ctypes.c_int32(0)
        _check(load().fastlbp_schedule_set(self._h, int(kind), _p(rk), ctypes.byref(n)))
        return int(n.value)

    def schedule_set_classes(self, edge_class, num_classes: int, arcs=()) -> int:
        """General preorder: class per edge and strict precedences (x, y) between classes."""
        ec = np.ascontiguousarray(edge_class, dtype=np.int32)
        if len(ec) != self.num_edges:
            raise FastLBPError(E_INVALID_ARG, "edge_class must have one entry per edge")
        ar = np.ascontiguousarray(np.asarray(arcs, dtype=np.int32).reshape(-1, 2))
        n = ctypes.c_int32(0)
        _check(load().fastlbp_schedule_set_classes(self._h, int(num_classes), _p(ec), len(ar),
                                                   _p(ar) if len(ar) else None, ctypes.byref(n)))
        return n.value

    def schedule_levels(self) -> np.ndarray:
        out = np.zeros(self.num_edges, dtype=np.int32)
        _check(load().fastlbp_schedule_levels(self._h, _p(out)))
        return out

    def evidence_set(self, vars_, values):
        v = np.ascontiguousarray(vars_, dtype=np.int32)
        x = np.ascontiguousarray(values, dtype=np.int8)
        if len(v) != len(x):
            raise FastLBPError(E_INVALID_ARG, "vars and values differ in length")
        _check(load().fastlbp_evidence_set(self._h, len(v), _p(v), _p(x)))

    def evidence_array(self, ev):
        """Sets the full evidence vector (-1 / 0 / 1 per variable)."""
        ev = np.asarray(ev, dtype=np.int8)
        self.evidence_set(np.arange(len(ev), dtype=np.int32), ev)

    def evidence_clear(self):
        _check(load().fastlbp_evidence_clear(self._h))

    def run(self, max_iters: int, tol: float = 0.0, damping: float = 0.0) -> dict:
        st = RunStats()
        _check(load().fastlbp_run(self._h, int(max_iters), float(tol), float(damping), ctypes.byref(st)))
        return st.as_dict()

    def run_adaptive(self, generator: str, groups: int, every: int, seed: int, max_iters: int, tol: float = 0.0,
                     damping: float = 0.0) -> dict:
        """fastlbp_run_adaptive: blocks of `every` iterations, each on the schedule the generator
        ("random" ordered groups or "residual"-driven ranks) draws before it."""
        gen = {"random": RANKS_RANDOM, "residual": RANKS_RESIDUAL}[generator]
        st = RunStats()
        _check(load().fastlbp_run_adaptive(self._h, gen, int(groups), int(every), ctypes.c_uint64(int(seed) & (2**64 - 1)),
                                           int(max_iters), float(tol), float(damping), ctypes.byref(st)))
        return st.as_dict()

    def run_noalloc(self, max_iters: int, tol: float = 0.0, damping: float = 0.0) -> dict:
        """fastlbp_run_noalloc: the same run without any allocation (fixed per-device scratch area)."""
        st = RunStats()
        _check(load().fastlbp_run_noalloc(self._h, int(max_iters), float(tol), float(damping), ctypes.byref(st)))
        return st.as_dict()

    def info(self) -> dict:
        """Sizes, residency and device memory of the handle (fastlbp_graph_get_info)."""
        r = GraphInfo()
        _check(load().fastlbp_graph_get_info(self._h, ctypes.byref(r)))
        return r.as_dict()

    def autotune(self, probe_iters: int = 4, damping: float = 0.0, cache_path=None) -> dict:
        """fastlbp_autotune: time a few launch choices on this graph and schedule, keep the fastest
        (cached under the graph's shape key in cache_path or FASTLBP_AUTOTUNE_CACHE)."""
        r = TuneResult()
        _check(load().fastlbp_autotune(self._h, int(probe_iters), float(damping), _path(cache_path), ctypes.byref(r)))
        return r.as_dict()

    def marginals(self) -> np.ndarray:
        out = np.zeros(self.num_vars)
        _check(load().fastlbp_marginals(self._h, _p(out)))
        return out

    def messages_get(self) -> np.ndarray:
        out = np.zeros(self.num_edges)
        _check(load().fastlbp_messages_get(self._h, _p(out)))
        return out

    def messages_set(self, p1):
        a = np.ascontiguousarray(p1, dtype=np.float64)
        if len(a) != self.num_edges:
            raise FastLBPError(E_INVALID_ARG, "one message per edge")
        _check(load().fastlbp_messages_set(self._h, _p(a)))

    def messages_reset(self):
        _check(load().fastlbp_messages_reset(self._h))

    def alarm_loop(self, alarm_vars, labels, max_rounds=None, max_iters=500, tol=1e-6, damping=0.0):
        """BINGO's interactive loop with a simulated user (fastlbp_alarm_loop): returns the
        inspection order (positions in alarm_vars), each pick's marginal and the loop's stats."""
        av = np.ascontiguousarray(alarm_vars, dtype=np.int32)
        lb = np.ascontiguousarray(labels, dtype=np.int8)
        if len(av) != len(lb):
            raise FastLBPError(E_INVALID_ARG, "one label per alarm")
        n = len(av) if max_rounds is None else int(max_rounds)
        order = np.zeros(max(n, 1), dtype=np.int32)
        prob = np.zeros(max(n, 1))
        st = AlarmStats()
        _check(load().fastlbp_alarm_loop(self._h, len(av), _p(av), _p(lb), n, int(max_iters), float(tol),
                                         float(damping), _p(order), _p(prob), ctypes.byref(st)))
        r = st.rounds
        return order[:r].copy(), prob[:r].copy(), st.as_dict()


def inversion_count(labels_in_order) -> int:
    """Pairs of inspected alarms where a false alarm comes before a true one (Section 5.3):
    the sum over false alarms of the true alarms inspected after them."""
    l = np.asarray(labels_in_order, dtype=np.int64)
    true_after = np.cumsum(l[::-1])[::-1] - l  # true alarms strictly after each position
    return int(((1 - l) * true_after).sum())


def rank_of_fraction(labels_in_order, frac: float, total_true: Optional[int] = None) -> int:
    """Interactions needed to find at least ceil(frac x total_true) true alarms (Rank-100%-T for
    frac = 1, Rank-90%-T for 0.9); -1 if the sequence does not reach that many."""
    l = np.asarray(labels_in_order, dtype=np.int64)
    total = int(l.sum()) if total_true is None else int(total_true)
    need = int(np.ceil(frac * total - 1e-9))
    if need <= 0:
        return 0
    hit = np.flatnonzero(np.cumsum(l) >= need)
    return int(hit[0]) + 1 if len(hit) else -1


class Server:
    """Continuous-batching query server (see include/fastlbp.h): requests on graph handles are
    admitted between steps and advanced side by side, one workgroup per run."""

    def __init__(self, precision: str = "fp32", device: int = 0, max_active: int = 256, step_iters: int = 2,
                 memory_budget: int = 0, step_levels=None):
        """step_levels: levels per step for each run (None: the library default, 0: step_iters)."""
        lib = load()
        o = ServerOptions()
        lib.fastlbp_server_options_default(ctypes.byref(o))
        o.device = int(device)
        o.precision = {"fp64": FP64, "fp32": FP32}[precision]
        o.max_active = int(max_active)
        o.step_iters = int(step_iters)
        o.memory_budget = int(memory_budget)
        if step_levels is not None:
            o.step_levels = int(step_levels)
        h = ctypes.c_void_p()
        _check(lib.fastlbp_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._nv = {}
        _LIVE_SERVERS.add(self)

    def submit(self, graph: "Graph", ev_vars=(), ev_vals=(), max_iters: int = 100, tol: float = 0.0,
               damping: float = 0.0) -> int:
        v = np.ascontiguousarray(ev_vars, dtype=np.int32)
        x = np.ascontiguousarray(ev_vals, dtype=np.int8)
        if len(v) != len(x):
            raise FastLBPError(E_INVALID_ARG, "vars and values differ in length")
        t = ctypes.c_uint64(0)
        _check(load().fastlbp_server_submit(self._h, graph._h, len(v), _p(v), _p(x), int(max_iters), float(tol),
                                            float(damping), ctypes.byref(t)))
        self._nv[t.value] = np.empty(graph.num_vars)  # receives the marginals
        return t.value

    def _collect(self, fn, ticket):
        p1 = self._nv.get(ticket)
        if p1 is None:
            p1 = np.empty(0)
        st = RunStats()
        lat = ctypes.c_double(0.0)
        rc = fn(self._h, ctypes.c_uint64(ticket), _p(p1), ctypes.byref(st), ctypes.byref(lat))
        if rc == 1:
            return None
        self._nv.pop(ticket, None)
        _check(rc)
        return p1, st.as_dict(), lat.value

    def poll(self, ticket: int):
        """None while pending, else (marginals, stats, latency_ms)."""
        return self._collect(load().fastlbp_server_poll, ticket)

    def wait(self, ticket: int):
        return self._collect(load().fastlbp_server_wait, ticket)

    def stats(self) -> dict:
        s = ServerStats()
        _check(load().fastlbp_server_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().fastlbp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_LIVE_SERVERS: "weakref.WeakSet[Server]" = weakref.WeakSet()


@atexit.register
def _close_servers():
    for s in list(_LIVE_SERVERS):
        try:
            s.close()
        except Exception:
            pass
