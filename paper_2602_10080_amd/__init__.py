"""Python binding of the MLMQ SSSP library (libmlmq.so, HIP for gfx950).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels. PyTorch provides device memory and streams. If the library is not
built it is compiled once; if it cannot be loaded every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np

from . import build as _build

_LIB_PATH = _build.LIB
_lib = None

OK = 0
ERR_INVALID_ARG = -1
ERR_OUT_OF_MEMORY = -2
ERR_DISTANCE_OVERFLOW = -3
ERR_QUEUE_CAPACITY = -4
ERR_TIMEOUT = -5
ERR_DEVICE = -6
ERR_CANCELED = -7
ERR_BUSY = -8
UNREACHABLE = 0xFFFFFFFF

L1_NONE, L1_VEC, L1_NEARFAR, L1_FILTER, L1_SLF = 0, 1, 2, 3, 4
RELAX_PRECHECK, RELAX_ATOMIC = 0, 1
L2_FIFO, L2_BUCKET, L2_PQ = 0, 1, 2
MEM_HOST, MEM_DEVICE = 0, 1
GRAPH_KEEP_ORDER, GRAPH_DEGREE_ORDER = 2, 4

# C-ABI entry points declared in include/mlmq.h
EXPORTS = (
    "mlmq_config_default", "mlmq_graph_create", "mlmq_graph_destroy", "mlmq_graph_info", "mlmq_graph_config",
    "mlmq_features_host", "mlmq_sssp", "mlmq_sssp_noalloc", "mlmq_bfs", "mlmq_check", "mlmq_latency_probe",
    "mlmq_sssp_batch",
    "mlmq_candidate_count", "mlmq_candidate_config", "mlmq_select_inputs", "mlmq_select_rank", "mlmq_select",
    "mlmq_autotune", "mlmq_server_create",
    "mlmq_server_submit", "mlmq_server_poll", "mlmq_server_wait", "mlmq_server_times",
    "mlmq_server_destroy", "mlmq_last_error",
)


class MlmqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mlmq error {code}: {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("status", ctypes.c_uint32), ("kernel_ms", ctypes.c_double),
        ("worker_ms", ctypes.c_double),
        ("expansions", ctypes.c_uint64), ("stale", ctypes.c_uint64), ("edges", ctypes.c_uint64),
        ("pushes", ctypes.c_uint64), ("l1_writes", ctypes.c_uint64), ("l1_reads", ctypes.c_uint64),
        ("l2_writes", ctypes.c_uint64), ("l2_reads", ctypes.c_uint64), ("hub_chunks", ctypes.c_uint64),
        ("flushes", ctypes.c_uint64), ("grid_wgs", ctypes.c_uint32), ("retries", ctypes.c_uint32),
        ("donations", ctypes.c_uint64), ("atomics", ctypes.c_uint64), ("wave_ms", ctypes.c_double),
        ("idle_ms", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "struct_size"}


class Config(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("l0_rows", ctypes.c_uint8), ("l1_type", ctypes.c_uint8),
        ("l2_type", ctypes.c_uint8), ("relax_mode", ctypes.c_uint8), ("l1_cap", ctypes.c_uint32),
        ("l1_flush_wb", ctypes.c_uint32), ("delta1", ctypes.c_uint32), ("delta2_log2", ctypes.c_uint32),
        ("bmax", ctypes.c_uint32), ("bnum", ctypes.c_uint32), ("th_v", ctypes.c_uint32),
        ("th_hub", ctypes.c_uint32), ("hub_chunk", ctypes.c_uint32), ("wg_size", ctypes.c_uint32),
        ("grid_wgs", ctypes.c_uint32), ("l2_capacity", ctypes.c_uint64), ("stream", ctypes.c_void_p),
        ("timeout_ms", ctypes.c_uint32), ("max_retries", ctypes.c_uint32),
        ("stats_out", ctypes.POINTER(Stats)), ("donate_min", ctypes.c_uint32), ("pnum", ctypes.c_uint32),
    ]

    KNOBS = ("l0_rows", "l1_type", "l2_type", "relax_mode", "l1_cap", "l1_flush_wb", "delta1", "delta2_log2", "bmax",
             "bnum", "th_v", "th_hub", "hub_chunk", "wg_size", "grid_wgs", "l2_capacity", "timeout_ms",
             "max_retries", "donate_min", "pnum")

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k in self.KNOBS}

    def copy(self, **kw) -> "Config":
        c = Config()
        ctypes.pointer(c)[0] = self
        for k, v in kw.items():
            setattr(c, k, v)
        return c


class Features(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("n", "nnz", "avg_deg", "max_deg", "std_deg", "avg_w", "std_w", "max_w")]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def _declare(lib):
    vp, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "mlmq_config_default": (ctypes.c_int, [ctypes.POINTER(Config)]),
        "mlmq_graph_create": (ctypes.c_int, [i32, i64, vp, vp, vp, u32, ctypes.POINTER(vp)]),
        "mlmq_graph_destroy": (None, [vp]),
        "mlmq_graph_config": (ctypes.c_int, [vp, ctypes.POINTER(Config)]),
        "mlmq_graph_info": (ctypes.c_int, [vp, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                           ctypes.POINTER(Features)]),
        "mlmq_features_host": (ctypes.c_int, [i32, i64, vp, vp, vp, ctypes.POINTER(Features)]),
        "mlmq_sssp": (ctypes.c_int, [vp, u32, vp, ctypes.POINTER(Config)]),
        "mlmq_sssp_noalloc": (ctypes.c_int, [vp, u32, vp, ctypes.POINTER(Config)]),
        "mlmq_bfs": (ctypes.c_int, [vp, u32, vp, ctypes.POINTER(Config)]),
        "mlmq_check": (ctypes.c_int, [vp, u32, vp, vp, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_float)]),
        "mlmq_latency_probe": (ctypes.c_int, [vp, u32, u32, vp, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double)]),
        "mlmq_sssp_batch": (ctypes.c_int, [vp, vp, vp, i32, vp, vp]),
        "mlmq_candidate_count": (i32, []),
        "mlmq_candidate_config": (ctypes.c_int, [vp, i32, ctypes.POINTER(Config)]),
        "mlmq_select_inputs": (ctypes.c_int, [ctypes.POINTER(Features), i32, ctypes.POINTER(ctypes.c_float)]),
        "mlmq_select_rank": (ctypes.c_int, [ctypes.POINTER(Features), vp, vp, i32]),
        "mlmq_select": (ctypes.c_int, [vp, ctypes.POINTER(Config)]),
        "mlmq_autotune": (ctypes.c_int, [vp, u32, ctypes.POINTER(Config)]),
        "mlmq_server_create": (ctypes.c_int, [vp, i32, u64, i32, ctypes.POINTER(Config), ctypes.POINTER(vp)]),
        "mlmq_server_submit": (ctypes.c_int, [vp, i32, u32, vp, ctypes.POINTER(u64)]),
        "mlmq_server_poll": (ctypes.c_int, [vp, u64, ctypes.POINTER(i32)]),
        "mlmq_server_wait": (ctypes.c_int, [vp, u64, u32]),
        "mlmq_server_times": (ctypes.c_int, [vp, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)]),
        "mlmq_server_destroy": (None, [vp]),
        "mlmq_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        try:
            f = getattr(lib, name)
        except AttributeError:
            continue  # reported by the export test; calling it raises AttributeError
        f.restype = res
        f.argtypes = args


def lib():
    """The loaded library (built on first use if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            _build.build()
        try:
            l = ctypes.CDLL(_LIB_PATH)
        except OSError as e:  # fail loudly: there is no other path
            raise RuntimeError(f"cannot load the MLMQ HIP library {_LIB_PATH}: {e}") from e
        _declare(l)
        _lib = l
    return _lib


def _check(rc: int) -> None:
    if rc != OK:
        raise MlmqError(rc, lib().mlmq_last_error().decode(errors="replace"))


def default_config(**overrides) -> Config:
    c = Config()
    c.struct_size = ctypes.sizeof(Config)
    _check(lib().mlmq_config_default(ctypes.byref(c)))
    for k, v in overrides.items():
        setattr(c, k, v)
    return c


def features(csr) -> dict:
    off = np.ascontiguousarray(csr.off, dtype=np.int32)
    col = np.ascontiguousarray(csr.col, dtype=np.int32)
    w = np.ascontiguousarray(csr.w, dtype=np.uint32)
    f = Features()
    _check(lib().mlmq_features_host(int(csr.n), int(col.size), off.ctypes.data, col.ctypes.data,
                                    w.ctypes.data, ctypes.byref(f)))
    return f.as_dict()


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        torch = _torch()
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


class Graph:
    """A device-resident graph. Build from any object with n, off, col, w
    (e.g. graphgen.Csr) or from arrays; torch CUDA tensors are read on device."""

    def __init__(self, n: int, off, col, w, keep_order: bool = False, degree_order: bool = False):
        self._h = ctypes.c_void_p()
        flags = MEM_HOST
        keep = []
        if hasattr(off, "is_cuda") and off.is_cuda:
            flags = MEM_DEVICE
            torch = _torch()
            off = off.to(torch.int32).contiguous()
            col = col.to(torch.int32).contiguous()
            w = w.contiguous()
            ptrs = (off.data_ptr(), col.data_ptr(), w.data_ptr())
            m = col.numel()
            keep = [off, col, w]
        else:
            off = np.ascontiguousarray(off, dtype=np.int64)
            if off[-1] >= 2**31:
                raise ValueError("graph too large for int32 offsets")
            off = off.astype(np.int32)
            col = np.ascontiguousarray(col, dtype=np.int32)
            w = np.ascontiguousarray(w, dtype=np.uint32)
            ptrs = (off.ctypes.data, col.ctypes.data, w.ctypes.data)
            m = col.size
            keep = [off, col, w]
        if keep_order:
            flags |= GRAPH_KEEP_ORDER
        if degree_order:
            flags |= GRAPH_DEGREE_ORDER
        _check(lib().mlmq_graph_create(int(n), int(m), *ptrs, flags, ctypes.byref(self._h)))
        del keep
        self.n = int(n)
        self.m = int(m)

    @classmethod
    def from_csr(cls, csr, keep_order: bool = False, degree_order: bool = False) -> "Graph":
        return cls(csr.n, csr.off, csr.col, csr.w, keep_order=keep_order, degree_order=degree_order)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("graph is closed")
        return self._h

    def config(self) -> Config:
        """The config a solve uses when none is given (tuned, else heuristic)."""
        c = Config()
        c.struct_size = ctypes.sizeof(Config)
        _check(lib().mlmq_graph_config(self.handle, ctypes.byref(c)))
        return c

    def features(self) -> dict:
        f = Features()
        _check(lib().mlmq_graph_info(self.handle, None, None, ctypes.byref(f)))
        return f.as_dict()

    def close(self) -> None:
        if self._h:
            lib().mlmq_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def new_dist(n: int):
    """A device buffer for n uint32 distances (int32 storage)."""
    torch = _torch()
    return torch.empty(n, dtype=torch.int32, device="cuda")


def to_numpy(dist) -> np.ndarray:
    """uint32 view of a distance buffer (torch tensor or numpy array)."""
    if hasattr(dist, "is_cuda"):
        dist = dist.detach().cpu().numpy()
    return np.ascontiguousarray(dist).view(np.uint32)


def sssp(graph: Graph, source: int, out=None, config: Optional[Config] = None, stream=None,
         stats: bool = False):
    """Shortest distances from source into out (device tensor allocated if None,
    or a host uint32 numpy array). config None = the graph's tuned/default
    config. Returns out, or (out, stats dict) when stats=True."""
    return _single("mlmq_sssp", graph, source, out, config, stream, stats)


def sssp_noalloc(graph: Graph, source: int, out, config: Optional[Config] = None, stream=None,
                 stats: bool = False):
    """mlmq_sssp_noalloc: the same solve with the library's fixed queue array
    (no allocation inside the call); out must be a device tensor of n 4-byte
    elements that the caller allocated."""
    if not hasattr(out, "is_cuda"):
        raise ValueError("out must be a CUDA tensor")
    return _single("mlmq_sssp_noalloc", graph, source, out, config, stream, stats)


def bfs(graph: Graph, source: int, out=None, config: Optional[Config] = None, stream=None,
        stats: bool = False):
    """Breadth-first levels (fewest edges) from source; weights are ignored.
    config None = the graph's config with a one-level near-far window and
    unit bucket width (what mlmq_bfs uses for a NULL config)."""
    if config is None:
        config = graph.config()
        config.delta1 = 1
        config.delta2_log2 = 0
    return _single("mlmq_bfs", graph, source, out, config, stream, stats)


def check(graph: Graph, source: int, dist, stream=None):
    """Optimality check of a device distance vector (mlmq_check): returns
    (violations, edge_pass_ms); 0 violations = dist is the exact
    shortest-distance vector from source (positive weights only)."""
    if not (hasattr(dist, "is_cuda") and dist.is_cuda and dist.numel() == graph.n and dist.element_size() == 4
            and dist.is_contiguous()):
        raise ValueError("dist must be a contiguous 4-byte CUDA tensor of n elements")
    bad = ctypes.c_uint64()
    ms = ctypes.c_float()
    _check(lib().mlmq_check(graph.handle, int(source), dist.data_ptr(), _stream_handle(stream), ctypes.byref(bad),
                            ctypes.byref(ms)))
    return int(bad.value), float(ms.value)


def latency_probe(graph: Graph, source: int, hops: int = 4096, stream=None):
    """(ns per dependent relaxation hop, ns per hand-off between two
    workgroups) measured on graph's device copy (mlmq_latency_probe)."""
    hop = ctypes.c_double()
    hand = ctypes.c_double()
    _check(lib().mlmq_latency_probe(graph.handle, int(source), int(hops), _stream_handle(stream), ctypes.byref(hop),
                                    ctypes.byref(hand)))
    return float(hop.value), float(hand.value)


def _single(fn: str, graph: Graph, source: int, out, config: Optional[Config], stream, stats: bool):
    if out is None:
        out = new_dist(graph.n)
    if hasattr(out, "is_cuda"):
        if (not out.is_cuda or out.numel() != graph.n or out.element_size() != 4
                or not out.is_contiguous()):
            raise ValueError("out must be a contiguous 4-byte CUDA tensor of n elements")
        ptr = out.data_ptr()
    else:
        if out.dtype != np.uint32 or out.size != graph.n or not out.flags.c_contiguous:
            raise ValueError("out must be a contiguous uint32 array of n elements")
        ptr = out.ctypes.data
    cfg = config.copy() if config is not None else graph.config()
    if hasattr(out, "is_cuda") or stream is not None:
        cfg.stream = _stream_handle(stream)
    st = None
    if stats:
        st = Stats()
        st.struct_size = ctypes.sizeof(Stats)
        cfg.stats_out = ctypes.pointer(st)
    _check(getattr(lib(), fn)(graph.handle, int(source), ptr, ctypes.byref(cfg)))
    if stats:
        return out, st.as_dict()
    return out


def sssp_batch(graphs: Sequence[Graph], sources: Sequence[int], outs=None,
               configs: Optional[Sequence[Optional[Config]]] = None, stream=None, stats: bool = False):
    """Solve many (graph, source) queries in one persistent launch.
    Returns (outs, statuses) or (outs, statuses, stats list)."""
    nq = len(graphs)
    if len(sources) != nq:
        raise ValueError("graphs and sources differ in length")
    if outs is None:
        outs = [new_dist(g.n) for g in graphs]
    gh = (ctypes.c_void_p * nq)(*[g.handle.value for g in graphs])
    src = (ctypes.c_uint32 * nq)(*[int(s) for s in sources])
    dp = (ctypes.c_void_p * nq)(*[o.data_ptr() for o in outs])
    st_list, keep = [], []
    for i in range(nq):
        base = configs[i] if configs is not None and configs[i] is not None else None
        c = base.copy() if base is not None else graphs[i].config()
        c.stream = _stream_handle(stream)
        if stats:
            s = Stats()
            s.struct_size = ctypes.sizeof(Stats)
            c.stats_out = ctypes.pointer(s)
            st_list.append(s)
        keep.append(c)
    cfg_arr = (ctypes.c_void_p * nq)(*[ctypes.addressof(c) for c in keep])
    status = (ctypes.c_int32 * nq)()
    rc = lib().mlmq_sssp_batch(gh, src, dp, nq, cfg_arr, status)
    if rc != OK and all(s == OK for s in status):
        _check(rc)
    res = (outs, list(status))
    if stats:
        return res + ([s.as_dict() for s in st_list],)
    return res


def autotune(graph: Graph, budget_ms: int = 2000, stream=None) -> Config:
    """Times the feature-driven default and the selector's top templates; the
    winner is cached in the library for this graph (used when no config is
    passed) and returned."""
    c = default_config()
    c.stream = _stream_handle(stream)
    _check(lib().mlmq_autotune(graph.handle, int(budget_ms), ctypes.byref(c)))
    c.stream = None
    return c


def candidate_count() -> int:
    return int(lib().mlmq_candidate_count())


def candidate_config(graph: Graph, t: int) -> Config:
    """Template t (or the feature-driven default for t = -1) as a config for graph."""
    c = default_config()
    _check(lib().mlmq_candidate_config(graph.handle, int(t), ctypes.byref(c)))
    return c


def _features_struct(f) -> Features:
    if isinstance(f, Features):
        return f
    s = Features()
    for k, _ in Features._fields_:
        setattr(s, k, float(f[k]))
    return s


def select_inputs(f, t: int) -> np.ndarray:
    """The selector's model inputs for template t on features f (host only)."""
    x = (ctypes.c_float * 20)()
    _check(lib().mlmq_select_inputs(ctypes.byref(_features_struct(f)), int(t), x))
    return np.frombuffer(x, dtype=np.float32).copy()


def select_rank(f) -> tuple:
    """(template ids best first, predicted relative performance per template)
    for features f (host only)."""
    k = candidate_count()
    order = np.empty(k, np.int32)
    scores = np.empty(k, np.float32)
    _check(lib().mlmq_select_rank(ctypes.byref(_features_struct(f)), order.ctypes.data, scores.ctypes.data, k))
    return order, scores


def select(graph: Graph) -> Config:
    """The selector's top template for graph (nothing is timed or cached)."""
    c = default_config()
    _check(lib().mlmq_select(graph.handle, ctypes.byref(c)))
    return c


class Server:
    """Continuous-batching SSSP server over resident graphs."""

    def __init__(self, graphs: Sequence[Graph], mem_budget_bytes: int, max_slots: int = 64,
                 config: Optional[Config] = None):
        self._h = ctypes.c_void_p()
        self.graphs = list(graphs)
        arr = (ctypes.c_void_p * len(graphs))(*[g.handle.value for g in graphs])
        cfg = config.copy() if config is not None else None
        _check(lib().mlmq_server_create(arr, len(graphs), int(mem_budget_bytes), int(max_slots),
                                        ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(self._h)))

    def submit(self, graph_id: int, source: int, out) -> int:
        t = ctypes.c_uint64()
        _check(lib().mlmq_server_submit(self._h, int(graph_id), int(source), out.data_ptr(), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> int:
        st = ctypes.c_int32()
        _check(lib().mlmq_server_poll(self._h, int(ticket), ctypes.byref(st)))
        return st.value

    def wait(self, ticket: int, timeout_ms: int = 60000) -> int:
        return int(lib().mlmq_server_wait(self._h, int(ticket), int(timeout_ms)))

    def times(self, ticket: int):
        a = ctypes.c_uint64()
        b = ctypes.c_uint64()
        _check(lib().mlmq_server_times(self._h, int(ticket), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def close(self) -> None:
        if self._h:
            lib().mlmq_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
