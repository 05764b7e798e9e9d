"""CPU oracle for single-source shortest paths.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use it; the GPU library never does, and the two share no
code. See ``oracle.c`` for what each function computes and which passage of
the paper it follows (Section 2.1: problem statement, Dijkstra, Bellman-Ford;
Section 5.7: breadth-first search).

Every function here is pinned by tests against things other than itself:
brute-force path enumeration, Floyd-Warshall, closed forms on grids, paths and
stars, the hand-worked redundant-wavefront example (Section 3.2) and
scipy.sparse.csgraph.dijkstra.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK = 0
ERR_INVALID_ARG = -1
ERR_OUT_OF_MEMORY = -2
ERR_DISTANCE_OVERFLOW = -3
CERT_BAD_SOURCE = -10
CERT_EDGE_VIOLATED = -11
CERT_UNSUPPORTED = -12
UNREACHABLE = 0xFFFFFFFF


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"oracle error {code} {msg}".strip())
        self.code = code


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        i64p = ctypes.POINTER(ctypes.c_int64)
        for name in ("oracle_dijkstra", "oracle_bellman_ford"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [i64, vp, vp, vp, i64, vp]
        lib.oracle_certificate.restype = ctypes.c_int
        lib.oracle_certificate.argtypes = [i64, vp, vp, vp, i64, vp, i64p, i64p]
        lib.oracle_reach_stats.restype = ctypes.c_int
        lib.oracle_reach_stats.argtypes = [i64, vp, vp, i64p, i64p]
        lib.oracle_bfs.restype = ctypes.c_int
        lib.oracle_bfs.argtypes = [i64, vp, vp, i64, vp]
        _lib = lib
    return _lib


def _csr_args(g):
    off = np.ascontiguousarray(g.off, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.uint32)
    return off, col, w


def _solve(fn_name: str, g, src: int, allow_overflow: bool) -> np.ndarray:
    off, col, w = _csr_args(g)
    dist = np.empty(g.n, dtype=np.uint32)
    rc = getattr(_load(), fn_name)(g.n, off.ctypes.data, col.ctypes.data, w.ctypes.data, int(src),
                                   dist.ctypes.data)
    if rc == ERR_DISTANCE_OVERFLOW and allow_overflow:
        return dist
    if rc != OK:
        raise OracleError(rc, fn_name)
    return dist


def dijkstra(g, src: int, allow_overflow: bool = False) -> np.ndarray:
    """Shortest distances from src (uint32, UNREACHABLE where no path)."""
    return _solve("oracle_dijkstra", g, src, allow_overflow)


def bellman_ford(g, src: int, allow_overflow: bool = False) -> np.ndarray:
    return _solve("oracle_bellman_ford", g, src, allow_overflow)


def bfs(g, src: int) -> np.ndarray:
    """Breadth-first levels from src (fewest edges; UNREACHABLE where no path)."""
    off, col, _ = _csr_args(g)
    level = np.empty(g.n, dtype=np.uint32)
    rc = _load().oracle_bfs(g.n, off.ctypes.data, col.ctypes.data, int(src), level.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "oracle_bfs")
    return level


def certificate(g, src: int, dist: np.ndarray):
    """Return (code, where, depth); code 0 iff dist is the shortest-distance vector."""
    off, col, w = _csr_args(g)
    d = np.ascontiguousarray(dist, dtype=np.uint32)
    if d.shape != (g.n,):
        raise ValueError("distance vector has the wrong length")
    where = ctypes.c_int64()
    depth = ctypes.c_int64()
    rc = _load().oracle_certificate(g.n, off.ctypes.data, col.ctypes.data, w.ctypes.data, int(src),
                                    d.ctypes.data, ctypes.byref(where), ctypes.byref(depth))
    return rc, where.value, depth.value


def reach_stats(g, dist: np.ndarray):
    """(n_reach, m_reach): finite vertices and directed edges leaving them."""
    off = np.ascontiguousarray(g.off, dtype=np.int64)
    d = np.ascontiguousarray(dist, dtype=np.uint32)
    nr = ctypes.c_int64()
    mr = ctypes.c_int64()
    rc = _load().oracle_reach_stats(g.n, off.ctypes.data, d.ctypes.data, ctypes.byref(nr), ctypes.byref(mr))
    if rc != OK:
        raise OracleError(rc, "reach_stats")
    return nr.value, mr.value
