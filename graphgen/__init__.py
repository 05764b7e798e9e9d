"""Seeded synthetic CSR graphs (input generation only).

This module holds no shortest-path arithmetic. It serves both the CPU oracle
(``oracle/``) and the GPU library, and neither of those imports the other.

Shapes stand in for the paper's workloads (Section 5.1, Table 4): road-like
grids (4-neighbour, each undirected edge dropped with probability p), meshes
(grids without drops), RMAT power-law graphs and uniform random graphs.
Weights are 1 + (hash mod wmax), one draw per undirected pair.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile libgraphgen.so with g++ (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c++17", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.gg_draw.restype = ctypes.c_uint64
        lib.gg_draw.argtypes = [ctypes.c_uint64] * 3
        lib.gg_set_threads.restype = ctypes.c_int
        lib.gg_set_threads.argtypes = [ctypes.c_int]
        lib.gg_grid.restype = ctypes.c_int64
        lib.gg_grid.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32,
                                ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.gg_rmat_build.restype = ctypes.c_int
        lib.gg_rmat_build.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                                      i64p, i64p]
        lib.gg_uniform_build.restype = ctypes.c_int
        lib.gg_uniform_build.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                                         ctypes.c_uint64, i64p, i64p]
        lib.gg_take.restype = ctypes.c_int
        lib.gg_take.argtypes = [ctypes.c_void_p] * 3
        _lib = lib
    return _lib


@dataclass
class Csr:
    """Directed graph in CSR form: row r's out-edges are col[off[r]:off[r+1]]."""
    n: int
    off: np.ndarray          # int64[n+1]
    col: np.ndarray          # int32[m]
    w: np.ndarray            # uint32[m]
    name: str = ""
    params: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.off[-1])

    def off32(self) -> np.ndarray:
        if self.m >= 2**31:
            raise ValueError("graph too large for int32 offsets")
        return self.off.astype(np.int32)

    def degrees(self) -> np.ndarray:
        return np.diff(self.off)


def draw(seed: int, stream: int, index: int) -> int:
    return int(_load().gg_draw(seed, stream, index))


def set_threads(t: int) -> int:
    return int(_load().gg_set_threads(int(t)))


def grid(rows: int, cols: int, p_drop: float = 0.0, wmax: int = 255, seed: int = 1) -> Csr:
    lib = _load()
    n = rows * cols
    off = np.empty(n + 1, dtype=np.int64)
    m = lib.gg_grid(rows, cols, float(p_drop), wmax, seed, off.ctypes.data, None, None)
    if m < 0:
        raise ValueError("bad grid parameters")
    col = np.empty(m, dtype=np.int32)
    w = np.empty(m, dtype=np.uint32)
    lib.gg_grid(rows, cols, float(p_drop), wmax, seed, off.ctypes.data, col.ctypes.data, w.ctypes.data)
    return Csr(n, off, col, w, name=f"grid{rows}x{cols}",
               params=dict(kind="grid", rows=rows, cols=cols, p_drop=p_drop, wmax=wmax, seed=seed))


def _take(n: int, m: int) -> tuple:
    off = np.empty(n + 1, dtype=np.int64)
    col = np.empty(m, dtype=np.int32)
    w = np.empty(m, dtype=np.uint32)
    _load().gg_take(off.ctypes.data, col.ctypes.data, w.ctypes.data)
    return off, col, w


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         permute: bool = True, wmax: int = 255, seed: int = 1) -> Csr:
    lib = _load()
    n = ctypes.c_int64()
    m = ctypes.c_int64()
    if lib.gg_rmat_build(scale, edge_factor, a, b, c, int(permute), wmax, seed,
                         ctypes.byref(n), ctypes.byref(m)) != 0:
        raise ValueError("bad rmat parameters")
    off, col, w = _take(n.value, m.value)
    return Csr(n.value, off, col, w, name=f"rmat{scale}",
               params=dict(kind="rmat", scale=scale, edge_factor=edge_factor, a=a, b=b, c=c,
                           permute=permute, wmax=wmax, seed=seed))


def uniform(n: int, npairs: int, wmax: int = 65535, seed: int = 1) -> Csr:
    lib = _load()
    nn = ctypes.c_int64()
    m = ctypes.c_int64()
    if lib.gg_uniform_build(n, npairs, wmax, seed, ctypes.byref(nn), ctypes.byref(m)) != 0:
        raise ValueError("bad uniform parameters")
    off, col, w = _take(nn.value, m.value)
    return Csr(nn.value, off, col, w, name=f"uniform{n}",
               params=dict(kind="uniform", n=n, npairs=npairs, wmax=wmax, seed=seed))


def from_edges(n: int, src, dst, w) -> Csr:
    """CSR from an explicit edge list (kept as given: self-loops and multi-edges stay)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    w = np.asarray(w, dtype=np.uint64)
    if src.size and (src.min() < 0 or src.max() >= n or dst.min() < 0 or dst.max() >= n):
        raise ValueError("vertex id out of range")
    if w.size and w.max() > 0xFFFFFFFF:
        raise ValueError("weight out of uint32 range")
    order = np.lexsort((dst, src))
    src, dst, w = src[order], dst[order], w[order]
    off = np.zeros(n + 1, dtype=np.int64)
    np.add.at(off, src + 1, 1)
    off = np.cumsum(off)
    return Csr(n, off, dst.astype(np.int32), w.astype(np.uint32), name="edges")


def random_small(n: int, nedges: int, wmax: int, rng: np.random.Generator, wmin: int = 0) -> Csr:
    """Tiny random multigraph (self-loops and parallel edges allowed) for brute-force tests."""
    src = rng.integers(0, n, nedges)
    dst = rng.integers(0, n, nedges)
    w = rng.integers(wmin, wmax + 1, nedges)
    return from_edges(n, src, dst, w)


def max_degree_vertex(g: Csr) -> int:
    """Highest out-degree vertex, ties to the smallest id."""
    return int(np.argmax(g.degrees()))


def sample_sources(g: Csr, k: int, seed: int) -> np.ndarray:
    """k distinct sources drawn uniformly from vertices with out-degree >= 1."""
    cand = np.nonzero(g.degrees() > 0)[0]
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cand, size=min(k, cand.size), replace=False)).astype(np.uint32)
