"""Seeded synthetic graph inputs shared by the GPU library and the CPU oracle.

Raw inputs only: R-MAT and grid edge lists (self-loops and duplicates kept),
integer edge weights 1..64, query sources and Poisson arrival times.  Nothing
here cleans, sorts or traverses a graph; each consumer does that itself.

R-MAT follows the experimental setup of the paper (Section 8, dataset
paragraph): (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), 2^scale vertices,
edge_factor * 2^scale generated edges, weights uniform integers in 1..64.
The 2-D grid (a stand-in for the paper's road networks) has vertex id
r * cols + c and 4-neighbour edges.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")

#: default seeds: graph structure, edge weights, query sources, arrivals
SEED_GRAPH = 1
SEED_WEIGHTS = 2
SEED_SOURCES = 3
SEED_ARRIVALS = 4

RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = True) -> str:
    """Compile libgraphgen.so in place (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, u64, p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        lib.gg_rmat_edges.argtypes = [ctypes.c_int, i64, u64, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, p, p]
        lib.gg_rmat_edges.restype = None
        lib.gg_grid_num_edges.argtypes = [i64, i64]
        lib.gg_grid_num_edges.restype = i64
        lib.gg_grid_edges.argtypes = [i64, i64, p, p]
        lib.gg_grid_edges.restype = None
        lib.gg_edge_weights.argtypes = [i64, p, p, i64, u64, p]
        lib.gg_edge_weights.restype = None
        lib.gg_touched.argtypes = [i64, p, p, i64, p]
        lib.gg_touched.restype = None
        lib.gg_sources.argtypes = [i64, p, i64, u64, p]
        lib.gg_sources.restype = i64
        lib.gg_splitmix64.argtypes = [u64]
        lib.gg_splitmix64.restype = u64
        lib.gg_uniform_ints.argtypes = [i64, u64, u64, p]
        lib.gg_uniform_ints.restype = None
        lib.gg_uniform_doubles.argtypes = [i64, u64, p]
        lib.gg_uniform_doubles.restype = None
        lib.gg_poisson_arrivals.argtypes = [i64, u64, ctypes.c_double, p]
        lib.gg_poisson_arrivals.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def splitmix64(x: int) -> int:
    return int(_load().gg_splitmix64(x))


def rmat_edges(scale: int, edge_factor: int = 16, seed: int = SEED_GRAPH,
               abc=RMAT_ABC):
    """Raw R-MAT edge list (src, dst) of edge_factor << scale int32 pairs."""
    m = edge_factor << scale
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    a, b, c = abc
    _load().gg_rmat_edges(scale, edge_factor, seed, a, b, c, _ptr(src), _ptr(dst))
    return src, dst


def grid_edges(rows: int, cols: int):
    """Each undirected 4-neighbour edge of a rows x cols grid, once."""
    lib = _load()
    m = lib.gg_grid_num_edges(rows, cols)
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    lib.gg_grid_edges(rows, cols, _ptr(src), _ptr(dst))
    return src, dst


def edge_weights(src: np.ndarray, dst: np.ndarray, n: int,
                 seed: int = SEED_WEIGHTS) -> np.ndarray:
    """Symmetric integer weights 1..64 as float32, one per raw edge."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    w = np.empty(src.shape[0], dtype=np.float32)
    _load().gg_edge_weights(src.shape[0], _ptr(src), _ptr(dst), n, seed, _ptr(w))
    return w


def touched(src: np.ndarray, dst: np.ndarray, n: int) -> np.ndarray:
    """Boolean mask of vertices incident to a non-self-loop edge."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    flags = np.empty(n, dtype=np.uint8)
    _load().gg_touched(src.shape[0], _ptr(src), _ptr(dst), n, _ptr(flags))
    return flags.astype(bool)


def sources(src: np.ndarray, dst: np.ndarray, n: int, k: int,
            seed: int = SEED_SOURCES) -> np.ndarray:
    """k distinct sources, uniform over vertices with degree > 0."""
    flags = touched(src, dst, n).astype(np.uint8)
    out = np.empty(max(k, 0), dtype=np.int32)
    got = _load().gg_sources(n, _ptr(flags), k, seed, _ptr(out))
    if got < 0:
        raise MemoryError("gg_sources: allocation failed")
    return out[:got]


def uniform_ints(count: int, bound: int, seed: int) -> np.ndarray:
    out = np.empty(count, dtype=np.int64)
    _load().gg_uniform_ints(count, seed, bound, _ptr(out))
    return out


def uniform_doubles(count: int, seed: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _load().gg_uniform_doubles(count, seed, _ptr(out))
    return out


def poisson_arrivals(count: int, rate: float, seed: int = SEED_ARRIVALS) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _load().gg_poisson_arrivals(count, seed, float(rate), _ptr(out))
    return out


@dataclasses.dataclass
class RawGraph:
    """A raw (uncleaned) edge list plus what consumers need to clean it."""
    name: str
    n: int
    src: np.ndarray
    dst: np.ndarray
    w: np.ndarray | None
    symmetric: bool  # True: consumers symmetrise; False: directed as given


def rmat(scale: int, edge_factor: int = 16, *, symmetric: bool = True,
         weights: bool = True, seed: int = SEED_GRAPH,
         wseed: int = SEED_WEIGHTS) -> RawGraph:
    n = 1 << scale
    src, dst = rmat_edges(scale, edge_factor, seed)
    w = edge_weights(src, dst, n, wseed) if weights else None
    kind = "rmat" if symmetric else "rmat_dir"
    return RawGraph(f"{kind}_s{scale}_e{edge_factor}", n, src, dst, w, symmetric)


def grid(rows: int, cols: int, *, weights: bool = True,
         wseed: int = SEED_WEIGHTS) -> RawGraph:
    n = rows * cols
    src, dst = grid_edges(rows, cols)
    w = edge_weights(src, dst, n, wseed) if weights else None
    return RawGraph(f"grid_{rows}x{cols}", n, src, dst, w, True)


def from_edges(name: str, n: int, src, dst, w=None, symmetric: bool = True) -> RawGraph:
    """Wraps a hand-written edge list (tests) in the same container."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float32)
    return RawGraph(name, n, src, dst, w, symmetric)
