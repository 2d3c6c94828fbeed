"""ORACLE — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct CPU implementations of what the GPU library
computes, written from the paper (GraphBLAST, Yang, Buluc and Owens):

* :func:`Adjacency` — graph cleaning of the experimental section (dataset
  table caption: self-loops and duplicate edges removed, undirected graphs
  symmetrised), built from the raw edge list by its own code.
* :func:`bfs` — level-synchronous BFS of Algorithm 1 as a queue BFS; levels
  are hop counts (the paper's 1-based d minus one), parents are the
  smallest-id neighbour one level up.
* :func:`sssp` — exact single-source shortest paths (Dijkstra), the result
  the paper's Bellman-Ford variant (Section 7.2) converges to.
* :func:`pagerank` — FP64 power iteration (Section 7.3) with uniform
  redistribution of dangling mass and an L1 stopping rule.
* :func:`pagerank_adaptive` — adaptive PageRank (PageRankDelta): the same
  iteration with converged vertices frozen (the masked form named in
  Sections 5.1 and 7.3).
* :func:`msbfs` — k independent BFS runs (multi-nodeset traversal).
* :func:`triangles` — triangle count and per-vertex counts by definition
  (Section 7.5), each triangle found once from its lowest edge.
* :mod:`oracle.mxv` — the plain-loop masked semiring mxv / vxm over
  dictionaries (small inputs), and :func:`mxv_dense` — the same definition
  in C over dense arrays (full-size inputs).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library and imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import mxv as mxv_mod  # noqa: F401  (re-export)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile liboracle.so in place (gcc -O2, single-threaded code)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra",
               "-pthread", "-o", _LIB + ".tmp", _SRC, "-lm"]
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
        p, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.oracle_adj_build.argtypes = [i64, i64, p, p, p, ctypes.c_int]
        lib.oracle_adj_build.restype = p
        lib.oracle_adj_free.argtypes = [p]
        lib.oracle_adj_free.restype = None
        lib.oracle_adj_nnz.argtypes = [p]
        lib.oracle_adj_nnz.restype = i64
        lib.oracle_adj_n.argtypes = [p]
        lib.oracle_adj_n.restype = i64
        lib.oracle_adj_copy.argtypes = [p, p, p, p]
        lib.oracle_adj_copy.restype = None
        lib.oracle_adj_transpose.argtypes = [p]
        lib.oracle_adj_transpose.restype = p
        lib.oracle_bfs.argtypes = [p, i32, p, p]
        lib.oracle_bfs.restype = i32
        lib.oracle_sssp.argtypes = [p, i32, p, p]
        lib.oracle_sssp.restype = i64
        lib.oracle_pagerank.argtypes = [p, f64, i32, f64, p, p]
        lib.oracle_pagerank.restype = i32
        lib.oracle_pagerank_adaptive.argtypes = [p, f64, i32, f64, f64, p, p, p, p]
        lib.oracle_pagerank_adaptive.restype = i32
        lib.oracle_triangles.argtypes = [p, p]
        lib.oracle_triangles.restype = i64
        lib.oracle_msbfs.argtypes = [p, i64, p, p, i32]
        lib.oracle_msbfs.restype = i32
        lib.oracle_mxv.argtypes = [p, i32, i32, p, p, p, p, p, p, i32, i32, p, p]
        lib.oracle_mxv.restype = i32
        lib.oracle_cc.argtypes = [p, p]
        lib.oracle_cc.restype = i64
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class Adjacency:
    """Cleaned adjacency lists of a raw edge list (rows ascending)."""

    def __init__(self, n, src, dst, w=None, symmetrise=True, _handle=None):
        lib = _load()
        self.n = int(n)
        if _handle is not None:
            self._h = _handle
        else:
            src = np.ascontiguousarray(src, dtype=np.int32)
            dst = np.ascontiguousarray(dst, dtype=np.int32)
            w = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
            self._h = lib.oracle_adj_build(self.n, src.shape[0], _ptr(src), _ptr(dst),
                                           _ptr(w), 1 if symmetrise else 0)
            if not self._h:
                raise ValueError("oracle_adj_build failed (bad vertex id or out of memory)")
        self.nnz = int(lib.oracle_adj_nnz(self._h))
        self.weighted = w is not None if _handle is None else None

    @classmethod
    def from_raw(cls, g):
        """From a graphgen.RawGraph."""
        return cls(g.n, g.src, g.dst, g.w, symmetrise=g.symmetric)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oracle_adj_free(h)
            self._h = None

    def arrays(self, weights=True):
        """(off int64[n+1], nbr int32[nnz], w float64[nnz] or None)."""
        off = np.empty(self.n + 1, dtype=np.int64)
        nbr = np.empty(self.nnz, dtype=np.int32)
        w = np.empty(self.nnz, dtype=np.float64) if weights else None
        _load().oracle_adj_copy(self._h, _ptr(off), _ptr(nbr), _ptr(w))
        return off, nbr, w

    def transpose(self):
        h = _load().oracle_adj_transpose(self._h)
        t = Adjacency(self.n, None, None, _handle=h)
        t.weighted = self.weighted
        return t


def bfs(adj: Adjacency, source: int, parents: bool = True):
    """(levels int32[n], parents int32[n] or None, number of levels)."""
    lev = np.empty(adj.n, dtype=np.int32)
    par = np.empty(adj.n, dtype=np.int32) if parents else None
    nl = _load().oracle_bfs(adj._h, int(source), _ptr(lev), _ptr(par))
    if nl < 0:
        raise ValueError("oracle_bfs: bad source")
    return lev, par, int(nl)


def sssp(adj: Adjacency, source: int):
    """(dist float32[n] with +inf unreached, dist float64[n], reached count)."""
    d32 = np.empty(adj.n, dtype=np.float32)
    d64 = np.empty(adj.n, dtype=np.float64)
    r = _load().oracle_sssp(adj._h, int(source), _ptr(d32), _ptr(d64))
    if r < 0:
        raise ValueError("oracle_sssp: bad source or unweighted graph")
    return d32, d64, int(r)


def pagerank(adj_out: Adjacency, alpha=0.85, max_iter=50, tol=1e-7):
    """(p float64[n], iterations run, last L1 delta); adj_out = out-edges."""
    p = np.empty(adj_out.n, dtype=np.float64)
    delta = ctypes.c_double(0.0)
    it = _load().oracle_pagerank(adj_out._h, float(alpha), int(max_iter), float(tol),
                                 _ptr(p), ctypes.byref(delta))
    if it < 0:
        raise ValueError("oracle_pagerank: bad input")
    return p, int(it), float(delta.value)


def pagerank_adaptive(adj_out: Adjacency, eps: float, alpha=0.85, max_iter=50, tol=1e-7):
    """Adaptive PageRank (PageRankDelta): (p float64[n], iterations run, last
    L1 delta, vertices still active, frozen_at int32[n] = iteration at which
    each vertex froze, 0 if never)."""
    p = np.empty(adj_out.n, dtype=np.float64)
    fz = np.empty(adj_out.n, dtype=np.int32)
    delta = ctypes.c_double(0.0)
    active = ctypes.c_int64(0)
    it = _load().oracle_pagerank_adaptive(adj_out._h, float(alpha), int(max_iter), float(tol),
                                          float(eps), _ptr(p), _ptr(fz), ctypes.byref(delta),
                                          ctypes.byref(active))
    if it < 0:
        raise ValueError("oracle_pagerank_adaptive: bad input")
    return p, int(it), float(delta.value), int(active.value), fz


def triangles(adj: Adjacency):
    """(triangle count, per-vertex counts int64[n]) of a symmetric adjacency."""
    pv = np.empty(adj.n, dtype=np.int64)
    t = _load().oracle_triangles(adj._h, _ptr(pv))
    if t < 0:
        raise ValueError("oracle_triangles: bad input")
    return int(t), pv


def cc(adj: Adjacency):
    """(labels int32[n], number of components): the smallest vertex id of
    each vertex's component (symmetric adjacency)."""
    lab = np.empty(adj.n, dtype=np.int32)
    c = _load().oracle_cc(adj._h, _ptr(lab))
    if c < 0:
        raise ValueError("oracle_cc: bad input")
    return lab, int(c)


def msbfs(adj: Adjacency, sources, nthreads: int = 1):
    """levels int32[k, n] of k independent BFS runs."""
    src = np.ascontiguousarray(sources, dtype=np.int32)
    lev = np.empty((src.shape[0], adj.n), dtype=np.int32)
    rc = _load().oracle_msbfs(adj._h, src.shape[0], _ptr(src), _ptr(lev), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_msbfs: bad source")
    return lev


# semiring and accumulator codes of oracle_mxv (the library's numbering)
MXV_SEMIRINGS = {"lor_land": 0, "min_plus_fp32": 1, "min_plus_fp64": 2, "plus_times_fp32": 3,
                 "plus_times_fp64": 4, "min_first_int32": 5, "min_second_int32": 6}
MXV_ACCUMS = {None: 0, "min": 1, "plus": 2, "lor": 3}
MXV_COMP, MXV_STRUCT, MXV_REPLACE = 1, 2, 8


def mxv_dense(rows: Adjacency, semiring: str, u_val, u_has, *, vec_first=False, w_val=None,
              w_has=None, mask_val=None, mask_has=None, flags=0, accum=None):
    """w<mask> = accum(w, A' u) by its definition over dense arrays (C loop,
    fp64).  `rows` holds the rows of A' (pass the transpose for a product
    over A^T); vec_first gives the vxm operand order.  Vectors are value
    arrays plus boolean presence arrays; mask_has None = no mask.  Returns
    (values float64[n], present bool[n])."""
    n = rows.n
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    u8 = lambda a: np.ascontiguousarray(a, dtype=np.uint8)
    uv, uh = f64(u_val), u8(u_has)
    wv = f64(np.zeros(n) if w_val is None else w_val)
    wh = u8(np.zeros(n) if w_has is None else w_has)
    mv = None if mask_val is None else f64(mask_val)
    mh = None if mask_has is None else u8(mask_has)
    out_v = np.empty(n, dtype=np.float64)
    out_h = np.empty(n, dtype=np.uint8)
    rc = _load().oracle_mxv(rows._h, MXV_SEMIRINGS[semiring], 1 if vec_first else 0, _ptr(uv),
                            _ptr(uh), _ptr(wv), _ptr(wh), _ptr(mv), _ptr(mh), int(flags),
                            MXV_ACCUMS[accum], _ptr(out_v), _ptr(out_h))
    if rc != 0:
        raise ValueError("oracle_mxv: bad input")
    return out_v, out_h.astype(bool)
