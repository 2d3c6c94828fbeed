"""ORACLE — TEST INFRASTRUCTURE ONLY.

Masked sparse matrix-matrix product in the dot-product form of the paper's
masked SpGEMM (Section 6.3.4) and the triangle-counting operand of Section
7.4, written from their definitions with scipy / numpy as plain steps:

* :func:`mxm_masked` — for every entry (i, j) of the mask M, the sum over
  k of A(i, k) * B(j, k) (PLUS_TIMES) or the number of common k (PLUS_PAIR):
  the full product A B^T by a library sparse matmul, then read at M's
  entries (0 where the rows share no index).
* :func:`lower_by_degree` — vertices renumbered by decreasing degree (ties
  by increasing id), the strict lower triangle of the symmetric adjacency.
* :func:`edge_counts` — for sampled entries (i, j) of such an L, the size of
  the intersection of rows i and j (one entry at a time, for graphs too
  large for the full product).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the GPU library.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _csr(n_rows, n_cols, rp, ci, vals=None):
    rp = np.asarray(rp, dtype=np.int64)
    ci = np.asarray(ci, dtype=np.int64)
    data = np.ones(ci.shape[0]) if vals is None else np.asarray(vals, dtype=np.float64)
    return sp.csr_matrix((data, ci, rp), shape=(n_rows, n_cols))


def mxm_masked(M, A, B, semiring: str):
    """M, A, B: (n_rows, n_cols, row_ptr, col_idx, values or None) tuples.
    Returns one float64 value per entry of M, in M's CSR order."""
    pair = semiring == "plus_pair_int32"
    Am = _csr(*A[:4], None if pair else A[4])
    Bm = _csr(*B[:4], None if pair else B[4])
    prod = (Am @ Bm.T).tocsr()
    n_rows, _, mrp, mci = M[:4]
    mrp = np.asarray(mrp, dtype=np.int64)
    rows = np.repeat(np.arange(n_rows), np.diff(mrp))
    if rows.shape[0] == 0:
        return np.zeros(0, dtype=np.float64)
    return np.asarray(prod[rows, np.asarray(mci, dtype=np.int64)]).ravel().astype(np.float64)


def mxm_abs_bound(M, A, B):
    """Per mask entry: (number of common indices, sum of |A(i,k) B(j,k)|),
    the two quantities of the floating-point error bound of a sum."""
    Ap = _csr(*A[:4], None)
    Bp = _csr(*B[:4], None)
    Aa = _csr(*A[:4], np.abs(np.asarray(A[4], dtype=np.float64)))
    Ba = _csr(*B[:4], np.abs(np.asarray(B[4], dtype=np.float64)))
    n_rows, _, mrp, mci = M[:4]
    mrp = np.asarray(mrp, dtype=np.int64)
    rows = np.repeat(np.arange(n_rows), np.diff(mrp))
    cols = np.asarray(mci, dtype=np.int64)
    if rows.shape[0] == 0:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.float64)
    cnt = np.asarray((Ap @ Bp.T).tocsr()[rows, cols]).ravel()
    mag = np.asarray((Aa @ Ba.T).tocsr()[rows, cols]).ravel()
    return cnt, mag


def lower_by_degree(n: int, off, nbr):
    """(row_ptr, col_idx, rank) of the strict lower triangle after
    renumbering by decreasing degree, ties by increasing id; off / nbr are
    a symmetric adjacency (numpy arrays)."""
    off = np.asarray(off, dtype=np.int64)
    nbr = np.asarray(nbr, dtype=np.int64)
    deg = np.diff(off)
    order = np.lexsort((np.arange(n), -deg))  # last key primary: degree desc
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)
    src = np.repeat(np.arange(n), deg)
    keep = rank[nbr] < rank[src]
    r, c = rank[src[keep]], rank[nbr[keep]]
    L = sp.csr_matrix((np.ones(r.shape[0]), (r, c)), shape=(n, n))
    L.sort_indices()
    return L.indptr.astype(np.int64), L.indices.astype(np.int64), rank


def edge_counts(rp, ci, entries):
    """|row i of L  intersect  row j of L| for each mask entry index e of L
    (i = the row holding entry e, j = ci[e])."""
    rp = np.asarray(rp, dtype=np.int64)
    ci = np.asarray(ci, dtype=np.int64)
    out = []
    for e in entries:
        i = int(np.searchsorted(rp, e, side="right") - 1)
        j = int(ci[e])
        out.append(np.intersect1d(ci[rp[i]:rp[i + 1]], ci[rp[j]:rp[j + 1]],
                                  assume_unique=True).shape[0])
    return np.asarray(out, dtype=np.int64)
