"""Pins for the BFS oracle (Algorithm 1; levels = the paper's d minus one).

Checked against things the oracle does not compute itself: boolean matrix
powers, scipy's hop-count shortest paths and connected components, closed
forms on paths, stars, cliques and grids, and the min-id parent rule
verified directly.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen
import oracle


def _dense(n, src, dst, symmetric=True):
    A = np.zeros((n, n), dtype=bool)
    for u, v in zip(src, dst):
        if u != v:
            A[u, v] = True
            if symmetric:
                A[v, u] = True
    return A


def _brute_levels(A, s):
    # level(v) = min{k : (A^k)(s, v) != 0}, by boolean matrix powers
    n = A.shape[0]
    lev = np.full(n, -1, dtype=np.int32)
    reach = np.zeros(n, dtype=bool)
    reach[s] = True
    lev[s] = 0
    cur = reach.copy()
    for k in range(1, n + 1):
        cur = (cur.astype(np.int64) @ A.astype(np.int64)) > 0  # row s of A^k
        new = cur & (lev < 0)
        lev[new] = k
        if not cur.any():
            break
    return lev


def _brute_parents(A, lev, s):
    n = A.shape[0]
    par = np.full(n, -1, dtype=np.int32)
    par[s] = s
    for v in range(n):
        if v == s or lev[v] < 0:
            continue
        cands = [u for u in range(n) if A[u, v] and lev[u] == lev[v] - 1]
        par[v] = min(cands)
    return par


@pytest.mark.parametrize("seed", range(12))
def test_bfs_matches_matrix_powers_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    m = int(rng.integers(0, 3 * n))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    symmetric = bool(seed % 3)
    A = _dense(n, src, dst, symmetric)
    adj = oracle.Adjacency(n, src, dst, symmetrise=symmetric)
    for s in range(0, n, max(1, n // 5)):
        lev, par, nl = oracle.bfs(adj, s)
        ref = _brute_levels(A, s)
        assert np.array_equal(lev, ref)
        assert np.array_equal(par, _brute_parents(A, ref, s))
        assert nl == ref.max() + 1


def test_bfs_closed_forms():
    # path 0-1-...-9
    k = 10
    adj = oracle.Adjacency(k, np.arange(k - 1), np.arange(1, k))
    lev, par, nl = oracle.bfs(adj, 0)
    assert np.array_equal(lev, np.arange(k)) and nl == k
    assert np.array_equal(par, np.concatenate([[0], np.arange(k - 1)]))
    # star with centre 0 and 7 leaves, from leaf 3
    adj = oracle.Adjacency(8, np.zeros(7, np.int32), np.arange(1, 8))
    lev, par, _ = oracle.bfs(adj, 3)
    assert lev.tolist() == [1, 2, 2, 0, 2, 2, 2, 2]
    assert par.tolist() == [3, 0, 0, 3, 0, 0, 0, 0]
    # clique of 6 from 4
    iu = np.triu_indices(6, 1)
    adj = oracle.Adjacency(6, iu[0], iu[1])
    lev, par, _ = oracle.bfs(adj, 4)
    assert lev.tolist() == [1, 1, 1, 1, 0, 1] and par.tolist() == [4] * 6
    # 5x5 grid from the corner: level r + c; parent = upper neighbour
    # (smaller id) when r > 0, else the left neighbour
    s_, d_ = graphgen.grid_edges(5, 5)
    adj = oracle.Adjacency(25, s_, d_)
    lev, par, _ = oracle.bfs(adj, 0)
    r, c = np.divmod(np.arange(25), 5)
    assert np.array_equal(lev, r + c)
    exp = np.where(r > 0, (r - 1) * 5 + c, r * 5 + c - 1)
    exp[0] = 0
    assert np.array_equal(par, exp)


def test_bfs_isolated_and_single_vertex():
    adj = oracle.Adjacency(1, np.zeros(0, np.int32), np.zeros(0, np.int32))
    lev, par, nl = oracle.bfs(adj, 0)
    assert lev.tolist() == [0] and par.tolist() == [0] and nl == 1
    # two components, self-loop and duplicates dropped
    adj = oracle.Adjacency(6, [0, 1, 1, 3, 4, 2], [1, 2, 2, 4, 4, 2])
    assert adj.nnz == 6
    lev, par, _ = oracle.bfs(adj, 3)
    assert lev.tolist() == [-1, -1, -1, 0, 1, -1]
    assert par.tolist() == [-1, -1, -1, 3, 3, -1]


def test_bfs_rmat_invariants_and_scipy():
    g = graphgen.rmat(12, weights=False)
    adj = oracle.Adjacency.from_raw(g)
    off, nbr, _ = adj.arrays(weights=False)
    rows = np.repeat(np.arange(g.n), np.diff(off))
    A = sp.csr_matrix((np.ones(adj.nnz), (rows, nbr)), shape=(g.n, g.n))
    lev, par, nl = oracle.bfs(adj, 0)
    # hop distances from scipy
    hops = csg.shortest_path(A, unweighted=True, indices=0)
    ref = np.where(np.isinf(hops), -1, hops).astype(np.int32)
    assert np.array_equal(lev, ref)
    # reached set = connected component of the source
    _, comp = csg.connected_components(A, directed=False)
    assert np.array_equal(lev >= 0, comp == comp[0])
    # |level(u) - level(v)| <= 1 on every edge with both ends reached
    both = (lev[rows] >= 0) & (lev[nbr] >= 0)
    assert np.all(np.abs(lev[rows][both] - lev[nbr][both]) <= 1)
    # parent rule: a neighbour one level up, and no smaller such neighbour
    reached = np.flatnonzero((lev > 0))
    for v in reached[:: max(1, len(reached) // 300)]:
        nb = nbr[off[v]:off[v + 1]]
        up = nb[lev[nb] == lev[v] - 1]
        assert par[v] == up.min()
    assert nl == lev.max() + 1


def test_adjacency_cleaning():
    adj = oracle.Adjacency(4, [0, 0, 1, 2, 3, 3], [1, 1, 0, 2, 0, 1],
                           w=[5, 3, 9, 1, 2, 2], symmetrise=True)
    off, nbr, w = adj.arrays()
    assert off.tolist() == [0, 2, 4, 4, 6]
    assert nbr.tolist() == [1, 3, 0, 3, 0, 1]
    # duplicates of (0,1) carry 5, 3, 9: the smallest survives
    assert w.tolist() == [3, 2, 3, 2, 2, 2]
    d = oracle.Adjacency(4, [0, 0, 1], [1, 1, 0], symmetrise=False)
    off, nbr, _ = d.arrays(weights=False)
    assert off.tolist() == [0, 1, 2, 2, 2] and nbr.tolist() == [1, 0]
    t = d.transpose()
    off, nbr, _ = t.arrays(weights=False)
    assert off.tolist() == [0, 1, 2, 2, 2] and nbr.tolist() == [1, 0]


@pytest.mark.parametrize("nthreads", [1, 8])
def test_msbfs_equals_stacked_single_source_runs(nthreads):
    """oracle.msbfs (k runs on a thread pool, query-major output) equals k
    separate oracle.bfs runs stacked row by row: random, repeated and
    isolated sources, k not a multiple of the thread count, a directed and
    an undirected graph.  A wrong row offset, a lost or doubled query, or a
    race on the shared work counter changes some row."""
    for g in (graphgen.rmat(11), graphgen.rmat(10, symmetric=False)):
        adj = oracle.Adjacency.from_raw(g)
        deg = np.diff(adj.arrays(weights=False)[0])
        rng = np.random.default_rng(7 + nthreads)
        k = 77
        src = rng.integers(0, g.n, k).astype(np.int32)
        src[5] = src[4]                              # repeated source
        src[9] = int(np.flatnonzero(deg == 0)[0])    # isolated source
        src[10] = 0                                  # the hub
        got = oracle.msbfs(adj, src, nthreads=nthreads)
        assert got.shape == (k, g.n)
        for q, s in enumerate(src):
            ref, _, _ = oracle.bfs(adj, int(s), parents=False)
            assert np.array_equal(got[q], ref), (q, int(s))
        # an independent check of a few rows: scipy hop counts
        off, nbr, _ = adj.arrays(weights=False)
        S = sp.csr_matrix((np.ones(nbr.size), nbr, off), shape=(g.n, g.n))
        hops = csg.shortest_path(S, unweighted=True, indices=src[:6])
        for q in range(6):
            want = np.where(np.isinf(hops[q]), -1, hops[q]).astype(np.int32)
            assert np.array_equal(got[q], want), q


def test_msbfs_rejects_bad_source():
    adj = oracle.Adjacency(4, np.array([0, 1]), np.array([1, 2]))
    with pytest.raises(ValueError):
        oracle.msbfs(adj, np.array([0, 4], np.int32))
