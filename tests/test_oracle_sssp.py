"""Pins for the SSSP oracle (the fixed point of the Bellman-Ford variant of
Section 7.2 is the exact shortest-path distance vector).

Checked against scipy's Dijkstra, a Floyd-Warshall recurrence, an optimality
certificate (triangle inequality plus a tight-edge tree back to the source),
and the unit-weight reduction to BFS levels.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen
import oracle


def _csr(adj):
    off, nbr, w = adj.arrays()
    rows = np.repeat(np.arange(adj.n), np.diff(off))
    return off, nbr, w, rows


def _floyd_warshall(n, rows, nbr, w):
    D = np.full((n, n), np.inf)
    np.fill_diagonal(D, 0.0)
    for r, c, x in zip(rows, nbr, w):
        D[r, c] = min(D[r, c], x)
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


@pytest.mark.parametrize("seed", range(8))
def test_sssp_floyd_warshall_small(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 60))
    m = int(rng.integers(0, 4 * n))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    w = rng.integers(1, 65, m).astype(np.float32)
    symmetric = bool(seed % 2)
    adj = oracle.Adjacency(n, src, dst, w, symmetrise=symmetric)
    _, nbr, ww, rows = _csr(adj)
    D = _floyd_warshall(n, rows, nbr, ww)
    for s in range(0, n, max(1, n // 4)):
        d32, d64, reached = oracle.sssp(adj, s)
        assert np.array_equal(d64, D[s])
        assert np.array_equal(d32, D[s].astype(np.float32))
        assert reached == int(np.isfinite(D[s]).sum())


def _certificate(adj, s, d):
    off, nbr, w, rows = _csr(adj)
    assert d[s] == 0
    du, dv = d[rows], d[nbr]
    fin = np.isfinite(du)
    # no edge can improve a distance
    assert np.all(dv[fin] <= du[fin] + w[fin])
    # every reached vertex other than s has a tight in-edge, and the tight
    # edges chosen (smallest tail) lead back to s (weights >= 1: no cycles)
    tight = fin & (dv == du + w)
    par = np.full(adj.n, -1)
    order = np.argsort(-rows[tight], kind="stable")
    par[nbr[tight][order]] = rows[tight][order]
    reached = np.flatnonzero(np.isfinite(d))
    for v in reached:
        if v != s:
            assert par[v] >= 0
    for v in reached[:: max(1, len(reached) // 200)]:
        steps = 0
        while v != s:
            v = par[v]
            steps += 1
            assert steps <= adj.n


def test_sssp_certificate_and_scipy_rmat():
    g = graphgen.rmat(12)
    adj = oracle.Adjacency.from_raw(g)
    d32, d64, _ = oracle.sssp(adj, 0)
    _certificate(adj, 0, d64)
    off, nbr, w, rows = _csr(adj)
    A = sp.csr_matrix((w, (rows, nbr)), shape=(g.n, g.n))
    ref = csg.dijkstra(A, indices=0)
    assert np.array_equal(d64, ref)
    assert np.array_equal(d32, ref.astype(np.float32))


def test_sssp_certificate_grid():
    g = graphgen.grid(40, 40)
    adj = oracle.Adjacency.from_raw(g)
    _, d64, reached = oracle.sssp(adj, 0)
    assert reached == 1600
    _certificate(adj, 0, d64)


def test_sssp_unit_weights_equal_bfs_levels():
    g = graphgen.rmat(11, weights=False)
    w = np.ones(g.src.shape[0], dtype=np.float32)
    adj = oracle.Adjacency(g.n, g.src, g.dst, w)
    d32, _, _ = oracle.sssp(adj, 5)
    lev, _, _ = oracle.bfs(adj, 5, parents=False)
    assert np.array_equal(np.where(np.isinf(d32), -1, d32).astype(np.int32), lev)


def test_sssp_unreached_is_inf():
    adj = oracle.Adjacency(4, [0, 2], [1, 3], w=[7.0, 3.0])
    d32, _, r = oracle.sssp(adj, 0)
    assert d32.tolist()[:2] == [0.0, 7.0] and np.isinf(d32[2]) and np.isinf(d32[3])
    assert r == 2
