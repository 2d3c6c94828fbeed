"""Pins for the PageRank oracle (Section 7.3, pull form; damping 0.85,
dangling mass spread uniformly, L1 stopping rule).

Checked against the exact fixed point from a dense linear solve, closed
forms (cycles, regular graphs and edgeless graphs give the uniform vector)
and invariants (sum 1, positivity, geometric convergence).
"""
import numpy as np
import pytest

import graphgen
import oracle


def _exact(n, src, dst, alpha):
    # column-stochastic M with dangling columns spread uniformly; solve
    # (I - alpha M) p = (1 - alpha)/n * 1
    A = np.zeros((n, n))
    for u, v in zip(src, dst):
        if u != v:
            A[u, v] = 1.0
    out = A.sum(1)
    M = np.zeros((n, n))
    for u in range(n):
        if out[u] > 0:
            M[:, u] = A[u] / out[u]
        else:
            M[:, u] = 1.0 / n
    return np.linalg.solve(np.eye(n) - alpha * M, np.full(n, (1 - alpha) / n))


@pytest.mark.parametrize("seed", range(8))
def test_pagerank_fixed_point(seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(2, 50))
    m = int(rng.integers(0, 4 * n))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    adj = oracle.Adjacency(n, src, dst, symmetrise=False)
    p, it, delta = oracle.pagerank(adj, 0.85, max_iter=400, tol=0.0)
    assert it == 400
    assert np.allclose(p, _exact(n, src, dst, 0.85), atol=1e-13, rtol=0)
    assert abs(p.sum() - 1) < 1e-12 and np.all(p > 0)


def test_pagerank_closed_forms():
    n = 7
    cyc = oracle.Adjacency(n, np.arange(n), (np.arange(n) + 1) % n, symmetrise=False)
    p, it, delta = oracle.pagerank(cyc, 0.85, 50, 1e-7)
    assert np.allclose(p, 1 / n, atol=1e-15) and it == 1 and delta == 0.0
    empty = oracle.Adjacency(5, np.zeros(0, np.int32), np.zeros(0, np.int32), symmetrise=False)
    p, it, _ = oracle.pagerank(empty, 0.85, 50, 1e-7)
    assert np.allclose(p, 0.2, atol=1e-15) and it == 1
    # a regular graph (a clique) also gives the uniform vector
    iu = np.triu_indices(6, 1)
    clique = oracle.Adjacency(6, iu[0], iu[1], symmetrise=True)
    p, _, _ = oracle.pagerank(clique, 0.85, 50, 1e-7)
    assert np.allclose(p, 1 / 6, atol=1e-15)


def test_pagerank_rmat_directed_invariants():
    g = graphgen.rmat(12, symmetric=False, weights=False)
    adj = oracle.Adjacency.from_raw(g)
    p, it, delta = oracle.pagerank(adj, 0.85, 50, 1e-7)
    assert 1 < it < 50 and delta < 1e-7
    assert abs(p.sum() - 1) < 1e-12 and np.all(p > 0)
    # the update is an L1 contraction with factor alpha, so each change is at
    # most alpha times the previous one; and the stop is the first iteration
    # whose change falls below the tolerance
    _, _, prev = oracle.pagerank(adj, 0.85, it - 1, 0.0)
    assert prev >= 1e-7
    assert delta <= 0.85 * prev * (1 + 1e-9)
