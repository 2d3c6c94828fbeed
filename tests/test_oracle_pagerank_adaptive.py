"""Pins for the adaptive PageRank oracle (PageRankDelta: PageRank whose mask
holds the converged vertices, Sections 5.1 and 7.3; a vertex freezes once
its change relative to the previous iterate is at most eps).

The oracle's trajectory is checked against the definition from outside:
the update of every still-active vertex is recomputed from the previous
iterate with a dense column-stochastic matrix (dangling columns spread
uniformly, frozen values included); the freeze rule is checked at the
iteration each vertex froze and for every vertex still active; frozen
values never change and the frozen set only grows; with eps = 0 nothing
freezes and the iterates are the dense power iteration's; closed forms
freeze everything at once; a tiny eps reaches the exact fixed point.
"""
import numpy as np
import pytest

import graphgen
import oracle

ALPHA = 0.85


def _dense_m(n, src, dst):
    A = np.zeros((n, n))
    for u, v in zip(src, dst):
        if u != v:
            A[u, v] = 1.0
    out = A.sum(1)
    M = np.zeros((n, n))
    for u in range(n):
        M[:, u] = A[u] / out[u] if out[u] > 0 else 1.0 / n
    return M


def _random(seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(3, 60))
    m = int(rng.integers(0, 4 * n))
    return n, rng.integers(0, n, m).astype(np.int32), rng.integers(0, n, m).astype(np.int32)


def _traj(adj, eps, k):
    """iterates p_0 .. p_k of the adaptive run (p_j = the run stopped after j
    iterations) and the full-run freeze iterations."""
    ps = [np.full(adj.n, 1.0 / adj.n)]
    for j in range(1, k + 1):
        p, it, _, _, _ = oracle.pagerank_adaptive(adj, eps, ALPHA, max_iter=j, tol=0.0)
        ps.append(p)
    return ps


@pytest.mark.parametrize("seed", range(6))
def test_eps_zero_is_power_iteration(seed):
    n, src, dst = _random(seed)
    adj = oracle.Adjacency(n, src, dst, symmetrise=False)
    M = _dense_m(n, src, dst)
    p, it, _, active, fz = oracle.pagerank_adaptive(adj, 0.0, ALPHA, max_iter=6, tol=0.0)
    q = np.full(n, 1.0 / n)
    for _ in range(it):
        q = (1 - ALPHA) / n + ALPHA * (M @ q)
    if np.all(fz == 0):
        assert it == 6 and active == n
        assert np.allclose(p, q, atol=1e-15, rtol=1e-13)
    else:  # only a vertex whose value stopped moving exactly may freeze at eps = 0
        assert np.allclose(p, q, atol=1e-15, rtol=1e-12)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("eps", [1e-1, 1e-2, 1e-3])
def test_trajectory_follows_definition(seed, eps):
    n, src, dst = _random(seed)
    adj = oracle.Adjacency(n, src, dst, symmetrise=False)
    M = _dense_m(n, src, dst)
    full, it, _, active, fz = oracle.pagerank_adaptive(adj, eps, ALPHA, max_iter=40, tol=0.0)
    ps = _traj(adj, eps, it)
    for j in range(1, it + 1):
        prev, cur = ps[j - 1], ps[j]
        frozen_before = (fz > 0) & (fz < j)
        live = ~frozen_before
        # frozen values stay; live ones take the update from the previous
        # iterate (frozen neighbours and frozen dangling mass included)
        assert np.array_equal(cur[frozen_before], prev[frozen_before])
        upd = (1 - ALPHA) / n + ALPHA * (M @ prev)
        assert np.allclose(cur[live], upd[live], atol=1e-15, rtol=1e-12)
        # freeze rule: exactly the live vertices whose change is within eps
        ch = np.abs(cur - prev)
        now = fz == j
        assert np.all(ch[now] <= eps * prev[now] * (1 + 1e-12))
        still = live & ~now
        assert np.all(ch[still] > eps * prev[still] * (1 - 1e-12))
        # the frozen set of a shorter run is a prefix of the full run's
        _, _, _, act_j, fz_j = oracle.pagerank_adaptive(adj, eps, ALPHA, max_iter=j, tol=0.0)
        assert np.array_equal(fz_j, np.where(fz <= j, fz, 0))
        assert act_j == int(np.sum((fz == 0) | (fz > j)))
    assert np.array_equal(full, ps[it])
    assert active == int(np.sum(fz == 0))
    assert active == 0 or it == 40


def test_closed_forms_freeze_at_once():
    n = 7
    cyc = oracle.Adjacency(n, np.arange(n), (np.arange(n) + 1) % n, symmetrise=False)
    empty = oracle.Adjacency(5, np.zeros(0, np.int32), np.zeros(0, np.int32), symmetrise=False)
    iu = np.triu_indices(6, 1)
    clique = oracle.Adjacency(6, iu[0], iu[1], symmetrise=True)
    for adj in (cyc, empty, clique):
        # the change is zero (up to rounding) at the first iteration, so even
        # eps = 0 freezes every vertex when the change is exactly zero
        for eps in (1e-9, 0.0):
            p, it, delta, active, fz = oracle.pagerank_adaptive(adj, eps, ALPHA, 50, 0.0)
            if eps == 0.0 and adj is clique:
                continue  # 1/6 is not exact in binary: rounding may move it
            assert it == 1 and active == 0 and np.all(fz == 1)
            assert np.allclose(p, 1 / adj.n, atol=1e-15) and delta < 1e-15


@pytest.mark.parametrize("seed", range(4))
def test_tiny_eps_reaches_fixed_point(seed):
    n, src, dst = _random(seed)
    adj = oracle.Adjacency(n, src, dst, symmetrise=False)
    M = _dense_m(n, src, dst)
    exact = np.linalg.solve(np.eye(n) - ALPHA * M, np.full(n, (1 - ALPHA) / n))
    p, it, _, _, _ = oracle.pagerank_adaptive(adj, 1e-12, ALPHA, max_iter=400, tol=0.0)
    assert np.abs(p - exact).sum() < 1e-9


def test_rmat_directed_shrinks_and_approximates():
    g = graphgen.rmat(11, symmetric=False, weights=False)
    adj = oracle.Adjacency.from_raw(g)
    ref, _, _ = oracle.pagerank(adj, ALPHA, 200, 0.0)
    errs = []
    for eps in (1e-2, 1e-3, 1e-4):
        p, it, _, active, fz = oracle.pagerank_adaptive(adj, eps, ALPHA, 100, 0.0)
        assert active == 0 and it < 100  # every vertex freezes
        # vertices freeze over several iterations, not all at once
        assert len(np.unique(fz)) > 3
        errs.append(np.abs(p - ref).sum())
    # a smaller threshold gives a closer result
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-3


def test_bad_input():
    adj = oracle.Adjacency(3, [0], [1], symmetrise=False)
    with pytest.raises(ValueError):
        oracle.pagerank_adaptive(adj, -1.0)
    with pytest.raises(ValueError):
        oracle.pagerank_adaptive(adj, float("nan"))
