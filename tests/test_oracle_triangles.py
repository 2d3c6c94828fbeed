"""Pins for the triangle-counting and masked-SpGEMM oracles (Sections 6.3.4
and 7.5).

The triangle count is checked against trace(A^3) / 6 and the per-vertex
counts against diag(A^3) / 2 (dense matrix powers), and against closed
forms: cliques C(n, 3), wheels, grids and bipartite graphs 0.  The masked
product is checked against a dense product read at the mask's entries, and
the degree-ordered lower triangle against its defining properties; the sum
of (L L^T) .* L over that L must equal the triangle count.
"""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import mxm as omxm


def _dense(n, src, dst):
    A = np.zeros((n, n), dtype=np.int64)
    for u, v in zip(src, dst):
        if u != v:
            A[u, v] = A[v, u] = 1
    return A


def _random(seed, n_max=40):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(1, n_max))
    m = int(rng.integers(0, 4 * n))
    return n, rng.integers(0, n, m).astype(np.int32), rng.integers(0, n, m).astype(np.int32)


@pytest.mark.parametrize("seed", range(12))
def test_triangles_match_matrix_powers(seed):
    n, src, dst = _random(seed)
    A = _dense(n, src, dst)
    A3 = A @ A @ A
    t, pv = oracle.triangles(oracle.Adjacency(n, src, dst, symmetrise=True))
    assert t == np.trace(A3) // 6
    assert np.array_equal(pv, np.diag(A3) // 2)


def test_triangles_closed_forms():
    for k in (3, 4, 7, 30):
        iu = np.triu_indices(k, 1)
        t, pv = oracle.triangles(oracle.Adjacency(k, iu[0], iu[1]))
        assert t == k * (k - 1) * (k - 2) // 6
        assert np.all(pv == (k - 1) * (k - 2) // 2)
    for k in (4, 5, 9):  # wheel: hub 0 joined to a k-cycle 1..k
        cyc = np.arange(1, k + 1)
        src = np.concatenate([np.zeros(k, np.int32), cyc])
        dst = np.concatenate([cyc, np.roll(cyc, -1)])
        t, pv = oracle.triangles(oracle.Adjacency(k + 1, src, dst))
        assert t == k and pv[0] == k and np.all(pv[1:] == 2)
    g = graphgen.grid(7, 9, weights=False)
    assert oracle.triangles(oracle.Adjacency.from_raw(g))[0] == 0
    a, b = np.meshgrid(np.arange(5), np.arange(5, 12))
    assert oracle.triangles(oracle.Adjacency(12, a.ravel(), b.ravel()))[0] == 0
    assert oracle.triangles(oracle.Adjacency(6, [], []))[0] == 0
    assert oracle.triangles(oracle.Adjacency(0, [], []))[0] == 0


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("semiring", ["plus_pair_int32", "plus_times_fp64"])
def test_mxm_masked_matches_dense(seed, semiring):
    rng = np.random.default_rng(500 + seed)
    r, kd, c = (int(x) for x in rng.integers(1, 30, 3))

    def rand_csr(nr, nc, dens):
        D = (rng.random((nr, nc)) < dens) * rng.integers(1, 9, (nr, nc)).astype(np.float64)
        rp = np.concatenate([[0], np.cumsum((D != 0).sum(1))])
        ci = np.nonzero(D)[1]
        return (nr, nc, rp, ci, D[D != 0]), D

    A, Ad = rand_csr(r, kd, 0.3)
    B, Bd = rand_csr(c, kd, 0.3)
    M, Md = rand_csr(r, c, 0.4)
    got = omxm.mxm_masked(M, A, B, semiring)
    Pa, Pb = (Ad, Bd) if semiring != "plus_pair_int32" else ((Ad != 0) * 1.0, (Bd != 0) * 1.0)
    full = Pa @ Pb.T
    mi, mj = np.nonzero(Md)
    assert np.array_equal(got, full[mi, mj])
    cnt, mag = omxm.mxm_abs_bound(M, A, B)
    assert np.array_equal(cnt, ((Ad != 0).astype(int) @ (Bd != 0).astype(int).T)[mi, mj])
    assert np.allclose(mag, (np.abs(Ad) @ np.abs(Bd).T)[mi, mj])


@pytest.mark.parametrize("scale", [8, 10, 12])
def test_lower_by_degree_and_tricount_identity(scale):
    g = graphgen.rmat(scale, weights=False)
    adj = oracle.Adjacency.from_raw(g)
    off, nbr, _ = adj.arrays(weights=False)
    n = adj.n
    rp, ci, rank = omxm.lower_by_degree(n, off, nbr)
    deg = np.diff(off)
    # rank: a permutation ordered by degree (desc), ties by id (asc)
    assert np.array_equal(np.sort(rank), np.arange(n))
    inv = np.empty(n, np.int64)
    inv[rank] = np.arange(n)
    d = deg[inv]
    assert np.all(d[:-1] >= d[1:])
    tie = d[:-1] == d[1:]
    assert np.all(inv[:-1][tie] < inv[1:][tie])
    # L: strict lower, sorted rows, each undirected edge once, short rows
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(ci < rows)
    assert all(np.all(np.diff(ci[rp[i]:rp[i + 1]]) > 0) for i in range(n))
    assert ci.shape[0] * 2 == adj.nnz
    assert np.diff(rp).max() <= np.sqrt(adj.nnz) + 1
    # sum of (L L^T) .* L = number of triangles; per-entry sampled counts agree
    L = (n, n, rp, ci, None)
    c = omxm.mxm_masked(L, L, L, "plus_pair_int32")
    t, _ = oracle.triangles(adj)
    assert int(c.sum()) == t
    ent = np.arange(0, ci.shape[0], max(1, ci.shape[0] // 300))
    assert np.array_equal(omxm.edge_counts(rp, ci, ent), c[ent].astype(np.int64))


def test_mxm_masked_empty_mask():
    A = (3, 4, np.array([0, 1, 1, 2]), np.array([0, 3]), np.array([1.0, 2.0]))
    M = (3, 3, np.zeros(4, np.int64), np.zeros(0, np.int64), None)
    assert omxm.mxm_masked(M, A, A, "plus_times_fp64").shape == (0,)
    cnt, mag = omxm.mxm_abs_bound(M, A, A)
    assert cnt.shape == (0,) and mag.shape == (0,)
