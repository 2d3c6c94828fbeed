"""Pins for the connected-components oracle (Section 7.4: components of an
undirected graph, each vertex labelled with its component).  The oracle's
label is the smallest vertex id of the component, the fixed point of the
min-label hooking and shortcutting iteration.

Checked against reachability by boolean matrix powers on tiny random
graphs, against scipy's connected_components (same partition, same count)
on R-MAT and random graphs, closed forms (path, edgeless, star, two
interleaved cliques) and invariants (a label is a vertex of the component
and its own label, no larger than the vertex, shared along every edge)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import graphgen
import oracle


def _adj(n, src, dst):
    return oracle.Adjacency(n, np.asarray(src, np.int32), np.asarray(dst, np.int32),
                            symmetrise=True)


def _random(seed, n_max=30):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(1, n_max))
    m = int(rng.integers(0, 2 * n))
    return n, rng.integers(0, n, m), rng.integers(0, n, m)


@pytest.mark.parametrize("seed", range(15))
def test_cc_matches_reachability(seed):
    n, src, dst = _random(seed)
    R = np.eye(n, dtype=bool)
    for u, v in zip(src, dst):
        R[u, v] = R[v, u] = True
    for _ in range(int(np.ceil(np.log2(max(n, 2)))) + 1):  # closure by squaring
        R = (R.astype(np.int64) @ R.astype(np.int64)) > 0
    want = np.array([np.flatnonzero(R[v])[0] for v in range(n)], dtype=np.int32)
    lab, c = oracle.cc(_adj(n, src, dst))
    assert np.array_equal(lab, want)
    assert c == len(set(want.tolist()))


@pytest.mark.parametrize("kind", ["rmat12", "rmat_dir_sym", "sparse_random"])
def test_cc_matches_scipy(kind):
    if kind == "rmat12":
        g = graphgen.rmat(12)
        src, dst, n = g.src, g.dst, g.n
    elif kind == "rmat_dir_sym":
        g = graphgen.rmat(11, symmetric=False)
        src, dst, n = g.src, g.dst, g.n
    else:
        rng = np.random.default_rng(9)
        n = 5000
        src, dst = rng.integers(0, n, 3000), rng.integers(0, n, 3000)
    lab, c = oracle.cc(_adj(n, src, dst))
    M = sp.coo_matrix((np.ones(len(src)), (np.asarray(src), np.asarray(dst))), shape=(n, n))
    nc, comp = connected_components(M, directed=True, connection="weak")
    assert c == nc
    # same partition: label -> scipy component is a bijection
    pairs = set(zip(lab.tolist(), comp.tolist()))
    assert len(pairs) == nc == len({a for a, _ in pairs}) == len({b for _, b in pairs})


def test_cc_closed_forms():
    lab, c = oracle.cc(_adj(7, range(6), range(1, 7)))  # path
    assert c == 1 and lab.tolist() == [0] * 7
    lab, c = oracle.cc(_adj(5, [], []))  # edgeless: every vertex alone
    assert c == 5 and lab.tolist() == list(range(5))
    lab, c = oracle.cc(_adj(6, [3, 3, 3, 3, 3], [0, 1, 2, 4, 5]))  # star
    assert c == 1 and lab.tolist() == [0] * 6
    # two cliques on interleaved ids (evens, odds) plus an isolated vertex 10
    ev = [(a, b) for a in range(0, 10, 2) for b in range(a + 2, 10, 2)]
    od = [(a, b) for a in range(1, 10, 2) for b in range(a + 2, 10, 2)]
    e = ev + od
    lab, c = oracle.cc(_adj(11, [x for x, _ in e], [y for _, y in e]))
    assert c == 3 and lab.tolist() == [0, 1] * 5 + [10]


@pytest.mark.parametrize("seed", range(5))
def test_cc_invariants(seed):
    g = graphgen.rmat(10 + seed % 3, seed=seed + 1)
    adj = oracle.Adjacency.from_raw(g)
    lab, c = oracle.cc(adj)
    off, nbr, _ = adj.arrays(weights=False)
    v = np.arange(g.n)
    assert np.all(lab <= v)
    assert np.array_equal(lab[lab], lab)
    src = np.repeat(v, np.diff(off))
    assert np.array_equal(lab[src], lab[nbr])
    assert c == int((lab == v).sum())
