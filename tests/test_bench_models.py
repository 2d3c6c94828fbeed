"""Byte models of bench.py (host-side arithmetic, no GPU): the early-exit
scan length against brute force, and the BFS byte model on a path graph
where every term can be counted by hand."""
import numpy as np

import bench
import graphgen
import oracle


def brute_first_hit(rp, ci, rows_mask, hit_col):
    total = 0
    for r in np.flatnonzero(rows_mask):
        nb = ci[rp[r]:rp[r + 1]]
        if nb.size == 0:
            continue
        hits = np.flatnonzero(hit_col[nb])
        total += int(hits[0]) + 1 if hits.size else int(nb.size)
    return total


def csr_of(raw):
    adj = oracle.Adjacency.from_raw(raw)
    rp, ci = adj.arrays()[:2]
    return np.asarray(rp, dtype=np.int64), np.asarray(ci, dtype=np.int64)


def test_first_hit_scan_matches_brute_force():
    g = graphgen.rmat(9)
    rp, ci = csr_of(g)
    rng = np.random.default_rng(5)
    for _ in range(5):
        rows = rng.random(g.n) < 0.4
        hit = rng.random(g.n) < 0.1
        assert bench.first_hit_scan(rp, ci, rows, hit) == brute_first_hit(rp, ci, rows, hit)


def test_path_graph_byte_model():
    # path 0-1-2-3: levels 0,1,2,3 from vertex 0, every level a push
    n = 4
    raw = graphgen.from_edges("path4", n, np.array([0, 1, 2]), np.array([1, 2, 3]))
    rp, ci = csr_of(raw)
    lev = np.array([0, 1, 2, 3])
    dirs = [1, 1, 1, 1]
    per = bench.bfs_bytes_per_level(rp, ci, lev, dirs, n)
    deg = np.diff(rp)
    for d in range(4):
        nxt = 1 if d < 3 else 0
        assert per[d] == 12 * 1 + 4 * deg[d] + n / 8 + n / 8 + 4 * nxt
    # parents: level 0's frontier is one vertex, so vertex 1's parent is
    # written with its level (4 bytes); levels 1 and 2 push from one vertex
    # each too (the path), so every parent is written at claim
    assert bench.parents_bytes(rp, ci, lev, dirs, [1, 1, 1, 1], n) == [4.0, 4.0, 4.0, 0.0]
    # with a frontier of several vertices at level 1, level 2's kernel finds
    # vertex 2's parent; pushing over the same CSR it reads the levels of the
    # two expanded neighbours [1, 3] (8) and writes the parent (4); level 2
    # (one vertex) still writes vertex 3's parent at claim (4)
    assert bench.parents_bytes(rp, ci, lev, dirs, [1, 2, 1, 1], n) == [4.0, 0.0, 8.0 + 4.0 + 4.0,
                                                                        0.0]
    # if level 2 pulls instead, it scans vertex 2's in-neighbours up to the
    # first one a level up: 12 + 8 x (neighbours [1, 3] -> 1 hits first: 1
    # edge), and the pull finds vertex 3's parent itself
    assert bench.parents_bytes(rp, ci, lev, [1, 1, 2, 1], [1, 2, 1, 1], n) == [4.0, 0.0, 20.0,
                                                                                0.0]
    # a directed graph always scans in-neighbours
    assert bench.parents_bytes(rp, ci, lev, dirs, [1, 2, 1, 1], n, symmetric=False) == [
        4.0, 0.0, 12.0 + 8.0 + 4.0, 0.0]
