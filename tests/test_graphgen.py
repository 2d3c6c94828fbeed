"""Input generator: determinism, shapes, value ranges (no method arithmetic)."""
import numpy as np

import graphgen


def test_splitmix64_reference_values():
    # First outputs of the splitmix64 stream seeded with 0 (the generator's
    # published reference sequence: state advances by the golden gamma).
    assert graphgen.splitmix64(0) == 0xE220A8397B1DCDAF
    assert graphgen.splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


def test_rmat_deterministic_and_in_range():
    s1, d1 = graphgen.rmat_edges(10, 16, seed=1)
    s2, d2 = graphgen.rmat_edges(10, 16, seed=1)
    s3, _ = graphgen.rmat_edges(10, 16, seed=7)
    assert s1.shape == (16 << 10,)
    assert np.array_equal(s1, s2) and np.array_equal(d1, d2)
    assert not np.array_equal(s1, s3)
    assert s1.min() >= 0 and s1.max() < 1024 and d1.min() >= 0 and d1.max() < 1024


def test_rmat_quadrant_frequencies():
    # the top-level bit of (src, dst) follows (a, b, c, d)
    s, d = graphgen.rmat_edges(12, 16, seed=1)
    hi = 1 << 11
    sb, db = s >= hi, d >= hi
    m = s.shape[0]
    freq = np.array([np.sum(~sb & ~db), np.sum(~sb & db), np.sum(sb & ~db), np.sum(sb & db)]) / m
    assert np.allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=0.01)
    # vertex 0 is the hub
    deg = np.bincount(np.concatenate([s, d]), minlength=1 << 12)
    assert deg.argmax() == 0


def test_grid_edges():
    s, d = graphgen.grid_edges(3, 4)
    assert s.shape[0] == 3 * 3 + 2 * 4
    pairs = set(zip(s.tolist(), d.tolist()))
    assert (0, 1) in pairs and (0, 4) in pairs and (10, 11) in pairs and (7, 11) in pairs
    assert all(abs(a - b) in (1, 4) for a, b in pairs)


def test_weights_symmetric_integer_range():
    s, d = graphgen.rmat_edges(10, 16)
    w = graphgen.edge_weights(s, d, 1024, seed=2)
    w_rev = graphgen.edge_weights(d, s, 1024, seed=2)
    assert np.array_equal(w, w_rev)
    assert w.min() >= 1 and w.max() <= 64
    assert np.all(w == np.round(w))
    assert len(np.unique(w)) == 64


def test_sources_distinct_and_touched():
    g = graphgen.rmat(10)
    src = graphgen.sources(g.src, g.dst, g.n, 64, seed=3)
    t = graphgen.touched(g.src, g.dst, g.n)
    assert src.shape == (64,)
    assert len(set(src.tolist())) == 64
    assert t[src].all()
    assert np.array_equal(src, graphgen.sources(g.src, g.dst, g.n, 64, seed=3))


def test_poisson_arrivals():
    t = graphgen.poisson_arrivals(20000, rate=100.0, seed=4)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 0.01) < 0.0005
