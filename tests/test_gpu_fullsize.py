"""GPU parity at the benchmark's full sizes, in the launch configuration
bench.py times: RMAT scale 22 (edge factor 16, symmetrised, weights 1..64),
the 3000 x 3000 grid, and PageRank on the directed RMAT scale 22 graph.

The oracle computes every output in full at these sizes (a few seconds
each), so the comparison is element by element, not sampled.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def grb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_01407_amd as g
    return g


@pytest.fixture(scope="module")
def rmat22(grb):
    g = graphgen.rmat(22)
    return grb.Matrix.from_raw(g), oracle.Adjacency.from_raw(g)


@pytest.fixture(scope="module")
def grid3000(grb):
    g = graphgen.grid(3000, 3000)
    return grb.Matrix.from_raw(g), oracle.Adjacency.from_raw(g)


MODES = [("auto_paper", 0, 0), ("auto_exact", 0, 1), ("push", 1, 0), ("pull", 2, 0)]


@pytest.mark.parametrize("mode", MODES, ids=[m[0] for m in MODES])
def test_bfs_rmat22(grb, rmat22, mode):
    A, adj = rmat22
    ref_lev, ref_par, nl = oracle.bfs(adj, 0)
    lev, par = grb.bfs(A, 0, desc=grb.descriptor(direction=mode[1], rule=mode[2]))
    assert np.array_equal(lev.cpu().numpy(), ref_lev)
    assert np.array_equal(par.cpu().numpy(), ref_par)
    st = grb.last_stats()
    assert st["iterations"] == nl
    # the first batch of levels covers the search, and the empty next
    # frontier of its last level ends it without another launch
    assert st["launches"] == nl


def test_bfs_rmat22_other_sources(grb, rmat22):
    A, adj = rmat22
    src, dst = graphgen.rmat_edges(22)
    srcs = graphgen.sources(src, dst, 1 << 22, 3)
    for s in srcs:
        ref_lev, ref_par, _ = oracle.bfs(adj, int(s))
        lev, par = grb.bfs(A, int(s), desc=grb.descriptor(rule=1))
        assert np.array_equal(lev.cpu().numpy(), ref_lev), s
        assert np.array_equal(par.cpu().numpy(), ref_par), s


def test_bfs_rmat22_low_degree_sources(grb, rmat22):
    """Sources of degree 9 and 309: level 1 is a push of several vertices,
    level 2 a pull whose frontier holds tens of millions of in-edges, so the
    level-2 vertices' parents come from the level-1 vertices' offers."""
    A, adj = rmat22
    for s in (1122651, 2886679, 2662536):
        ref_lev, ref_par, _ = oracle.bfs(adj, s)
        lev, par = grb.bfs(A, s, desc=grb.descriptor(rule=1, flags=grb.GRB_PROFILE))
        st = grb.last_stats()
        assert st["direction"][:3] == [1, 1, 2], (s, st["direction"])
        assert np.array_equal(lev.cpu().numpy(), ref_lev), s
        assert np.array_equal(par.cpu().numpy(), ref_par), s


@pytest.mark.parametrize("rule", [0, 1])
def test_sssp_rmat22(grb, rmat22, rule):
    A, adj = rmat22
    ref, _, _ = oracle.sssp(adj, 0)
    dist = grb.sssp(A, 0, desc=grb.descriptor(rule=rule))
    assert np.array_equal(dist.cpu().numpy(), ref)


def test_sssp_rmat22_forced_pull(grb, rmat22):
    """Every round pulled (the benchmark's forced-pull run): the pull forms
    that gather a distance per edge, test the frontier bit first, or load
    only members' weights all run at full size."""
    A, adj = rmat22
    ref, _, _ = oracle.sssp(adj, 0)
    dist = grb.sssp(A, 0, desc=grb.descriptor(direction=2, flags=grb.GRB_PROFILE))
    st = grb.last_stats()
    assert st["pulls"] == st["iterations"] and st["pushes"] == 0
    assert np.array_equal(dist.cpu().numpy(), ref)


def _to_words(bits):
    b = np.packbits(bits.astype(np.uint8), bitorder="little")
    b = np.concatenate([b, np.zeros((-len(b)) % 8, np.uint8)])
    return b.view(np.int64)


def _vector(grb, vals, has, dtype):
    n = has.shape[0]
    v = grb.Vector(n, dtype)
    v.values[:n] = torch.from_numpy(vals.astype(np.uint8)).to(v.values.device)
    words = _to_words(has)
    v.bitmap[: len(words)] = torch.from_numpy(words).to(v.values.device)
    return v


SWEEP = [(1e-4, 0.0), (1e-2, 0.5), (0.05, 0.0), (0.2, 0.5)]


@pytest.mark.parametrize("pq", SWEEP, ids=[f"p{p}_q{q}" for p, q in SWEEP])
def test_mxv_sweep_rmat22(grb, rmat22, pq):
    """Points of the benchmark's mxv sweep, element by element against the
    oracle's dense-array product: w<not m, struct, replace> = A u over
    LOR_LAND, u random of density p (a tenth of its entries false), m a
    random set of density q, w holding stale entries that REPLACE must clear
    outside the mask; forced push, forced pull and automatic."""
    A, adj = rmat22
    p, q = pq
    n = A.nrows
    rng = np.random.default_rng(int(p * 1e6) * 7 + int(q * 10))
    u_has = rng.random(n) < p
    u_val = u_has & (rng.random(n) >= 0.1)
    m_has = rng.random(n) < q
    w_has = rng.random(n) < 0.3
    w_val = w_has & (rng.random(n) < 0.5)
    flags = grb.GRB_MASK_COMP | grb.GRB_MASK_STRUCT | grb.GRB_REPLACE
    ref_v, ref_h = oracle.mxv_dense(adj, "lor_land", u_val, u_has, w_val=w_val, w_has=w_has,
                                    mask_val=m_has, mask_has=m_has, flags=flags)
    U = _vector(grb, u_val, u_has, torch.uint8)
    Mk = _vector(grb, m_has, m_has, torch.uint8)
    ws = grb.workspace(grb.OP_MXV, A)
    for direction in (1, 2, 0):
        W = _vector(grb, w_val, w_has, torch.uint8)
        grb.mxv(W, Mk, None, "lor_land", A, U,
                desc=grb.descriptor(direction=direction, rule=1, flags=flags), ws=ws)
        torch.cuda.synchronize()
        words = W.bitmap.cpu().numpy().view(np.uint8)
        got_h = np.unpackbits(words, bitorder="little")[:n].astype(bool)
        assert np.array_equal(got_h, ref_h), (direction, int((got_h != ref_h).sum()))
        got_v = W.values[:n].cpu().numpy()
        assert np.array_equal(got_v[ref_h] != 0, ref_v[ref_h] != 0), direction


def test_grid3000_bfs_sssp(grb, grid3000):
    A, adj = grid3000
    ref_lev, ref_par, nl = oracle.bfs(adj, 0)
    lev, par = grb.bfs(A, 0)
    assert nl == 5999
    assert np.array_equal(lev.cpu().numpy(), ref_lev)
    assert np.array_equal(par.cpu().numpy(), ref_par)
    # the level loop's barriers given up from the start (hand-over at level 1)
    lev, par = grb.bfs(A, 0, desc=grb.descriptor(flags=grb.GRB_LOOP_NO_WAIT))
    assert np.array_equal(lev.cpu().numpy(), ref_lev)
    assert np.array_equal(par.cpu().numpy(), ref_par)
    ref, _, _ = oracle.sssp(adj, 0)
    dist = grb.sssp(A, 0)
    assert np.array_equal(dist.cpu().numpy(), ref)
    # bucketed rounds (multi-workgroup loop), also with its barriers given up
    for flags in (0, grb.GRB_LOOP_NO_WAIT):
        dist = grb.sssp(A, 0, delta=2048.0, desc=grb.descriptor(flags=flags))
        assert np.array_equal(dist.cpu().numpy(), ref), flags


def test_pagerank_rmat22_directed(grb):
    g = graphgen.rmat(22, symmetric=False, weights=False)
    adj = oracle.Adjacency.from_raw(g)
    ref, it, _ = oracle.pagerank(adj, 0.85, 50, 1e-7)
    P = grb.Matrix.from_raw(g, weights=False)
    p32, it32, _ = grb.pagerank(P, dtype=torch.float32, max_iter=it, tol=0.0)
    p64, it64, _ = grb.pagerank(P, dtype=torch.float64, max_iter=it, tol=0.0)
    assert it32 == it and it64 == it
    err32 = np.abs(p32.cpu().numpy().astype(np.float64) - ref).sum()
    err64 = np.abs(p64.cpu().numpy() - ref).sum()
    assert err32 <= 1e-5, err32
    assert err64 <= 1e-10, err64
    _, it_auto, _ = grb.pagerank(P, dtype=torch.float64, max_iter=50, tol=1e-7)
    assert it_auto == it
    # adaptive form (converged vertices frozen), as the benchmark runs it
    aref, ait, _, aact, _ = oracle.pagerank_adaptive(adj, 1e-4, 0.85, 50, 1e-7)
    a32, it32, _, act32 = grb.pagerank_adaptive(P, 1e-4, dtype=torch.float32, max_iter=ait,
                                                tol=0.0)
    a64, it64, _, act64 = grb.pagerank_adaptive(P, 1e-4, dtype=torch.float64, max_iter=ait,
                                                tol=0.0)
    assert it64 == ait and act64 == aact
    err32 = np.abs(a32.cpu().numpy().astype(np.float64) - aref).sum()
    err64 = np.abs(a64.cpu().numpy() - aref).sum()
    assert err32 <= 1e-5, err32
    assert err64 <= 1e-10, err64


def test_tricount_rmat22(grb):
    """Triangle count of RMAT-22: the degree-ordered operand equals the
    oracle's, sampled per-edge counts (row intersections) match the
    oracle's one by one, and the fused count equals the sum of the product."""
    from oracle import mxm as omxm
    g = graphgen.rmat(22, weights=False)
    adj = oracle.Adjacency.from_raw(g)
    off, nbr, _ = adj.arrays(weights=False)
    rp, ci, rank = grb.lower_by_degree(g.n, g.src, g.dst)
    orp, oci, orank = omxm.lower_by_degree(g.n, off, nbr)
    assert np.array_equal(rank, orank)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    del off, nbr, orp, oci
    L = grb.Matrix(g.n, g.n, rp, ci, None, symmetric=False)
    t = grb.tricount(L)
    c = grb.mxm_masked(L, L, L, "plus_pair_int32")
    assert int(c.to(torch.int64).sum()) == t
    rng = np.random.default_rng(11)
    ent = rng.choice(ci.shape[0], 3000, replace=False)
    got = c[torch.from_numpy(ent).to(c.device)].cpu().numpy().astype(np.int64)
    assert np.array_equal(got, omxm.edge_counts(rp, ci, ent))
