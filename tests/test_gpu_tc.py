"""GPU parity: grb_tricount and grb_mxm_masked against the oracle.

Triangle counts and PLUS_PAIR products are integers and must match exactly;
PLUS_TIMES products must lie within the floating-point error bound of a sum
of m products (|error| <= (m + 1) u / (1 - (m + 1) u) * sum |a b|, u the
unit roundoff).  Graphs are seeded R-MAT (a, b, c, d = 0.57, 0.19, 0.19,
0.05), grids, cliques, wheels and degenerate cases; a renumbering that puts
a 5000-entry row on the searched side exercises the path for rows longer
than the LDS copy.
"""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import mxm as omxm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def grb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_01407_amd as g
    return g


def _graph(kind):
    if kind.startswith("rmat"):
        return graphgen.rmat(int(kind[4:]), weights=False)
    if kind == "grid":
        return graphgen.grid(30, 41, weights=False)
    if kind == "clique":
        iu = np.triu_indices(70, 1)
        return graphgen.from_edges(kind, 70, iu[0], iu[1])
    if kind == "wheel":
        k = 2000
        cyc = np.arange(1, k + 1)
        return graphgen.from_edges(kind, k + 1, np.concatenate([np.zeros(k, np.int64), cyc]),
                                   np.concatenate([cyc, np.roll(cyc, -1)]))
    if kind == "two_comp":
        return graphgen.from_edges(kind, 12, [0, 1, 2, 5, 6, 7, 8], [1, 2, 0, 6, 7, 5, 9])
    if kind == "empty":
        return graphgen.from_edges(kind, 9, [], [])
    if kind == "single":
        return graphgen.from_edges(kind, 1, [], [])
    raise ValueError(kind)


def _lower(grb, n, rp, ci):
    return grb.Matrix(n, n, rp, ci, None, symmetric=False)


@pytest.mark.parametrize("kind", ["rmat10", "rmat12", "rmat14", "grid", "clique", "wheel",
                                  "two_comp", "empty", "single"])
def test_tricount_parity(grb, kind):
    g = _graph(kind)
    adj = oracle.Adjacency.from_raw(g)
    t, _ = oracle.triangles(adj)
    rp, ci, rank = grb.lower_by_degree(g.n, g.src, g.dst)
    L = _lower(grb, g.n, rp, ci)
    assert grb.tricount(L) == t
    c = grb.mxm_masked(L, L, L, "plus_pair_int32")
    Lt = (g.n, g.n, rp, ci, None)
    ref = omxm.mxm_masked(Lt, Lt, Lt, "plus_pair_int32")
    assert np.array_equal(c.cpu().numpy().astype(np.int64), ref.astype(np.int64))
    assert int(c.to(torch.int64).sum()) == t
    # repeatable
    assert grb.tricount(L) == t


@pytest.mark.parametrize("kind", ["rmat12", "wheel"])
def test_tricount_any_numbering(grb, kind):
    """The count does not depend on the numbering; numbering by decreasing
    id puts the hubs' whole neighbourhoods on the searched side (the wheel's
    hub row has 2000 entries, past the LDS copy)."""
    g = _graph(kind)
    adj = oracle.Adjacency.from_raw(g)
    t, _ = oracle.triangles(adj)
    off, nbr, _ = adj.arrays(weights=False)
    n = adj.n
    new = n - 1 - np.arange(n)  # decreasing id
    src = np.repeat(np.arange(n), np.diff(off))
    keep = new[nbr] < new[src]
    r, cc = new[src[keep]], new[nbr[keep]]
    order = np.lexsort((cc, r))
    r, cc = r[order], cc[order]
    rp = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=n))]).astype(np.int32)
    L = _lower(grb, n, rp, cc.astype(np.int32))
    assert np.diff(rp).max() > 1024 or kind != "wheel"
    assert grb.tricount(L) == t
    c = grb.mxm_masked(L, L, L, "plus_pair_int32")
    Lt = (n, n, rp, cc, None)
    assert np.array_equal(c.cpu().numpy().astype(np.int64),
                          omxm.mxm_masked(Lt, Lt, Lt, "plus_pair_int32").astype(np.int64))


def _rand_csr(rng, nr, nc, dens, long_rows=(), f32=True):
    rows, cols = [], []
    for i in range(nr):
        k = int(rng.binomial(nc, dens)) if i not in long_rows else min(nc, 1500)
        cs = np.sort(rng.choice(nc, size=k, replace=False))
        rows.append(np.full(k, i))
        cols.append(cs)
    ci = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    rp = np.concatenate([[0], np.cumsum([len(c) for c in cols])]).astype(np.int32)
    vals = rng.standard_normal(ci.shape[0])
    if f32:
        vals = vals.astype(np.float32).astype(np.float64)
    return rp, ci, vals


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("semiring", ["plus_times_fp32", "plus_times_fp64", "plus_pair_int32"])
def test_mxm_masked_parity(grb, seed, semiring):
    rng = np.random.default_rng(700 + seed)
    r, c, k = 300, 250, 2000
    f32 = semiring == "plus_times_fp32"
    arp, aci, av = _rand_csr(rng, r, k, 0.05, long_rows=(3, 77), f32=f32)
    brp, bci, bv = _rand_csr(rng, c, k, 0.05, long_rows=(5,), f32=f32)
    mrp, mci, _ = _rand_csr(rng, r, c, 0.1)
    vdt = np.float32 if f32 else np.float64
    A = grb.Matrix(r, k, arp, aci, av.astype(vdt), symmetric=False)
    B = grb.Matrix(c, k, brp, bci, bv.astype(vdt), symmetric=False)
    M = grb.Matrix(r, c, mrp, mci, None, symmetric=False)
    got = grb.mxm_masked(M, A, B, semiring).cpu().numpy().astype(np.float64)
    Mt, At, Bt = (r, c, mrp, mci, None), (r, k, arp, aci, av), (c, k, brp, bci, bv)
    ref = omxm.mxm_masked(Mt, At, Bt, semiring)
    if semiring == "plus_pair_int32":
        assert np.array_equal(got, ref)
        return
    cnt, mag = omxm.mxm_abs_bound(Mt, At, Bt)
    u = 2.0 ** -24 if f32 else 2.0 ** -53
    m = cnt + 1
    bound = m * u / (1 - m * u) * mag
    assert np.all(np.abs(got - ref) <= bound * 1.0001 + 1e-300)


def test_mxm_masked_edge_cases(grb):
    # empty mask; mask rows whose A row is empty; B rows empty
    A = grb.Matrix(3, 4, np.array([0, 0, 2, 3], np.int32), np.array([1, 3, 2], np.int32),
                   np.array([2.0, 3.0, 5.0]), symmetric=False)
    B = grb.Matrix(2, 4, np.array([0, 2, 2], np.int32), np.array([1, 3], np.int32),
                   np.array([7.0, 11.0]), symmetric=False)
    M = grb.Matrix(3, 2, np.array([0, 2, 4, 5], np.int32), np.array([0, 1, 0, 1, 0], np.int32),
                   None, symmetric=False)
    got = grb.mxm_masked(M, A, B, "plus_times_fp64").cpu().numpy()
    # row 0 of A is empty; A(1,:)·B(0,:) = 2*7 + 3*11; B row 1 is empty; A(2,:)·B(0,:) = 0
    assert np.array_equal(got, [0.0, 0.0, 47.0, 0.0, 0.0])
    E = grb.Matrix(3, 2, np.zeros(4, np.int32), np.zeros(0, np.int32), None, symmetric=False)
    assert grb.mxm_masked(E, A, B, "plus_times_fp64").numel() == 0
    with pytest.raises(grb.GrbError):
        grb.mxm_masked(M, B, A, "plus_times_fp64")  # dimension mismatch
    with pytest.raises(grb.GrbError):
        grb.mxm_masked(M, A, B, "plus_times_fp32")  # values are fp64
    with pytest.raises(grb.GrbError):
        grb.mxm_masked(M, A, B, "min_plus_fp64")


@pytest.mark.parametrize("semiring", ["plus_pair_int32", "plus_times_fp64"])
def test_mxm_masked_wide_columns(grb, semiring):
    """Columns past the structure-only kernel's LDS bitmap (65,536): rows of
    A with a short tail above it (kept in LDS) and with a long one (more
    than 256 entries, searched in place)."""
    rng = np.random.default_rng(77)
    r, c, k = 64, 48, 300_000
    rows_a = []
    for i in range(r):
        lo = rng.choice(65_536, size=int(rng.integers(0, 200)), replace=False)
        n_hi = 600 if i % 3 == 0 else int(rng.integers(0, 40))  # long / short tails
        hi = rng.choice(np.arange(65_536, k), size=n_hi, replace=False)
        rows_a.append(np.sort(np.concatenate([lo, hi])))
    rows_b = []
    for j in range(c):
        pool = np.concatenate([rows_a[j % r], rng.choice(k, size=300, replace=False)])
        rows_b.append(np.unique(rng.choice(pool, size=min(len(pool), 500), replace=False)))

    def csr(rows):
        rp = np.concatenate([[0], np.cumsum([len(x) for x in rows])]).astype(np.int32)
        ci = np.concatenate(rows).astype(np.int32)
        return rp, ci, rng.integers(1, 5, ci.shape[0]).astype(np.float64)

    arp, aci, av = csr(rows_a)
    brp, bci, bv = csr(rows_b)
    M = np.ones((r, c), dtype=bool)
    mrp = np.arange(0, r * c + 1, c, dtype=np.int32)
    mci = np.tile(np.arange(c, dtype=np.int32), r)
    A = grb.Matrix(r, k, arp, aci, av, symmetric=False)
    B = grb.Matrix(c, k, brp, bci, bv, symmetric=False)
    Mm = grb.Matrix(r, c, mrp, mci, None, symmetric=False)
    got = grb.mxm_masked(Mm, A, B, semiring).cpu().numpy().astype(np.float64)
    ref = omxm.mxm_masked((r, c, mrp, mci, None), (r, k, arp, aci, av), (c, k, brp, bci, bv),
                          semiring)
    assert np.array_equal(got, ref)  # integer-valued products: exact in fp64
    assert M.sum() == got.shape[0]
