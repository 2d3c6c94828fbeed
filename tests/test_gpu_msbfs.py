"""GPU parity of the batched multi-source BFS (grb_msbfs) against k
independent oracle BFS runs: every (vertex, query) level must match, in
every direction mode and query-tile width, for full and partial 64-query
words, repeated sources and isolated sources."""
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
def rmat14(grb):
    g = graphgen.rmat(14)
    return g, grb.Matrix.from_raw(g), oracle.Adjacency.from_raw(g)


@pytest.mark.parametrize("k", [1, 64, 100, 512])
@pytest.mark.parametrize("mode", [(0, 0), (0, 1), (1, 0), (2, 0)],
                         ids=["auto_paper", "auto_exact", "push", "pull"])
def test_msbfs_rmat14(grb, rmat14, k, mode):
    g, A, adj = rmat14
    src = graphgen.sources(g.src, g.dst, g.n, k, seed=3)
    if k > 3:
        src[1] = src[0]  # repeated source
        deg = np.diff(adj.arrays(weights=False)[0])
        src[2] = int(np.flatnonzero(deg == 0)[0])  # isolated source
    ref = oracle.msbfs(adj, src, nthreads=8)
    W = (k + 63) // 64
    # every tile the autotuner may pick: query words per pass (clamped to
    # the batch) by launch width (0 = the default width)
    for kt in sorted({min(x, W) for x in (0, 1, 2, 4, 8)}):
        for grid in (0, 1024, 4096):
            lev = grb.msbfs(A, src, words_per_pass=kt, grid=grid,
                            desc=grb.descriptor(direction=mode[0], rule=mode[1]))
            got = lev.cpu().numpy().T
            assert np.array_equal(got, ref), (k, mode, kt, grid)


def test_msbfs_grid_and_directed(grb):
    for g in (graphgen.grid(40, 70), graphgen.rmat(12, symmetric=False)):
        A = grb.Matrix.from_raw(g)
        adj = oracle.Adjacency.from_raw(g)
        src = np.arange(0, g.n, max(1, g.n // 70))[:70].astype(np.int32)
        ref = oracle.msbfs(adj, src, nthreads=8)
        for direction in (0, 1, 2):
            lev = grb.msbfs(A, src, desc=grb.descriptor(direction=direction))
            assert np.array_equal(lev.cpu().numpy().T, ref), (g.name, direction)


def test_msbfs_matches_single_source(grb, rmat14):
    g, A, adj = rmat14
    src = graphgen.sources(g.src, g.dst, g.n, 8, seed=5)
    lev = grb.msbfs(A, src).cpu().numpy()
    for q, s in enumerate(src):
        single, _ = grb.bfs(A, int(s), parents=False)
        assert np.array_equal(lev[:, q], single.cpu().numpy())
