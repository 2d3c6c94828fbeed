"""GPU parity of connected components (grb_cc, FastSV hooking and
shortcutting driven by the library's min-second product): every vertex's
label equals the oracle's (the smallest vertex id of its component) on
R-MAT, grid, sparse random graphs with many components, edge cases and a
directed matrix (weak components), in every direction mode of the product,
and at RMAT scale 22."""
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


def _graph(name):
    if name == "rmat14":
        return graphgen.rmat(14)
    if name == "rmat18":
        return graphgen.rmat(18)
    if name == "grid":
        return graphgen.grid(33, 70)
    if name == "sparse":  # many components, sizes from 1 to thousands
        rng = np.random.default_rng(31)
        n = 40000
        src, dst = rng.integers(0, n, 22000), rng.integers(0, n, 22000)
        return graphgen.from_edges(name, n, src, dst, np.ones(22000))
    if name == "path":
        k = 3000
        return graphgen.from_edges(name, k, np.arange(k - 1)[::-1], np.arange(1, k)[::-1],
                                   np.ones(k - 1))
    if name == "two_comp":
        return graphgen.from_edges(name, 133, [0, 1, 2, 3, 10, 11, 12, 130],
                                   [1, 2, 3, 0, 11, 12, 13, 131], np.ones(8))
    if name == "empty":
        return graphgen.from_edges(name, 70, [], [], [])
    if name == "single":
        return graphgen.from_edges(name, 1, [], [], [])
    if name == "rmat_dir":
        return graphgen.rmat(12, symmetric=False)
    raise KeyError(name)


NAMES = ["rmat14", "rmat18", "grid", "sparse", "path", "two_comp", "empty", "single", "rmat_dir"]


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("direction", [0, 1, 2], ids=["auto", "push", "pull"])
def test_cc_parity(grb, name, direction):
    g = _graph(name)
    A = grb.Matrix.from_raw(g)
    # weak components: the oracle symmetrises the edge list
    ref, ncomp = oracle.cc(oracle.Adjacency(g.n, g.src, g.dst, symmetrise=True))
    lab, it = grb.cc(A, desc=grb.descriptor(direction=direction))
    got = lab.cpu().numpy()
    assert np.array_equal(got, ref), (name, direction, it)
    assert int((got == np.arange(g.n)).sum()) == ncomp
    assert it >= 1 or g.n == 0


def test_cc_iteration_cap(grb):
    g = _graph("path")
    A = grb.Matrix.from_raw(g)
    lab, it = grb.cc(A, desc=grb.descriptor(max_iter=2))
    assert it == 2
    got = lab.cpu().numpy()
    # labels after two iterations: vertex ids of the path, no smaller than
    # the final label (0) and never above the vertex itself
    assert np.all(got >= 0) and np.all(got <= np.arange(g.n))
    full, it_full = grb.cc(A)
    assert it_full > 2 and int(full.max()) == 0


def test_cc_rmat22(grb):
    g = graphgen.rmat(22, weights=False)
    A = grb.Matrix.from_raw(g, weights=False)
    ref, ncomp = oracle.cc(oracle.Adjacency.from_raw(g))
    lab, it = grb.cc(A)
    assert np.array_equal(lab.cpu().numpy(), ref), it
