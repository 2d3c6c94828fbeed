"""GPU test of grb_bfs_noalloc, the BFS entry point that allocates nothing
(its workspace is a file-scope device array): through the C ABI, its levels
and parents equal grb_bfs's (the entry point with a caller workspace) on
two calls in a row, the second on a smaller graph; a graph past the array's
size is refused with GRB_INSUFFICIENT_SPACE."""
import ctypes

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


def noalloc(grb, A, source, desc=None):
    f = grb.C_FUNCTIONS["grb_bfs_noalloc"]
    lev = torch.empty(max(A.nrows, 1), dtype=torch.int32, device="cuda")
    par = torch.empty(max(A.nrows, 1), dtype=torch.int32, device="cuda")
    code = f(ctypes.c_void_p(lev.data_ptr()), ctypes.c_void_p(par.data_ptr()), A.handle,
             int(source), ctypes.byref(desc) if desc is not None else None,
             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return code, lev[: A.nrows], par[: A.nrows]


def test_noalloc_equals_bfs_two_calls(grb):
    for scale, src, rule in ((16, 0, 1), (12, 5, 0)):  # second call: a smaller input
        g = graphgen.rmat(scale)
        A = grb.Matrix.from_raw(g)
        code, lev, par = noalloc(grb, A, src, grb.descriptor(rule=rule))
        assert code == 0
        ref_lev, ref_par = grb.bfs(A, src, desc=grb.descriptor(rule=rule))
        assert torch.equal(lev, ref_lev) and torch.equal(par, ref_par), scale
        ol, op, _ = oracle.bfs(oracle.Adjacency.from_raw(g), src)
        assert np.array_equal(lev.cpu().numpy(), ol) and np.array_equal(par.cpu().numpy(), op)
    # a high-diameter graph (the one-workgroup level loop) after them
    g = graphgen.grid(70, 40)
    A = grb.Matrix.from_raw(g)
    code, lev, par = noalloc(grb, A, 17)
    ref_lev, ref_par = grb.bfs(A, 17)
    assert code == 0 and torch.equal(lev, ref_lev) and torch.equal(par, ref_par)


def test_noalloc_refuses_graphs_past_its_array(grb):
    n = (1 << 24) + 1
    A = grb.Matrix(n, n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), None, symmetric=True)
    code, _, _ = noalloc(grb, A, 0)
    assert code == 9
