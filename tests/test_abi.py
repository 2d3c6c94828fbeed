"""C ABI checks that need no GPU: the library loads, exports every function
include/grb.h declares, validates arguments on the host before any HIP call,
and its host CSR builder agrees with the oracle's independent adjacency."""
import ctypes
import os
import re

import numpy as np
import pytest

import graphgen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "grb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(grb_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def grb():
    import paper_1908_01407_amd as g
    return g


def test_every_declared_symbol_is_exported(grb):
    names = _declared()
    assert "grb_mxv" in names and "grb_vxm" in names and "grb_bfs" in names
    lib = ctypes.CDLL(grb.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wires each of them
    assert set(names) <= set(grb.C_FUNCTIONS), set(names) - set(grb.C_FUNCTIONS)


def test_error_strings_and_version(grb):
    assert grb.grb_version() >= 100
    for code in range(12):
        assert grb.grb_error_string(code)
    assert b"unknown" in grb.grb_error_string(99)


def test_descriptor_defaults(grb):
    d = grb.descriptor()
    assert d.direction == 0 and d.switch_rule == 0 and d.switch_denominator == 10
    assert d.flags == 0 and d.max_iter == 0


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: creation only stores pointers


def _create(grb, n=4, nnz=3, rp=FAKE, ci=FAKE, vals=None, vt=2, trp=None, tci=None, tv=None,
            flags=0):
    h = ctypes.c_void_p()
    rc = grb.grb_matrix_create(ctypes.byref(h), n, n, nnz, rp, ci, vals, vt, trp, tci, tv, flags)
    return rc, h


def test_matrix_create_validation(grb):
    assert _create(grb, n=-1)[0] == 4
    assert _create(grb, nnz=2**31)[0] == 4
    assert _create(grb, rp=None)[0] == 3
    assert _create(grb, flags=0x80)[0] == 4
    assert _create(grb, vals=FAKE, vt=0)[0] == 4  # bool values are not a matrix type
    assert _create(grb, flags=1, trp=FAKE, tci=FAKE)[0] == 4  # symmetric + transpose
    assert _create(grb, trp=None, tci=FAKE)[0] == 4
    rc, h = _create(grb, flags=1)
    assert rc == 0
    n = ctypes.c_int64()
    assert grb.grb_matrix_nrows(h, ctypes.byref(n)) == 0 and n.value == 4
    assert grb.grb_matrix_nvals(h, ctypes.byref(n)) == 0 and n.value == 3
    sz = ctypes.c_size_t()
    assert grb.grb_matrix_meta_size(h, ctypes.byref(sz)) == 0 and sz.value > 0
    # products and drivers refuse an unprepared matrix before touching the GPU
    assert grb.grb_bfs(FAKE, None, h, 0, None, FAKE, 1 << 20, None) == 2
    assert grb.grb_sssp(FAKE, h, 0, None, FAKE, 1 << 20, None) == 2
    assert grb.grb_sssp_delta(FAKE, h, 0, 64.0, None, FAKE, 1 << 20, None) == 2
    it = ctypes.c_int32()
    assert grb.grb_pagerank(FAKE, 2, h, 0.85, 5, 0.0, ctypes.byref(it), None, None, FAKE,
                            1 << 20, None) == 2
    assert grb.grb_pagerank_adaptive(FAKE, 2, h, 0.85, 5, 0.0, 1e-3, ctypes.byref(it), None,
                                     None, None, FAKE, 1 << 20, None) == 2
    for bad in (-1e-3, float("nan"), float("inf")):  # bad threshold: refused first
        assert grb.grb_pagerank_adaptive(FAKE, 2, h, 0.85, 5, 0.0, bad, ctypes.byref(it), None,
                                         None, None, FAKE, 1 << 20, None) == 4
    assert grb.grb_matrix_free(ctypes.byref(h)) == 0 and not h.value
    assert grb.grb_bfs(FAKE, None, None, 0, None, FAKE, 1 << 20, None) == 2


def test_vector_and_workspace_validation(grb):
    h = ctypes.c_void_p()
    assert grb.grb_vector_create(ctypes.byref(h), -1, 2, FAKE, FAKE, None, None) == 4
    assert grb.grb_vector_create(ctypes.byref(h), 10, 7, FAKE, FAKE, None, None) == 4
    # no presence storage (neither bitmap nor list), or half a list
    assert grb.grb_vector_create(ctypes.byref(h), 10, 2, FAKE, None, None, None) == 3
    assert grb.grb_vector_create(ctypes.byref(h), 10, 2, FAKE, None, FAKE, None) == 3
    assert grb.grb_vector_create(ctypes.byref(h), 10, 2, FAKE, None, None, FAKE) == 3
    # values may be absent (every entry 1); list-only and both forms
    assert grb.grb_vector_create(ctypes.byref(h), 10, 2, None, FAKE, None, None) == 0
    assert grb.grb_vector_free(ctypes.byref(h)) == 0
    assert grb.grb_vector_create(ctypes.byref(h), 10, 2, FAKE, None, FAKE, FAKE) == 0
    assert grb.grb_vector_free(ctypes.byref(h)) == 0
    assert grb.grb_vector_create(ctypes.byref(h), 10, 2, FAKE, FAKE, FAKE, FAKE) == 0
    assert grb.grb_vector_free(ctypes.byref(h)) == 0
    assert grb.grb_vector_create(ctypes.byref(h), 10, 2, FAKE, FAKE, None, None) == 0
    n = ctypes.c_int64()
    assert grb.grb_vector_size(h, ctypes.byref(n)) == 0 and n.value == 10
    assert grb.grb_vector_nvals(h, ctypes.byref(n), None, 0, None) == 9  # workspace too small
    # extract: argument errors are caught before any device work
    assert grb.grb_vector_extract(h, None, None, 5, None, None, 0, None) == 3
    assert grb.grb_vector_extract(h, None, None, -1, ctypes.byref(n), None, 0, None) == 4
    assert grb.grb_vector_extract(h, None, None, 5, ctypes.byref(n), None, 0, None) == 9
    assert grb.grb_vector_extract(None, None, None, 5, ctypes.byref(n), None, 0, None) == 2
    assert grb.grb_vector_free(ctypes.byref(h)) == 0
    sz = ctypes.c_size_t()
    assert grb.grb_workspace_size(1, None, 0, ctypes.byref(sz)) == 2
    assert grb.grb_workspace_size(5, None, 0, ctypes.byref(sz)) == 0 and sz.value >= 64
    assert grb.grb_workspace_size(7, None, 1000, ctypes.byref(sz)) == 0 and sz.value > 12000
    assert grb.grb_workspace_size(7, None, -1, ctypes.byref(sz)) == 4
    rc, m = _create(grb, n=1000, nnz=5000, flags=1)
    for op in (0, 1, 2):
        assert grb.grb_workspace_size(op, m, 0, ctypes.byref(sz)) == 0 and sz.value > 0
    assert grb.grb_workspace_size(3, m, 3, ctypes.byref(sz)) == 4
    grb.grb_matrix_free(ctypes.byref(m))


@pytest.mark.parametrize("kind", ["rmat", "rmat_dir", "grid", "tiny"])
def test_csr_builder_matches_oracle_adjacency(grb, kind):
    if kind == "rmat":
        g = graphgen.rmat(12)
    elif kind == "rmat_dir":
        g = graphgen.rmat(11, symmetric=False)
    elif kind == "grid":
        g = graphgen.grid(17, 23)
    else:
        g = graphgen.from_edges("tiny", 5, [0, 0, 1, 3, 3, 4, 2], [1, 1, 0, 3, 4, 3, 0],
                                [9, 2, 5, 1, 7, 3, 4], symmetric=True)
    rp, ci, w = grb.csr_from_edges(g.n, g.src, g.dst, g.w, symmetrise=g.symmetric)
    adj = oracle.Adjacency.from_raw(g)
    off, nbr, ow = adj.arrays()
    assert np.array_equal(rp.astype(np.int64), off)
    assert np.array_equal(ci, nbr)
    assert np.array_equal(w.astype(np.float64), ow)


def test_csr_builder_errors(grb):
    with pytest.raises(grb.GrbError) as e:
        grb.csr_from_edges(4, [0, 5], [1, 2])
    assert e.value.code == 5
    rp, ci, w = grb.csr_from_edges(3, [], [], None)
    assert rp.tolist() == [0, 0, 0, 0] and ci.size == 0 and w is None


@pytest.mark.parametrize("kind", ["rmat10", "rmat12", "grid", "clique", "empty"])
def test_lower_by_degree_matches_oracle(grb, kind):
    """grb_csr_lower_by_degree (host setup of triangle counting) gives the
    oracle's degree-ordered strict lower triangle exactly."""
    from oracle import mxm as omxm
    if kind.startswith("rmat"):
        g = graphgen.rmat(int(kind[4:]), weights=False)
    elif kind == "grid":
        g = graphgen.grid(9, 11, weights=False)
    elif kind == "clique":
        iu = np.triu_indices(40, 1)
        g = graphgen.from_edges("clique", 40, iu[0], iu[1])
    else:
        g = graphgen.from_edges("empty", 5, [], [])
    adj = oracle.Adjacency.from_raw(g)
    off, nbr, _ = adj.arrays(weights=False)
    rp, ci, rank = grb.lower_by_degree(g.n, g.src, g.dst)
    orp, oci, orank = omxm.lower_by_degree(g.n, off, nbr)
    assert np.array_equal(rank, orank)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)


def test_mxm_argument_errors(grb):
    rc, h = _create(grb, flags=1)
    assert rc == 0
    it = ctypes.c_int64()
    # masked products refuse semirings they do not provide, before any launch
    assert grb.grb_mxm_masked(FAKE, h, h, h, 1, None, FAKE, 1 << 20, None) == 8
    assert grb.grb_mxm_masked(FAKE, h, h, h, 99, None, FAKE, 1 << 20, None) == 4
    assert grb.grb_mxm_masked(FAKE, h, h, h, 3, None, FAKE, 1 << 20, None) == 6  # no fp32 values
    assert grb.grb_mxm_masked(FAKE, None, h, h, 7, None, FAKE, 1 << 20, None) == 2
    assert grb.grb_mxm_masked(FAKE, h, h, h, 7, None, FAKE, 16, None) == 9  # workspace too small
    assert grb.grb_tricount(None, h, None, FAKE, 1 << 20, None) == 3
    assert grb.grb_tricount(ctypes.byref(it), None, None, FAKE, 1 << 20, None) == 2
    d = grb.descriptor(flags=grb.GRB_MASK_COMP)
    assert grb.grb_tricount(ctypes.byref(it), h, ctypes.byref(d), FAKE, 1 << 20, None) == 8
    sz = ctypes.c_size_t()
    assert grb.grb_workspace_size(6, None, 0, ctypes.byref(sz)) == 0 and sz.value >= 8
    assert grb.grb_matrix_free(ctypes.byref(h)) == 0


def test_stream_handle_lookup(grb, monkeypatch):
    """The binding passes the current stream's raw handle: through torch's
    raw-handle call for the current device when torch has it, else through
    the public Stream object; an explicit stream's handle is used as given."""
    import types

    calls = []
    fast = types.SimpleNamespace(
        _C=types.SimpleNamespace(_cuda_getCurrentRawStream=lambda dev: calls.append(dev) or 0x5000 + dev),
        cuda=types.SimpleNamespace(current_device=lambda: 3,
                                   current_stream=lambda: pytest.fail("public path taken")))
    monkeypatch.setattr(grb, "_torch", lambda: fast)
    assert grb._stream(None).value == 0x5003 and calls == [3]
    slow = types.SimpleNamespace(
        _C=types.SimpleNamespace(),
        cuda=types.SimpleNamespace(current_stream=lambda: types.SimpleNamespace(cuda_stream=0x77)))
    monkeypatch.setattr(grb, "_torch", lambda: slow)
    assert grb._stream(None).value == 0x77
    assert grb._stream(types.SimpleNamespace(cuda_stream=0x99)).value == 0x99
