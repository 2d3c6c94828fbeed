"""GPU tests of the vector forms of the C ABI: the sparse (list) form of
grb_vector_create (sorted indices + device count) as a product's input,
mask and output, and grb_vector_extract (device -> host tuples).

A product whose operands are given as lists must give exactly what the
same product gives on the bitmap forms, and what the plain-loop oracle
gives; the list of an output must hold its present indices in order.
"""
import ctypes
import zlib

import numpy as np
import pytest

import graphgen
from oracle import mxv as M

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def grb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_01407_amd as g
    return g


SEMI = {"lor_land": ("lor_land", torch.uint8), "min_plus": ("min_plus_fp32", torch.float32),
        "plus_times": ("plus_times_fp32", torch.float32),
        "min_first": ("min_first_int32", torch.int32),
        "plus_times_fp64": ("plus_times_fp64", torch.float64)}
ONAME = {"plus_times_fp64": "plus_times"}


def seed(*key):
    return zlib.crc32(repr(key).encode())


def rand_entries(rng, n, p, semiring):
    out = {}
    for i in np.flatnonzero(rng.random(n) < p):
        if semiring == "lor_land":
            out[int(i)] = bool(rng.integers(0, 2))
        elif semiring == "min_first":
            out[int(i)] = int(rng.integers(0, 50))
        else:
            out[int(i)] = float(rng.integers(0, 9))
    return out


def make_vec(grb, n, dtype, entries, form):
    """form: 'bitmap', 'list' (list only) or 'both'."""
    v = grb.Vector(n, dtype, dense=form != "list", sparse=form != "bitmap")
    v.set_any(entries)
    return v


def test_extract_roundtrip(grb):
    rng = np.random.default_rng(7)
    n = 5000
    for form in ("bitmap", "list", "both"):
        for dt in (torch.uint8, torch.int32, torch.float32, torch.float64):
            ent = {int(i): (1 if dt == torch.uint8 else float(rng.integers(1, 100)))
                   for i in np.flatnonzero(rng.random(n) < 0.1)}
            v = make_vec(grb, n, dt, ent, form)
            idx, val = v.extract()
            assert idx.tolist() == sorted(ent), (form, dt)
            assert [float(x) for x in val] == [float(ent[i]) for i in sorted(ent)], (form, dt)
            code, nv = v.extract_code(capacity=len(ent) - 1)
            assert code == 9 and nv == len(ent)  # GRB_INSUFFICIENT_SPACE, count still reported
    e = grb.Vector(0, torch.float32)
    assert e.extract()[0].size == 0


def test_list_and_bitmap_agree_with_oracle(grb):
    """Random small products with the input, mask and output in every
    combination of forms: equal results, equal to the oracle."""
    for sname, (lib_name, dt) in SEMI.items():
        rng = np.random.default_rng(seed("forms", sname))
        for trial in range(12):
            n = int(rng.integers(1, 300))
            dens = float(rng.uniform(0.0, 0.1))
            triples = []
            for i in range(n):
                for j in np.flatnonzero(rng.random(n) < dens):
                    triples.append((i, int(j), int(rng.integers(1, 9))))
            rp, ci, v = _csr(n, triples)
            trp, tci, tv = _csr(n, [(j, i, x) for i, j, x in triples])
            if dt == torch.float64:
                v, tv = v.astype(np.float64), tv.astype(np.float64)
            A = grb.Matrix(n, n, rp, ci, v, trp, tci, tv, symmetric=False)
            u = rand_entries(rng, n, float(rng.uniform(0, 0.5)), ONAME.get(sname, sname))
            w_old = rand_entries(rng, n, 0.3, ONAME.get(sname, sname))
            mask = {i: 1 for i in range(n) if rng.random() < 0.5}
            comp = bool(trial % 2)
            replace = trial % 3 == 0
            flags = (grb.GRB_MASK_COMP if comp else 0) | (grb.GRB_REPLACE if replace else 0) | \
                grb.GRB_MASK_STRUCT
            ref = M.mxv(n, triples, u, semiring=ONAME.get(sname, sname), w_old=w_old, mask=mask,
                        complement=comp, structural=True, replace=replace)
            for direction in (0, 1, 2):
                for uf, mf, wf in (("bitmap", "bitmap", "bitmap"), ("list", "bitmap", "bitmap"),
                                   ("both", "list", "both"), ("list", "list", "list")):
                    U = make_vec(grb, n, dt, u, uf)
                    Mk = make_vec(grb, n, torch.uint8, mask, mf)
                    W = make_vec(grb, n, dt, w_old, wf)
                    grb.mxv(W, Mk, None, lib_name, A, U,
                            desc=grb.descriptor(direction=direction, rule=trial % 2, flags=flags))
                    got = W.to_dict()
                    key = (sname, trial, direction, uf, mf, wf)
                    assert set(got) == set(ref), key
                    for i in ref:
                        assert float(got[i]) == float(ref[i]), key
                    if W.indices is not None:
                        cnt = int(W.count.cpu()[0])
                        lst = W.indices[:cnt].cpu().numpy().tolist()
                        assert lst == sorted(ref), key


def _csr(n, triples):
    if not triples:
        return np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32)
    t = np.array(sorted(triples), dtype=np.float64)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, t[:, 0].astype(np.int64) + 1, 1)
    return np.cumsum(rp).astype(np.int32), t[:, 1].astype(np.int32), t[:, 2].astype(np.float32)


def test_list_input_rmat(grb):
    """R-MAT 13 with hub rows beyond the piece length: a list-only input
    gives the bitmap input's result in every direction (OR and min-plus)."""
    g = graphgen.rmat(13)
    rp, ci, w = grb.csr_from_edges(g.n, g.src, g.dst, g.w, symmetrise=True)
    A = grb.Matrix(g.n, g.n, rp, ci, w, symmetric=True)
    rng = np.random.default_rng(3)
    for sname in ("lor_land", "min_plus"):
        lib_name, dt = SEMI[sname]
        for p in (0.001, 0.05, 0.6):
            u = rand_entries(rng, g.n, p, sname)
            outs = []
            for form in ("bitmap", "list"):
                for direction in (0, 1, 2):
                    U = make_vec(grb, g.n, dt, u, form)
                    W = grb.Vector(g.n, dt)
                    grb.mxv(W, None, None, lib_name, A, U, desc=grb.descriptor(direction=direction))
                    outs.append(W.to_dict())
            assert all(o == outs[0] for o in outs), (sname, p)


def test_vector_form_errors(grb):
    f = grb.C_FUNCTIONS["grb_vector_create"]
    h = ctypes.c_void_p()
    ind = torch.zeros(10, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    vals = torch.zeros(10, dtype=torch.float32, device="cuda")
    # indices without a count, and no presence storage at all
    assert f(ctypes.byref(h), 10, grb.GRB_FP32, ctypes.c_void_p(vals.data_ptr()), None,
             ctypes.c_void_p(ind.data_ptr()), None) == 3
    assert f(ctypes.byref(h), 10, grb.GRB_FP32, ctypes.c_void_p(vals.data_ptr()), None, None,
             None) == 3
    # build on a list-only vector: its owner writes it
    v = grb.Vector(10, torch.float32, dense=False, sparse=True)
    idx = torch.tensor([1, 2], dtype=torch.int32, device="cuda")
    code = grb.C_FUNCTIONS["grb_vector_build"](v.handle, ctypes.c_void_p(idx.data_ptr()), None, 2,
                                               None)
    assert code == 8
    # an output without values
    A = grb.Matrix(10, 10, np.arange(11, dtype=np.int32), np.arange(10, dtype=np.int32),
                   np.ones(10, np.float32), symmetric=True)
    U = grb.Vector(10, torch.float32)
    U.set({1: 1.0})
    W = grb.Vector(10, torch.float32, values=False)
    ws = grb.workspace(grb.OP_MXV, A)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = grb.C_FUNCTIONS["grb_mxv"](W.handle, None, 0, grb.SEMIRINGS["min_plus_fp32"], A.handle,
                                      U.handle, None, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                      s)
    assert code == 4


def test_fill_clear_build_keep_list(grb):
    n = 1000
    v = grb.Vector(n, torch.float32, dense=True, sparse=True)
    v.set({5: 1.0, 900: 2.0, 77: 3.0})
    assert v.indices[: int(v.count.cpu()[0])].cpu().tolist() == [5, 77, 900]
    v.fill(4.0)
    assert int(v.count.cpu()[0]) == n
    assert v.indices.cpu().tolist() == list(range(n))
    idx, val = v.extract()
    assert idx.tolist() == list(range(n)) and set(val.tolist()) == {4.0}
    v.clear()
    assert int(v.count.cpu()[0]) == 0 and v.extract()[0].size == 0
    # a vector without values reads as 1 everywhere
    u = grb.Vector(n, torch.float32, values=False)
    u.set({3: None, 4: None})
    idx, val = u.extract()
    assert idx.tolist() == [3, 4] and val.tolist() == [1.0, 1.0]
