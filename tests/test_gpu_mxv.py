"""GPU parity of grb_mxv / grb_vxm against the plain-loop oracle.

Random small matrices (empty rows, hub rows, isolated columns) with every
semiring x mask (none / value / structural, complemented or not) x accum x
REPLACE x transpose x direction (push / pull / auto).  Values are small
integers so every semiring is exact in any summation order; the results
must match element by element.  Larger R-MAT inputs check push = pull and
rows longer than the pull split threshold.  The fp64 semirings run the
same cases with float64 vectors; argument errors are checked for their
codes and for leaving the output untouched.
"""
import ctypes
import json
import os
import zlib

import numpy as np
import pytest

import graphgen
from oracle import mxv as M

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def grb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_01407_amd as g
    return g


# test name -> (library semiring, oracle semiring)
GRB_NAME = {"lor_land": "lor_land", "min_plus": "min_plus_fp32", "plus_times": "plus_times_fp32",
            "min_first": "min_first_int32", "min_second": "min_second_int32",
            "min_plus_fp64": "min_plus_fp64", "plus_times_fp64": "plus_times_fp64"}
ORACLE_NAME = {"min_plus_fp64": "min_plus", "plus_times_fp64": "plus_times"}
ACCUM = {"lor_land": "lor", "min_plus": "min", "plus_times": "plus", "min_first": "min",
         "min_second": "min", "min_plus_fp64": "min", "plus_times_fp64": "plus"}


def oname(semiring):
    return ORACLE_NAME.get(semiring, semiring)


def vec_dtype(semiring):
    return {"lor_land": torch.uint8, "min_plus": torch.float32, "plus_times": torch.float32,
            "min_first": torch.int32, "min_second": torch.int32,
            "min_plus_fp64": torch.float64, "plus_times_fp64": torch.float64}[semiring]


def fixed_seed(*key):
    """Seed derived from the case's name (stable across processes)."""
    return zlib.crc32(repr(key).encode())


def csr(n_rows, triples):
    if not triples:
        return np.zeros(n_rows + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32)
    t = np.array(triples, dtype=np.float64)
    order = np.lexsort((t[:, 1], t[:, 0]))
    t = t[order]
    rows = t[:, 0].astype(np.int64)
    rp = np.zeros(n_rows + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp).astype(np.int32), t[:, 1].astype(np.int32), t[:, 2].astype(np.float32)


def device_matrix(grb, n_rows, n_cols, triples, valued=True, fp64=False):
    rp, ci, v = csr(n_rows, triples)
    trp, tci, tv = csr(n_cols, [(j, i, x) for (i, j, x) in triples])
    if fp64:
        v, tv = v.astype(np.float64), tv.astype(np.float64)
    return grb.Matrix(n_rows, n_cols, rp, ci, v if valued else None, trp, tci,
                      tv if valued else None, symmetric=False)


def rand_vec(rng, n, p, semiring):
    out = {}
    for i in range(n):
        if rng.random() < p:
            if semiring == "lor_land":
                out[i] = bool(rng.integers(0, 2))
            elif semiring in ("min_first", "min_second"):
                out[i] = int(rng.integers(0, 50))
            else:
                out[i] = float(rng.integers(0, 20))
    return out


def rand_matrix(rng, n_rows, n_cols, density, semiring, hub=False):
    triples = []
    for i in range(n_rows):
        for j in range(n_cols):
            if rng.random() < density:
                val = int(rng.integers(0, 3)) if semiring == "lor_land" else int(rng.integers(1, 9))
                triples.append((i, j, val))
    if hub and n_rows:
        h = int(rng.integers(0, n_rows))
        have = {j for (i, j, _) in triples if i == h}
        triples += [(h, j, 1) for j in range(n_cols) if j not in have]
    return triples


def check_case(grb, rng, semiring, is_vxm, direction, n_rows, n_cols, trial, valued=True):
    triples = rand_matrix(rng, n_rows, n_cols, float(rng.uniform(0.0, 0.5)), oname(semiring),
                          hub=trial % 5 == 0)
    transpose = trial % 3 == 2
    out_rows = (n_cols if not transpose else n_rows) if is_vxm else (n_rows if not transpose
                                                                      else n_cols)
    in_len = n_rows + n_cols - out_rows
    A = device_matrix(grb, n_rows, n_cols, triples, valued=valued,
                      fp64=vec_dtype(semiring) == torch.float64)
    o_triples = triples if valued else [(i, j, 1) for (i, j, _) in triples]
    u = rand_vec(rng, in_len, float(rng.uniform(0, 1)), oname(semiring))
    w_old = rand_vec(rng, out_rows, 0.5, oname(semiring))
    mask = None if trial % 4 == 0 else {i: int(rng.integers(0, 3)) for i in range(out_rows)
                                        if rng.random() < 0.6}
    comp = trial % 3 == 1
    struct = trial % 5 == 3
    accum = ACCUM[semiring] if trial % 2 else None
    replace = trial % 7 < 3
    dt = vec_dtype(semiring)
    W = grb.Vector(out_rows, dt)
    W.set(w_old)
    U = grb.Vector(in_len, dt)
    U.set(u)
    Mk = None
    if mask is not None:
        Mk = grb.Vector(out_rows, torch.int32)
        Mk.set(mask)
    flags = ((grb.GRB_MASK_COMP if comp else 0) | (grb.GRB_MASK_STRUCT if struct else 0) |
             (grb.GRB_REPLACE if replace else 0) | (grb.GRB_TRAN_A if transpose else 0))
    d = grb.descriptor(direction=direction, flags=flags, rule=trial % 2)
    if is_vxm:
        grb.vxm(W, Mk, accum, GRB_NAME[semiring], U, A, desc=d)
    else:
        grb.mxv(W, Mk, accum, GRB_NAME[semiring], A, U, desc=d)
    torch.cuda.synchronize()
    fn = M.vxm if is_vxm else M.mxv
    ref = fn(out_rows, o_triples, u, semiring=oname(semiring), w_old=w_old, mask=mask,
             complement=comp, structural=struct, accum=accum, replace=replace,
             transpose=transpose)
    got = W.to_dict()
    assert set(got) == set(ref), (trial, sorted(got), sorted(ref))
    for i in ref:
        assert float(got[i]) == float(ref[i]), (trial, i, got[i], ref[i])


@pytest.mark.parametrize("semiring", list(GRB_NAME))
@pytest.mark.parametrize("is_vxm", [False, True], ids=["mxv", "vxm"])
@pytest.mark.parametrize("direction", [0, 1, 2], ids=["auto", "push", "pull"])
def test_mxv_random_small(grb, semiring, is_vxm, direction):
    rng = np.random.default_rng(fixed_seed(semiring, is_vxm, direction))
    for trial in range(24):
        n_rows = int(rng.integers(1, 150))
        n_cols = int(rng.integers(1, 150))
        check_case(grb, rng, semiring, is_vxm, direction, n_rows, n_cols, trial,
                   valued=trial % 6 != 5)


def test_running_example(grb):
    with open(os.path.join(GOLDEN, "running_example_bfs_step.json")) as f:
        ex = json.load(f)
    n = ex["n"]
    A = device_matrix(grb, n, n, [(u, v, 1) for u, v in ex["edges"]], valued=False)
    for direction in (0, 1, 2):
        f_ = grb.Vector(n, torch.uint8)
        f_.set({i: True for i in ex["frontier"]})
        vis = grb.Vector(n, torch.uint8)
        vis.set({i: True for i in ex["visited"]})
        nxt = grb.Vector(n, torch.uint8)
        d = grb.descriptor(direction=direction, flags=grb.GRB_MASK_COMP | grb.GRB_REPLACE)
        grb.vxm(nxt, vis, None, "lor_land", f_, A, desc=d)
        assert sorted(nxt.to_dict()) == ex["next_frontier"]


@pytest.mark.parametrize("semiring", ["lor_land", "min_plus", "min_first", "min_second",
                                      "min_plus_fp64", "plus_times_fp64"])
def test_push_equals_pull_rmat(grb, semiring):
    """Exact semirings: the two directions agree bit for bit on an R-MAT graph
    whose hub rows exceed the pull split threshold, and match the oracle."""
    g = graphgen.rmat(13)
    rp, ci, w = grb.csr_from_edges(g.n, g.src, g.dst, g.w, symmetrise=True)
    if vec_dtype(semiring) == torch.float64:
        w = w.astype(np.float64)
    A = grb.Matrix(g.n, g.n, rp, ci, w, symmetric=True)
    assert np.diff(rp).max() > 2048
    rng = np.random.default_rng(11)
    triples = [(int(i), int(j), float(x)) for i, (s, e) in enumerate(zip(rp[:-1], rp[1:]))
               for j, x in zip(ci[s:e], w[s:e])]
    for p in (0.001, 0.05, 0.6):
        u = rand_vec(rng, g.n, p, oname(semiring))
        if semiring == "plus_times_fp64":  # small integers: every sum exact in any order
            u = {i: float(int(x) % 4) for i, x in u.items()}
        mask = {i: 1 for i in range(g.n) if rng.random() < 0.3}
        outs = []
        for direction in (1, 2, 0):
            U = grb.Vector(g.n, vec_dtype(semiring))
            U.set(u)
            Mk = grb.Vector(g.n, torch.int32)
            Mk.set(mask)
            W = grb.Vector(g.n, vec_dtype(semiring))
            grb.mxv(W, Mk, None, GRB_NAME[semiring], A, U,
                    desc=grb.descriptor(direction=direction, flags=grb.GRB_MASK_COMP))
            outs.append(W.to_dict())
        assert outs[0] == outs[1] == outs[2]
        ref = M.mxv(g.n, triples, u, semiring=oname(semiring), mask=mask, complement=True)
        assert set(outs[0]) == set(ref)
        for i in ref:
            assert float(outs[0][i]) == float(ref[i])


def _dense_vector(grb, vals, has, dtype):
    """A device vector from value and presence arrays (presence as bitmap words)."""
    n = has.shape[0]
    v = grb.Vector(n, dtype)
    npdt = {torch.uint8: np.uint8, torch.float32: np.float32, torch.int32: np.int32}[dtype]
    v.values[:n] = torch.from_numpy(np.where(has, vals, 0).astype(npdt)).to(v.values.device)
    b = np.packbits(has.astype(np.uint8), bitorder="little")
    b = np.concatenate([b, np.zeros((-len(b)) % 8, np.uint8)]).view(np.int64)
    v.bitmap[: len(b)] = torch.from_numpy(b).to(v.values.device)
    return v


@pytest.mark.parametrize("semiring", ["lor_land", "min_plus_fp32"])
def test_push_ragged_blocks(grb, semiring):
    """Forced push, pull and automatic products on a graph of 19,493
    vertices: not a multiple of the compaction block (4,096 positions) nor
    of 64, with edges into the last partial word and its last vertex in
    every input.  Complemented structural mask with REPLACE, then an
    accumulating product into an existing output without REPLACE (outputs
    outside the mask kept); element by element against the oracle."""
    import oracle
    base = graphgen.rmat(14)
    n = 16384 + 3 * 1024 + 37
    rng = np.random.default_rng(fixed_seed("ragged", semiring))
    k = 4000
    src = np.concatenate([base.src, rng.integers(16384, n, k), [n - 1]])
    dst = np.concatenate([base.dst, rng.integers(0, n, k), [0]])
    w = np.concatenate([base.w, rng.integers(1, 65, k + 1)])
    g = graphgen.from_edges("ragged", n, src, dst, w)
    A = grb.Matrix.from_raw(g)
    adj = oracle.Adjacency.from_raw(g)
    dt = torch.uint8 if semiring == "lor_land" else torch.float32
    ws = grb.workspace(grb.OP_MXV, A)
    comp = grb.GRB_MASK_COMP | grb.GRB_MASK_STRUCT
    for p in (2e-3, 0.05, 0.7):
        u_has = rng.random(n) < p
        u_has[n - 1] = True
        if semiring == "lor_land":
            u_val = (rng.random(n) >= 0.1).astype(np.float64)
        else:
            u_val = rng.integers(0, 20, n).astype(np.float64)
        m_has = rng.random(n) < 0.3
        w_has = rng.random(n) < 0.2
        w_val = np.ones(n) if semiring == "lor_land" else rng.integers(0, 30, n).astype(np.float64)
        accum = "lor" if semiring == "lor_land" else "min"
        U = _dense_vector(grb, u_val, u_has, dt)
        Mk = _dense_vector(grb, m_has.astype(np.float64), m_has, torch.uint8)
        for flags, acc in ((comp | grb.GRB_REPLACE, None), (comp, accum)):
            ref_v, ref_h = oracle.mxv_dense(
                adj, semiring, u_val, u_has, w_val=w_val if acc else None,
                w_has=w_has if acc else None, mask_val=m_has, mask_has=m_has, flags=flags,
                accum=acc)
            for direction in (1, 2, 0):
                W = (_dense_vector(grb, w_val, w_has, dt) if acc else grb.Vector(n, dt))
                grb.mxv(W, Mk, acc, semiring, A, U,
                        desc=grb.descriptor(direction=direction, flags=flags), ws=ws)
                torch.cuda.synchronize()
                words = W.bitmap.cpu().numpy().view(np.uint8)
                got_h = np.unpackbits(words, bitorder="little")[:n].astype(bool)
                case = (p, flags, direction)
                assert np.array_equal(got_h, ref_h), (case, int((got_h != ref_h).sum()))
                assert not np.unpackbits(words, bitorder="little")[n:].any(), case
                got_v = W.values[:n].cpu().numpy().astype(np.float64)
                if semiring == "lor_land":
                    assert np.array_equal(got_v[ref_h] != 0, ref_v[ref_h] != 0), case
                else:
                    assert np.array_equal(got_v[ref_h], ref_v[ref_h]), case


def test_plus_times_float_tolerance(grb):
    """Real-valued plus-times: both directions within the summation bound
    gamma_m * sum |a u| of the fp64 result; pull repeats bit for bit."""
    g = graphgen.rmat(12, symmetric=False)
    rng = np.random.default_rng(3)
    rp, ci, _ = grb.csr_from_edges(g.n, g.src, g.dst, None, symmetrise=False)
    vals = rng.standard_normal(ci.size).astype(np.float32)
    trp, tci, tv = csr(g.n, [(int(j), int(i), float(x)) for i, (s, e) in
                             enumerate(zip(rp[:-1], rp[1:])) for j, x in zip(ci[s:e], vals[s:e])])
    A = grb.Matrix(g.n, g.n, rp, ci, vals, trp, tci, tv)
    u = {i: float(rng.standard_normal()) for i in range(g.n) if rng.random() < 0.7}
    uv = np.zeros(g.n)
    for i, x in u.items():
        uv[i] = np.float32(x)
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    exact = np.zeros(g.n)
    absum = np.zeros(g.n)
    np.add.at(exact, rows, vals.astype(np.float64) * uv[ci])
    np.add.at(absum, rows, np.abs(vals.astype(np.float64) * uv[ci]))
    deg = np.diff(rp)
    gamma = deg * 2.0**-24 / (1 - deg * 2.0**-24)
    # t(i) exists iff row i has a stored entry at a present index of u
    present_u = np.zeros(g.n, bool)
    present_u[list(u)] = True
    want_has = np.zeros(g.n, bool)
    np.logical_or.at(want_has, rows, present_u[ci])
    res = []
    for direction in (1, 2, 2):
        U = grb.Vector(g.n, torch.float32)
        U.set(u)
        W = grb.Vector(g.n, torch.float32)
        grb.mxv(W, None, None, "plus_times_fp32", A, U, desc=grb.descriptor(direction=direction))
        got_has = np.zeros(g.n, bool)
        got_has[list(W.to_dict())] = True
        assert np.array_equal(got_has, want_has), direction
        res.append(W.values.cpu().numpy().astype(np.float64)[: g.n])
    for r in res:
        touched = np.flatnonzero(want_has)
        assert np.all(np.abs(r[touched] - exact[touched]) <= gamma[touched] * absum[touched]
                      + 1e-30)
    assert np.array_equal(res[1], res[2])


def test_mxv_argument_errors(grb):
    """Each argument error returns its code before anything is enqueued:
    the output's values and presence bits stay as they were."""
    n = 40
    triples = [(i, (i * 7 + 3) % n, 1.0) for i in range(n)]
    A = device_matrix(grb, n, n, triples)
    ws = grb.workspace(grb.OP_MXV, A)
    U = grb.Vector(n, torch.float32)
    U.set({1: 2.0, 5: 3.0})
    W = grb.Vector(n, torch.float32)
    W.set({0: 9.0, 7: 4.0})
    before = W.to_dict()
    fn = grb.C_FUNCTIONS["grb_mxv"]
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call(w, mask, accum, sr, a, u, desc=None, wsb=ws, nbytes=None):
        return fn(w.handle, mask.handle if mask is not None else None, accum, sr, a.handle,
                  u.handle, ctypes.byref(desc) if desc is not None else None,
                  ctypes.c_void_p(wsb.data_ptr()), wsb.numel() if nbytes is None else nbytes, s)

    sr = grb.SEMIRINGS
    W_short = grb.Vector(n - 1, torch.float32)
    W_int = grb.Vector(n, torch.int32)
    bad_desc = grb.descriptor()
    bad_desc.reserved[0] = 1
    cases = [
        ("output length", call(W_short, None, 0, sr["min_plus_fp32"], A, U), 7),
        ("output type", call(W_int, None, 0, sr["min_plus_fp32"], A, U), 6),
        ("accum not the semiring's add", call(W, None, grb.ACCUMS["plus"], sr["min_plus_fp32"],
                                               A, U), 6),
        ("input aliases output", call(W, None, 0, sr["min_plus_fp32"], A, W), 4),
        ("mask aliases output", call(W, W, 0, sr["min_plus_fp32"], A, U), 4),
        ("semiring out of range", call(W, None, 0, 99, A, U), 4),
        ("structure-only pair semiring", call(W, None, 0, sr["plus_pair_int32"], A, U), 8),
        ("descriptor reserved field", call(W, None, 0, sr["min_plus_fp32"], A, U, bad_desc), 4),
        ("workspace too small", call(W, None, 0, sr["min_plus_fp32"], A, U, nbytes=64), 9),
    ]
    for name, got, want in cases:
        assert got == want, (name, got, want)
    torch.cuda.synchronize()
    assert W.to_dict() == before
    assert fn(None, None, 0, 1, A.handle, U.handle, None, None, 0, s) == 2
    assert grb.C_FUNCTIONS["grb_stream_check"](s) == 0
