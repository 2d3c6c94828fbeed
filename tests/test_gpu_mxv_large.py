"""Pull and automatic grb_mxv on R-MAT 18 and 20 (262,144 and 1,048,576
columns, long rows cut into pieces), element by element against the
oracle's dense-array product: sparse inputs, clustered runs with every
other column absent, and a dense input; OR, min-plus (fp32, fp64) and
min-select semirings, with and without a complemented structural mask."""
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


@pytest.fixture(scope="module", params=[18, 20], ids=["rmat18", "rmat20"])
def graph(grb, request):
    g = graphgen.rmat(request.param)
    return grb.Matrix.from_raw(g), oracle.Adjacency.from_raw(g)


SEMIRINGS = {"lor_land": torch.uint8, "min_plus_fp32": torch.float32,
             "min_plus_fp64": torch.float64, "min_second_int32": torch.int32}


def _words(bits):
    b = np.packbits(bits.astype(np.uint8), bitorder="little")
    b = np.concatenate([b, np.zeros((-len(b)) % 8, np.uint8)])
    return b.view(np.int64)


def _vector(grb, vals, has, dtype):
    n = has.shape[0]
    v = grb.Vector(n, dtype)
    v.values[:n] = torch.from_numpy(np.where(has, vals, 0).astype(
        {torch.uint8: np.uint8, torch.float32: np.float32, torch.float64: np.float64,
         torch.int32: np.int32}[dtype])).to(v.values.device)
    w = _words(has)
    v.bitmap[: len(w)] = torch.from_numpy(w).to(v.values.device)
    return v


def _input(kind, n, rng):
    if kind == "sparse":
        has = rng.random(n) < 1e-3
    elif kind == "clustered":
        has = np.zeros(n, bool)
        for s in rng.integers(0, n - 100, 40):
            has[s: s + 100: 2] = True
    else:
        has = rng.random(n) < 0.6
    return has


@pytest.mark.parametrize("kind", ["sparse", "clustered", "dense"])
@pytest.mark.parametrize("semiring", list(SEMIRINGS))
def test_pull_large_inputs(grb, graph, semiring, kind):
    A, adj = graph
    n = A.nrows
    rng = np.random.default_rng(n + len(kind) * 31 + len(semiring))
    u_has = _input(kind, n, rng)
    if semiring == "lor_land":
        u_val = (rng.random(n) >= 0.1).astype(np.float64)
    else:
        u_val = rng.integers(0, 20, n).astype(np.float64)
    m_has = rng.random(n) < 0.3
    dt = SEMIRINGS[semiring]
    U = _vector(grb, u_val, u_has, dt)
    ws = grb.workspace(grb.OP_MXV, A)
    for masked in (False, True):
        flags = grb.GRB_MASK_COMP | grb.GRB_MASK_STRUCT if masked else 0
        ref_v, ref_h = oracle.mxv_dense(adj, semiring, u_val, u_has,
                                        mask_val=m_has if masked else None,
                                        mask_has=m_has if masked else None, flags=flags)
        Mk = _vector(grb, m_has.astype(np.float64), m_has, torch.uint8) if masked else None
        for direction in (2, 0):
            W = grb.Vector(n, dt)
            grb.mxv(W, Mk, None, semiring, A, U,
                    desc=grb.descriptor(direction=direction, flags=flags), ws=ws)
            torch.cuda.synchronize()
            words = W.bitmap.cpu().numpy().view(np.uint8)
            got_h = np.unpackbits(words, bitorder="little")[:n].astype(bool)
            assert np.array_equal(got_h, ref_h), (direction, masked,
                                                  int((got_h != ref_h).sum()))
            got_v = W.values[:n].cpu().numpy().astype(np.float64)
            if semiring == "lor_land":
                assert np.array_equal(got_v[ref_h] != 0, ref_v[ref_h] != 0), (direction, masked)
            else:
                assert np.array_equal(got_v[ref_h], ref_v[ref_h]), (direction, masked)
