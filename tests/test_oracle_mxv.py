"""Pins for the plain-loop mxv / vxm oracle.

* the paper's running example (Figure 4 caption): one masked BFS step;
* scipy sparse products for plus-times (library routine);
* an independent dense-array formulation for every semiring, mask mode,
  accumulator, REPLACE and transpose on random tiny inputs;
* fixed points: iterating boolean vxm with the complemented visited mask
  gives the BFS levels of the queue oracle, and iterating min-plus vxm with
  accum = min gives Dijkstra's distances;
* the dense-array C loop (oracle.mxv_dense, used at full sizes) equals the
  pinned dictionary form on random tiny inputs for every semiring and flag.
"""
import json
import math
import os
import zlib

import numpy as np
import pytest
import scipy.sparse as sp

import graphgen
import oracle
from oracle import mxv as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_running_example_bfs_step():
    with open(os.path.join(GOLDEN, "running_example_bfs_step.json")) as f:
        ex = json.load(f)
    A = [(u, v, 1) for u, v in ex["edges"]]
    f_ = {i: True for i in ex["frontier"]}
    vis = {i: True for i in ex["visited"]}
    nb = M.vxm(ex["n"], A, f_, semiring="lor_land")
    assert sorted(nb) == ex["neighbours"]
    nxt = M.vxm(ex["n"], A, f_, semiring="lor_land", mask=vis, complement=True,
                replace=True)
    assert sorted(nxt) == ex["next_frontier"]
    # same result as mxv on the transposed matrix
    nxt2 = M.mxv(ex["n"], A, f_, semiring="lor_land", mask=vis, complement=True,
                 replace=True, transpose=True)
    assert nxt2 == nxt


def _rand_problem(rng, n_rows, n_cols, density=0.3):
    A = []
    for i in range(n_rows):
        for j in range(n_cols):
            if rng.random() < density:
                A.append((i, j, int(rng.integers(1, 9))))
    return A


def _rand_vec(rng, n, p, kind):
    v = {}
    for i in range(n):
        if rng.random() < p:
            if kind == "bool":
                v[i] = bool(rng.integers(0, 2))
            elif kind == "int":
                v[i] = int(rng.integers(0, 50))
            else:
                v[i] = float(rng.integers(0, 20))
    return v


def _dense_ref(n_out, A, u, semiring, w_old, mask, comp, struct, accum, replace,
               transpose, vxm):
    """Array formulation: build the full product table, reduce along axis."""
    n_in = n_out  # square test matrices
    Av = np.full((n_in, n_in), np.nan)
    for (i, j, a) in A:
        Av[i, j] = a
    if transpose:
        Av = Av.T
    if vxm:
        Av = Av.T  # w(j) = sum_i u(i) (x) A(i, j)  ==  (A^T u)(j)
    uv = np.full(n_in, np.nan)
    for j, x in u.items():
        uv[j] = float(x)
    pres = ~np.isnan(Av) & ~np.isnan(uv)[None, :]
    t_has = pres.any(axis=1)[:n_out]
    if semiring == "lor_land":
        prod = (np.nan_to_num(Av) != 0) & (np.nan_to_num(uv) != 0)[None, :]
        t = np.where(pres, prod, False).any(axis=1).astype(float)
    elif semiring == "min_plus":
        t = np.where(pres, Av + uv[None, :], np.inf).min(axis=1)
    elif semiring == "plus_times":
        t = np.where(pres, Av * uv[None, :], 0.0).sum(axis=1)
    elif semiring in ("min_first", "min_second"):
        # operand order: mxv multiplies A(i,j) (x) u(j); vxm u(i) (x) A(i,j)
        first_is_matrix = not vxm
        pick_matrix = (semiring == "min_first") == first_is_matrix
        val = np.broadcast_to(Av if pick_matrix else uv[None, :], Av.shape)
        t = np.where(pres, val, np.inf).min(axis=1)
    t = t[:n_out]
    old_has = np.array([i in w_old for i in range(n_out)])
    old = np.array([float(w_old.get(i, 0)) for i in range(n_out)])
    if accum is None:
        z_has, z = t_has, t
    else:
        op = {"min": np.minimum, "plus": np.add, "lor": np.logical_or}[accum]
        both = t_has & old_has
        z = np.where(both, op(old, t), np.where(t_has, t, old)).astype(float)
        z_has = t_has | old_has
    if mask is None:
        allowed = np.ones(n_out, bool)
    else:
        present = np.array([i in mask for i in range(n_out)])
        nz = np.array([i in mask and mask[i] != 0 for i in range(n_out)])
        allowed = (present if struct else nz) != comp
    out = {}
    for i in range(n_out):
        if allowed[i]:
            if z_has[i]:
                out[i] = z[i]
        elif not replace and old_has[i]:
            out[i] = old[i]
    return out


SEMI_KIND = {"lor_land": "bool", "min_plus": "float", "plus_times": "float",
             "min_first": "int", "min_second": "int"}
SEMI_ACCUM = {"lor_land": [None, "lor"], "min_plus": [None, "min"],
              "plus_times": [None, "plus"], "min_first": [None, "min"],
              "min_second": [None, "min"]}


@pytest.mark.parametrize("semiring", list(SEMI_KIND))
@pytest.mark.parametrize("vxm", [False, True])
def test_mxv_against_dense_formulation(semiring, vxm):
    rng = np.random.default_rng(zlib.crc32(repr((semiring, vxm)).encode()))
    fn = M.vxm if vxm else M.mxv
    for trial in range(40):
        n = int(rng.integers(1, 9))
        A = _rand_problem(rng, n, n, density=float(rng.uniform(0.05, 0.6)))
        kind = SEMI_KIND[semiring]
        u = _rand_vec(rng, n, float(rng.uniform(0, 1)), kind)
        w_old = _rand_vec(rng, n, 0.5, kind)
        mask = None if trial % 4 == 0 else _rand_vec(rng, n, 0.6, "int")
        comp = bool(trial % 3 == 1)
        struct = bool(trial % 5 == 2)
        accum = SEMI_ACCUM[semiring][trial % 2]
        replace = bool(trial % 7 < 3)
        transpose = bool(trial % 6 >= 3)
        got = fn(n, A, u, semiring=semiring, w_old=w_old, mask=mask, complement=comp,
                 structural=struct, accum=accum, replace=replace, transpose=transpose)
        ref = _dense_ref(n, A, u, semiring, w_old, mask, comp, struct, accum, replace,
                         transpose, vxm)
        assert set(got) == set(ref), (trial, got, ref)
        for i in got:
            assert float(got[i]) == ref[i], (trial, i, got[i], ref[i])


def test_plus_times_matches_scipy():
    rng = np.random.default_rng(5)
    n = 30
    A = _rand_problem(rng, n, n, 0.2)
    u = {j: float(rng.standard_normal()) for j in range(n) if rng.random() < 0.7}
    rows, cols, vals = zip(*A)
    S = sp.csr_matrix((np.array(vals, float), (rows, cols)), shape=(n, n))
    uv = np.zeros(n)
    for j, x in u.items():
        uv[j] = x
    got = M.mxv(n, A, u, semiring="plus_times")
    ref = S @ uv
    touched = set(np.flatnonzero(abs(S) @ (uv != 0)))
    assert set(got) == touched
    for i in got:
        assert math.isclose(got[i], ref[i], rel_tol=1e-12, abs_tol=1e-12)
    got_t = M.vxm(n, A, u, semiring="plus_times")
    ref_t = S.T @ uv
    for i in got_t:
        assert math.isclose(got_t[i], ref_t[i], rel_tol=1e-12, abs_tol=1e-12)


def test_iterated_vxm_gives_bfs_and_sssp():
    g = graphgen.rmat(7)
    adj = oracle.Adjacency.from_raw(g)
    off, nbr, w = adj.arrays()
    A_bool = [(u, int(v), 1) for u in range(g.n) for v in nbr[off[u]:off[u + 1]]]
    A_w = [(u, int(v), float(x)) for u in range(g.n)
           for v, x in zip(nbr[off[u]:off[u + 1]], w[off[u]:off[u + 1]])]
    s = 0
    # BFS: f <- f A .* not(visited)
    lev = {s: 0}
    f = {s: True}
    d = 0
    while f:
        d += 1
        f = M.vxm(g.n, A_bool, f, semiring="lor_land", mask=dict.fromkeys(lev, 1),
                  complement=True, replace=True)
        for v in f:
            lev[v] = d
    ref, _, _ = oracle.bfs(adj, s, parents=False)
    got = np.full(g.n, -1)
    for v, l in lev.items():
        got[v] = l
    assert np.array_equal(got, ref)
    # Bellman-Ford: dist <- min(dist, dist A) until nothing changes
    dist = {s: 0.0}
    while True:
        new = M.vxm(g.n, A_w, dist, semiring="min_plus", w_old=dist, accum="min")
        if new == dist:
            break
        dist = new
    d32, _, _ = oracle.sssp(adj, s)
    got = np.full(g.n, np.inf, dtype=np.float32)
    for v, x in dist.items():
        got[v] = x
    assert np.array_equal(got, d32)


DENSE_NAME = {"lor_land": "lor_land", "min_plus": "min_plus_fp64",
              "plus_times": "plus_times_fp64", "min_first": "min_first_int32",
              "min_second": "min_second_int32"}


@pytest.mark.parametrize("semiring", list(SEMI_KIND))
@pytest.mark.parametrize("vxm", [False, True])
def test_dense_c_loop_matches_dictionary_form(semiring, vxm):
    """oracle.mxv_dense (C, dense arrays) against the pinned dictionary
    oracle, every mask mode, accum, REPLACE and transpose; matrices without
    self-loops (the adjacency builder drops them), values 0 allowed for the
    Boolean semiring (false entries)."""
    rng = np.random.default_rng(zlib.crc32(repr(("dense", semiring, vxm)).encode()))
    kind = SEMI_KIND[semiring]
    for trial in range(40):
        n = int(rng.integers(1, 24))
        A = [(i, j, (int(rng.integers(0, 3)) if kind == "bool" else int(rng.integers(1, 9))))
             for i in range(n) for j in range(n) if i != j and rng.random() < 0.3]
        u = _rand_vec(rng, n, float(rng.uniform(0, 1)), kind)
        w_old = _rand_vec(rng, n, 0.5, kind)
        mask = None if trial % 4 == 0 else _rand_vec(rng, n, 0.6, "int")
        comp, struct = trial % 3 == 1, trial % 5 == 2
        accum = SEMI_ACCUM[semiring][trial % 2]
        replace, transpose = trial % 7 < 3, trial % 6 >= 3
        fn = M.vxm if vxm else M.mxv
        ref = fn(n, A, u, semiring=semiring, w_old=w_old, mask=mask, complement=comp,
                 structural=struct, accum=accum, replace=replace, transpose=transpose)
        src = np.array([t[0] for t in A], np.int32)
        dst = np.array([t[1] for t in A], np.int32)
        wts = np.array([t[2] for t in A], np.float32)
        adj = oracle.Adjacency(n, src, dst, wts, symmetrise=False)
        # rows of the operand: mxv reads A (A^T when transposed), vxm reads A^T (A)
        rows = adj if vxm == transpose else adj.transpose()

        def dense(d):
            v, h = np.zeros(n), np.zeros(n, bool)
            for i, x in d.items():
                v[i], h[i] = float(x), True
            return v, h

        uv, uh = dense(u)
        wv, wh = dense(w_old)
        mv, mh = dense(mask) if mask is not None else (None, None)
        flags = ((oracle.MXV_COMP if comp else 0) | (oracle.MXV_STRUCT if struct else 0) |
                 (oracle.MXV_REPLACE if replace else 0))
        val, has = oracle.mxv_dense(rows, DENSE_NAME[semiring], uv, uh, vec_first=vxm,
                                    w_val=wv, w_has=wh, mask_val=mv, mask_has=mh, flags=flags,
                                    accum=accum)
        assert set(np.flatnonzero(has)) == set(ref), (trial, sorted(ref))
        for i in ref:
            assert val[i] == float(ref[i]), (trial, i, val[i], ref[i])
