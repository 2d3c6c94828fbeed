"""GPU parity: grb_bfs / grb_sssp / grb_pagerank against the CPU oracle.

BFS levels and parents and SSSP distances (integer weights, sums < 2^24)
must match bit for bit in every direction mode; PageRank fp32 within L1
1e-5 and fp64 within L1 1e-10 of the FP64 oracle at the same iteration
count.  Inputs are seeded synthetic graphs of the paper's kinds (R-MAT with
a, b, c, d = 0.57, 0.19, 0.19, 0.05 and integer weights 1..64) plus grids and
hand-built degenerate graphs.
"""
import os

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


_CACHE = {}


def graph(name):
    """(raw graph, oracle adjacency) by name, built once per session."""
    if name in _CACHE:
        return _CACHE[name]
    if name.startswith("rmat_dir"):
        g = graphgen.rmat(int(name.split("_")[2]), symmetric=False)
    elif name.startswith("rmat"):
        g = graphgen.rmat(int(name.split("_")[1]))
    elif name.startswith("grid"):
        r, c = name.split("_")[1].split("x")
        g = graphgen.grid(int(r), int(c))
    elif name == "path":
        k = 300
        g = graphgen.from_edges(name, k, np.arange(k - 1), np.arange(1, k),
                                np.full(k - 1, 3.0))
    elif name == "star":  # one row far longer than the split threshold
        k = 5001
        g = graphgen.from_edges(name, k, np.zeros(k - 1), np.arange(1, k),
                                1 + np.arange(k - 1) % 64)
    elif name == "clique":
        iu = np.triu_indices(70, 1)
        g = graphgen.from_edges(name, 70, iu[0], iu[1], 1 + (iu[0] + iu[1]) % 64)
    elif name == "two_comp":
        src = [0, 1, 2, 3, 10, 11, 12, 130]
        dst = [1, 2, 3, 0, 11, 12, 13, 131]
        g = graphgen.from_edges(name, 133, src, dst, [5, 1, 2, 9, 1, 1, 1, 4])
    elif name == "lowdeg":
        # random sparse graph (max degree far below the one-workgroup loop's
        # limit) whose frontier outgrows that loop's lists after a few levels
        k = 120000
        rng = np.random.default_rng(21)
        src = rng.integers(0, k, 3 * k)
        dst = rng.integers(0, k, 3 * k)
        g = graphgen.from_edges(name, k, src, dst, 1 + (src * 7 + dst) % 64)
    elif name == "empty":
        g = graphgen.from_edges(name, 70, [], [], [])
    elif name == "single":
        g = graphgen.from_edges(name, 1, [], [], [])
    else:
        raise KeyError(name)
    adj = oracle.Adjacency.from_raw(g)
    _CACHE[name] = (g, adj)
    return _CACHE[name]


_MATS = {}


def matrix(grb, name):
    if name not in _MATS:
        g, _ = graph(name)
        _MATS[name] = grb.Matrix.from_raw(g)
    return _MATS[name]


MODES = [("auto_paper", 0, 0), ("auto_exact", 0, 1), ("push", 1, 0), ("pull", 2, 0)]
SMALL = ["rmat_14", "rmat_18", "rmat_dir_12", "grid_33x70", "path", "star", "clique",
         "two_comp", "empty", "single", "lowdeg"]


def _sources(name, n):
    if name == "two_comp":
        return [0, 10, 132]  # 132 is isolated
    if name in ("empty", "single"):
        return [0]
    rng = np.random.default_rng(7)
    return [0] + rng.integers(0, n, 2).tolist()


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("mode", MODES, ids=[m[0] for m in MODES])
def test_bfs_parity(grb, name, mode):
    g, adj = graph(name)
    A = matrix(grb, name)
    _, direction, rule = mode
    for s in _sources(name, g.n):
        d = grb.descriptor(direction=direction, rule=rule)
        lev, par = grb.bfs(A, s, desc=d)
        ref_lev, ref_par, nl = oracle.bfs(adj, s)
        assert np.array_equal(lev.cpu().numpy(), ref_lev), (name, s)
        assert np.array_equal(par.cpu().numpy(), ref_par), (name, s)
        st = grb.last_stats()
        assert st["iterations"] == nl
        if direction:
            assert set(st["direction"]) <= {direction}


@pytest.mark.parametrize("name", ["rmat_14", "rmat_dir_12", "grid_33x70"])
def test_bfs_direction_sequence_and_work(grb, name):
    """Per level: frontier size, its degree sum and the direction the paper's
    rule picks (pull iff 10 |f| > n) follow from the oracle's levels."""
    g, adj = graph(name)
    A = matrix(grb, name)
    off, _, _ = adj.arrays(weights=False)
    deg = np.diff(off)
    ref_lev, _, nl = oracle.bfs(adj, 0, parents=False)
    for rule in (0, 1):
        grb.bfs(A, 0, parents=False, desc=grb.descriptor(rule=rule))
        st = grb.last_stats()
        assert st["iterations"] == nl
        for d in range(nl):
            f = np.flatnonzero(ref_lev == d)
            assert st["frontier"][d] == f.size
            assert st["edges"][d] == deg[f].sum()
            pull = (10 * f.size > g.n) if rule == 0 else (10 * deg[f].sum() > adj.nnz)
            assert st["direction"][d] == (2 if pull else 1), (rule, d)


def test_bfs_level_cap_low_degree(grb):
    """A level cap inside the multi-workgroup loop (grid) and after it handed
    the frontier to the level kernel (lowdeg): levels up to the cap, parents
    of every reached vertex by the min-id rule."""
    for name, caps in (("grid_33x70", (1, 5, 40)), ("lowdeg", (3, 8, 9))):
        g, adj = graph(name)
        A = matrix(grb, name)
        ref_lev, ref_par, nl = oracle.bfs(adj, 0)
        for cap in caps:
            lev, par = grb.bfs(A, 0, desc=grb.descriptor(max_iter=cap))
            want = np.where(ref_lev <= cap, ref_lev, -1)
            assert np.array_equal(lev.cpu().numpy(), want), (name, cap)
            wpar = np.where(ref_lev <= cap, ref_par, -1)
            assert np.array_equal(par.cpu().numpy(), wpar), (name, cap)


def test_bfs_first_batch_follows_last_depth(grb):
    """The number of level launches queued before the first read-back is the
    random-graph estimate ceil(ln n / ln(nnz / n)) + 1, raised to the depth
    of the last search on the same matrix (at most twice the estimate).  A
    deep search followed by shallow ones still gives the oracle's levels
    and parents; the extra launches find an empty frontier."""
    import math
    name = "rmat_14"
    g, adj = graph(name)
    A = matrix(grb, name)
    est = min(64, math.ceil(math.log(g.n) / math.log(adj.nnz / g.n)) + 1)
    off, _, _ = adj.arrays(weights=False)
    deg = np.diff(off)
    # the deepest of a few sources of degree 1
    cands = np.flatnonzero(deg == 1)[:40]
    depths = [oracle.bfs(adj, int(v), parents=False)[2] for v in cands]
    deep = int(cands[int(np.argmax(depths))])
    prev = None
    for s in (deep, 0, 0, deep):
        lev, par = grb.bfs(A, s)
        ref_lev, ref_par, nl = oracle.bfs(adj, s)
        assert np.array_equal(lev.cpu().numpy(), ref_lev), s
        assert np.array_equal(par.cpu().numpy(), ref_par), s
        st = grb.last_stats()
        assert st["iterations"] == nl
        if prev is not None:
            first = max(est, min(prev, 2 * est))
            if nl <= first:  # one batch: every queued launch ran
                assert st["launches"] == first, (s, prev, nl)
        prev = nl


@pytest.mark.parametrize("name", ["grid_33x70", "path", "lowdeg", "two_comp"])
def test_bfs_loop_barrier_given_up(grb, name):
    """The multi-workgroup level loop's failure path, forced from the host
    (GRB_LOOP_NO_WAIT: every barrier is given up at its first unfinished
    poll, as when some of its workgroups are not resident): the search
    continues in the level kernels and gives the oracle's levels and parents."""
    g, adj = graph(name)
    A = matrix(grb, name)
    for s in _sources(name, g.n):
        ref_lev, ref_par, nl = oracle.bfs(adj, s)
        for cap in (0, 2, 7):
            lev, par = grb.bfs(A, s, desc=grb.descriptor(flags=grb.GRB_LOOP_NO_WAIT,
                                                         max_iter=cap))
            want = ref_lev if cap == 0 else np.where(ref_lev <= cap, ref_lev, -1)
            wpar = ref_par if cap == 0 else np.where(ref_lev <= cap, ref_par, -1)
            assert np.array_equal(lev.cpu().numpy(), want), (name, s, cap)
            assert np.array_equal(par.cpu().numpy(), wpar), (name, s, cap)
            if cap == 0:
                assert grb.last_stats()["iterations"] == nl


@pytest.mark.parametrize("name", ["rmat_14", "grid_33x70", "star"])
def test_bfs_repeatable(grb, name):
    A = matrix(grb, name)
    a = [t.cpu().numpy() for t in grb.bfs(A, 0)]
    b = [t.cpu().numpy() for t in grb.bfs(A, 0)]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


SSSP_GRAPHS = ["rmat_14", "rmat_18", "rmat_dir_12", "grid_33x70", "path", "star", "clique",
               "two_comp", "empty", "single", "lowdeg"]


@pytest.mark.parametrize("name", SSSP_GRAPHS)
@pytest.mark.parametrize("mode", MODES, ids=[m[0] for m in MODES])
def test_sssp_parity(grb, name, mode):
    g, adj = graph(name)
    A = matrix(grb, name)
    _, direction, rule = mode
    for s in _sources(name, g.n):
        dist = grb.sssp(A, s, desc=grb.descriptor(direction=direction, rule=rule))
        ref, _, _ = oracle.sssp(adj, s)
        assert np.array_equal(dist.cpu().numpy(), ref), (name, s)


def test_sssp_pull_modes(grb):
    """A forced-pull SSSP whose rounds span the three pull forms (chosen by
    the share of edges leaving the frontier: below 1/32 member-only weight
    loads, below 1/4 a frontier-bit test before the distance gather, else a
    gather per edge) reaches the oracle's distances."""
    g, adj = graph("rmat_14")
    A = matrix(grb, "rmat_14")
    dist = grb.sssp(A, 0, desc=grb.descriptor(direction=grb.DIR_PULL, flags=grb.GRB_PROFILE))
    st = grb.last_stats()
    ref, _, _ = oracle.sssp(adj, 0)
    assert np.array_equal(dist.cpu().numpy(), ref)
    assert all(d == grb.DIR_PULL for d in st["direction"])
    share = [e / A.nnz for e in st["edges"]]
    assert any(x < 1 / 32 for x in share), share
    assert any(1 / 32 <= x < 1 / 4 for x in share), share
    assert any(x >= 1 / 4 for x in share), share


@pytest.mark.parametrize("name", SSSP_GRAPHS)
@pytest.mark.parametrize("delta", [1.0, 7.5, 64.0, 1e6])
def test_sssp_delta_parity(grb, name, delta):
    # bucketed rounds reach the same exact distances for any bucket width
    g, adj = graph(name)
    A = matrix(grb, name)
    for s in _sources(name, g.n):
        dist = grb.sssp(A, s, delta=delta)
        ref, _, _ = oracle.sssp(adj, s)
        assert np.array_equal(dist.cpu().numpy(), ref), (name, s, delta)


def test_sssp_delta_round_cap_low_degree(grb):
    """A round cap inside the multi-workgroup loop (grid) and after it handed
    the pending set to the round kernel (lowdeg): the capped distances are
    never below the exact ones and run to them with enough rounds, and the
    round records agree with the rounds run."""
    for name, caps in (("grid_33x70", (3, 40)), ("lowdeg", (4, 30))):
        g, adj = graph(name)
        A = matrix(grb, name)
        ref, _, _ = oracle.sssp(adj, 0)
        for delta in (7.5, 256.0):
            for cap in caps:
                dist = grb.sssp(A, 0, delta=delta, desc=grb.descriptor(max_iter=cap))
                got = dist.cpu().numpy()
                assert np.all(got >= ref), (name, delta, cap)
                st = grb.last_stats()
                assert st["iterations"] <= cap
            full = grb.sssp(A, 0, delta=delta).cpu().numpy()
            assert np.array_equal(full, ref), (name, delta)


@pytest.mark.parametrize("name", ["grid_33x70", "path", "lowdeg", "two_comp"])
def test_sssp_delta_loop_barrier_given_up(grb, name):
    """The multi-workgroup bucket-round loop's failure path, forced from the
    host (GRB_LOOP_NO_WAIT): the pending set goes to the round kernel at the
    first barrier and the distances are the oracle's."""
    g, adj = graph(name)
    A = matrix(grb, name)
    for s in _sources(name, g.n):
        ref, _, _ = oracle.sssp(adj, s)
        for delta in (7.5, 256.0):
            dist = grb.sssp(A, s, delta=delta,
                            desc=grb.descriptor(flags=grb.GRB_LOOP_NO_WAIT))
            assert np.array_equal(dist.cpu().numpy(), ref), (name, s, delta)


def test_sssp_negative_weights_rejected(grb):
    g = graphgen.from_edges("neg", 4, [0, 1, 2], [1, 2, 3], [1.0, -2.0, 3.0])
    A = grb.Matrix.from_raw(g)
    with pytest.raises(grb.GrbError) as e:
        grb.sssp(A, 0)
    assert e.value.code == 4
    with pytest.raises(grb.GrbError) as e:
        grb.sssp(A, 0, delta=2.0)
    assert e.value.code == 4


def test_sssp_delta_argument_errors(grb):
    A = matrix(grb, "rmat_14")
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(grb.GrbError):
            grb.sssp(A, 0, delta=bad)
    with pytest.raises(grb.GrbError):
        grb.sssp(A, 0, delta=64.0, desc=grb.descriptor(direction=grb.DIR_PULL))


@pytest.mark.parametrize("name", ["rmat_dir_12", "rmat_dir_14"])
def test_pagerank_parity(grb, name):
    g, adj = graph(name)
    A = matrix(grb, name)
    ref, it, delta = oracle.pagerank(adj, 0.85, 50, 1e-7)
    p32, it32, d32 = grb.pagerank(A, dtype=torch.float32, max_iter=it, tol=0.0)
    p64, it64, d64 = grb.pagerank(A, dtype=torch.float64, max_iter=it, tol=0.0)
    assert it32 == it and it64 == it
    assert np.abs(p32.cpu().numpy().astype(np.float64) - ref).sum() <= 1e-5
    assert np.abs(p64.cpu().numpy() - ref).sum() <= 1e-10
    # the device-side stopping rule stops where the oracle stops
    _, it_auto, _ = grb.pagerank(A, dtype=torch.float64, max_iter=50, tol=1e-7)
    assert it_auto == it
    # bitwise repeatable
    q32, _, _ = grb.pagerank(A, dtype=torch.float32, max_iter=it, tol=0.0)
    assert torch.equal(p32, q32)


def _adaptive_schedule(adj, fz, it):
    """per iteration j = 1..it: (vertices active entering it, their in-edges,
    vertices active after it), from the oracle's freeze iterations"""
    _, nbr, _ = adj.arrays(weights=False)
    indeg = np.bincount(nbr, minlength=adj.n)
    rows = []
    for j in range(1, it + 1):
        live = (fz == 0) | (fz >= j)
        after = (fz == 0) | (fz > j)
        rows.append((int(live.sum()), int(indeg[live].sum()), int(after.sum())))
    return rows


def _directed_star():
    star = graph("star")[0]
    g = graphgen.from_edges("dstar", star.n, star.src, star.dst, symmetric=False)
    return g, oracle.Adjacency(star.n, star.src, star.dst, symmetrise=False)


@pytest.mark.parametrize("name", ["rmat_dir_12", "rmat_dir_14", "star_dir"])
@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_pagerank_adaptive_parity(grb, name, eps):
    if name == "star_dir":  # in-rows far longer than the piece size
        g, adj = _directed_star()
        A = grb.Matrix.from_raw(g, weights=False)
    else:
        g, adj = graph(name)
        A = matrix(grb, name)
    ref, it, delta, active, fz = oracle.pagerank_adaptive(adj, eps, 0.85, 50, 1e-7)
    p64, it64, d64, a64 = grb.pagerank_adaptive(A, eps, dtype=torch.float64, max_iter=it,
                                                tol=0.0)
    st = grb.last_stats()
    p32, it32, d32, a32 = grb.pagerank_adaptive(A, eps, dtype=torch.float32, max_iter=it,
                                                tol=0.0)
    assert it64 == it and a64 == active
    assert np.abs(p64.cpu().numpy() - ref).sum() <= 1e-10
    assert np.abs(p32.cpu().numpy().astype(np.float64) - ref).sum() <= 1e-5
    # per iteration: active rows, their in-edges, active after (fp64 run)
    sched = _adaptive_schedule(adj, fz, it)
    assert st["iterations"] == it
    assert [(f, e) for f, e, _ in sched] == list(zip(st["frontier"], st["edges"]))
    assert all(d == 2 for d in st["direction"])
    # the device-side stopping rule stops where the oracle stops
    _, it_auto, _, a_auto = grb.pagerank_adaptive(A, eps, dtype=torch.float64, max_iter=50,
                                                  tol=1e-7)
    assert it_auto == it and a_auto == active
    # bitwise repeatable
    q32, _, _, _ = grb.pagerank_adaptive(A, eps, dtype=torch.float32, max_iter=it, tol=0.0)
    assert torch.equal(p32, q32)


def test_pagerank_adaptive_edge_cases(grb):
    n = 9
    cyc = graphgen.from_edges("cyc", n, np.arange(n), (np.arange(n) + 1) % n, symmetric=False)
    A = grb.Matrix.from_raw(cyc, weights=False)
    for dt in (torch.float32, torch.float64):
        p, it, delta, active = grb.pagerank_adaptive(A, 1e-6, dtype=dt, max_iter=50, tol=0.0)
        assert it == 1 and active == 0
        assert np.allclose(p.cpu().numpy(), 1 / n, atol=1e-7)
    # eps = 0 on a graph that never stands still: every iteration is plain PageRank
    g, adj = graph("rmat_dir_12")
    B = matrix(grb, "rmat_dir_12")
    ref, it, _ = oracle.pagerank(adj, 0.85, 6, 0.0)
    p, it2, _, active = grb.pagerank_adaptive(B, 0.0, dtype=torch.float64, max_iter=6, tol=0.0)
    _, _, _, oact, _ = oracle.pagerank_adaptive(adj, 0.0, 0.85, 6, 0.0)
    assert it2 == 6 and active == oact
    if oact == adj.n:
        assert np.abs(p.cpu().numpy() - ref).sum() <= 1e-12
    # max_iter = 0: no iteration, p = 1/n
    p, it3, _, active = grb.pagerank_adaptive(B, 1e-3, dtype=torch.float64, max_iter=0)
    assert it3 == 0 and active == adj.n
    assert np.allclose(p.cpu().numpy(), 1 / adj.n, atol=1e-18)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(grb.GrbError):
            grb.pagerank_adaptive(B, bad)


def test_pagerank_closed_forms(grb):
    n = 9
    cyc = graphgen.from_edges("cyc", n, np.arange(n), (np.arange(n) + 1) % n, symmetric=False)
    A = grb.Matrix.from_raw(cyc, weights=False)
    p, it, delta = grb.pagerank(A, dtype=torch.float64, max_iter=50, tol=1e-7)
    assert it == 1 and np.allclose(p.cpu().numpy(), 1 / n, atol=1e-15)
    star = graph("star")[0]
    S = grb.Matrix.from_raw(graphgen.from_edges("st", star.n, star.src, star.dst,
                                                symmetric=False), weights=False)
    adj = oracle.Adjacency(star.n, star.src, star.dst, symmetrise=False)
    ref, it, _ = oracle.pagerank(adj, 0.85, 50, 1e-7)
    p, it2, _ = grb.pagerank(S, dtype=torch.float64, max_iter=50, tol=1e-7)
    assert it2 == it
    assert np.abs(p.cpu().numpy() - ref).sum() <= 1e-10


def test_package_imported_before_torch():
    """Importing the package before torch leaves torch's kernels working
    (the package loads torch before its library, so both share torch's HIP
    runtime); a fresh process, BFS levels checked against the oracle."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import paper_1908_01407_amd as grb, graphgen, oracle, numpy as np, torch\n"
            "g = graphgen.rmat(10)\n"
            "lev, par = grb.bfs(grb.Matrix.from_raw(g), 0)\n"
            "ref = oracle.bfs(oracle.Adjacency.from_raw(g), 0)[0]\n"
            "x = torch.arange(8, device='cuda').sum().item()\n"
            "assert np.array_equal(lev.cpu().numpy(), ref) and x == 28\n"
            "print('ok')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=100)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-3000:]


def test_loops_concurrent_streams(grb):
    """Device-side level loops of several searches at once: two host threads,
    each with its own stream and workspace, run BFS and bucketed SSSP on a
    grid (hundreds of levels, so the loops' kernels overlap on the device);
    every result equals the oracle's."""
    import threading

    g = graphgen.grid(300, 300)
    adj = oracle.Adjacency.from_raw(g)
    A = grb.Matrix.from_raw(g)
    torch.cuda.synchronize()
    ref_lev, ref_par, _ = oracle.bfs(adj, 0)
    ref_d, _, _ = oracle.sssp(adj, 0)
    errors = []

    def work(seed):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                wsb = grb.workspace(grb.OP_BFS, A)
                wss = grb.workspace(grb.OP_SSSP, A)
                for i in range(3):
                    if (i + seed) % 2 == 0:
                        lev, par = grb.bfs(A, 0, ws=wsb, stream=s)
                        s.synchronize()
                        if not (np.array_equal(lev.cpu().numpy(), ref_lev)
                                and np.array_equal(par.cpu().numpy(), ref_par)):
                            errors.append(("bfs", seed, i))
                    else:
                        dist = grb.sssp(A, 0, delta=64.0, ws=wss, stream=s)
                        s.synchronize()
                        if not np.array_equal(dist.cpu().numpy(), ref_d):
                            errors.append(("sssp", seed, i))
        except Exception as e:  # reported below
            errors.append(("exception", seed, repr(e)))

    threads = [threading.Thread(target=work, args=(t,)) for t in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
