"""GPU serving: BFS queries that join running lane sessions mid-flight and
SSSP queries in concurrent slots return exactly what each query returns
alone (BFS levels equal single-source BFS, SSSP distances bitwise equal)
and match the oracle; with a budget that admits one session at a time the
memory pool never exceeds it and the results are unchanged."""
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
def graphs(grb):
    raws = {"r12": graphgen.rmat(12), "r14": graphgen.rmat(14), "g60": graphgen.grid(60, 60)}
    return (raws, {k: grb.Matrix.from_raw(g) for k, g in raws.items()},
            {k: oracle.Adjacency.from_raw(g) for k, g in raws.items()})


def trace(raws, n_q, rate, seed):
    from paper_1908_01407_amd.serve import Query
    names = sorted(raws)
    arr = graphgen.poisson_arrivals(n_q, rate=rate, seed=seed)
    kind = graphgen.uniform_ints(n_q, 10, seed=seed + 2)
    gsel = graphgen.uniform_ints(n_q, len(names), seed=seed + 3)
    qs = []
    for i in range(n_q):
        g = names[int(gsel[i])]
        srcs = graphgen.sources(raws[g].src, raws[g].dst, raws[g].n, 1, seed=100 + i)
        qs.append(Query(qid=i, kind="bfs" if kind[i] < 7 else "sssp", graph=g,
                        source=int(srcs[0]), arrival=float(arr[i])))
    return qs


def check(grb, graphs, qs):
    _, mats, adjs = graphs
    for q in qs:
        A = mats[q.graph]
        if q.kind == "bfs":
            alone, _ = grb.bfs(A, q.source, parents=False)
            ref, _, _ = oracle.bfs(adjs[q.graph], q.source, parents=False)
        else:
            alone = grb.sssp(A, q.source)
            ref, _, _ = oracle.sssp(adjs[q.graph], q.source)
        got = q.result.numpy()
        assert np.array_equal(got, alone.cpu().numpy()), (q.qid, q.kind, q.graph, q.batch,
                                                           q.joined_level)
        assert np.array_equal(got, ref), (q.qid, q.kind, q.graph)


def test_results_same_alone_and_in_mix(grb, graphs):
    from paper_1908_01407_amd.serve import GpuExecutor, Server
    raws, mats, _ = graphs
    qs = trace(raws, 240, 3000.0, 4)
    ex = GpuExecutor(mats, budget=1 << 30, slots=4, sssp_delta={"g60": 64.0})
    srv = Server(ex, slots=4, lanes=64, level_chunk={"g60": 8})
    st = srv.run(qs, realtime=True)
    assert st["failed"] == 0
    assert st["mean_batch"] > 1.0  # BFS queries shared sessions
    # some joined a session that was already past its first level
    assert any(q.joined_level > 0 for q in qs if q.kind == "bfs")
    check(grb, graphs, qs)


def test_budget_admits_one_session_at_a_time(grb, graphs):
    from paper_1908_01407_amd.serve import GpuExecutor, Server
    raws, mats, _ = graphs
    probe = GpuExecutor(mats, budget=1 << 20, slots=1)
    need = max(probe.footprint_session(g, 64) for g in mats)
    extra = max(probe.footprint_sssp(g) for g in mats)
    del probe
    budget = need + extra + 4096
    qs = trace(raws, 120, 5000.0, 14)
    ex = GpuExecutor(mats, budget=budget, slots=2, sssp_delta={"g60": 64.0})
    srv = Server(ex, slots=2, lanes=64, level_chunk={"g60": 8}, session_share=1.0)
    st = srv.run(qs, realtime=True)
    assert st["failed"] == 0
    assert st["pool_peak_bytes"] <= budget
    assert st["max_sessions"] <= 2 and st["deferred_admissions"] > 0
    check(grb, graphs, qs)
