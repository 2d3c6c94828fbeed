"""GPU serving: queries admitted into concurrent slots with batching on
arrival return exactly what each query returns alone (BFS levels equal
single-source BFS, SSSP distances bitwise equal), and match the oracle."""
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


def test_results_same_alone_and_in_mix(grb):
    from paper_1908_01407_amd.serve import GpuExecutor, Query, Server

    raws = {"r12": graphgen.rmat(12), "r14": graphgen.rmat(14), "g60": graphgen.grid(60, 60)}
    graphs = {k: grb.Matrix.from_raw(g) for k, g in raws.items()}
    adjs = {k: oracle.Adjacency.from_raw(g) for k, g in raws.items()}
    names = sorted(raws)
    n_q = 240
    arr = graphgen.poisson_arrivals(n_q, rate=3000.0, seed=4)
    kind = graphgen.uniform_ints(n_q, 10, seed=6)
    gsel = graphgen.uniform_ints(n_q, len(names), seed=7)
    qs = []
    for i in range(n_q):
        g = names[int(gsel[i])]
        srcs = graphgen.sources(raws[g].src, raws[g].dst, raws[g].n, 1, seed=100 + i)
        qs.append(Query(qid=i, kind="bfs" if kind[i] < 7 else "sssp", graph=g,
                        source=int(srcs[0]), arrival=float(arr[i])))
    ex = GpuExecutor(graphs, slots=4, max_batch=16, sssp_delta={"g60": 64.0})
    srv = Server(ex, budget=1 << 34, slots=4, max_batch=16)
    st = srv.run(qs, realtime=True)
    assert st["failed"] == 0
    assert st["mean_batch"] > 1.0  # some BFS queries were batched on arrival
    for q in qs:
        A = graphs[q.graph]
        if q.kind == "bfs":
            alone, _ = grb.bfs(A, q.source, parents=False)
            ref, _, _ = oracle.bfs(adjs[q.graph], q.source, parents=False)
        else:
            alone = grb.sssp(A, q.source)
            ref, _, _ = oracle.sssp(adjs[q.graph], q.source)
        got = q.result.numpy()
        assert np.array_equal(got, alone.cpu().numpy()), (q.qid, q.kind, q.graph, q.batch)
        assert np.array_equal(got, ref), (q.qid, q.kind, q.graph)
