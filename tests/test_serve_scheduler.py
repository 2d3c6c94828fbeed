"""Serving scheduler on the CPU with a fake executor: admission under the
memory budget, slot limit, FIFO head, batching on arrival, slot reuse,
error isolation and oversized queries."""
import threading

import pytest

import graphgen
from paper_1908_01407_amd.serve import FakeExecutor, Query, Scheduler, Server


def mk(qid, kind, graph, t=0.0, src=0):
    return Query(qid=qid, kind=kind, graph=graph, source=src, arrival=t)


def test_fifo_head_and_batching():
    s = Scheduler(lambda k, g, b: 10 * b, budget=1000, slots=4, max_batch=3)
    qs = [mk(0, "bfs", "a"), mk(1, "sssp", "a"), mk(2, "bfs", "b"), mk(3, "bfs", "a"),
          mk(4, "bfs", "a"), mk(5, "bfs", "a")]
    for q in qs:
        s.submit(q)
    it = s.next_item()
    assert [q.qid for q in it.queries] == [0, 3, 4]  # head + later BFS on graph a, max 3
    it2 = s.next_item()
    assert [q.qid for q in it2.queries] == [1]       # SSSP alone
    it3 = s.next_item()
    assert [q.qid for q in it3.queries] == [2]
    it4 = s.next_item()
    assert [q.qid for q in it4.queries] == [5]
    assert s.next_item() is None                     # slots exhausted (4 running)
    s.release(it)
    assert s.next_item() is None                     # nothing waiting
    for it_ in (it2, it3, it4):
        s.release(it_)
    assert s.idle()


def test_budget_shrinks_batch_and_blocks():
    s = Scheduler(lambda k, g, b: 100 * b, budget=250, slots=8, max_batch=8)
    for i in range(6):
        s.submit(mk(i, "bfs", "a"))
    it = s.next_item()
    assert len(it.queries) == 2 and s.used == 200    # shrunk to fit 250
    assert s.next_item() is None                     # 50 left: even one query (100) waits
    s.release(it)
    it = s.next_item()
    assert len(it.queries) == 2


def test_oversized_query_fails_instead_of_blocking():
    s = Scheduler(lambda k, g, b: 10**9, budget=100, slots=2)
    s.submit(mk(0, "sssp", "huge"))
    it = s.next_item()
    assert it.queries[0].error and it.footprint == 0
    s.release(it)
    assert s.idle()


def test_server_respects_budget_and_slots():
    ex = FakeExecutor({"a": 10, "b": 30}, service_s=0.003)
    seen_max = [0]
    budget = 100

    class Watch(FakeExecutor):
        pass

    srv = Server(ex, budget=budget, slots=3, max_batch=4)
    orig = srv.sched.next_item

    def watched():
        it = orig()
        seen_max[0] = max(seen_max[0], srv.sched.used)
        return it

    srv.sched.next_item = watched
    arr = graphgen.poisson_arrivals(200, rate=2000.0, seed=4)
    kinds = graphgen.uniform_ints(200, 10, seed=5)
    qs = [mk(i, "bfs" if kinds[i] < 7 else "sssp", "a" if i % 3 else "b", float(arr[i]))
          for i in range(200)]
    st = srv.run(qs, realtime=True)
    assert st["failed"] == 0 and st["queries"] == 200
    assert all(q.result == (q.kind, q.graph, q.source) for q in qs)
    assert seen_max[0] <= budget
    assert ex.max_concurrent <= 3
    assert st["mean_batch"] >= 1.0 and st["p99_ms"] >= st["p50_ms"] > 0
    assert set(st["by_graph"]) == {"a", "b"}


def test_error_isolation():
    ex = FakeExecutor({"a": 1}, service_s=0.001, fail_ids={5})
    srv = Server(ex, budget=100, slots=2, max_batch=1)
    qs = [mk(i, "bfs", "a") for i in range(12)]
    st = srv.run(qs, realtime=False)
    assert st["failed"] == 1
    assert qs[5].error and "injected" in qs[5].error
    assert all(q.error is None and q.result for q in qs if q.qid != 5)


def test_no_starvation_under_continuous_load():
    # a stream of graph-a BFS queries must not starve an SSSP on graph b
    ex = FakeExecutor({"a": 1, "b": 1}, service_s=0.001)
    srv = Server(ex, budget=1000, slots=2, max_batch=8)
    qs = [mk(i, "bfs", "a", t=0.0001 * i) for i in range(100)]
    qs.insert(10, mk(1000, "sssp", "b", t=0.00105))
    st = srv.run(qs, realtime=True)
    victim = next(q for q in qs if q.qid == 1000)
    later = [q for q in qs if q.arrival > victim.arrival + 0.002]
    assert st["failed"] == 0
    assert all(victim.start <= q.start for q in later)
