"""Serving logic on the CPU with a fake executor: the device memory pool,
BFS queries joining running lane sessions at level boundaries and retiring
independently, admission bound by the memory budget (sessions and SSSP
queries wait, oversized work fails), error isolation, no starvation, and
the one-at-a-time FIFO mode."""
import pytest

import graphgen
from paper_1908_01407_amd.serve import DevicePool, FakeExecutor, Query, Server


def mk(qid, kind, graph, t=0.0, src=0):
    return Query(qid=qid, kind=kind, graph=graph, source=src, arrival=t)


def test_pool_first_fit_and_coalesce():
    p = DevicePool(4096, align=256)
    a = p.alloc(100)
    b = p.alloc(1000)
    c = p.alloc(256)
    assert (a, b, c) == (0, 256, 1280) and p.used == 256 + 1024 + 256
    assert p.alloc(4096) is None
    p.release(b, 1000)
    assert p.alloc(1024) == 256          # first fit reuses the hole
    p.release(256, 1024)
    p.release(a, 100)
    p.release(c, 256)
    assert p.free == [(0, 4096)] and p.used == 0   # all coalesced
    assert p.peak == 1536
    assert not p.fits_ever(5000) and p.fits_ever(4096)


def test_lanes_join_running_sessions():
    ex = FakeExecutor({"a": 10}, budget=1000, level_s=0.001, depth=6)
    srv = Server(ex, slots=2, lanes=8)
    arr = graphgen.poisson_arrivals(60, rate=3000.0, seed=4)
    qs = [mk(i, "bfs", "a", float(arr[i]), src=i) for i in range(60)]
    st = srv.run(qs, realtime=True)
    assert st["failed"] == 0
    assert all(q.result == ("bfs", "a", q.source) for q in qs)
    # queries joined sessions that were already past level 0, lanes were
    # reused, and never more than 8 ran at once in a session
    assert any(q.joined_level > 0 for q in qs)
    assert max(q.batch for q in qs) <= 8 and st["mean_batch"] > 1.0
    used_lanes = [l for (_, _, ls) in ex.joins for l in ls]
    assert len(used_lanes) == 60 and max(used_lanes) < 8


def test_budget_binds_sessions_and_queries():
    # a session needs 40 bytes of 64: one at a time; the other graph's BFS
    # queries and the SSSP queries wait for memory
    ex = FakeExecutor({"a": 10, "b": 10}, budget=64 * 256, level_s=0.0005)
    ex.footprint_session = lambda g, lanes: 40 * 256
    ex.footprint_sssp = lambda g: 30 * 256
    srv = Server(ex, slots=3, lanes=4)
    arr = graphgen.poisson_arrivals(80, rate=4000.0, seed=5)
    kinds = graphgen.uniform_ints(80, 10, seed=6)
    qs = [mk(i, "bfs" if kinds[i] < 7 else "sssp", "a" if i % 2 else "b", float(arr[i]), src=i)
          for i in range(80)]
    st = srv.run(qs, realtime=True)
    assert st["failed"] == 0 and st["queries"] == 80
    assert all(q.result == (q.kind, q.graph, q.source) for q in qs)
    assert st["max_sessions"] == 1
    assert st["deferred_admissions"] > 0
    assert st["pool_peak_bytes"] <= 64 * 256 and ex.max_used <= 64 * 256


def test_oversized_work_fails_instead_of_blocking():
    ex = FakeExecutor({"huge": 10**9, "a": 1}, budget=1000)
    srv = Server(ex, slots=2, lanes=4)
    qs = [mk(0, "sssp", "huge"), mk(1, "bfs", "huge"), mk(2, "bfs", "a"), mk(3, "sssp", "a")]
    st = srv.run(qs, realtime=False)
    assert st["failed"] == 2
    assert qs[0].error and qs[1].error and qs[2].error is None and qs[3].error is None


def test_error_isolation():
    ex = FakeExecutor({"a": 1}, budget=1000, fail_ids={5})
    srv = Server(ex, slots=2, lanes=4)
    qs = [mk(i, "sssp", "a") for i in range(12)] + [mk(20 + i, "bfs", "a", src=i)
                                                    for i in range(6)]
    st = srv.run(qs, realtime=False)
    assert st["failed"] == 1
    assert qs[5].error and "injected" in qs[5].error
    assert all(q.error is None and q.result for q in qs if q.qid != 5)


def test_no_starvation_under_continuous_load():
    # a stream of graph-a BFS queries must not starve an SSSP on graph b
    ex = FakeExecutor({"a": 1, "b": 1}, budget=1000, service_s=0.001, level_s=0.0002)
    srv = Server(ex, slots=2, lanes=8)
    qs = [mk(i, "bfs", "a", t=0.0001 * i, src=i) for i in range(100)]
    qs.insert(10, mk(1000, "sssp", "b", t=0.00105))
    st = srv.run(qs, realtime=True)
    victim = next(q for q in qs if q.qid == 1000)
    assert st["failed"] == 0
    assert victim.end - victim.arrival < 0.05


def test_fifo_mode_runs_one_query_at_a_time():
    ex = FakeExecutor({"a": 1, "b": 1}, budget=1000, service_s=0.001)
    srv = Server(ex, lane_mode=False)
    qs = [mk(i, "bfs" if i % 3 else "sssp", "a" if i % 2 else "b", t=0.0) for i in range(20)]
    st = srv.run(qs, realtime=False)
    assert st["failed"] == 0 and ex.max_concurrent == 1
    assert all(q.batch == 1 for q in qs)
    order = sorted(qs, key=lambda q: q.start)
    assert [q.qid for q in order] == list(range(20))


def test_sessions_rotate_when_another_graph_waits_for_memory():
    # one session fits the budget; graph a's queue never empties, yet the
    # BFS query on graph b gets a session after a's quantum and drain
    ex = FakeExecutor({"a": 10, "b": 10}, budget=48 * 256, level_s=0.0005, depth=4)
    ex.footprint_session = lambda g, lanes: 40 * 256
    srv = Server(ex, slots=1, lanes=4, session_quantum=0.01)
    qs = [mk(i, "bfs", "a", t=0.0005 * i, src=i) for i in range(400)]
    qs.append(mk(1000, "bfs", "b", t=0.002, src=1))
    st = srv.run(qs, realtime=True)
    victim = next(q for q in qs if q.qid == 1000)
    assert st["failed"] == 0 and st["max_sessions"] == 1
    assert st["session_drains"] >= 1
    assert all(q.result == ("bfs", q.graph, q.source) for q in qs)
    # without rotation b would wait for a's whole stream (0.2 s)
    assert victim.end - victim.arrival < 0.08


def test_single_bfs_graphs_run_in_slots():
    # BFS queries of a graph named in single_bfs run alone in the slots (no
    # session), the other graph's BFS queries still join lane sessions
    ex = FakeExecutor({"grid": 10, "rmat": 10}, budget=4096 * 256, level_s=0.0005)
    srv = Server(ex, slots=2, lanes=8, single_bfs={"grid"})
    arr = graphgen.poisson_arrivals(60, rate=4000.0, seed=8)
    qs = [mk(i, "bfs", "grid" if i % 3 == 0 else "rmat", float(arr[i]), src=i)
          for i in range(60)]
    st = srv.run(qs, realtime=True)
    assert st["failed"] == 0
    assert all(q.result == ("bfs", q.graph, q.source) for q in qs)
    assert all(q.batch == 1 for q in qs if q.graph == "grid")
    joined = {g for (g, _, _) in ex.joins}
    assert joined == {"rmat"}
