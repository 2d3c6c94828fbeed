"""Query serving over resident graphs with continuous batching.

Graphs stay resident in HBM.  BFS and SSSP queries arrive over time and are
admitted as memory and execution resources free up:

* BFS queries run in lane sessions (grb_msbfs_session_*): one session per
  graph keeps `lanes` query lanes of a batched multi-source BFS running on
  its own stream; at every level boundary the waiting BFS queries of that
  graph join free lanes, and a lane retires as soon as its own frontier is
  empty (its result is extracted and the lane is free again), so the batch
  never drains before new queries start;
* SSSP queries run one per execution slot (grb_sssp, or grb_sssp_delta on
  the graphs given a bucket width), the oldest first, each slot on its own
  stream; so do the BFS queries of the graphs named in `single_bfs`
  (high-diameter graphs, where a batched level costs several single-source
  levels and thousands of levels make a session slower per query than a
  BFS alone);
* memory: every session's workspace, level block and extraction buffer and
  every SSSP query's workspace and output are carved from one device pool
  of `budget` bytes (:class:`DevicePool`) and returned when they finish, so
  the device memory in use never exceeds the budget.  Work that does not
  fit waits (counted as deferred) until memory is released;
* fairness: while another graph's BFS queries wait for memory to open a
  session, a session that has been open for `session_quantum` seconds
  takes no new queries, finishes the ones it holds and closes; its graph
  then queues behind the waiting graph (the drain time counts as its
  oldest waiting arrival), so large sessions rotate instead of holding the
  pool for as long as their own queue stays non-empty.

Sessions and slots overlap on the device.  A BFS result equals the query
alone (levels exactly equal single-source BFS, whatever level it joined
at), SSSP is deterministic.  With ``lane_mode=False`` the server is the
one-query-at-a-time FIFO baseline (one slot, single-source BFS and SSSP).

The scheduling logic is host code, tested on the CPU with
:class:`FakeExecutor`; :class:`GpuExecutor` binds it to the library.
"""
from __future__ import annotations

import bisect
import collections
import ctypes
import dataclasses
import threading
import time


@dataclasses.dataclass
class Query:
    qid: int
    kind: str          # "bfs" or "sssp"
    graph: str
    source: int
    arrival: float     # seconds, on the server clock
    start: float = -1.0
    end: float = -1.0
    result: object = None
    error: str | None = None
    batch: int = 0     # lanes busy in its session when it joined (1 outside sessions)
    joined_level: int = -1  # session level at which it joined (-1 outside sessions)


class DevicePool:
    """First-fit allocator over one buffer of `size` bytes (offsets aligned
    to `align`); free blocks coalesce on release.  Host bookkeeping only:
    the executor maps offsets to device memory.  Thread-safe."""

    def __init__(self, size: int, align: int = 256):
        self.size = int(size)
        self.align = int(align)
        self.free = [(0, self.size)]  # sorted (offset, length)
        self.used = 0
        self.peak = 0
        self.lock = threading.Lock()

    def _round(self, n: int) -> int:
        return max(self.align, (int(n) + self.align - 1) // self.align * self.align)

    def alloc(self, nbytes: int):
        """Offset of a block of at least nbytes, or None if none is free."""
        n = self._round(nbytes)
        with self.lock:
            for i, (off, ln) in enumerate(self.free):
                if ln >= n:
                    if ln == n:
                        self.free.pop(i)
                    else:
                        self.free[i] = (off + n, ln - n)
                    self.used += n
                    self.peak = max(self.peak, self.used)
                    return off
        return None

    def release(self, off: int, nbytes: int) -> None:
        n = self._round(nbytes)
        with self.lock:
            i = bisect.bisect_left(self.free, (off, 0))
            self.free.insert(i, (off, n))
            # coalesce with the neighbours
            if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
                self.free[i] = (self.free[i][0], self.free[i][1] + self.free[i + 1][1])
                self.free.pop(i + 1)
            if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
                self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
                self.free.pop(i)
            self.used -= n

    def fits_ever(self, nbytes: int) -> bool:
        return self._round(nbytes) <= self.size


@dataclasses.dataclass
class _Session:
    graph: str
    mem: int
    nbytes: int
    lanes: int
    opened: float = 0.0
    draining: bool = False
    thread: threading.Thread | None = None


class Server:
    """Runs a query trace over an executor (see the module text)."""

    def __init__(self, executor, slots: int = 4, lanes: int = 64, lane_mode: bool = True,
                 level_chunk: dict | None = None, session_share: float = 0.5,
                 session_quantum: float = 0.05, single_bfs=()):
        self.ex = executor
        self.session_share = float(session_share)
        self.session_quantum = float(session_quantum)
        self.single_bfs = set(single_bfs)
        self.blocked = False    # a graph's BFS queries wait for memory to open a session
        self.requeued = {}      # graph -> time its session drained to make room
        self.drains = 0
        self.pool = executor.pool
        self.slots = 1 if not lane_mode else int(slots)
        self.lanes = int(lanes)
        self.lane_mode = lane_mode
        self.level_chunk = dict(level_chunk or {})
        self.cv = threading.Condition()
        self.wait_sssp = collections.deque()   # lane mode: SSSP queries; FIFO mode: all
        self.wait_bfs = collections.defaultdict(collections.deque)
        self.sessions: dict = {}
        self.pending = 0
        self.deferred = 0       # admissions that had to wait for memory
        self.max_sessions = 0
        self.stop = False
        self.t0 = 0.0

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # ---- admission ------------------------------------------------------------
    def _fail(self, q: Query, msg: str):
        q.error = msg
        q.start = q.end = self.now()
        self.pending -= 1

    def lanes_for(self, g: str) -> int:
        """Lanes of a session on graph g: `lanes`, halved (down to 1) until
        the session takes at most `session_share` of the memory budget, so
        that large graphs still get sessions and leave room for other work."""
        k = self.lanes
        cap = int(self.pool.size * self.session_share)
        while k > 1 and self.ex.footprint_session(g, k) > cap:
            k //= 2
        return k

    def _open_sessions(self):
        """Opens sessions for graphs with waiting BFS queries (oldest first)
        while memory allows; called with the lock held."""
        cand = [(max(dq[0].arrival, self.requeued.get(g, 0.0)), g)
                for g, dq in self.wait_bfs.items() if dq and g not in self.sessions]
        self.blocked = False
        for _, g in sorted(cand):
            k = self.lanes_for(g)
            need = self.ex.footprint_session(g, k)
            if not self.pool.fits_ever(need):
                dq = self.wait_bfs[g]
                while dq:
                    self._fail(dq.popleft(), "footprint exceeds the memory budget")
                continue
            off = self.pool.alloc(need)
            if off is None:
                self.deferred += 1
                self.blocked = True
                break  # oldest first: later graphs wait too
            self.requeued.pop(g, None)
            s = _Session(g, off, need, k, opened=self.now())
            self.sessions[g] = s
            self.max_sessions = max(self.max_sessions, len(self.sessions))
            s.thread = threading.Thread(target=self._drive, args=(s,), daemon=True)
            s.thread.start()

    def submit(self, q: Query):
        with self.cv:
            self.pending += 1
            if self.lane_mode and q.kind == "bfs" and q.graph not in self.single_bfs:
                self.wait_bfs[q.graph].append(q)
                self._open_sessions()
            else:
                self.wait_sssp.append(q)
            self.cv.notify_all()

    # ---- slot workers (SSSP; everything in FIFO mode) ----------------------------
    def _take(self):
        """Head query and its memory, or None; called with the lock held."""
        if not self.wait_sssp:
            return None
        q = self.wait_sssp[0]
        need = (self.ex.footprint_sssp(q.graph) if q.kind == "sssp"
                else self.ex.footprint_bfs(q.graph))
        if not self.pool.fits_ever(need):
            self.wait_sssp.popleft()
            self._fail(q, "footprint exceeds the memory budget")
            self.cv.notify_all()
            return self._take()
        off = self.pool.alloc(need)
        if off is None:
            self.deferred += 1
            return None
        self.wait_sssp.popleft()
        return q, off, need

    def _worker(self, slot: int):
        while True:
            with self.cv:
                got = self._take()
                while got is None and not self.stop:
                    self.cv.wait(timeout=0.002)
                    got = self._take()
                if got is None:
                    return
            q, off, need = got
            q.start = self.now()
            q.batch = 1
            try:
                if q.kind == "sssp":
                    self.ex.run_sssp(slot, q, off)
                else:
                    self.ex.run_bfs(slot, q, off)
            except Exception as e:  # per-query error isolation
                q.error = f"{type(e).__name__}: {e}"
            q.end = self.now()
            self.pool.release(off, need)
            with self.cv:
                self.pending -= 1
                if self.lane_mode:
                    self._open_sessions()
                self.cv.notify_all()

    # ---- session drivers ------------------------------------------------------------
    def _drive(self, s: _Session):
        g = s.graph
        chunk = int(self.level_chunk.get(g, 1))
        busy = {}
        free = list(range(s.lanes - 1, -1, -1))
        h = None
        level = 0
        try:
            h = self.ex.session_open(g, s.lanes, s.mem)
            while True:
                with self.cv:
                    joins = []
                    dq = self.wait_bfs[g]
                    if (not s.draining and self.blocked
                            and self.now() - s.opened >= self.session_quantum):
                        s.draining = True  # make room for the waiting graph
                        self.drains += 1
                    while free and dq and not s.draining:
                        joins.append((free.pop(), dq.popleft()))
                    if not joins and not busy:
                        break
                if joins:
                    t = self.now()
                    nbusy = len(busy) + len(joins)
                    for lane, q in joins:
                        q.start = t
                        q.batch = nbusy
                        q.joined_level = level
                        busy[lane] = q
                    self.ex.session_join(h, [l for l, _ in joins], [q.source for _, q in joins])
                done, ran = self.ex.session_step(h, chunk)
                level += ran
                if done:
                    qs = [busy[l] for l in done]
                    self.ex.session_finish(h, done, qs)
                    t = self.now()
                    for l in done:
                        busy.pop(l).end = t
                        free.append(l)
                    with self.cv:
                        self.pending -= len(done)
                        self.cv.notify_all()
        except Exception as e:  # the session's queries fail, the server goes on
            msg = f"{type(e).__name__}: {e}"
            with self.cv:
                for q in busy.values():
                    q.error = msg
                    q.end = self.now()
                self.pending -= len(busy)
                busy.clear()
        finally:
            if h is not None:
                try:
                    self.ex.session_close(h)
                except Exception:
                    pass
            with self.cv:
                del self.sessions[g]
                if s.draining:
                    self.requeued[g] = self.now()
                self.pool.release(s.mem, s.nbytes)
                self._open_sessions()
                self.cv.notify_all()

    # ---- trace -------------------------------------------------------------------
    def run(self, queries: list, realtime: bool = True, progress=None) -> dict:
        """Submits each query at its arrival time (realtime) or all at once,
        waits for all to finish and returns latency statistics.  `progress`
        (optional) is called with the number of queries submitted so far,
        every 1000 submissions."""
        self.stop = False
        self.t0 = time.perf_counter()
        workers = [threading.Thread(target=self._worker, args=(s,), daemon=True)
                   for s in range(self.slots)]
        for w in workers:
            w.start()
        submitted = 0
        for q in sorted(queries, key=lambda x: x.arrival):
            if realtime:
                delay = q.arrival - self.now()
                if delay > 0:
                    time.sleep(delay)
            else:
                q.arrival = self.now()
            self.submit(q)
            submitted += 1
            if progress is not None and submitted % 1000 == 0:
                progress(submitted)
        with self.cv:
            while self.pending > 0:
                self.cv.wait(timeout=0.005)
            self.stop = True
            self.cv.notify_all()
        for w in workers:
            w.join()
        for s in list(self.sessions.values()):
            if s.thread is not None:
                s.thread.join()
        makespan = max(q.end for q in queries) - min(q.arrival for q in queries)
        st = summarize(queries, makespan)
        st["deferred_admissions"] = self.deferred
        st["session_drains"] = self.drains
        st["max_sessions"] = self.max_sessions
        st["pool_peak_bytes"] = self.pool.peak
        return st


def _pct(xs, p):
    if not xs:
        return None
    xs = sorted(xs)
    i = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return round(xs[i], 3)


def summarize(queries, makespan: float) -> dict:
    ok = [q for q in queries if q.error is None]
    lat = [(q.end - q.arrival) * 1e3 for q in ok]
    out = {"queries": len(queries), "failed": len(queries) - len(ok),
           "qps": round(len(ok) / makespan, 2) if makespan > 0 else None,
           "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
           "mean_batch": round(sum(q.batch for q in ok) / max(len(ok), 1), 2)}
    for kind in ("bfs", "sssp"):
        lk = [(q.end - q.arrival) * 1e3 for q in ok if q.kind == kind]
        out[kind] = {"n": len(lk), "p50_ms": _pct(lk, 50), "p99_ms": _pct(lk, 99)}
    by = collections.defaultdict(list)
    for q in ok:
        by[(q.graph, q.kind)].append((q.end - q.arrival) * 1e3)
    out["by_graph"] = {}
    for (g, k), v in sorted(by.items()):
        out["by_graph"].setdefault(g, {})[k] = {"n": len(v), "p50_ms": _pct(v, 50),
                                                "p99_ms": _pct(v, 99)}
    return out


class GpuExecutor:
    """Runs queries with the library.  One device buffer of `budget` bytes
    is the memory pool every admitted session or query carves its workspace
    and outputs from; graphs are resident `Matrix` objects."""

    def __init__(self, graphs: dict, budget: int, slots: int = 4, keep_results: bool = True,
                 sssp_delta: dict | None = None, extract_lanes: int = 8):
        import torch

        import paper_1908_01407_amd as grb

        self.grb = grb
        self.torch = torch
        self.graphs = graphs
        self.keep = keep_results
        # graph -> bucket width: SSSP on these graphs uses grb_sssp_delta
        self.sssp_delta = dict(sssp_delta or {})
        self.extract_lanes = int(extract_lanes)
        self.pool = DevicePool(budget)
        self.buf = torch.empty(int(budget), dtype=torch.uint8, device="cuda")
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.spare = []  # streams of closed sessions, reused
        self.lock = threading.Lock()
        # the exact switch rule (frontier degree sum against nnz): results are
        # the same under either rule, and on these graphs it is the faster
        self.desc = grb.descriptor(rule=grb.SWITCH_EXACT)

    # memory ------------------------------------------------------------------------
    def _ws_bytes(self, op, A, k):
        n = ctypes.c_size_t()
        self.grb.check(self.grb._lib.grb_workspace_size(op, A.handle, k, ctypes.byref(n)))
        return n.value

    @staticmethod
    def _a(x):
        return (int(x) + 255) // 256 * 256

    def _carve(self, off, nbytes, dtype, shape=None):
        t = self.buf[off: off + nbytes]
        t = t.view(dtype)
        return t if shape is None else t[: int(self.torch.tensor(shape).prod())].view(*shape)

    def footprint_sssp(self, g):
        A = self.graphs[g]
        return self._a(self._ws_bytes(self.grb.OP_SSSP, A, 0)) + self._a(4 * A.nrows)

    def footprint_bfs(self, g):
        A = self.graphs[g]
        return self._a(self._ws_bytes(self.grb.OP_BFS, A, 0)) + self._a(4 * A.nrows)

    def footprint_session(self, g, lanes):
        A = self.graphs[g]
        return (self._a(self._ws_bytes(self.grb.OP_MSBFS, A, lanes)) + self._a(4 * A.nrows * lanes)
                + self._a(4 * A.nrows * min(lanes, self.extract_lanes)))

    # single queries ------------------------------------------------------------------
    def run_sssp(self, slot, q, off):
        grb, torch = self.grb, self.torch
        A = self.graphs[q.graph]
        n = A.nrows
        wsb = self._a(self._ws_bytes(grb.OP_SSSP, A, 0))
        ws = self.buf[off: off + wsb]
        dist = self.buf[off + wsb: off + wsb + 4 * n].view(torch.float32)
        s = self.streams[slot]
        delta = self.sssp_delta.get(q.graph)
        if delta is None:
            grb.check(grb._lib.grb_sssp(grb._ptr(dist), A.handle, int(q.source),
                                        ctypes.byref(self.desc), grb._ptr(ws), ws.numel(),
                                        grb._stream(s)), "grb_sssp")
        else:
            grb.check(grb._lib.grb_sssp_delta(grb._ptr(dist), A.handle, int(q.source),
                                              float(delta), ctypes.byref(self.desc),
                                              grb._ptr(ws), ws.numel(), grb._stream(s)),
                      "grb_sssp_delta")
        if self.keep:
            q.result = dist.cpu()  # (synchronises the stream)
        else:
            s.synchronize()

    def run_bfs(self, slot, q, off):
        grb, torch = self.grb, self.torch
        A = self.graphs[q.graph]
        n = A.nrows
        wsb = self._a(self._ws_bytes(grb.OP_BFS, A, 0))
        ws = self.buf[off: off + wsb]
        lev = self.buf[off + wsb: off + wsb + 4 * n].view(torch.int32)
        s = self.streams[slot]
        grb.check(grb._lib.grb_bfs(grb._ptr(lev), None, A.handle, int(q.source),
                                   ctypes.byref(self.desc), grb._ptr(ws), ws.numel(),
                                   grb._stream(s)), "grb_bfs")
        if self.keep:
            q.result = lev.cpu()
        else:
            s.synchronize()

    # lane sessions -------------------------------------------------------------------
    def session_open(self, g, lanes, off):
        grb, torch = self.grb, self.torch
        A = self.graphs[g]
        n = A.nrows
        wsb = self._a(self._ws_bytes(grb.OP_MSBFS, A, lanes))
        lvb = self._a(4 * n * lanes)
        ws = self.buf[off: off + wsb]
        levels = self.buf[off + wsb: off + wsb + 4 * n * lanes].view(torch.int32).view(n, lanes)
        xb = 4 * n * min(lanes, self.extract_lanes)
        out = self.buf[off + wsb + lvb: off + wsb + lvb + xb].view(torch.int32)
        with self.lock:
            s = self.spare.pop() if self.spare else torch.cuda.Stream()
        sess = grb.MsbfsSession(A, lanes, desc=self.desc, ws=ws, levels=levels, stream=s)
        return {"sess": sess, "out": out, "n": n, "stream": s}

    def session_join(self, h, lanes, sources):
        h["sess"].join(lanes, sources)

    def session_step(self, h, levels):
        return h["sess"].step(levels)

    def session_finish(self, h, lanes, queries):
        n, m = h["n"], self.extract_lanes
        for i in range(0, len(lanes), m):
            part = lanes[i: i + m]
            out = h["out"][: len(part) * n].view(len(part), n)
            h["sess"].extract(part, out=out)  # (synchronises the stream)
            if self.keep:
                host = out.cpu()
                for j, q in enumerate(queries[i: i + m]):
                    q.result = host[j].clone()

    def session_close(self, h):
        h["sess"] = None
        with self.lock:
            self.spare.append(h["stream"])


class FakeExecutor:
    """CPU stand-in for scheduler tests: SSSP and single BFS take a fixed
    service time; a session query runs for 1 + (source mod depth) levels of
    `level_s` seconds each.  Records concurrency and memory in use; can fail
    chosen query ids."""

    def __init__(self, sizes: dict, budget: int, service_s: float = 0.002, level_s: float = 0.0005,
                 depth: int = 5, fail_ids=()):
        self.sizes = sizes
        self.pool = DevicePool(budget)
        self.service_s = service_s
        self.level_s = level_s
        self.depth = depth
        self.fail_ids = set(fail_ids)
        self.lock = threading.Lock()
        self.concurrent = 0
        self.max_concurrent = 0
        self.max_used = 0
        self.joins = []  # (graph, level of the session when they joined, lanes)

    def footprint_sssp(self, g):
        return 2 * self.sizes[g]

    def footprint_bfs(self, g):
        return self.sizes[g]

    def footprint_session(self, g, lanes):
        return self.sizes[g] * 4

    def _enter(self):
        with self.lock:
            self.concurrent += 1
            self.max_concurrent = max(self.max_concurrent, self.concurrent)
            self.max_used = max(self.max_used, self.pool.used)

    def _leave(self):
        with self.lock:
            self.concurrent -= 1

    def run_sssp(self, slot, q, off):
        self._enter()
        try:
            time.sleep(self.service_s)
            if q.qid in self.fail_ids:
                raise RuntimeError("injected failure")
            q.result = (q.kind, q.graph, q.source)
        finally:
            self._leave()

    run_bfs = run_sssp

    def session_open(self, g, lanes, off):
        self._enter()
        return {"g": g, "left": {}, "level": 0}

    def session_join(self, h, lanes, sources):
        with self.lock:
            self.joins.append((h["g"], h["level"], list(lanes)))
        for l, s in zip(lanes, sources):
            h["left"][l] = 1 + int(s) % self.depth

    def session_step(self, h, levels):
        ran = 0
        done = []
        for _ in range(levels):
            if not h["left"]:
                break
            time.sleep(self.level_s)
            ran += 1
            h["level"] += 1
            for l in list(h["left"]):
                h["left"][l] -= 1
                if h["left"][l] == 0:
                    del h["left"][l]
                    done.append(l)
        with self.lock:
            self.max_used = max(self.max_used, self.pool.used)
        return done, ran

    def session_finish(self, h, lanes, queries):
        bad = [q.qid for q in queries if q.qid in self.fail_ids]
        for q in queries:
            q.result = (q.kind, q.graph, q.source)
        if bad:
            raise RuntimeError("injected failure")

    def session_close(self, h):
        self._leave()
