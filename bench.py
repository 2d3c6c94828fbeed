#!/usr/bin/env python3
"""Benchmark of the masked semiring mxv library on one MI355X.

Headline (one JSON line on stdout): direction-optimised BFS from vertex 0 on
a symmetrised R-MAT graph, scale 22, edge factor 16, (a, b, c, d) =
(0.57, 0.19, 0.19, 0.05), int32 CSR, Boolean semiring, levels and parents.
A step is one full BFS; value = stored entries of the symmetrised CSR per
second of BFS (the paper's TEPS convention, Section 8), in GTEPS.

The JSON line also carries:
* roofline: HBM roofline of the BFS level kernel k_bfs_level (the step's dominant
  kernel): algorithmic bytes of all its launches in K steps divided by their
  summed duration (HIP events recorded by the library on the launch stream,
  in a second pass over the same K steps so that the events do not slow the
  headline pass), against 8 TB/s;
* cpu_baseline: the CPU oracle (single-threaded queue BFS with the
  min-id parent pass) timed on this host on the same graph;
* extras: SSSP on the same graph (Bellman-Ford rounds and bucketed), BFS/SSSP
  on a 3000x3000 grid, PageRank and adaptive PageRank on a directed R-MAT
  scale 22 graph (fp32 and fp64), triangle counting on R-MAT scales 18 and
  22, batched BFS and the serving loop, each with its own timing.

Other modes: --rocprof-summary DIR prints a per-kernel summary of rocprofv3
CSV output (kernel stats and FETCH_SIZE / WRITE_SIZE counters).
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# algorithmic byte models (what the method must move, not what the kernel did)
# ---------------------------------------------------------------------------

def first_hit_scan(rp, ci, rows_mask, hit_col):
    """Edges a scan with early exit must read: for every row in rows_mask,
    the position of its first neighbour with hit_col[neighbour] plus one, or
    its full degree when there is none (one vectorised step per edge
    position, over the rows still scanning)."""
    deg = np.diff(rp).astype(np.int64)
    rows = np.flatnonzero(rows_mask & (deg > 0))
    starts = rp[rows].astype(np.int64)
    lens = deg[rows]
    total, k = 0, 0
    while rows.size:
        total += rows.size
        hit = hit_col[ci[starts + k]]
        keep = ~hit & (lens > k + 1)
        rows, starts, lens = rows[keep], starts[keep], lens[keep]
        k += 1
    return total


def parents_bytes(rp, ci, lev, directions, frontier, n, symmetric=True):
    """Bytes of the parent work per level kernel.  A push from a one-vertex
    frontier writes each found vertex's parent with its level (4 bytes each,
    charged to that level).  After a push from several vertices the next
    level's kernel finds the parents of its frontier: when it pushes over the
    same CSR (symmetric graph), from the edges it expands anyway, reading the
    level of every expanded neighbour (4 per edge) and writing the parent
    (4); otherwise by scanning each vertex's in-neighbours up to the first
    one a level up: row extents (8), ids and levels of the scanned
    neighbours (8 each) and the parent (4).  Charged to that next level.
    Pull levels find parents while they scan."""
    deg = np.diff(rp).astype(np.int64)
    out = [0.0] * len(directions)
    for d, dr in enumerate(directions):
        if dr != 1:
            continue
        nxt = lev == d + 1
        cnt = int(nxt.sum())
        if not cnt:
            continue
        if frontier[d] == 1:
            out[d] += 4.0 * cnt
        elif d + 1 < len(out):
            if symmetric and directions[d + 1] == 1:
                out[d + 1] += 4.0 * int(deg[nxt].sum()) + 4.0 * cnt
            else:
                out[d + 1] += 12.0 * cnt + 8.0 * first_hit_scan(rp, ci, nxt, lev == d)
    return out


def bfs_bytes_per_level(rp, ci, lev, directions, n):
    """Per-level algorithmic bytes of a BFS level given the direction run.
    push: frontier ids and row extents 12|f|, neighbour ids 4*sum deg(f),
          visited bitmap probe n/8, next bitmap n/8, level 4|next| (parents
          in parents_bytes).
    pull: visited n/8, frontier bitmap n/8, row extents 8R of candidate rows,
          neighbour ids 4*E_scan (early exit), next bitmap n/8, 8|next|."""
    deg = np.diff(rp).astype(np.int64)
    out = []
    for d, dr in enumerate(directions):
        f = lev == d
        nf = int(f.sum())
        nxt = int((lev == d + 1).sum())
        if dr == 1:
            b = 12 * nf + 4 * int(deg[f].sum()) + n / 8 + n / 8 + 4 * nxt
        else:
            cand = ((lev < 0) | (lev > d)) & (deg > 0)
            e_scan = first_hit_scan(rp, ci, cand, f)
            b = 3 * n / 8 + 8 * int(cand.sum()) + 4 * e_scan + 8 * nxt
        out.append(float(b))
    return out


# ---------------------------------------------------------------------------
# rocprofv3 summaries
# ---------------------------------------------------------------------------

# sources whose change invalidates counter readings of the BFS level kernel
KERNEL_SOURCES = ["paper_1908_01407_amd/csrc/grb_bfs.hip", "paper_1908_01407_amd/csrc/grb_device.h",
                  "paper_1908_01407_amd/csrc/grb_internal.h", "paper_1908_01407_amd/csrc/grb_api.cpp"]
COUNTERS_FILE = "profiles/k_bfs_level_rmat22_counters.txt"


def kernel_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic():
    """HBM bytes per k_bfs_level launch from the committed counter summary,
    or None when it is missing or the kernel's sources changed since."""
    path = os.path.join(ROOT, COUNTERS_FILE)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("sources_sha256") != kernel_sources_digest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def short_name(name):
    """Kernel name without namespaces' noise and argument lists (60 chars)."""
    name = name.replace("(anonymous namespace)::", "")
    if "elementwise_kernel" in name:
        return "torch_elementwise_kernel" + ("(mul)" if "Mul" in name or "mul" in name else "")
    return name.split("(")[0][:60]


def serve_report(paths):
    """Markdown tables of the serving runs in the given bench output files
    (one JSON line each): per load point and budget, p50/p99 per query type
    and graph, batched sessions against the FIFO server."""
    out = []
    for path in paths:
        with open(path) as f:
            d = json.loads([ln for ln in f.read().splitlines() if ln.startswith("{")][-1])
        sv = d.get("serving", d if "saturation" in d else None)  # bench line or --serve-out
        if not sv:
            continue
        out.append(f"## {os.path.basename(path)}: budget {sv['budget_bytes'] >> 20} MiB, "
                   f"{sv['queries_per_point']} queries per point, {sv['mix']}")
        sat = sv["saturation"]
        if "batched" in sat:
            out.append(f"saturation (all queries at once): batched {sat['batched']['qps']} q/s, "
                       f"FIFO {sat['fifo']['qps']} q/s")
        else:
            out.append(f"saturation rate given: {sat['batched_qps_given']} q/s ({sat['note']})")
        out.append(f"session lanes: {sv['session_lanes']}")
        graphs = sorted(sv["graphs"])

        def rows(tag, st):
            r = [f"| {tag} | all | {st['p50_ms']} | {st['p99_ms']} | {st['qps']} |"]
            for kind in ("bfs", "sssp"):
                r.append(f"| {tag} | {kind} | {st[kind]['p50_ms']} | {st[kind]['p99_ms']} | |")
                for g in graphs:
                    x = st["by_graph"].get(g, {}).get(kind)
                    if x:
                        r.append(f"| {tag} | {kind} {g} (n={x['n']}) | {x['p50_ms']} | "
                                 f"{x['p99_ms']} | |")
            return r
        for pt in sv.get("points", []):
            b, f = pt["batched"], pt["fifo"]
            out.append("")
            out.append(f"### load {pt['load_of_batched_saturation']} x saturation = "
                       f"{pt['rate_qps']} q/s (batched: deferred {b['deferred_admissions']}, "
                       f"drains {b.get('session_drains', 0)}, max sessions {b['max_sessions']}, "
                       f"pool peak {b['pool_peak_bytes'] >> 20} MiB, mean batch {b['mean_batch']})")
            out.append("| server | queries | p50 ms | p99 ms | q/s |")
            out.append("|---|---|---|---|---|")
            out += rows("batched", b) + rows("FIFO", f)
        for sw in sv.get("budget_sweep", []):
            st = sw["stats"]
            out.append("")
            out.append(f"### budget {sw['budget_bytes'] >> 20} MiB at 0.75 x saturation "
                       f"(deferred {st['deferred_admissions']}, drains "
                       f"{st.get('session_drains', 0)}, max sessions {st['max_sessions']}, "
                       f"pool peak {st['pool_peak_bytes'] >> 20} MiB)")
            out.append("| server | queries | p50 ms | p99 ms | q/s |")
            out.append("|---|---|---|---|---|")
            out += rows("batched", st)
        out.append("")
    return "\n".join(out)


MXV_STAGES = [("k_mxv_init", "mxv_init"), ("k_compact", "compact"), ("k_mxv_list_prep", "list_prep"),
              ("k_mxv_prep", "mxv_prep"), ("k_mxv_push", "mxv_push"), ("k_mxv_merge", "mxv_merge"),
              ("k_mxv_sweep", "mxv_pull"), ("k_mxv_fixup", "mxv_pull_fixup")]


def mxv_trace_summary(d, counter=None):
    """Per-stage figures of the mxv sweep from a rocprofv3 run (csv) of a
    bench run: kernel durations (us) from the kernel trace, or, with
    `counter`, that counter's KiB per dispatch from the counter collection.
    Calls start at each k_mxv_init and come in the sweep's order (q, p,
    direction; one warm-up and five timed calls each); the table gives the
    mean of the timed calls."""
    pattern = "*counter_collection.csv" if counter else "*kernel_trace.csv"
    paths = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    disp = {}  # dispatch -> [order key, kernel name, value]
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                if counter:
                    if r["Counter_Name"] != counter:
                        continue
                    key = int(r["Dispatch_Id"])
                    e = disp.setdefault(key, [key, r["Kernel_Name"], 0.0])
                    e[2] += float(r["Counter_Value"])
                else:
                    key = int(r["Start_Timestamp"])
                    us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                    disp[(key, r["Dispatch_Id"])] = [key, r["Kernel_Name"], us]
    calls = []
    for _, name, val in sorted(disp.values(), key=lambda e: e[0]):
        stage = next((st for k, st in MXV_STAGES if k + "(" in name or k + "<" in name), None)
        if stage is None:
            continue
        if stage == "mxv_init":
            calls.append({})
        if not calls:
            continue
        calls[-1][stage] = calls[-1].get(stage, 0.0) + val
    points = [(q, p, c) for q in (0.0, 0.5) for p in (1e-4, 1e-3, 1e-2, 0.05, 0.2, 0.5)
              for c in ("push", "pull", "auto")]
    if len(calls) < 6 * len(points):
        return f"expected {6 * len(points)} mxv calls in the run, found {len(calls)}"
    calls = calls[: 6 * len(points)]  # the sweep runs first; later products (CC) follow
    names = [st for _, st in MXV_STAGES]
    out = [f"{'q':>4s} {'p':>7s} {'call':>6s} " + " ".join(f"{n:>14s}" for n in names)
           + f" {'sum':>9s}"]
    for i, (q, p, c) in enumerate(points):
        grp = calls[6 * i + 1: 6 * i + 6]
        mean = {n: sum(g.get(n, 0.0) for g in grp) / len(grp) for n in names}
        out.append(f"{q:4.1f} {p:7g} {c:>6s} " + " ".join(f"{mean[n]:14.1f}" for n in names)
                   + f" {sum(mean.values()):9.1f}")
    return "\n".join(out)


def _counter_means(d, counter):
    """{kernel short name: (dispatches, mean KiB per dispatch)} of one counter
    in the rocprofv3 counter collection(s) under d."""
    per = {}
    for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                key = (short_name(r["Kernel_Name"]), r["Dispatch_Id"])
                per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    agg = {}
    for (k, _), v in per.items():
        a = agg.setdefault(k, [0, 0.0])
        a[0] += 1
        a[1] += v
    return {k: (n, v / n) for k, (n, v) in agg.items()}


def bfs_counters_file(fetch_dir, write_dir, bench_json):
    """The k_bfs_level counter summary (the file bench.py reads its traffic
    figure from) from two rocprofv3 --pmc runs of bench.py --calibrate-copy
    (FETCH_SIZE, then WRITE_SIZE) and the bench output of one of them."""
    fe = _counter_means(fetch_dir, "FETCH_SIZE")
    wr = _counter_means(write_dir, "WRITE_SIZE")
    with open(bench_json) as f:
        b = json.loads([ln for ln in f.read().splitlines() if ln.startswith("{")][-1])
    alg = float(b["roofline"]["algorithmic_bytes_per_launch"])
    cal = "torch_elementwise_kernel(mul)"
    sf = 262144.0 / fe[cal][1]
    sw = 262144.0 / wr[cal][1]
    kf, kw = fe["grb::k_bfs_level"][1], wr["grb::k_bfs_level"][1]
    traffic = (kf * sf + kw * sw) * 1024.0
    out = ["k_bfs_level on RMAT-22: HBM traffic from rocprofv3 counters",
           "(FETCH_SIZE and WRITE_SIZE, KiB per dispatch, one run each)", "",
           "commands (from the repository root on the GPU host):"]
    for c, dd in (("FETCH_SIZE", "pmc_fetch"), ("WRITE_SIZE", "pmc_write")):
        out.append(f"  export TMPDIR=/tmp; R=$GRAFT_REPO_ROOT; cd /tmp && rocprofv3 --pmc {c} "
                   f"--output-format csv -d $R/gpurun_out/{dd} -o run -- python3 $R/bench.py "
                   "--no-extras --no-msbfs --no-serve --no-cpu-baseline --headline-only --rule exact "
                   "--steps 3 --warmup 1 --calibrate-copy")
    out += ["  python bench.py --bfs-counters gpurun_out/pmc_fetch gpurun_out/pmc_write "
            "<bench output of the FETCH_SIZE run>", "",
            f"Each run does 1 warm-up, 3 timed and 3 profiled BFS runs "
            f"({fe['grb::k_bfs_level'][0] // 7} level launches each)",
            "and, last, one streaming kernel of known size (torch elementwise multiply",
            "over 64 Mi fp32: 256 MiB read, 256 MiB written).", ""]
    out.append(f"{'kernel':40s} {'counter':>12s} {'dispatches':>10s} {'KiB/dispatch':>14s}")
    for name, tab, c in (("fetch", fe, "FETCH_SIZE"), ("write", wr, "WRITE_SIZE")):
        for k in sorted(tab):
            out.append(f"{k:40s} {c:>12s} {tab[k][0]:10d} {tab[k][1]:14.1f}")
    out += ["", "calibration (streaming kernel, 262144 KiB each way):",
            f"  FETCH_SIZE reads {fe[cal][1]:.1f} KiB -> scale {sf:.4f}",
            f"  WRITE_SIZE reads {wr[cal][1]:.1f} KiB -> scale {sw:.4f}",
            "k_bfs_level per launch (average over the launches of a BFS):",
            f"  fetched {kf:.1f} KiB x {sf:.4f} + written {kw:.1f} KiB x {sw:.4f}",
            f"  = {traffic / 1e6:.2f} MB per launch, against {alg / 1e6:.2f} MB of algorithmic bytes",
            f"  ({traffic / alg:.1f}x): cache-line granularity of the random gathers (row",
            "  starts of candidate rows, frontier and visited words) and the level / parent",
            "  stores of scattered vertices", "",
            f"traffic_bytes_per_launch: {int(round(traffic))}",
            f"sources_sha256: {kernel_sources_digest()}",
            "sources: " + ", ".join(KERNEL_SOURCES)]
    return "\n".join(out)


def bfs_trace(d):
    """Kernels of one BFS (the second-to-last in the trace) from a rocprofv3
    kernel trace (csv) of a bench run: start, duration and the gap before
    each launch, in us from the BFS's first kernel."""
    rows = []
    for path in sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)):
        with open(path) as f:
            rows += [r for r in csv.DictReader(f)
                     if "k_bfs_start" in r["Kernel_Name"] or "k_bfs_level" in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    starts = [i for i, r in enumerate(rows) if "k_bfs_start" in r["Kernel_Name"]]
    if len(starts) < 2:
        return "fewer than two BFS runs in the trace"
    grp = rows[starts[-2]: starts[-1]]
    t0 = int(grp[0]["Start_Timestamp"])
    out, prev_end = [], t0
    for r in grp:
        b, e = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        out.append(f"{short_name(r['Kernel_Name']):22s} start={(b - t0) / 1e3:8.2f} us  "
                   f"dur={(e - b) / 1e3:7.2f} us  gap={(b - prev_end) / 1e3:6.2f} us")
        prev_end = e
    return "\n".join(out)


def rocprof_summary(d):
    lines = []
    for path in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
        lines.append(f"# kernel stats: {os.path.relpath(path, d)}")
        with open(path) as f:
            rows = list(csv.DictReader(f))
        rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
        lines.append(f"{'kernel':60s} {'calls':>7s} {'total_us':>11s} {'avg_us':>9s} {'pct':>6s}")
        for r in rows:
            name = short_name(r["Name"])
            lines.append(f"{name:60s} {int(r['Calls']):7d} {float(r['TotalDurationNs'])/1e3:11.1f} "
                         f"{float(r['AverageNs'])/1e3:9.2f} {float(r['Percentage']):6.2f}")
    for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        lines.append(f"# counters: {os.path.relpath(path, d)}")
        agg = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                key = (short_name(r["Kernel_Name"]), r["Counter_Name"])
                a = agg.setdefault(key, [0, 0.0, set()])
                a[1] += float(r["Counter_Value"])
                a[2].add(r.get("Dispatch_Id", r.get("Correlation_Id", "")))
        lines.append(f"{'kernel':60s} {'counter':>12s} {'dispatches':>10s} {'KiB/dispatch':>14s}")
        for (k, c), (_, v, ids) in sorted(agg.items(), key=lambda x: -x[1][1]):
            nd = max(len(ids), 1)
            lines.append(f"{k:60s} {c:>12s} {nd:10d} {v / nd:14.1f}")
    return "\n".join(lines)


# ---------------------------------------------------------------------------
# measurements
# ---------------------------------------------------------------------------

def timed(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def host_info():
    cpu = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu": cpu, "logical_cpus": os.cpu_count()}


def mxv_sweep(grb, torch, A, rp, ci):
    """Forced-push, forced-pull and automatic grb_mxv on the same graph:
    w<not m, replace> = A' u over LOR_LAND with a structural mask, u a random
    frontier of density p, m a random visited set of density q.  Algorithmic
    bytes per product:
      push: frontier bitmap n/8, list and row extents 16|u|, column ids
            4 sum deg(u), mask and output bitmaps 2n/8, values 1 per output;
      pull: mask, frontier and output bitmaps 3n/8, row extents 8 per
            allowed non-empty row, column ids 4 E_scan (first frontier hit),
            values 1 per output."""
    n = A.nrows
    deg = np.diff(rp).astype(np.int64)
    rng = np.random.default_rng(5)
    out = []

    def make(bits, dtype):
        v = grb.Vector(n, dtype)
        idx = torch.from_numpy(np.flatnonzero(bits).astype(np.int64)).to(v.values.device)
        v.values[idx] = 1
        words = np.packbits(bits.astype(np.uint8), bitorder="little")
        words = np.concatenate([words, np.zeros((-len(words)) % 8, np.uint8)]).view(np.int64)
        v.bitmap[: len(words)] = torch.from_numpy(words).to(v.values.device)
        return v

    ws = grb.workspace(grb.OP_MXV, A)
    for q in (0.0, 0.5):
        mask_bits = rng.random(n) < q
        for p in (1e-4, 1e-3, 1e-2, 0.05, 0.2, 0.5):
            u_bits = rng.random(n) < p
            U = make(u_bits, torch.uint8)
            Mk = make(mask_bits, torch.uint8)
            W = grb.Vector(n, torch.uint8)
            allowed = ~mask_bits
            nxt_rows = allowed & (deg > 0)
            e_scan = first_hit_scan(rp, ci, nxt_rows, u_bits)
            hit = np.zeros(n, bool)
            src = np.repeat(np.arange(n), deg)
            hit[src[u_bits[ci]]] = True
            n_out = int((hit & allowed).sum())
            nu = int(u_bits.sum())
            push_b = n / 8 + 16 * nu + 4 * int(deg[u_bits].sum()) + 2 * n / 8 + n_out
            pull_b = 3 * n / 8 + 8 * int(nxt_rows.sum()) + 4 * e_scan + n_out
            row = {"frontier_density": p, "mask_density": q, "frontier": nu,
                   "push_edges": int(deg[u_bits].sum()), "pull_edges_scanned": int(e_scan)}
            for name, dr in (("push", 1), ("pull", 2), ("auto", 0)):
                d = grb.descriptor(direction=dr, rule=1,
                                   flags=grb.GRB_MASK_COMP | grb.GRB_MASK_STRUCT | grb.GRB_REPLACE)
                run = lambda: grb.mxv(W, Mk, None, "lor_land", A, U, desc=d, ws=ws)
                run()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(5):
                    run()
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / 5
                row[f"{name}_ms"] = round(ms, 4)
                if name != "auto":
                    b = push_b if name == "push" else pull_b
                    row[f"{name}_gbs"] = round(b / (ms / 1e3) / 1e9, 1)
                    row[f"{name}_frac_hbm"] = round(b / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
            out.append(row)
            log(f"[bench] mxv sweep p={p} q={q}: push {row['push_ms']} ms "
                f"({row['push_frac_hbm']}), pull {row['pull_ms']} ms ({row['pull_frac_hbm']}), "
                f"auto {row['auto_ms']} ms")
            del U, Mk, W, src
    return out


def bench_extras(grb, graphgen, torch, args):
    ex = {}
    if not args.no_sweep:
        ex["mxv_sweep_rmat22"] = mxv_sweep(grb, torch, args._A, args._rp, args._ci)
    # SSSP on the same R-MAT graph (min-plus, weights 1..64)
    A = args._A
    ws = grb.workspace(grb.OP_SSSP, A)
    for name, rule in (("paper", 0), ("exact", 1)):
        d = grb.descriptor(rule=rule)
        grb.sssp(A, 0, desc=d, ws=ws)
        ms = timed(lambda: grb.sssp(A, 0, desc=d, ws=ws), args.extra_steps, torch)
        st = grb.last_stats()
        ex[f"sssp_rmat{args.scale}_{name}"] = {
            "ms": round(ms, 4), "gteps": round(A.nnz / ms / 1e6, 3),
            "rounds": st["iterations"], "pushes": st["pushes"], "pulls": st["pulls"]}
    dp = grb.descriptor(rule=1, flags=grb.GRB_PROFILE)
    grb.sssp(A, 0, desc=dp, ws=ws)
    st = grb.last_stats()
    ex[f"sssp_rmat{args.scale}_kernels"] = {
        "expand_ms_push": round(st["expand_ms_push"], 4),
        "expand_ms_pull": round(st["expand_ms_pull"], 4),
        "per_round_ms": [round(x, 4) for x in st["kernel_ms"]],
        "direction": st["direction"], "frontier": st["frontier"], "edges": st["edges"]}
    # SSSP pull as masked SpMV over the whole graph: bytes of one full pull round
    # (col + weight of every stored entry, row extents, frontier bitmap, distances)
    dpull = grb.descriptor(direction=2, flags=grb.GRB_PROFILE)
    grb.sssp(A, 0, desc=dpull, ws=ws)
    st = grb.last_stats()
    n = A.nrows
    if st["kernel_ms"]:
        rounds = len(st["kernel_ms"])
        tot_ms = sum(st["kernel_ms"])
        bytes_round = 8 * A.nnz + 4 * (n + 1) + 4 * n + 4 * n + n / 4
        ex[f"sssp_rmat{args.scale}_forced_pull"] = {
            "rounds": rounds, "ms": round(tot_ms, 4),
            "bytes_per_round_model": bytes_round,
            "gbs": round(bytes_round * rounds / (tot_ms / 1e3) / 1e9, 1),
            "frac_hbm": round(bytes_round * rounds / (tot_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "note": "per round: col_idx + weight of every stored entry (8 B), row extents, "
                    "frontier distances (gathered, counted once), distances read, candidate "
                    "and next-frontier bitmaps"}
    del ws
    # connected components (FastSV on the generic product) on the same graph
    wsc = grb.workspace(grb.OP_CC, A)
    grb.cc(A, ws=wsc)
    ms = timed(lambda: grb.cc(A, ws=wsc), args.extra_steps, torch)
    lab, it = grb.cc(A, ws=wsc)
    lab = lab.cpu().numpy()
    ex[f"cc_rmat{args.scale}"] = {
        "ms": round(ms, 4), "iterations": it,
        "components": int((lab == np.arange(lab.size)).sum()),
        "note": "FastSV: per iteration one MIN_SECOND pull product with MIN accumulate, "
                "hooking, shortcutting and grandparents; the last iteration finds no change"}
    del wsc, lab
    # grid 3000 x 3000
    if not args.no_grid:
        gg = graphgen.grid(3000, 3000)
        G = grb.Matrix.from_raw(gg)
        wsb = grb.workspace(grb.OP_BFS, G)
        wss = grb.workspace(grb.OP_SSSP, G)
        grb.bfs(G, 0, ws=wsb)
        ms = timed(lambda: grb.bfs(G, 0, ws=wsb), 2, torch)
        st = grb.last_stats()
        ex["bfs_grid3000"] = {"ms": round(ms, 3), "levels": st["iterations"],
                              "us_per_level": round(ms * 1e3 / max(st["iterations"], 1), 2),
                              "gteps": round(G.nnz / ms / 1e6, 4)}
        grb.sssp(G, 0, ws=wss)
        ms = timed(lambda: grb.sssp(G, 0, ws=wss), 2, torch)
        st = grb.last_stats()
        ex["sssp_grid3000"] = {"ms": round(ms, 3), "rounds": st["iterations"],
                               "us_per_round": round(ms * 1e3 / max(st["iterations"], 1), 2),
                               "gteps": round(G.nnz / ms / 1e6, 4)}
        # bucketed rounds (grb_sssp_delta), same distances
        for delta in (512.0, 2048.0):
            grb.sssp(G, 0, ws=wss, delta=delta)
            ms = timed(lambda: grb.sssp(G, 0, ws=wss, delta=delta), 2, torch)
            st = grb.last_stats()
            ex[f"sssp_grid3000_delta{int(delta)}"] = {
                "ms": round(ms, 3), "rounds": st["iterations"],
                "us_per_round": round(ms * 1e3 / max(st["iterations"], 1), 2),
                "gteps": round(G.nnz / ms / 1e6, 4)}
        del G, wsb, wss
    # PageRank on a directed R-MAT graph
    if not args.no_pr:
        gd = graphgen.rmat(args.scale, symmetric=False, weights=False)
        P = grb.Matrix.from_raw(gd, weights=False)
        res = {}
        p64, it64, _ = grb.pagerank(P, dtype=torch.float64, max_iter=50, tol=1e-7)
        for dt, name in ((torch.float32, "fp32"), (torch.float64, "fp64")):
            ws = grb.workspace(grb.OP_PAGERANK, P, 2 if dt == torch.float64 else 1)
            grb.pagerank(P, dtype=dt, max_iter=50, tol=1e-7, ws=ws)
            ms = timed(lambda: grb.pagerank(P, dtype=dt, max_iter=50, tol=1e-7, ws=ws),
                       args.extra_steps, torch)
            p, it, delta = grb.pagerank(P, dtype=dt, max_iter=50, tol=1e-7, ws=ws,
                                        desc=grb.descriptor(flags=grb.GRB_PROFILE))
            st = grb.last_stats()
            # kernels of the iterations that ran (the batch of eight launched
            # iterations ends with some that return at once after convergence)
            kk = st["kernel_ms"][:it] or [st["expand_ms_all"] / max(st["launches"], 1)]
            kms = float(np.mean(kk))
            n = P.nrows
            esz = 8 if dt == torch.float64 else 4
            # per iteration: col_idx of every in-edge, row extents, x gather
            # working set once, p read + write, out-degree row extents, x write
            bytes_it = 4 * P.nnz + 4 * (n + 1) + esz * n + 2 * esz * n + 4 * (n + 1) + esz * n
            res[name] = {"ms_total": round(ms, 4), "iterations": it,
                         "ms_per_iter": round(ms / max(it, 1), 4),
                         "spmv_kernel_ms": round(kms, 4),
                         "spmv_kernel_gbs": round(bytes_it / (kms / 1e3) / 1e9, 1),
                         "spmv_kernel_frac_hbm": round(bytes_it / (kms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                         "gteps_per_iter": round(P.nnz / (ms / max(it, 1)) / 1e6, 3)}
            if name == "fp32":
                res[name]["l1_vs_gpu_fp64"] = float(
                    (p.double() - p64).abs().sum().item())
            # adaptive form: converged vertices frozen (relative change <= eps)
            for eps in (1e-4, 1e-5):
                grb.pagerank_adaptive(P, eps, dtype=dt, max_iter=50, tol=1e-7, ws=ws)
                ms_a = timed(lambda: grb.pagerank_adaptive(P, eps, dtype=dt, max_iter=50,
                                                           tol=1e-7, ws=ws),
                             args.extra_steps, torch)
                q, it_a, _, act = grb.pagerank_adaptive(P, eps, dtype=dt, max_iter=50, tol=1e-7,
                                                        ws=ws)
                st = grb.last_stats()
                res[f"{name}_adaptive_eps{eps:g}"] = {
                    "ms_total": round(ms_a, 4), "iterations": it_a, "active_left": act,
                    "edges_touched": int(sum(st["edges"])),
                    "edges_touched_vs_plain": round(sum(st["edges"]) / (P.nnz * it), 4),
                    "l1_vs_gpu_fp64_plain": float((q.double() - p64).abs().sum().item())}
            del ws
        res["nnz"] = P.nnz
        res["iterations_fp64_reference"] = it64
        ex[f"pagerank_rmat{args.scale}_dir"] = res
        del P
    # triangle counting: the sum of L L^T .* L (degree-ordered lower triangle)
    if not args.no_tc:
        for sc in sorted({18, args.scale}):
            g = graphgen.rmat(sc, weights=False)
            rp, ci, _ = grb.lower_by_degree(g.n, g.src, g.dst)  # setup, untimed
            L = grb.Matrix(g.n, g.n, rp, ci, None, symmetric=False)
            ws = grb.workspace(grb.OP_MXM, None)
            t = grb.tricount(L, ws=ws)
            ms = timed(lambda: grb.tricount(L, ws=ws), args.extra_steps, torch)
            grb.tricount(L, ws=ws, desc=grb.descriptor(flags=grb.GRB_PROFILE))
            kms = grb.last_stats()["expand_ms_all"]
            # membership probes: every entry of row j of L, once per row i
            # holding j (entries of L equal to j)
            lr = np.diff(rp).astype(np.int64)
            probes = int(np.sum(lr * np.bincount(ci, minlength=g.n)))
            ex[f"tricount_rmat{sc}"] = {
                "ms": round(ms, 3), "kernel_ms": round(kms, 3), "triangles": t,
                "nnz_lower": int(ci.shape[0]), "probes": probes,
                "gprobes_per_s": round(probes / (kms / 1e3) / 1e9, 1),
                "edges_per_s_g": round(2 * ci.shape[0] / (ms / 1e3) / 1e9, 3)}
            del L, ws
    return ex


def bench_msbfs(grb, graphgen, torch, args):
    """Batched multi-source BFS (k = 64 and 512, R-MAT 20 and 22) with tiles
    from the autotuner, against 64 sequential single-source BFS runs."""
    from paper_1908_01407_amd import tune

    res = {}
    for scale in args.msbfs_scales:
        if scale == args.scale:
            g, A = args._g, args._A
        else:
            g = graphgen.rmat(scale, weights=False)
            A = grb.Matrix.from_raw(g, weights=False)
        ws1 = grb.workspace(grb.OP_BFS, A)
        for k in args.msbfs_k:
            src = graphgen.sources(g.src, g.dst, g.n, k, seed=3)
            best = tune.tune_msbfs(A, src, cache_path=args.tune_cache, repeats=2, log=log)
            wsk = grb.workspace(grb.OP_MSBFS, A, k)
            lev = torch.empty((A.nrows, k), dtype=torch.int32, device="cuda")
            dbest = grb.descriptor(rule=tune.RULES[best.get("rule", "paper")])
            run = lambda: grb.msbfs(A, src, words_per_pass=best["words_per_pass"],
                                    grid=best["grid"], desc=dbest, ws=wsk, levels=lev)
            run()
            ms = timed(run, args.extra_steps, torch)
            st = grb.last_stats()
            seq_src = src[:64]
            dseq = grb.descriptor(rule=grb.SWITCH_EXACT)  # the faster rule for one source
            ms_seq = timed(lambda: [grb.bfs(A, int(s), parents=False, desc=dseq, ws=ws1)
                                    for s in seq_src], 1, torch)
            per_src_seq = ms_seq / len(seq_src)
            # algorithmic floor of the batch: every (vertex, query) level is
            # written once (4 B), and each level streams the CSR once per pass
            # of query words (4 B per column id, 8 B per row extent pair)
            reached = int((lev >= 0).sum().item())
            W = (k + 63) // 64
            passes = -(-W // min(best["words_per_pass"] or W, 8))
            grb.msbfs(A, src, words_per_pass=best["words_per_pass"], grid=best["grid"],
                      desc=grb.descriptor(rule=tune.RULES[best.get("rule", "paper")],
                                          flags=grb.GRB_PROFILE), ws=wsk, levels=lev)
            stp = grb.last_stats()
            nlev = stp["iterations"]
            floor_b = 4 * reached + nlev * passes * (4 * A.nnz + 8 * A.nrows)
            # the same floor level by level: (vertex, query) pairs reached at
            # each level, counted in blocks of rows
            hist = np.zeros(nlev + 1, np.int64)
            for r0 in range(0, A.nrows, 1 << 18):
                blk = (lev[r0: r0 + (1 << 18)] + 1).flatten().long()
                hist += torch.bincount(blk, minlength=nlev + 1).cpu().numpy()[: nlev + 1]
            lvl_b = [int(4 * hist[l + 1] + passes * (4 * A.nnz + 8 * A.nrows))
                     for l in range(nlev)]
            kern_ms = stp["expand_ms_all"]
            # the timed batch's first 64 queries equal the sequential runs
            for q, s in enumerate(seq_src):
                single, _ = grb.bfs(A, int(s), parents=False, desc=dseq, ws=ws1)
                if not torch.equal(single, lev[:, q]):
                    raise RuntimeError(f"batched BFS rmat{scale} k={k}: query {q} differs "
                                       "from its single-source BFS")
            res[f"rmat{scale}_k{k}"] = {
                "ms": round(ms, 3), "levels": st["iterations"],
                "sources_per_s": round(k / ms * 1e3, 1),
                "gteps": round(k * A.nnz / ms / 1e6, 2),
                "tile": {"words_per_pass": best["words_per_pass"], "grid": best["grid"],
                         "rule": best.get("rule", "paper")},
                "sequential_ms_per_source": round(per_src_seq, 4),
                "speedup_vs_sequential": round(per_src_seq * k / ms, 2),
                "k_ms_level": {"launches": stp["launches"],
                               "avg_launch_us": round(kern_ms / max(stp["launches"], 1) * 1e3, 2),
                               "per_level_us": [round(x * 1e3, 1) for x in stp["kernel_ms"]],
                               "direction": stp["direction"][:nlev]},
                "bytes_floor": floor_b,
                "per_level_bytes_floor": lvl_b,
                "per_level_floor_gbs": [round(b / (t * 1e-3) / 1e9, 1) if t > 0 else None
                                        for b, t in zip(lvl_b, stp["kernel_ms"])],
                "floor_gbs": round(floor_b / (kern_ms / 1e3) / 1e9, 1),
                "floor_frac_hbm": round(floor_b / (kern_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                "floor_model": "4 B per reached (vertex, query) level + per level and pass of "
                               "query words 4 B per column id and 8 B per row extent pair"}
            del wsk, lev
        del ws1
    return res


def bench_serve(grb, graphgen, torch, args):
    """Serving: six resident graphs, Poisson arrivals, 70% BFS / 30% SSSP.
    BFS queries join lane sessions of their graph at level boundaries and
    retire on their own; SSSP queries run in slots; every session and query
    carves its memory from one pool of the HBM budget (admission binds when
    the pool is full).  Compared with a one-query-at-a-time FIFO server at
    the same arrival rates.  The full protocol (--serve-full) sweeps the
    load over {0.25, 0.5, 0.75, 0.9, 1.1} x saturation with 10,000 queries
    per point and the budget over 1-8 GiB."""
    from paper_1908_01407_amd.serve import GpuExecutor, Query, Server

    raws = {f"rmat{s}": (args._g if s == args.scale else graphgen.rmat(s)) for s in (16, 18, 20, 22)}
    raws["grid2000"] = graphgen.grid(2000, 2000)
    raws["grid3000"] = graphgen.grid(3000, 3000)
    graphs = {k: (args._A if k == f"rmat{args.scale}" else grb.Matrix.from_raw(g))
              for k, g in raws.items()}
    names = sorted(graphs)
    cand = {k: np.flatnonzero(graphgen.touched(g.src, g.dst, g.n)) for k, g in raws.items()}

    def trace(nq, rate, seed):
        arr = graphgen.poisson_arrivals(nq, rate=rate, seed=4 + seed)
        kind = graphgen.uniform_ints(nq, 10, seed=50 + seed)
        gs = graphgen.uniform_ints(nq, len(names), seed=60 + seed)
        pick = graphgen.uniform_doubles(nq, seed=70 + seed)
        qs = []
        for i in range(nq):
            gname = names[int(gs[i])]
            c = cand[gname]
            qs.append(Query(qid=i, kind="bfs" if kind[i] < 7 else "sssp", graph=gname,
                            source=int(c[min(int(pick[i] * c.size), c.size - 1)]),
                            arrival=float(arr[i])))
        return qs

    # high-diameter graphs: bucketed SSSP, several BFS levels per session step
    deltas = {"grid2000": 512.0, "grid3000": 512.0}
    chunks = {"grid2000": 16, "grid3000": 16}
    # their BFS queries run alone in the slots: thousands of levels make a
    # lane session slower per query than a single-source BFS
    single = {"grid2000", "grid3000"}
    full = args.serve_full
    nq = 10000 if full else args.serve_queries
    loads = args.serve_load
    if loads is None:
        loads = [0.25, 0.5, 0.75, 0.9, 1.1] if full else [0.5, 0.9]
    sweep_gib = args.serve_sweep
    if sweep_gib is None:
        sweep_gib = [1, 2, 4, 8] if full else []
    budget = args.serve_budget

    def prog(tag):
        return lambda k: log(f"[bench] serve {tag}: {k} queries submitted")

    def checkpoint():
        if args.serve_out:
            with open(args.serve_out, "w") as f:
                json.dump(out, f)

    def batched(bud):
        ex = GpuExecutor(graphs, budget=bud, slots=args.serve_slots, keep_results=False,
                         sssp_delta=deltas)
        return ex, (lambda: Server(ex, slots=args.serve_slots, lanes=64, level_chunk=chunks,
                                   single_bfs=single))

    ex, mk = batched(budget)
    fifo_ex = GpuExecutor(graphs, budget=budget, slots=1, keep_results=False, sssp_delta=deltas)
    fifo = lambda: Server(fifo_ex, lane_mode=False)
    out = {"graphs": {k: {"n": A.nrows, "nnz": A.nnz} for k, A in graphs.items()},
           "mix": "70% BFS / 30% SSSP, graph and source uniform, Poisson arrivals",
           "budget_bytes": budget, "queries_per_point": nq,
           "session_lanes": {g: mk().lanes_for(g) for g in names}}
    mk().run(trace(4 * len(names), 1e6, 99), realtime=False)  # warm-up
    fifo().run(trace(2 * len(names), 1e6, 98), realtime=False)
    if args.serve_sat is None:
        sat = mk().run(trace(nq, 1e9, 0), realtime=False, progress=prog("saturation"))
        fifo_sat = fifo().run(trace(max(nq // 4, 200), 1e9, 0), realtime=False,
                              progress=prog("fifo saturation"))
        out["saturation"] = {"batched": sat, "fifo": fifo_sat}
        checkpoint()
        log(f"[bench] serve saturation: batched {sat['qps']} q/s, fifo {fifo_sat['qps']} q/s")
        qps = sat["qps"]
    else:
        qps = float(args.serve_sat)
        out["saturation"] = {"batched_qps_given": qps,
                             "note": "measured by an earlier run of the same protocol"}
    points = []
    for frac in loads:
        rate = frac * qps
        b = mk().run(trace(nq, rate, 1), realtime=True, progress=prog(f"load {frac}"))
        f = fifo().run(trace(nq, rate, 1), realtime=True, progress=prog(f"fifo load {frac}"))
        points.append({"rate_qps": round(rate, 1), "load_of_batched_saturation": frac,
                       "batched": b, "fifo": f})
        out["points"] = points
        checkpoint()
        log(f"[bench] serve rate {rate:.1f}: batched p50 {b['p50_ms']} p99 {b['p99_ms']} "
            f"(deferred {b['deferred_admissions']}, drains {b['session_drains']}) "
            f"| fifo p50 {f['p50_ms']} p99 {f['p99_ms']}")
    out["points"] = points
    if sweep_gib:
        # budget sweep at 0.75 x saturation
        sweep = []
        for bud in (int(b * (1 << 30)) for b in sweep_gib):
            del ex
            torch.cuda.empty_cache()
            ex, mkb = batched(bud)
            r = mkb().run(trace(nq, 0.75 * qps, 2), realtime=True, progress=prog(f"budget {bud}"))
            sweep.append({"budget_bytes": bud, "stats": r})
            out["budget_sweep"] = sweep
            checkpoint()
            log(f"[bench] serve budget {bud >> 20} MiB: p50 {r['p50_ms']} p99 {r['p99_ms']} "
                f"qps {r['qps']} deferred {r['deferred_admissions']}")
        out["budget_sweep"] = sweep
    return out


def cpu_oracle_other(g, graphgen, args):
    """The oracle timed on this host's cores for the other workloads, each on
    a bounded sample: SSSP (Dijkstra, one core), connected components (one
    core), PageRank (FP64 power iteration, one core, three iterations),
    batched BFS (64 sources, one query per thread on all cores) and the
    serving mix (64 queries of the six graphs, one per thread on all
    cores)."""
    import concurrent.futures as cf

    import oracle
    cores = max(1, min(16, os.cpu_count() or 1))
    res = {"host": host_info()["cpu"], "cores_available": cores}
    adj = oracle.Adjacency.from_raw(g)
    t0 = time.perf_counter()
    oracle.sssp(adj, 0)
    t = time.perf_counter() - t0
    res["sssp_rmat"] = {"ms": round(t * 1e3, 1), "gteps": round(adj.nnz / t / 1e9, 4), "cores": 1,
                        "sample": f"one Dijkstra from vertex 0 on RMAT-{args.scale}"}
    t0 = time.perf_counter()
    _, ncc = oracle.cc(adj)
    t = time.perf_counter() - t0
    res["cc_rmat"] = {"ms": round(t * 1e3, 1), "components": ncc, "cores": 1,
                      "sample": f"minimum-label components of RMAT-{args.scale}, one core"}
    gd = graphgen.rmat(args.scale, symmetric=False, weights=False)
    adjd = oracle.Adjacency.from_raw(gd)
    t0 = time.perf_counter()
    oracle.pagerank(adjd, 0.85, 3, 0.0)
    t = (time.perf_counter() - t0) / 3
    res["pagerank_rmat_dir"] = {"ms_per_iter": round(t * 1e3, 1), "cores": 1,
                                "gteps_per_iter": round(adjd.nnz / t / 1e9, 4),
                                "sample": "3 FP64 iterations (the sweep of all in-edges each)"}
    del adjd, gd
    src = graphgen.sources(g.src, g.dst, g.n, 64, seed=3)
    t0 = time.perf_counter()
    oracle.msbfs(adj, src, nthreads=cores)
    t = time.perf_counter() - t0
    res["batched_bfs_rmat_k64"] = {"ms": round(t * 1e3, 1), "sources_per_s": round(64 / t, 2),
                                   "cores": cores,
                                   "sample": f"64 sources on RMAT-{args.scale}, one BFS per thread"}
    # serving mix: 64 queries over the six graphs, one per thread
    raws = {f"rmat{s}": (g if s == args.scale else graphgen.rmat(s)) for s in (16, 18, 20)}
    raws["grid2000"] = graphgen.grid(2000, 2000)
    adjs = {k: (adj if v is g else oracle.Adjacency.from_raw(v)) for k, v in raws.items()}
    adjs[f"rmat{args.scale}"] = adj
    names = sorted(adjs)
    kind = graphgen.uniform_ints(64, 10, seed=50)
    gs = graphgen.uniform_ints(64, len(names), seed=60)
    jobs = []
    for i in range(64):
        a = adjs[names[int(gs[i])]]
        jobs.append((a, 0 if kind[i] < 7 else 1, int(i * 7919) % a.n))

    def one(job):
        a, k, s = job
        return oracle.bfs(a, s, parents=False) if k == 0 else oracle.sssp(a, s)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as pool:
        list(pool.map(one, jobs))
    t = time.perf_counter() - t0
    res["serving_mix"] = {"queries_per_s": round(64 / t, 2), "cores": cores,
                          "sample": "64 queries (70% BFS / 30% SSSP) over RMAT 16/18/20/"
                                    f"{args.scale} and the 2000^2 grid, one per thread"}
    return res


def cpu_baseline(g, A_nnz, args):
    import oracle
    adj = oracle.Adjacency.from_raw(g)
    runs, t_total = 0, 0.0
    while runs < 1 or (t_total < args.cpu_seconds and runs < 20):
        t0 = time.perf_counter()
        oracle.bfs(adj, 0)
        t_total += time.perf_counter() - t0
        runs += 1
    per = t_total / runs
    return {"value": round(A_nnz / per / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{runs} full BFS runs (queue BFS + min-id parent pass) from vertex 0 on "
                      f"the same RMAT-{args.scale} graph; {per * 1e3:.1f} ms per BFS; "
                      f"host {host_info()['cpu']}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--rule", choices=("auto", "paper", "exact"), default="auto",
                    help="direction switch rule of the timed BFS (auto: the faster one, "
                         "measured; results are identical under either)")
    ap.add_argument("--extra-steps", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the BFS runs from other sources and on RMAT-14 (so that a "
                         "profile of the level kernel holds the headline BFS alone)")
    ap.add_argument("--no-grid", action="store_true")
    ap.add_argument("--no-pr", action="store_true")
    ap.add_argument("--no-tc", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-msbfs", action="store_true")
    ap.add_argument("--msbfs-scales", type=int, nargs="*", default=[20, 22])
    ap.add_argument("--msbfs-k", type=int, nargs="*", default=[64, 512])
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file caching autotuned batched-BFS tiles (default: none)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-queries", type=int, default=600)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget", type=int, default=2 << 30,
                    help="device memory of the serving pool in bytes (default 2 GiB)")
    ap.add_argument("--serve-full", action="store_true",
                    help="full serving protocol: 10,000 queries per point, five loads, "
                         "budget sweep (minutes of GPU time)")
    ap.add_argument("--serve-load", type=float, nargs="*", default=None,
                    help="loads as fractions of the batched saturation rate (default 0.5 0.9; "
                         "with --serve-full 0.25 0.5 0.75 0.9 1.1)")
    ap.add_argument("--serve-sweep", type=float, nargs="*", default=None,
                    help="budgets in GiB of the sweep at 0.75 x saturation (default: none; "
                         "with --serve-full 1 2 4 8)")
    ap.add_argument("--serve-out", metavar="JSON", default=None,
                    help="write the serving results to this file after every measured point")
    ap.add_argument("--serve-sat", type=float, default=None,
                    help="batched saturation rate (q/s) of an earlier run of the same protocol: "
                         "skips measuring it, so the protocol can be split over several runs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 256 MiB device copy (counter calibration)")
    ap.add_argument("--rocprof-summary", metavar="DIR")
    ap.add_argument("--mxv-trace", metavar="DIR",
                    help="print the per-stage table of the mxv sweep from a rocprofv3 kernel trace")
    ap.add_argument("--mxv-counter", metavar="COUNTER",
                    help="with --mxv-trace: the table of this counter (KiB per dispatch) from a "
                         "rocprofv3 --pmc run instead of durations")
    ap.add_argument("--bfs-trace", metavar="DIR",
                    help="print the kernels of one BFS from a rocprofv3 kernel trace")
    ap.add_argument("--bfs-counters", metavar=("FETCH_DIR", "WRITE_DIR", "BENCH_JSON"), nargs=3,
                    help="print the k_bfs_level counter summary from two --pmc runs")
    ap.add_argument("--serve-report", metavar="BENCH_JSON", nargs="+",
                    help="print markdown tables of the serving runs in these bench outputs")
    args = ap.parse_args()

    if args.serve_report:
        print(serve_report(args.serve_report))
        return 0
    if args.mxv_trace:
        print(mxv_trace_summary(args.mxv_trace, args.mxv_counter))
        return 0
    if args.bfs_counters:
        print(bfs_counters_file(*args.bfs_counters))
        return 0
    if args.bfs_trace:
        print(bfs_trace(args.bfs_trace))
        return 0

    if args.rocprof_summary:
        print(rocprof_summary(args.rocprof_summary))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU "
              "sharding of this workload (by rows of the output, by query for batched BFS and "
              "serving) is not built.",
              file=sys.stderr)
        return 2

    import torch

    import graphgen
    import paper_1908_01407_amd as grb

    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        return 1
    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    log(f"[bench] generating RMAT-{args.scale}")
    g = graphgen.rmat(args.scale)
    log(f"[bench] building CSR ({time.perf_counter() - t_setup:.1f}s)")
    A = grb.Matrix.from_raw(g)
    args._A = A
    args._g = g
    n, nnz = A.nrows, A.nnz
    log(f"[bench] n={n} nnz={nnz} ({time.perf_counter() - t_setup:.1f}s)")
    ws = grb.workspace(grb.OP_BFS, A)

    # pick the switch rule by measurement (results are identical either way)
    rule_ms = {}
    if args.rule == "auto":
        for rule in (0, 1):
            d = grb.descriptor(rule=rule)
            for _ in range(max(args.warmup, 1)):
                grb.bfs(A, 0, desc=d, ws=ws)
            rule_ms[rule] = round(timed(lambda: grb.bfs(A, 0, desc=d, ws=ws), 5, torch), 4)
        rule = min(rule_ms, key=rule_ms.get)
    else:
        rule = 0 if args.rule == "paper" else 1
    desc = grb.descriptor(rule=rule)
    dprof = grb.descriptor(rule=rule, flags=grb.GRB_PROFILE)
    out_bufs = (torch.empty(n, dtype=torch.int32, device="cuda"),
                torch.empty(n, dtype=torch.int32, device="cuda"))
    for _ in range(args.warmup):
        grb.bfs(A, 0, desc=desc, ws=ws, out=out_bufs)

    # timed region: K full BFS runs (levels and parents), inputs resident
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lev, par = grb.bfs(A, 0, desc=desc, ws=ws, out=out_bufs)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) / args.steps * 1e3
    value = nnz / (ms_per_step / 1e3) / 1e9
    log(f"[bench] BFS {ms_per_step:.4f} ms/step -> {value:.2f} GTEPS (rule {rule})")

    # the same K runs again with the library's HIP events around every level
    # kernel (on the launch stream): the kernel durations for the roofline
    # (the events add host and queue work, so this pass is not the headline)
    launches, exp_ms = 0, 0.0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        lev, par = grb.bfs(A, 0, desc=dprof, ws=ws, out=out_bufs)
        st = grb.last_stats()
        launches += st["launches"]
        exp_ms += st["expand_ms_all"]
    torch.cuda.synchronize()
    ms_profiled = (time.perf_counter() - t1) / args.steps * 1e3

    # algorithmic bytes of the expand launches of one BFS
    levels = lev.cpu().numpy()
    rp = A.row_ptr.cpu().numpy()
    ci = A.col_idx.cpu().numpy()
    args._rp, args._ci = rp, ci
    per_level = bfs_bytes_per_level(rp, ci, levels, st["direction"], n)
    par = parents_bytes(rp, ci, levels, st["direction"], st["frontier"], n)
    per_level = [b + p for b, p in zip(per_level, par)]
    bytes_step = sum(per_level)
    achieved = bytes_step * args.steps / (exp_ms / 1e3) / 1e9
    reached = int((levels >= 0).sum())
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": counter_traffic(),
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by a "
                        "streaming kernel of known size)",
        "algorithmic_bytes_per_launch": round(bytes_step * args.steps / max(launches, 1)),
        "kernel": "k_bfs_level",
        "region": "second pass of the K timed steps with per-level HIP events "
                  f"({ms_profiled:.4f} ms/step with the events)",
        "launches_per_step": launches / args.steps,
        "avg_launch_us": round(exp_ms / launches * 1e3, 3),
        "algorithmic_bytes_per_step": bytes_step,
        "per_level": [{"level": i, "dir": "push" if st["direction"][i] == 1 else "pull",
                       "frontier": st["frontier"][i], "edges": st["edges"][i],
                       "bytes": per_level[i], "kernel_us": round(st["kernel_ms"][i] * 1e3, 2)}
                      for i in range(len(per_level))] + (
            [{"level": len(per_level), "dir": "empty level (ends the search)", "bytes": 0.0,
              "kernel_us": round((st["expand_ms_all"] - sum(st["kernel_ms"])) * 1e3, 2)}]
            if st["launches"] > len(per_level) else []),
    }
    out = {
        "metric": f"BFS GTEPS at RMAT-{args.scale} (direction-optimised, from vertex 0)",
        "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"DO-BFS from vertex 0 on symmetrised RMAT scale {args.scale}, "
                               f"edge factor 16, (a,b,c,d)=(0.57,0.19,0.19,0.05), int32 CSR, "
                               f"levels+parents",
                   "n": n, "nnz": nnz, "levels": st["iterations"],
                   "switch_rule": "paper" if rule == 0 else "exact",
                   "rule_ms": {("paper" if r == 0 else "exact"): v for r, v in rule_ms.items()},
                   "gteps_graph500": round(
                       (int(np.diff(rp)[levels >= 0].sum()) // 2) / (ms_per_step / 1e3) / 1e9, 3),
                   "reached": reached},
        "roofline": roofline,
    }
    # the practical HBM ceiling beside the 8 TB/s peak: a 1 GiB device copy
    cp_src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    cp_dst = torch.empty_like(cp_src)
    cp_dst.copy_(cp_src)
    cp_ms = timed(lambda: cp_dst.copy_(cp_src), 5, torch)
    copy_gbs = 2 * (1 << 30) / (cp_ms / 1e3) / 1e9
    del cp_src, cp_dst
    out["roofline"]["copy_ceiling_gbs"] = round(copy_gbs, 1)
    out["roofline"]["frac_of_copy_ceiling"] = round(achieved / copy_gbs, 5)
    # the headline workload from three other sources (random, degree > 0)
    other = []
    for s in ([] if args.headline_only else graphgen.sources(g.src, g.dst, g.n, 3, seed=3)):
        grb.bfs(A, int(s), desc=desc, ws=ws, out=out_bufs)
        ms_s = timed(lambda: grb.bfs(A, int(s), desc=desc, ws=ws, out=out_bufs), 5, torch)
        other.append({"source": int(s), "ms": round(ms_s, 4), "levels": grb.last_stats()["iterations"],
                      "gteps": round(nnz / (ms_s / 1e3) / 1e9, 2)})
    out["config"]["other_sources"] = other
    # C1: the small configuration, a latency line (microseconds per BFS)
    if not args.headline_only:
        g14 = graphgen.rmat(14)
        A14 = grb.Matrix.from_raw(g14)
        ws14 = grb.workspace(grb.OP_BFS, A14)
        out14 = (torch.empty(A14.nrows, dtype=torch.int32, device="cuda"),
                 torch.empty(A14.nrows, dtype=torch.int32, device="cuda"))
        for _ in range(3):
            grb.bfs(A14, 0, desc=desc, ws=ws14, out=out14)
        ms14 = timed(lambda: grb.bfs(A14, 0, desc=desc, ws=ws14, out=out14), 10, torch)
        out["rmat14_bfs"] = {
            "us_per_bfs": round(ms14 * 1e3, 2), "levels": grb.last_stats()["iterations"],
            "gteps": round(A14.nnz / (ms14 / 1e3) / 1e9, 3), "runs": 10, "warmup": 3,
            "note": "levels + parents from vertex 0; L2-resident, a latency figure"}
        del A14, ws14, out14
    if args.calibrate_copy:
        # a plain streaming kernel of known traffic for the counter scale:
        # reads 256 MiB and writes 256 MiB (torch's elementwise multiply)
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        out["calibration_kernel"] = "torch elementwise mul, 256 MiB read + 256 MiB written"
    if not args.no_extras:
        log("[bench] extras")
        out["extras"] = bench_extras(grb, graphgen, torch, args)
    if not args.no_msbfs:
        log("[bench] batched BFS")
        out["batched_bfs"] = bench_msbfs(grb, graphgen, torch, args)
    if not args.no_serve:
        log("[bench] serving")
        out["serving"] = bench_serve(grb, graphgen, torch, args)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(g, nnz, args)
        if not args.no_extras:
            log("[bench] oracle baselines of the other workloads")
            out["cpu_oracle_other"] = cpu_oracle_other(g, graphgen, args)
    out["host"] = host_info()
    out["gpu"] = torch.cuda.get_device_name(0)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
