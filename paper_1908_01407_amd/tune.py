"""Autotuner for the batched multi-source BFS tile shape.

grb_msbfs streams every level once per pass over `words_per_pass` query
words (64 queries each, at most 8 per pass) with `grid` workgroups per pass,
and picks push or pull per level with the descriptor's switch rule.  Wider
passes re-read each adjacency list fewer times and gather whole frontier
rows per edge; narrower passes keep the gathered frontier block (n x
words_per_pass x 8 bytes) small enough to stay in the caches.  The best
shape and rule depend on the graph, k and the device, so they are measured:
every candidate runs the real batch on the real graph and the fastest is
cached in a JSON file keyed by device, graph size and k.  A candidate is
eligible only if its levels equal a reference run's bit for bit (the
default tile, itself checked against single-source BFS on its first
queries).
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "grb_mi355x_tune.json")


RULES = {"paper": 0, "exact": 1}


def candidates(k: int):
    W = (k + 63) // 64
    kts = sorted({w for w in (1, 2, 4, 8, min(W, 8)) if w <= W})
    grids = (1024, 2048, 4096)
    return [(kt, g, r) for kt in kts for g in grids for r in RULES]


def _key(A, k, device_name):
    return f"{device_name}|n={A.nrows}|nnz={A.nnz}|k={k}"


def tune_msbfs(A, sources, *, repeats: int = 2, cache_path: str | None = DEFAULT_CACHE,
               force: bool = False, log=None):
    """Returns {"words_per_pass", "grid", "rule", "ms", "table"} for this
    graph and batch size ("rule": "paper" or "exact"), measuring candidates
    unless the cache already has them."""
    import torch

    import paper_1908_01407_amd as grb

    k = len(sources)
    dev = torch.cuda.get_device_name(A.device)
    key = _key(A, k, dev)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if not force and key in cache:
        return cache[key]
    ws = grb.workspace(grb.OP_MSBFS, A, k)
    levels = torch.empty((A.nrows, k), dtype=torch.int32, device=A.device)
    # reference levels: the default tile, its first queries checked against
    # single-source BFS runs (a different kernel); every candidate must then
    # reproduce the reference block exactly, or it is not eligible
    ref = grb.msbfs(A, sources, ws=ws).clone()
    src_host = [int(s) for s in (sources.tolist() if hasattr(sources, "tolist") else sources)]
    ws1 = grb.workspace(grb.OP_BFS, A)
    for q in range(min(k, 4)):
        single, _ = grb.bfs(A, src_host[q], parents=False, ws=ws1)
        if not torch.equal(single, ref[:, q]):
            raise RuntimeError(f"batched BFS query {q} differs from single-source BFS")
    del ws1
    table = []
    for kt, g, rule in candidates(k):
        desc = grb.descriptor(rule=RULES[rule])
        grb.msbfs(A, sources, words_per_pass=kt, grid=g, desc=desc, ws=ws, levels=levels)
        torch.cuda.synchronize()
        if not torch.equal(levels, ref):
            if log:
                log(f"[tune] kt={kt} grid={g} rule={rule}: levels differ, rejected")
            table.append({"words_per_pass": kt, "grid": g, "rule": rule, "ms": None,
                          "rejected": True})
            continue
        t0 = time.perf_counter()
        for _ in range(repeats):
            grb.msbfs(A, sources, words_per_pass=kt, grid=g, desc=desc, ws=ws, levels=levels)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / repeats * 1e3
        table.append({"words_per_pass": kt, "grid": g, "rule": rule, "ms": round(ms, 4)})
        if log:
            log(f"[tune] kt={kt} grid={g} rule={rule}: {ms:.3f} ms")
    ok = [r for r in table if r["ms"] is not None]
    if not ok:
        raise RuntimeError("no batched-BFS tile reproduced the reference levels")
    best = min(ok, key=lambda r: r["ms"])
    res = {"words_per_pass": best["words_per_pass"], "grid": best["grid"], "rule": best["rule"],
           "ms": best["ms"], "table": table}
    cache[key] = res
    if cache_path:
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            with open(cache_path + ".tmp", "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(cache_path + ".tmp", cache_path)
        except OSError:
            pass
    return res
