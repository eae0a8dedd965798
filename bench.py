#!/usr/bin/env python3
"""Exact k-NN throughput of the Random Ball Cover hot path on one MI355X.

Workload: n=1,000,000 database points, d=64, on a random 8-dim linear
subspace (N(0,1) coordinates, random orthonormal embedding) plus N(0, 0.01^2)
noise; m=10,000 queries from the same generator; n_r=1,000 representatives
drawn uniformly (seeded); Euclidean metric, k=1.  All data synthetic, seeded.

One step = the whole exact-RBC job on one batch, inputs resident in HBM:
rbc_build (BF(X, R) ownership, counting sort, radii) + rbc_search of the
10,000 queries (stage 1, pruning, grouping, grouped stage-2 tile, shortlist
re-score and certificate).  `value` = queries per second of that step.
Also reported: search-only throughput with the index resident, brute force
(bf_search) on the same batch, the other metric/k combinations, the
roofline of the dominant kernel (the grouped stage-2 distance tile) from the
library's own HIP event timer, and the CPU FP64 oracle timed on a sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_MFMA_PEAK_TF = 157.3   # MI355X dense fp32 matrix peak
ALU_PEAK_TOPS = 78.6        # fp32 VALU lane-operations per second (157.3 TFLOP/s counts an FMA as 2)


def profiled_traffic(kernel, grid_threads=None):
    """HBM bytes per launch of `kernel` (launched with grid_threads work-items,
    when given) from the committed rocprofv3 summaries (FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy's counts), or None when there is no such
    summary or the kernel's sources changed since it was taken."""
    import glob
    import hashlib

    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            line = line.strip()
            if not (line.startswith("{") and '"traffic_bytes"' in line):
                continue
            rec = json.loads(line)
            if rec.get("kernel") != kernel:
                continue
            if grid_threads is not None and rec.get("grid_threads") != grid_threads:
                continue
            h = hashlib.sha256()
            try:
                for f in rec["sources"]:
                    with open(os.path.join(ROOT, f), "rb") as fh:
                        h.update(fh.read())
            except OSError:
                return None
            return rec["traffic_bytes"] if h.hexdigest() == rec["sha256"] else None
    return None


def _progress(what):
    print(json.dumps({"progress": what}), file=sys.stderr, flush=True)


def _timed(fn, steps, warmup, sync):
    for _ in range(warmup):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) * 1e3 / steps


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--metric", default="l2", choices=["l2", "l1"])
    ap.add_argument("--k", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=1000,
                    help="queries of the oracle's timed search sample (0: skip the CPU baseline)")
    ap.add_argument("--extra", action="store_true",
                    help="also time the other metric / k combinations")
    ap.add_argument("--serving", action="store_true",
                    help="also run the serving workload (resident 2M x 96 index, Poisson "
                         "arrivals at three rates) and report p50/p99 latency and QPS")
    ap.add_argument("--configs", action="store_true",
                    help="also run the one-shot workload (2M x 128 clustered integer data) and the "
                         "4M x 128 brute force / exact RBC per precision (fp32, bf16, fp8)")
    ap.add_argument("--sweep", action="store_true",
                    help="also sweep the approximate variant's eps and the number of "
                         "representatives n_r on the headline workload")
    ap.add_argument("--range", action="store_true",
                    help="also time the range search on the headline index at radii that hold "
                         "about 1, 20 and 200 points per query")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy (byte-counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path (sharding the "
              "lists by representative is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_1103_2635_amd as rbc

    dev = torch.device("cuda", 0)
    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": a.numel() * 4}))
        return

    name = "sub8"
    w = datagen.WORKLOADS[name]
    X = datagen.database(name)
    Q = datagen.queries(name)
    reps = datagen.representatives(name)
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    m, d = Q.shape
    n = X.shape[0]
    sync = torch.cuda.synchronize
    metric, k = args.metric, args.k

    out = (torch.empty((m, k), dtype=torch.int64, device=dev),
           torch.empty((m, k), dtype=torch.float32, device=dev))
    bf_ws = torch.empty(rbc.bf_search_workspace_size(m, n, d, k, metric), dtype=torch.uint8,
                        device=dev)

    # ---- tile autotuning (library call, before any timing): the stage-2 and
    # pass-1 configuration of the exact search and the BF tile shape
    tuning = {}
    if metric == "l2":
        _progress("autotune")
        ix0 = rbc.rbc_build(Xd, w.n_r, metric=metric, rep_idx=reps)
        tuning["rbc_search"] = rbc.autotune_search(ix0, Qd, k)
        ix0.free()
        tuning["bf_search"] = rbc.autotune_bf(Qd, Xd, k, metric)

    # ---- the step: build + search
    holder = {}

    def step():
        ix = rbc.rbc_build(Xd, w.n_r, metric=metric, rep_idx=reps)
        ws = holder.get("ws")
        if ws is None:
            ws = holder["ws"] = torch.empty(rbc.rbc_search_workspace_size(ix, m, k), dtype=torch.uint8,
                                            device=dev)
        rbc.rbc_search(ix, Qd, k, out=out, workspace=ws)
        old = holder.get("ix")
        if old is not None:
            old.free()
        holder["ix"] = ix

    for _ in range(args.warmup):
        step()
    sync()
    rbc.timer_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    sync()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    tile_ms, tile_n = rbc.timer_read("tile_items")
    kernel_ms = {kn: rbc.timer_read(kn) for kn in ("stage1", "pass1", "prune", "worklist", "finalize",
                                                   "fallback")}
    rbc.timer_enable(False)
    ix = holder["ix"]

    # ---- search only (index resident) and its counters
    ws = holder["ws"]
    search_ms = _timed(lambda: rbc.rbc_search(ix, Qd, k, out=out, workspace=ws), args.steps,
                       args.warmup, sync)
    build_ms = _timed(lambda: rbc.rbc_build(Xd, w.n_r, metric=metric, rep_idx=reps).free(), 3, 1,
                      sync)
    stats = rbc.new_stats()
    rbc.rbc_search(ix, Qd, k, out=out, workspace=ws, stats=stats)
    sync()
    st = stats.cpu().numpy()
    cand = int(st[rbc.STAT_CAND])
    pairs = int(st[rbc.STAT_PAIRS])
    items = int(st[rbc.STAT_ITEMS])
    slots = int(st[rbc.STAT_SLOTS])

    # ---- brute force on the same batch, with its tile timed by the library
    rbc.timer_enable(True)
    bf_ms = _timed(lambda: rbc.bf_search(Qd, Xd, k, metric, out=out, workspace=bf_ws), args.steps,
                   args.warmup, sync)
    bf_tile_ms, bf_tile_n = rbc.timer_read("tile")
    rbc.timer_enable(False)

    def roof(flops_or_elems, ms):
        if metric == "l2":
            ach = flops_or_elems / (ms * 1e-3) / 1e12
            return {"bound": "mfma", "achieved": round(ach, 2), "peak": FP32_MFMA_PEAK_TF,
                    "unit": "TFLOP/s", "frac": round(ach / FP32_MFMA_PEAK_TF, 4)}
        ach = flops_or_elems / (ms * 1e-3) / 1e12   # lane-ops (2 per element)
        return {"bound": "alu", "achieved": round(ach, 2), "peak": ALU_PEAK_TOPS,
                "unit": "Tops/s", "frac": round(ach / ALU_PEAK_TOPS, 4)}

    per_pair = 2 * d  # l2: one multiply-add per feature (2 flops); l1: subtract + abs-add
    tile_avg = tile_ms / max(tile_n, 1)
    # stage 2 scores, for each work item, its queries against the run of rows
    # of its list that the two-pass bound leaves (pairs); that is the work
    roofline = roof(per_pair * pairs, tile_avg)
    kname = "tile_valu_items"
    tuned = tuning.get("rbc_search", {})
    if metric == "l2":
        kname = ("tile_l2_mfma32_items" if tuned.get("shape") == 32 else
                 "tile_l2_mfma_items32q" if tuned.get("item_queries") == 32 else
                 "tile_l2_mfma_items")
    roofline["traffic"] = (profiled_traffic("void rbc::%s<4, 4>(rbc::TileArgs)" % kname,
                                            256 * tuned.get("blocks", 1024))
                           if (metric, k) == ("l2", 1) else None)
    roofline["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated)"
    roofline["kernel"] = kname + " (RBC stage 2)"
    roofline["avg_ms"] = round(tile_avg, 4)
    roofline["algorithmic_units"] = ("2*d per (query, row) pair scored: sum over items of "
                                     "queries x rows of the item's run = %d pairs, %d flops per "
                                     "launch" % (pairs, per_pair * pairs))
    bf_avg = bf_tile_ms / max(bf_tile_n, 1)
    bf_roof = roof(per_pair * m * n, bf_avg)
    bf_roof["avg_ms"] = round(bf_avg, 4)
    bf_k = "tile_l2_mfma32" if tuning.get("bf_search", {}).get("shape") == 32 else "tile_l2_mfma"
    bf_roof["kernel"] = ("%s (brute force)" % bf_k) if metric == "l2" else "tile_valu (brute force)"
    bf_roof["traffic"] = (profiled_traffic("void rbc::%s<4, 4>(rbc::TileArgs)" % bf_k)
                          if (metric, k) == ("l2", 1) else None)

    extra = {}
    if args.extra:
        for mt, kk in (("l2", 1), ("l2", 10), ("l1", 1), ("l1", 10)):
            ix2 = rbc.rbc_build(Xd, w.n_r, metric=mt, rep_idx=reps)
            o2 = (torch.empty((m, kk), dtype=torch.int64, device=dev),
                  torch.empty((m, kk), dtype=torch.float32, device=dev))
            ws2 = torch.empty(rbc.rbc_search_workspace_size(ix2, m, kk), dtype=torch.uint8, device=dev)
            bws2 = torch.empty(rbc.bf_search_workspace_size(m, n, d, kk, mt), dtype=torch.uint8,
                               device=dev)
            s_ms = _timed(lambda: rbc.rbc_search(ix2, Qd, kk, out=o2, workspace=ws2), 5, 2, sync)
            b_ms = _timed(lambda: rbc.bf_search(Qd, Xd, kk, mt, out=o2, workspace=bws2), 5, 2, sync)
            extra["%s_k%d" % (mt, kk)] = {"rbc_search_qps": round(m / s_ms * 1e3, 1),
                                         "bf_qps": round(m / b_ms * 1e3, 1),
                                         "rbc_search_ms": round(s_ms, 3), "bf_ms": round(b_ms, 3)}
            ix2.free()

    # ---- CPU FP64 oracle on a bounded sample (build on the full database)
    cpu = None
    if args.cpu_sample > 0:
        import oracle

        samp = min(args.cpu_sample, m)
        t0 = time.perf_counter()
        oix = oracle.rbc_build_exact(X, reps, metric)
        t_build = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.rbc_search_exact(Q[:samp], X, oix, k, metric)
        t_search = time.perf_counter() - t0
        job_s = t_build + t_search * m / samp
        cpu = {"value": round(m / job_s, 2), "unit": "queries/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "exact RBC build on all %d points (%.1f s) + search of the first %d of "
                         "%d queries (%.1f s), scaled to the %d-query job" % (
                             n, t_build, samp, m, t_search, m)}

    serving = run_serving(rbc, torch, dev) if args.serving else None
    _progress("optional sections")
    configs = run_configs(rbc, torch, dev) if args.configs else None
    sweep = run_sweeps(rbc, torch, dev, Xd, Qd, w, reps) if args.sweep else None
    rng_line = run_range(rbc, torch, dev, Xd, Qd, w, reps) if args.range else None

    line = {
        "metric": "exact k-NN queries/s (n=1M, d=64), RBC build+search vs BF, recall 1.0",
        "value": round(m / ms_step * 1e3, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sub8: n=1,000,000 d=64, 8-dim subspace + N(0,0.01^2) noise, "
                               "m=10,000 queries, n_r=1,000, %s, k=%d" % (metric, k),
                   "n": n, "d": d, "m": m, "n_r": w.n_r, "metric": metric, "k": k,
                   "parallelism": "single GPU"},
        "search_only_qps": round(m / search_ms * 1e3, 1),
        "search_ms": round(search_ms, 3),
        "build_ms": round(build_ms, 3),
        "bf_qps": round(m / bf_ms * 1e3, 1),
        "bf_ms": round(bf_ms, 3),
        "rbc_vs_bf": round(bf_ms / ms_step, 3),
        "candidates_per_query": round(cand / m, 1),
        "candidate_fraction": round(cand / (m * n), 4),
        "pairs_scored_per_query": round(pairs / m, 1),
        "stage2_items": items,
        "stage2_rows_per_item": round(slots / 64 / max(items, 1), 1),
        "stage2_slot_use": round(pairs / max(slots, 1), 4),
        "fallback_queries": int(st[rbc.STAT_FALLBACK]),
        "kernel_ms_per_step": {kn: round(v[0] / args.steps, 4) for kn, v in kernel_ms.items()},
        "tuning": tuning,
        "roofline": roofline,
        "bf_roofline": bf_roof,
        "cpu_baseline": cpu,
    }
    if extra:
        line["paths"] = extra
    if serving:
        line["serving"] = serving
    if configs:
        line["configs"] = configs
    if sweep:
        line["sweeps"] = sweep
    if rng_line:
        line["range"] = rng_line
    print(json.dumps(line))


def run_sweeps(rbc, torch, dev, Xd, Qd, w, reps):
    """On the headline workload (L2, k = 1):
    - the approximate variant: prune_eps in {0, 0.1, 0.25, 0.5, 1, 2}: search
      time, candidates, recall@1 against brute force and the mean rank of the
      returned point (points strictly closer, counted among the 64 nearest);
    - the number of representatives: n_r from 250 to 8,000 (uniform draws),
      exact search: build and search time, candidates per query."""
    import numpy as np

    import datagen

    sync = torch.cuda.synchronize
    m = Qd.shape[0]
    n = Xd.shape[0]
    out = {}
    bi, bd = rbc.bf_search(Qd, Xd, 64, "l2")
    sync()
    bd64 = bd.cpu().numpy()
    bi1 = bi[:, 0].cpu().numpy()
    ix = rbc.rbc_build(Xd, w.n_r, rep_idx=reps)
    ws = torch.empty(rbc.rbc_search_workspace_size(ix, m, 1), dtype=torch.uint8, device=dev)
    o = (torch.empty((m, 1), dtype=torch.int64, device=dev),
         torch.empty((m, 1), dtype=torch.float32, device=dev))
    eps_rows = []
    _progress("sweep eps")
    for eps in (0.0, 0.1, 0.25, 0.5, 1.0, 2.0):
        ms = _timed(lambda: rbc.rbc_search(ix, Qd, 1, out=o, workspace=ws, prune_eps=eps), 5, 2,
                    sync)
        st = rbc.new_stats()
        rbc.rbc_search(ix, Qd, 1, out=o, workspace=ws, prune_eps=eps, stats=st)
        sync()
        ri = o[0][:, 0].cpu().numpy()
        rd = o[1][:, 0].cpu().numpy()
        rank = (bd64 < rd[:, None] * (1 - 1e-6)).sum(1)
        eps_rows.append({"eps": eps, "search_ms": round(ms, 3), "qps": round(m / ms * 1e3, 1),
                         "candidate_fraction": round(float(st.cpu().numpy()[rbc.STAT_CAND]) / (m * n), 4),
                         "recall_at_1": round(float(np.mean((ri == bi1) | (rank == 0))), 4),
                         "mean_rank": round(float(rank.mean()), 3), "max_rank_capped_64": int(rank.max())})
    ix.free()
    out["approximate_eps"] = eps_rows
    nr_rows = []
    for n_r in (250, 500, 1000, 2000, 4000, 8000):
        _progress("sweep n_r %d" % n_r)
        rr = datagen.random_reps(n, n_r, seed=23)
        b_ms = _timed(lambda: rbc.rbc_build(Xd, n_r, rep_idx=rr).free(), 2, 1, sync)
        ix = rbc.rbc_build(Xd, n_r, rep_idx=rr)
        ws = torch.empty(rbc.rbc_search_workspace_size(ix, m, 1), dtype=torch.uint8, device=dev)
        s_ms = _timed(lambda: rbc.rbc_search(ix, Qd, 1, out=o, workspace=ws), 5, 2, sync)
        st = rbc.new_stats()
        rbc.rbc_search(ix, Qd, 1, out=o, workspace=ws, stats=st)
        sync()
        stn = st.cpu().numpy()
        nr_rows.append({"n_r": n_r, "build_ms": round(b_ms, 3), "search_ms": round(s_ms, 3),
                        "step_qps": round(m / (b_ms + s_ms) * 1e3, 1),
                        "candidates_per_query": round(float(stn[rbc.STAT_CAND]) / m, 1),
                        "lists_per_query": round(float(stn[rbc.STAT_LISTS]) / m, 1)})
        ix.free()
        del ws
    out["n_r"] = nr_rows
    out["workload"] = "sub8: n=1,000,000 d=64, m=10,000, l2, k=1"
    return out


def run_range(rbc, torch, dev, Xd, Qd, w, reps):
    """Range search on the headline index (L2): for radii equal to the median
    1st, 20th and 200th nearest-neighbour distance of 256 queries, the time
    of the two calls (count, then fill + sort; the caller reads the total in
    between), points per query, and the library's kernel times."""
    import numpy as np

    sync = torch.cuda.synchronize
    m = Qd.shape[0]
    _, bd = rbc.bf_search(Qd[:256].contiguous(), Xd, 200, "l2")
    sync()
    bd = bd.cpu().numpy()
    ix = rbc.rbc_build(Xd, w.n_r, rep_idx=reps)
    ws = torch.empty(rbc.rbc_range_workspace_size(ix, m, Qd.stride(0)), dtype=torch.uint8,
                     device=dev)
    rows = []
    for kth in (1, 20, 200):
        _progress("range %d" % kth)
        radius = float(np.median(bd[:, kth - 1]))
        holder = {}

        def call():
            holder["r"] = rbc.rbc_range_search(ix, Qd, radius, workspace=ws)

        ms = _timed(call, 5, 2, sync)
        total = int(holder["r"][0][-1].item())
        rbc.timer_enable(True)
        call()
        sync()
        kern = {kn: round(rbc.timer_read(kn)[0], 4)
                for kn in ("stage1", "prune", "worklist", "range_tile", "range_sort")}
        rbc.timer_enable(False)
        rows.append({"radius": round(radius, 5), "points_per_query": round(total / m, 2),
                     "ms": round(ms, 3), "qps": round(m / ms * 1e3, 1), "kernel_ms": kern})
    ix.free()
    return {"workload": "sub8: n=1,000,000 d=64, m=10,000, l2, n_r=1,000 (index resident)",
            "radii": rows}


MFMA_PEAK_TF = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}


def run_configs(rbc, torch, dev):
    """One-shot RBC on zipf128 (n=2,000,000 d=128 clustered integer data,
    m=20,000, n_r=1,414, s=2,000, L2, k=1): build and search time, recall and
    mean rank error against brute force.  Brute force and exact RBC on sub16
    (n=4,000,000 d=128, 16-dim subspace, m=50,000, n_r=2,000, L2, k in
    {1, 10}) in fp32, bf16 and fp8: queries/s and the ranking tile's fraction
    of its own precision's matrix peak (2 d flops per scored pair)."""
    import numpy as np

    import datagen

    sync = torch.cuda.synchronize
    res = {}
    # ---- one-shot
    w = datagen.WORKLOADS["zipf128"]
    X = torch.from_numpy(datagen.database("zipf128")).to(dev)
    Q = torch.from_numpy(datagen.queries("zipf128")).to(dev)
    reps = datagen.representatives("zipf128")
    m, d = Q.shape
    build_ms = _timed(lambda: rbc.rbc_build(X, w.n_r, mode="oneshot", s=w.s, rep_idx=reps).free(),
                      3, 1, sync)
    ix = rbc.rbc_build(X, w.n_r, mode="oneshot", s=w.s, rep_idx=reps)
    out = (torch.empty((m, 1), dtype=torch.int64, device=dev),
           torch.empty((m, 1), dtype=torch.float32, device=dev))
    ws = torch.empty(rbc.rbc_search_workspace_size(ix, m, 1), dtype=torch.uint8, device=dev)
    s_ms = _timed(lambda: rbc.rbc_search(ix, Q, 1, out=out, workspace=ws), 10, 3, sync)
    got_i, got_d = out[0].clone(), out[1].clone()
    bi, bd = rbc.bf_search(Q, X, 1, "l2")
    sync()
    # rank of the returned point: points strictly closer than it (exact BF distances)
    recall = float((got_d[:, 0] <= bd[:, 0]).float().mean())
    res["oneshot_zipf128"] = {
        "workload": "zipf128: n=2,000,000 d=128 integer clustered (2,000 Zipf(1.1) centres), "
                    "m=20,000, n_r=1,414, s=2,000, l2, k=1",
        "build_ms": round(build_ms, 3), "search_ms": round(s_ms, 3),
        "search_qps": round(m / s_ms * 1e3, 1),
        "recall_at_1": round(recall, 5),
        "exact_match_ids": round(float((got_i[:, 0] == bi[:, 0]).float().mean()), 5)}
    ix.free()
    del X, Q, ws
    torch.cuda.empty_cache()
    # ---- brute force and exact RBC per precision
    w = datagen.WORKLOADS["sub16"]
    Xh = datagen.database("sub16")
    X = torch.from_numpy(Xh).to(dev)
    del Xh
    Q = torch.from_numpy(datagen.queries("sub16")).to(dev)
    reps = datagen.representatives("sub16")
    m, d = Q.shape
    n = X.shape[0]
    ix = rbc.rbc_build(X, w.n_r, rep_idx=reps, precisions=("bf16", "fp8"))
    for prec in ("fp32", "bf16", "fp8"):
        for k in (1, 10):
            out = (torch.empty((m, k), dtype=torch.int64, device=dev),
                   torch.empty((m, k), dtype=torch.float32, device=dev))
            bws = torch.empty(rbc.bf_search_workspace_size(m, n, d, k, "l2", precision=prec),
                              dtype=torch.uint8, device=dev)
            rbc.timer_enable(True)
            b_ms = _timed(lambda: rbc.bf_search(Q, X, k, "l2", out=out, workspace=bws,
                                                precision=prec), 3, 1, sync)
            t_ms, t_n = rbc.timer_read("tile")
            rbc.timer_enable(False)
            bi = out[0].clone()
            del bws
            stats = rbc.new_stats()
            rbc.bf_search(Q, X, k, "l2", out=out, workspace=None, precision=prec, stats=stats)
            sync()
            fb = int(stats.cpu().numpy()[rbc.STAT_FALLBACK])
            tile_avg = t_ms / max(t_n, 1)
            ach = 2.0 * d * m * n / (tile_avg * 1e-3) / 1e12
            rws = torch.empty(rbc.rbc_search_workspace_size(ix, m, k, precision=prec),
                              dtype=torch.uint8, device=dev)
            rbc.timer_enable(True)
            r_ms = _timed(lambda: rbc.rbc_search(ix, Q, k, out=out, workspace=rws, precision=prec),
                          3, 1, sync)
            rt_ms, rt_n = rbc.timer_read("tile_items")
            rbc.timer_enable(False)
            st2 = rbc.new_stats()
            rbc.rbc_search(ix, Q, k, out=out, workspace=rws, precision=prec, stats=st2)
            sync()
            st2 = st2.cpu().numpy()
            del rws
            torch.cuda.empty_cache()
            r_avg = rt_ms / max(rt_n, 1)
            r_ach = 2.0 * d * float(st2[rbc.STAT_CAND]) / (r_avg * 1e-3) / 1e12
            res["sub16_%s_k%d" % (prec, k)] = {
                "bf_ms": round(b_ms, 2), "bf_qps": round(m / b_ms * 1e3, 1),
                "bf_tile": {"avg_ms": round(tile_avg, 3), "achieved_tflops": round(ach, 1),
                            "peak_tflops": MFMA_PEAK_TF[prec],
                            "frac": round(ach / MFMA_PEAK_TF[prec], 4)},
                "bf_fallback_queries": fb,
                "rbc_search_ms": round(r_ms, 2), "rbc_search_qps": round(m / r_ms * 1e3, 1),
                "rbc_tile": {"avg_ms": round(r_avg, 3), "achieved_tflops": round(r_ach, 1),
                             "frac": round(r_ach / MFMA_PEAK_TF[prec], 4)},
                "rbc_candidate_fraction": round(float(st2[rbc.STAT_CAND]) / (m * n), 4),
                "rbc_fallback_queries": int(st2[rbc.STAT_FALLBACK])}
            print(json.dumps({"progress": "sub16 %s k=%d" % (prec, k)}), file=sys.stderr, flush=True)
    ix.free()
    res["sub16_workload"] = ("sub16: n=4,000,000 d=128, 16-dim subspace + N(0,0.02^2), m=50,000, "
                             "n_r=2,000, l2")
    return res


def run_serving(rbc, torch, dev, n_requests=2000, precisions=("fp32", "bf16")):
    """Serving workload: resident exact index over n=2,000,000 d=96 (12-dim
    subspace + N(0,0.01^2)), n_r=1,414; a 200,000-query pool; request sizes
    round(exp(N(4, 1.5^2))) clipped to [1, 4096], k uniform in {1, 10};
    Poisson arrivals at 0.3, 0.6, 0.9 of the measured saturation rate; four
    execution streams, batches of at most 4,096 queries."""
    import numpy as np

    import datagen
    from paper_1103_2635_amd.serving import GpuExecutor, Request, Scheduler, latency_stats, replay

    w = datagen.WORKLOADS["sub12"]
    X = torch.from_numpy(datagen.database("sub12")).to(dev)
    pool = torch.from_numpy(datagen.queries("sub12")).to(dev)
    reps = datagen.representatives("sub12")
    ix = rbc.rbc_build(X, w.n_r, rep_idx=reps, precisions=precisions)
    out = {"workload": "sub12: n=2,000,000 d=96, n_r=1,414, pool 200,000, sizes lognormal(4,1.5) "
                       "clipped [1,4096], k in {1,10}, 4 streams, max batch 4096"}
    for prec in precisions:
        def search(Q, k, o, ws, prec=prec):
            rbc.rbc_search(ix, Q, k, out=o, workspace=ws, precision=prec)

        def ws_fn(m, k, prec=prec):
            return rbc.rbc_search_workspace_size(ix, m, k, precision=prec)

        res = {}
        _progress("serving %s" % prec)
        # saturation: every request of a trace arrives at once
        t, sizes, ks, offs = datagen.arrival_trace("sub12", 1.0, n_requests, pool.shape[0])
        ex = GpuExecutor(pool, search, ws_fn, 4, max_batch=4096, max_k=10)

        def run(times):
            sched = Scheduler(ex, 4, mem_budget=8 << 30, max_batch=4096)
            reqs = [Request(i, int(offs[i]), int(sizes[i]), int(ks[i]), float(times[i]))
                    for i in range(len(times))]
            done = replay(sched, reqs, time.perf_counter, lambda s: time.sleep(0))
            torch.cuda.synchronize()
            return latency_stats(done)
        run(np.zeros(200))  # warm-up of streams and allocator
        sat = run(np.zeros(n_requests))
        res["saturation_qps"] = round(sat["qps"], 1)
        mean_size = float(np.mean(sizes))
        for frac in (0.3, 0.6, 0.9):
            _progress("serving %s load %.1f" % (prec, frac))
            rate = frac * sat["qps"] / mean_size
            tt, _, _, _ = datagen.arrival_trace("sub12", rate, n_requests, pool.shape[0])
            st = run(tt)
            res["load_%.1f" % frac] = {k2: round(v, 3) for k2, v in st.items()}
        out[prec] = res
    ix.free()
    return out


if __name__ == "__main__":
    main()
