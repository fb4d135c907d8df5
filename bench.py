#!/usr/bin/env python3
"""Throughput of scoring a partition with the full no-ground-truth metric set
(Q, Qds with its split penalty, and the six measures of Section II-B3) on an
LFR-style graph of 10,000,000 nodes (degree exponent 2, average degree 20, maximum
1,000; community-size exponent 1, sizes 50-5,000; mixing 0.3), on one MI355X.

One step = one synchronous cq_score_partition call over the resident graph and label
array: every kernel of the scoring path plus the copy of the result to the host.
Value = stored CSR entries (2|E|) per second, in GEdges/s.

Prints one JSON line.  ``roofline`` reports the dominant kernel: its duration comes from
HIP events on the library's stream around that kernel alone, recorded inside the timed
steps (every timed stage costs a few microseconds of device time, so the other stages
are timed in separate steps before them: ``stage_ms_all_timed``); ``cpu_baseline``
times the CPU oracle on the same graph on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "GEdges/s scoring full metric set at 10M/100M nodes; served p50/p99 latency"
HBM_PEAK_GBS = 8000.0
WEIGHTED_MAX_LABELS = 32768  # label ids a weighted score can take (its direct LDS table)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_l10m.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1507_05492_amd", "csrc", f) for f in ("cq_kernels.hpp", "cq_device.hpp")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n: int, nnz: int) -> int:
    # what the scoring path must move: every stored CSR entry once (4 B) and, per node,
    # its row offset and its label once (8 B)
    return 4 * nnz + 8 * n


def kernel_names(L: int, blocked: bool) -> dict:
    """Profiler names of the unweighted kernels of each stage (namespace dropped)."""
    lt = "unsigned short" if L <= 65535 else "unsigned int"
    priv = "true" if L <= 131072 else "false"  # LDS-private node histograms (in label ranges)
    return {"edge_gather": f"k_gather_blocked<{lt}, false>" if blocked else f"k_gather<{priv}, {lt}, false>",
            "group_count": f"k_groups<ScoreVis, {lt}>",
            "node_pass": f"k_node_scatter<{lt}>" if blocked else f"k_node_priv<true, {lt}, true>",
            "final_reduce": "k_score_final1", "column_scan": "k_colscan", "scan_order": "k_scan_order"}


def traffic_for(kernel: str):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated),
    valid only if the kernels are unchanged since the counters were taken."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="l10m", choices=["l10m", "s100m", "m100k_mu0.3", "batch256", "serve"],
                    help="batch256: 256 LFR-style graphs x 4 partitions as one batch; serve: Poisson request "
                         "load on a resident 100M-node graph plus 64 graphs (each prints its own JSON line)")
    ap.add_argument("--serve-requests", type=int, default=10000, help="requests per load point and stream seed (serve)")
    ap.add_argument("--serve-seeds", default="3,5", help="comma-separated request-stream seeds (serve)")
    ap.add_argument("--seed", type=int, default=21)
    ap.add_argument("--order", default="locality", choices=["locality", "input"],
                    help="graph storage order: 'locality' loads with CQ_GRAPH_REORDER (default), 'input' keeps node ids")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="l10m: skip the reassigned/random partitions and the 100M-node line")
    ap.add_argument("--no-s100m", action="store_true", help="l10m: skip the 100M-node line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (a known-size reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; scoring across several GPUs is not implemented",
                          "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    from cqgen import CONFIGS, lfr_graph
    from paper_1507_05492_amd import cq

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.workload == "batch256":
        return bench_batch(args, log)
    if args.workload == "serve":
        return bench_serve(args, log)

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del src, dst

    params = CONFIGS[args.workload]
    t = time.perf_counter()
    g = lfr_graph(params, args.seed, device="cuda")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    n, nnz, L = g.n, g.nnz, g.num_labels
    log(f"graph {args.workload}: n={n} nnz={nnz} K={L} generated in {gen_s:.1f}s")

    ctx = cq.Context(0)
    labels = g.labels

    def timed_run(graph, steps, warmup, labels=labels, L=L):
        """Warmup, then a few steps with every stage timed (the stage breakdown and the
        dominant stage), then the timed steps with events around the dominant stage only:
        each timed stage costs a few microseconds of device time.  Returns the result,
        ms per timed step, the dominant stage, its average ms in the timed steps, and the
        breakdown {stage: ms}."""
        ws = ctx.workspace(graph.workspace_size(L))
        for _ in range(warmup):
            cq.score_partition(graph, labels, L, workspace=ws)
        cq.cq_context_enable_timing(ctx.handle, True)
        for _ in range(max(3, steps // 4)):
            cq.score_partition(graph, labels, L, workspace=ws)
        breakdown = {k: v[0] / v[1] for k, v in cq.cq_context_stage_times(ctx.handle).items()}
        dom = max(breakdown, key=breakdown.get)
        cq.cq_context_time_stages(ctx.handle, 1 << cq.stage_id(dom))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res, _, _ = cq.score_partition(graph, labels, L, workspace=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tot, cnt = cq.cq_context_stage_times(ctx.handle)[dom]
        cq.cq_context_enable_timing(ctx.handle, False)
        return res, (t1 - t0) * 1e3 / steps, dom, tot / cnt, breakdown

    # reference: the graph kept in its input node order
    other = "input" if args.order == "locality" else "locality"
    gref = cq.Graph(ctx, g.row_ptr, g.col_idx, reorder=(other == "locality"))
    r_ref, ms_ref, _, _, _ = timed_run(gref, max(3, args.steps // 4), 1)
    gref.close()

    torch.cuda.synchronize()
    t = time.perf_counter()
    graph = cq.Graph(ctx, g.row_ptr, g.col_idx, reorder=(args.order == "locality"))
    load_ms = (time.perf_counter() - t) * 1e3
    log(f"graph load ({args.order} order): {load_ms:.1f} ms")
    ws = ctx.workspace(graph.workspace_size(L))
    r, ms_per_step, dom, dom_ms, stage_avg = timed_run(graph, args.steps, args.warmup)
    assert r_ref == r, "results differ between storage orders"
    gedges = nnz / (ms_per_step * 1e-3) / 1e9
    # The steps above are synchronous calls: each one waits for its result struct in host
    # memory.  The same steps back to back on the stream, each result left in device
    # memory (cq_score_partition_async), give the device-side rate.
    import ctypes
    rsz = ctypes.sizeof(cq.ScoreResult)
    dres = torch.empty(rsz, dtype=torch.uint8, device="cuda")

    def one_async():  # raises on an error status
        cq.cq_score_partition_async(ctx.handle, graph.handle, labels.data_ptr(), L, ws.data_ptr(), ws.numel(),
                                    dres.data_ptr())

    for _ in range(3):
        one_async()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_async()
    torch.cuda.synchronize()
    ms_async = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"{ms_async:.3f} ms/step back to back without waiting for each result")
    log(f"{ms_per_step:.3f} ms/step, {gedges:.1f} GEdges/s; {dom} {dom_ms:.3f} ms; stages (all timed) " +
        ", ".join(f"{k}={v:.3f}ms" for k, v in stage_avg.items()))
    blocked = graph.stats["reordered"] == cq.CQ_GRAPH_REORDER  # renumbered and stored in column blocks
    kernel_of = kernel_names(L, blocked)
    abytes = algorithmic_bytes(n, nnz)
    achieved = abytes / (dom_ms * 1e-3) / 1e9
    roofline = {
        "bound": "hbm", "kernel": kernel_of.get(dom, dom), "stage": dom,
        "avg_ms": round(dom_ms, 4),
        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "algorithmic_bytes": abytes,
        "step_frac": round(abytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "traffic": traffic_for(kernel_of.get(dom, dom)),
        "stage_ms_all_timed": {k: round(v, 4) for k, v in stage_avg.items()},
    }

    # comparison path on the same node set (ground truth vs 10% reassigned), for context
    from cqgen import perturb_labels
    pert = perturb_labels(labels, L, 0.10, 1010)
    cws = ctx.workspace(max(cq.cq_compare_workspace_size(n, L, L), ws.numel()))
    for _ in range(2):
        cr, _ = cq.compare_partitions(ctx, labels, L, pert, L, workspace=cws)
    torch.cuda.synchronize()
    tc = time.perf_counter()
    csteps = max(3, args.steps // 4)
    for _ in range(csteps):
        cr, _ = cq.compare_partitions(ctx, labels, L, pert, L, workspace=cws)
    torch.cuda.synchronize()
    cmp_ms = (time.perf_counter() - tc) * 1e3 / csteps

    # the same graph with seeded symmetric edge weights (weighted Q/Qds/measures), for
    # context; weighted scoring takes at most WEIGHTED_MAX_LABELS label ids
    wres, wms = None, None
    if L <= WEIGHTED_MAX_LABELS:
        from cqgen import edge_weights
        wts = edge_weights(g.row_ptr, g.col_idx, args.seed)
        wgraph = cq.Graph(ctx, g.row_ptr, g.col_idx, reorder=(args.order == "locality"), weights=wts)
        wsteps = max(3, args.steps // 4)
        wres, wms, _, _, wstages = timed_run(wgraph, wsteps, 2)
        wgraph.close()
        del wts
        log(f"weighted: {wms:.3f} ms/step; stages (all timed) " + ", ".join(f"{k}={v:.3f}ms" for k, v in wstages.items()))

    # partitions that do not follow the stored node order, on the same loaded graph
    parts = {}
    if args.workload == "l10m" and not args.no_extra:
        from cqgen import random_labels
        for name, lab in (("reassigned_30pct", perturb_labels(labels, L, 0.30, 3030)),
                          ("random", random_labels(n, L, 3131, device="cuda"))):
            pr, pms, pdom, pdom_ms, pst = timed_run(graph, max(5, args.steps // 4), 2, labels=lab)
            parts[name] = {"ms_per_step": round(pms, 4), "GEdges_per_s": round(nnz / (pms * 1e-3) / 1e9, 2),
                           "Q": pr["Q"], "dominant": pdom, "stage_ms_all_timed": {k: round(v, 4) for k, v in pst.items()},
                           "labels": lab}
            log(f"partition {name}: {pms:.3f} ms/step; " + ", ".join(f"{k}={v:.3f}ms" for k, v in pst.items()))

    cpu = None
    check = None
    cpu_threaded = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle.parity import score_mismatches

        rp, ci, lab = g.row_ptr.cpu().numpy(), g.col_idx.cpu().numpy(), labels.cpu().numpy()
        oracle.lib()
        log("oracle on the host (full graph, one thread)")
        t = time.perf_counter()
        o = oracle.score(rp, ci, lab, L, want_pairs=False)
        cpu_s = time.perf_counter() - t
        host = host_info()
        cpu = {"value": round(nnz / cpu_s / 1e9, 5), "unit": "GEdges/s", "cores": 1, "kind": "oracle",
               "sample": f"whole {args.workload} graph (n={n}, 2|E|={nnz}), one partition, single-threaded C oracle",
               "seconds": round(cpu_s, 2), **host}
        bad = score_mismatches(r, o.result)
        check = "match" if not bad else "MISMATCH: " + "; ".join(bad)
        for name, pt in parts.items():
            op = oracle.score(rp, ci, pt["labels"].cpu().numpy(), L, want_pairs=False)
            pr, _, _ = cq.score_partition(graph, pt["labels"], L)
            bad = score_mismatches(pr, op.result)
            pt["oracle_check"] = "match" if not bad else "MISMATCH: " + "; ".join(bad)
        cpu_threaded = threaded_cpu(rp, ci, lab, L, nnz, log)
    for pt in parts.values():
        pt.pop("labels", None)

    out = {
        "metric": METRIC, "value": round(gedges, 2), "unit": "GEdges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"lfr_{args.workload}", "n": n, "nnz": nnz, "m": nnz // 2, "communities": L,
                   "seed": args.seed, "partition": "ground truth", "avg_degree": round(nnz / n, 2),
                   "max_degree": g.stats["max_degree"], "mu": params.mu, "epilogue": "f64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "aux": {"graph_order": args.order, "graph_load_ms": round(load_ms, 2), "generate_s": round(gen_s, 2),
                f"ms_per_step_{other}_order": round(ms_ref, 4),
                "ms_per_step_async": round(ms_async, 4),
                "GEdges_per_s_async": round(nnz / (ms_async * 1e-3) / 1e9, 2),
                "compare_ms": round(cmp_ms, 4), "compare_Gnodes_per_s": round(n / (cmp_ms * 1e-3) / 1e9, 3),
                "weighted_ms_per_step": None if wms is None else round(wms, 4),
                "weighted_GEdges_per_s": None if wms is None else round(nnz / (wms * 1e-3) / 1e9, 2),
                "weighted_Q": None if wres is None else wres["Q"], "weighted_Qds": None if wres is None else wres["Qds"],
                "oracle_check": check,
                "Q": r["Q"], "Qds": r["Qds"],
                "partitions": parts or None,
                "cpu_threaded": cpu_threaded},
    }
    graph.close()
    del ws, cws
    if args.workload == "l10m" and not args.no_extra and not args.no_s100m:
        torch.cuda.empty_cache()
        out["aux"]["s100m"] = big_graph_leg(args, ctx, cq, timed_run_factory, log)
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def host_info() -> dict:
    import cpubase

    return {"host_cores": os.cpu_count(), "host_threads_usable": cpubase.host_threads(), "cpu_model": cpubase.cpu_model()}


def threaded_cpu(rp, ci, lab, L, nnz, log) -> dict:
    """The multi-threaded CPU scoring (cpubase, the paper's community-per-thread layout) at
    one thread and at all usable host threads: speedup T1/Tp and efficiency speedup/p as
    the paper defines them (Eqs. 10-11)."""
    import cpubase

    T = cpubase.host_threads()
    cpubase.lib()
    times = {}
    for t in sorted({1, T}):
        log(f"threaded CPU scoring, {t} thread(s)")
        t0 = time.perf_counter()
        cpubase.score(rp, ci, lab, L, t)
        times[t] = time.perf_counter() - t0
    sp = times[1] / times[T]
    return {"threads": T, "seconds_1": round(times[1], 3), f"seconds_{T}": round(times[T], 3),
            "GEdges_per_s": round(nnz / times[T] / 1e9, 4), "speedup": round(sp, 2), "efficiency": round(sp / T, 3),
            "kind": "pthreads, communities assigned to threads by id (the paper's shared-memory layout)",
            **host_info()}


def timed_run_factory(ctx, cq, graph, labels, L):
    """Same timing protocol as the main line's timed_run, for another graph."""
    import torch

    def run(steps, warmup):
        ws = ctx.workspace(graph.workspace_size(L))
        for _ in range(warmup):
            cq.score_partition(graph, labels, L, workspace=ws)
        cq.cq_context_enable_timing(ctx.handle, True)
        for _ in range(max(2, steps // 2)):
            cq.score_partition(graph, labels, L, workspace=ws)
        breakdown = {k: v[0] / v[1] for k, v in cq.cq_context_stage_times(ctx.handle).items()}
        dom = max(breakdown, key=breakdown.get)
        cq.cq_context_time_stages(ctx.handle, 1 << cq.stage_id(dom))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res, _, _ = cq.score_partition(graph, labels, L, workspace=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tot, cnt = cq.cq_context_stage_times(ctx.handle)[dom]
        cq.cq_context_enable_timing(ctx.handle, False)
        return res, (t1 - t0) * 1e3 / steps, dom, tot / cnt, breakdown

    return run


def big_graph_leg(args, ctx, cq, factory, log) -> dict:
    """The 100M-node graph (average degree 10, maximum 1,000, communities 50-10,000,
    mixing 0.3): step time, dominant kernel against the HBM roofline, the comparison of
    two 1e8-node partitions, and the oracle's check of the score."""
    import torch

    from cqgen import CONFIGS, lfr_graph, perturb_labels

    t = time.perf_counter()
    g = lfr_graph(CONFIGS["s100m"], args.seed, device="cuda")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    n, nnz, L = g.n, g.nnz, g.num_labels
    log(f"graph s100m: n={n} nnz={nnz} K={L} generated in {gen_s:.1f}s")
    t = time.perf_counter()
    graph = cq.Graph(ctx, g.row_ptr, g.col_idx, reorder=True)
    load_ms = (time.perf_counter() - t) * 1e3
    r, ms, dom, dom_ms, st = factory(ctx, cq, graph, g.labels, L)(5, 1)
    blocked = graph.stats["reordered"] == cq.CQ_GRAPH_REORDER
    abytes = algorithmic_bytes(n, nnz)
    log(f"s100m: {ms:.3f} ms/step; " + ", ".join(f"{k}={v:.3f}ms" for k, v in st.items()))
    pert = perturb_labels(g.labels, L, 0.10, 1010)
    cws = ctx.workspace(cq.cq_compare_workspace_size(n, L, L))
    cq.compare_partitions(ctx, g.labels, L, pert, L, workspace=cws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        cq.compare_partitions(ctx, g.labels, L, pert, L, workspace=cws)
    torch.cuda.synchronize()
    cmp_ms = (time.perf_counter() - t) * 1e3 / 3
    del cws, pert
    graph.close()
    out = {"workload": "lfr_s100m", "n": n, "nnz": nnz, "communities": L, "seed": args.seed,
           "max_degree": g.stats["max_degree"], "graph_order": "locality (no column blocks above 2^24 nodes)",
           "graph_load_ms": round(load_ms, 1), "ms_per_step": round(ms, 4),
           "GEdges_per_s": round(nnz / (ms * 1e-3) / 1e9, 2),
           "roofline": {"bound": "hbm", "kernel": kernel_names(L, blocked).get(dom, dom), "stage": dom,
                        "avg_ms": round(dom_ms, 4), "achieved": round(abytes / (dom_ms * 1e-3) / 1e9, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(abytes / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "algorithmic_bytes": abytes, "step_frac": round(abytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
           "stage_ms_all_timed": {k: round(v, 4) for k, v in st.items()},
           "compare_ms": round(cmp_ms, 3), "compare_Gnodes_per_s": round(n / (cmp_ms * 1e-3) / 1e9, 3),
           "Q": r["Q"], "Qds": r["Qds"], "oracle_check": None}
    if not args.no_cpu_baseline:
        import oracle
        from oracle.parity import score_mismatches

        log("s100m: oracle on the host (whole graph, one thread)")
        t = time.perf_counter()
        o = oracle.score(g.row_ptr.cpu().numpy(), g.col_idx.cpu().numpy(), g.labels.cpu().numpy(), L, want_pairs=False)
        out["oracle_seconds"] = round(time.perf_counter() - t, 1)
        bad = score_mismatches(r, o.result)
        out["oracle_check"] = "match" if not bad else "MISMATCH: " + "; ".join(bad)
    del g
    torch.cuda.empty_cache()
    return out


def bench_batch(args, log) -> int:
    """256 LFR-style graphs (n log-uniform in [5e3, 5e5], average degree U[10, 30],
    mixing U[0.1, 0.5], seeds 31000+i) x 4 partitions (ground truth and 5/15/30 %
    reassigned) = 1024 tasks.  One step = one replay of the batch's HIP graph; compared
    with the same 1024 tasks scored one call at a time (synchronous calls, and
    asynchronous calls back to back on one stream)."""
    import ctypes

    import numpy as np
    import torch

    from cqgen import LFRParams, lfr_graph, perturb_labels
    from paper_1507_05492_amd import cq

    rng = np.random.default_rng(31)
    ctx = cq.Context(0)
    t = time.perf_counter()
    tasks, graphs = [], []
    total_nnz = 0
    for i in range(256):
        n = int(np.exp(rng.uniform(np.log(5e3), np.log(5e5))))
        avg = float(rng.uniform(10, 30))
        mu = float(rng.uniform(0.1, 0.5))
        p = LFRParams(n, avg, int(5 * avg), 2.0, 1.0, 20, max(40, min(1000, n // 5)), mu)
        g = lfr_graph(p, 31000 + i, device="cuda")
        G = cq.Graph(ctx, g.row_ptr, g.col_idx, reorder=(args.order == "locality"))
        graphs.append((g, G))
        parts = [g.labels] + [perturb_labels(g.labels, g.num_labels, f, 310000 + 10 * i + k).contiguous()
                              for k, f in enumerate((0.05, 0.15, 0.30))]
        for lab in parts:
            tasks.append((G, lab, g.num_labels))
            total_nnz += g.nnz
        if (i + 1) % 32 == 0:
            log(f"batch: {i + 1} of 256 graphs generated and loaded")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    log(f"batch: {len(tasks)} tasks over {len(graphs)} graphs, sum 2|E| = {total_nnz}, built in {gen_s:.1f}s")

    t = time.perf_counter()
    b = cq.Batch(ctx, tasks, autotune=True, use_graph=True)
    plan_s = time.perf_counter() - t
    for _ in range(args.warmup):
        res = b.run_sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t0) * 1e3 / args.steps
    res = b.run_sync()

    # one call at a time, asynchronous and back to back on one stream
    ws_bytes = max(G.workspace_size(L) for G, _, L in tasks)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    rsz = ctypes.sizeof(cq.ScoreResult)
    outs = torch.empty(len(tasks) * rsz, dtype=torch.uint8, device="cuda")

    def one_at_a_time_async():
        for i, (G, lab, L) in enumerate(tasks):
            cq.cq_score_partition_async(ctx.handle, G.handle, lab.data_ptr(), L, ws.data_ptr(), ws_bytes,
                                        outs.data_ptr() + i * rsz)

    one_at_a_time_async()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(1, args.steps // 4)
    for _ in range(reps):
        one_at_a_time_async()
    torch.cuda.synchronize()
    ms_async = (time.perf_counter() - t0) * 1e3 / reps
    host = outs.cpu().numpy().tobytes()
    async_res = [cq.as_dict(cq.ScoreResult.from_buffer_copy(host[i * rsz:(i + 1) * rsz])) for i in range(len(tasks))]
    # one call at a time, synchronous (what a per-request caller does)
    t0 = time.perf_counter()
    sync_res = [cq.score_partition(G, lab, L, workspace=ws)[0] for G, lab, L in tasks]
    torch.cuda.synchronize()
    ms_sync = (time.perf_counter() - t0) * 1e3
    equal = all({k: v for k, v in r.items() if k != "status"} == a for r, a in zip(res, async_res))
    equal = equal and all({k: v for k, v in r.items() if k != "status"} == {k: v for k, v in s_.items() if k != "status"}
                          for r, s_ in zip(res, sync_res))
    out = {
        "metric": "batched GEdges/s, 1024 (graph, partition) tasks in one HIP graph replay",
        "value": round(total_nnz / (ms_batch * 1e-3) / 1e9, 2), "unit": "GEdges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_batch, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "lfr_batch_256x4", "graphs": len(graphs), "tasks": len(tasks),
                   "sum_nnz": total_nnz, "sum_n": sum(g.n for g, _ in graphs) * 4, "graph_order": args.order},
        "one_at_a_time": {"async_ms": round(ms_async, 3), "sync_ms": round(ms_sync, 3),
                          "speedup_vs_async": round(ms_async / ms_batch, 2),
                          "speedup_vs_sync": round(ms_sync / ms_batch, 2), "results_equal": bool(equal)},
        "tuning": b.tuning, "plan_s": round(plan_s, 3), "build_s": round(gen_s, 1),
    }
    print(json.dumps(out), flush=True)
    b.close()
    return 0


def bench_serve(args, log) -> int:
    """Serving: a resident LFR-style graph of 100M nodes (average degree 10, maximum 1,000,
    community sizes 50-10,000, mixing 0.3) plus 64 graphs with n log-uniform in
    [1e4, 1e6]; requests are 70 % scoring / 30 % comparison, 10 % of them on the big
    graph, with label sets = ground truth or 5/15/30 % reassigned (pinned host memory).
    Saturated throughput is measured with all requests submitted at once; then Poisson
    arrivals at 25/50/75/90 % of it.  The same request streams go to a one-at-a-time
    FIFO server (one slot, no grouping) for comparison."""
    import threading

    import numpy as np
    import torch

    from cqgen import CONFIGS, LFRParams, lfr_graph, perturb_labels
    from paper_1507_05492_amd import cq

    rng = np.random.default_rng(41)
    ctx = cq.Context(0)
    t = time.perf_counter()
    graphs = []  # (n, nnz, num_labels, Graph, [pinned label sets])

    def add(g, reorder=True):
        G = cq.Graph(ctx, g.row_ptr, g.col_idx, reorder=reorder)
        sets = [g.labels] + [perturb_labels(g.labels, g.num_labels, f, 4100 + int(100 * f)) for f in (0.05, 0.15, 0.30)]
        pins = [s_.cpu().pin_memory() for s_ in sets]
        graphs.append((g.n, g.nnz, g.num_labels, G, pins))

    big = lfr_graph(CONFIGS["s100m"], 41, device="cuda")
    add(big)
    big_nnz = big.nnz
    del big
    for i in range(64):
        n = int(np.exp(rng.uniform(np.log(1e4), np.log(1e6))))
        avg = float(rng.uniform(10, 30))
        p = LFRParams(n, avg, int(5 * avg), 2.0, 1.0, 20, max(40, min(1000, n // 5)), 0.3)
        add(lfr_graph(p, 4200 + i, device="cuda"))
    torch.cuda.synchronize()
    log(f"serve: 1 + 64 resident graphs built in {time.perf_counter() - t:.1f}s (big graph 2|E| = {big_nnz})")

    def make_stream(m, seed):
        r = np.random.default_rng(seed)
        out = []
        for _ in range(m):
            gi = 0 if r.random() < 0.10 else int(r.integers(1, len(graphs)))
            kind = "score" if r.random() < 0.70 else "compare"
            li = int(r.integers(0, 4)) if kind == "score" else int(r.integers(1, 4))
            out.append((kind, gi, li))
        return out

    def entries(req):
        kind, gi, _ = req
        n, nnz = graphs[gi][0], graphs[gi][1]
        return nnz if kind == "score" else n

    def run(server, stream, rate, arrival_seed=7):
        """rate None: submit everything at once.  Returns (wall s, per-request results)."""
        tickets = [None] * len(stream)
        arrivals = None
        if rate:
            gaps = np.random.default_rng(arrival_seed).exponential(1.0 / rate, len(stream))
            arrivals = np.cumsum(gaps)
        server.reset_stats()
        t0 = time.perf_counter()

        def submitter():
            for i, (kind, gi, li) in enumerate(stream):
                if arrivals is not None:
                    while time.perf_counter() - t0 < arrivals[i]:
                        pass
                n, nnz, L, G, pins = graphs[gi]
                if kind == "score":
                    tickets[i] = server.submit_score(G, pins[li], L)
                else:
                    tickets[i] = server.submit_compare(pins[0], L, pins[li], L)

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        outs = [server.wait(tk) for tk in tickets]
        wall = time.perf_counter() - t0
        return wall, outs, server.stats()

    seeds = [int(x) for x in args.serve_seeds.split(",") if x]
    fracs = (0.25, 0.50, 0.75, 0.90)
    points = {}
    for name, slots, batch in (("continuous", 4, 32), ("fifo_one_at_a_time", 1, 1)):
        srv = cq.Server(ctx, num_slots=slots, max_batch=batch, memory_budget=24 << 30, small_nnz=8_000_000)
        warm = make_stream(64, 1)
        run(srv, warm, None)
        res = {"per_seed": {}}
        sat_rates = []
        for seed in seeds:
            sat_stream = make_stream(args.serve_requests, 100 + seed)
            wall, outs, st = run(srv, sat_stream, None)
            assert all(o["status"] == cq.CQ_OK for o in outs)
            sat_rates.append(len(sat_stream) / wall)
            res["per_seed"][str(seed)] = {
                "saturated_req_per_s": round(len(sat_stream) / wall, 1),
                "saturated_GEdges_per_s": round(sum(entries(q) for q in sat_stream) / wall / 1e9, 2),
                "saturated_p50_ms": round(st["p50_ms"], 3), "saturated_p99_ms": round(st["p99_ms"], 3),
                "launches": st["launches"], "grouped_requests": st["grouped_requests"], "loads": []}
            log(f"serve[{name}] seed {seed} saturated: {len(sat_stream) / wall:.1f} req/s "
                f"({wall:.1f} s for {len(sat_stream)} requests)")
        res["saturated_req_per_s"] = round(float(np.mean(sat_rates)), 1)
        # the same absolute arrival rates for both servers: fractions of the continuous server's saturation
        base_rate = points.get("continuous", {}).get("saturated_req_per_s", res["saturated_req_per_s"])
        for seed in seeds:
            for frac in fracs:
                rate = frac * base_rate
                stream = make_stream(args.serve_requests, seed)
                wall, outs, st = run(srv, stream, rate, arrival_seed=1000 + seed)
                assert all(o["status"] == cq.CQ_OK for o in outs)
                res["per_seed"][str(seed)]["loads"].append({
                    "offered_req_per_s": round(rate, 1), "fraction_of_continuous_saturation": frac,
                    "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                    "achieved_req_per_s": round(len(stream) / wall, 1), "seconds": round(wall, 1),
                    "GEdges_per_s": round(sum(entries(q) for q in stream) / wall / 1e9, 2)})
                log(f"serve[{name}] seed {seed} load {frac:.2f}: {wall:.1f} s, p50 {st['p50_ms']:.2f} ms "
                    f"p99 {st['p99_ms']:.2f} ms")
        res["loads"] = []
        for k, frac in enumerate(fracs):
            per = [res["per_seed"][str(sd)]["loads"][k] for sd in seeds]
            p99 = [x["p99_ms"] for x in per]
            p50 = [x["p50_ms"] for x in per]
            res["loads"].append({"fraction_of_continuous_saturation": frac,
                                 "offered_req_per_s": per[0]["offered_req_per_s"],
                                 "p50_ms_mean": round(float(np.mean(p50)), 3),
                                 "p99_ms_mean": round(float(np.mean(p99)), 3),
                                 "p99_ms_min": min(p99), "p99_ms_max": max(p99),
                                 "achieved_req_per_s_mean": round(float(np.mean([x["achieved_req_per_s"] for x in per])), 1)})
        points[name] = res
        srv.close()

    # results in the mix equal results alone (a sample of the saturated stream)
    check = make_stream(40, 2)
    srv = cq.Server(ctx, num_slots=4, max_batch=32, memory_budget=24 << 30, small_nnz=8_000_000)
    _, outs, _ = run(srv, check, None)
    same = True
    for (kind, gi, li), o in zip(check, outs):
        n, nnz, L, G, pins = graphs[gi]
        if kind == "score":
            a, _, _ = cq.score_partition(G, pins[li].cuda(), L)
            got = o["score"]
        else:
            a, _ = cq.compare_partitions(ctx, pins[0].cuda(), L, pins[li].cuda(), L)
            got = o["compare"]
        a.pop("status")
        same = same and got == a
    srv.close()
    c = points["continuous"]
    out = {
        "metric": "served p50/p99 latency (ms) at 75% of saturation, continuous batching",
        "value": c["loads"][2]["p99_ms_mean"], "unit": "ms (p99, mean over stream seeds)", "n_gpus": 1,
        "higher_is_better": False,
        "data": "synthetic", "dtype": "u32",
        "config": {"workload": "lfr_serve_100m_plus_64", "big_graph_nnz": big_nnz, "graphs": len(graphs),
                   "requests_per_point": args.serve_requests, "stream_seeds": seeds, "mix": "70% score / 30% compare, 10% on the 100M graph"},
        "continuous": points["continuous"], "fifo_one_at_a_time": points["fifo_one_at_a_time"],
        "results_same_alone_and_in_mix": bool(same),
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
