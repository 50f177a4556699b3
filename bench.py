#!/usr/bin/env python3
"""Benchmark of the streamed subgraph pass on one MI355X.

Headline workload (the largest single-GPU one): connected components by
min-label propagation on a seeded R-MAT graph of scale 24 (edge factor 32,
symmetrized: 1.02 G arcs), in-edge pages, with the library's page slots
capped at 1/4 of the graph bytes so the pages stream from pinned host memory
every pass (Seraph's out-of-GPU-memory regime); its uniform-random twin
(same vertex and edge counts, the dense always-active regime) is the second
leg. The library numbers vertices internally by descending degree (results
are returned in the input's ids). One step = one CC solve to convergence
through the C ABI (sr_run), labels checked bit-exact against union-find.

Prints one JSON line: solve GTEPS (arcs / time to convergence, page
streaming included as the paper times it), the roofline of the sweep kernel
(its algorithmic bytes over its HIP-event time, against the 8 TB/s HBM
peak), the host-to-device rate of the page stream, and the CPU oracle timed
on the host: synchronous label propagation over all host cores (the CPU
baseline, core count and CPU model stated) and single-thread union-find.
Further legs: streamed SSSP on R-MAT scale 22, PageRank on scale 16, the
batched PPR set and the query server.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
H2D_PEAK_GBS = 64.0        # PCIe 5.0 x16, one direction, nominal
METRIC = "GTEPS & HBM GB/s fraction per subgraph pass; batched/served vs plain solves/s"


def kernel_traffic(name):
    """HBM traffic of a launch of the sweep kernel, from the rocprofv3 counter
    summary committed under profiles/ (FETCH_SIZE and WRITE_SIZE per dispatch,
    scaled by the copy-kernel calibration). None when the kernel sources have
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name + "_traffic.json")
    if not os.path.exists(path):
        return None, None
    j = json.load(open(path))
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1806_00762_amd", "csrc", f), "rb").read())
    if h.hexdigest() != j["source_sha256"]:
        return None, None
    return j["traffic_bytes_per_launch"], j["algo_bytes_per_launch_same_runs"]


def sssp_inner(args):
    """Re-sweeps per window step of the streamed SSSP leg: 4 (under the
    deterministic schedule 2 needs a fifth pass and 8 re-sweeps windows
    whose gains later passes would make anyway: 3.02 / 3.74 / 3.52 GTEPS)."""
    return args.inner or 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info():
    """CPU of the host the benchmark runs on: logical CPUs, the ones this
    process may use, and the model name."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "model": model}


def sync():
    import torch
    torch.cuda.synchronize()


def _cc_leg(args, g, workload, traffic_name, cpu=True):
    """Streamed CC on a symmetric graph: pages within a quarter of the graph
    bytes (plus the vertex state: label, predictor state and in-edge bit per
    vertex), strong prediction, the heterogeneous model of Section 3.1 (the
    host takes over once the vertices a pass would attempt are few), timed
    solves; labels checked bit-exact against the oracle's union-find (timed,
    one thread) and, with cpu=True, the multi-core CPU baseline timed too."""
    import oracle
    import paper_1806_00762_amd as sr
    gbytes = 4 * (g.n + 1) + 4 * g.m
    budget = gbytes // 4 + 5 * g.n + g.n // 8 + (1 << 20)
    ctx = sr.Context(0, budget)
    t = time.perf_counter()
    G = ctx.load(g, symmetric=True, reorder=args.order == "degree")
    G.partition(0, args.slots)
    info = G.info()
    log(f"[bench] {workload}: loaded+partitioned in {time.perf_counter() - t:.1f}s: {info['num_parts']} pages, "
        f"budget {budget / 1e6:.1f} MB, graph {gbytes / 1e6:.1f} MB")
    # the fixed schedule (a window is re-swept until a sweep changes nothing, at
    # most max_inner_iters times) does not depend on when a copy lands, so a
    # profiled run makes the same sweeps as the timed one
    inner = args.inner or 8
    run_kw = dict(pvu="strong", max_inner_iters=inner, force_stream=True, copy_depth=args.copy_depth,
                  wide_pages=args.wide_pages, deterministic=args.schedule == "fixed",
                  hetero=not args.no_host_stage)
    device_only = None
    if not args.no_host_stage:
        # the same solves with device passes only (the pass that proves
        # convergence streams every page again), before the timed ones, so
        # that a profile's last launches are those of the timed solves
        dkw = dict(run_kw, hetero=False)
        G.run("cc", **dkw)
        sync()
        t1 = time.perf_counter()
        dst = [G.run("cc", **dkw) for _ in range(args.steps)]
        sync()
        del1 = time.perf_counter() - t1
        dlab = G.values()
        device_only = {"gteps": round(g.m * args.steps / del1 / 1e9, 4),
                       "ms_per_step": round(del1 * 1e3 / args.steps, 3), "passes_per_solve": dst[-1]["passes"],
                       "h2d_bytes_per_solve": sum(x["h2d_bytes"] for x in dst) // args.steps}
        log(f"[bench] {workload} device passes only: {device_only}")
    for i in range(args.warmup):
        st = G.run("cc", **run_kw)
        log(f"[bench] {workload} warmup {i}: {st['wall_ms']:.1f} ms, passes {st['passes']}")
    sync()
    t0 = time.perf_counter()
    stats = [G.run("cc", **run_kw) for _ in range(args.steps)]
    sync()
    elapsed = time.perf_counter() - t0
    lab = G.values()
    st = stats[-1]
    if device_only is not None:
        assert np.array_equal(dlab, lab)
    log(f"[bench] {workload}: {elapsed * 1e3 / args.steps:.1f} ms per solve, passes {st['passes']} sweeps "
        f"{st['sweeps']} kernel {st['kernel_ms']:.1f} ms h2d {st['h2d_ms']:.1f} ms ({st['h2d_bytes'] / 1e9:.2f} GB)")
    sweep_ms = sum(x["sweep_kernel_ms"] for x in stats)
    kernel_ms = sum(x["kernel_ms"] for x in stats)
    algo_bytes = sum(x["algo_bytes"] for x in stats)
    sweeps = sum(x["sweeps"] for x in stats)
    launches = sum(x["sweep_launches"] for x in stats)
    h2d_bytes = sum(x["h2d_bytes"] for x in stats)
    h2d_ms = sum(x["h2d_ms"] for x in stats)
    scanned = sum(x["edges_scanned"] for x in stats)
    narrow = sum(x["edges_narrow"] for x in stats)
    achieved = algo_bytes / (sweep_ms * 1e-3) / 1e9
    traffic, traffic_algo = kernel_traffic(traffic_name)
    out = {
        "value": round(g.m * args.steps / elapsed / 1e9, 4),
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "config": {"workload": workload, "n": g.n, "m": g.m, "pages": info["num_parts"], "slots": args.slots,
                   "device_budget_bytes": budget, "graph_bytes": gbytes, "pvu": "strong",
                   "max_inner_iters": inner, "copy_depth": args.copy_depth,
                   "vertex_order": "degree descending (labels in input ids)" if args.order == "degree"
                   else "input",
                   "page_image": "full-width" if args.wide_pages else "split-width when smaller",
                   "schedule": "fixed re-entry (until no change, <= max_inner_iters)" if args.schedule == "fixed"
                   else "re-entry until the next page lands",
                   "narrow_edge_frac": round(narrow / max(scanned, 1), 4),
                   "host_stage": "off" if args.no_host_stage else
                   "on (the host pulls the vertices a pass would attempt once at most n/512 remain)"},
        "roofline": {"bound": "hbm", "kernel": "sweep_kernel<CC>",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "target_frac": 0.6, "traffic": traffic,
                     "traffic_algo_bytes_per_launch": traffic_algo,
                     # per launch of the sweep kernel (what a kernel trace averages over), a
                     # launch into a window that had stopped changing included
                     "launches": launches, "sweeps": sweeps,
                     "algo_bytes_per_launch": round(algo_bytes / max(launches, 1)),
                     "avg_launch_us": round(sweep_ms * 1e3 / max(launches, 1), 2),
                     "close_kernel_avg_us": round((kernel_ms - sweep_ms) * 1e3 / max(launches, 1), 2)},
        "h2d": {"achieved": round(h2d_bytes / (h2d_ms * 1e-3) / 1e9, 2) if h2d_ms else None,
                "peak": H2D_PEAK_GBS, "unit": "GB/s",
                "frac": round(h2d_bytes / (h2d_ms * 1e-3) / 1e9 / H2D_PEAK_GBS, 4) if h2d_ms else None,
                "bytes_per_solve": h2d_bytes // args.steps},
        "scan_gteps": round(scanned / (sweep_ms * 1e-3) / 1e9, 3),
        "passes_per_solve": st["passes"],
        "sweeps_per_solve": st["sweeps"],
        "timed_sweeps": sweeps,
        "kernel_busy_frac": round(kernel_ms / (elapsed * 1e3), 3),
        "host_stage": {"entries_per_solve": round(sum(x["sparse_entries"] for x in stats) / args.steps, 2),
                       "finished_solves": sum(x["sparse_stage"] for x in stats),
                       "list": st["sparse_frontier"], "edges_per_solve": st["sparse_relaxations"],
                       "rounds": st["sparse_rounds"], "value_bytes_copied": st["sparse_copy_bytes"],
                       "ms_per_solve": round(sum(x["sparse_ms"] for x in stats) / args.steps, 3)},
        "device_passes_only": device_only,
    }
    G.close()
    ctx.close()
    t = time.perf_counter()
    ref = oracle.cc(g)
    tu = time.perf_counter() - t
    out["parity"] = "bit-exact" if np.array_equal(ref, lab) else f"MISMATCH {int(np.sum(ref != lab))}"
    single = {"value": round(g.m / tu / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
              "sample": f"one union-find solve of the whole graph ({tu:.1f} s, one thread)"}
    if cpu and not args.no_cpu:
        t = time.perf_counter()
        lp, iters, used = oracle.cc_labelprop_parallel(g)
        tl = time.perf_counter() - t
        assert np.array_equal(lp, ref)
        out["cpu_baseline"] = {"value": round(g.m / tl / 1e9, 5), "unit": "GTEPS", "cores": used, "kind": "oracle",
                               "sample": f"one synchronous label-propagation solve of the whole graph over "
                                         f"{used} OpenMP threads ({iters} iterations, {tl:.1f} s), labels equal "
                                         f"to union-find",
                               "host": host_info(), "single_thread": single}
    else:
        out["cpu_single_thread"] = single
    log(f"[bench] {workload}: parity {out['parity']}, union-find {tu:.1f}s")
    return out


def bench_cc24(args):
    """The headline: streamed CC on the scale-24 R-MAT graph, then its uniform twin."""
    import gc
    import graphgen
    t = time.perf_counter()
    g = graphgen.recipes.cc_rmat_s24()
    log(f"[bench] generated rmat24 ef32 sym n={g.n} m={g.m} in {time.perf_counter() - t:.1f}s")
    head = _cc_leg(args, g, "cc_rmat24_ef32_sym_streamed_budget_quarter", "sweep_kernel_cc_rmat24_streamed")
    del g
    gc.collect()
    res = {
        "metric": METRIC,
        "value": head.pop("value"),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
    }
    res.update(head)
    if not args.no_twin:
        t = time.perf_counter()
        g = graphgen.recipes.cc_uniform_s24()
        log(f"[bench] generated uniform24 twin n={g.n} m={g.m} in {time.perf_counter() - t:.1f}s")
        twin = _cc_leg(args, g, "cc_uniform24_m2^29_sym_streamed_budget_quarter",
                       "sweep_kernel_cc_uniform24_streamed", cpu=False)
        twin["solve_gteps"] = twin.pop("value")
        res["uniform_twin"] = twin
        del g
        gc.collect()
    return res


def bench_sssp22(args):
    import graphgen
    import paper_1806_00762_amd as sr
    t = time.perf_counter()
    g = graphgen.recipes.sssp_s22()
    log(f"[bench] generated rmat22 n={g.n} m={g.m} in {time.perf_counter() - t:.1f}s")
    gbytes = 4 * (g.n + 1) + 8 * g.m
    budget = gbytes // 4
    ctx = sr.Context(0, budget)
    t = time.perf_counter()
    G = ctx.load(g, reorder=args.order == "degree")
    G.partition(0, args.slots)
    info = G.info()
    log(f"[bench] loaded+partitioned in {time.perf_counter() - t:.1f}s: {info['num_parts']} pages, "
        f"budget {budget / 1e6:.1f} MB, graph {gbytes / 1e6:.1f} MB")
    # the fixed schedule (see the CC leg) makes profiled runs sweep as the timed ones do
    inner = sssp_inner(args)
    run_kw = dict(source=0, pvu=args.pvu, max_inner_iters=inner, force_stream=True,
                  copy_depth=args.copy_depth, wide_pages=args.wide_pages,
                  deterministic=args.schedule == "fixed")
    for i in range(args.warmup):
        st = G.run("sssp", **run_kw)
        log(f"[bench] warmup {i}: {st['wall_ms']:.1f} ms, passes {st['passes']}")
    sync()
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        stats.append(G.run("sssp", **run_kw))
    sync()
    elapsed = time.perf_counter() - t0
    dist = G.values()
    for i, st in enumerate(stats):
        log(f"[bench] step {i}: wall {st['wall_ms']:.1f} ms passes {st['passes']} sweeps {st['sweeps']} "
            f"kernel {st['kernel_ms']:.2f} ms h2d {st['h2d_ms']:.1f} ms ({st['h2d_bytes'] / 1e6:.0f} MB)")
    kernel_ms = sum(s["kernel_ms"] for s in stats)
    sweep_ms = sum(s["sweep_kernel_ms"] for s in stats)
    algo_bytes = sum(s["algo_bytes"] for s in stats)
    sweeps = sum(s["sweeps"] for s in stats)
    launches = sum(s["sweep_launches"] for s in stats)
    h2d_bytes = sum(s["h2d_bytes"] for s in stats)
    h2d_ms = sum(s["h2d_ms"] for s in stats)
    scanned = sum(s["edges_scanned"] for s in stats)
    narrow = sum(s["edges_narrow"] for s in stats)
    # the sweep kernel alone moves the algorithmic bytes (events on its stream
    # around it; the one-block close kernel after it is reported separately)
    achieved = algo_bytes / (sweep_ms * 1e-3) / 1e9
    traffic, traffic_algo = kernel_traffic("sweep_kernel_sssp_rmat22_streamed")
    res = {
        "metric": METRIC,
        "value": round(g.m * args.steps / elapsed / 1e9, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "sssp_rmat22_ef16_w1-255_src0_streamed_budget_quarter",
                   "n": g.n, "m": g.m, "pages": info["num_parts"], "slots": args.slots,
                   "device_budget_bytes": budget, "graph_bytes": gbytes,
                   "pvu": args.pvu, "max_inner_iters": inner, "copy_depth": args.copy_depth,
                   "vertex_order": "in-degree descending (results in input ids)" if args.order == "degree"
                   else "input",
                   "page_image": "full-width" if args.wide_pages else "split-width",
                   "schedule": "fixed re-entry (until no change, <= max_inner_iters)" if args.schedule == "fixed"
                   else "re-entry until the next page lands",
                   "narrow_edge_frac": round(narrow / max(scanned, 1), 4)},
        "roofline": {"bound": "hbm", "kernel": "sweep_kernel<SSSP>",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "target_frac": 0.6, "traffic": traffic,
                     "traffic_algo_bytes_per_launch": traffic_algo,
                     # per launch of the sweep kernel (what a kernel trace averages over), a
                     # launch into a window that had stopped changing included
                     "launches": launches, "sweeps": sweeps,
                     "algo_bytes_per_launch": round(algo_bytes / max(launches, 1)),
                     "avg_launch_us": round(sweep_ms * 1e3 / max(launches, 1), 2),
                     "close_kernel_avg_us": round((kernel_ms - sweep_ms) * 1e3 / max(launches, 1), 2)},
        "h2d": {"achieved": round(h2d_bytes / (h2d_ms * 1e-3) / 1e9, 2) if h2d_ms else None,
                "peak": H2D_PEAK_GBS, "unit": "GB/s",
                "frac": round(h2d_bytes / (h2d_ms * 1e-3) / 1e9 / H2D_PEAK_GBS, 4) if h2d_ms else None,
                "bytes_per_solve": h2d_bytes // args.steps},
        "scan_gteps": round(scanned / (sweep_ms * 1e-3) / 1e9, 3),
        "passes_per_solve": stats[-1]["passes"],
        "sweeps_per_solve": stats[-1]["sweeps"],
    }
    if not args.no_other:
        other = "weak" if args.pvu == "strong" else "strong"
        okw = dict(run_kw, pvu=other)
        G.run("sssp", **okw)
        sync()
        t0 = time.perf_counter()
        ost = [G.run("sssp", **okw) for _ in range(args.steps)]
        sync()
        oel = time.perf_counter() - t0
        assert np.array_equal(G.values(), dist)
        res["pvu_" + other] = {"solve_gteps": round(g.m * args.steps / oel / 1e9, 4),
                               "ms_per_solve": round(oel * 1e3 / args.steps, 3),
                               "passes_per_solve": ost[-1]["passes"],
                               "h2d_bytes_per_solve": ost[-1]["h2d_bytes"],
                               "sweep_GBps": round(sum(s["algo_bytes"] for s in ost) /
                                                   (sum(s["sweep_kernel_ms"] for s in ost) * 1e-3) / 1e9, 1)}
    if args.order == "degree" and not args.no_other and args.input_order:
        # the same solve with the input's vertex numbering
        ctxn = sr.Context(0, budget)
        Gn = ctxn.load(g)
        Gn.partition(0, args.slots)
        Gn.run("sssp", **run_kw)
        sync()
        t0 = time.perf_counter()
        nst = [Gn.run("sssp", **run_kw) for _ in range(args.steps)]
        sync()
        nel = time.perf_counter() - t0
        assert np.array_equal(Gn.values(), dist)
        res["input_order"] = {"solve_gteps": round(g.m * args.steps / nel / 1e9, 4),
                              "ms_per_solve": round(nel * 1e3 / args.steps, 3),
                              "pages": Gn.info()["num_parts"], "passes_per_solve": nst[-1]["passes"],
                              "h2d_bytes_per_solve": nst[-1]["h2d_bytes"],
                              "sweep_GBps": round(sum(s["algo_bytes"] for s in nst) /
                                                  (sum(s["sweep_kernel_ms"] for s in nst) * 1e-3) / 1e9, 1)}
        Gn.close()
        ctxn.close()
    if not args.no_hetero:
        # heterogeneous model of Section 3.1: the host finishes from a small frontier
        hkw = dict(run_kw, pvu="strong", hetero=True)
        for _ in range(max(1, args.warmup)):
            G.run("sssp", **hkw)
        sync()
        t0 = time.perf_counter()
        hst = [G.run("sssp", **hkw) for _ in range(args.steps)]
        sync()
        hel = time.perf_counter() - t0
        assert np.array_equal(G.values(), dist)
        h = hst[-1]
        res["hetero"] = {"solve_gteps": round(g.m * args.steps / hel / 1e9, 4),
                         "ms_per_solve": round(hel * 1e3 / args.steps, 3),
                         "device_passes": h["passes"], "sparse_stage": h["sparse_stage"],
                         "sparse_frontier": h["sparse_frontier"], "sparse_rounds": h["sparse_rounds"],
                         "sparse_relaxations": h["sparse_relaxations"], "sparse_ms": round(h["sparse_ms"], 3),
                         "sparse_value_bytes_copied": h["sparse_copy_bytes"],
                         "h2d_bytes_per_solve": h["h2d_bytes"],
                         "note": "device dense passes + host push sparse stage; not the headline value"}
        log(f"[bench] hetero: {res['hetero']}")
    probe = gather_probe(args, g, G, dist)
    res["roofline"]["gather_probe"] = probe
    res["roofline"]["sweep_scan_vs_probe"] = round(res["scan_gteps"] / probe["edges_per_s"], 3)
    log(f"[bench] gather probe: {probe}")
    if not args.no_other:
        res["bfs_early_break"] = bench_bfs_early_break(args, g, G)
        log(f"[bench] bfs early break: {res['bfs_early_break']}")
    if args.ablation:
        res["ablation"] = ablation(args, G, info["num_parts"], dist)
    if args.resident:
        ctx2 = sr.Context(0, 0)
        G2 = ctx2.load(g, reorder=args.order == "degree")
        G2.partition(1, 4)
        G2.run("sssp", source=0, pvu=args.pvu)
        sync()
        t0 = time.perf_counter()
        rs = [G2.run("sssp", source=0, pvu=args.pvu) for _ in range(args.steps)]
        sync()
        el = time.perf_counter() - t0
        km = sum(s["sweep_kernel_ms"] for s in rs)
        ab = sum(s["algo_bytes"] for s in rs)
        res["resident"] = {"solve_gteps": round(g.m * args.steps / el / 1e9, 3),
                           "ms_per_solve": round(el * 1e3 / args.steps, 3),
                           "sweep_GBps": round(ab / (km * 1e-3) / 1e9, 1),
                           "sweep_frac": round(ab / (km * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "sweeps_per_solve": rs[-1]["sweeps"]}
        assert np.array_equal(G2.values(), dist)
        G2.close()
        ctx2.close()
    if not args.no_cpu:
        import oracle
        solves = 0
        t0 = time.perf_counter()
        while True:
            ref = oracle.sssp(g, 0)
            solves += 1
            tc = time.perf_counter() - t0
            # as a secondary leg one solve gives parity and a single-thread rate
            if tc >= args.cpu_seconds or args.headline != "sssp22":
                break
        res["cpu_baseline"] = {"value": round(g.m * solves / tc / 1e9, 5), "unit": "GTEPS", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{solves} full Dijkstra solves of the same graph from vertex 0 "
                                         f"({tc:.1f} s, one thread)"}
        res["parity"] = "bit-exact" if np.array_equal(ref, dist) else f"MISMATCH {int(np.sum(ref != dist))}"
    G.close()
    ctx.close()
    return res


def ablation(args, G, parts, dist):
    """Section 5.4 schedules on the same streamed pages (same page count):
    baseline = two slots, each page swept once per pass; rsi = two slots, each
    page re-entered MRT = 2 times (the paper's MRT for SSSP); psi = the
    pipelined window of S-1 pages with adaptive re-entry, prediction off; then
    psi with each predictor. Reports solve time, passes, sweeps, streamed bytes,
    and for the weak predictor the per-pass changed / skipped vertices (the
    status curves of Fig. 10)."""
    scheds = [("baseline", 2, 1, True, "off", 1), ("rsi_mrt2", 2, 2, True, "off", 1),
              ("psi", args.slots, sssp_inner(args), False, "off", 1),
              ("psi_strong", args.slots, sssp_inner(args), False, "strong", 1),
              ("psi_weak", args.slots, sssp_inner(args), False, "weak", 1),
              ("psi_strong_depth2", args.slots, sssp_inner(args), False, "strong", 2)]
    out = {}
    for name, slots, inner, fixed, pvu, depth in scheds:
        G.partition(parts, slots)
        kw = dict(source=0, pvu=pvu, max_inner_iters=inner, force_stream=True, fixed_inner=fixed,
                  copy_depth=depth)
        G.run("sssp", **kw)
        sync()
        t0 = time.perf_counter()
        st = G.run("sssp", **kw)
        sync()
        el = time.perf_counter() - t0
        assert np.array_equal(G.values(), dist), name
        row = {"ms_per_solve": round(el * 1e3, 2), "passes": st["passes"], "sweeps": st["sweeps"],
               "edges_scanned": st["edges_scanned"], "h2d_bytes": st["h2d_bytes"],
               "kernel_ms": round(st["kernel_ms"], 2), "h2d_ms": round(st["h2d_ms"], 2)}
        if pvu != "off":
            tr = G.sweeps()
            np_ = st["passes"]
            row["per_pass_changed"] = [sum(r["changed"] for r in tr if r["pass"] == k) for k in range(np_)]
            row["per_pass_skipped"] = [sum(r["skipped"] for r in tr if r["pass"] == k) for k in range(np_)]
        out[name] = row
        log(f"[bench] ablation {name}: {row['ms_per_solve']} ms, {row['passes']} passes, {row['sweeps']} sweeps")
    G.partition(parts, args.slots)
    return out


def bench_probe(args):
    """The gather probe alone on the streamed SSSP workload's edge words
    (R-MAT scale 22, device numbering): for hardware counters on the bare
    gather (sr_probe_gather, 20 timed launches)."""
    import graphgen
    import oracle
    import paper_1806_00762_amd as sr
    g = graphgen.recipes.sssp_s22()
    ctx = sr.Context(0, 0)
    G = ctx.load(g, reorder=args.order == "degree")
    G.partition(0, args.slots)
    dist = oracle.sssp(g, 0)
    out = gather_probe(args, g, G, dist)
    G.close()
    ctx.close()
    return out


def gather_probe(args, g, G, dist):
    """The sweep's practical ceiling: the same edge words in the same order
    (all pages of the graph, vertices as numbered on the device) and the same
    value array, read with the sweep kernel's tiling by a kernel that only
    gathers (no gate, no reduction, no writes): sr_probe_gather."""
    import paper_1806_00762_amd as sr
    info = G.info()
    words, packed = [], False
    for p in range(info["num_parts"]):
        pg = G.page(p)
        w = pg["src"].astype(np.uint32)
        if pg["src_packed"]:
            packed = True
            w = w | (pg["weights"].astype(np.uint32) << np.uint32(24))
        words.append(w)
    words = np.concatenate(words)
    vals = dist
    if args.order == "degree":
        _, caller_of = G.order()
        vals = dist[caller_of]
    ctx = sr.Context(0, 0)
    ms, _ = sr.probe_gather(ctx, words, 0x00FFFFFF if packed else 0xFFFFFFFF, vals.astype(np.uint32), repeats=20)
    ctx.close()
    rate = words.size / (ms * 1e-3)
    return {"kernel": "gather_probe_kernel", "edges": int(words.size), "ms_per_launch": round(ms, 4),
            "edges_per_s": round(rate / 1e9, 2), "unit_edges": "G/s",
            "GBps_8B_per_edge": round(8 * rate / 1e9, 1)}


def bench_bfs_early_break(args, g, G):
    """BFS from vertex 0 on the same graph with strong prediction, resident
    (each sweep closes a pass) and streamed like the headline solve, with
    and without the dense-pull early break; levels checked against the
    oracle's queue BFS."""
    import oracle
    import paper_1806_00762_amd as sr
    ref = oracle.bfs(g, 0)
    out = {"workload": "bfs_rmat22_ef16_src0", "parity": "bit-exact"}
    ctx_r = sr.Context(0, 0)
    Gr = ctx_r.load(g, reorder=args.order == "degree")
    Gr.partition(1, 4)
    legs = (("resident", Gr, dict(source=0, pvu="strong")),
            ("streamed", G, dict(source=0, pvu="strong", max_inner_iters=sssp_inner(args), force_stream=True,
                                 copy_depth=args.copy_depth)))
    for name, H, kw in legs:
        row = {}
        for tag, eb in (("break", True), ("full", False)):
            H.run("bfs", early_break=eb, **kw)
            sync()
            t0 = time.perf_counter()
            sts = [H.run("bfs", early_break=eb, **kw) for _ in range(args.steps)]
            sync()
            el = (time.perf_counter() - t0) / args.steps
            assert np.array_equal(H.values(), ref), (name, tag)
            km = sum(s["kernel_ms"] for s in sts) / args.steps
            row[tag] = {"ms_per_solve": round(el * 1e3, 3), "solve_gteps": round(g.m / el / 1e9, 3),
                        "kernel_ms": round(km, 3), "passes": sts[-1]["passes"], "sweeps": sts[-1]["sweeps"],
                        "edges_read": sts[-1]["edges_scanned"]}
        out[name] = row
    Gr.close()
    ctx_r.close()
    return out


def bench_pagerank16(args):
    """PageRank on R-MAT scale 16 (4 equal-byte pages, up to 4 sweeps per page
    per pass, L1 < 1e-9, resident): no prediction, weak prediction, weak
    prediction with a change tolerance (updates below it count as failed
    attempts), and PageRank-delta (residual propagation, then the rank-form
    verification passes) without and with a send threshold and with weak
    prediction; each checked against the FP64 oracle."""
    import graphgen
    import oracle
    import paper_1806_00762_amd as sr
    g = graphgen.recipes.pagerank_s16()
    ref, _, _ = oracle.pagerank(g, tol=1e-13)
    ctx = sr.Context(0, 0)
    G = ctx.load(g, reorder=args.order == "degree")
    G.partition(4, 4)
    out = {"workload": "pagerank_rmat16_ef16_4pages_inner4_tol1e-9", "n": g.n, "m": g.m}
    for name, pvu, eps, delta in (("off", "off", 0.0, False), ("weak", "weak", 0.0, False),
                                  ("weak_eps1e-9", "weak", 1e-9, False),
                                  ("delta", "off", 0.0, True), ("delta_eps1e-10", "off", 1e-10, True),
                                  ("delta_weak_eps1e-10", "weak", 1e-10, True)):
        kw = dict(pvu=pvu, pr_change_eps=eps, max_inner_iters=4, tol_l1=1e-9, pr_delta=delta)
        G.run("pagerank", **kw)
        sync()
        t0 = time.perf_counter()
        sts = [G.run("pagerank", **kw) for _ in range(args.steps)]
        sync()
        el = (time.perf_counter() - t0) / args.steps
        x = G.values().view(np.float32).astype(np.float64)
        st = sts[-1]
        out[name] = {"ms_per_solve": round(el * 1e3, 3), "solve_gteps": round(g.m / el / 1e9, 3),
                     "edges_swept_gteps": round(g.m * st["sweeps"] / el / 1e9, 2),
                     "sweeps": st["sweeps"], "vertex_pulls": st["vertices_attempted"],
                     "delta_passes": st["pr_delta_passes"], "verify_passes": st["verify_passes"],
                     "max_abs": float(np.max(np.abs(x - ref))), "dtype": "f32"}
    G.close()
    ctx.close()
    return out


def bench_lattice(args):
    """Page skipping on a high-diameter graph with locality: SSSP from a corner
    of a 1024 x 1024 lattice (weights 1-9), pages streamed through 4 slots
    within a quarter of the graph bytes, with and without skipping the pages
    no changed vertex points into."""
    import graphgen
    import oracle
    import paper_1806_00762_amd as sr
    g = graphgen.grid(1024, 1024, weights=(1, 9, 2024))
    ref = oracle.sssp(g, 0)
    budget = (4 * (g.n + 1) + 8 * g.m) // 4
    ctx = sr.Context(0, budget)
    G = ctx.load(g)
    G.partition(0, 4)
    out = {"workload": "sssp_grid1024x1024_w1-9_corner_streamed_budget_quarter", "n": g.n, "m": g.m,
           "pages": G.info()["num_parts"]}
    for name, skip in (("all_pages", False), ("skip_clean", True)):
        kw = dict(source=0, pvu="strong", force_stream=True, copy_depth=2, skip_clean=skip, max_passes=100000)
        G.run("sssp", **kw)
        sync()
        t0 = time.perf_counter()
        st = G.run("sssp", **kw)
        sync()
        el = time.perf_counter() - t0
        assert np.array_equal(G.values(), ref), name
        out[name] = {"ms_per_solve": round(el * 1e3, 2), "passes": st["passes"], "sweeps": st["sweeps"],
                     "h2d_bytes": st["h2d_bytes"], "pages_skipped": st["pages_skipped"],
                     "solve_gteps": round(g.m / el / 1e9, 4)}
    out["parity"] = "bit-exact"
    G.close()
    ctx.close()
    return out


def bench_batched(args):
    """256 personalized-PageRank instances over 32 R-MAT graphs (scales 12-20,
    edge factor 8/16/32), 8 seeds per graph: one batched call vs a loop of
    single-instance solves on the same GPU."""
    import graphgen
    import oracle
    import paper_1806_00762_amd as sr
    t = time.perf_counter()
    graphs = [graphgen.recipes.batched_graph(i) for i in range(32)]
    log(f"[bench] batched: generated 32 graphs, m total {sum(g.m for g in graphs)} in {time.perf_counter() - t:.1f}s")
    ctx = sr.Context(0, 0)
    Gs = [ctx.load(g, reorder=args.order == "degree") for g in graphs]
    for G in Gs:
        G.partition(1, 4)
    insts = []
    for gi, g in enumerate(graphs):
        for s in graphgen.sources_with_outedges(g, 8, seed=2000 + gi):
            insts.append((gi, int(s)))
    _, _, bs0 = sr.batch_run(ctx, [(Gs[gi], "ppr", s) for gi, s in insts])   # warm-up and autotune
    sync()
    t0 = time.perf_counter()
    outs, per, bs = sr.batch_run(ctx, [(Gs[gi], "ppr", s) for gi, s in insts])
    sync()
    tb = time.perf_counter() - t0
    # plain: the same instances one solve at a time through sr_run
    # (a strided sample, so every graph size is represented)
    stride = max(1, len(insts) // args.plain_sample)
    sample = insts[::stride]
    nplain = len(sample)
    Gs[insts[0][0]].run("ppr", source=insts[0][1], pvu="off", max_inner_iters=1)
    sync()
    t0 = time.perf_counter()
    for gi, s in sample:
        Gs[gi].run("ppr", source=s, pvu="off", max_inner_iters=1)
    sync()
    tp = (time.perf_counter() - t0) / nplain
    # accuracy: max-abs against the FP64 oracle's own solve of every instance
    # (oracle solves in a thread pool over the host cores)
    from concurrent.futures import ThreadPoolExecutor

    def err_of(k):
        gi, s = insts[k]
        ref, _, _ = oracle.pagerank(graphs[gi], seed=s, tol=1e-13)
        return float(np.max(np.abs(outs[k].view(np.float32).astype(np.float64) - ref)))

    with ThreadPoolExecutor(max(1, min(16, host_info()["usable_cpus"] or 1))) as ex:
        errs = list(ex.map(err_of, range(len(insts))))
    exact_max, nexact = max(errs), len(errs)
    for G in Gs:
        G.close()
    ctx.close()
    return {"workload": "ppr256_over_32_rmat_s12-20_ef8-32", "instances": len(insts), "vertex_order": args.order,
            "solves_per_s": round(len(insts) / tb, 1), "batched_ms": round(tb * 1e3, 2),
            "plain_solves_per_s": round(1.0 / tp, 1), "plain_sample": nplain,
            "speedup_vs_plain": round(tp * len(insts) / tb, 2),
            "sweeps": bs["sweeps"],
            "schedule": {"group_width": bs["group_width"], "rounds": bs["rounds"], "grid_blocks": bs["grid_blocks"],
                         "grab": bs["grab"], "widths_timed": bs0["width_candidates"],
                         "tuning_call_wall_ms": round(bs0["wall_ms"], 1)},
            "sweep_GBps": round(bs["algo_bytes"] / (bs["kernel_ms"] * 1e-3) / 1e9, 1) if bs["kernel_ms"] else None,
            "max_abs_exact": exact_max, "max_abs_exact_instances": nexact, "dtype": "f32"}


def _serve_stream(srv, graphs, reqs, arr, timeout, check):
    """Submit reqs at arrival times arr (s) from a producer thread and poll
    until all are done; returns (latencies ms, elapsed s, outputs of check)."""
    import threading
    nreq = len(reqs)
    tickets = [None] * nreq
    t0 = time.perf_counter()

    def producer():
        for i, (gi, algo, s) in enumerate(reqs):
            delay = arr[i] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets[i] = srv.submit(gi, algo, s)

    th = threading.Thread(target=producer)
    th.start()
    outs = {i: np.empty(graphs[reqs[i][0]].n, dtype=np.uint32) for i in check}
    lat = [None] * nreq
    pending = set(range(nreq))
    while pending:
        for i in list(pending):
            if tickets[i] is None:
                continue
            done, l = srv.poll(tickets[i], outs.get(i))
            if done:
                lat[i] = l
                pending.discard(i)
        time.sleep(0.0002)
        if time.perf_counter() - t0 > timeout:
            break
    th.join()
    return lat, time.perf_counter() - t0, outs


def _requests(graphs, nreq, rate, seed):
    import graphgen
    arr = graphgen.poisson_arrivals(rate, nreq, seed=seed)
    pick = graphgen.bounded_draws(seed + 1, 1, nreq, 0, 2)
    kind = graphgen.bounded_draws(seed + 2, 1, nreq, 0, 1)
    srcs = [graphgen.sources_with_outedges(graphs[gi], nreq, seed=seed + 3 + gi) for gi in range(3)]
    reqs = [(int(pick[i]), "sssp" if kind[i] == 0 else "bfs", int(srcs[int(pick[i])][i])) for i in range(nreq)]
    return arr, reqs


def bench_served(args):
    """Poisson stream of SSSP/BFS queries over 3 resident R-MAT graphs (scales
    20, 22, 23; ef 16; weights [1, 255]) through the continuous-batching
    server, vs solo solves of the same queries. The offered 2000/s overloads
    the server, so a second, shorter stream at 70% of the achieved rate gives
    the latency of a server that keeps up."""
    import graphgen
    import oracle
    import paper_1806_00762_amd as sr
    t = time.perf_counter()
    graphs = [graphgen.recipes.serving_graph(s) for s in (20, 22, 23)]
    log(f"[bench] served: generated graphs in {time.perf_counter() - t:.1f}s")
    ctx = sr.Context(0, 0)
    Gs = [ctx.load(g, reorder=args.order == "degree") for g in graphs]
    for G in Gs:
        G.partition(1, 4)
    nreq = args.requests
    arr, reqs = _requests(graphs, nreq, args.rate, 4000)
    srv = sr.Server(ctx, Gs, state_budget_bytes=0, slots=args.serve_slots)
    check = set(range(0, nreq, max(1, nreq // 12)))
    lat, elapsed, outs = _serve_stream(srv, graphs, reqs, arr, args.served_timeout, check)
    st1 = srv.stats()
    ok = 0
    for i in check:
        gi, algo, s = reqs[i]
        if lat[i] is None:
            continue
        ref = oracle.sssp(graphs[gi], s) if algo == "sssp" else oracle.bfs(graphs[gi], s)
        ok += int(np.array_equal(outs[i], ref))
    done_lat = np.array([x for x in lat if x is not None])
    achieved = done_lat.size / elapsed
    # a rate the server sustains
    rate2 = max(1.0, 0.7 * achieved)
    n2 = int(min(nreq, max(200, rate2 * 4)))
    arr2, reqs2 = _requests(graphs, n2, rate2, 4100)
    lat2, el2, _ = _serve_stream(srv, graphs, reqs2, arr2, args.served_timeout, set())
    lat2 = np.array([x for x in lat2 if x is not None])
    st = srv.stats()
    srv.close()
    # plain: the same kind of queries solved one at a time
    nplain = args.plain_sample
    Gs[0].run("sssp", source=reqs[0][2] if reqs[0][0] == 0 else 0)
    sync()
    tp0 = time.perf_counter()
    for gi, algo, s in reqs[:nplain]:
        Gs[gi].run(algo, source=s)
    sync()
    tp = (time.perf_counter() - tp0) / nplain
    for G in Gs:
        G.close()
    ctx.close()
    return {"workload": "poisson2000_sssp_bfs_rmat20_22_23_ef16", "requests": nreq, "vertex_order": args.order,
            "completed": int(done_lat.size), "offered_qps": args.rate,
            "achieved_qps": round(achieved, 1),
            "p50_ms": round(float(np.percentile(done_lat, 50)), 2) if done_lat.size else None,
            "p99_ms": round(float(np.percentile(done_lat, 99)), 2) if done_lat.size else None,
            "sustained": {"offered_qps": round(rate2, 1), "requests": n2, "completed": int(lat2.size),
                          "achieved_qps": round(lat2.size / el2, 1),
                          "p50_ms": round(float(np.percentile(lat2, 50)), 2) if lat2.size else None,
                          "p99_ms": round(float(np.percentile(lat2, 99)), 2) if lat2.size else None},
            "plain_solves_per_s": round(1.0 / tp, 1), "plain_sample": nplain,
            "sweeps": st["sweeps"], "slots_per_graph": st["slots_per_graph"],
            # the sweep replays of the offered-rate stream: algorithmic bytes
            # (shared edge words, offsets and bins per live graph and sweep,
            # one 16-bit value per scanned in-edge and query) over their
            # HIP-event time
            "sweep": {"replays": st1["sweeps"], "ms_per_replay": round(st1["kernel_ms"] / max(st1["sweeps"], 1), 3),
                      "device_busy_frac": round(st1["kernel_ms"] * 1e-3 / elapsed, 3),
                      "algo_GBps": round(st1["algo_bytes"] / (st1["kernel_ms"] * 1e-3) / 1e9, 1)
                      if st1["kernel_ms"] else None,
                      "frac_hbm_peak": round(st1["algo_bytes"] / (st1["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                      if st1["kernel_ms"] else None},
            "narrow_fallbacks": st["narrow_fallbacks"],
            "checked_vs_oracle": f"{ok}/{len(check)} bit-exact"}


def copy_calibration():
    """A plain streaming kernel of known size: out = in * 1 over 2^28 float32
    (1 GiB read + 1 GiB written per launch), 5 launches. Its HBM counters
    scale the sweep's counters to bytes; its rate is the measured copy peak."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        torch.mul(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    return {"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 6,
            "ms_per_launch": round(ms, 4), "copy_GBps": round(8 * n / (ms * 1e-3) / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--inner", type=int, default=0,
                    help="max re-sweeps per window step (0: 8 for the CC legs, 4 for the SSSP leg)")
    ap.add_argument("--pvu", default="strong",
                    help="predictor of the timed solves (the other one is reported beside it)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--resident", action="store_true", help="also time the resident solve")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and served legs")
    ap.add_argument("--plain-sample", type=int, default=32)
    ap.add_argument("--requests", type=int, default=20000)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain copy kernel of known size (for HBM counter scaling)")
    ap.add_argument("--served-timeout", type=float, default=90.0)
    ap.add_argument("--only", choices=["batched", "served", "lattice", "pagerank16", "probe"],
                    help="run one extra leg alone and print its JSON object")
    ap.add_argument("--copy-depth", type=int, default=2,
                    help="page copies kept in flight ahead of the window (1 = the paper's layout)")
    ap.add_argument("--no-other", action="store_true", help="skip the other predictor's and order's solves")
    ap.add_argument("--order", choices=["degree", "input"], default="degree",
                    help="internal vertex numbering of the headline graph (results are in input ids)")
    ap.add_argument("--no-hetero", action="store_true", help="skip the host sparse stage leg")
    ap.add_argument("--no-host-stage", action="store_true",
                    help="CC legs without the heterogeneous model's host stage (device passes only)")
    ap.add_argument("--headline", choices=["cc24", "sssp22"], default="cc24",
                    help="workload of the headline line: streamed CC on R-MAT scale 24 (and its uniform "
                         "twin), or streamed SSSP on R-MAT scale 22")
    ap.add_argument("--no-twin", action="store_true", help="skip the uniform twin of the CC workload")
    ap.add_argument("--no-sssp", action="store_true", help="skip the streamed SSSP leg")
    ap.add_argument("--input-order", action="store_true",
                    help="also time the streamed SSSP solve with the input's vertex numbering")
    ap.add_argument("--wide-pages", action="store_true",
                    help="stream full-width pages instead of split-width images")
    ap.add_argument("--ablation", action="store_true",
                    help="also time the Section 5.4 schedules (baseline, re-entry, pipelined, +predictors)")
    ap.add_argument("--schedule", choices=["fixed", "copy"], default="fixed",
                    help="streamed windows: re-swept until no change (fixed, timing-independent) or until "
                         "the next page has landed (copy)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU work of the oracle baseline (repeated solves)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the engine runs on a single device; "
              "run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.init()
    if args.copy_calibration:
        print(json.dumps(copy_calibration()), flush=True)
        return
    if args.only:
        # one extra leg alone (for profiling it): its JSON object only
        fn = {"batched": bench_batched, "served": bench_served, "lattice": bench_lattice,
              "pagerank16": bench_pagerank16, "probe": bench_probe}[args.only]
        print(json.dumps(fn(args)), flush=True)
        return
    if args.headline == "cc24":
        res = bench_cc24(args)
        log(f"[bench] headline cc24: {res['value']} GTEPS")
        if not args.no_sssp:
            s22 = bench_sssp22(args)
            for k in ("metric", "unit", "n_gpus", "steps", "warmup", "higher_is_better", "scaling",
                      "vs_baseline", "data"):
                s22.pop(k, None)
            s22["solve_gteps"] = s22.pop("value")
            res["sssp22"] = s22
            log(f"[bench] sssp22: {s22['solve_gteps']} GTEPS")
    else:
        res = bench_sssp22(args)
    if not args.no_extras:
        res["pagerank16"] = bench_pagerank16(args)
        log(f"[bench] pagerank16: {res['pagerank16']}")
        res["lattice"] = bench_lattice(args)
        log(f"[bench] lattice: {res['lattice']}")
        res["batched"] = bench_batched(args)
        log(f"[bench] batched: {res['batched']}")
        res["served"] = bench_served(args)
        log(f"[bench] served: {res['served']}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
