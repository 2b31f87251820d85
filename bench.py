#!/usr/bin/env python3
"""Benchmark of PCPM PageRank on one MI355X.

Workload: PageRank (d = 0.85, dangling mass spread uniformly, FP32 ranks,
FP64 residual) on a directed RMAT graph of scale 24 with edge factor 16
(a, b, c = 0.57, 0.19, 0.19; self-loops and duplicate edges dropped), random
node labels, partitions of 16384 nodes, iterated to an L1 residual below 1e-6.
A step is one solve from the uniform vector; the graph and its partition-node
graph are resident in HBM before the timed region starts.  The same graph with
in-degree-sorted labels (relabelled on the GPU by pcpm_relabel, whose time is
reported) is measured as well and reported under "indegree".

The timed region holds the solves only; per-kernel averages (and the
roofline figure taken from them) come from a separate pass of solves with a
HIP event pair around every launch.

Further legs (in "detail"): the sparse matrix-vector product over the PNG
with random edge weights on the main graph (Sec. 3.5), the learned warm
start against the uniform start
on the main graph (network weights shipped with the package, trained on other
RMAT graphs), batched personalised PageRank on RMAT-22 with 8/32/64 seed sets
against one vector at a time, 16 RMAT graphs of uneven size in one handle
against one handle per graph, and the paper's scale of graph (RMAT-26 EF 24
with 1.58B edges, and a uniform graph of 50M nodes and 1B edge draws) for
20 iterations each, as in the paper's Table 5 protocol.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import re
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS/iter + HBM GB/s; time to L1 resid 1e-6, warm vs cold init"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def solve_tol(args):
    return 0.0 if args.iters > 0 else args.tol


def solve_iters(args):
    return args.iters if args.iters > 0 else args.max_iters


def workload_name(args):
    if args.graph == "uniform":
        g = f"a uniform random directed graph of {args.nodes} nodes and {args.draws} edge draws (seed {args.seed})"
    else:
        labels = ("random node labels" if args.labels == "random" else
                  "random node labels, then in-degree order from pcpm_relabel")
        g = (f"RMAT scale {args.scale}, edge factor {args.edge_factor:g} (a,b,c=.57,.19,.19, seed {args.seed}), "
             f"{labels}")
    stop = f"{args.iters} iterations" if args.iters > 0 else f"to L1 residual {args.tol:g}"
    return f"PageRank d={args.d} {stop} on {g}, partition {1 << args.part_log2} nodes"


def relabel_detail(P, torch, r, c, reps=3):
    """In-degree-sorted labels from pcpm_relabel on the device-resident graph;
    returns the relabelled CSR (host) and the median relabel time in ms."""
    rt = torch.from_numpy(r).cuda()
    ct = torch.from_numpy(c).cuda()
    P.relabel(rt, ct, key="in")
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        perm, ro, co = P.relabel(rt, ct, key="in")
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    rl_ms = sorted(ts)[len(ts) // 2] * 1e3
    log(f"[indegree] pcpm_relabel (in-degree order) {rl_ms:.1f} ms")
    ri, ci = ro.cpu().numpy(), co.cpu().numpy()
    del rt, ct, perm, ro, co
    torch.cuda.empty_cache()
    return ri, ci, rl_ms


def measure(P, torch, r, c, args, label, tol=None, max_iters=None, update_order=None):
    """Build the PNG, warm up, time `steps` solves with nothing but the solves
    in the timed region, then run a separate pass of solves with per-launch
    HIP events for the per-kernel averages."""
    from paper_1709_07122_amd import commmodel as cm

    tol = solve_tol(args) if tol is None else tol
    max_iters = solve_iters(args) if max_iters is None else max_iters
    update_order = args.update_order if update_order is None else update_order
    n, m = len(r) - 1, len(c)
    rt = torch.from_numpy(r).cuda()
    ct = torch.from_numpy(c).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    png = P.build_png(rt, ct, part_log2=args.part_log2, update_order=update_order)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    del rt, ct
    info = png.info
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        P.pagerank(png, d=args.d, tol=tol, max_iters=max_iters, out=out, want_hist=False)
    log(f"[{label}] n={n} m={m} q={info['q']} k={info['k']} E'={info['eprime']} "
        f"r={m / max(info['eprime'], 1):.3f} updates in {'PNG' if info['update_order'] == 2 else 'bin'} order "
        f"build={build_s * 1e3:.1f} ms")

    # timed region: the solves only (no per-launch events), in the default
    # launch mode (one launch per phase)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, step_s = [], []
    for _ in range(args.steps):
        ts = time.perf_counter()
        res = P.pagerank(png, d=args.d, tol=tol, max_iters=max_iters, out=out, want_hist=False)
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - ts)
        iters.append(res.iters)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0

    # the same solves in one persistent launch each (for comparison)
    persist_ms = None
    if png.launch_grid > 0 and not args.no_persistent:
        png.set_launch(2)
        P.pagerank(png, d=args.d, tol=tol, max_iters=max_iters, out=out, want_hist=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            P.pagerank(png, d=args.d, tol=tol, max_iters=max_iters, out=out, want_hist=False)
        torch.cuda.synchronize()
        persist_ms = (time.perf_counter() - t0) / args.steps * 1e3
    # per-kernel table: events around every launch, one launch per phase
    png.set_launch(1)
    ev_steps = max(2, args.steps // 4)
    P.timing_enable(True)
    te = time.perf_counter()
    ev_iters = 0
    for _ in range(ev_steps):
        ev_iters += P.pagerank(png, d=args.d, tol=tol, max_iters=max_iters, out=out, want_hist=False).iters
    torch.cuda.synchronize()
    ev_ms = (time.perf_counter() - te) / ev_steps * 1e3
    P.timing_enable(False)
    kt = P.timing_collect()
    png.set_launch(0)

    tot_iters = sum(iters)
    sec_per_iter = total_s / tot_iters
    eprime, nseg = info["eprime"], info["nseg"]
    kernels = {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1)} for k, v in kt.items()}
    png_order = info["update_order"] == 2
    g_bytes = cm.gather_bytes(n, m, eprime, nseg=nseg, png_order=png_order)
    s_bytes = cm.scatter_bytes(n, eprime, nseg, png_order=png_order)
    it_bytes = g_bytes + s_bytes
    eq5 = cm.pcpm_comm(n, m, info["k"], m / max(eprime, 1))
    kern_iter_ms = sum(v[1] for name, v in kt.items() if name != "pcpm_init") / max(ev_iters, 1)
    g_ms = kernels.get("pcpm_gather", {"avg_ms": float("nan")})["avg_ms"]
    s_ms = kernels.get("pcpm_scatter", {"avg_ms": float("nan")})["avg_ms"]
    result = {
        "n": n, "m": m, "q": info["q"], "k": info["k"], "eprime": eprime, "r": m / max(eprime, 1),
        "iters": iters[-1], "ms_per_step": total_s / args.steps * 1e3, "ms_per_iter": sec_per_iter * 1e3,
        "gteps": m / sec_per_iter / 1e9, "time_to_tol_ms": total_s / args.steps * 1e3,
        "ms_per_step_median": sorted(step_s)[len(step_s) // 2] * 1e3,
        "gteps_median": m * iters[-1] / sorted(step_s)[len(step_s) // 2] / 1e9,
        "alg_bytes_per_iter": it_bytes, "alg_bytes_per_edge": it_bytes / m, "eq5_bytes_per_edge": eq5 / m,
        "hbm_gbs_alg": it_bytes / sec_per_iter / 1e9,
        "iteration_frac_of_peak": it_bytes / sec_per_iter / 1e9 / HBM_PEAK_GBS,
        "build_ms": build_s * 1e3,
        "launch": "per_phase", "launch_grid": png.launch_grid, "ms_per_step_persistent_launch": persist_ms,
        "kernel_ms_per_step": kern_iter_ms * iters[-1],
        "kernels": kernels, "kernel_pass": {"launch": "per_phase", "solves": ev_steps,
                                            "ms_per_step_with_events": ev_ms, "kernel_ms_per_iter": kern_iter_ms},
        "gather_bytes": g_bytes, "scatter_bytes": s_bytes,
        "gather_frac_of_peak": g_bytes / (g_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "scatter_frac_of_peak": s_bytes / (s_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "update_order": "png" if png_order else "bin",
        "split_bins": info["split_bins"], "gather_items": info["gather_items"],
        "scatter_items": info["scatter_items"],
    }
    log(f"[{label}] iters={iters} {result['ms_per_step']:.3f} ms/solve, {result['gteps']:.1f} GTEPS, "
        f"{result['hbm_gbs_alg']:.0f} GB/s (algorithmic, {result['iteration_frac_of_peak']:.3f} of peak); "
        f"sum of kernel times {kern_iter_ms * iters[-1]:.3f} ms/solve; one persistent launch "
        f"{persist_ms if persist_ms is None else round(persist_ms, 3)} ms/solve; with events {ev_ms:.3f} ms/solve")
    for k, v in sorted(kernels.items()):
        log(f"    {k:16s} launches={v['launches']:5d} avg={v['avg_ms'] * 1e3:9.1f} us")
    return result, out.cpu().numpy(), png


def paper_scale_detail(P, torch, args, kind):
    """The paper's protocol on its scale of graph: 20 iterations from the
    uniform start, q = 16384, automatic update order (Table 5's GTEPS =
    edges / one iteration's time)."""
    import graphgen

    t = time.perf_counter()
    if kind == "rmat26":
        r, c = graphgen.rmat(26, 24, seed=3, relabel="random")
        name = "RMAT scale 26, edge factor 24 (a,b,c=.57,.19,.19, seed 3), random node labels"
    else:
        r, c = graphgen.uniform(50_000_000, 1_000_000_000, seed=4)
        name = "uniform random directed graph, 50M nodes, 1B edge draws (seed 4)"
    log(f"generated {kind}: n={len(r) - 1} m={len(c)} in {time.perf_counter() - t:.1f} s")
    res, _, png = measure(P, torch, r, c, args, kind, tol=0.0, max_iters=20, update_order=0)
    png.close()
    del r, c
    torch.cuda.empty_cache()
    res["graph"] = name
    res["protocol"] = "20 iterations from the uniform start, q = 16384"
    return res


def spmv_detail(P, torch, r, c, args, reps=20):
    """SpMV over the PNG (Sec. 3.5) on the main graph with seeded random edge
    weights (uniform in [-1, 1)) and x uniform in [-1, 1): per-kernel event
    times of `reps` calls, the weighted gather against the HBM roofline, and
    y against the FP64 oracle within the bound of pcpm_spmv."""
    import numpy as np
    from paper_1709_07122_amd import commmodel as cm

    n, m = len(r) - 1, len(c)
    rng = np.random.default_rng(args.seed + 1000)
    w = rng.uniform(-1.0, 1.0, m).astype(np.float32)
    x = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    rt, ct, wt, xt = (torch.from_numpy(a).cuda() for a in (r, c, w, x))
    png = P.build_png(rt, ct, part_log2=args.part_log2, weights=wt)
    info = png.info
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    for _ in range(3):
        P.spmv(png, xt, out=y)
    torch.cuda.synchronize()
    P.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        P.spmv(png, xt, out=y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    P.timing_enable(False)
    kt = P.timing_collect()
    kernels = {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1)} for k, v in kt.items()}
    ep, nseg = info["eprime"], info["nseg"]
    po = info["update_order"] == 2
    g_bytes = cm.spmv_gather_bytes(n, m, ep, nseg=nseg, png_order=po)
    total = cm.spmv_bytes(n, m, ep, nseg, png_order=po)
    g_ms = kernels.get("pcpm_spmv_gather", {"avg_ms": float("nan")})["avg_ms"]
    res = {"graph": "the main graph, weights uniform in [-1, 1)", "ms_per_call": dt * 1e3, "gteps": m / dt / 1e9,
           "alg_bytes_per_call": total, "hbm_gbs_alg": total / dt / 1e9, "kernels": kernels,
           "gather_bytes": g_bytes, "gather_gbs": g_bytes / (g_ms * 1e-3) / 1e9,
           "gather_frac_of_peak": g_bytes / (g_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if not args.no_cpu_baseline:
        import oracle

        tc = time.perf_counter()
        ref = oracle.spmv(r, c, x, w)
        cpu_s = time.perf_counter() - tc
        res["cpu_baseline"] = {"value": m / cpu_s / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
                               "sample": "one FP64 SpMV of the oracle (numpy, one thread) on the same graph",
                               "sec_per_call": cpu_s}
        got = y.cpu().numpy().astype(np.float64)
        indeg = np.bincount(c, minlength=n)
        aw = np.abs(w.astype(np.float64))
        xmax = float(np.abs(x).max())
        wcol = float(np.bincount(c, weights=aw, minlength=n).max())
        sbits = min(50 - int(np.ceil(np.log2(aw.max() * xmax))), 62 - int(np.ceil(np.log2(wcol * xmax))))
        ratio = float((np.abs(got - ref) / (indeg * 2.0 ** -(sbits - 1) + 2.0 ** -23 * np.abs(ref) + 2.0 ** -150)).max())
        res["parity"] = {"max_err_over_bound": ratio, "max_abs_err": float(np.abs(got - ref).max())}
    png.close()
    log(f"[spmv] {dt * 1e3:.3f} ms/call, {res['gteps']:.1f} GTEPS, weighted gather {res['gather_gbs']:.0f} GB/s "
        f"({res['gather_frac_of_peak']:.3f} of peak)" + (f", error/bound {res['parity']['max_err_over_bound']:.3f}, "
                                                          f"oracle {res['cpu_baseline']['sec_per_call'] * 1e3:.0f} ms"
                                                          if "parity" in res else ""))
    for k, v in sorted(kernels.items()):
        log(f"    {k:18s} launches={v['launches']:5d} avg={v['avg_ms'] * 1e3:9.1f} us")
    return res


def warm_detail(P, torch, png, args):
    """Time to tol from the uniform start and from the learned start (the
    committed network), on the graph of the main measurement."""
    from paper_1709_07122_amd import warmstart as ws

    params = ws.load(ws.DEFAULT_WEIGHTS)
    res = ws.compare(png, params, d=args.d, tol=args.tol, reps=max(1, args.steps))
    kern = res.get("warm_kernels", {})
    pred = (kern.get("pcpm_ws_predict") or {}).get("total_ms")
    fwd = (kern.get("pcpm_ws_forward_on_features") or {}).get("total_ms")
    soft = (kern.get("pcpm_ws_init") or {}).get("total_ms")
    us = lambda v: "n/a" if v is None else f"{v * 1e3:.1f} us"
    log(f"[warm] cold {res['cold_iters']} iters {res['cold_ms']:.2f} ms; warm {res['warm_iters']} iters "
        f"{res['warm_ms']:.2f} ms ({res['warm_ms_first']:.2f} ms with the in-degree count); MLP forward on the "
        f"feature matrix {us(fwd)}, fused prediction (features + forward) {us(pred)}, softmax {us(soft)}")
    return res


def warm_eval_detail(P, torch, args, seeds=(2000, 2001, 2002, 2003)):
    """The learned warm start on the held-out RMAT-24 graphs (EF 16, random
    labels): iterations and time to tol from the uniform start and from the
    committed network's start vector, per graph."""
    import graphgen
    from paper_1709_07122_amd import warmstart as ws

    params = ws.load(ws.DEFAULT_WEIGHTS)
    rows = []
    for sd in seeds:
        r, c = graphgen.rmat(24, 16, seed=sd, relabel="random")
        png = P.build_png(torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda(), part_log2=args.part_log2)
        row = {"seed": sd, **ws.compare(png, params, d=args.d, tol=args.tol, reps=max(1, args.steps // 2))}
        row["warm_incl_count_over_cold"] = row["warm_ms_first"] / row["cold_ms"]
        rows.append(row)
        png.close()
        log(f"[warm-eval] seed {sd}: cold {row['cold_iters']} iters {row['cold_ms']:.2f} ms; warm {row['warm_iters']} "
            f"iters {row['warm_ms']:.2f} ms ({row['warm_ms_first']:.2f} ms with the in-degree count, "
            f"{row['warm_incl_count_over_cold']:.3f} of cold)")
        del r, c
    return {"graphs": "RMAT-24 EF16 random labels, seeds 2000-2003 (not in the training set)", "rows": rows}


def _timed(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3, out


def ppr_detail(P, torch, args):
    """Batched personalised PageRank on RMAT-22 (EF 16, random labels) with
    k = 8, 32, 64 seed sets of 1-100 nodes, partition size from the autotuner,
    against the same k vectors solved one at a time."""
    import numpy as np

    import graphgen
    from paper_1709_07122_amd import autotune

    r, c = graphgen.rmat(22, 16, seed=args.ppr_seed, relabel="random")
    n, m = len(r) - 1, len(c)
    rt, ct = torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()
    png1, one = autotune.build(rt, ct, vectors=1)
    rows = []
    for k in (8, 32, 64):
        png, tune = autotune.build(rt, ct, vectors=k)
        off, seeds = graphgen.seed_sets(n, k, seed=k)
        reps = max(1, args.steps // 2)
        b_ms, res = _timed(torch, lambda: P.ppr_batch(png, off, seeds, tol=args.tol, max_iters=args.max_iters), reps)
        p_ms = None
        if png.launch_grid > 0 and not args.no_persistent:
            png.set_launch(2)
            try:
                p_ms, _ = _timed(torch, lambda: P.ppr_batch(png, off, seeds, tol=args.tol,
                                                            max_iters=args.max_iters), reps)
            except P.PCPMError as e:
                p_ms = f"error: {e}"
            png.set_launch(0)
        singles = [(np.array([0, off[j + 1] - off[j]], np.int32), seeds[off[j]:off[j + 1]]) for j in range(k)]

        def one_by_one():
            return [P.ppr_batch(png1, o, s, tol=args.tol, max_iters=args.max_iters) for o, s in singles]

        s_ms, sres = _timed(torch, one_by_one, reps)
        vec_iters = int(res.iters.sum())
        # per-kernel table of one batch (events around every launch); a launch
        # of the gather serves one tile of kt vector slots: 2m + 4kt E' + 8kt n
        # algorithmic bytes (IDs, updates, fixed-point slice out as ranks and
        # residual inputs)
        P.timing_enable(True)
        P.ppr_batch(png, off, seeds, tol=args.tol, max_iters=args.max_iters)
        torch.cuda.synchronize()
        P.timing_enable(False)
        kt_tab = {name: {"launches": v[0], "avg_ms": v[1] / max(1, v[0])} for name, v in P.timing_collect().items()}
        ktw = tune.tile_width
        ep = png.info["eprime"]
        g_bytes = 2 * m + 4 * ktw * ep + 8 * ktw * n
        g_avg = kt_tab.get("pcpm_ppr_gather", {}).get("avg_ms")
        g_gbs = g_bytes / (g_avg * 1e-3) / 1e9 if g_avg else None
        rows.append({"k": k, "part_log2": tune.part_log2, "update_order": tune.update_order,
                     "scatter_chunk": tune.scatter_chunk, "gather_chunk": tune.gather_chunk,
                     "tune_ms_per_vector_iter": tune.ms_per_iter, "tune_table": tune.table,
                     "tile_width": tune.tile_width, "batched_ms": b_ms, "batched_persistent_launch_ms": p_ms,
                     "one_at_a_time_ms": s_ms, "one_at_a_time_part_log2": one.part_log2,
                     "one_at_a_time_update_order": one.update_order,
                     "one_at_a_time_chunks": [one.scatter_chunk, one.gather_chunk],
                     "speedup": s_ms / b_ms, "iters_mean": float(res.iters.mean()), "iters_max": int(res.iters.max()),
                     "converged": bool(res.converged), "vector_gteps": m * vec_iters / (b_ms * 1e-3) / 1e9,
                     "single_iters_mean": float(np.mean([x.iters[0] for x in sres])),
                     "kernels": kt_tab, "eprime": ep, "gather_bytes_per_launch": g_bytes, "gather_gbs": g_gbs,
                     "gather_frac_of_peak": None if g_gbs is None else g_gbs / HBM_PEAK_GBS})
        log(f"[ppr] k={k} q=2^{tune.part_log2} order {tune.update_order} width {tune.tile_width}: {b_ms:.2f} ms batched "
            f"(one persistent launch {p_ms} ms) "
            f"vs {s_ms:.2f} ms one at a time (q=2^{one.part_log2} order {one.update_order}, {s_ms / b_ms:.2f}x), "
            f"{rows[-1]['vector_gteps']:.1f} vector-GTEPS; gather "
            + (f"{g_avg * 1e3:.1f} us/launch ({g_gbs / HBM_PEAK_GBS:.3f} of peak)" if g_avg else "not timed"))
        png.close()
    png1.close()
    return {"graph": f"RMAT-22 EF16 seed {args.ppr_seed} random labels", "n": n, "m": m, "tol": args.tol, "rows": rows}


def multigraph_detail(P, torch, args):
    """16 RMAT graphs (scale 14-20, edge factor 8-32, seeds 100-115, both
    extremes present) solved to tol in one handle, against one handle per
    graph solved in turn; partition size, update order and work-item chunks
    from the autotuner (q = 2^12..2^14)."""
    import numpy as np

    import graphgen

    graphs, shapes = graphgen.uneven_rmat_batch(16, seed=100)
    scales = [s for s, _ in shapes]
    efs = [e for _, e in shapes]
    m_tot = sum(len(c) for _, c in graphs)
    from paper_1709_07122_amd import autotune

    r, c, off, sizes = P.union_csr(graphs, 14)  # offsets divisible by every candidate q
    png, tune = autotune.build(torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda(), candidates=(12, 13, 14),
                               graph_node_off=off, graph_nodes=sizes)
    pl = tune.part_log2
    reps = max(1, args.steps // 2)
    u_ms, res = _timed(torch, lambda: P.pagerank(png, d=args.d, tol=args.tol, max_iters=args.max_iters,
                                                 want_hist=False), reps)
    it, resid = png.graph_results()
    pp_ms = None
    if png.launch_grid > 0 and not args.no_persistent:
        png.set_launch(2)
        pp_ms, _ = _timed(torch, lambda: P.pagerank(png, d=args.d, tol=args.tol, max_iters=args.max_iters,
                                                    want_hist=False), reps)
    png.set_launch(1)
    P.timing_enable(True)
    P.pagerank(png, d=args.d, tol=args.tol, max_iters=args.max_iters, want_hist=False)
    torch.cuda.synchronize()
    P.timing_enable(False)
    kern_ms = sum(v[1] for name, v in P.timing_collect().items() if name != "pcpm_init")
    png.close()
    singles = [P.build_png(torch.from_numpy(rg).cuda(), torch.from_numpy(cg).cuda(), part_log2=pl)
               for rg, cg in graphs]
    s_ms, sres = _timed(torch, lambda: [P.pagerank(g, d=args.d, tol=args.tol, max_iters=args.max_iters,
                                                   want_hist=False) for g in singles], reps)
    for g in singles:
        g.close()
    edge_iters = sum(len(c) * int(i) for (_, c), i in zip(graphs, it))
    out = {"graphs": [{"scale": int(sc), "edge_factor": int(ef), "n": len(r) - 1, "m": len(c), "iters": int(i)}
                      for (r, c), sc, ef, i in zip(graphs, scales, efs, it)],
           "part_log2": pl, "update_order": tune.update_order, "scatter_chunk": tune.scatter_chunk,
           "gather_chunk": tune.gather_chunk, "tune_table": tune.table,
           "m_total": m_tot, "one_handle_ms": u_ms, "launch": "per_phase",
           "one_handle_kernel_ms": kern_ms, "one_handle_persistent_launch_ms": pp_ms,
           "one_handle_per_graph_ms": s_ms,
           "speedup": s_ms / u_ms, "gteps": edge_iters / (u_ms * 1e-3) / 1e9, "all_converged": bool(np.all(resid < args.tol))}
    log(f"[multi] 16 graphs, m={m_tot}, q=2^{pl}: {u_ms:.2f} ms in one handle (kernels {kern_ms:.2f} ms; one "
        f"persistent launch {pp_ms} ms) vs {s_ms:.2f} ms one by one ({s_ms / u_ms:.2f}x), {out['gteps']:.1f} GTEPS")
    return out


def kernel_source_key(src: str) -> str:
    """sha256 prefix of kernel source code with its comments and whitespace
    removed: edits to comments leave the key (and the counters) valid."""
    import hashlib

    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = re.sub(r"\s+", " ", src).strip()
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", "pcpm_rmat24_random.json")))
        src = open(os.path.join(ROOT, "paper_1709_07122_amd", "csrc", "pcpm_iter.hip")).read()
    except OSError:
        return None
    if kernel_source_key(src) != prof.get("kernel_source_key"):
        return None
    k = prof["kernels"].get(kernel)
    return None if k is None else int(k["traffic_bytes"])


def copy_gbs(torch, nbytes=1 << 30, reps=5):
    """Achieved bandwidth of a plain device-to-device copy (bytes read plus
    written per second), timed with events on the current stream."""
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    return 2 * nbytes / (ms * 1e-3) / 1e9


def stream_gbs(P, torch, nbytes=4 << 30, reps=5):
    """Achieved rates of the library's plain HBM streams (pcpm_hbm_stream:
    read, write, copy, with and without non-temporal stores), bytes moved
    per second from HIP events on the launch stream."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    out = {}
    for kind in P._pcpm.STREAM_KINDS:
        size = nbytes // 2 if kind.startswith("copy") else nbytes
        P.hbm_stream(kind, src, dst, size)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            P.hbm_stream(kind, src, dst, size)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b) / reps
        moved = 2 * size if kind.startswith("copy") else size
        out[kind] = round(moved / (ms * 1e-3) / 1e9, 1)
    del src, dst
    torch.cuda.empty_cache()
    log("[stream] " + ", ".join(f"{k} {v:.0f} GB/s" for k, v in out.items()))
    return out


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = None
    return {"nproc": os.cpu_count(), "affinity_cpus": aff, "model": model}


def calibrate_copy(torch):
    """A plain copy kernel of known size: 2 GiB read + 2 GiB written per launch."""
    nbytes = 2 << 30
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "ms": dt * 1e3,
                      "gbs_read_plus_write": 2 * nbytes / dt / 1e9}))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--graph", choices=("rmat", "uniform"), default="rmat")
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--nodes", type=int, default=50_000_000, help="uniform graph: nodes")
    ap.add_argument("--draws", type=int, default=1_000_000_000, help="uniform graph: edge draws")
    ap.add_argument("--iters", type=int, default=0, help="fixed iteration count (0: iterate to --tol)")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="oracle iterations of the CPU baseline (0: as many as the GPU solve took, at least 100, "
                         "about 10 s of host work at RMAT-24)")
    ap.add_argument("--edge-factor", type=float, default=16)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--part-log2", type=int, default=14)
    ap.add_argument("--d", type=float, default=0.85)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iters", type=int, default=200)
    ap.add_argument("--no-indegree", action="store_true", help="skip the in-degree-sorted labelling")
    ap.add_argument("--labels", choices=("random", "indegree"), default="random",
                    help="labelling of the main RMAT graph (indegree: relabelled on the GPU, no separate leg)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the personalised and multi-graph legs")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm start leg")
    ap.add_argument("--no-spmv", action="store_true", help="skip the weighted SpMV leg")
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip the comparison runs in one persistent (cooperative) launch")
    ap.add_argument("--no-paper-scale", action="store_true",
                    help="skip the 20-iteration legs on RMAT-26 EF24 and the uniform 50M/1B graph")
    ap.add_argument("--update-order", type=int, default=0, choices=(0, 1, 2),
                    help="storage order of the updates: 0 automatic, 1 bin order, 2 PNG order")
    ap.add_argument("--ppr-seed", type=int, default=5)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 2 GiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        calibrate_copy(torch)
        return

    import graphgen
    import paper_1709_07122_amd as P

    torch.cuda.set_device(0)
    t = time.perf_counter()
    if args.graph == "uniform":
        raw_r = raw_c = None
        r, c = graphgen.uniform(args.nodes, args.draws, seed=args.seed)
        n = len(r) - 1
        args.no_indegree = args.no_warm = True
    else:
        raw_r, raw_c = graphgen.rmat(args.scale, args.edge_factor, 0.57, 0.19, 0.19, seed=args.seed)
        n = len(raw_r) - 1
        perm = np.empty(n, dtype=np.int32)
        graphgen._load().gg_perm_random(n, (args.seed * 7919 + 17) & (2**64 - 1), perm.ctypes.data)
        r, c = graphgen.apply_labels(raw_r, raw_c, perm)
        raw_r = raw_c = None
    log(f"generated {args.graph}: n={n} m={len(c)} in {time.perf_counter() - t:.1f} s")
    main_name = "random"
    if args.graph == "rmat" and args.labels == "indegree":
        r, c, rl_ms = relabel_detail(P, torch, r, c)
        main_name = "indegree"
        args.no_indegree = args.no_warm = True

    main_res, x_gpu, png = measure(P, torch, r, c, args, main_name)
    if main_name == "indegree":
        main_res["relabel_ms"] = rl_ms
    detail = {main_name: main_res}
    warm = None
    if not args.no_warm and args.iters == 0:
        warm = warm_detail(P, torch, png, args)
        detail["warm_start"] = warm
    cpu_iters = args.cpu_iters if args.cpu_iters > 0 else max(main_res["iters"], 100)
    if not args.no_cpu_baseline and cpu_iters != main_res["iters"]:
        x_gpu = P.pagerank(png, d=args.d, tol=0.0, max_iters=cpu_iters, want_hist=False).pr.cpu().numpy()
    png.close()
    if not args.no_indegree:
        ri, ci, rl_ms = relabel_detail(P, torch, r, c)
        ind_res, _, png_i = measure(P, torch, ri, ci, args, "indegree")
        png_i.close()
        ind_res["relabel_ms"] = rl_ms
        detail["indegree"] = ind_res
        del ri, ci

    if not args.no_warm and args.iters == 0 and args.graph == "rmat":
        detail["warm_eval"] = warm_eval_detail(P, torch, args)
    if not args.no_spmv:
        detail["spmv"] = spmv_detail(P, torch, r, c, args)
    if not args.no_batched:
        detail["ppr"] = ppr_detail(P, torch, args)
        detail["multigraph"] = multigraph_detail(P, torch, args)
    if not args.no_paper_scale and args.graph == "rmat" and args.scale < 26:
        detail["rmat26"] = paper_scale_detail(P, torch, args, "rmat26")
        detail["uniform"] = paper_scale_detail(P, torch, args, "uniform")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        iters = cpu_iters
        t = time.perf_counter()
        o = oracle.pagerank(r, c, d=args.d, iters=iters)
        wall = time.perf_counter() - t
        x_ref = o.x
        l1 = float(np.abs(x_gpu.astype(np.float64) - x_ref).sum())
        big = x_ref > 1.0 / n
        rel = float((np.abs(x_gpu.astype(np.float64) - x_ref)[big] / x_ref[big]).max())
        detail["parity"] = {"l1": l1, "max_rel_above_1_over_n": rel, "iters": iters}
        cpu = {"value": len(c) / o.sec_per_iter / 1e9, "unit": "GTEPS", "cores": threads(), "kind": "oracle",
               "sample": f"the same graph, {iters} FP64 pull iterations of the oracle, transpose excluded "
                         f"({wall:.1f} s wall incl. transpose)",
               "sec_per_iter": o.sec_per_iter, "host": host_info()}
        log(f"oracle: {o.sec_per_iter * 1e3:.1f} ms/iter on {threads()} threads; parity L1={l1:.2e} rel={rel:.2e}")

    g = main_res["kernels"].get("pcpm_gather", {"avg_ms": float("nan")})
    achieved = main_res["gather_bytes"] / (g["avg_ms"] * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(main_res["gteps"], 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": workload_name(args),
            "n": main_res["n"], "m": main_res["m"], "q": main_res["q"], "k": main_res["k"],
            "eprime": main_res["eprime"], "tol": solve_tol(args), "iters": main_res["iters"], "d": args.d,
        },
        "roofline": {
            "bound": "hbm", "kernel": "pcpm_gather", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (counter_traffic("pcpm::k_gather<1024, 0, %s>" % (
                "true" if main_res["update_order"] == "png" else "false")) if args.graph == "rmat" and args.part_log2 == 14
                        and args.scale == 24 and args.edge_factor == 16 and args.seed == 2 and args.labels == "random"
                        else None),
            "bytes_per_launch": main_res["gather_bytes"], "avg_launch_ms": g["avg_ms"],
        },
        "cpu_baseline": cpu,
        "hbm_gbs_algorithmic": round(main_res["hbm_gbs_alg"], 1),
        "copy_gbs": round(copy_gbs(torch), 1),
        "stream_gbs": stream_gbs(P, torch),
        "time_to_tol_ms": None if warm is None else {
            "cold": round(warm["cold_ms"], 3), "warm": round(warm["warm_ms"], 3),
            "warm_incl_indegree_count": round(warm["warm_ms_first"], 3),
            "cold_iters": warm["cold_iters"], "warm_iters": warm["warm_iters"]},
        "detail": detail,
    }
    print(json.dumps(line, default=lambda o: None if isinstance(o, float) and math.isnan(o) else o))


if __name__ == "__main__":
    main()
