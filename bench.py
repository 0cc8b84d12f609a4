#!/usr/bin/env python
"""MFBC benchmark on one MI355X: betweenness-centrality TEPS.

A *step* is one MFBC run (Algorithm 3) over the workload's whole source
list: every batch's forward products, counting product and backward
products, and the lambda reduction, all in libmfbc's HIP kernels.  The graph
and the source list are resident in HBM before the timed region; graph
generation and loading are not timed.

    TEPS = n_sources * m / (seconds per step),  m = unique undirected edges.

The JSON line also carries the roofline of the dominant kernel (algorithmic
bytes of its launches, from the frontier counters, over its HIP-event time)
and the CPU oracle's TEPS on a bounded sample of the same sources.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, AMD published

WORKLOADS = {
    # weighted R-MAT scale 20 (the headline): 1024 sources in batches of 256
    "rmat20_w255": dict(kind="rmat", scale=20, ef=16, wrange=(1, 255), seed=3,
                        n_sources=1024, source_seed=103, batch=256, cpu_sample=256),
    # dense Erdos-Renyi, same weights and sources
    "er32k_k512_w255": dict(kind="er", n=32768, k=512, wrange=(1, 255), seed=4,
                            n_sources=1024, source_seed=104, batch=256, cpu_sample=1024),
    # unweighted R-MAT scale 16, approximate BC from 4096 sources
    "rmat16_unw": dict(kind="rmat", scale=16, ef=16, wrange=None, seed=2,
                       n_sources=4096, source_seed=102, batch=512, cpu_sample=4096),
    # Erdos-Renyi n=1024, exact BC over all sources in batches of 64
    "er1024_w100": dict(kind="er", n=1024, k=8, wrange=(1, 100), seed=1,
                        n_sources=None, source_seed=None, batch=64, cpu_sample=None),
    # monoid fixpoints on the headline graph and sources: shortest distances
    # (min, +w) and hop levels (min, +1) from 1024 sources in batches of 256
    "sssp_rmat20_w255": dict(kind="fixpoint", op="sssp", scale=20, ef=16, wrange=(1, 255), seed=3,
                             n_sources=1024, source_seed=103, batch=256, cpu_sample=6),
    "bfs_rmat20": dict(kind="fixpoint", op="bfs", scale=20, ef=16, wrange=(1, 255), seed=3,
                       n_sources=1024, source_seed=103, batch=256, cpu_sample=10),
    # the same graph and sources with the other two algebras of the generic
    # product: widest-path bottlenecks (max, min(a, w)) and binary32 sums of
    # 1/w (min, a + 1/w)
    "widest_rmat20_w255": dict(kind="fixpoint", op="widest", scale=20, ef=16, wrange=(1, 255), seed=3,
                               n_sources=1024, source_seed=103, batch=256, cpu_sample=4),
    "resist_rmat20_w255": dict(kind="fixpoint", op="resist", scale=20, ef=16, wrange=(1, 255), seed=3,
                               n_sources=1024, source_seed=103, batch=256, cpu_sample=4),
    # batched form: 256 ER / R-MAT graphs, n log-uniform in [200, 20000], average
    # degree uniform in [4, 64], weights 1..100, exact BC of every graph
    "batched256": dict(kind="many", count=256, seed0=1000, cpu_sample=48),
    # served form: 8 resident weighted R-MAT graphs (scales 14..20 and a second
    # 17), Poisson requests for BC contributions or dependencies of 16..1024
    # sources, continuous batching of source columns vs one request at a time
    "served8": dict(kind="serve", scales=(14, 15, 16, 17, 18, 19, 20, 17), seed0=2000,
                    trace_seed=2100, width=256, heavy_plain=True),
}


def make_graph(spec):
    from paper_1609_07008_amd import graphgen as gg
    if spec["kind"] in ("rmat", "fixpoint"):
        return gg.rmat_graph(spec["scale"], spec["ef"], spec["seed"], wrange=spec["wrange"])
    return gg.er_graph(spec["n"], spec["k"], spec["seed"], spec["wrange"])


def make_sources(g, spec):
    import numpy as np
    from paper_1609_07008_amd import graphgen as gg
    if spec["n_sources"] is None:
        return np.arange(g.n, dtype=np.int32)
    return gg.pick_sources(g, spec["n_sources"], spec["source_seed"])


KERNEL_SOURCES = ("pull.h", "products.h", "kernels.hip", "monoid.hip", "mfbc_internal.h")


def kernel_sha(csrc=None):
    """Hash of the kernel sources with comments and blank space removed (so a
    record of measured traffic outlives edits that do not change the code)."""
    import re
    csrc = csrc or os.path.join(ROOT, "paper_1609_07008_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def stored_traffic(workload, kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, if still valid."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_sha") != kernel_sha():
        return None            # the kernel changed since the counters were taken
    return rec.get("hbm_bytes_per_launch")


def copy_rate_gbs(torch, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Bytes per second a plain device-to-device copy moves (read + write):
    the practical ceiling of HBM traffic on this GPU, measured after the
    timed region next to the kernel's own rate."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return round(2 * nbytes / (ms * 1e-3) / 1e9, 1)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(g, src, sample, m, one_thread_sample=8):
    """The C oracle (Brandes, FP64, OpenMP over sources) on the host: a bounded
    sample of the workload's sources on every host thread, and a smaller one
    on one thread."""
    import numpy as np
    import oracle
    k = src.size if sample is None else min(sample, src.size)
    s = np.ascontiguousarray(src[:k])
    threads = oracle.brandes_threads()
    t0 = time.perf_counter()
    oracle.brandes(g, s, per_source=False, nthreads=threads)
    dt = time.perf_counter() - t0
    k1 = min(one_thread_sample, k)
    t0 = time.perf_counter()
    oracle.brandes(g, np.ascontiguousarray(src[:k1]), per_source=False, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": k * m / dt, "unit": "TEPS", "cores": threads, "kind": "oracle",
            "sample": f"{k} of the workload's {src.size} sources (C Brandes, FP64, "
                      f"OpenMP over sources), {dt:.2f} s",
            "cpu": cpu_model(),
            "one_thread": {"value": k1 * m / dt1, "unit": "TEPS", "sources": k1, "seconds": round(dt1, 3)}}


def relaxation_census(dg, d_src, batch, g):
    """Relaxations (Section 5's flops of each product: every frontier entry
    combined along each of its arcs) of one MFBC run over the source list, from
    an untimed traced run: forward products from the recorded per-product
    counts; the counting product relaxes every reachable (source, vertex)
    along its arcs; every backward product relaxes each non-source entry of
    its frontier, and each reachable non-source entry enters exactly once."""
    import torch
    deg = torch.as_tensor(g.row_ptr[1:] - g.row_ptr[:-1], device="cuda", dtype=torch.int64)
    fwd = cnt = bwd = 0
    products = 0
    for b0 in range(0, d_src.numel(), batch):
        sb = d_src[b0:b0 + batch]
        f = dg.forward(sb, trace=True, frontiers=False, max_products=dg.n + 2)
        fwd += int(f["relax"].sum())
        products += f["products"]
        reach = f["dist"] != 0x7FFFFFFF
        cnt += int((reach.to(torch.int64) * deg).sum())
        bwd += int((reach.to(torch.int64) * deg).sum() - deg[sb.long()].sum())
        del f, reach
    return {"forward": fwd, "counting": cnt, "backward": bwd, "total": fwd + cnt + bwd,
            "forward_products": products}


def run_many(args, spec):
    """Batched form: one persistent launch over every graph, against one
    mfbc_bc launch sequence per graph on the same GPU (batches of 64 and 256)."""
    import numpy as np
    import torch
    from paper_1609_07008_amd import graphgen as gg
    from paper_1609_07008_amd import mfbc

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    gs = gg.batched_suite(spec["count"], spec["seed0"])
    dgs = [mfbc.DeviceGraph(g) for g in gs]
    srcs = [torch.arange(g.n, dtype=torch.int32, device="cuda") for g in gs]
    outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for g in gs]
    work = sum(g.n * g.m for g in gs)
    print(f"[bench] batched: {len(gs)} graphs, sum n = {sum(g.n for g in gs)}, "
          f"sum n*m = {work:.3e}, setup {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    from paper_1609_07008_amd import autotune
    cache = autotune.load_cache()
    if args.tune or "job_width" not in cache.get("many", {}) or "many_plan" not in cache:
        pick = list(range(0, len(gs), 4))           # every fourth graph
        autotune.tune_many([dgs[i] for i in pick], [srcs[i] for i in pick], cache=cache,
                           verbose=True)
        autotune.save_cache(cache)
    cfg = autotune.many_config(cache)
    plans = autotune.apply_many_plans(dgs, cache)
    if args.block_threads:
        cfg["block_threads"] = args.block_threads
    if args.blocks:
        cfg["blocks"] = args.blocks
    for _ in range(args.warmup):
        mfbc.bc_many(dgs, srcs, outs=outs, **cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mfbc.bc_many(dgs, srcs, outs=outs, **cfg)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    st = mfbc.bc_many.last_stats
    # the plain per-graph method on the same GPU, at two batch sizes; the
    # speedup is taken against the faster one
    plain = {}
    for d, g in zip(dgs, gs):                      # the per-graph path runs its own tuned plans
        autotune.apply_plan(d, g, cache) or d.set_plan()
    for batch in (() if args.no_baseline else (64, 256)):
        for d, s, o in zip(dgs, srcs, outs):
            d.bc(s, batch, out=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for d, s, o in zip(dgs, srcs, outs):
            d.bc(s, batch, out=o)
        torch.cuda.synchronize()
        plain[batch] = time.perf_counter() - t0
        print(f"[bench] per-graph launch sequences, batch {batch}: {plain[batch]:.2f} s",
              file=sys.stderr, flush=True)
    best = min(plain, key=plain.get) if plain else None
    el_plain = plain[best] if plain else float("nan")
    line = {
        "metric": "BC TEPS (sources x edges / s) at 1 GPU", "value": work / el, "unit": "TEPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched256", "graphs": len(gs), "sum_n": int(sum(g.n for g in gs)),
                   "sum_m": int(sum(g.m for g in gs)), "launch": cfg,
                   "plans_by_size": {b: {"run_arcs": p[0], "run_verts": p[1]} for b, p in plans.items()},
                   "fwd_products": st["fwd_products"], "bwd_products": st["bwd_products"]},
        "per_graph_baseline": {"value": work / el_plain, "unit": "TEPS", "ms": el_plain * 1e3,
                               "method": f"one mfbc_bc launch sequence per graph, batch {best} "
                                         f"(the faster of 64 and 256)",
                               "ms_by_batch": {str(b): t * 1e3 for b, t in plain.items()}},
        "speedup_vs_per_graph": el_plain / el,
        "roofline": None, "cpu_baseline": None,
    }
    if not args.no_cpu:
        import oracle
        rng = np.random.default_rng(5)
        pick = rng.choice(len(gs), size=min(spec["cpu_sample"], len(gs)), replace=False)
        threads = oracle.brandes_threads()
        t0 = time.perf_counter()
        w = 0
        for i in pick:
            g = gs[int(i)]
            oracle.brandes(g, np.arange(g.n, dtype=np.int32), per_source=False, nthreads=threads)
            w += g.n * g.m
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": w / dt, "unit": "TEPS", "cores": threads, "kind": "oracle",
                                "sample": f"{len(pick)} of the {len(gs)} graphs, all sources, {dt:.2f} s"}
    for d in dgs:
        d.close()
    print(json.dumps(line), flush=True)


def run_serve(args, spec):
    import numpy as np
    import torch
    from paper_1609_07008_amd import graphgen as gg
    from paper_1609_07008_amd import mfbc, serve

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    gs = [gg.rmat_graph(sc, 16, spec["seed0"] + i, wrange=(1, 255))
          for i, sc in enumerate(spec["scales"])]
    dgs = [mfbc.DeviceGraph(g) for g in gs]
    foot = sum(serve.footprint(d, spec["width"]) for d in dgs)
    print(f"[bench] served: {len(gs)} graphs, server state {foot / 2**30:.1f} GiB, "
          f"setup {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    nreq = args.requests

    def trace(rate, seed):
        return serve.make_requests(gs, nreq, rate, seed)

    def work(reqs):
        return sum(r.sources.size * gs[r.graph].m for r in reqs)

    # saturation rate of the plain method: every request queued at time 0
    sat = trace(1e9, spec["trace_seed"])
    for r in sat:
        r.arrival = 0.0
    serve.run_fifo(dgs, sat[: min(40, nreq)], realtime=False)          # warm-up
    t1 = time.perf_counter()
    serve.run_fifo(dgs, sat, realtime=False)
    rate_sat = nreq / (time.perf_counter() - t1)
    print(f"[bench] plain method saturates at {rate_sat:.2f} requests/s", file=sys.stderr, flush=True)
    # servers admitted by memory footprint within a budget of 80% of the free
    # device memory, up to the workload's width per graph
    lag = None if args.light_lag < 0 else args.light_lag
    width = args.serve_width or spec["width"]
    heavy_plain = spec["heavy_plain"] and not args.no_heavy_plain
    eng = serve.ServeEngine(dgs, budget_bytes=args.serve_budget or None, max_width=width,
                            light_lag=lag, heavy_plain=heavy_plain)
    out = {}
    for frac in (0.5, 0.9):
        reqs = trace(frac * rate_sat, spec["trace_seed"] + int(frac * 10))
        t1 = time.perf_counter()
        eng.run(reqs)
        el = time.perf_counter() - t1
        res = {"served": dict(serve.latency_stats(reqs), teps=work(reqs) / el, wall_s=el)}
        print(f"[bench] load {frac}: served p50/p99 {res['served']['p50_ms']:.1f}/"
              f"{res['served']['p99_ms']:.1f} ms ({eng.steps} steps so far)", file=sys.stderr, flush=True)
        reqs2 = trace(frac * rate_sat, spec["trace_seed"] + int(frac * 10))
        t1 = time.perf_counter()
        serve.run_fifo(dgs, reqs2)
        el2 = time.perf_counter() - t1
        res["fifo"] = dict(serve.latency_stats(reqs2), teps=work(reqs2) / el2, wall_s=el2)
        print(f"[bench] load {frac}: fifo p50/p99 {res['fifo']['p50_ms']:.1f}/"
              f"{res['fifo']['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
        out[f"load_{frac}"] = res
    main_res = out["load_0.9"]["served"]
    line = {
        "metric": "BC TEPS (sources x edges / s) at 1 GPU; serving p50/p99 latency",
        "value": main_res["teps"], "unit": "TEPS", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": main_res["wall_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "served8", "graphs": [g.name for g in gs], "requests": nreq,
                   "width": width, "saturation_rate_plain": rate_sat, "light_lag_s": lag,
                   "heavy_plain": heavy_plain,
                   "admission": {"budget_bytes": eng.mem.budget, "peak_bytes": eng.mem.peak,
                                 "rejected": eng.rejected, "steps": eng.steps,
                                 "merged": eng.merged}},
        "serving": out, "roofline": None, "cpu_baseline": None,
    }
    eng.close()
    for d in dgs:
        d.close()
    print(json.dumps(line), flush=True)


def run_fixpoint(args, spec):
    """Monoid fixpoint (mfbc_fixpoint) over the workload's sources, batch by batch."""
    import numpy as np
    import torch
    from paper_1609_07008_amd import autotune, mfbc

    torch.cuda.set_device(0)
    g = make_graph(spec)
    src = make_sources(g, spec)
    batch = args.batch or spec["batch"]
    dg = mfbc.DeviceGraph(g)
    autotune.apply_plan(dg, g, autotune.load_cache())
    d_src = torch.as_tensor(src, device="cuda")
    vtype = torch.float32 if spec["op"] == "resist" else torch.int32
    out = torch.empty((batch, g.n), dtype=vtype, device="cuda")
    print(f"[bench] {args.workload}: n={g.n} m={g.m} sources={src.size} batch={batch}",
          file=sys.stderr, flush=True)

    def step(stats):
        prods = 0
        for b0 in range(0, src.size, batch):
            sb = d_src[b0:b0 + batch]
            _, p = dg.fixpoint(sb, spec["op"], out=out[:sb.numel()])
            prods += p
            if stats is not None:
                for k, v in dg.stats().items():
                    stats[k] = stats.get(k, 0) + v
        return prods

    for i in range(args.warmup):
        step(None)
        torch.cuda.synchronize()
    dg.enable_timing(1 if args.stats else 2)      # 2: events around the product kernels only
    tot = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        prods = step(tot)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dg.enable_timing(False)
    print(f"[bench] {args.steps} steps in {elapsed:.3f}s, {prods} products per step",
          file=sys.stderr, flush=True)
    ms, alg, launches = tot["fwd_pull_ms"], tot["fwd_alg_bytes"], tot["fwd_pull_launches"]
    achieved = alg / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    line = {
        "metric": f"{spec['op'].upper()} TEPS (sources x edges / s) at 1 GPU",
        "value": src.size * g.m / (elapsed / args.steps), "unit": "TEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if spec["op"] == "resist" else "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": g.name, "n": g.n, "m": g.m,
                   "n_sources": int(src.size), "batch": batch, "op": spec["op"]},
        "roofline": {"bound": "hbm", "kernel": "k_mono_pull", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": stored_traffic(args.workload, "k_mono_pull"),
                     "launches": int(launches), "avg_launch_us": round(ms / max(launches, 1) * 1e3, 2),
                     "alg_bytes_per_launch": round(alg / max(launches, 1)),
                     "copy_gbs": copy_rate_gbs(torch)},
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        from oracle.frontier import InArcs, fixpoint
        k = min(spec["cpu_sample"], src.size)
        t1 = time.perf_counter()
        arcs = InArcs(g, unit_weights=spec["op"] == "bfs")
        for s in src[:k]:
            fixpoint(g, int(s), spec["op"], arcs=arcs)
        dt = time.perf_counter() - t1
        line["cpu_baseline"] = {"value": k * g.m / dt, "unit": "TEPS", "cores": 1, "kind": "oracle",
                                "sample": f"{k} of the workload's {src.size} sources (numpy "
                                          f"relaxation to the fixpoint, one source at a time), {dt:.2f} s"}
    dg.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat20_w255", choices=sorted(WORKLOADS))
    ap.add_argument("--batch", type=int, default=None, help="override the batch size")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-census", action="store_true",
                    help="skip the untimed traced run that counts relaxations (for profiler runs)")
    ap.add_argument("--stats", action="store_true", help="print per-kernel stats to stderr")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (calibrates the "
                         "HBM byte counters of rocprofv3) and exit")
    ap.add_argument("--tune", action="store_true", help="re-run the autotuner before timing")
    ap.add_argument("--lanes", type=int, default=-1,
                    help="batches of one call run at once (1..4; 0 = by size; default: tuned)")
    ap.add_argument("--no-baseline", action="store_true",
                    help="batched form: skip the per-graph comparison")
    ap.add_argument("--requests", type=int, default=2000, help="served form: requests per trace")
    ap.add_argument("--serve-width", type=int, default=0,
                    help="served form: widest column server per graph (multiple of 128; 0: the workload's)")
    ap.add_argument("--no-heavy-plain", action="store_true",
                    help="served form: heavy graphs get column servers too (by default their "
                         "requests run whole through the plain path)")
    ap.add_argument("--light-lag", type=float, default=-1.0,
                    help="served form: light requests arriving this many seconds after the oldest "
                         "unfinished heavy request wait for it (negative: off)")
    ap.add_argument("--serve-budget", type=int, default=0,
                    help="served form: device-memory budget of the column servers in bytes "
                         "(0 = 80%% of the free memory)")
    ap.add_argument("--block-threads", type=int, default=0, help="batched form: threads per workgroup")
    ap.add_argument("--blocks", type=int, default=0, help="batched form: persistent workgroups")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        torch.cuda.set_device(0)
        a = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X; "
              "a multi-GPU run (source batches sharded over GPUs, one allreduce of lambda) "
              "is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1609_07008_amd import mfbc

    spec = WORKLOADS[args.workload]
    if spec["kind"] == "many":
        run_many(args, spec)
        return
    if spec["kind"] == "serve":
        run_serve(args, spec)
        return
    if spec["kind"] == "fixpoint":
        run_fixpoint(args, spec)
        return
    batch = args.batch or spec["batch"]
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    g = make_graph(spec)
    src = make_sources(g, spec)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    dg = mfbc.DeviceGraph(g)
    from paper_1609_07008_amd import autotune
    cache = autotune.load_cache()
    if args.tune or not autotune.apply_plan(dg, g, cache):
        best, _ = autotune.tune_plan(dg, g, src, batch, cache=cache, verbose=True)
        autotune.save_cache(cache)
    if args.lanes >= 0:
        dg.set_lanes(args.lanes)
    d_src = torch.as_tensor(src, device="cuda")
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t_load = time.perf_counter() - t0
    print(f"[bench] {args.workload}: n={g.n} m={g.m} arcs={g.arcs} sources={src.size} "
          f"batch={batch} gen {t_gen:.1f}s load {t_load:.1f}s", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        dg.bc(d_src, batch, out=out)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    # events around the forward product kernels only (the dominant kernel of
    # every BC workload here: every event costs the stream a few microseconds,
    # 4.2 ms of a 7.6 ms step on the 1,024-vertex graph with all kernels
    # timed); --stats times every kernel
    dg.enable_timing(1 if args.stats else 2)
    tot = {}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        dg.bc(d_src, batch, out=out)
        st = dg.stats()
        for k, v in st.items():
            tot[k] = tot.get(k, 0) + v
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    dg.enable_timing(False)
    print(f"[bench] {args.steps} steps in {elapsed:.3f}s", file=sys.stderr, flush=True)

    ms_step = elapsed / args.steps * 1e3
    teps = src.size * g.m / (elapsed / args.steps)
    census = None if args.no_census else relaxation_census(dg, d_src, batch, g)
    if census:
        print(f"[bench] relaxations per step: {census}", file=sys.stderr, flush=True)

    kernels = {
        "k_fwd_pull": (tot["fwd_pull_ms"], tot["fwd_alg_bytes"], tot["fwd_pull_launches"]),
        "k_bwd_pull": (tot["bwd_pull_ms"], tot["bwd_alg_bytes"], tot["bwd_pull_launches"]),
        "k_bwd_count": (tot["count_ms"], tot["count_alg_bytes"], tot["count_launches"]),
    }
    dom = max(kernels, key=lambda k: kernels[k][0])
    ms, alg, launches = kernels[dom]
    achieved = alg / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    traffic = stored_traffic(args.workload, dom)
    # batches of two or more column groups run the forward product two groups per wave
    label = "k_fwd_pull_w" if dom == "k_fwd_pull" and min(batch, src.size) > 64 else dom
    avg_us = ms / max(launches, 1) * 1e3
    roofline = {"bound": "hbm", "kernel": label, "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "launches": int(launches),
                "avg_launch_us": round(avg_us, 2),
                "alg_bytes_per_launch": round(alg / max(launches, 1)),
                "achieved_basis": "algorithmic bytes (frontier-counter model) per launch / "
                                  "HIP-event kernel time per launch",
                "traffic_rate_gbs": (round(traffic / (avg_us * 1e-6) / 1e9, 1)
                                     if traffic else None),
                "copy_gbs": copy_rate_gbs(torch)}
    if args.stats:
        for k, (kms, kb, kl) in kernels.items():
            print(f"[bench] {k}: {kms / args.steps:.2f} ms/step over {kl // args.steps} launches, "
                  f"{kb / max(kms, 1e-9) / 1e6:.1f} GB/s algorithmic", file=sys.stderr)
        print("[bench] stats " + json.dumps({k: v / args.steps for k, v in tot.items()}),
              file=sys.stderr)

    line = {
        "metric": "BC TEPS (sources x edges / s) at 1 GPU",
        "value": teps,
        "unit": "TEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": g.name, "n": g.n, "m": g.m,
                   "arcs": g.arcs, "weights": None if spec["wrange"] is None else list(spec["wrange"]),
                   "n_sources": int(src.size), "batch": batch,
                   "fwd_products_per_step": tot["fwd_products"] / args.steps,
                   "bwd_products_per_step": tot["bwd_products"] / args.steps},
        "relaxations_per_step": census["total"] if census else None,
        "relaxations_per_s": census["total"] / (elapsed / args.steps) if census else None,
        "relaxations": census,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(g, src, spec["cpu_sample"], g.m)
    dg.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
