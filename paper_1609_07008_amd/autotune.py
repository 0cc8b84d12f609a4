"""Autotuner for the work decomposition and launch shapes, measured on the device.

Knobs (none changes results beyond floating-point summation order, only speed):
  * per graph: the pull-task decomposition of ``mfbc_set_plan`` -- light rows
    grouped into runs of at most ``run_verts`` rows and about ``run_arcs``
    arcs (hub rows are always cut into slices) -- and, for graphs whose
    products are too small to fill the device, the number of batches of one
    ``mfbc_bc`` call that run at once (``mfbc_set_lanes``);
  * batched form: threads per workgroup, persistent workgroups and sources
    per job (64, or 128 on the paired products) of ``mfbc_bc_many`` for the
    whole launch, and the run sizes of the graphs of each size class inside
    it (``many_bucket``).

Choices are cached per device architecture and graph-size bucket (vertex
count, average degree, weighted or not) in ``tuned_<arch>.json`` next to
this module, so a later run applies them without measuring again.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))

PLAN_CANDIDATES = [(64, 1), (128, 4), (256, 16), (512, 16), (256, 64), (512, 64), (1024, 64),
                   (2048, 64)]
MANY_CANDIDATES = [(512, 4), (256, 8), (256, 6), (512, 2)]      # (threads, workgroups per CU)
MANY_WIDTHS = (64, 128)                                          # sources per job
MANY_PLAN_CANDIDATES = [(0, 0), (64, 1), (128, 4), (256, 16), (1024, 64), (4096, 64)]   # (0, 0): size default


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def cache_path(arch: str = None) -> str:
    return os.path.join(_HERE, f"tuned_{arch or _arch()}.json")


def load_cache(arch: str = None) -> dict:
    p = cache_path(arch)
    if not os.path.exists(p):
        return {}
    with open(p) as fh:
        return json.load(fh)


def save_cache(cache: dict, arch: str = None):
    p = cache_path(arch)
    tmp = p + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, p)


def bucket(n: int, arcs: int, weighted: bool) -> str:
    k = max(arcs / max(n, 1), 1.0)
    return f"n2^{int(math.ceil(math.log2(max(n, 2))))}_k2^{int(round(math.log2(k)))}_{'w' if weighted else 'u'}"


def graph_bucket(g) -> str:
    return bucket(g.n, g.arcs, g.w is not None)


def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


LANE_CANDIDATES = (1, 2, 4)
# lanes are tuned only where one product of a batch is small next to the
# device (arcs x column groups below this): on large products concurrent
# batches only share the memory bandwidth, and each kernel's own duration --
# the denominator of its roofline figure -- would stretch
LANE_TUNE_MAX = 1 << 25


def tune_plan(dg, g, sources, batch: int, reps: int = 2, cache: dict = None, verbose=False):
    """Pick the run sizes of one graph by timing mfbc_bc on one batch of
    sources, then (small products only) the lane count on up to four batches."""
    import torch
    src = torch.as_tensor(np.ascontiguousarray(sources[:batch], dtype=np.int32), device="cuda")
    res = {}
    dg.set_lanes(1)
    for ra, rv in PLAN_CANDIDATES:
        dg.set_plan(run_arcs=ra, run_verts=rv)
        res[(ra, rv)] = _time(lambda: dg.bc(src, batch), reps)
        if verbose:
            print(f"[tune] {g.name} run_arcs={ra} run_verts={rv}: {res[(ra, rv)] * 1e3:.2f} ms",
                  file=sys.stderr, flush=True)
    best = min(res, key=res.get)
    dg.set_plan(run_arcs=best[0], run_verts=best[1])
    lanes = 0
    ncg = -(-min(batch, len(sources)) // 64)
    if g.arcs * ncg < LANE_TUNE_MAX:
        src4 = torch.as_tensor(np.ascontiguousarray(sources[:4 * batch], dtype=np.int32),
                               device="cuda")
        lres = {}
        for L in LANE_CANDIDATES:
            dg.set_lanes(L)
            lres[L] = _time(lambda: dg.bc(src4, batch), reps)
            if verbose:
                print(f"[tune] {g.name} lanes={L}: {lres[L] * 1e3:.2f} ms", file=sys.stderr, flush=True)
        lanes = min(lres, key=lres.get)
    dg.set_lanes(lanes if lanes else 1)
    if cache is not None:
        cache.setdefault("plan", {})[graph_bucket(g)] = {"run_arcs": best[0], "run_verts": best[1],
                                                         "lanes": lanes if lanes else 1,
                                                         "ms": res[best] * 1e3}
    return best, res


def apply_plan(dg, g, cache: dict) -> bool:
    """Set a graph's plan (and lane count) from the cache (returns False if
    its bucket is unknown)."""
    e = cache.get("plan", {}).get(graph_bucket(g))
    if not e:
        return False
    dg.set_plan(run_arcs=e["run_arcs"], run_verts=e["run_verts"])
    if "lanes" in e:
        dg.set_lanes(e["lanes"])
    return True


def many_bucket(n: int) -> str:
    """Size class of a graph in the batched form (vertex count)."""
    return "n<=2^10" if n <= 1024 else ("n<=2^12" if n <= 4096 else "n>2^12")


def tune_many(dgs, srcs, reps: int = 1, cache: dict = None, verbose=False):
    """Pick the batched form's launch (threads, workgroups per CU, sources
    per job) on (a sample of) its graphs, then the run sizes of each size
    class: the class's graphs alone, in the chosen launch, under each plan."""
    import torch
    from . import mfbc
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    outs = [torch.empty(d.n, dtype=torch.float64, device="cuda") for d in dgs]
    for d in dgs:
        d.set_plan()
    res = {}
    for width in MANY_WIDTHS:
        for threads, per_cu in MANY_CANDIDATES:
            cfg = dict(block_threads=threads, blocks=per_cu * cus, job_width=width)
            key = (threads, per_cu, width)
            res[key] = _time(lambda: mfbc.bc_many(dgs, srcs, outs=outs, **cfg), reps)
            if verbose:
                print(f"[tune] many threads={threads} per_cu={per_cu} job_width={width}: "
                      f"{res[key]:.3f} s", file=sys.stderr, flush=True)
    best = min(res, key=res.get)
    cfg = dict(block_threads=best[0], blocks=best[1] * cus, job_width=best[2])
    plans = {}
    classes = {}
    for i, d in enumerate(dgs):
        classes.setdefault(many_bucket(d.n), []).append(i)
    for b, idx in sorted(classes.items()):
        sub = [dgs[i] for i in idx]
        ssrc = [srcs[i] for i in idx]
        sout = [outs[i] for i in idx]
        pres = {}
        for ra, rv in MANY_PLAN_CANDIDATES:
            for d in sub:
                d.set_plan(run_arcs=ra, run_verts=rv)
            pres[(ra, rv)] = _time(lambda: mfbc.bc_many(sub, ssrc, outs=sout, **cfg), reps)
            if verbose:
                print(f"[tune] many {b} ({len(sub)} graphs) run_arcs={ra} run_verts={rv}: "
                      f"{pres[(ra, rv)] * 1e3:.1f} ms", file=sys.stderr, flush=True)
        pb = min(pres, key=pres.get)
        for d in sub:
            d.set_plan(run_arcs=pb[0], run_verts=pb[1])
        plans[b] = {"run_arcs": pb[0], "run_verts": pb[1], "ms": pres[pb] * 1e3,
                    "graphs_tuned_on": len(sub)}
    if cache is not None:
        cache["many"] = {"block_threads": best[0], "per_cu": best[1], "job_width": best[2],
                         "s": res[best]}
        cache["many_plan"] = plans
    return best, res


def many_config(cache: dict) -> dict:
    import torch
    e = cache.get("many")
    if not e:
        return {}
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    return {"block_threads": e["block_threads"], "blocks": e["per_cu"] * cus,
            "job_width": e.get("job_width", 64)}


def apply_many_plans(dgs, cache: dict) -> dict:
    """Set every graph's run sizes from its size class's tuned plan (the size
    default where the class is unknown); returns the plans applied per class."""
    plans = cache.get("many_plan", {})
    used = {}
    for d in dgs:
        b = many_bucket(d.n)
        e = plans.get(b)
        if e:
            d.set_plan(run_arcs=e["run_arcs"], run_verts=e["run_verts"])
            used[b] = (e["run_arcs"], e["run_verts"])
        else:
            d.set_plan()
    return used
