"""Served form: a request loop over resident graphs with continuous batching.

Requests ask for the betweenness contribution of a source set S on one graph
(``kind="bc"``: lambda_S(v) = sum_{s in S} delta(s, v), f64[n]) or for the
dependencies of S at a few target vertices (``kind="dep"``: delta(s, t),
f64[|S|][T]).  Every resident graph has a column server (``mfbc_server_*`` in
``include/mfbc.h``): its 64-column groups move independently through the
forward loop, the counting product and the backward loop, so the sources of
requests that arrive while others are running fill a group as soon as one is
free (several small requests share one group) and share every launch with
the groups already running.  Admission is by device memory: the servers'
widths are chosen so that their footprints fit a budget; requests then wait
in a FIFO per graph for a free group.

The loop is host code (Python) around the C ABI; all product work runs in the
library's HIP kernels.  ``run_fifo`` is the reference schedule: one request
at a time, in arrival order, through the plain per-batch entry points.
"""
from __future__ import annotations

import ctypes
import time
from collections import deque
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import mfbc as _m

_P = ctypes.c_void_p
_I32, _I64 = ctypes.c_int32, ctypes.c_int64

SERVER_SIGNATURES = {
    "mfbc_server_footprint": ([_P, _I32, _P], ctypes.c_int),
    "mfbc_server_create": ([_P, _I32, ctypes.POINTER(_P)], ctypes.c_int),
    "mfbc_server_free": ([_P], ctypes.c_int),
    "mfbc_server_free_columns": ([_P], ctypes.c_int),
    "mfbc_server_active_columns": ([_P], ctypes.c_int),
    "mfbc_server_admit": ([_P, _P, _I32, _P, _P], ctypes.c_int),
    "mfbc_server_step_launch": ([_P, _P], ctypes.c_int),
    "mfbc_server_step_query": ([_P], ctypes.c_int),
    "mfbc_server_step_finish": ([_P, _P, _P, _P], ctypes.c_int),
    "mfbc_server_harvest_bc": ([_P, _P, _I32, _P, _P], ctypes.c_int),
    "mfbc_server_harvest_dep": ([_P, _P, _I32, _P, _I32, _P, _P], ctypes.c_int),
}


def _lib():
    lib = _m.load_library()
    if not getattr(lib, "_server_sigs", False):
        for name, (args, res) in SERVER_SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        lib._server_sigs = True
    return lib


def footprint(dg, width: int) -> int:
    b = ctypes.c_int64(0)
    _m._check(_lib().mfbc_server_footprint(dg.handle, width, ctypes.byref(b)))
    return int(b.value)


class ColumnServer:
    """One ``mfbc_server``: `width` source columns over a resident graph."""

    def __init__(self, dg, width: int = 256, stream=None):
        import torch
        self.torch = torch
        self.dg = dg
        self.width = width
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = ctypes.c_void_p()
        _m._check(_lib().mfbc_server_create(dg.handle, width, ctypes.byref(h)))
        self.h = h
        self.launched = False
        self._done = np.zeros(width, dtype=np.int32)

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def close(self):
        if getattr(self, "h", None):
            _lib().mfbc_server_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def free_columns(self) -> int:
        r = _lib().mfbc_server_free_columns(self.h)
        if r < 0:
            _m._check(r)
        return r

    def active_columns(self) -> int:
        r = _lib().mfbc_server_active_columns(self.h)
        if r < 0:
            _m._check(r)
        return r

    def admit(self, sources) -> np.ndarray:
        src = np.ascontiguousarray(sources, dtype=np.int32)
        cols = np.empty(src.size, dtype=np.int32)
        _m._check(_lib().mfbc_server_admit(self.h, src.ctypes.data_as(_P), src.size,
                                           cols.ctypes.data_as(_P), self._s()))
        return cols

    def step_launch(self):
        _m._check(_lib().mfbc_server_step_launch(self.h, self._s()))
        self.launched = True

    def ready(self) -> bool:
        r = _lib().mfbc_server_step_query(self.h)
        if r < 0:
            _m._check(r)
        return r == 1

    def step_finish(self) -> np.ndarray:
        self.launched = False
        nd = ctypes.c_int32(0)
        _m._check(_lib().mfbc_server_step_finish(self.h, self._done.ctypes.data_as(_P),
                                                 ctypes.byref(nd), self._s()))
        return self._done[:nd.value].copy()

    def _order_after_caller(self):
        # destination buffers are produced (zeroed) on the caller's stream
        self.stream.wait_stream(self.torch.cuda.current_stream())

    def _order_before_caller(self):
        # ... and consumed there once harvested
        self.torch.cuda.current_stream().wait_stream(self.stream)

    def harvest_bc(self, cols, dests):
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        ptrs = (ctypes.c_void_p * len(dests))(*[d.data_ptr() for d in dests])
        self._order_after_caller()
        _m._check(_lib().mfbc_server_harvest_bc(self.h, cols.ctypes.data_as(_P), cols.size,
                                                ctypes.cast(ptrs, _P), self._s()))
        self._order_before_caller()

    def harvest_dep(self, cols, targets, outs):
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        ptrs = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        self._order_after_caller()
        _m._check(_lib().mfbc_server_harvest_dep(self.h, cols.ctypes.data_as(_P), cols.size,
                                                 ctypes.c_void_p(targets.data_ptr()),
                                                 targets.numel(), ctypes.cast(ptrs, _P),
                                                 self._s()))
        self._order_before_caller()


@dataclass
class Request:
    rid: int
    graph: int
    kind: str                      # "bc" or "dep"
    sources: np.ndarray
    targets: Optional[np.ndarray] = None
    arrival: float = 0.0           # seconds after the start of the run
    # filled by the loop
    out: object = None
    placed: int = 0
    harvested: int = 0
    done: float = -1.0
    cols: dict = field(default_factory=dict)   # column -> index of the source in `sources`


class ServeEngine:
    """Resident graphs, each with a column server, and the request loop."""

    def __init__(self, dgraphs, widths):
        import torch
        self.torch = torch
        self.dgraphs = list(dgraphs)
        self.servers = [ColumnServer(dg, w) for dg, w in zip(self.dgraphs, widths)]
        self.steps = 0

    def close(self):
        for s in self.servers:
            s.close()

    def _alloc(self, r: Request):
        t = self.torch
        dg = self.dgraphs[r.graph]
        if r.kind == "bc":
            r.out = t.zeros(dg.n, dtype=t.float64, device="cuda")
        else:
            r.out = t.zeros((r.sources.size, r.targets.size), dtype=t.float64, device="cuda")
            r._targets = t.as_tensor(np.ascontiguousarray(r.targets, dtype=np.int32), device="cuda")

    def run(self, requests: List[Request], realtime: bool = True, on_step=None):
        """Serve `requests` (arrival times in seconds); returns them with `done` set.

        Each graph's server advances on its own: whenever its step has
        completed, finished columns are harvested, queued sources take the
        free columns and the next step is launched -- a small graph never
        waits for a step of a large one.
        """
        t = self.torch
        pending = sorted(requests, key=lambda r: r.arrival)
        nxt = 0
        queues = [deque() for _ in self.servers]
        owner = [dict() for _ in self.servers]           # column -> request
        left = len(pending)
        t.cuda.synchronize()
        t0 = time.perf_counter()
        while left:
            now = time.perf_counter() - t0 if realtime else float("inf")
            while nxt < len(pending) and pending[nxt].arrival <= now:
                r = pending[nxt]
                self._alloc(r)
                if r.sources.size == 0:          # nothing to compute: the zero result
                    r.done = time.perf_counter() - t0
                    left -= 1
                else:
                    queues[r.graph].append(r)
                nxt += 1
            busy = False
            for gi, srv in enumerate(self.servers):
                if srv.launched:
                    if not srv.ready():
                        busy = True
                        continue
                    done = srv.step_finish()
                    if done.size:
                        left -= self._harvest(srv, gi, done, owner, t0)
                q = queues[gi]
                free = srv.free_columns()
                while q and free:
                    r = q[0]
                    k = min(free, r.sources.size - r.placed)
                    cols = srv.admit(r.sources[r.placed:r.placed + k])
                    for j, c in enumerate(cols):
                        owner[gi][int(c)] = r
                        r.cols[int(c)] = r.placed + j
                    r.placed += k
                    free -= k
                    if r.placed == r.sources.size:
                        q.popleft()
                if srv.active_columns() > 0:
                    srv.step_launch()
                    self.steps += 1
                    busy = True
            if on_step is not None:
                on_step(self)
            if not busy and nxt < len(pending):
                wait = pending[nxt].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.002))
        return requests

    def _harvest(self, srv, gi, done, owner, t0) -> int:
        """Harvest finished columns; returns the number of requests completed."""
        by_req = {}
        for c in done:
            r = owner[gi].pop(int(c))
            by_req.setdefault(id(r), (r, []))[1].append(int(c))
        bc_cols, bc_dest = [], []
        for r, cols in by_req.values():
            if r.kind == "bc":
                bc_cols += cols
                bc_dest += [r.out] * len(cols)
            else:
                srv.harvest_dep(cols, r._targets, [r.out[r.cols[c]] for c in cols])
            r.harvested += len(cols)
        if bc_cols:
            srv.harvest_bc(bc_cols, bc_dest)
        tnow = time.perf_counter() - t0
        finished = 0
        for r, cols in by_req.values():
            if r.harvested == r.sources.size:
                r.done = tnow
                finished += 1
        return finished


def run_fifo(dgraphs, requests: List[Request], batch: int = 256, realtime: bool = True):
    """Reference schedule: each request alone, in arrival order, through the
    plain per-batch entry points (mfbc_bc, mfbc_forward + mfbc_backward)."""
    import torch
    pending = sorted(requests, key=lambda r: r.arrival)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in pending:
        if realtime:
            wait = r.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        dg = dgraphs[r.graph]
        src = torch.as_tensor(np.ascontiguousarray(r.sources, dtype=np.int32), device="cuda")
        if r.kind == "bc":
            r.out = dg.bc(src, batch)
        else:
            tg = torch.as_tensor(np.ascontiguousarray(r.targets, dtype=np.int64), device="cuda")
            rows = []
            for b0 in range(0, src.numel(), batch):
                bs = src[b0:b0 + batch]
                f = dg.forward(bs)
                d = dg.backward(bs, f["dist"], f["sigma"])["delta"]
                rows.append(d[:, tg])
                del f, d
            r.out = torch.cat(rows, dim=0) if rows else \
                torch.zeros((0, tg.numel()), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        r.done = time.perf_counter() - t0
    return requests


def latency_stats(requests) -> dict:
    lat = np.array([r.done - r.arrival for r in requests])
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3)}


def make_requests(graphs, count: int, rate: float, seed: int, smin: int = 16, smax: int = 1024,
                  dep_fraction: float = 0.5, max_targets: int = 64) -> List[Request]:
    """Poisson request trace over `graphs` (seeded; uses graphgen's trace)."""
    from .graphgen import pick_sources, poisson_trace
    t, gidx, ns = poisson_trace(rate, count, len(graphs), seed, smin, smax)
    rng = np.random.default_rng(seed + 1)
    out = []
    for i in range(count):
        g = graphs[int(gidx[i])]
        k = min(int(ns[i]), int((g.degree > 0).sum()))
        src = pick_sources(g, k, int(rng.integers(0, 2**31 - 1)))
        kind = "dep" if rng.random() < dep_fraction else "bc"
        tg = None
        if kind == "dep":
            tg = rng.choice(g.n, size=min(max_targets, g.n), replace=False).astype(np.int32)
        out.append(Request(i, int(gidx[i]), kind, src, tg, float(t[i])))
    return out
