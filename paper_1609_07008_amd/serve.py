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
import threading
import time
from collections import deque
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

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
    "mfbc_server_set_rounds": ([_P, _I32], ctypes.c_int),
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

    def __init__(self, dg, width: int = 256, stream=None, rounds: int = 0):
        import torch
        self.torch = torch
        self.dg = dg
        self.width = width
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = ctypes.c_void_p()
        _m._check(_lib().mfbc_server_create(dg.handle, width, ctypes.byref(h)))
        self.h = h
        if rounds:
            _m._check(_lib().mfbc_server_set_rounds(h, int(rounds)))
        self.launched = False
        self.owned = 0             # columns admitted and not yet harvested
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
    started: float = -1.0          # when its first source was admitted or its plain run began
    error: Optional[str] = None    # set when the request was rejected (nothing computed)
    cols: dict = field(default_factory=dict)   # column -> index of the source in `sources`


class MemoryBudget:
    """Admission of column servers by device-memory footprint (host logic only).

    ``footprint(g, w)`` gives the bytes a server of ``w`` columns (a multiple
    of 64) on graph ``g`` allocates.  ``acquire`` decides the width of a new
    server for ``g`` given the columns its waiting sources need and which other
    servers are idle, keeping the sum of live footprints within ``budget``.
    """

    def __init__(self, budget: int, footprint, max_width: int = 256):
        if max_width < 64 or max_width % 64:
            raise ValueError("max_width must be a positive multiple of 64")
        self.budget = int(budget)
        self.footprint = footprint
        self.max_width = max_width
        self.live = {}            # graph -> (width, bytes)
        self.last_use = {}        # graph -> logical time of the last step
        self.clock = 0
        self.peak = 0             # largest sum of live footprints seen

    @property
    def used(self) -> int:
        return sum(b for _, b in self.live.values())

    def fits_ever(self, g) -> bool:
        """Whether a 64-column server of g fits the whole budget."""
        return self.footprint(g, 64) <= self.budget

    def touch(self, g):
        self.clock += 1
        self.last_use[g] = self.clock

    def acquire(self, g, want_cols: int, idle) -> Tuple[Optional[int], list]:
        """Width for a new server of g (None: wait) and the idle servers to
        release first.  ``idle(h)`` tells whether graph h's server holds no
        column in use."""
        assert g not in self.live
        want = min(self.max_width, max(64, -(-int(want_cols) // 64) * 64))
        free = self.budget - self.used
        widths = list(range(want, 0, -64))
        for w in widths:                       # widest that fits without releasing anything
            if self.footprint(g, w) <= free:
                return w, []
        victims = sorted((h for h in self.live if h != g and idle(h)),
                         key=lambda h: self.last_use.get(h, 0))
        for w in widths:                       # then release idle servers, oldest first
            need = self.footprint(g, w)
            f, ev = free, []
            for h in victims:
                if f >= need:
                    break
                ev.append(h)
                f += self.live[h][1]
            if f >= need:
                return w, ev
        return None, []

    def add(self, g, width: int):
        self.live[g] = (width, self.footprint(g, width))
        self.touch(g)
        self.peak = max(self.peak, self.used)

    def remove(self, g):
        self.live.pop(g, None)


def default_budget(fraction: float = 0.8) -> int:
    """A fraction of the device memory free now."""
    import torch
    return int(torch.cuda.mem_get_info()[0] * fraction)


class ServeEngine:
    """Resident graphs, column servers admitted by memory footprint, and the
    request loop.

    ``widths``: one fixed server per graph of the given widths (created up
    front; their footprints must fit the budget).  Without it, servers are
    created on demand by ``MemoryBudget`` (``budget_bytes``, default 80% of
    the free device memory; widths up to ``max_width``)."""

    def __init__(self, dgraphs, widths=None, budget_bytes: Optional[int] = None,
                 max_width: int = 256, server_factory=None, footprint_fn=None,
                 device: str = "cuda", heavy_arcs: Optional[int] = 1 << 22, max_heavy: int = 1,
                 light_lag: Optional[float] = None, heavy_plain: bool = False, plain_batch: int = 256,
                 plain_fn=None, plain_many_fn=None, plain_merge: bool = True,
                 light_yield: Optional[float] = None):
        """``server_factory(dgraph, width)`` and ``footprint_fn(dgraph, width)``
        default to ColumnServer and mfbc_server_footprint (other executors
        can be plugged in, e.g. to test the scheduling on the CPU);
        ``device``: where request results are allocated.

        Heavy graphs (more than ``heavy_arcs`` arcs; None: no graph is heavy)
        advance one step at a time in order of their oldest request: at most
        ``max_heavy`` of their servers have steps in flight, chosen by the
        arrival of the oldest request they hold or queue, while light graphs'
        servers run alongside.  Sharing the device between several heavy
        graphs would stretch each of their requests (every one of their
        products is bound by the memory bandwidth the others also use); light
        graphs' products take little of it and keep their short latency.

        ``light_lag`` (seconds; None: off): a light graph's request that
        arrived more than this after the oldest unfinished heavy request is
        not admitted until that heavy request is done (columns already
        admitted run on), so light work never queues ahead of an older
        heavy request for long -- the heavy request sees the device much as
        it would in arrival order, and light requests older than it still
        run alongside.

        ``heavy_plain``: heavy graphs get no column server; their requests
        run whole, one at a time in arrival order, through the plain path
        (``plain_fn(dgraph, request, plain_batch)``, default run_plain) on
        the worker's own stream, while light graphs' servers run alongside.
        The plain path's workspace (the footprint of a ``plain_batch``-wide
        server) is reserved in the budget up front.

        ``plain_merge``: when the oldest request of a heavy graph is a BC sum,
        queued BC requests of the same graph that fit the free column groups
        of its last batch run with it in one call
        (``plain_many_fn(dgraph, requests, plain_batch)``, default
        run_plain_many: mfbc_bc_requests), so they add no batch of their
        own.  A caller-supplied ``plain_fn`` without ``plain_many_fn`` turns
        merging off.

        ``light_yield`` (seconds; None: off): while a heavy request is in
        service, a light graph launches a step only if its oldest unfinished
        request arrived at least this long ago -- heavy requests get the
        device to themselves unless light work has waited that long."""
        import torch
        self.torch = torch
        self.device = device
        self.dgraphs = list(dgraphs)
        self.factory = server_factory or ColumnServer
        fp = footprint_fn or footprint
        budget = (default_budget() if budget_bytes is None else int(budget_bytes))
        self.mem = MemoryBudget(budget, lambda gi, w: fp(self.dgraphs[gi], w), max_width)
        self.fixed = widths is not None
        self.servers = [None] * len(self.dgraphs)
        self.steps = 0
        self.rejected = 0
        self.heavy = [heavy_arcs is not None and getattr(dg, "arcs", 0) > heavy_arcs
                      for dg in self.dgraphs]
        self.max_heavy = max_heavy
        self.light_lag = light_lag
        self.heavy_plain = heavy_plain
        self.plain_batch = plain_batch
        self.plain_fn = plain_fn or run_plain
        self.plain_many_fn = plain_many_fn or (run_plain_many if plain_fn is None else None)
        self.plain_merge = plain_merge and self.plain_many_fn is not None
        self.merged = 0                 # requests that ran inside an older request's batch
        self.light_yield = light_yield
        self.light_shared = 0           # light steps decided while a heavy request was in service
        if heavy_plain:
            need = sum(fp(dg, plain_batch) for dg, h in zip(self.dgraphs, self.heavy) if h)
            if need > self.mem.budget:
                raise _m.MfbcError(_m.MFBC_ENOMEM, f"plain workspaces need {need} bytes, "
                                                   f"budget {budget}")
            for gi, h in enumerate(self.heavy):
                if h:
                    self.mem.add(gi, plain_batch)
        if self.fixed:
            need = sum(fp(dg, w) for dg, w in zip(self.dgraphs, widths))
            if need > self.mem.budget:
                raise _m.MfbcError(_m.MFBC_ENOMEM, f"servers need {need} bytes, budget {budget}")
            for gi, w in enumerate(widths):
                self._open(gi, w)

    def _open(self, gi: int, width: int):
        self.servers[gi] = self.factory(self.dgraphs[gi], width)
        self.mem.add(gi, width)

    def _close(self, gi: int):
        if self.servers[gi] is not None:
            self.servers[gi].close()
            self.servers[gi] = None
        self.mem.remove(gi)

    def close(self):
        for gi in range(len(self.servers)):
            self._close(gi)

    def _alloc(self, r: Request):
        t = self.torch
        dg = self.dgraphs[r.graph]
        if r.kind == "bc":
            r.out = t.zeros(dg.n, dtype=t.float64, device=self.device)
        else:
            r.out = t.zeros((r.sources.size, r.targets.size), dtype=t.float64, device=self.device)
            r._targets = t.as_tensor(np.ascontiguousarray(r.targets, dtype=np.int32),
                                     device=self.device)

    def _idle(self, gi: int) -> bool:
        s = self.servers[gi]
        return (s is not None and not getattr(s, "busy", False) and not s.launched
                and s.owned == 0 and s.active_columns() == 0)

    def run(self, requests: List[Request], realtime: bool = True, on_step=None):
        """Serve `requests` (arrival times in seconds); returns them with `done` set.

        The calling thread releases requests at their arrival times; one worker
        thread per graph drives that graph's server: it admits queued sources
        into free columns, launches a step, waits for it (the library call
        releases the interpreter lock, so graphs progress in parallel) and
        harvests the columns that finished -- a small graph never waits for a
        step of a large one.  A graph without a server gets one when the
        memory budget allows (see MemoryBudget); a request whose graph cannot
        fit a server within the whole budget completes at once with ``error``
        set and no result.  Heavy graphs take turns (see __init__).
        ``on_step(engine)`` is called after every step, under the engine's lock.
        """
        t = self.torch
        pending = sorted(requests, key=lambda r: r.arrival)
        G = len(self.dgraphs)
        self._queues = [deque() for _ in range(G)]
        self._owner = [dict() for _ in range(G)]      # column -> request, per graph
        self._active = [dict() for _ in range(G)]     # id -> request with columns in flight
        self._oldest = [float("inf")] * G             # arrival of the oldest request held
        self._left = len(pending)
        self._stop = False
        self._err = None
        self._token = None                            # heavy graph allowed to step
        cv = threading.Condition()
        self._cv = cv
        if self.device == "cuda":
            t.cuda.synchronize()
        t0 = time.perf_counter()
        self._t0 = t0
        workers = [threading.Thread(target=self._plain_worker if (self.heavy_plain and self.heavy[gi])
                                    else self._worker, args=(gi, on_step), daemon=True)
                   for gi in range(G)]
        for w in workers:
            w.start()
        try:
            for r in pending:
                if realtime:
                    wait = r.arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(wait)
                if r.sources.size and not self.fixed and not self.mem.fits_ever(r.graph):
                    with cv:
                        r.error = (f"ENOMEM: a 64-column server of graph {r.graph} needs "
                                   f"{self.mem.footprint(r.graph, 64)} bytes, the budget is "
                                   f"{self.mem.budget}")
                        r.done = time.perf_counter() - t0
                        self.rejected += 1
                        self._left -= 1
                        cv.notify_all()
                    continue
                self._alloc(r)
                with cv:
                    if r.sources.size == 0:          # nothing to compute: the zero result
                        r.done = time.perf_counter() - t0
                        self._left -= 1
                    else:
                        self._queues[r.graph].append(r)
                        self._oldest[r.graph] = min(self._oldest[r.graph], r.arrival)
                    cv.notify_all()
            with cv:
                while self._left > 0 and self._err is None:
                    cv.wait(timeout=0.5)
        finally:
            with cv:
                self._stop = True
                cv.notify_all()
            for w in workers:
                w.join()
        if self._err is not None:
            raise self._err
        return requests

    def _may_step(self, gi: int) -> bool:
        """Heavy graphs: only the one holding the oldest request steps, one at a
        time.  Light graphs: always, or (light_yield) while no heavy request is
        in service."""
        if not self.heavy[gi]:
            if self.light_yield is None or self._token is None:
                return True
            return time.perf_counter() - self._t0 - self._oldest[gi] >= self.light_yield
        if self._token is not None and self._token != gi:
            return False
        mine = self._oldest[gi]
        return all(not self.heavy[h] or h == gi or self._oldest[h] >= mine
                   for h in range(len(self.dgraphs)))

    def _may_admit(self, gi: int, r) -> bool:
        """Light graphs: `r` waits while a heavy request older than
        r.arrival - light_lag is unfinished (see __init__)."""
        if self.heavy[gi] or self.light_lag is None:
            return True
        oldest_heavy = min((self._oldest[h] for h in range(len(self.dgraphs)) if self.heavy[h]),
                           default=float("inf"))
        return r.arrival <= oldest_heavy + self.light_lag

    def _refresh_oldest(self, gi: int):
        ages = [r.arrival for r in self._queues[gi]] + [r.arrival for r in self._active[gi].values()]
        self._oldest[gi] = min(ages) if ages else float("inf")

    def _worker(self, gi: int, on_step):
        cv = self._cv
        q = self._queues[gi]
        try:
            while True:
                admits = []
                with cv:
                    while True:
                        if self._stop:
                            return
                        srv = self.servers[gi]
                        active = srv is not None and srv.active_columns() > 0
                        ready = bool(q) and self._may_admit(gi, q[0])
                        if (ready or active) and self._may_step(gi):
                            if srv is None:
                                srv = self._acquire(gi)
                            if srv is not None:
                                break
                        cv.wait(timeout=0.05)
                    srv.busy = True
                    if self.heavy[gi]:
                        self._token = gi
                    elif self._token is not None:
                        self.light_shared += 1     # a light step alongside a heavy request
                    # queued sources fill the free columns (their requests in arrival order)
                    free = srv.free_columns()
                    while q and free and self._may_admit(gi, q[0]):
                        r = q[0]
                        k = min(free, r.sources.size - r.placed)
                        admits.append((r, r.placed, k))
                        if r.placed == 0:
                            r.started = time.perf_counter() - self._t0
                        r.placed += k
                        free -= k
                        self._active[gi][id(r)] = r
                        if r.placed == r.sources.size:
                            q.popleft()
                for r, p0, k in admits:
                    cols = srv.admit(r.sources[p0:p0 + k])
                    for j, c in enumerate(cols):
                        self._owner[gi][int(c)] = r
                        r.cols[int(c)] = p0 + j
                    srv.owned += k
                finished = 0
                if srv.active_columns() > 0:
                    srv.step_launch()
                    done = srv.step_finish()
                    if done.size:
                        finished = self._harvest(srv, gi, done, self._owner, self._t0)
                with cv:
                    srv.busy = False
                    self.steps += 1
                    self.mem.touch(gi)
                    if self._token == gi:
                        self._token = None
                    self._left -= finished
                    self._refresh_oldest(gi)
                    if on_step is not None:
                        on_step(self)
                    cv.notify_all()
        except BaseException as e:             # surfaced by run()
            with cv:
                self._err = e
                self._stop = True
                cv.notify_all()

    def _plain_worker(self, gi: int, on_step):
        """Heavy graph under heavy_plain: whole requests, oldest first among the
        heavy graphs, one at a time, on this thread's own stream."""
        cv = self._cv
        q = self._queues[gi]
        t = self.torch
        stream = t.cuda.Stream() if self.device == "cuda" else None
        try:
            while True:
                with cv:
                    while True:
                        if self._stop:
                            return
                        if q and self._may_step(gi):
                            break
                        cv.wait(timeout=0.05)
                    self._token = gi
                    run = [q.popleft()]
                    if self.plain_merge and run[0].kind == "bc":
                        run += self._bc_mates(q, run[0])
                        self.merged += len(run) - 1
                    now = time.perf_counter() - self._t0
                    for r in run:
                        r.placed = r.sources.size
                        r.started = now
                        self._active[gi][id(r)] = r
                self._run_plain(gi, run, stream)
                with cv:
                    now = time.perf_counter() - self._t0
                    for r in run:
                        r.done = now
                        del self._active[gi][id(r)]
                    self.steps += 1
                    if self._token == gi:
                        self._token = None
                    self._left -= len(run)
                    self._refresh_oldest(gi)
                    if on_step is not None:
                        on_step(self)
                    cv.notify_all()
        except BaseException as e:             # surfaced by run()
            with cv:
                self._err = e
                self._stop = True
                cv.notify_all()

    def _bc_mates(self, q, head) -> list:
        """Queued BC requests (arrival order, under the lock) whose column
        groups fit the free groups of the last batch of `head`; removed from q."""
        per = max(1, self.plain_batch // 64)
        used = -(-head.sources.size // 64)
        free = (-used) % per if used else 0
        mates = []
        for r in list(q):
            if free == 0:
                break
            k = -(-r.sources.size // 64)
            if r.kind == "bc" and 0 < k <= free:
                mates.append(r)
                free -= k
        if mates:
            taken = {id(r) for r in mates}
            keep = [r for r in q if id(r) not in taken]
            q.clear()
            q.extend(keep)
        return mates

    def _run_plain(self, gi: int, run: list, stream):
        def go():
            if len(run) > 1:
                self.plain_many_fn(self.dgraphs[gi], run, self.plain_batch)
            else:
                self.plain_fn(self.dgraphs[gi], run[0], self.plain_batch)
        if stream is not None:
            with self.torch.cuda.stream(stream):
                go()
            stream.synchronize()
        else:
            go()

    def _acquire(self, gi: int):
        """A server for graph gi within the memory budget (under the lock), or None."""
        q = self._queues[gi]
        want = sum(r.sources.size - r.placed for r in q)
        head = q[0].arrival if q else float("inf")

        def evictable(h):
            # an idle server may go if its graph has nothing waiting that
            # arrived before this graph's oldest request
            hq = self._queues[h]
            return self._idle(h) and (not hq or hq[0].arrival > head)

        width, evict = self.mem.acquire(gi, want, evictable)
        if width is None:
            return None
        for h in evict:
            self._close(h)
        self._open(gi, width)
        return self.servers[gi]

    def _harvest(self, srv, gi, done, owner, t0) -> int:
        """Harvest finished columns; returns the number of requests completed."""
        by_req = {}
        for c in done:
            r = owner[gi].pop(int(c))
            by_req.setdefault(id(r), (r, []))[1].append(int(c))
        srv.owned -= len(done)
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
                self._active[gi].pop(id(r), None)
                finished += 1
        return finished


def run_plain(dg, r: Request, batch: int = 256):
    """One request through the plain per-batch entry points on the current
    stream: mfbc_bc for a BC sum, mfbc_forward + mfbc_backward per batch and
    a gather of delta at the targets for a dependency request."""
    import torch
    src = torch.as_tensor(np.ascontiguousarray(r.sources, dtype=np.int32), device="cuda")
    if r.kind == "bc":
        r.out = dg.bc(src, batch)
        return
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


def run_plain_many(dg, reqs: List[Request], batch: int = 256):
    """BC requests of one graph in one mfbc_bc_requests call on the current
    stream: each request's sources in whole column groups, the requests
    sharing batches."""
    outs = dg.bc_requests([r.sources for r in reqs], batch)
    for r, o in zip(reqs, outs):
        r.out = o


def run_fifo(dgraphs, requests: List[Request], batch: int = 256, realtime: bool = True):
    """Reference schedule: each request alone, in arrival order, through the
    plain per-batch entry points (run_plain)."""
    import torch
    pending = sorted(requests, key=lambda r: r.arrival)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in pending:
        if realtime:
            wait = r.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        r.started = time.perf_counter() - t0
        run_plain(dgraphs[r.graph], r, batch)
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
