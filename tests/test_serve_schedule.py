"""Served-form scheduling on the CPU (no GPU): admission of column servers by
memory footprint (MemoryBudget) and the request loop of ServeEngine driven
by a fake executor whose columns finish after a known number of steps.

Checked: the live servers' footprints never exceed the budget; widths shrink
to what fits; idle servers are released oldest first, busy ones never;
requests wait while memory is taken and complete once it frees up; requests
whose graph cannot fit 64 columns in the whole budget are rejected; every
request's result is assembled from exactly its own columns."""
import threading
import time
from dataclasses import dataclass

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1609_07008_amd.serve import MemoryBudget, Request, ServeEngine  # noqa: E402


def fp_linear(base, per_col):
    return lambda g, w: base[g] + per_col[g] * w


def test_widest_width_that_fits():
    mem = MemoryBudget(1000, fp_linear([100, 100], [2, 2]), max_width=256)
    assert mem.acquire(0, 1000, lambda h: False) == (256, [])     # 100 + 512 fits
    mem.add(0, 256)
    assert mem.used == 612
    # 388 left: 192 columns take 484, 128 take 356
    assert mem.acquire(1, 300, lambda h: False) == (128, [])
    assert mem.acquire(1, 10, lambda h: False) == (64, [])        # as wide as needed only


def test_waits_while_busy_and_releases_idle_oldest_first():
    fp = fp_linear([0, 0, 0], [1, 1, 1])
    mem = MemoryBudget(256, fp, max_width=128)
    mem.add(0, 128)
    mem.add(1, 128)
    assert mem.acquire(2, 64, lambda h: False) == (None, [])      # everything busy: wait
    mem.touch(0)                                                  # graph 1 is now the oldest
    width, evict = mem.acquire(2, 64, lambda h: True)
    assert (width, evict) == (64, [1])
    width, evict = mem.acquire(2, 256, lambda h: True)            # needs both released
    assert width == 128 and evict == [1]
    width, evict = mem.acquire(2, 256, lambda h: h == 0)          # only graph 0 is idle
    assert width == 128 and evict == [0]


def test_graph_that_never_fits():
    mem = MemoryBudget(100, fp_linear([50, 10], [1, 1]))
    assert not mem.fits_ever(0)                                   # 50 + 64 > 100
    assert mem.fits_ever(1)


@dataclass
class FakeGraph:
    n: int


class FakeServer:
    """Columns finish `steps_for(source)` steps after admission; harvest
    adds one to dest[v] for v = source (bc) or writes 1 at target 0 (dep)."""

    live = []

    def __init__(self, dg, width):
        self.dg, self.width = dg, width
        self.rem = np.full(width, -1)
        self.src = np.full(width, -1)
        self.launched = False
        self.owned = 0
        self.ready_after = 0
        self.log = FakeServer.live
        self.log.append(self)
        self.closed = False

    @staticmethod
    def steps_for(s):
        return 2 + int(s) % 5

    def free_columns(self):
        return int((self.rem < 0).sum())

    def active_columns(self):
        return int((self.rem > 0).sum())

    def admit(self, sources):
        free = np.flatnonzero(self.rem < 0)[:len(sources)]
        assert free.size == len(sources)
        self.rem[free] = [self.steps_for(s) for s in sources]
        self.src[free] = sources
        return free.astype(np.int32)

    heavy_flying = 0               # heavy servers between step_launch and step_finish
    max_heavy_flying = 0
    light_during_heavy = 0         # light steps run while a heavy step was in flight
    lock = threading.Lock()

    def step_launch(self):
        assert not self.launched
        self.launched = True
        with FakeServer.lock:
            if getattr(self.dg, "arcs", 0) > 1000:
                FakeServer.heavy_flying += 1
                FakeServer.max_heavy_flying = max(FakeServer.max_heavy_flying,
                                                  FakeServer.heavy_flying)
            elif FakeServer.heavy_flying:
                FakeServer.light_during_heavy += 1

    def ready(self):
        return True

    def step_finish(self):
        time.sleep(0.001)              # a step takes a little while
        with FakeServer.lock:
            if getattr(self.dg, "arcs", 0) > 1000:
                FakeServer.heavy_flying -= 1
        self.launched = False
        act = self.rem > 0
        self.rem[act] -= 1
        done = np.flatnonzero(act & (self.rem == 0))
        return done.astype(np.int32)

    def harvest_bc(self, cols, dests):
        for c, d in zip(cols, dests):
            d[int(self.src[c])] += 1.0
            self.rem[c] = -1

    def harvest_dep(self, cols, targets, outs):
        for c, o in zip(cols, outs):
            o[0] = float(self.src[c])
            self.rem[c] = -1

    def close(self):
        self.closed = True


def test_engine_respects_budget_and_completes_every_request():
    """The budget holds one server at a time (any two exceed it), so every
    switch between graphs releases an idle server first."""
    FakeServer.live.clear()
    graphs = [FakeGraph(50), FakeGraph(60), FakeGraph(40), FakeGraph(70)]
    per_col = [1, 2, 3, 100]                         # graph 3 never fits
    fp = lambda dg, w: 200 + per_col[graphs.index(dg)] * w   # noqa: E731
    budget = 400
    peak = []
    eng = ServeEngine(graphs, budget_bytes=budget, max_width=256, server_factory=FakeServer,
                      footprint_fn=fp, device="cpu")
    rng = np.random.default_rng(1)
    reqs = []
    for i in range(60):
        gi = int(rng.integers(0, 4))
        k = int(rng.integers(1, 150))
        src = rng.integers(0, graphs[gi].n, size=k).astype(np.int32)
        kind = "bc" if i % 3 else "dep"
        tg = np.array([0, 1], dtype=np.int32) if kind == "dep" else None
        reqs.append(Request(i, gi, kind, src, tg, 0.0))
    eng.run(reqs, realtime=False, on_step=lambda e: peak.append(e.mem.used))
    assert max(peak) <= budget and eng.mem.peak <= budget
    for r in reqs:
        assert r.done >= 0
        if r.graph == 3:
            assert r.error and r.error.startswith("ENOMEM") and r.out is None
            continue
        assert r.error is None
        if r.kind == "bc":
            want = np.bincount(r.sources, minlength=graphs[r.graph].n).astype(float)
            assert np.array_equal(r.out.numpy(), want), r.rid
        else:
            assert np.array_equal(r.out[:, 0].numpy(), r.sources.astype(float)), r.rid
    assert eng.rejected == sum(r.graph == 3 for r in reqs)
    # three graphs were served through one server slot: servers were released
    assert sum(s.closed for s in FakeServer.live) >= 2
    eng.close()


def test_fixed_widths_must_fit_the_budget():
    graphs = [FakeGraph(10), FakeGraph(10)]
    from paper_1609_07008_amd import mfbc
    with pytest.raises(mfbc.MfbcError) as e:
        ServeEngine(graphs, widths=[64, 64], budget_bytes=100, server_factory=FakeServer,
                    footprint_fn=lambda dg, w: w, device="cpu")
    assert e.value.code == mfbc.MFBC_ENOMEM
    eng = ServeEngine(graphs, widths=[64, 64], budget_bytes=128, server_factory=FakeServer,
                      footprint_fn=lambda dg, w: w, device="cpu")
    eng.close()


@dataclass
class FakeSized:
    n: int
    arcs: int


def test_heavy_graphs_advance_one_at_a_time_oldest_first():
    """At most one heavy graph's server has a step in flight; light graphs
    run alongside; the heavy graph holding the oldest request goes first and
    every request completes with its own result."""
    FakeServer.live.clear()
    graphs = [FakeSized(40, 100), FakeSized(50, 10_000), FakeSized(60, 20_000), FakeSized(30, 50)]
    eng = ServeEngine(graphs, budget_bytes=10**9, max_width=128, server_factory=FakeServer,
                      footprint_fn=lambda dg, w: w, device="cpu", heavy_arcs=1000, max_heavy=1)
    assert eng.heavy == [False, True, True, False]
    FakeServer.heavy_flying = FakeServer.max_heavy_flying = FakeServer.light_during_heavy = 0
    rng = np.random.default_rng(4)
    reqs = []
    for i in range(40):
        gi = int(rng.integers(0, 4))
        src = rng.integers(0, graphs[gi].n, size=int(rng.integers(1, 90))).astype(np.int32)
        reqs.append(Request(i, gi, "bc", src, None, 0.0))
    eng.run(reqs, realtime=False)
    assert FakeServer.max_heavy_flying == 1
    assert FakeServer.light_during_heavy > 0                  # light work overlaps heavy work
    for r in reqs:
        want = np.bincount(r.sources, minlength=graphs[r.graph].n).astype(float)
        assert np.array_equal(r.out.numpy(), want), r.rid
    eng.close()


class TickServer(FakeServer):
    """FakeServer that stamps admissions and harvests with a global counter."""

    tick = 0
    first_admit = {}
    last_harvest = {}
    tick_lock = threading.Lock()

    def admit(self, sources):
        cols = super().admit(sources)
        with TickServer.tick_lock:
            TickServer.tick += 1
            for c in cols:
                TickServer.first_admit.setdefault(self.req_of(int(c)), TickServer.tick)
        return cols

    def req_of(self, c):
        return (id(self.dg), int(self.src[c]))

    def harvest_bc(self, cols, dests):
        with TickServer.tick_lock:
            TickServer.tick += 1
            for c in cols:
                TickServer.last_harvest[self.req_of(int(c))] = TickServer.tick
        super().harvest_bc(cols, dests)


def test_light_requests_wait_behind_older_heavy_ones():
    """With light_lag = 0 a light graph's request is first admitted only after
    every heavy request that arrived before it has finished; without the rule
    light requests overtake (so the check has teeth)."""
    def run(lag):
        FakeServer.live.clear()
        TickServer.tick = 0
        TickServer.first_admit.clear()
        TickServer.last_harvest.clear()
        graphs = [FakeSized(40, 100), FakeSized(50, 10_000), FakeSized(30, 50)]
        eng = ServeEngine(graphs, budget_bytes=10**9, max_width=128, server_factory=TickServer,
                          footprint_fn=lambda dg, w: w, device="cpu", heavy_arcs=1000, light_lag=lag)
        reqs = []
        rng = np.random.default_rng(9)
        for i in range(30):
            gi = [1, 0, 2][i % 3]
            # one source per request, distinct per graph: (graph, source) names the request
            reqs.append(Request(i, gi, "bc", np.array([i], dtype=np.int32), None, float(i)))
        rng.shuffle(reqs)
        eng.run(reqs, realtime=False)
        for r in reqs:
            want = np.bincount(r.sources, minlength=graphs[r.graph].n).astype(float)
            assert np.array_equal(r.out.numpy(), want), r.rid
        key = lambda r: (id(graphs[r.graph]), int(r.sources[0]))    # noqa: E731
        late = 0
        for lt in reqs:
            if eng.heavy[lt.graph]:
                continue
            for h in reqs:
                if eng.heavy[h.graph] and h.arrival < lt.arrival:
                    late += TickServer.first_admit[key(lt)] < TickServer.last_harvest[key(h)]
        eng.close()
        return late
    assert run(0.0) == 0
    assert run(None) > 0


def test_heavy_plain_runs_whole_requests_in_arrival_order():
    """heavy_plain: heavy graphs' requests run whole through the plain
    function, one at a time and in arrival order across the heavy graphs,
    while light graphs' servers keep stepping; the plain workspaces are
    reserved in the budget."""
    FakeServer.live.clear()
    graphs = [FakeSized(40, 100), FakeSized(50, 10_000), FakeSized(60, 20_000), FakeSized(30, 50)]
    state = {"flying": 0, "max": 0, "order": [], "light_steps_during": 0}
    lock = threading.Lock()

    def plain(dg, r, batch):
        with lock:
            state["flying"] += 1
            state["max"] = max(state["max"], state["flying"])
            state["order"].append(r.arrival)
        time.sleep(0.003)
        r.out = torch.as_tensor(np.bincount(r.sources, minlength=dg.n).astype(float))
        with lock:
            state["flying"] -= 1

    class CountingServer(FakeServer):
        def step_launch(self):
            super().step_launch()
            with lock:
                state["light_steps_during"] += state["flying"] > 0

    eng = ServeEngine(graphs, budget_bytes=10_000, max_width=128, server_factory=CountingServer,
                      footprint_fn=lambda dg, w: w, device="cpu", heavy_arcs=1000,
                      heavy_plain=True, plain_batch=256, plain_fn=plain)
    assert eng.mem.used == 2 * 256                     # the two heavy graphs' plain workspaces
    rng = np.random.default_rng(8)
    reqs = []
    for i in range(40):
        gi = int(rng.integers(0, 4))
        src = rng.integers(0, graphs[gi].n, size=int(rng.integers(1, 90))).astype(np.int32)
        reqs.append(Request(i, gi, "bc", src, None, float(i)))
    eng.run(reqs, realtime=False)
    for r in reqs:
        want = np.bincount(r.sources, minlength=graphs[r.graph].n).astype(float)
        assert np.array_equal(r.out.numpy(), want), r.rid
    assert state["max"] == 1
    assert state["order"] == sorted(state["order"])   # heavy requests in arrival order
    assert state["light_steps_during"] > 0            # light servers step alongside
    assert all(s.dg.arcs <= 1000 for s in FakeServer.live)   # no server for a heavy graph
    eng.close()
    with pytest.raises(Exception):
        ServeEngine(graphs, budget_bytes=300, server_factory=CountingServer, footprint_fn=lambda dg, w: w,
                    device="cpu", heavy_arcs=1000, heavy_plain=True, plain_fn=plain)


def test_heavy_bc_requests_merge_into_the_oldest_requests_last_batch():
    """heavy_plain with merging: when the oldest queued request of a heavy
    graph is a BC sum, queued BC requests of the same graph that fit the free
    64-column groups of its last batch run in the same call; dependency
    requests and requests that do not fit are left in arrival order.  Every
    request completes with its own result."""
    FakeServer.live.clear()
    graphs = [FakeSized(40, 100), FakeSized(50, 10_000)]
    calls = []
    lock = threading.Lock()

    def result(dg, r):
        return torch.as_tensor(np.bincount(r.sources, minlength=dg.n).astype(float))

    def plain(dg, r, batch):
        with lock:
            calls.append([r.rid])
        time.sleep(0.002)
        r.out = result(dg, r)

    def plain_many(dg, reqs, batch):
        with lock:
            calls.append([r.rid for r in reqs])
        time.sleep(0.002)
        for r in reqs:
            r.out = result(dg, r)

    eng = ServeEngine(graphs, budget_bytes=10_000, max_width=128, server_factory=FakeServer,
                      footprint_fn=lambda dg, w: w, device="cpu", heavy_arcs=1000,
                      heavy_plain=True, plain_batch=256, plain_fn=plain, plain_many_fn=plain_many)
    rng = np.random.default_rng(3)
    sizes = [100, 30, 20, 70, 10, 200, 64, 5, 130, 1]     # sources; 64 per column group
    kinds = ["bc", "bc", "dep", "bc", "bc", "bc", "bc", "bc", "bc", "bc"]
    reqs = []
    for i, (k, kind) in enumerate(zip(sizes, kinds)):
        src = rng.integers(0, 50, size=k).astype(np.int32)
        tg = np.array([1, 2], dtype=np.int32) if kind == "dep" else None
        reqs.append(Request(i, 1, kind, src, tg, 0.0))
    reqs.append(Request(99, 0, "bc", np.array([1, 2, 3], dtype=np.int32), None, 0.0))
    eng.run(reqs, realtime=False)
    byid = {r.rid: r for r in reqs}
    for r in reqs:
        if r.kind == "bc":
            assert np.array_equal(r.out.numpy(), result(graphs[r.graph], r).numpy()), r.rid
    groups = lambda rid: -(-byid[rid].sources.size // 64)
    seen = [rid for c in calls for rid in c]
    assert sorted(seen) == sorted(r.rid for r in reqs if r.graph == 1)
    merged = [c for c in calls if len(c) > 1]
    assert merged, "queued BC requests were never merged"
    for c in calls:
        head, mates = c[0], c[1:]
        if mates:
            assert byid[head].kind == "bc" and all(byid[m].kind == "bc" for m in mates)
            free = (-groups(head)) % 4
            assert sum(groups(m) for m in mates) <= free
            assert all(m > head for m in mates)        # mates arrived after the head
    heads = [c[0] for c in calls]
    assert heads == sorted(heads)                      # heads in arrival order
    eng.close()


def test_light_graphs_yield_to_heavy_requests():
    """light_yield: while a heavy request runs on the plain path, light
    graphs launch no step unless their oldest request has waited the given
    time; with a long wait no light step is decided while a heavy request
    is in service, and every request still completes with its own result."""
    FakeServer.live.clear()
    graphs = [FakeSized(40, 100), FakeSized(50, 10_000)]

    def plain(dg, r, batch):
        time.sleep(0.01)
        r.out = torch.as_tensor(np.bincount(r.sources, minlength=dg.n).astype(float))

    eng = ServeEngine(graphs, budget_bytes=10_000, max_width=128, server_factory=FakeServer,
                      footprint_fn=lambda dg, w: w, device="cpu", heavy_arcs=1000,
                      heavy_plain=True, plain_batch=256, plain_fn=plain, light_yield=60.0)
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(24):
        gi = i % 2
        src = rng.integers(0, graphs[gi].n, size=int(rng.integers(1, 60))).astype(np.int32)
        reqs.append(Request(i, gi, "bc", src, None, 0.0))
    eng.run(reqs, realtime=False)
    for r in reqs:
        want = np.bincount(r.sources, minlength=graphs[r.graph].n).astype(float)
        assert np.array_equal(r.out.numpy(), want), r.rid
    assert eng.light_shared == 0               # no light step decided during a heavy request
    eng.close()
