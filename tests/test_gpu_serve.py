"""Served form: continuous batching of source columns over resident graphs.

Every request's result is checked against the CPU oracle, and the same
request served alone against it served in a mix with others (the bar of the
served form: equal within the stated tolerance)."""
import numpy as np
import pytest

import oracle
from paper_1609_07008_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_07008_amd import mfbc, serve
    mfbc.load_library()
    graphs = [gg.rmat_graph(10, 8, 21, wrange=(1, 255)), gg.er_graph(700, 6, 22, (1, 50)),
              gg.rmat_graph(9, 16, 23)]
    dgs = [mfbc.DeviceGraph(g) for g in graphs]
    yield t, mfbc, serve, graphs, dgs
    for d in dgs:
        d.close()


def rel_close(got, want, tol, what=""):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    zero = want == 0
    assert np.count_nonzero(got[zero]) == 0, f"{what}: zeros must be exact"
    if (~zero).any():
        err = np.abs(got[~zero] - want[~zero]) / np.abs(want[~zero])
        assert err.max() <= tol, f"{what}: max rel err {err.max():.3e}"


def reference(graphs, r):
    g = graphs[r.graph]
    if r.kind == "bc":
        return oracle.brandes(g, r.sources, per_source=False)["lambda"]
    d = oracle.brandes(g, r.sources)["delta"]
    return d[:, r.targets]


def test_served_results_match_oracle_and_alone(env):
    t, mfbc, serve, graphs, dgs = env
    reqs = serve.make_requests(graphs, 24, rate=1e9, seed=5, smin=3, smax=150)
    eng = serve.ServeEngine(dgs, [128, 64, 192])
    eng.run(reqs, realtime=False)
    for r in reqs:
        assert r.done >= 0
        rel_close(r.out.cpu().numpy(), reference(graphs, r), 1e-10, f"request {r.rid} ({r.kind})")
    # each request alone gives the same result as in the mix
    for r in reqs[:8]:
        alone = serve.Request(r.rid, r.graph, r.kind, r.sources, r.targets, 0.0)
        eng.run([alone], realtime=False)
        rel_close(alone.out.cpu().numpy(), r.out.cpu().numpy(), 1e-12, f"alone vs mix {r.rid}")
    eng.close()


def test_served_requests_wider_than_the_server(env):
    """A request with more sources than columns is admitted piece by piece."""
    t, mfbc, serve, graphs, dgs = env
    g = graphs[0]
    src = gg.pick_sources(g, 300, 8)
    r = serve.Request(0, 0, "bc", src, None, 0.0)
    eng = serve.ServeEngine(dgs[:1], [64])
    eng.run([r], realtime=False)
    rel_close(r.out.cpu().numpy(), oracle.brandes(g, src, per_source=False)["lambda"], 1e-10)
    eng.close()


def test_served_distances_past_16_bits(env):
    """Shortest-path distances beyond 16 bits (a heavy path, up to 76,245):
    the counting product reads the full tau; results against the oracle."""
    t, mfbc, serve, graphs, dgs = env
    g = gg.path_graph(300, w=255)
    dg = mfbc.DeviceGraph(g)
    src = np.arange(0, 300, 3, dtype=np.int32)          # 100 sources: one pair of groups
    r = serve.Request(0, 0, "bc", src, None, 0.0)
    eng = serve.ServeEngine([dg], [128])
    eng.run([r], realtime=False)
    rel_close(r.out.cpu().numpy(), oracle.brandes(g, src, per_source=False)["lambda"], 1e-10)
    eng.close()
    dg.close()


def test_fifo_reference_schedule(env):
    t, mfbc, serve, graphs, dgs = env
    reqs = serve.make_requests(graphs, 6, rate=1e9, seed=9, smin=4, smax=40)
    serve.run_fifo(dgs, reqs, batch=64, realtime=False)
    for r in reqs:
        rel_close(r.out.cpu().numpy(), reference(graphs, r), 1e-10, f"fifo {r.rid}")


def test_server_rejects_misuse(env):
    t, mfbc, serve, graphs, dgs = env
    s = serve.ColumnServer(dgs[1], 64)
    with pytest.raises(mfbc.MfbcError):
        s.admit(np.arange(65, dtype=np.int32))            # more sources than columns
    with pytest.raises(mfbc.MfbcError):
        s.admit(np.array([graphs[1].n], dtype=np.int32))  # out of range
    with pytest.raises(mfbc.MfbcError):
        s.step_finish()                                   # nothing in flight
    s.close()


def test_cohort_admission(env):
    """Sources join a pair of 64-column groups only until its first step is
    launched; a running pair takes none, a free pair next to it does, and
    both give the oracle's results."""
    t, mfbc, serve, graphs, dgs = env
    g = graphs[1]
    s = serve.ColumnServer(dgs[1], 256)
    a_src = gg.pick_sources(g, 10, 31)
    b_src = gg.pick_sources(g, 64, 32)
    assert s.free_columns() == 256
    ca = s.admit(a_src[:4])
    ca = np.concatenate([ca, s.admit(a_src[4:])])          # same pair, before the launch
    assert np.all(ca // 128 == ca[0] // 128)
    assert s.free_columns() == 256 - 10
    s.step_launch()
    done = list(s.step_finish())
    assert s.free_columns() == 128                          # the running pair is closed
    with pytest.raises(mfbc.MfbcError):
        s.admit(b_src[:1].repeat(129))
    cb = s.admit(b_src)                                     # the other pair, mid-loop of the first
    assert np.all(cb // 128 != ca[0] // 128)
    out_a = t.zeros(g.n, dtype=t.float64, device="cuda")
    out_b = t.zeros(g.n, dtype=t.float64, device="cuda")
    owner = {int(c): out_a for c in ca}
    owner.update({int(c): out_b for c in cb})
    left = set(owner)
    for _ in range(10 * g.n):
        fin = [c for c in done if c in left]
        if fin:
            s.harvest_bc(fin, [owner[c] for c in fin])
            left -= set(fin)
        if not left:
            break
        s.step_launch()
        done = list(s.step_finish())
    assert not left
    t.cuda.synchronize()
    rel_close(out_a.cpu().numpy(), oracle.brandes(g, a_src, per_source=False)["lambda"], 1e-10, "a")
    rel_close(out_b.cpu().numpy(), oracle.brandes(g, b_src, per_source=False)["lambda"], 1e-10, "b")
    assert s.free_columns() == 256
    s.close()


def test_server_reports_path_count_overflow(env):
    t, mfbc, serve, graphs, dgs = env
    g = gg.diamond_chain(1100)
    dg = mfbc.DeviceGraph(g)
    s = serve.ColumnServer(dg, 64)
    s.admit(np.array([0], dtype=np.int32))
    with pytest.raises(mfbc.MfbcError) as e:
        for _ in range(3 * 1100 + 10):
            s.step_launch()
            s.step_finish()
    assert e.value.code == mfbc.MFBC_EOVERFLOW
    s.close()
    dg.close()


def test_empty_requests_complete(env):
    t, mfbc, serve, graphs, dgs = env
    reqs = [serve.Request(0, 0, "bc", np.zeros(0, dtype=np.int32), None, 0.0),
            serve.Request(1, 1, "dep", np.zeros(0, dtype=np.int32), np.array([1, 2], dtype=np.int32), 0.0),
            serve.Request(2, 1, "bc", gg.pick_sources(graphs[1], 5, 3), None, 0.0)]
    eng = serve.ServeEngine(dgs[:2], [64, 64])
    eng.run(reqs, realtime=False)
    assert all(r.done >= 0 for r in reqs)
    assert float(reqs[0].out.abs().sum()) == 0.0 and tuple(reqs[1].out.shape) == (0, 2)
    rel_close(reqs[2].out.cpu().numpy(),
              oracle.brandes(graphs[1], reqs[2].sources, per_source=False)["lambda"], 1e-10)
    eng.close()


def test_set_plan_refused_while_a_server_is_attached(env):
    t, mfbc, serve, graphs, dgs = env
    g = gg.er_graph(200, 5, 41, (1, 9))
    dg = mfbc.DeviceGraph(g)
    s = serve.ColumnServer(dg, 64)
    with pytest.raises(mfbc.MfbcError) as e:
        dg.set_plan(heavy=4, slice=2)                 # would need more hub slots than s holds
    assert e.value.code == mfbc.MFBC_EINVAL
    s.close()
    dg.set_plan(heavy=4, slice=2)                     # fine once the server is gone
    dg.close()


def test_free_graph_refused_while_a_server_is_attached(env):
    t, mfbc, serve, graphs, dgs = env
    g = gg.er_graph(200, 5, 42, (1, 9))
    dg = mfbc.DeviceGraph(g)
    s = serve.ColumnServer(dg, 64)
    with pytest.raises(mfbc.MfbcError) as e:
        dg.close()                                    # the server still uses the graph
    assert e.value.code == mfbc.MFBC_EINVAL and dg.handle
    src = gg.pick_sources(g, 3, 5)                    # the server still runs to the oracle's result
    cols = s.admit(src)
    out = t.zeros(g.n, dtype=t.float64, device="cuda")
    left = set(int(c) for c in cols)
    for _ in range(10 * g.n):
        s.step_launch()
        fin = [c for c in s.step_finish() if c in left]
        if fin:
            s.harvest_bc(fin, [out] * len(fin))
            left -= set(fin)
        if not left:
            break
    assert not left
    t.cuda.synchronize()
    rel_close(out.cpu().numpy(), oracle.brandes(g, src, per_source=False)["lambda"], 1e-10)
    s.close()
    dg.close()                                        # freed once the server is gone
    assert dg.handle is None


def test_served_hub_rows_alone_and_in_the_mix(env):
    """Rows cut into slices (a star and plans with tiny hub thresholds) run
    the served form's hub merges; every request against the oracle, and
    alone == in the mix."""
    t, mfbc, serve, graphs, dgs = env
    gs = [gg.star_graph(3000), gg.rmat_graph(10, 8, 21, wrange=(1, 255))]
    ds = [mfbc.DeviceGraph(g) for g in gs]
    ds[1].set_plan(run_arcs=64, run_verts=8, heavy=16, slice=8)
    reqs = serve.make_requests(gs, 16, rate=1e9, seed=17, smin=3, smax=130)
    eng = serve.ServeEngine(ds, [128, 192])
    eng.run(reqs, realtime=False)
    for r in reqs:
        rel_close(r.out.cpu().numpy(), reference(gs, r), 1e-10, f"request {r.rid} ({r.kind})")
    for r in reqs[:6]:
        alone = serve.Request(r.rid, r.graph, r.kind, r.sources, r.targets, 0.0)
        eng.run([alone], realtime=False)
        rel_close(alone.out.cpu().numpy(), r.out.cpu().numpy(), 1e-12, f"alone vs mix {r.rid}")
    eng.close()
    for d in ds:
        d.close()


def test_served_admission_by_memory_budget(env):
    """A budget that holds about one server at a time: requests on three
    graphs wait for memory, servers are released and created as they go, the
    live footprint never exceeds the budget, every result matches the oracle;
    a graph whose smallest server exceeds the budget is rejected (ENOMEM)."""
    t, mfbc, serve, graphs, dgs = env
    fps = [serve.footprint(d, 64) for d in dgs]
    big = gg.rmat_graph(14, 16, 44, wrange=(1, 255))
    dbig = mfbc.DeviceGraph(big)
    budget = max(fps) + min(fps) // 2
    assert serve.footprint(dbig, 64) > budget
    allg = graphs + [big]
    reqs = serve.make_requests(graphs, 18, rate=1e9, seed=23, smin=3, smax=100)
    reqs.append(serve.Request(99, 3, "bc", gg.pick_sources(big, 10, 1), None, 0.0))
    peak = []
    eng = serve.ServeEngine(dgs + [dbig], budget_bytes=budget, max_width=128)
    eng.run(reqs, realtime=False, on_step=lambda e: peak.append(e.mem.used))
    assert max(peak) <= budget and eng.mem.peak <= budget
    for r in reqs:
        if r.graph == 3:
            assert r.error and r.error.startswith("ENOMEM")
            continue
        assert r.error is None
        rel_close(r.out.cpu().numpy(), reference(allg, r), 1e-10, f"request {r.rid} ({r.kind})")
    assert eng.rejected == 1
    eng.close()
    dbig.close()


def test_served_at_workload_sizes(env):
    """Resident weighted R-MAT graphs of the served workload's scales 14..17
    (edge factor 16, weights 1..255; their hub rows are split) plus the
    scale-20 graph with small requests, servers of 256 columns: every request
    against the oracle, and a few alone == in the mix."""
    import time
    t, mfbc, serve, graphs, dgs = env
    scales = (14, 15, 16, 17, 20)
    gs = [gg.rmat_graph(sc, 16, 2000 + i, wrange=(1, 255)) for i, sc in enumerate(scales[:-1])]
    gs.append(gg.rmat_graph(20, 16, 2006, wrange=(1, 255)))
    ds = [mfbc.DeviceGraph(g) for g in gs]
    reqs = serve.make_requests(gs[:-1], 20, rate=1e9, seed=2101, smin=16, smax=300)
    for i, k in enumerate((16, 40)):
        reqs.append(serve.Request(100 + i, 4, "bc" if i == 0 else "dep",
                                  gg.pick_sources(gs[4], k, 7 + i),
                                  None if i == 0 else np.arange(0, 64, dtype=np.int32) * 997, 0.0))
    t0 = time.perf_counter()
    eng = serve.ServeEngine(ds, [256] * len(ds))
    eng.run(reqs, realtime=False)
    print(f"[serve] {len(reqs)} requests served in {time.perf_counter() - t0:.1f}s", flush=True)
    for r in reqs:
        rel_close(r.out.cpu().numpy(), reference(gs, r), 1e-10, f"request {r.rid} ({r.kind})")
    for r in reqs[:3] + reqs[-1:]:
        alone = serve.Request(r.rid, r.graph, r.kind, r.sources, r.targets, 0.0)
        eng.run([alone], realtime=False)
        rel_close(alone.out.cpu().numpy(), r.out.cpu().numpy(), 1e-12, f"alone vs mix {r.rid}")
    eng.close()
    for d in ds:
        d.close()


@pytest.mark.parametrize("rounds", [1, 3, 8])
def test_rounds_per_step_do_not_change_results(env, rounds):
    """A step runs 1..8 rounds of products (later rounds skip on the device
    once a loop has ended); every request against the oracle."""
    t, mfbc, serve, graphs, dgs = env
    reqs = serve.make_requests(graphs, 14, rate=1e9, seed=31 + rounds, smin=2, smax=140)
    eng = serve.ServeEngine(dgs, [128, 64, 192],
                            server_factory=lambda dg, w: serve.ColumnServer(dg, w, rounds=rounds))
    eng.run(reqs, realtime=False)
    for r in reqs:
        rel_close(r.out.cpu().numpy(), reference(graphs, r), 1e-10, f"rounds={rounds} request {r.rid}")
    eng.close()


def test_heavy_graphs_through_the_plain_path(env):
    """heavy_plain: the graphs above the heavy threshold run whole requests
    through the plain path on their own streams while the others are served
    by column servers; every request against the oracle, the heavy ones
    also against run_fifo's result."""
    t, mfbc, serve, graphs, dgs = env
    heavy_arcs = dgs[1].arcs                                # graphs 0 and 2 heavy, 1 light
    reqs = serve.make_requests(graphs, 30, rate=1e9, seed=12, smin=3, smax=300)
    eng = serve.ServeEngine(dgs, budget_bytes=4 << 30, max_width=128, heavy_arcs=heavy_arcs,
                            heavy_plain=True)
    assert eng.heavy == [True, False, True]
    eng.run(reqs, realtime=False)
    print(f"[serve] heavy_plain: {eng.merged} requests merged into older ones' batches", flush=True)
    assert eng.merged > 0                    # queued BC requests shared batches (mfbc_bc_requests)
    for r in reqs:
        rel_close(r.out.cpu().numpy(), reference(graphs, r), 1e-10, f"request {r.rid} ({r.kind})")
    fifo = [serve.Request(r.rid, r.graph, r.kind, r.sources, r.targets, 0.0) for r in reqs
            if eng.heavy[r.graph]][:6]
    serve.run_fifo(dgs, fifo, realtime=False)
    for f in fifo:
        r = next(x for x in reqs if x.rid == f.rid)
        rel_close(r.out.cpu().numpy(), f.out.cpu().numpy(), 1e-12, f"plain vs fifo {r.rid}")
    eng.close()
