"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (same graphs, seeds, source lists, batch sizes and the
work decomposition the benchmark applies from the tuning cache).

  * ER n=1024 (weights 1..100), exact BC over all 1024 sources, batch 64:
    every lambda entry; every column's frontier at every product of one batch.
  * R-MAT scale 16 unweighted, 4096 sources, batch 512: every lambda entry;
    every column of the first batch for tau / sigma / delta / backward
    frontier index; the product counts; sampled columns' frontiers.
  * R-MAT scale 20 (weights 1..255) and ER n=32768 k=512 (weights 1..255),
    1024 sources, batch 256: lambda over all 1024 sources against the oracle;
    tau / sigma / delta of all 256 columns of the first batch, compared in
    chunks of 16 sources; frontier membership at every product for sampled
    columns of that batch.
"""
import time

import numpy as np
import pytest

import oracle
from oracle import frontier
from paper_1609_07008_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def mfbc(torch):
    from paper_1609_07008_amd import mfbc as m
    m.load_library()
    return m


def rel_close(got, want, tol, what=""):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, what
    zero = want == 0
    nbad = int(np.count_nonzero(got[zero] != 0))
    assert nbad == 0, f"{what}: {nbad} entries should be exactly 0"
    if (~zero).any():
        err = np.abs(got[~zero] - want[~zero]) / np.abs(want[~zero])
        assert err.max() <= tol, f"{what}: max rel err {err.max():.3e}"


def host_dist(d, inf):
    d = np.asarray(d).astype(np.int64)
    d[d == inf] = -1
    return d


def device_graph(mfbc, g):
    """Load g and apply the work decomposition the benchmark applies."""
    from paper_1609_07008_amd import autotune
    dg = mfbc.DeviceGraph(g)
    autotune.apply_plan(dg, g, autotune.load_cache())
    return dg


def log(msg):
    print(f"[configs] {msg}", flush=True)


def full_batch_checks(torch, mfbc, dg, g, src, batch, frontier_cols, chunk=16):
    threads = oracle.brandes_threads()
    b0 = src[:batch]
    t0 = time.perf_counter()
    f = dg.forward(b0)
    b = dg.backward(b0, f["dist"], f["sigma"], trace=True)
    log(f"{g.name}: forward+backward of {batch} columns, {f['products']} + {b['products']} products")
    for c0 in range(0, batch, chunk):
        cols = slice(c0, min(batch, c0 + chunk))
        ref = oracle.brandes(g, b0[cols], nthreads=threads)
        d = host_dist(f["dist"][cols].cpu().numpy(), mfbc.INF_DIST)
        assert np.array_equal(d, ref["dist"]), f"distances, columns {c0}.."
        rel_close(f["sigma"][cols].cpu().numpy(), ref["sigma"], 1e-12, f"sigma, columns {c0}..")
        rel_close(b["delta"][cols].cpu().numpy(), ref["delta"], 1e-10, f"delta, columns {c0}..")
        assert np.array_equal(b["step"][cols].cpu().numpy(), ref["height"]), f"heights {c0}.."
    log(f"{g.name}: tau/sigma/delta/heights of all {batch} columns match "
        f"({time.perf_counter() - t0:.1f}s)")
    # frontier membership: the whole batch traced, sampled columns checked
    t0 = time.perf_counter()
    ft = dg.forward(b0, trace=True, max_products=f["products"])
    assert ft["products"] == f["products"]
    assert torch.equal(ft["dist"], f["dist"]) and torch.equal(ft["sigma"], f["sigma"])
    arcs = frontier.InArcs(g)
    for c in frontier_cols:
        want = frontier.forward_frontiers(g, int(b0[c]), arcs=arcs)
        assert len(want) <= f["products"]
        rows = mfbc.DeviceGraph.frontier_rows(ft["fbits"][:, c, :].cpu().numpy(), g.n)
        for j in range(1, f["products"] + 1):
            w = want[j - 1] if j <= len(want) else np.zeros(g.n, bool)
            assert np.array_equal(rows[j - 1], w), f"column {c}, frontier {j}"
    log(f"{g.name}: frontiers of columns {list(frontier_cols)} at all {f['products']} products "
        f"match ({time.perf_counter() - t0:.1f}s)")
    del f, b, ft


def lambda_all_sources(mfbc, dg, g, src, batch):
    t0 = time.perf_counter()
    lam = dg.bc(src, batch).cpu().numpy()
    t1 = time.perf_counter()
    ref = oracle.brandes(g, src, per_source=False, nthreads=oracle.brandes_threads())["lambda"]
    t2 = time.perf_counter()
    rel_close(lam, ref, 1e-10, "lambda")
    log(f"{g.name}: lambda over {src.size} sources matches (GPU {t1 - t0:.2f}s, oracle "
        f"{t2 - t1:.1f}s on {oracle.brandes_threads()} threads)")


def test_er1024_exact_bc(torch, mfbc):
    g = gg.er_graph(1024, 8, 1, (1, 100))
    src = np.arange(g.n, dtype=np.int32)
    dg = device_graph(mfbc, g)
    lambda_all_sources(mfbc, dg, g, src, 64)
    # one batch of 64: every column, every product's frontier
    from tests.helpers import expected_forward
    f = dg.forward(src[:64], trace=True)
    products, member, nnz, relax = expected_forward(g, src[:64])
    assert f["products"] == products
    fb = mfbc.DeviceGraph.frontier_rows(f["fbits"][:products].cpu().numpy(), g.n)
    for j in range(1, products + 1):
        assert np.array_equal(fb[j - 1], member(j)), f"frontier {j}"
    assert f["nnz"].tolist() == nnz and f["relax"].tolist() == relax
    dg.close()


def test_rmat16_unweighted_4096_sources(torch, mfbc):
    g = gg.rmat_graph(16, 16, 2)
    src = gg.pick_sources(g, 4096, 102)
    dg = device_graph(mfbc, g)
    log(f"rmat16 m={g.m}")
    lambda_all_sources(mfbc, dg, g, src, 512)
    st = dg.stats()
    assert st["batches"] == 8
    full_batch_checks(torch, mfbc, dg, g, src, 512, frontier_cols=[0, 211, 511], chunk=64)
    # unweighted: the forward frontiers are BFS levels, one product per level
    # plus the one that finds nothing; backward: the counting product plus
    # one per DAG height level below the source's
    b0 = src[:512]
    r = oracle.brandes(g, b0, nthreads=oracle.brandes_threads())
    f = dg.forward(b0)
    bw = dg.backward(b0, f["dist"], f["sigma"])
    assert f["products"] == int(r["dist"].max()) + 1
    assert bw["products"] == frontier.backward_products(r["height"], b0)
    dg.close()


def test_rmat20_weighted_full(torch, mfbc):
    g = gg.rmat_graph(20, 16, 3, wrange=(1, 255))
    src = gg.pick_sources(g, 1024, 103)
    log(f"rmat20 m={g.m}")
    dg = device_graph(mfbc, g)
    lambda_all_sources(mfbc, dg, g, src, 256)
    full_batch_checks(torch, mfbc, dg, g, src, 256, frontier_cols=[0, 77, 130, 255])
    dg.close()


def test_er32k_dense_weighted_full(torch, mfbc):
    g = gg.er_graph(32768, 512, 4, (1, 255))
    src = gg.pick_sources(g, 1024, 104)
    log(f"er32k m={g.m}")
    dg = device_graph(mfbc, g)
    lambda_all_sources(mfbc, dg, g, src, 256)
    full_batch_checks(torch, mfbc, dg, g, src, 256, frontier_cols=[3, 128, 200])
    dg.close()
