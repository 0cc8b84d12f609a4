"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (same graphs, seeds, source lists and batch sizes).

  * ER n=1024 (weights 1..100), exact BC over all 1024 sources, batch 64:
    every lambda entry against the oracle.
  * R-MAT scale 16 unweighted, 4096 sources, batch 512: every lambda entry;
    sampled columns of the first batch for tau / sigma; the product bound.
  * R-MAT scale 20 (weights 1..255) and ER n=32768 k=512 (weights 1..255),
    1024 sources, batch 256: sampled columns of a full batch against
    single-source oracle runs (tau, sigma, delta), lambda over a sample of
    sources, and lambda over all 1024 sources against the sum of the
    per-batch dependencies (a property that holds at any size).
"""
import numpy as np
import pytest

import oracle
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


def test_er1024_exact_bc(torch, mfbc):
    g = gg.er_graph(1024, 8, 1, (1, 100))
    src = np.arange(g.n, dtype=np.int32)
    dg = mfbc.DeviceGraph(g)
    lam = dg.bc(src, 64).cpu().numpy()
    rel_close(lam, oracle.brandes(g, src, per_source=False)["lambda"], 1e-10, "lambda")
    dg.close()


def test_rmat16_unweighted_4096_sources(torch, mfbc):
    g = gg.rmat_graph(16, 16, 2)
    src = gg.pick_sources(g, 4096, 102)
    dg = mfbc.DeviceGraph(g)
    print(f"[rmat16] m={g.m}", flush=True)
    lam = dg.bc(src, 512).cpu().numpy()
    ref = oracle.brandes(g, src, per_source=False, nthreads=oracle.brandes_threads())
    rel_close(lam, ref["lambda"], 1e-10, "lambda")
    st = dg.stats()
    assert st["batches"] == 8
    # every column of the first batch: tau bit-exact, sigma and delta to the bar
    b0 = src[:512]
    f = dg.forward(b0)
    bw = dg.backward(b0, f["dist"], f["sigma"], trace=True)
    r = oracle.brandes(g, b0, nthreads=oracle.brandes_threads())
    assert np.array_equal(host_dist(f["dist"].cpu().numpy(), mfbc.INF_DIST), r["dist"])
    rel_close(f["sigma"].cpu().numpy(), r["sigma"], 1e-12, "sigma")
    rel_close(bw["delta"].cpu().numpy(), r["delta"], 1e-10, "delta")
    assert np.array_equal(bw["step"].cpu().numpy(), r["height"])
    # unweighted: the forward frontiers are BFS levels, one product per level
    # plus the one that finds nothing; backward: the counting product plus
    # one per DAG height level below the source's
    assert f["products"] == int(r["dist"].max()) + 1
    assert bw["products"] == 1 + int(r["height"].max())
    dg.close()


def _sampled_full_batch(torch, mfbc, g, src, batch, seed):
    dg = mfbc.DeviceGraph(g)
    b0 = src[:batch]
    f = dg.forward(b0)
    b = dg.backward(b0, f["dist"], f["sigma"])
    cols = np.sort(np.random.default_rng(seed).choice(batch, size=6, replace=False))
    ref = oracle.brandes(g, b0[cols], nthreads=6)
    d = host_dist(f["dist"][cols].cpu().numpy(), mfbc.INF_DIST)
    assert np.array_equal(d, ref["dist"]), "distances"
    rel_close(f["sigma"][cols].cpu().numpy(), ref["sigma"], 1e-12, "sigma")
    rel_close(b["delta"][cols].cpu().numpy(), ref["delta"], 1e-10, "delta")
    del f, b
    # lambda over a sample of sources (one batch) against the oracle
    sample = b0[cols]
    lam_s = dg.bc(sample, batch).cpu().numpy()
    rel_close(lam_s, ref["lambda"], 1e-10, "lambda over sampled sources")
    # lambda over all sources == sum over batches of the dependencies
    lam = dg.bc(src, batch)
    acc = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    for i in range(0, src.size, batch):
        bs = src[i:i + batch]
        f = dg.forward(bs)
        b = dg.backward(bs, f["dist"], f["sigma"])
        acc += b["delta"].sum(dim=0)
        del f, b
    rel_close(lam.cpu().numpy(), acc.cpu().numpy(), 1e-12, "lambda vs sum of deltas")
    dg.close()


def test_rmat20_weighted_sampled(torch, mfbc):
    g = gg.rmat_graph(20, 16, 3, wrange=(1, 255))
    src = gg.pick_sources(g, 1024, 103)
    print(f"[rmat20] m={g.m}", flush=True)
    _sampled_full_batch(torch, mfbc, g, src, 256, 1)


def test_er32k_dense_weighted_sampled(torch, mfbc):
    g = gg.er_graph(32768, 512, 4, (1, 255))
    src = gg.pick_sources(g, 1024, 104)
    print(f"[er32k] m={g.m}", flush=True)
    _sampled_full_batch(torch, mfbc, g, src, 256, 2)
