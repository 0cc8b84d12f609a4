"""Batched form (many graphs, one persistent launch) against the per-graph
C ABI and the CPU oracle, on graphs of uneven sizes, kinds and weights."""
import numpy as np
import pytest

import oracle
from paper_1609_07008_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mfbc():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_07008_amd import mfbc as m
    m.load_library()
    return m


def rel_close(got, want, tol, what=""):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    zero = want == 0
    assert np.count_nonzero(got[zero]) == 0, f"{what}: zeros must be exact"
    if (~zero).any():
        err = np.abs(got[~zero] - want[~zero]) / np.abs(want[~zero])
        assert err.max() <= tol, f"{what}: max rel err {err.max():.3e}"


def suite():
    gs = gg.batched_suite(count=10, seed0=7000, nmin=50, nmax=1500)
    gs.append(gg.star_graph(1500))                     # a hub row that is split
    gs.append(gg.csr_from_edges(3, [], [], None, "no_arcs"))
    gs.append(gg.diamond_chain(20))
    gs.append(gg.path_graph(300, w=255))               # distances past 16 bits
    return gs


@pytest.mark.parametrize("threads,width", [(256, 64), (512, 64), (256, 128), (512, 128)])
def test_bc_many_matches_oracle_and_per_graph(mfbc, threads, width):
    gs = suite()
    dgs = [mfbc.DeviceGraph(g) for g in gs]
    srcs = [np.arange(g.n, dtype=np.int32) for g in gs]
    srcs[0] = srcs[0][::3].copy()                       # a partial source list
    srcs[1] = srcs[1][:70].copy()                       # a job whose second group is short
    print(f"[batched] threads={threads} job_width={width}", flush=True)
    out = mfbc.bc_many(dgs, srcs, block_threads=threads, blocks=37, job_width=width)
    for g, dg, s, o in zip(gs, dgs, srcs, out):
        lam = o.cpu().numpy()
        ref = oracle.brandes(g, s, per_source=False)["lambda"]
        rel_close(lam, ref, 1e-10, g.name)
        if s.size:
            rel_close(lam, dg.bc(s, width).cpu().numpy(), 1e-12, g.name + " vs per-graph")
    again = mfbc.bc_many(dgs, srcs, block_threads=threads, blocks=11, job_width=width)
    for a, b in zip(out, again):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), "job-order sums are deterministic"
    for d in dgs:
        d.close()


def test_bc_many_weighted_and_unweighted_mixed(mfbc):
    gs = [gg.er_graph(400, 6, 1, (1, 100)), gg.er_graph(300, 5, 2), gg.rmat_graph(9, 8, 3),
          gg.rmat_graph(9, 8, 4, wrange=(1, 9))]
    dgs = [mfbc.DeviceGraph(g) for g in gs]
    srcs = [gg.pick_sources(g, 100, 5) for g in gs]
    out = mfbc.bc_many(dgs, srcs)
    for g, s, o in zip(gs, srcs, out):
        rel_close(o.cpu().numpy(), oracle.brandes(g, s, per_source=False)["lambda"], 1e-10, g.name)
    st = mfbc.bc_many.last_stats
    assert st["fwd_products"] > 0 and st["bwd_products"] > 0
    for d in dgs:
        d.close()


def test_bc_many_rejects_bad_sources(mfbc):
    g = gg.er_graph(50, 4, 3, (1, 5))
    dg = mfbc.DeviceGraph(g)
    with pytest.raises(mfbc.MfbcError) as e:
        mfbc.bc_many([dg], [np.array([0, 50], dtype=np.int32)])
    assert e.value.code == mfbc.MFBC_EINVAL
    with pytest.raises(mfbc.MfbcError) as e:
        mfbc.bc_many([dg], [np.array([0, 1], dtype=np.int32)], block_threads=1024)
    assert e.value.code == mfbc.MFBC_EINVAL
    with pytest.raises(mfbc.MfbcError) as e:
        mfbc.bc_many([dg], [np.array([0, 1], dtype=np.int32)], job_width=96)
    assert e.value.code == mfbc.MFBC_EINVAL
    dg.close()


def test_bc_many_at_batched_workload_sizes(mfbc):
    """Graphs of the batched workload itself (n up to 19,900, average degree
    up to 60, ER and R-MAT, weights 1..100), in the launch shape the
    benchmark uses: all-source results against one mfbc_bc per graph, the
    largest graph against the oracle over all its sources, and every graph
    against the oracle on a sampled source list."""
    import time
    import torch
    from paper_1609_07008_amd import autotune
    specs = gg.batched_specs()
    order = sorted(range(len(specs)), key=lambda i: -specs[i][1])
    rng = np.random.default_rng(11)
    pick = order[:5] + sorted(rng.choice(order[5:], size=10, replace=False).tolist())
    gs = [gg.batched_graph(i, specs[i]) for i in pick]
    print(f"[batched] graphs {[(g.name, g.n, g.m) for g in gs]}", flush=True)
    dgs = [mfbc.DeviceGraph(g) for g in gs]
    cfg = autotune.many_config(autotune.load_cache())
    srcs = [torch.arange(g.n, dtype=torch.int32, device="cuda") for g in gs]
    out = mfbc.bc_many(dgs, srcs, **cfg)
    for g, dg, s, o in zip(gs, dgs, srcs, out):
        rel_close(o.cpu().numpy(), dg.bc(s, 256).cpu().numpy(), 1e-10, g.name + " vs per-graph")
    # both job widths at the workload's sizes
    for width in (64, 128):
        other = mfbc.bc_many(dgs, srcs, **dict(cfg, job_width=width))
        for g, o, o2 in zip(gs, out, other):
            rel_close(o2.cpu().numpy(), o.cpu().numpy(), 1e-10, f"{g.name} job_width={width}")
    t0 = time.perf_counter()
    big = gs[0]
    ref = oracle.brandes(big, np.arange(big.n, dtype=np.int32), per_source=False,
                         nthreads=oracle.brandes_threads())["lambda"]
    rel_close(out[0].cpu().numpy(), ref, 1e-10, big.name + " all sources")
    print(f"[batched] {big.name}: all {big.n} sources match the oracle "
          f"({time.perf_counter() - t0:.1f}s)", flush=True)
    sample = [gg.pick_sources(g, min(128, int((g.degree > 0).sum())), 40 + i)
              for i, g in enumerate(gs)]
    out2 = mfbc.bc_many(dgs, sample, **cfg)
    for g, s, o in zip(gs, sample, out2):
        ref = oracle.brandes(g, s, per_source=False, nthreads=oracle.brandes_threads())["lambda"]
        rel_close(o.cpu().numpy(), ref, 1e-10, g.name + " sampled sources")
    for d in dgs:
        d.close()
