"""Monoid fixpoints (mfbc_fixpoint): SSSP distances, BFS hop levels,
widest-path bottlenecks (int32, max / min) and binary32 sums of 1/w.

Bars: values bit-exact against the CPU oracle (Brandes' distances for SSSP
and BFS; the oracle's hop-indexed fixpoint, pinned by brute force over
paths and walks, for the widest and reciprocal-sum instances -- binary32
compared bit for bit), product counts equal to the oracle's
strict-improvement frontier definition (the largest over the batch's
sources), at small sizes over several tiles and a ragged tail, with split
hub rows, and on sampled sources at the benchmark's size and launch
configuration.
"""
import numpy as np
import pytest

import oracle
from oracle.frontier import InArcs
from oracle.frontier import fixpoint as oracle_fixpoint
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


def unweighted(g):
    u, v, _ = g.edges()
    return gg.csr_from_edges(g.n, u, v, None, g.name + "_unw")


def graphs():
    two = gg.er_graph(150, 4, 31, (1, 9))
    u2, v2, w2 = two.edges()
    disc = gg.csr_from_edges(2 * 150 + 5, np.concatenate([u2, u2 + 150]),
                             np.concatenate([v2, v2 + 150]), np.concatenate([w2, w2]), "disconnected")
    return {
        "er1024_w100": gg.er_graph(1024, 8, 1, (1, 100)),
        "rmat11_w255": gg.rmat_graph(11, 16, 6, wrange=(1, 255)),
        "rmat10_unw": gg.rmat_graph(10, 8, 5),
        "grid20x30": gg.grid_graph(20, 30),
        "path300": gg.path_graph(300, w=4),
        "star200": gg.star_graph(200),
        "disconnected": disc,
    }


GRAPHS = graphs()


def host(d, inf):
    d = d.cpu().numpy().astype(np.int64)
    d[d == inf] = -1
    return d


def pick(g, nb, seed):
    return np.random.default_rng(seed).integers(0, g.n, size=nb).astype(np.int32)


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("nb", [1, 64, 130])
def test_sssp_and_bfs_parity(mfbc, name, nb):
    g = GRAPHS[name]
    src = pick(g, nb, 300 + nb)
    print(f"[fixpoint] {name} nb={nb}", flush=True)
    dg = mfbc.DeviceGraph(g)
    d, prods = dg.fixpoint(src, "sssp")
    ref = oracle.brandes(g, src)["dist"]
    assert np.array_equal(host(d, mfbc.INF_DIST), ref)
    assert prods == max(oracle_fixpoint(g, int(s), "sssp")[1] for s in np.unique(src))
    h, prods = dg.fixpoint(src, "bfs")
    ref = oracle.brandes(unweighted(g), src)["dist"]
    assert np.array_equal(host(h, mfbc.INF_DIST), ref)
    assert prods == int(ref.max()) + 1
    dg.close()


def oracle_rows(g, src, op, arcs=None):
    """The oracle's values for each source of the list and the batch's product count."""
    arcs = arcs or InArcs(g)
    refs = {int(s): oracle_fixpoint(g, int(s), op, arcs=arcs) for s in np.unique(src)}
    return np.stack([refs[int(s)][0] for s in src]), max(r[1] for r in refs.values())


def same_values(got, want, op):
    got = got.cpu().numpy()
    if op == "resist":
        return got.dtype == np.float32 and np.array_equal(got.view(np.uint32),
                                                         want.astype(np.float32).view(np.uint32))
    return np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("nb", [1, 64, 130])
def test_widest_and_resist_parity(mfbc, name, nb):
    g = GRAPHS[name]
    src = pick(g, nb, 500 + nb)
    print(f"[fixpoint] widest/resist {name} nb={nb}", flush=True)
    dg = mfbc.DeviceGraph(g)
    arcs = InArcs(g)
    for op in ("widest", "resist"):
        d, prods = dg.fixpoint(src, op)
        want, wprods = oracle_rows(g, src, op, arcs)
        assert same_values(d, want, op), op
        assert prods == wprods, op
    dg.close()


def test_fixpoint_plans_and_errors(mfbc):
    g = GRAPHS["rmat11_w255"]
    dg = mfbc.DeviceGraph(g)
    src = pick(g, 100, 9)
    ref = oracle.brandes(g, src)["dist"]
    others = {op: oracle_rows(g, src, op) for op in ("widest", "resist")}
    for plan in [(64, 1, 0, 0), (0, 0, 8, 4), (1, 64, 2, 1)]:
        dg.set_plan(*plan)
        d, _ = dg.fixpoint(src, "sssp")
        assert np.array_equal(host(d, mfbc.INF_DIST), ref), plan
        for op, (want, wprods) in others.items():
            d, prods = dg.fixpoint(src, op)
            assert same_values(d, want, op) and prods == wprods, (op, plan)
    lib = mfbc.load_library()
    import ctypes
    import torch
    out = torch.empty((1, g.n), dtype=torch.int32, device="cuda")
    s = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = lib.mfbc_fixpoint(dg.handle, 7, ctypes.c_void_p(s.data_ptr()), 1,
                           ctypes.c_void_p(out.data_ptr()), None, None)
    assert rc == mfbc.MFBC_EINVAL
    with pytest.raises(mfbc.MfbcError):
        dg.fixpoint(np.array([g.n], dtype=np.int32), "bfs")
    dg.close()


@pytest.fixture(scope="module")
def rmat20():
    return gg.rmat_graph(20, 16, 3, wrange=(1, 255))


@pytest.mark.parametrize("op", ["sssp", "bfs"])
def test_full_size_sampled(mfbc, rmat20, op):
    """R-MAT scale 20 (w 1..255), 256 sources in one call, as the benchmark
    runs it; eight sampled sources checked row by row against the oracle."""
    g = rmat20
    src = gg.pick_sources(g, 1024, 103)[:256].astype(np.int32)
    dg = mfbc.DeviceGraph(g)
    d, prods = dg.fixpoint(src, op)
    rows = [0, 1, 63, 64, 127, 128, 200, 255]
    gg_ = g if op == "sssp" else unweighted(g)
    ref = oracle.brandes(gg_, src[rows])["dist"]
    got = host(d, mfbc.INF_DIST)[rows]
    assert np.array_equal(got, ref)
    assert prods >= oracle_fixpoint(gg_, int(src[0]), op)[1]
    dg.close()


@pytest.mark.parametrize("op", ["widest", "resist"])
def test_full_size_sampled_widest_resist(mfbc, rmat20, op):
    """R-MAT scale 20 (w 1..255), 256 sources in one call; two sampled rows
    (one in each pair of column groups) against the oracle's fixpoint, and
    the product count no smaller than theirs."""
    g = rmat20
    src = gg.pick_sources(g, 1024, 103)[:256].astype(np.int32)
    dg = mfbc.DeviceGraph(g)
    d, prods = dg.fixpoint(src, op)
    arcs = InArcs(g)
    for r in (5, 190):
        want, k = oracle_fixpoint(g, int(src[r]), op, arcs=arcs)
        assert same_values(d[r:r + 1], want[None, :], op), r
        assert prods >= k
    print(f"[fixpoint] rmat20 {op}: {prods} products, rows 5 and 190 match", flush=True)
    dg.close()


@pytest.mark.parametrize("nb", [1, 130])
def test_fixpoints_on_a_directed_graph(mfbc, nb):
    """Directed R-MAT (weights 1..50): every algebra follows the arcs from
    the source (the product pulls over in-arcs); values and product counts
    against the oracle, which groups the out-arcs by head."""
    g = gg.directed_rmat_graph(10, 8, 31, wrange=(1, 50))
    src = pick(g, nb, 700 + nb)
    print(f"[fixpoint] directed nb={nb}", flush=True)
    dg = mfbc.DeviceGraph(g, directed=True)
    arcs = InArcs(g)
    for op in ("sssp", "widest", "resist"):
        d, prods = dg.fixpoint(src, op)
        want, wprods = oracle_rows(g, src, op, arcs)
        if op == "sssp":
            want = np.where(want >= (1 << 60), mfbc.INF_DIST, want)
        assert same_values(d, want, op), op
        assert prods == wprods, op
    h, prods = dg.fixpoint(src, "bfs")
    want, wprods = oracle_rows(g, src, "bfs", InArcs(g, unit_weights=True))
    assert same_values(h, np.where(want >= (1 << 60), mfbc.INF_DIST, want), "bfs") and prods == wprods
    dg.close()
