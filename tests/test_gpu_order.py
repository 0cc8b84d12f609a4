"""The library's internal vertex order (descending degree) is invisible.

Every entry point is run on the same graph loaded twice, once renumbered
(the default) and once with MFBC_KEEP_ORDER: integer results (distances,
frontier membership, backward frontier indices, product counts, fixpoint
values) are bit-identical between the two and to the CPU oracle; sigma,
delta and lambda match the oracle within relative 1e-12 / 1e-10.
"""
import ctypes

import numpy as np
import pytest

import oracle
from tests.helpers import expected_forward
from paper_1609_07008_amd import graphgen as gg

pytestmark = pytest.mark.gpu

SIGMA_TOL = 1e-12
DELTA_TOL = 1e-10


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
    assert got.shape == want.shape, what
    zero = want == 0
    assert np.all(got[zero] == 0), f"{what}: entries should be exactly 0"
    if (~zero).any():
        err = np.abs(got[~zero] - want[~zero]) / np.abs(want[~zero])
        assert err.max() <= tol, f"{what}: max rel err {err.max():.3e}"


def host_dist(d, inf):
    d = d.cpu().numpy().astype(np.int64)
    d[d == inf] = -1
    return d


def hubby():
    """A star of 3000 leaves over a sparse random graph: one hub row, split
    into slices, lands at device id 0."""
    k = 3000
    star = gg.star_graph(k)
    extra = gg.er_graph(k + 1, 3, 8, None)
    u1, v1, _ = star.edges()
    u2, v2, _ = extra.edges()
    a, b = np.concatenate([u1, u2]), np.concatenate([v1, v2])
    key = np.unique(np.minimum(a, b) * (k + 1) + np.maximum(a, b))
    w = np.random.default_rng(1).integers(1, 4, size=key.size)
    # the hub is the LAST vertex, so the renumbering moves it
    lo, hi = key // (k + 1), key % (k + 1)
    return gg.csr_from_edges(k + 1, k - lo, k - hi, w, "hub_last")


GRAPHS = {
    "rmat11_w255": (gg.rmat_graph(11, 16, 6, wrange=(1, 255)), False),
    "rmat10_unw": (gg.rmat_graph(10, 8, 5), False),
    "hub_last": (hubby(), False),
    "directed_rmat10": (gg.directed_rmat_graph(10, 8, 12, wrange=(1, 50)), True),
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_every_entry_point_in_caller_order(mfbc, name):
    g, directed = GRAPHS[name]
    src = np.random.default_rng(7).integers(0, g.n, size=130).astype(np.int32)
    print(f"[order] {name}", flush=True)
    ref = oracle.brandes(g, src)
    lam_ref = oracle.brandes(g, src, per_source=False)["lambda"]
    products = expected_forward(g, src)[0]
    got = {}
    for keep in (False, True):
        dg = mfbc.DeviceGraph(g, directed=directed, keep_order=keep)
        f = dg.forward(src, trace=True)
        assert np.array_equal(host_dist(f["dist"], mfbc.INF_DIST), ref["dist"]), keep
        rel_close(f["sigma"].cpu().numpy(), ref["sigma"], SIGMA_TOL, f"sigma keep={keep}")
        assert f["products"] == products
        b = dg.backward(src, f["dist"], f["sigma"], trace=True)
        rel_close(b["delta"].cpu().numpy(), ref["delta"], DELTA_TOL, f"delta keep={keep}")
        assert np.array_equal(b["step"].cpu().numpy(), ref["height"]), keep
        # backward from the oracle's forward arrays (the import transpose)
        import torch
        d_in = torch.tensor(np.where(ref["dist"] < 0, mfbc.INF_DIST, ref["dist"]).astype(np.int32),
                            device="cuda")
        s_in = torch.tensor(ref["sigma"], dtype=torch.float64, device="cuda")
        b2 = dg.backward(src, d_in, s_in)
        rel_close(b2["delta"].cpu().numpy(), ref["delta"], DELTA_TOL, f"delta(import) keep={keep}")
        rel_close(dg.bc(src, 64).cpu().numpy(), lam_ref, DELTA_TOL, f"lambda keep={keep}")
        sp, _ = dg.fixpoint(src, "sssp")
        bf, _ = dg.fixpoint(src, "bfs")
        got[keep] = dict(fbits=f["fbits"].cpu().numpy(), nnz=f["nnz"].tolist(),
                         relax=f["relax"].tolist(),
                         step=b["step"].cpu().numpy(), sssp=sp.cpu().numpy(),
                         bfs=bf.cpu().numpy(), bprod=b["products"])
        dg.close()
    for k in got[False]:
        assert np.array_equal(np.asarray(got[False][k]), np.asarray(got[True][k])), k
    sssp = got[False]["sssp"].astype(np.int64)
    assert np.array_equal(np.where(sssp == mfbc.INF_DIST, -1, sssp), ref["dist"])


def test_batched_mixes_orders(mfbc):
    """One persistent launch over graphs loaded in both orders."""
    import torch
    gs = [gg.er_graph(300, 6, 3, (1, 20)), gg.rmat_graph(9, 8, 4, wrange=(1, 20)),
          gg.er_graph(500, 4, 5, (1, 20))]
    dgs = [mfbc.DeviceGraph(g, keep_order=(i % 2 == 1)) for i, g in enumerate(gs)]
    srcs = [torch.arange(g.n, dtype=torch.int32, device="cuda") for g in gs]
    outs = mfbc.bc_many(dgs, srcs)
    for g, o in zip(gs, outs):
        lam = oracle.brandes(g, np.arange(g.n, dtype=np.int32), per_source=False)["lambda"]
        rel_close(o.cpu().numpy(), lam, DELTA_TOL, g.name)
    for d in dgs:
        d.close()


def test_load_flags_are_checked(mfbc):
    g = gg.path_graph(4)
    lib = mfbc.load_library()
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    for flags in (mfbc.MFBC_KEEP_ORDER, 8, mfbc.MFBC_UNDIRECTED | 8, 3):
        h = ctypes.c_void_p()
        rc = lib.mfbc_load_graph(g.n, int(rp[-1]), rp.ctypes.data_as(ctypes.c_void_p),
                                 col.ctypes.data_as(ctypes.c_void_p), None, flags, None,
                                 ctypes.byref(h))
        assert rc == mfbc.MFBC_EINVAL, flags
