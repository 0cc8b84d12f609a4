"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: distances, frontier membership, backward frontier indices and product
counts bit-exact; sigma within relative 1e-12; delta and lambda within
relative 1e-10 elementwise, zeros exact.  Inputs are seeded graphs of the
paper's workload families (R-MAT, Erdos-Renyi, weighted and unweighted) plus
small structured graphs and edge cases.
"""
import numpy as np
import pytest

import oracle
from oracle.frontier import backward_products
from paper_1609_07008_amd import graphgen as gg
from tests.helpers import expected_forward

pytestmark = pytest.mark.gpu

SIGMA_TOL = 1e-12
DELTA_TOL = 1e-10


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
    bad = np.flatnonzero(got[zero] != 0)
    assert bad.size == 0, f"{what}: {bad.size} entries should be exactly 0"
    if (~zero).any():
        err = np.abs(got[~zero] - want[~zero]) / np.abs(want[~zero])
        assert err.max() <= tol, f"{what}: max rel err {err.max():.3e}"


def host_dist(d, inf):
    d = d.cpu().numpy().astype(np.int64)
    d[d == inf] = -1
    return d


def graphs():
    u, v, w = zip(*[(0, 1, 1), (0, 2, 1), (1, 3, 1), (2, 3, 1), (3, 4, 2), (0, 4, 5), (1, 4, 3)])
    two = gg.er_graph(150, 4, 31, (1, 9))
    u2, v2, w2 = two.edges()
    disc = gg.csr_from_edges(2 * 150 + 5, np.concatenate([u2, u2 + 150]),
                             np.concatenate([v2, v2 + 150]), np.concatenate([w2, w2]), "disconnected")
    return {
        "golden5": gg.csr_from_edges(5, u, v, w, "golden5"),
        "er1024_w100": gg.er_graph(1024, 8, 1, (1, 100)),
        "er600_unw": gg.er_graph(600, 10, 2),
        "rmat10_unw": gg.rmat_graph(10, 8, 5),
        "rmat11_w255": gg.rmat_graph(11, 16, 6, wrange=(1, 255)),
        "rmat12_w3": gg.rmat_graph(12, 16, 7, wrange=(1, 3)),
        "grid20x30": gg.grid_graph(20, 30),
        "path300": gg.path_graph(300, w=4),
        "star200": gg.star_graph(200),
        "diamonds40": gg.diamond_chain(40),
        "disconnected": disc,
        # frontier rows past the 16-bit tuple's weight range: all long along
        # a heavy path, a mix of short and long rows with wide weights
        "path400_w97": gg.path_graph(400, w=97),
        "er800_w3000": gg.er_graph(800, 6, 9, (1, 3000)),
        # distances past 16 bits (the counting product's compact tau copy
        # holds finite values up to 65533): up to 76,245 along a heavy path;
        # exactly 65533 at most; exactly 65534 and 65535 (the compact
        # copy's two reserved codes)
        "path300_w255": gg.path_graph(300, w=255),
        "ladder_65533": gg.csr_from_edges(3, [0, 1], [1, 2], [65532, 1], "ladder_65533"),
        "ladder_65535": gg.csr_from_edges(4, [0, 1, 2], [1, 2, 3], [65533, 1, 1], "ladder_65535"),
    }


GRAPHS = graphs()
NB = [1, 5, 64, 65, 130, 256]     # 256: four groups, one wide forward group


@pytest.fixture(scope="module")
def dgraphs(mfbc):
    out = {k: mfbc.DeviceGraph(g) for k, g in GRAPHS.items()}
    yield out
    for d in out.values():
        d.close()


def pick(g, nb, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, g.n, size=nb).astype(np.int32)     # repeats allowed


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("nb", NB)
def test_forward_parity(torch, mfbc, dgraphs, name, nb):
    g = GRAPHS[name]
    src = pick(g, nb, 100 + nb)
    print(f"[forward] {name} nb={nb}", flush=True)
    f = dgraphs[name].forward(src, trace=True)
    ref = oracle.brandes(g, src)
    assert np.array_equal(host_dist(f["dist"], mfbc.INF_DIST), ref["dist"])
    rel_close(f["sigma"].cpu().numpy(), ref["sigma"], SIGMA_TOL, "sigma")
    check_frontiers(mfbc, g, src, f)


def check_frontiers(mfbc, g, src, f):
    """Every product's frontier, bit-exact, against Lemma 1's sets; the
    product count, frontier sizes and relaxations per product."""
    products, member, nnz, relax = expected_forward(g, src)
    assert f["products"] == products
    fb = mfbc.DeviceGraph.frontier_rows(f["fbits"][:products].cpu().numpy(), g.n)
    for j in range(1, products + 1):
        assert np.array_equal(fb[j - 1], member(j)), f"frontier {j} of {products}"
    assert f["nnz"].tolist() == nnz
    assert f["relax"].tolist() == relax


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("nb", [1, 64, 130, 260])
def test_backward_parity(torch, mfbc, dgraphs, name, nb):
    g = GRAPHS[name]
    src = pick(g, nb, 200 + nb)
    print(f"[backward] {name} nb={nb}", flush=True)
    ref = oracle.brandes(g, src)
    f = dgraphs[name].forward(src)
    b = dgraphs[name].backward(src, f["dist"], f["sigma"], trace=True)
    rel_close(b["delta"].cpu().numpy(), ref["delta"], DELTA_TOL, "delta")
    assert np.array_equal(b["step"].cpu().numpy(), ref["height"])
    # counting product + one per height level of a non-source vertex + the
    # product that finds nothing (the source has no predecessor, so its own
    # entry feeds no product)
    assert b["products"] == backward_products(ref["height"], src)


@pytest.mark.parametrize("name", list(GRAPHS))
def test_backward_from_oracle_forward(torch, mfbc, dgraphs, name):
    """MFBr alone, fed the oracle's tau and sigma."""
    g = GRAPHS[name]
    src = pick(g, 70, 7)
    ref = oracle.brandes(g, src)
    d = ref["dist"].copy()
    d[d < 0] = mfbc.INF_DIST
    dist = torch.as_tensor(d.astype(np.int32), device="cuda")
    sig = torch.as_tensor(ref["sigma"], device="cuda")
    b = dgraphs[name].backward(src, dist, sig, trace=True)
    rel_close(b["delta"].cpu().numpy(), ref["delta"], DELTA_TOL, "delta")
    assert np.array_equal(b["step"].cpu().numpy(), ref["height"])


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("batch", [1, 7, 64, 100, 256])
def test_bc_parity(torch, mfbc, dgraphs, name, batch):
    g = GRAPHS[name]
    src = np.arange(g.n, dtype=np.int32) if g.n <= 1100 else pick(g, 600, 3)
    if batch == 1 and src.size > 200:
        src = src[:200]
    print(f"[bc] {name} batch={batch} sources={src.size}", flush=True)
    lam = dgraphs[name].bc(src, batch).cpu().numpy()
    ref = oracle.brandes(g, src, per_source=False)["lambda"]
    rel_close(lam, ref, DELTA_TOL, "lambda")


@pytest.mark.parametrize("name", ["rmat11_w255", "er600_unw", "path300_w255", "star200", "disconnected"])
@pytest.mark.parametrize("batch", [64, 256])
def test_bc_requests_one_sum_per_list(torch, mfbc, dgraphs, name, batch):
    """mfbc_bc_requests: several source lists sharing batches, each in whole
    64-column groups (lists spanning two and three batches, an empty list, a
    one-source list, repeats); every list's sum against the oracle and
    against mfbc_bc on the same list."""
    g = GRAPHS[name]
    dg = dgraphs[name]
    rng = np.random.default_rng(41)
    lists = [rng.integers(0, g.n, size=k).astype(np.int32) for k in (30, 0, 1, 130, 64, 7, 200)]
    print(f"[bc_requests] {name} batch={batch}", flush=True)
    outs = dg.bc_requests(lists, batch)
    assert len(outs) == len(lists)
    for L, o in zip(lists, outs):
        got = o.cpu().numpy()
        if L.size == 0:
            assert np.all(got == 0)
            continue
        rel_close(got, oracle.brandes(g, L, per_source=False)["lambda"], DELTA_TOL, f"list of {L.size}")
        rel_close(got, dg.bc(L, batch).cpu().numpy(), 1e-12, f"list of {L.size} vs mfbc_bc")


def test_bc_requests_rejects_bad_arguments(torch, mfbc, dgraphs):
    dg = dgraphs["golden5"]
    with pytest.raises(mfbc.MfbcError) as e:
        dg.bc_requests([np.array([0, 1], dtype=np.int32)], 100)        # not a multiple of 64
    assert e.value.code == mfbc.MFBC_EINVAL
    with pytest.raises(mfbc.MfbcError) as e:
        dg.bc_requests([np.array([0], dtype=np.int32), np.array([5], dtype=np.int32)], 64)
    assert e.value.code == mfbc.MFBC_EINVAL                            # source outside [0, n)
    assert dg.bc_requests([], 64) == []
    # device tensors are accepted as lists too
    t_lists = [torch.as_tensor(np.array([0, 1, 2], dtype=np.int32), device="cuda")]
    rel_close(dg.bc_requests(t_lists, 64)[0].cpu().numpy(),
              oracle.brandes(GRAPHS["golden5"], np.array([0, 1, 2], dtype=np.int32), per_source=False)["lambda"],
              DELTA_TOL, "tensor list")


def test_bc_deterministic_and_batch_invariant(torch, mfbc, dgraphs):
    g = GRAPHS["rmat11_w255"]
    dg = dgraphs["rmat11_w255"]
    src = pick(g, 300, 9)
    a = dg.bc(src, 128).cpu().numpy()
    b = dg.bc(src, 128).cpu().numpy()
    assert np.array_equal(a, b), "same call must give bitwise-equal lambda"
    c = dg.bc(src, 37).cpu().numpy()
    rel_close(c, a, 1e-12, "batch invariance")


def test_duplicate_sources_count_per_occurrence(torch, mfbc, dgraphs):
    g = GRAPHS["er1024_w100"]
    dg = dgraphs["er1024_w100"]
    src = np.array([5, 9, 5, 5, 700], dtype=np.int32)
    lam = dg.bc(src, 2).cpu().numpy()
    rel_close(lam, oracle.brandes(g, src, per_source=False)["lambda"], DELTA_TOL, "dups")


def test_empty_source_list_gives_zero(torch, mfbc, dgraphs):
    dg = dgraphs["golden5"]
    lam = dg.bc(torch.empty(0, dtype=torch.int32, device="cuda"), 4).cpu().numpy()
    assert np.all(lam == 0)


@pytest.mark.parametrize("g", [
    gg.csr_from_edges(1, [], [], None, "single"),
    gg.csr_from_edges(2, [0], [1], [7], "edge"),
    gg.csr_from_edges(6, [], [], None, "no_arcs"),
    gg.complete_graph(9, w=2),
], ids=lambda g: g.name)
def test_tiny_and_degenerate_graphs(torch, mfbc, g):
    dg = mfbc.DeviceGraph(g)
    src = np.arange(g.n, dtype=np.int32)
    ref = oracle.brandes(g, src)
    f = dg.forward(src)
    assert np.array_equal(host_dist(f["dist"], mfbc.INF_DIST), ref["dist"])
    rel_close(f["sigma"].cpu().numpy(), ref["sigma"], SIGMA_TOL, "sigma")
    b = dg.backward(src, f["dist"], f["sigma"])
    rel_close(b["delta"].cpu().numpy(), ref["delta"], DELTA_TOL, "delta")
    rel_close(dg.bc(src, 3).cpu().numpy(), ref["lambda"], DELTA_TOL, "lambda")
    dg.close()


def test_directed_graph(torch, mfbc):
    g = gg.directed_rmat_graph(10, 8, 12, wrange=(1, 50))
    dg = mfbc.DeviceGraph(g, directed=True)
    src = pick(g, 150, 4)
    ref = oracle.brandes(g, src)
    f = dg.forward(src, trace=True)
    assert np.array_equal(host_dist(f["dist"], mfbc.INF_DIST), ref["dist"])
    rel_close(f["sigma"].cpu().numpy(), ref["sigma"], SIGMA_TOL, "sigma")
    check_frontiers(mfbc, g, src, f)
    b = dg.backward(src, f["dist"], f["sigma"], trace=True)
    rel_close(b["delta"].cpu().numpy(), ref["delta"], DELTA_TOL, "delta")
    assert np.array_equal(b["step"].cpu().numpy(), ref["height"])
    rel_close(dg.bc(src, 64).cpu().numpy(), ref["lambda"], DELTA_TOL, "lambda")
    # the same sources as three lists sharing batches
    parts = [src[:40], src[40:41], src[41:]]
    for L, o in zip(parts, dg.bc_requests(parts, 128)):
        rel_close(o.cpu().numpy(), oracle.brandes(g, L, per_source=False)["lambda"], DELTA_TOL,
                  f"list of {L.size}")
    dg.close()


def test_hub_rows_are_split_and_merged(torch, mfbc):
    """Stars and a dense hub exercise the sliced-row path (rows > 1024 arcs)."""
    k = 5000
    star = gg.star_graph(k)
    extra = gg.er_graph(k + 1, 3, 8, None)
    u1, v1, _ = star.edges()
    u2, v2, _ = extra.edges()
    key = np.unique(np.minimum(np.concatenate([u1, u2]), np.concatenate([v1, v2])) * (k + 1) +
                    np.maximum(np.concatenate([u1, u2]), np.concatenate([v1, v2])))
    rng = np.random.default_rng(1)
    g = gg.csr_from_edges(k + 1, key // (k + 1), key % (k + 1),
                          rng.integers(1, 4, size=key.size), "hubby")
    dg = mfbc.DeviceGraph(g)
    src = np.concatenate([[0], pick(g, 99, 2)]).astype(np.int32)
    ref = oracle.brandes(g, src)
    f = dg.forward(src)
    assert np.array_equal(host_dist(f["dist"], mfbc.INF_DIST), ref["dist"])
    rel_close(f["sigma"].cpu().numpy(), ref["sigma"], SIGMA_TOL, "sigma")
    b = dg.backward(src, f["dist"], f["sigma"], trace=True)
    rel_close(b["delta"].cpu().numpy(), ref["delta"], DELTA_TOL, "delta")
    assert np.array_equal(b["step"].cpu().numpy(), ref["height"])
    rel_close(dg.bc(src, 64).cpu().numpy(), ref["lambda"], DELTA_TOL, "lambda")
    # the same sources as three lists sharing batches
    parts = [src[:40], src[40:41], src[41:]]
    for L, o in zip(parts, dg.bc_requests(parts, 128)):
        rel_close(o.cpu().numpy(), oracle.brandes(g, L, per_source=False)["lambda"], DELTA_TOL,
                  f"list of {L.size}")
    dg.close()


def test_errors_are_reported(torch, mfbc, dgraphs):
    dg = dgraphs["golden5"]
    with pytest.raises(mfbc.MfbcError) as e:
        dg.forward(np.array([0, 5], dtype=np.int32))
    assert e.value.code == mfbc.MFBC_EINVAL
    with pytest.raises(mfbc.MfbcError) as e:
        dg.bc(np.array([1, -1], dtype=np.int32), 2)
    assert e.value.code == mfbc.MFBC_EINVAL
    with pytest.raises(mfbc.MfbcError) as e:
        dg.bc(np.array([1], dtype=np.int32), 0)
    assert e.value.code == mfbc.MFBC_EINVAL
    # the handle still works after rejected calls
    f = dg.forward(np.array([0], dtype=np.int32))
    assert f["dist"].cpu().numpy().tolist() == [[0, 1, 1, 2, 4]]


PLANS = [(64, 1, 0, 0), (4096, 64, 0, 0), (0, 0, 8, 4), (0, 0, 64, 16), (1, 64, 2, 1), (700, 3, 40, 7)]


@pytest.mark.parametrize("name", ["rmat12_w3", "er600_unw", "star200"])
def test_results_do_not_depend_on_plan(torch, mfbc, name):
    """Work decompositions (runs of 1..64 rows, rows sliced down to 1 arc)
    give the same results: every plan against the oracle."""
    g = GRAPHS[name]
    dg = mfbc.DeviceGraph(g)
    src = pick(g, 130, 41)
    ref = oracle.brandes(g, src)
    lam_ref = oracle.brandes(g, src, per_source=False)["lambda"]
    for plan in PLANS:
        print(f"[plan] {name} {plan}", flush=True)
        dg.set_plan(*plan)
        f = dg.forward(src)
        assert np.array_equal(host_dist(f["dist"], mfbc.INF_DIST), ref["dist"]), plan
        rel_close(f["sigma"].cpu().numpy(), ref["sigma"], SIGMA_TOL, f"sigma {plan}")
        b = dg.backward(src, f["dist"], f["sigma"], trace=True)
        rel_close(b["delta"].cpu().numpy(), ref["delta"], DELTA_TOL, f"delta {plan}")
        assert np.array_equal(b["step"].cpu().numpy(), ref["height"]), plan
        rel_close(dg.bc(src, 64).cpu().numpy(), lam_ref, DELTA_TOL, f"lambda {plan}")
    for bad in [(0, 65, 0, 0), (0, 0, (1 << 24) + 1, 0), ((1 << 24) + 1, 0, 0, 0)]:
        with pytest.raises(mfbc.MfbcError) as e:
            dg.set_plan(*bad)
        assert e.value.code == mfbc.MFBC_EINVAL
    dg.close()


def test_path_count_overflow_is_reported(torch, mfbc):
    """1100 diamonds in series: 2^1100 shortest paths end to end, past
    binary64.  MFBF and MFBC report EOVERFLOW; the fixpoint, which carries no
    counts, still gives the distances."""
    g = gg.diamond_chain(1100)
    dg = mfbc.DeviceGraph(g)
    src = np.array([0], dtype=np.int32)
    with pytest.raises(mfbc.MfbcError) as e:
        dg.forward(src)
    assert e.value.code == mfbc.MFBC_EOVERFLOW
    with pytest.raises(mfbc.MfbcError) as e:
        dg.bc(src, 64)
    assert e.value.code == mfbc.MFBC_EOVERFLOW
    d, _ = dg.fixpoint(src, "sssp")
    assert host_dist(d, mfbc.INF_DIST)[0, 3 * 1100] == 2 * 1100
    # a chain of 1000 diamonds (2^1000 paths) stays finite and exact
    g2 = gg.diamond_chain(1000)
    dg2 = mfbc.DeviceGraph(g2)
    f = dg2.forward(src)
    assert f["sigma"].cpu().numpy()[0, 3 * 1000] == 2.0 ** 1000
    dg.close()
    dg2.close()


def test_workspace_enomem_is_reported_and_recoverable(torch, mfbc):
    """A batch whose state cannot fit device memory (2^20 sources in one batch
    on 100,000 vertices: several TB) is refused with MFBC_ENOMEM before any
    product runs, and the graph then serves an ordinary call."""
    g = gg.er_graph(100_000, 4, 5, (1, 9))
    dg = mfbc.DeviceGraph(g)
    src = torch.randint(0, g.n, (1 << 20,), dtype=torch.int32, device="cuda",
                        generator=torch.Generator(device="cuda").manual_seed(3))
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    with pytest.raises(mfbc.MfbcError) as e:
        dg.bc(src, 1 << 20, out=out)
    assert e.value.code == mfbc.MFBC_ENOMEM
    assert "allocation" in str(e.value)
    s64 = src[:64].contiguous()
    lam = dg.bc(s64, 64).cpu().numpy()
    ref = oracle.brandes(g, s64.cpu().numpy(), per_source=False)["lambda"]
    rel_close(lam, ref, DELTA_TOL, "lambda after ENOMEM")
    dg.close()


@pytest.mark.parametrize("name", ["er1024_w100", "rmat11_w255", "er600_unw", "path300", "hubby"])
def test_lanes_give_the_oracle_lambda(torch, mfbc, dgraphs, name):
    """Batches of one call run on 1..4 lanes (streams with their own
    workspaces): every lane count and a ragged last batch give the oracle's
    lambda, and a repeated call with the same lane count is bitwise equal."""
    if name == "hubby":
        g = gg.star_graph(3000)
        dg = mfbc.DeviceGraph(g)
    else:
        g, dg = GRAPHS[name], dgraphs[name]
    src = np.arange(g.n, dtype=np.int32) if g.n <= 1100 else pick(g, 700, 3)
    ref = oracle.brandes(g, src, per_source=False)["lambda"]
    for lanes in (1, 2, 3, 4):
        dg.set_lanes(lanes)
        for batch in (64, 150):
            print(f"[lanes] {name} lanes={lanes} batch={batch}", flush=True)
            lam = dg.bc(src, batch).cpu().numpy()
            rel_close(lam, ref, DELTA_TOL, f"lanes={lanes} batch={batch}")
        a = dg.bc(src, 64).cpu().numpy()
        b = dg.bc(src, 64).cpu().numpy()
        assert np.array_equal(a, b), f"lanes={lanes}: repeated call differs"
    st = dg.stats()
    assert st["batches"] == (src.size + 63) // 64
    dg.set_lanes(0)
    with pytest.raises(mfbc.MfbcError) as e:
        dg.set_lanes(5)
    assert e.value.code == mfbc.MFBC_EINVAL
    if name == "hubby":
        dg.close()
