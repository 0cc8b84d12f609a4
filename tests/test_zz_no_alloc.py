"""mfbc_bc_noalloc (batch state in the library's static scratch) against
mfbc_bc on the same inputs, through the C ABI: two calls in a row, the
second with a smaller input, each to the parity bar of lambda (relative
1e-10 elementwise, zeros exact); sizes beyond the scratch are rejected with
MFBC_ENOMEM before any device work; the call allocates no device memory."""
import numpy as np
import pytest

from paper_1609_07008_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_07008_amd import mfbc as m
    m.load_library()
    return t, m


def rel_close(got, want, tol, what=""):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, what
    zero = want == 0
    assert np.count_nonzero(got[zero]) == 0, f"{what}: zeros must be exact"
    if (~zero).any():
        err = np.abs(got[~zero] - want[~zero]) / np.abs(want[~zero])
        assert err.max() <= tol, f"{what}: max rel err {err.max():.3e}"


def test_noalloc_matches_bc_on_two_calls(env):
    t, mfbc = env
    # set-up: the first call on a device loads the library's code object (and
    # with it the static scratch) and takes the scratch's address
    tiny = mfbc.DeviceGraph(gg.path_graph(5))
    tiny.bc_noalloc(t.arange(5, dtype=t.int32, device="cuda"), 5,
                    t.zeros(5, dtype=t.float64, device="cuda"))
    tiny.close()
    big = gg.er_graph(1024, 8, 1, (1, 100))             # all sources, batches of 64
    small = gg.er_graph(300, 6, 11, (1, 20))            # 100 sources, one batch of 2 groups
    cases = [(big, np.arange(big.n, dtype=np.int32), 64),
             (small, np.arange(0, 300, 3, dtype=np.int32), 128)]
    for g, src, batch in cases:
        print(f"[noalloc] n={g.n} sources={src.size} batch={batch}", flush=True)
        dg = mfbc.DeviceGraph(g)
        d_src = t.as_tensor(src, device="cuda")
        out = t.full((g.n,), -1.0, dtype=t.float64, device="cuda")
        t.cuda.synchronize()
        free0 = t.cuda.mem_get_info()[0]
        dg.bc_noalloc(d_src, batch, out)
        t.cuda.synchronize()
        free1 = t.cuda.mem_get_info()[0]
        # the plain path would allocate a workspace of a few MB here
        assert free1 >= free0 - (1 << 20), f"device memory went down by {free0 - free1} bytes"
        ref = dg.bc(d_src, batch).cpu().numpy()
        rel_close(out.cpu().numpy(), ref, 1e-10, f"n={g.n}")
        dg.close()


def test_noalloc_rejects_oversized_state(env):
    t, mfbc = env
    g = gg.rmat_graph(16, 16, 2)
    dg = mfbc.DeviceGraph(g)
    src = t.as_tensor(gg.pick_sources(g, 512, 102), device="cuda")
    out = t.zeros(g.n, dtype=t.float64, device="cuda")
    with pytest.raises(mfbc.MfbcError) as e:
        dg.bc_noalloc(src, 512, out)
    assert e.value.code == mfbc.MFBC_ENOMEM
    assert "static scratch" in str(e.value)
    dg.close()
    # a source outside [0, n) is found on the device
    g2 = gg.er_graph(300, 6, 11, (1, 20))
    dg2 = mfbc.DeviceGraph(g2)
    out2 = t.zeros(g2.n, dtype=t.float64, device="cuda")
    with pytest.raises(mfbc.MfbcError) as e:
        dg2.bc_noalloc(t.as_tensor(np.array([0, g2.n], dtype=np.int32), device="cuda"), 2, out2)
    assert e.value.code == mfbc.MFBC_EINVAL
    dg2.close()
