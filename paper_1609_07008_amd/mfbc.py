"""Thin ctypes binding of ``libmfbc.so`` (C ABI in ``include/mfbc.h``).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of MFBF, MFBr and MFBC runs in the library's HIP kernels.
There is no fallback: if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfbc.so")

MFBC_OK, MFBC_EINVAL, MFBC_ENOMEM, MFBC_EDEVICE, MFBC_EOVERFLOW = 0, -1, -2, -3, -4
MFBC_UNDIRECTED, MFBC_DIRECTED, MFBC_KEEP_ORDER = 1, 2, 4
INF_DIST = 0x7FFFFFFF
OP_SSSP, OP_BFS, OP_WIDEST, OP_RESIST = 0, 1, 2, 3
FIXPOINT_OPS = {"sssp": OP_SSSP, "bfs": OP_BFS, "widest": OP_WIDEST, "resist": OP_RESIST}

# Every entry point declared in include/mfbc.h, with its ctypes signature.
_P = ctypes.c_void_p
_I32, _I64, _U32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
SIGNATURES = {
    "mfbc_load_graph": ([_I32, _I64, _P, _P, _P, _U32, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "mfbc_free_graph": ([_P], ctypes.c_int),
    "mfbc_forward": ([_P, _P, _I32, _P, _P, _P, _P], ctypes.c_int),
    "mfbc_backward": ([_P, _P, _I32, _P, _P, _P, _P, _P], ctypes.c_int),
    "mfbc_bc": ([_P, _P, _I64, _I32, _P, _P], ctypes.c_int),
    "mfbc_bc_noalloc": ([_P, _P, _I64, _I32, _P, _P], ctypes.c_int),
    "mfbc_bc_requests": ([_P, _P, _P, _I32, _I32, _P, _P], ctypes.c_int),
    "mfbc_set_lanes": ([_P, _I32], ctypes.c_int),
    "mfbc_forward_trace": ([_P, _P, _I32, _P, _P, _P, _I32, _P, _P, _P, _P], ctypes.c_int),
    "mfbc_backward_trace": ([_P, _P, _I32, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "mfbc_get_stats": ([_P, _P], ctypes.c_int),
    "mfbc_enable_timing": ([_P, ctypes.c_int], ctypes.c_int),
    "mfbc_set_plan": ([_P, _I32, _I32, _I32, _I32], ctypes.c_int),
    "mfbc_graph_info": ([_P, _P, _P, _P], ctypes.c_int),
    "mfbc_bc_many": ([_I32, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "mfbc_fixpoint": ([_P, _I32, _P, _I32, _P, _P, _P], ctypes.c_int),
    "mfbc_last_error": ([], ctypes.c_char_p),
}


class MfbcStats(ctypes.Structure):
    _fields_ = [(k, _I64) for k in (
        "fwd_products", "bwd_products", "fwd_entries", "bwd_entries", "batches",
        "fwd_outputs", "bwd_outputs", "fwd_active_vertices", "fwd_active_arcs",
        "bwd_active_vertices", "bwd_active_arcs", "fwd_pull_launches", "bwd_pull_launches",
        "count_launches")] + [(k, ctypes.c_double) for k in (
        "fwd_pull_ms", "fwd_merge_ms", "count_ms", "bwd_pull_ms", "bwd_merge_ms", "other_ms",
        "fwd_alg_bytes", "bwd_alg_bytes", "count_alg_bytes")]


class MfbcManyConfig(ctypes.Structure):
    _fields_ = [("block_threads", _I32), ("blocks", _I32), ("job_width", _I32)]


class MfbcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mfbc error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmfbc.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        # load torch's HIP runtime first, so that the library binds to the same
        # one (a second runtime in the process would not share devices/streams)
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != MFBC_OK:
        msg = load_library().mfbc_last_error().decode(errors="replace")
        raise MfbcError(rc, msg)


def _stream(torch, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class DeviceGraph:
    """A graph resident on the current HIP device (handle of ``mfbc_load_graph``)."""

    def __init__(self, g, directed: Optional[bool] = None, keep_order: bool = False):
        """``keep_order``: store vertices in the caller's order instead of the
        library's descending-degree order (results are the same either way,
        up to the summation order of floating-point sums)."""
        import torch
        self._torch = torch
        lib = load_library()
        if directed is None:
            directed = type(g).__name__ == "DiGraph"
        rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(g.col, dtype=np.int32)
        w = None if g.w is None else np.ascontiguousarray(g.w, dtype=np.int32)
        h = ctypes.c_void_p()
        rc = lib.mfbc_load_graph(
            int(g.n), int(rp[-1]), rp.ctypes.data_as(_P), col.ctypes.data_as(_P),
            None if w is None else w.ctypes.data_as(_P),
            (MFBC_DIRECTED if directed else MFBC_UNDIRECTED) | (MFBC_KEEP_ORDER if keep_order else 0),
            _stream(torch), ctypes.byref(h))
        _check(rc)
        self.handle = h
        self.n = int(g.n)
        self.arcs = int(rp[-1])
        self.m = self.arcs if directed else self.arcs // 2
        self.directed = bool(directed)

    def close(self):
        """Free the graph; raises (and keeps the graph) while a server made on
        it is still open."""
        if getattr(self, "handle", None):
            _check(load_library().mfbc_free_graph(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _src(self, sources):
        t = self._torch
        if isinstance(sources, t.Tensor):
            assert sources.dtype == t.int32 and sources.is_cuda and sources.is_contiguous()
            return sources
        return t.as_tensor(np.asarray(sources, dtype=np.int32), device="cuda")

    def forward(self, sources, trace: bool = False, max_products: Optional[int] = None,
                frontiers: bool = True, stream=None):
        """MFBF for a batch: dist int32[nb][n], sigma float64[nb][n], products.

        ``trace``: also ``nnz`` (frontier entries per product), ``relax``
        (relaxations per product) and, if ``frontiers``, ``fbits``: int64
        [max_products][nb][(n+63)//64] membership bitmaps of each product's
        frontier (see ``frontier_rows``).  ``max_products`` defaults to
        min(n + 2, 4096)."""
        t = self._torch
        lib = load_library()
        src = self._src(sources)
        nb = src.numel()
        dist = t.empty((nb, self.n), dtype=t.int32, device="cuda")
        sigma = t.empty((nb, self.n), dtype=t.float64, device="cuda")
        prods = ctypes.c_int32(0)
        out = {"dist": dist, "sigma": sigma}
        if trace:
            if max_products is None:
                max_products = min(self.n + 2, 4096)
            words = (self.n + 63) // 64
            fbits = (t.zeros((max_products, nb, words), dtype=t.int64, device="cuda")
                     if frontiers else None)
            nnz = np.zeros(max_products, dtype=np.int64)
            relax = np.zeros(max_products, dtype=np.int64)
            rc = lib.mfbc_forward_trace(self.handle, _ptr(src), nb, _ptr(dist), _ptr(sigma),
                                        _ptr(fbits), max_products, nnz.ctypes.data_as(_P),
                                        relax.ctypes.data_as(_P), ctypes.byref(prods),
                                        _stream(t, stream))
            out.update(fbits=fbits, nnz=nnz, relax=relax)
        else:
            rc = lib.mfbc_forward(self.handle, _ptr(src), nb, _ptr(dist), _ptr(sigma),
                                  ctypes.byref(prods), _stream(t, stream))
        _check(rc)
        out["products"] = prods.value
        if trace:
            k = min(prods.value, max_products)
            out["nnz"] = out["nnz"][:k]
            out["relax"] = out["relax"][:k]
        return out

    @staticmethod
    def frontier_rows(fbits_host: np.ndarray, n: int) -> np.ndarray:
        """Unpack host bitmaps [..., words] (from ``forward(trace=True)``) to bool [..., n]."""
        b = np.ascontiguousarray(fbits_host).view(np.uint64)
        bits = np.unpackbits(b.view(np.uint8), axis=-1, bitorder="little")
        return bits[..., :n].astype(bool)

    def fixpoint(self, sources, op: str = "sssp", out=None, stream=None):
        """Monoid relaxation to a fixpoint (mfbc_fixpoint) and the product
        count: int32[nb][n] distances ("sssp"), hop levels ("bfs") or
        bottleneck widths ("widest"), or float32[nb][n] sums of 1/w ("resist")."""
        t = self._torch
        code = FIXPOINT_OPS[op]
        src = self._src(sources)
        nb = src.numel()
        if out is None:
            dtype = t.float32 if code == OP_RESIST else t.int32
            out = t.empty((nb, self.n), dtype=dtype, device="cuda")
        prods = ctypes.c_int32(0)
        _check(load_library().mfbc_fixpoint(self.handle, code, _ptr(src), nb, _ptr(out),
                                            ctypes.byref(prods), _stream(t, stream)))
        return out, prods.value

    def backward(self, sources, dist, sigma, trace: bool = False, stream=None):
        """MFBr from a forward result: delta float64[nb][n], products."""
        t = self._torch
        lib = load_library()
        src = self._src(sources)
        nb = src.numel()
        delta = t.empty((nb, self.n), dtype=t.float64, device="cuda")
        prods = ctypes.c_int32(0)
        out = {"delta": delta}
        if trace:
            step = t.empty((nb, self.n), dtype=t.int32, device="cuda")
            rc = lib.mfbc_backward_trace(self.handle, _ptr(src), nb, _ptr(dist), _ptr(sigma),
                                         _ptr(delta), _ptr(step), ctypes.byref(prods),
                                         _stream(t, stream))
            out["step"] = step
        else:
            rc = lib.mfbc_backward(self.handle, _ptr(src), nb, _ptr(dist), _ptr(sigma),
                                   _ptr(delta), ctypes.byref(prods), _stream(t, stream))
        _check(rc)
        out["products"] = prods.value
        return out

    def bc(self, sources, batch: int, out=None, stream=None):
        """MFBC: lambda float64[n] over the listed sources in batches of ``batch``."""
        t = self._torch
        src = self._src(sources)
        if out is None:
            out = t.empty(self.n, dtype=t.float64, device="cuda")
        rc = load_library().mfbc_bc(self.handle, _ptr(src), src.numel(), int(batch), _ptr(out),
                                    _stream(t, stream))
        _check(rc)
        return out

    def bc_requests(self, source_lists, batch: int = 256, outs=None, stream=None):
        """mfbc_bc_requests: one lambda float64[n] per list of sources, the
        lists sharing batches (each list in whole groups of 64 columns)."""
        t = self._torch
        lists = [np.ascontiguousarray(x.detach().cpu().numpy() if isinstance(x, t.Tensor) else np.asarray(x),
                                      dtype=np.int32).ravel() for x in source_lists]
        first = np.zeros(len(lists) + 1, dtype=np.int64)
        if lists:
            first[1:] = np.cumsum([x.size for x in lists])
        src = self._src(np.concatenate(lists) if lists else np.zeros(0, dtype=np.int32))
        if outs is None:
            outs = [t.empty(self.n, dtype=t.float64, device="cuda") for _ in lists]
        ptrs = (ctypes.c_void_p * max(1, len(outs)))(*[o.data_ptr() for o in outs])
        rc = load_library().mfbc_bc_requests(self.handle, _ptr(src), first.ctypes.data_as(ctypes.c_void_p),
                                             len(lists), int(batch), ptrs, _stream(t, stream))
        _check(rc)
        return outs

    def bc_noalloc(self, sources, batch: int, out, stream=None):
        """mfbc_bc_noalloc: MFBC with the batch state in the library's static
        scratch (no device allocation); ``out`` float64[n] is caller-provided."""
        t = self._torch
        src = self._src(sources)
        rc = load_library().mfbc_bc_noalloc(self.handle, _ptr(src), src.numel(), int(batch),
                                            _ptr(out), _stream(t, stream))
        _check(rc)
        return out

    def set_plan(self, run_arcs: int = 0, run_verts: int = 0, heavy: int = 0, slice: int = 0):
        """Work decomposition of the products (0 = size-based default)."""
        _check(load_library().mfbc_set_plan(self.handle, run_arcs, run_verts, heavy, slice))

    def set_lanes(self, lanes: int = 0):
        """Batches of one bc() call run at once (1..4; 0 = by graph size)."""
        _check(load_library().mfbc_set_lanes(self.handle, int(lanes)))

    def enable_timing(self, mode=1):
        """Kernel timing with HIP events on the call's stream: 0 (or False) off;
        1 (or True) every product kernel and merge; 2 only the forward and
        fixpoint product kernels."""
        _check(load_library().mfbc_enable_timing(self.handle, int(mode)))

    def stats(self) -> dict:
        s = MfbcStats()
        _check(load_library().mfbc_get_stats(self.handle, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in MfbcStats._fields_}


def bc_many(graphs, sources, block_threads: int = 0, blocks: int = 0, job_width: int = 0,
            outs=None, stream=None):
    """Batched form: lambda of every graph over its source list, one persistent launch.

    ``graphs``: DeviceGraph list; ``sources``: one int32 source list (numpy
    or CUDA tensor) per graph; ``job_width``: sources per job, 64 or 128
    (0 = 64).  Returns a list of float64[n_i] tensors.
    """
    import torch
    lib = load_library()
    G = len(graphs)
    srcs = [g._src(s) for g, s in zip(graphs, sources)]
    if outs is None:
        outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for g in graphs]
    handles = (ctypes.c_void_p * G)(*[g.handle.value for g in graphs])
    sp = (ctypes.c_void_p * G)(*[t.data_ptr() for t in srcs])
    ns = (ctypes.c_int64 * G)(*[t.numel() for t in srcs])
    op = (ctypes.c_void_p * G)(*[t.data_ptr() for t in outs])
    cfg = MfbcManyConfig(block_threads, blocks, job_width)
    st = MfbcStats()
    rc = lib.mfbc_bc_many(G, ctypes.cast(handles, _P), ctypes.cast(sp, _P), ctypes.cast(ns, _P),
                          ctypes.cast(op, _P), ctypes.byref(cfg), ctypes.byref(st),
                          _stream(torch, stream))
    _check(rc)
    bc_many.last_stats = {"fwd_products": st.fwd_products, "bwd_products": st.bwd_products}
    return outs
