"""ctypes wrapper of the C Brandes oracle (``brandes.c``) -- test infrastructure only.

Computes, for each listed source s, tau(s,.), sigma(s,.), delta(s,.) and the
shortest-path-DAG heights, and lambda = sum_s delta(s,.) (Section 2.4 and
Theorem 1: MFBC's output equals this definition).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "brandes.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def library_path() -> str:
    return _LIB


def build_library(verbose: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (-O3, OpenMP, portable x86-64)."""
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_library()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_bc.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int64, P, P, P, P, P,
                                  ctypes.c_int32]
        lib.oracle_bc.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def brandes(g, sources, per_source: bool = True, nthreads: int = 0) -> dict:
    """Run the oracle on graph ``g`` (graphgen.Graph or DiGraph) for ``sources``.

    Returns a dict with ``lambda`` (float64[n]) and, if ``per_source``,
    ``dist`` (int64[k][n], -1 = unreachable), ``sigma`` (float64[k][n]),
    ``delta`` (float64[k][n], delta(s,s) = 0) and ``height`` (int32[k][n]).
    """
    lib = _load()
    n = int(g.n)
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
    k = src.size
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = None if g.w is None else np.ascontiguousarray(g.w, dtype=np.int32)
    lam = np.zeros(n, dtype=np.float64)
    out = {"lambda": lam}
    dist = sigma = delta = height = None
    if per_source:
        dist = np.empty((k, n), np.int64)
        sigma = np.empty((k, n), np.float64)
        delta = np.empty((k, n), np.float64)
        height = np.empty((k, n), np.int32)
        out.update(dist=dist, sigma=sigma, delta=delta, height=height)
    rc = lib.oracle_bc(n, _ptr(rp), _ptr(col), _ptr(w), _ptr(src), k, _ptr(lam),
                       _ptr(dist), _ptr(sigma), _ptr(delta), _ptr(height), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_bc failed (bad source or out of memory)")
    return out


def brandes_threads() -> int:
    """Host threads available to this process (the CPU affinity mask)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1
