"""Frontier sets in closed form -- test infrastructure only.

Forward (Algorithm 1, Lemma 1 and its proof, Section 4.1.3).  Let l_j(v) be
the least weight of a walk from s to v with exactly j arcs (l_0(s) = 0, all
else INF) and L_j = min_{i <= j} l_i.  Product j of MFBF (F_0 = {s}) yields
the frontier

    F_j = { v : l_j(v) < INF  and  l_j(v) <= L_{j-1}(v) }:

a least-weight j-arc walk reaching v no heavier than anything found with
fewer arcs; its prefix is again such a walk, so it is produced from F_{j-1}.
Once some F_j is empty, every later one is too, so the number of products
MFBF performs is the first j with F_j empty.  For unweighted graphs F_j is
the j-th level of a breadth-first search.

Backward (Algorithm 2, Lemma 2, Section 4.2.3).  A reachable vertex enters
backward frontier B_k, k = 0, 1, ..., when k is its height in the
shortest-path DAG of s (0 for a vertex with no successor, else 1 + the
greatest height of its successors); heights come from the Brandes oracle.
"""
from __future__ import annotations

import numpy as np

INF = np.int64(1) << 60


def forward_frontiers(g, s: int, max_products: int = 1 << 20):
    """F_1, F_2, ... (bool[n] each, the last one empty) for source ``s``."""
    n = g.n
    u = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr))
    v = g.col.astype(np.int64)
    w = np.ones(u.size, np.int64) if g.w is None else g.w.astype(np.int64)
    ell = np.full(n, INF, dtype=np.int64)
    ell[s] = 0
    L = ell.copy()
    out = []
    for _ in range(max_products):
        cand = np.where(ell[u] < INF, ell[u] + w, INF)
        nxt = np.full(n, INF, dtype=np.int64)
        np.minimum.at(nxt, v, cand)
        F = (nxt < INF) & (nxt <= L)
        out.append(F)
        L = np.minimum(L, nxt)
        ell = nxt
        if not F.any():
            return out
    raise RuntimeError("frontier did not empty")


def backward_heights(height_row: np.ndarray) -> list:
    """B_0, B_1, ... (bool[n] each) from one source's DAG heights (-1 = unreachable)."""
    h = np.asarray(height_row)
    top = int(h.max()) if h.size else -1
    return [h == k for k in range(top + 1)]


def fixpoint(g, s: int, op: str = "sssp", max_products: int = 1 << 20):
    """Relaxation to a fixpoint with (+) = min over strict-improvement frontiers.

    Section 3's product C = A (+).f B with (+) = min and the action
    f(a, w) = a + w ("sssp") or a + 1 ("bfs"), iterated as Algorithm 1
    iterates it but without multiplicities, so an entry joins frontier j only
    when product j lowers it:  F_j = { v : l_j(v) < L_{j-1}(v) }  with l_j,
    L_j as above (arc weights, or 1 for "bfs").  Returns (L, products): the
    final values (INF where unreachable) and the index of the first product
    whose frontier is empty.  After an empty F_j every later one is empty
    too (l_{j+1}(v) >= min_u L_{j-1}(u) + w(u, v) >= L_j(v)).
    """
    n = g.n
    u = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr))
    v = g.col.astype(np.int64)
    if op == "bfs" or g.w is None:
        w = np.ones(u.size, np.int64)
    elif op == "sssp":
        w = g.w.astype(np.int64)
    else:
        raise ValueError(op)
    ell = np.full(n, INF, dtype=np.int64)
    ell[s] = 0
    L = ell.copy()
    for j in range(1, max_products + 1):
        cand = np.where(ell[u] < INF, ell[u] + w, INF)
        nxt = np.full(n, INF, dtype=np.int64)
        np.minimum.at(nxt, v, cand)
        F = nxt < L
        L = np.minimum(L, nxt)
        ell = nxt
        if not F.any():
            return L, j
    raise RuntimeError("fixpoint not reached")
