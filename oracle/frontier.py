"""Frontier sets and hop-indexed relaxations -- test infrastructure only.

Forward (Algorithm 1, Lemma 1 and its proof, Section 4.1.3).  Let l_j(v) be
the least weight of a walk from s to v with exactly j arcs (l_0(s) = 0, all
else INF) and L_j = min_{i <= j} l_i.  Product j of MFBF (F_0 = {s}) yields
the frontier

    F_j = { v : l_j(v) < INF  and  l_j(v) <= L_{j-1}(v) }:

a least-weight j-arc walk reaching v no heavier than anything found with
fewer arcs; its prefix is again such a walk, so it is produced from F_{j-1}.
Once some F_j is empty, every later one is too, so the number of products
MFBF performs is the first j with F_j empty.  For unweighted graphs F_j is
the j-th level of a breadth-first search.  The relaxations of product j
(Section 5's flops of a product) are the arcs leaving the entries of
F_{j-1}: sum over v in F_{j-1} of the out-degree of v.

l_j follows from l_{j-1} by one step of the definition, l_j(v) = min over
arcs u -> v of l_{j-1}(u) + w(u, v), evaluated here over the arcs grouped by
their head (numpy's minimum.reduceat over each head's in-arcs).

Backward (Algorithm 2, Lemma 2, Section 4.2.3).  A reachable vertex enters
backward frontier B_k, k = 0, 1, ..., when k is its height in the
shortest-path DAG of s (0 for a vertex with no successor, else 1 + the
greatest height of its successors); heights come from the Brandes oracle.
The source has no predecessor, so its own entry feeds no product; the
backward loop over a batch therefore ends with the product that reads the
greatest height of a non-source vertex: 1 (counting product) + that height
+ 1 products, or 1 if no non-source vertex is reachable (backward_products).
"""
from __future__ import annotations

import numpy as np

INF = np.int64(1) << 60


class InArcs:
    """Arcs of g grouped by head: tail[], weight[] in head order, and the
    first arc of every head that has one (for reduceat)."""

    def __init__(self, g, unit_weights: bool = False):
        n = g.n
        u = np.repeat(np.arange(n, dtype=np.int64), np.diff(np.asarray(g.row_ptr, np.int64)))
        v = np.asarray(g.col, np.int64)
        w = (np.ones(u.size, np.int64) if (g.w is None or unit_weights)
             else np.asarray(g.w, np.int64))
        order = np.argsort(v, kind="stable")
        self.n = n
        self.tail = u[order]
        self.weight = w[order]
        counts = np.bincount(v, minlength=n)
        starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
        self.has = counts > 0
        self.starts = starts[self.has]
        self.outdeg = np.diff(np.asarray(g.row_ptr, np.int64))

    def step(self, ell: np.ndarray) -> np.ndarray:
        """l_next(v) = min over arcs u -> v of ell(u) + w(u, v) (INF if none)."""
        nxt = np.full(self.n, INF, dtype=np.int64)
        if self.tail.size:
            cand = ell[self.tail] + self.weight
            nxt[self.has] = np.minimum.reduceat(cand, self.starts)
        return np.minimum(nxt, INF)

    def step_widest(self, ell: np.ndarray) -> np.ndarray:
        """b_next(v) = max over arcs u -> v of min(ell(u), w(u, v)) (0 if none)."""
        nxt = np.zeros(self.n, dtype=np.int64)
        if self.tail.size:
            cand = np.minimum(ell[self.tail], self.weight)
            nxt[self.has] = np.maximum.reduceat(cand, self.starts)
        return nxt

    def step_resist(self, ell: np.ndarray) -> np.ndarray:
        """r_next(v) = min over arcs u -> v of ell(u) + 1/w(u, v), in binary32
        (numpy's float32 division and addition round to nearest); inf if none."""
        nxt = np.full(self.n, np.inf, dtype=np.float32)
        if self.tail.size:
            recip = np.float32(1.0) / self.weight.astype(np.float32)
            cand = ell[self.tail] + recip
            nxt[self.has] = np.minimum.reduceat(cand, self.starts)
        return nxt


def forward_frontiers(g, s: int, max_products: int = 1 << 20, arcs: InArcs = None):
    """F_1, F_2, ... (bool[n] each, the last one empty) for source ``s``."""
    arcs = arcs or InArcs(g)
    ell = np.full(g.n, INF, dtype=np.int64)
    ell[s] = 0
    L = ell.copy()
    out = []
    for _ in range(max_products):
        nxt = arcs.step(ell)
        F = (nxt < INF) & (nxt <= L)
        out.append(F)
        L = np.minimum(L, nxt)
        ell = nxt
        if not F.any():
            return out
    raise RuntimeError("frontier did not empty")


def forward_relaxations(g, s: int, frontiers, arcs: InArcs = None) -> list:
    """Relaxations of products 1, 2, ...: out-degree sums over F_0 = {s}, F_1, ..."""
    outdeg = (arcs.outdeg if arcs is not None
              else np.diff(np.asarray(g.row_ptr, np.int64)))
    prev = [np.asarray([s])] + [np.flatnonzero(F) for F in frontiers[:-1]]
    return [int(outdeg[p].sum()) for p in prev]


def backward_heights(height_row: np.ndarray) -> list:
    """B_0, B_1, ... (bool[n] each) from one source's DAG heights (-1 = unreachable)."""
    h = np.asarray(height_row)
    top = int(h.max()) if h.size else -1
    return [h == k for k in range(top + 1)]


def backward_products(heights: np.ndarray, sources) -> int:
    """Backward products of a batch (counting product included) from its DAG heights."""
    h = np.array(heights, dtype=np.int64, copy=True)
    src = np.asarray(sources, dtype=np.int64)
    h[np.arange(src.size), src] = -1          # the source's own entry feeds no product
    top = int(h.max()) if h.size else -1
    return 1 if top < 0 else top + 2


WIDE_INF = np.int64(0x7FFFFFFF)   # the source's own (unbounded) width


def fixpoint(g, s: int, op: str = "sssp", max_products: int = 1 << 20, arcs: InArcs = None):
    """Relaxation to a fixpoint over strict-improvement frontiers.

    Section 3's product C = A (+).f B iterated as Algorithm 1 iterates it but
    without multiplicities, so an entry joins frontier j only when product j
    improves it.  With l_j(v) the best value of a walk from s to v with
    exactly j arcs and L_j the best over i <= j:

      "sssp"    (+) = min, f(a, w) = a + w; l_0(s) = 0, INF elsewhere
      "bfs"     the same with every weight 1 (hop counts)
      "widest"  (+) = max, f(a, w) = min(a, w); l_0(s) = WIDE_INF, 0 ("no
                walk") elsewhere: the bottleneck of the widest walk
      "resist"  (+) = min, f(a, w) = a + 1/w in binary32, l_0(s) = 0, inf
                elsewhere (binary32 addition of a positive term is monotone,
                so the best over walks is reached by the recurrence below)

    F_j = { v : l_j(v) strictly better than L_{j-1}(v) }.  Returns (L,
    products): the final values (int64; float32 for "resist") and the index
    of the first product whose frontier is empty.  After an empty F_j every
    later one is empty too (l_{j+1}(v) = best over u of f(l_j(u), w), and
    every l_j(u) is no better than L_{j-1}(u), whose images are already in
    L_j(v)).  ``arcs`` may pass g's InArcs (unit weights for "bfs") to reuse.
    """
    if op not in ("sssp", "bfs", "widest", "resist"):
        raise ValueError(op)
    arcs = arcs or InArcs(g, unit_weights=(op == "bfs"))
    if op == "widest":
        ell = np.zeros(g.n, dtype=np.int64)
        ell[s] = WIDE_INF
        step, better, best = arcs.step_widest, np.greater, np.maximum
    elif op == "resist":
        ell = np.full(g.n, np.inf, dtype=np.float32)
        ell[s] = 0.0
        step, better, best = arcs.step_resist, np.less, np.minimum
    else:
        ell = np.full(g.n, INF, dtype=np.int64)
        ell[s] = 0
        step, better, best = arcs.step, np.less, np.minimum
    L = ell.copy()
    for j in range(1, max_products + 1):
        nxt = step(ell)
        F = better(nxt, L)
        L = best(L, nxt)
        ell = nxt
        if not F.any():
            return L, j
    raise RuntimeError("fixpoint not reached")
