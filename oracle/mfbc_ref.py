"""Algorithms 1-3 (MFBF, MFBr, MFBC) written out plainly -- test infrastructure only.

A slow, dense, numpy transcription of the method's *steps* (Section 4), used
to pin what the GPU path must produce at every iteration: the frontier sets
of each product, the product counts, and the final T, Z and lambda.  Nothing
is blocked, fused or reordered beyond the algorithms themselves.

Notation (Section 4): a batch of n_b sources; matrices are stored [n_b][n]
(row s = source column s of the paper's n x n_b matrices).  A multpath is
(w, m); a centpath is (w, p, c).  An absent entry of a sparse matrix is the
identity of its monoid: (INF, 0) for multpaths (the min-monoid), "no entry"
for centpaths (the max-monoid, identity (-INF, 0, 0)).

Readings of the paper's text that this module takes (each is argued where
the deviation from the literal text matters):
  * T(s, s) = (0, 1) and the first frontier is {s} carrying (0, 1): the
    literal initialisation (A(s, v), 1) would give the source a cycle weight
    and count spurious successors in MFBr.  The products are therefore
    numbered j = 1, 2, ... with F_0 = {s}.
  * A multpath with weight INF is absent (multiplicity 0), so unreachable
    vertices never enter a frontier and the loop terminates.
  * A frontier carries the multiplicity of the product (the newly found
    paths), not the accumulated T; ties with T are kept.
  * MFBr's counter starts at the number of successors (the initial centpath
    used to count carries c = 1 per successor; Z's own entry starts at
    c = 0), so leaves start the first backward frontier.
  * Unreachable vertices take no part in MFBr.
  * lambda excludes the source's own term (sigma(s, t, s) = 0 in the
    definition of Section 2.4).
"""
from __future__ import annotations

import numpy as np

INF = np.int64(1) << 60


def _arcs(g):
    """Arc list (u -> v, weight) of graph g (out-arcs of the CSR rows)."""
    u = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    v = g.col.astype(np.int64)
    w = np.ones(u.size, np.int64) if g.w is None else g.w.astype(np.int64)
    return u, v, w


def _multpath_product(Fw, Fm, u, v, w, n):
    """G = F (+,f) A over the multpath monoid (Section 4.1).

    G(s, y) = sum-over-monoid of f(F(s, x), A(x, y)) with f(a, w) = (a.w + w, a.m);
    the monoid keeps the least weight and adds the multiplicities of ties.
    Layout [n_b][n]; returns (Gw, Gm).
    """
    nb = Fw.shape[0]
    src_w = Fw[:, u]                                    # [nb][arcs]
    present = src_w < INF
    cand_w = np.where(present, src_w + w[None, :], INF)
    cand_m = np.where(present, Fm[:, u], 0.0)
    GwT = np.full((n, nb), INF, dtype=np.int64)
    np.minimum.at(GwT, v, cand_w.T)
    Gw = GwT.T.copy()
    tie = present & (cand_w == Gw[:, v])
    GmT = np.zeros((n, nb), dtype=np.float64)
    np.add.at(GmT, v, np.where(tie, cand_m, 0.0).T)
    Gm = GmT.T.copy()
    Gm[Gw >= INF] = 0.0
    return Gw, Gm


def _multpath_accumulate(Tw, Tm, Gw, Gm):
    """T := T (+) G elementwise with the multpath monoid."""
    less = Gw < Tw
    tie = (Gw == Tw) & (Gw < INF)
    Tm2 = np.where(less, Gm, np.where(tie, Tm + Gm, Tm))
    Tw2 = np.minimum(Tw, Gw)
    return Tw2, Tm2


def mfbf(g, sources, trace: bool = True):
    """Algorithm 1 (MFBF) for the listed sources.

    Returns dict: dist int64[nb][n] (-1 = unreachable), sigma float64[nb][n],
    products (number of products performed, the last one yielding an empty
    frontier), and if ``trace`` a list ``frontiers`` of bool[nb][n], one per
    product j = 1..products (membership of F_j).
    """
    n = g.n
    src = np.asarray(sources, dtype=np.int64)
    nb = src.size
    u, v, w = _arcs(g)
    Tw = np.full((nb, n), INF, dtype=np.int64)
    Tm = np.zeros((nb, n), dtype=np.float64)
    Tw[np.arange(nb), src] = 0
    Tm[np.arange(nb), src] = 1.0
    Fw, Fm = Tw.copy(), Tm.copy()          # first frontier: the sources themselves
    frontiers = []
    products = 0
    while (Fw < INF).any():
        Gw, Gm = _multpath_product(Fw, Fm, u, v, w, n)
        products += 1
        Tw, Tm = _multpath_accumulate(Tw, Tm, Gw, Gm)
        # new frontier: entries of G that are present and not heavier than T
        keep = (Gm != 0) & (Gw < INF) & ~(Gw > Tw)
        Fw = np.where(keep, Gw, INF)
        Fm = np.where(keep, Gm, 0.0)
        if trace:
            frontiers.append(keep.copy())
    dist = np.where(Tw < INF, Tw, -1)
    out = {"dist": dist, "sigma": Tm, "products": products}
    if trace:
        out["frontiers"] = frontiers
    return out


def _centpath_product(Bw, Bp, Bc, u, v, w, n, nb):
    """C = B (x,g) A^T over the centpath monoid (Section 4.2).

    C(s, x) = max-monoid over arcs x -> y of g(B(s, y), A(x, y)) with
    g(a, w) = (a.w - w, a.p, a.c); the monoid keeps the greatest weight and
    adds p and c of ties.  Absent entries (Bw = -INF) contribute nothing.
    """
    # arc x -> y in the CSR: u = x (output row), v = y (frontier vertex)
    src_w = Bw[:, v]
    present = src_w > -INF
    cand_w = np.where(present, src_w - w[None, :], -INF)
    CwT = np.full((n, nb), -INF, dtype=np.int64)
    np.maximum.at(CwT, u, cand_w.T)
    Cw = CwT.T.copy()
    tie = present & (cand_w == Cw[:, u])
    CpT = np.zeros((n, nb))
    CcT = np.zeros((n, nb), dtype=np.int64)
    np.add.at(CpT, u, np.where(tie, Bp[:, v], 0.0).T)
    np.add.at(CcT, u, np.where(tie, Bc[:, v], 0).T)
    return Cw, CpT.T.copy(), CcT.T.copy()


def _centpath_accumulate(Zw, Zp, Zc, Cw, Cp, Cc):
    """Z := Z (x) C elementwise with the centpath (max) monoid."""
    more = Cw > Zw
    tie = (Cw == Zw) & (Cw > -INF)
    Zp2 = np.where(more, Cp, np.where(tie, Zp + Cp, Zp))
    Zc2 = np.where(more, Cc, np.where(tie, Zc + Cc, Zc))
    return np.maximum(Zw, Cw), Zp2, Zc2


def mfbr(g, sources, dist, sigma, trace: bool = True):
    """Algorithm 2 (MFBr) from MFBF's output (dist, sigma).

    Returns dict: zeta float64[nb][n] (0 where unreachable), products (count
    of backward products including the counting product), and if ``trace``
    ``step`` int32[nb][n]: the index k of the backward frontier B_k that
    (s, v) entered (k = 0 for the leaves found by the counting product),
    -1 for unreachable entries.
    """
    n = g.n
    src = np.asarray(sources, dtype=np.int64)
    nb = src.size
    u, v, w = _arcs(g)
    reach = dist >= 0
    tau = np.where(reach, dist, -INF).astype(np.int64)
    # counting product: every reachable entry is present with (tau, 0, 1)
    Bw = tau.copy()
    Bp = np.zeros((nb, n))
    Bc = np.where(reach, 1, 0).astype(np.int64)
    Cw, Cp, Cc = _centpath_product(Bw, Bp, Bc, u, v, w, n, nb)
    products = 1
    Zw, Zp, Zc = tau.copy(), np.zeros((nb, n)), np.zeros((nb, n), np.int64)
    Zw, Zp, Zc = _centpath_accumulate(Zw, Zp, Zc, Cw, Cp, Cc)
    step = np.full((nb, n), -1, dtype=np.int32)
    inv_sigma = np.where(reach, 1.0 / np.where(reach, sigma, 1.0), 0.0)
    # first frontier: the leaves (counter 0)
    front = reach & (Zc == 0)
    step[front] = 0
    Bw = np.where(front, tau, -INF)
    Bp = np.where(front, inv_sigma, 0.0)
    Bc = np.where(front, -1, 0).astype(np.int64)
    k = 0
    while front.any():
        Cw, Cp, Cc = _centpath_product(Bw, Bp, Bc, u, v, w, n, nb)
        products += 1
        Zc = np.where(reach & (Zc == 0), -1, Zc)      # turn off counters already used
        Zw, Zp, Zc = _centpath_accumulate(Zw, Zp, Zc, Cw, Cp, Cc)
        k += 1
        front = reach & (Zc == 0)
        step[front] = k
        Bw = np.where(front, tau, -INF)
        Bp = np.where(front, Zp + inv_sigma, 0.0)
        Bc = np.where(front, -1, 0).astype(np.int64)
    zeta = np.where(reach, Zp, 0.0)
    out = {"zeta": zeta, "products": products}
    if trace:
        out["step"] = step
    return out


def mfbc(g, sources, batch: int):
    """Algorithm 3 (MFBC): lambda over ``sources`` in batches of ``batch``.

    lambda(v) += zeta(s, v) * sigma(s, v) for every source s of every batch,
    except the source's own term (v = s).  A ragged last batch is allowed.
    """
    src = np.asarray(sources, dtype=np.int64)
    lam = np.zeros(g.n)
    for b0 in range(0, src.size, batch):
        bs = src[b0:b0 + batch]
        f = mfbf(g, bs, trace=False)
        r = mfbr(g, bs, f["dist"], f["sigma"], trace=False)
        dep = r["zeta"] * f["sigma"]
        dep[np.arange(bs.size), bs] = 0.0
        lam += dep.sum(axis=0)
    return lam
