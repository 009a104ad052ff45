"""Oracle, part 6: the minimum cut that turns the MRF capacities into a segmentation
(Section 4), closing the loop of Section 6 (the previous segmentation feeds f).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Integer arithmetic.

Section 4: the MAP labelling of the MRF is the minimum s-t cut of a graph with one
vertex per pixel, t-links from the source and to the sink weighted by the first
likelihood and prior terms, and a pair of directed n-links of equal weight between
8-neighbours.  Readings taken here:

* the source side is the object (label 1): a pixel left on the sink side pays its
  label-0 cost c(s, v) = U0, a pixel on the source side pays c(v, t) = U1, and each
  8-neighbour pair with different labels pays its pairwise capacity once (both directed
  n-links carry it);
* capacities are integers: q(c) = rint(float32(c) * float32(scale)) (round half to
  even, in FP32), clamped to [0, 2^24], so that the flow value is exact;
* among the minimum cuts the labelling is the one with the largest object: a pixel is
  background exactly when it can still reach the sink in the residual graph of a
  maximum flow (that set is the same for every maximum flow).
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

CAP_MAX = 1 << 24
# n-link directions as (dy, dx) with the pairwise plane that holds each one's capacity
# at its upper-left end: E, S, SE at the pixel itself, SW at the pixel itself.
DIRS = ((0, 1), (1, 0), (1, 1), (1, -1))


def quantise(x: np.ndarray, scale: float) -> np.ndarray:
    """Integer capacities: FP32 product, rounded half to even, clamped to [0, 2^24]."""
    v = np.rint(np.asarray(x, dtype=np.float32) * np.float32(scale)).astype(np.float64)
    return np.clip(v, 0, CAP_MAX).astype(np.int64)


def edges(H: int, W: int, pw: np.ndarray):
    """(u, v, w) for every in-frame 8-neighbour pair, u the pixel holding the capacity."""
    us, vs, ws = [], [], []
    for d, (dy, dx) in enumerate(DIRS):
        for y in range(H):
            y2 = y + dy
            if not 0 <= y2 < H:
                continue
            xs = np.arange(W)
            x2 = xs + dx
            ok = (x2 >= 0) & (x2 < W)
            us.append(y * W + xs[ok])
            vs.append(y2 * W + x2[ok])
            ws.append(pw[d, y, xs[ok]])
    if not us:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(us), np.concatenate(vs), np.concatenate(ws).astype(np.int64)


def energy(labels: np.ndarray, cs: np.ndarray, ct: np.ndarray, pw: np.ndarray) -> int:
    """Cost of a labelling: U0 of background pixels, U1 of object pixels, the pairwise
    capacity of every pair with different labels (integers)."""
    H, W = labels.shape
    lab = labels.reshape(-1).astype(bool)
    e = int(cs.reshape(-1)[~lab].sum()) + int(ct.reshape(-1)[lab].sum())
    u, v, w = edges(H, W, pw)
    return e + int(w[lab[u] != lab[v]].sum())


def min_cut(cs: np.ndarray, ct: np.ndarray, pw: np.ndarray) -> Tuple[int, np.ndarray]:
    """Maximum flow value and the labelling with the largest object among the minimum
    cuts.  cs, ct: [H][W] integer t-link capacities (source->pixel = U0, pixel->sink =
    U1); pw: [4][H][W] integer n-link capacities (E, S, SE, SW)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import maximum_flow
    H, W = cs.shape
    N = H * W
    s, t = N, N + 1
    u, v, w = edges(H, W, pw)
    pix = np.arange(N)
    rows = np.concatenate([np.full(N, s), pix, u, v])
    cols = np.concatenate([pix, np.full(N, t), v, u])
    caps = np.concatenate([cs.reshape(-1), ct.reshape(-1), w, w]).astype(np.int64)
    keep = caps > 0
    rows, cols, caps = rows[keep], cols[keep], caps[keep]
    if caps.size and caps.max() > np.iinfo(np.int32).max:
        raise ValueError("capacity exceeds int32")
    G = csr_matrix((caps.astype(np.int32), (rows, cols)), shape=(N + 2, N + 2))
    G.sum_duplicates()
    res = maximum_flow(G, s, t, method="dinic")
    # residual capacity of u -> v: cap(u, v) - flow(u, v), the flow being skew-symmetric;
    # the vertices that reach t in the residual graph are those t reaches in its transpose
    from scipy.sparse.csgraph import breadth_first_order
    R = (G.astype(np.int64) - res.flow.astype(np.int64)).tocsr()
    R.data = (R.data > 0).astype(np.int8)
    R.eliminate_zeros()
    order = breadth_first_order(R.T.tocsr(), t, directed=True, return_predecessors=False)
    reach = np.zeros(N + 2, dtype=bool)
    reach[order] = True
    labels = (~reach[:N]).reshape(H, W).astype(np.uint8)
    return int(res.flow_value), labels


def min_cut_brute(cs: np.ndarray, ct: np.ndarray, pw: np.ndarray) -> Tuple[int, np.ndarray]:
    """Every labelling of a tiny grid: the minimum energy and the union of the objects of
    all minimisers."""
    H, W = cs.shape
    N = H * W
    best, union = None, np.zeros(N, dtype=bool)
    for k in range(1 << N):
        lab = np.array([(k >> i) & 1 for i in range(N)], dtype=np.uint8).reshape(H, W)
        e = energy(lab, cs, ct, pw)
        if best is None or e < best:
            best, union = e, lab.reshape(-1).astype(bool).copy()
        elif e == best:
            union |= lab.reshape(-1).astype(bool)
    return best, union.reshape(H, W).astype(np.uint8)


def segment(unary: np.ndarray, pairwise: np.ndarray, scale: float) -> Tuple[int, np.ndarray]:
    """The cut of float capacities: U0, U1 = unary[0], unary[1]; pairwise [4][H][W]."""
    return min_cut(quantise(unary[0], scale), quantise(unary[1], scale), quantise(pairwise, scale))
