"""FP64 oracle, part 2: saliency-based observation, Kalman prior update, MRF capacities.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy float64.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import numpy as np

from .saliency import OracleParams, blur, geometry, saliency, upsample


def border_mask(H: int, W: int, width: int) -> np.ndarray:
    """True on the ring of `width` pixels along the frame edge (reading R7)."""
    m = np.zeros((H, W), dtype=bool)
    if width > 0:
        m[:width, :] = True
        m[-width:, :] = True
        m[:, :width] = True
        m[:, -width:] = True
    return m


# -- O10: the saliency-based observation q_t (Section 5; readings R1, R7, R8, R18)
def observation(S: np.ndarray, p: OracleParams, H: int, W: int, c_max: int):
    """q = clamp(up_{c_max -> 0}(S / max S), eps, 1 - eps), with q = eps on the border
    ring (the prior at the frame edge is close to 0).  If max S <= flat_tol the map
    carries no information and q = 0.5 (the paper's "no label" prior) inside the frame.

    Returns (q, info) where info holds m = max S, the first row-major argmax, the
    unclamped upsampled map and the mask of pixels where the clamp is inactive."""
    m = float(S.max())
    xstar = int(np.argmax(S))
    ring = border_mask(H, W, p.border)
    if m <= p.flat_tol:
        q = np.full((H, W), 0.5)
        free = np.zeros((H, W), dtype=bool)
        u = None
    else:
        u = upsample(S / m, c_max, H, W)
        q = np.clip(u, p.eps, 1.0 - p.eps)
        free = (u > p.eps) & (u < 1.0 - p.eps)
    q[ring] = p.eps
    free &= ~ring
    return q, {"m": m, "xstar": xstar, "u": u, "free": free, "flat": m <= p.flat_tol}


# -- O11: the Kalman prior update (Section 6; readings R2-R6)
def kalman_gains(T: int, Q: float, R: float) -> Tuple[np.ndarray, np.ndarray]:
    """Scalar gain and variance sequences: K_0 = 1, P_0 = R; for t >= 1
    a = P_{t-1} + Q, K_t = a / (a + R), P_t = R * K_t.  With R = sigma_1^2 and
    Q = sigma_2^2 this is the paper's recursion: the weight of q is K_t and
    sigma_xi^2(t) = P_t."""
    K = np.zeros(T)
    P = np.zeros(T)
    for t in range(T):
        if t == 0:
            K[t], P[t] = 1.0, R
        else:
            a = P[t - 1] + Q
            K[t] = a / (a + R)
            P[t] = R * K[t]
    return K, P


def prior_clip(qs: Sequence[np.ndarray], p: OracleParams,
               segs: Optional[Sequence[Optional[np.ndarray]]] = None):
    """pi_0 = q_0; for t >= 1, f = G * pi_{t-1} (or G * seg_{t-1} when the previous
    segmentation is supplied), pi_t = f + K_t (q_t - f); pi_t = eps on the border ring.
    The variance is carried per pixel and checked to stay spatially uniform.

    Returns (pis, fs, K) with fs[0] = None."""
    T = len(qs)
    H, W = qs[0].shape
    ring = border_mask(H, W, p.border)
    pis: List[np.ndarray] = []
    fs: List[Optional[np.ndarray]] = []
    Kseq = np.zeros(T)
    P = None
    for t in range(T):
        q = qs[t]
        if t == 0:
            pi = q.copy()
            P = np.full((H, W), p.r)
            K = np.ones((H, W))
            fs.append(None)
        else:
            src = None if segs is None else segs[t]
            f = blur(pis[-1] if src is None else np.asarray(src, dtype=np.float64))
            a = P + p.q
            K = a / (a + p.r)
            pi = f + K * (q - f)
            P = p.r * K
            fs.append(f)
        if not np.all(P == P.flat[0]):
            raise AssertionError("Kalman variance lost spatial uniformity")
        Kseq[t] = K.flat[0]
        pi[ring] = p.eps
        pis.append(pi)
    return pis, fs, Kseq


# -- O12: MRF capacities (Section 4, Eqs. 1-4; readings R19-R21)
DIRECTIONS = ((0, 1), (1, 0), (1, 1), (1, -1))      # E, S, SE, SW as (dy, dx)


def mrf_weights(rgb: np.ndarray, prior: np.ndarray, p: OracleParams):
    """Unary costs by label, U1 = -ln max(pi, eps) and U0 = -ln(1 - min(pi, 1 - eps)),
    and one symmetric contrast-sensitive capacity per unordered 8-neighbour pair,
    w = potts + lam * exp(-beta ||C_x - C_y||^2) / ||x - y||, with C the RGB value and
    beta = 1 / (2 * mean ||dC||^2) over all in-frame pairs (0 if that mean is 0).
    pairwise[d][y][x] links (y, x) to (y + dy, x + dx) and is 0 when that is outside.

    Returns (unary [2][H][W], pairwise [4][H][W], beta)."""
    pi = np.asarray(prior, dtype=np.float64)
    U1 = -np.log(np.maximum(pi, p.eps))
    U0 = -np.log1p(-np.minimum(pi, 1.0 - p.eps))
    H, W = pi.shape
    C = rgb.astype(np.float64)
    total, count = 0.0, 0
    d2s = []
    for dy, dx in DIRECTIONS:
        d2 = np.zeros((H, W))
        valid = np.zeros((H, W), dtype=bool)
        for y in range(H):
            y2 = y + dy
            if not 0 <= y2 < H:
                continue
            for_x = np.arange(W)
            x2 = for_x + dx
            ok = (x2 >= 0) & (x2 < W)
            xs = for_x[ok]
            diff = C[y, xs] - C[y2, xs + dx]
            d2[y, xs] = (diff * diff).sum(axis=1)
            valid[y, xs] = True
        total += d2[valid].sum()
        count += int(valid.sum())
        d2s.append((d2, valid, float(np.hypot(dy, dx))))
    mean = total / count if count else 0.0
    beta = 1.0 / (2.0 * mean) if mean > 0 else 0.0
    pair = np.zeros((4, H, W))
    for d, (d2, valid, dist) in enumerate(d2s):
        pair[d] = np.where(valid, p.potts + p.lam * np.exp(-beta * d2) / dist, 0.0)
    return np.stack([U0, U1]), pair, beta


def run_clip(frames: np.ndarray, p: OracleParams, segs=None, with_mrf: bool = False):
    """Whole path over a clip: saliency, observation and Kalman update per frame.

    Returns dict with S [T][Hc][Wc], C [T][8][Hc][Wc], q, pi [T][H][W], K [T],
    obs info per frame and, with_mrf, unary/pairwise/beta per frame."""
    T, H, W = frames.shape[:3]
    geo = geometry(H, W, p)
    Ss, Cs, qs, infos = [], [], [], []
    for t in range(T):
        S, C = saliency(frames[t], frames[t - 1] if t > 0 else None, p)
        q, info = observation(S, p, H, W, geo.c_max)
        Ss.append(S)
        Cs.append(C)
        qs.append(q)
        infos.append(info)
    pis, fs, K = prior_clip(qs, p, segs)
    out = {"S": np.stack(Ss), "C": np.stack(Cs), "q": np.stack(qs), "pi": np.stack(pis),
           "f": fs, "K": K, "info": infos, "geometry": geo}
    if with_mrf:
        us, ps, bs = [], [], []
        for t in range(T):
            u, pw, b = mrf_weights(frames[t], pis[t], p)
            us.append(u)
            ps.append(pw)
            bs.append(b)
        out["unary"] = np.stack(us)
        out["pairwise"] = np.stack(ps)
        out["beta"] = np.array(bs)
    return out
