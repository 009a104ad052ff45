"""FP64 oracle, part 1: the Itti-style saliency map.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy float64.

The paper computes the saliency map of each frame with Itti's model, using
intensity, colour-opponent, orientation and motion features (Section 3); on the GPU
it splits the work into pixel-wise feature extraction, Gaussian pyramids, a
normalisation built on global and local extrema, and a weighted addition of maps
(Section 7.2).  The paper gives no further formulas for these steps, so the
definitions below are the readings recorded with the design notes; each function
names the reading it implements.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

CHANNELS = ("I", "RG", "BY", "O0", "O45", "O90", "O135", "M")
ORIENTATIONS_DEG = (0.0, 45.0, 90.0, 135.0)
# 5-tap binomial low-pass used for every pyramid step and for f = G * pi (reading R11).
BINOMIAL5 = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0


@dataclasses.dataclass
class OracleParams:
    depth: Optional[int] = None                 # None -> floor(log2 min(H, W)) - 1
    centers: Tuple[int, ...] = (1, 2)
    deltas: Tuple[int, ...] = (2, 3)
    weights: Tuple[float, ...] = (1.0,) * 8     # channel order CHANNELS
    q: float = 1e-3                              # Kalman process variance Q (= sigma_2^2)
    r: float = 1e-1                              # Kalman observation variance R (= sigma_1^2)
    eps: float = 1e-4
    border: int = 1
    lam: float = 1.0                             # contrast weight of the pairwise term
    potts: float = 0.0                           # constant of the Potts prior xi_2
    block: int = 8                               # block size of the local maxima in N(.)
    flat_tol: float = 1e-5
    gabor_lambda: float = 4.0
    gabor_sigma: float = 2.0
    gabor_radius: int = 6


@dataclasses.dataclass
class Geometry:
    H: int
    W: int
    depth: int
    pairs: List[Tuple[int, int]]       # (c, s) centre-surround pairs with s <= depth
    sizes: List[Tuple[int, int]]       # level l -> (H_l, W_l), l = 0..depth
    c_min: int
    c_max: int
    top: int                           # deepest level any pair uses

    @property
    def used_levels(self) -> List[int]:
        return sorted({c for c, _ in self.pairs} | {s for _, s in self.pairs})


def geometry(H: int, W: int, p: OracleParams) -> Geometry:
    """Pyramid depth and centre-surround pairs (readings R12, R28): default depth
    floor(log2 min(H, W)) - 1; pairs (c, c + delta) whose surround level exceeds the
    depth are dropped; level sizes halve with ceil."""
    if H < 1 or W < 1:
        raise ValueError("empty frame")
    depth = p.depth if p.depth is not None else int(math.floor(math.log2(min(H, W)))) - 1
    pairs = [(c, c + d) for c in p.centers for d in p.deltas if c + d <= depth]
    if not pairs:
        raise ValueError("no centre-surround pair fits the pyramid depth")
    sizes = [(H, W)]
    for _ in range(depth):
        h, w = sizes[-1]
        sizes.append(((h + 1) // 2, (w + 1) // 2))
    c_min = min(c for c, _ in pairs)
    c_max = max(c for c, _ in pairs)
    top = max(s for _, s in pairs)
    return Geometry(H, W, depth, pairs, sizes, c_min, c_max, top)


# -- O1/O2: features (Section 3, Section 7.2 "pixel-wise computation"; readings R9, R10, R26)
def colour_max(rgb: np.ndarray) -> int:
    """Largest R8+G8+B8 over the frame, as an integer."""
    return int(rgb.astype(np.int64).sum(axis=2).max())


def features(rgb: np.ndarray, rgb_prev: Optional[np.ndarray], smax: int,
             chrom: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """Level-0 intensity, red-green and blue-yellow opponents, and frame-difference motion.

    I = (r+g+b)/3 with r, g, b in [0, 1].  Colours are normalised by I only where the
    pixel is bright enough: 10*(R8+G8+B8) > max over the frame (an integer test);
    elsewhere r' = g' = b' = 0.  Broadly tuned channels R, G, B, Y are clamped at 0
    and combined into RG = R - G and BY = B - Y.  Motion is |I_t - I_{t-1}| (0 for the
    first frame).  A given chrom mask replaces the threshold test (an integer decision,
    constant under small changes of real-valued frames)."""
    f = rgb.astype(np.float64) / 255.0
    r, g, b = f[..., 0], f[..., 1], f[..., 2]
    # I = (r + g + b) / 3 evaluated as (R8 + G8 + B8) / 765: one rounding of the byte sum,
    # so pixels with equal sums get bitwise equal intensities (and equal frames zero motion)
    s8f = rgb.astype(np.float64).sum(axis=2)
    inten = s8f / 765.0
    if chrom is None:
        s8 = rgb.astype(np.int64).sum(axis=2)
        chrom = 10 * s8 > smax
    safe = np.where(chrom, inten, 1.0)
    rp = np.where(chrom, r / safe, 0.0)
    gp = np.where(chrom, g / safe, 0.0)
    bp = np.where(chrom, b / safe, 0.0)
    R = np.maximum(0.0, rp - (gp + bp) / 2.0)
    G = np.maximum(0.0, gp - (rp + bp) / 2.0)
    B = np.maximum(0.0, bp - (rp + gp) / 2.0)
    Y = np.maximum(0.0, np.minimum(rp, gp) - bp)
    if rgb_prev is None:
        M = np.zeros_like(inten)
    else:
        M = np.abs(s8f - rgb_prev.astype(np.float64).sum(axis=2)) / 765.0
    return {"I": inten, "RG": R - G, "BY": B - Y, "M": M}


# -- O3: Gaussian pyramid (Section 7.2, filter convolution formula; reading R11)
def blur(X: np.ndarray) -> np.ndarray:
    """G * X: the 5x5 binomial (outer product of (1,4,6,4,1)/16) with clamp-to-edge."""
    H, W = X.shape
    ys, xs = np.arange(H), np.arange(W)
    out = np.zeros_like(X, dtype=np.float64)
    for i in range(-2, 3):
        yy = np.clip(ys + i, 0, H - 1)
        for j in range(-2, 3):
            xx = np.clip(xs + j, 0, W - 1)
            out += BINOMIAL5[i + 2] * BINOMIAL5[j + 2] * X[np.ix_(yy, xx)]
    return out


def reduce_level(X: np.ndarray) -> np.ndarray:
    """One pyramid step: blur, then keep even rows and columns (size ceil(n/2))."""
    return blur(X)[::2, ::2]


def pyramid(X: np.ndarray, top: int) -> List[np.ndarray]:
    levels = [np.asarray(X, dtype=np.float64)]
    for _ in range(top):
        levels.append(reduce_level(levels[-1]))
    return levels


# -- O4: Gabor orientation features (Section 3 "orientation", Section 7.2; reading R15)
def gabor_kernel(theta_deg: float, lam: float = 4.0, sigma: float = 2.0, radius: int = 6) -> np.ndarray:
    """h[v][u] = e(u,v)*cos(2 pi (u cos t + v sin t)/lam) - c*e(u,v), e = exp(-(u^2+v^2)/(2 sigma^2)),
    c chosen so the taps sum to zero; u is the column offset (x, right), v the row
    offset (y, down); even (cosine) phase."""
    u = np.arange(-radius, radius + 1, dtype=np.float64)
    U, V = np.meshgrid(u, u)              # U varies along columns, V along rows
    t = math.radians(theta_deg)
    e = np.exp(-(U * U + V * V) / (2.0 * sigma * sigma))
    carrier = np.cos(2.0 * math.pi * (U * math.cos(t) + V * math.sin(t)) / lam)
    c = (e * carrier).sum() / e.sum()
    return e * carrier - c * e


def gabor(X: np.ndarray, h: np.ndarray) -> np.ndarray:
    """out[y][x] = sum_{u,v} h[v][u] * X[clamp(y+v)][clamp(x+u)] (direct 2-D sum)."""
    H, W = X.shape
    r = h.shape[0] // 2
    ys, xs = np.arange(H), np.arange(W)
    out = np.zeros_like(X, dtype=np.float64)
    for v in range(-r, r + 1):
        yy = np.clip(ys + v, 0, H - 1)
        for u in range(-r, r + 1):
            xx = np.clip(xs + u, 0, W - 1)
            out += h[v + r, u + r] * X[np.ix_(yy, xx)]
    return out


# -- O5/O6: cross-scale centre-surround (Section 3; readings R9b, R13)
def upsample(X: np.ndarray, d: int, Ht: int, Wt: int) -> np.ndarray:
    """Bilinear sample of X at (y / 2^d, x / 2^d) for the Ht x Wt target grid;
    coordinates clamped to the source, second tap min(i0 + 1, size - 1)."""
    Hs, Ws = X.shape
    scale = float(2 ** d)
    fy = np.clip(np.arange(Ht, dtype=np.float64) / scale, 0.0, Hs - 1.0)
    fx = np.clip(np.arange(Wt, dtype=np.float64) / scale, 0.0, Ws - 1.0)
    y0 = np.floor(fy).astype(np.int64)
    x0 = np.floor(fx).astype(np.int64)
    y1 = np.minimum(y0 + 1, Hs - 1)
    x1 = np.minimum(x0 + 1, Ws - 1)
    wy = (fy - y0)[:, None]
    wx = (fx - x0)[None, :]
    top = (1.0 - wx) * X[np.ix_(y0, x0)] + wx * X[np.ix_(y0, x1)]
    bot = (1.0 - wx) * X[np.ix_(y1, x0)] + wx * X[np.ix_(y1, x1)]
    return (1.0 - wy) * top + wy * bot


def centre_surround(Xc: np.ndarray, Xs: np.ndarray, d: int) -> np.ndarray:
    """F(c, s) = |X(c) - up_{s->c} X(s)| (the same minus form for every channel)."""
    return np.abs(Xc - upsample(Xs, d, Xc.shape[0], Xc.shape[1]))


# -- O7: N(.) (Section 7.2 "normalization function utilizing the global and local
#    extrema", block extrema as in the min/max search listing; readings R16, R16b)
def normalise(X: np.ndarray, flat_tol: float = 1e-5, block: int = 8) -> np.ndarray:
    """Rescale to [0, 1] by the global min and max, then weight by (1 - mbar)^2 where
    mbar is the mean of the block maxima (block x block tiles from (0, 0), partial at
    the edges) with one instance of the global maximum removed.  A map whose range is
    at most flat_tol is returned as zeros."""
    X = np.asarray(X, dtype=np.float64)
    mn, mx = float(X.min()), float(X.max())
    if mx - mn <= flat_tol:
        return np.zeros_like(X)
    Y = (X - mn) / (mx - mn)
    H, W = Y.shape
    bmax = []
    for by in range(0, H, block):
        for bx in range(0, W, block):
            bmax.append(float(Y[by:by + block, bx:bx + block].max()))
    nb = len(bmax)
    mbar = (sum(bmax) - 1.0) / (nb - 1) if nb > 1 else 0.0
    return Y * (1.0 - mbar) ** 2


# -- O8/O9: across-scale sum, conspicuity, saliency (Section 7.2 "weighted addition")
def chromatic_mask(rgb: np.ndarray) -> np.ndarray:
    """The pixels bright enough for colour normalisation: 10 (R8+G8+B8) > max (R8+G8+B8)."""
    s8 = np.asarray(rgb).astype(np.int64).sum(axis=2)
    return 10 * s8 > int(s8.max())


def saliency(rgb: np.ndarray, rgb_prev: Optional[np.ndarray], p: OracleParams,
             want_intermediate: bool = False, chrom: Optional[np.ndarray] = None):
    """Saliency map S (at level c_max) and the conspicuity maps C_k of one frame.

    Returns (S, C) with C of shape [8][H_cmax][W_cmax] in CHANNELS order; with
    want_intermediate also a dict of every stage (for stage-isolated parity)."""
    H, W = rgb.shape[:2]
    geo = geometry(H, W, p)
    smax = colour_max(rgb) if chrom is None else -1
    feats = features(rgb, rgb_prev, smax, chrom)
    base = {k: pyramid(feats[k], geo.top) for k in ("I", "RG", "BY", "M")}
    used = geo.used_levels
    orient = {}
    for th in ORIENTATIONS_DEG:
        h = gabor_kernel(th, p.gabor_lambda, p.gabor_sigma, p.gabor_radius)
        orient[th] = {l: gabor(base["I"][l], h) for l in used}
    level_maps = {
        "I": base["I"], "RG": base["RG"], "BY": base["BY"], "M": base["M"],
        "O0": orient[0.0], "O45": orient[45.0], "O90": orient[90.0], "O135": orient[135.0],
    }
    Hc, Wc = geo.sizes[geo.c_max]
    C = np.zeros((8, Hc, Wc))
    cs_maps: Dict[Tuple[str, int, int], np.ndarray] = {}
    fbar_maps: Dict[str, np.ndarray] = {}
    for k, name in enumerate(CHANNELS):
        fbar = np.zeros((Hc, Wc))
        for (c, s) in geo.pairs:
            F = centre_surround(level_maps[name][c], level_maps[name][s], s - c)
            cs_maps[(name, c, s)] = F
            Nf = normalise(F, p.flat_tol, p.block)
            for _ in range(geo.c_max - c):
                Nf = reduce_level(Nf)
            fbar += Nf
        fbar_maps[name] = fbar
        C[k] = normalise(fbar, p.flat_tol, p.block)
    w = np.asarray(p.weights, dtype=np.float64)
    S = np.tensordot(w, C, axes=1)
    if not want_intermediate:
        return S, C
    inter = {"geometry": geo, "smax": smax, "features": feats, "base": base,
             "orient": orient, "cs": cs_maps, "fbar": fbar_maps}
    return S, C, inter
