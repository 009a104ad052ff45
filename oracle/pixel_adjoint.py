"""FP64 oracle, part 7: the adjoint of the whole chain down to the frames' pixels.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy float64.

This extends the adjoint of the prior chain (adjoint.py, which stops at the saliency map)
through the saliency model of Section 3 / Section 7.2: the weighted sum, N(.), the
across-scale sum, centre-surround, the Gabor maps, the Gaussian pyramid and the level-0
features, to dL/d frame_t for every frame (the motion feature also reaches frame t-1).
Frames are treated as real-valued RGB on the 0..255 scale; the gradient is per unit of
that scale.  Conventions where the forward is not differentiable:

* the chromatic mask (an integer threshold) and the colour maximum are held fixed;
* N(.): the global minimum, the global maximum and each 8x8 block maximum pass their
  gradient to one position: the first in row-major order whose value lies within
  TIE = 2^-20 of the map's range of the extreme.  Maps fed to N(.) hold exact ties at their
  extrema wherever a centre-surround difference vanishes identically (a static background
  has zero motion over whole regions); there the loss has no unique gradient, and the
  tolerance makes the choice among the tied positions independent of rounding.  A map at
  or below flat_tol passes none (N = 0);
* |D| of a centre-surround difference D = X(c) - up X(s): its derivative is taken as 0
  wherever |D| <= SIGN_BAND = 2^-16 of the pair's scale (the largest |value| of X(c) and
  X(s)), and as sign(D) elsewhere.  D vanishes identically wherever both levels are flat
  (the motion map of a constant-colour object moving over a constant background is a
  plateau), and at the minimum of |D| over a large map it can lie below the rounding error
  of FP32 maps; in both cases FP32 cannot fix the sign, and 0 is the derivative a central
  difference sees at an exact zero.  sign_band = 0 gives the plain sign(D) with sign(0) = 0;
* |.| of the frame difference: sign(0) = 0; max(0, .) passes nothing at 0; min(r', g')
  passes to r' on ties;
* the branches of the features are decided on the frame values themselves, where they
  are exact (for 8-bit frames, integer comparisons): on a chromatic pixel R' = r' - (g' +
  b')/2 > 0 exactly when 2R - G - B > 0 (likewise for G and B), Y' > 0 when min(R, G) > B,
  the min takes r' when R <= G, and the motion's sign is that of (R+G+B)_t - (R+G+B)_{t-1}.
  Evaluating r' = R / I first would let rounding pick the branch wherever the exact value
  sits on the kink (2R = G + B holds for about one pixel in two hundred).
"""
from __future__ import annotations

from typing import Dict, List, Optional, Tuple

import numpy as np

from .adjoint import blur_adjoint, mse_mask_loss, prior_chain_backward, prior_chain_forward, upsample_adjoint
from .saliency import (CHANNELS, ORIENTATIONS_DEG, OracleParams, chromatic_mask, gabor_kernel, geometry,
                       saliency, upsample)


def reduce_adjoint(G: np.ndarray, Hf: int, Wf: int) -> np.ndarray:
    """Transpose of reduce_level from an Hf x Wf map: insert G at the even positions,
    then the transpose of the clamped blur."""
    Z = np.zeros((Hf, Wf))
    Z[::2, ::2] = G
    return blur_adjoint(Z)


def gabor_adjoint(G: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Transpose of the clamped correlation gabor(X, h): each tap sends its weighted
    output back to the clamped position it read."""
    H, W = G.shape
    r = h.shape[0] // 2
    ys, xs = np.arange(H), np.arange(W)
    out = np.zeros((H, W))
    for v in range(-r, r + 1):
        yy = np.clip(ys + v, 0, H - 1)
        for u in range(-r, r + 1):
            xx = np.clip(xs + u, 0, W - 1)
            np.add.at(out, np.ix_(yy, xx), h[v + r, u + r] * G)
    return out


TIE = 2.0 ** -20


def normalise_vjp(X: np.ndarray, gN: np.ndarray, flat_tol: float = 1e-5, block: int = 8) -> np.ndarray:
    """dL/dX given dL/dN(X), N(X) = Y (1 - mbar)^2, Y = (X - mn) / (mx - mn), mbar the mean
    of the block maxima of Y with one global maximum removed."""
    X = np.asarray(X, dtype=np.float64)
    mn, mx = float(X.min()), float(X.max())
    if mx - mn <= flat_tol:
        return np.zeros_like(X)
    rng = mx - mn
    Y = (X - mn) / rng
    H, W = Y.shape
    pos, bvals = [], []
    for by in range(0, H, block):
        for bx in range(0, W, block):
            blk = Y[by:by + block, bx:bx + block]
            bm = float(blk.max())
            k = int(np.argmax((blk >= bm - TIE).reshape(-1)))
            pos.append((by + k // blk.shape[1], bx + k % blk.shape[1]))
            bvals.append(bm)
    nb = len(bvals)
    mbar = (sum(bvals) - 1.0) / (nb - 1) if nb > 1 else 0.0
    A = (1.0 - mbar) ** 2
    gY = gN * A
    if nb > 1:
        gb = -2.0 * (1.0 - mbar) * float((gN * Y).sum()) / (nb - 1)
        for (y, x) in pos:
            gY[y, x] += gb
    gX = gY / rng
    gmn = float((gY * (Y - 1.0)).sum()) / rng
    gmx = -float((gY * Y).sum()) / rng
    gX.flat[int(np.argmax((Y <= TIE).reshape(-1)))] += gmn
    gX.flat[int(np.argmax((Y >= 1.0 - TIE).reshape(-1)))] += gmx
    return gX


def feature_vjp(rgb: np.ndarray, rgb_prev: Optional[np.ndarray], chrom: np.ndarray, gI: np.ndarray,
                gRG: np.ndarray, gBY: np.ndarray, gM: np.ndarray):
    """Level-0 features back to the frame (and, through motion, the previous frame)."""
    v = np.asarray(rgb, dtype=np.float64)
    R8, G8, B8 = v[..., 0], v[..., 1], v[..., 2]
    f = v / 255.0
    r, g, b = f[..., 0], f[..., 1], f[..., 2]
    inten = (r + g + b) / 3.0
    safe = np.where(chrom, inten, 1.0)
    # branches from the frame values (exact for 8-bit frames)
    aR = chrom & (2 * R8 - G8 - B8 > 0)
    aG = chrom & (2 * G8 - R8 - B8 > 0)
    aB = chrom & (2 * B8 - R8 - G8 > 0)
    aY = chrom & (np.minimum(R8, G8) - B8 > 0)
    rfirst = R8 <= G8
    gR, gG, gB, gYc = gRG, -gRG, gBY, -gBY
    guR = np.where(aR, gR, 0.0)
    guG = np.where(aG, gG, 0.0)
    guB = np.where(aB, gB, 0.0)
    guY = np.where(aY, gYc, 0.0)
    grp = guR - 0.5 * guG - 0.5 * guB
    ggp = -0.5 * guR + guG - 0.5 * guB
    gbp = -0.5 * guR - 0.5 * guG + guB - guY
    grp = grp + np.where(rfirst, guY, 0.0)
    ggp = ggp + np.where(rfirst, 0.0, guY)
    gIt = np.array(gI, dtype=np.float64)
    g_prev = None
    if rgb_prev is not None:
        vp = np.asarray(rgb_prev, dtype=np.float64)
        sg = np.sign((R8 + G8 + B8) - (vp[..., 0] + vp[..., 1] + vp[..., 2])) * gM
        gIt = gIt + sg
        g_prev = np.repeat((-sg / 3.0)[..., None], 3, axis=2) / 255.0
    # r' = r / I on chromatic pixels
    gr = np.where(chrom, grp / safe, 0.0)
    gg = np.where(chrom, ggp / safe, 0.0)
    gb = np.where(chrom, gbp / safe, 0.0)
    gIt = gIt - np.where(chrom, (grp * r + ggp * g + gbp * b) / (safe * safe), 0.0)
    gr, gg, gb = gr + gIt / 3.0, gg + gIt / 3.0, gb + gIt / 3.0
    return np.stack([gr, gg, gb], axis=2) / 255.0, g_prev


def _levels_to_frame(gX, geo, p: OracleParams, rgb, rgb_prev, chrom):
    """Gabor transposes into the intensity, pyramid-step transposes down to level 0, then
    the features back to the frame (gX is consumed)."""
    for th, name in zip(ORIENTATIONS_DEG, ("O0", "O45", "O90", "O135")):
        h = gabor_kernel(th, p.gabor_lambda, p.gabor_sigma, p.gabor_radius)
        for l in geo.used_levels:
            gX["I"][l] += gabor_adjoint(gX[name][l], h)
    for name in ("I", "RG", "BY", "M"):
        for l in range(geo.top, 0, -1):
            gX[name][l - 1] += reduce_adjoint(gX[name][l], *geo.sizes[l - 1])
    return feature_vjp(rgb, rgb_prev, chrom, gX["I"][0], gX["RG"][0], gX["BY"][0], gX["M"][0])


SIGN_BAND = 2.0 ** -16


def _extreme_positions(F: np.ndarray, p: OracleParams) -> List[int]:
    """Flat indices that take N(.)'s extreme terms: the minimum and each block maximum
    (tie-tolerant, as in normalise_vjp).  The maximum's position has |D| at its largest."""
    Y = (F - F.min()) / (F.max() - F.min())
    out = [int(np.argmax((Y <= TIE).reshape(-1)))]
    H, W = F.shape
    for by in range(0, H, p.block):
        for bx in range(0, W, p.block):
            blk = Y[by:by + p.block, bx:bx + p.block]
            k = int(np.argmax((blk >= blk.max() - TIE).reshape(-1)))
            out.append((by + k // blk.shape[1]) * W + bx + k % blk.shape[1])
    return sorted(set(out))


def saliency_vjp(rgb: np.ndarray, rgb_prev: Optional[np.ndarray], gS: np.ndarray, p: OracleParams,
                 chrom: np.ndarray, sign_band: float = SIGN_BAND, edge_terms: bool = False):
    """(dL/d rgb, dL/d rgb_prev or None) for dL/dS = gS, through Section 3's model.

    With edge_terms, also the terms an FP32 evaluation may place on the other side of the
    sign band: every position taking an extreme term of N(.) (a large gradient) whose |D|
    lies within a factor of two of the band's edge, as (label, kept, dL/d rgb part, dL/d
    rgb_prev part) of that position's contribution with its gradient kept (sign(D) gF);
    kept says whether this result includes it."""
    S, C, inter = saliency(rgb, rgb_prev, p, want_intermediate=True, chrom=chrom)
    geo = inter["geometry"]
    base, orient = inter["base"], inter["orient"]
    maps = {"I": base["I"], "RG": base["RG"], "BY": base["BY"], "M": base["M"],
            "O0": orient[0.0], "O45": orient[45.0], "O90": orient[90.0], "O135": orient[135.0]}
    zero = lambda: {k: {l: np.zeros(geo.sizes[l]) for l in range(geo.top + 1)} for k in CHANNELS}
    gX = zero()
    spikes = []
    w = np.asarray(p.weights, dtype=np.float64)
    for k, name in enumerate(CHANNELS):
        gFbar = normalise_vjp(inter["fbar"][name], w[k] * gS, p.flat_tol, p.block)
        for (c, s) in geo.pairs:
            g = gFbar
            for l in range(geo.c_max - 1, c - 1, -1):
                g = reduce_adjoint(g, *geo.sizes[l])
            F = inter["cs"][(name, c, s)]
            gF = normalise_vjp(F, g, p.flat_tol, p.block)
            D = maps[name][c] - upsample(maps[name][s], s - c, *geo.sizes[c])
            band = sign_band * max(float(np.abs(maps[name][c]).max()), float(np.abs(maps[name][s]).max()))
            gD = np.where(D > band, gF, np.where(D < -band, -gF, 0.0))
            gX[name][c] += gD
            gX[name][s] += upsample_adjoint(-gD, s - c, *geo.sizes[s])
            if edge_terms and band > 0 and F.max() - F.min() > p.flat_tol:
                W = F.shape[1]
                for a in _extreme_positions(F, p):
                    if 0.5 * band <= abs(D.flat[a]) <= 2.0 * band and gF.flat[a] != 0.0:
                        e = np.zeros(geo.sizes[c])
                        e.flat[a] = np.sign(D.flat[a]) * gF.flat[a]
                        spikes.append((f"{name} ({c},{s}) at {divmod(a, W)}", abs(D.flat[a]) > band, name, c, s, e))
    g, gp = _levels_to_frame(gX, geo, p, rgb, rgb_prev, chrom)
    if not edge_terms:
        return g, gp
    terms = []
    for label, kept, name, c, s, e in spikes:
        gx = zero()
        gx[name][c] += e
        gx[name][s] += upsample_adjoint(-e, s - c, *geo.sizes[s])
        terms.append((label, kept) + tuple(_levels_to_frame(gx, geo, p, rgb, rgb_prev, chrom)))
    return g, gp, terms


def clip_loss(frames: np.ndarray, masks: np.ndarray, p: OracleParams, chroms: List[np.ndarray]) -> float:
    """Masked-MSE loss of the prior over a clip of real-valued frames (fixed masks)."""
    T, H, W = frames.shape[:3]
    geo = geometry(H, W, p)
    C = np.stack([saliency(frames[t], frames[t - 1] if t else None, p, chrom=chroms[t])[1] for t in range(T)])
    tape = prior_chain_forward(C, p.weights, p.q, p.r, p, H, W, geo.c_max)
    return mse_mask_loss(np.stack(tape["pi"]), masks)[0]


def frame_gradients(frames: np.ndarray, masks: np.ndarray, p: OracleParams,
                    sign_band: float = SIGN_BAND, edge_terms: bool = False):
    """Loss and dL/d frames [T][H][W][3] of the masked-MSE prior loss (Section 6 prior with
    the stand-in f, frames on the 0..255 scale).  With edge_terms also the sign band's edge
    terms of every frame (see saliency_vjp), each as (frame, label, kept, contribution to
    dL/d frames [T][H][W][3])."""
    frames = np.asarray(frames)
    T, H, W = frames.shape[:3]
    geo = geometry(H, W, p)
    chroms = [chromatic_mask(frames[t]) for t in range(T)]
    C = np.stack([saliency(frames[t], frames[t - 1] if t else None, p, chrom=chroms[t])[1] for t in range(T)])
    tape = prior_chain_forward(C, p.weights, p.q, p.r, p, H, W, geo.c_max)
    loss, gpi = mse_mask_loss(np.stack(tape["pi"]), masks)
    _, _, _, gS = prior_chain_backward(tape, C, gpi, p, want_gS=True)
    grad = np.zeros(frames.shape, dtype=np.float64)
    edges = []
    for t in range(T):
        res = saliency_vjp(frames[t], frames[t - 1] if t else None, gS[t], p, chroms[t], sign_band, edge_terms)
        grad[t] += res[0]
        if res[1] is not None:
            grad[t - 1] += res[1]
        for label, kept, dg, dgp in (res[2] if edge_terms else ()):
            full = np.zeros(frames.shape, dtype=np.float64)
            full[t] = dg
            if dgp is not None:
                full[t - 1] = dgp
            edges.append((t, label, kept, full))
    if edge_terms:
        return loss, grad, edges
    return loss, grad
