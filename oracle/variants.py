"""FP64 oracle, part 4: the variants of the prior (Sections 3, 4, 6 and 8.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy float64.

* f by distance transform (Section 6 names Gaussian smoothing or a distance transform
  as the image processing f that turns the previous segmentation into a grey image):
  f(A, x) = exp(-d(x)^2 / (2 sigma_d^2)) with d(x) the Euclidean distance from pixel x
  to the nearest object pixel of A (0 on the object; f = 0 everywhere when A holds no
  object pixel).  When no segmentation is supplied, the stand-in A = [pi_{t-1} > 1/2].
* The manual prior of Section 4 (used by the "Manual" baseline of Section 8.1 for the
  first frame): p(A_x = 1) = 1 where the user labelled x as object, eps where labelled
  background, 0.5 where no label is given; label codes 1, 0 and anything else.  It
  replaces pi_0 (variance P_0 = R); the border ring of the saliency-based prior is not
  applied to it.
* The stochastic saliency map of Section 3: a Kalman filter that takes the saliency
  map as its observation, each pixel a Gaussian N(mu_t, P_t).  Reading: a per-pixel
  scalar random-walk filter on S_t (level c_max) with process variance Q_s and
  observation variance R_s, mu_0 = S_0, P_0 = R_s, and the same gain recursion as the
  prior update; the observation q_t of the prior is then taken from mu_t instead of
  S_t.  The eye-focusing density (signal detection theory, the HMM of eye movements)
  stays out.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from .prior import border_mask, kalman_gains, observation
from .saliency import OracleParams, blur, geometry, saliency


def distance_sq(seg: np.ndarray) -> np.ndarray:
    """Squared Euclidean distance from every pixel to the nearest nonzero pixel of seg
    (brute force over all object pixels; +inf everywhere when there is none)."""
    seg = np.asarray(seg) != 0
    H, W = seg.shape
    oy, ox = np.nonzero(seg)
    out = np.full((H, W), np.inf)
    if oy.size == 0:
        return out
    ys = np.arange(H, dtype=np.float64)[:, None]
    xs = np.arange(W, dtype=np.float64)[None, :]
    for k in range(0, oy.size, 256):
        dy = ys[None, :, :] - oy[k:k + 256, None, None].astype(np.float64)
        dx = xs[None, :, :] - ox[k:k + 256, None, None].astype(np.float64)
        out = np.minimum(out, (dy * dy + dx * dx).min(axis=0))
    return out


def f_distance(seg: np.ndarray, sigma: float) -> np.ndarray:
    """f(A, x) = exp(-d(x)^2 / (2 sigma^2)); 0 where no object pixel exists."""
    d2 = distance_sq(seg)
    with np.errstate(over="ignore"):
        return np.where(np.isinf(d2), 0.0, np.exp(-d2 / (2.0 * sigma * sigma)))


def manual_prior(labels: np.ndarray, eps: float) -> np.ndarray:
    """p(A_x = 1) from manual labels: 1 -> 1, 0 -> eps, anything else -> 0.5."""
    lab = np.asarray(labels)
    return np.where(lab == 1, 1.0, np.where(lab == 0, eps, 0.5))


def stochastic_saliency(Ss: Sequence[np.ndarray], Qs: float, Rs: float):
    """Per-pixel Kalman filter of the saliency maps: returns (mu [T][Hc][Wc], P [T])."""
    T = len(Ss)
    K, P = kalman_gains(T, Qs, Rs)
    mus: List[np.ndarray] = []
    for t in range(T):
        S = np.asarray(Ss[t], dtype=np.float64)
        mus.append(S.copy() if t == 0 else mus[-1] + K[t] * (S - mus[-1]))
    return np.stack(mus), P


def prior_clip_variant(qs: Sequence[np.ndarray], p: OracleParams, f_mode: int = 0, dt_sigma: float = 2.0,
                       segs: Optional[Sequence[Optional[np.ndarray]]] = None,
                       pi0: Optional[np.ndarray] = None):
    """The prior recursion of Section 6 with the chosen f (0: binomial blur of the
    previous segmentation or prior; 1: distance transform) and optionally a manual
    first-frame prior pi0 (then q_0 is not used).  Returns (pis, fs, K)."""
    T = len(qs)
    H, W = qs[0].shape
    ring = border_mask(H, W, p.border)
    K, _ = kalman_gains(T, p.q, p.r)
    pis: List[np.ndarray] = []
    fs: List[Optional[np.ndarray]] = []
    for t in range(T):
        if t == 0:
            if pi0 is not None:
                pis.append(np.asarray(pi0, dtype=np.float64).copy())
                fs.append(None)
                continue
            pi = np.array(qs[0], dtype=np.float64)
            f = None
        else:
            seg = None if segs is None else segs[t]
            if f_mode == 0:
                src = pis[-1] if seg is None else np.asarray(seg, dtype=np.float64)
                f = blur(src)
            else:
                A = (pis[-1] > 0.5) if seg is None else (np.asarray(seg) != 0)
                f = f_distance(A, dt_sigma)
            pi = f + K[t] * (qs[t] - f)
        pi[ring] = p.eps
        pis.append(pi)
        fs.append(f)
    return pis, fs, K


def run_clip_variant(frames: np.ndarray, p: OracleParams, f_mode: int = 0, dt_sigma: float = 2.0,
                     ssm: Optional[tuple] = None, segs=None, manual: Optional[np.ndarray] = None):
    """Whole path over a clip with the variants: ssm = (Q_s, R_s) filters S before the
    observation; manual gives the labels of the first frame's prior."""
    T, H, W = frames.shape[:3]
    geo = geometry(H, W, p)
    Ss = [saliency(frames[t], frames[t - 1] if t else None, p)[0] for t in range(T)]
    obs = Ss
    mu, Pm = None, None
    if ssm is not None:
        # the stochastic map starts at the first saliency map it filters: frame 1 when the
        # first frame's prior comes from manual labels
        first = 0 if manual is None else 1
        mu, Pm = stochastic_saliency(Ss[first:], ssm[0], ssm[1])
        obs = list(Ss[:first]) + list(mu)
    qs = [observation(obs[t], p, H, W, geo.c_max)[0] for t in range(T)]
    pi0 = None if manual is None else manual_prior(manual, p.eps)
    pis, fs, K = prior_clip_variant(qs, p, f_mode, dt_sigma, segs, pi0)
    return {"S": np.stack(Ss), "mu": mu, "mu_var": Pm, "q": np.stack(qs), "pi": np.stack(pis), "f": fs,
            "K": K, "geometry": geo}
