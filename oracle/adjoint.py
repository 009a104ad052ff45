"""FP64 oracle, part 3: adjoint of the prior chain and central finite differences.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy float64.

The differentiable parameters are the eight channel weights w of the saliency sum,
and the Kalman variances Q and R of the prior update (Section 6).  The conspicuity
maps C_k do not depend on them, so the chain is

    S_t = sum_k w_k C_{k,t}  ->  q_t = clamp(up(S_t / max S_t))  ->  pi_t (Kalman)  ->  loss.

Loss used for fitting (reading R22): L = mean over t, x of (pi_t - mask_t)^2.
"""
from __future__ import annotations

from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from .prior import border_mask, kalman_gains, observation
from .saliency import BINOMIAL5, OracleParams, blur


def mse_mask_loss(pis: np.ndarray, masks: np.ndarray) -> Tuple[float, np.ndarray]:
    """L = mean (pi - mask)^2 and dL/dpi."""
    pis = np.asarray(pis, dtype=np.float64)
    d = pis - masks.astype(np.float64)
    return float((d * d).mean()), 2.0 * d / d.size


def blur_adjoint(V: np.ndarray) -> np.ndarray:
    """G^T V for the clamp-to-edge blur: every tap of the forward sum sends its
    weighted input back to the clamped position it read from."""
    H, W = V.shape
    out = np.zeros_like(V, dtype=np.float64)
    ys, xs = np.arange(H), np.arange(W)
    for i in range(-2, 3):
        yy = np.clip(ys + i, 0, H - 1)
        for j in range(-2, 3):
            xx = np.clip(xs + j, 0, W - 1)
            np.add.at(out, np.ix_(yy, xx), BINOMIAL5[i + 2] * BINOMIAL5[j + 2] * V)
    return out


def upsample_adjoint(G: np.ndarray, d: int, Hs: int, Ws: int) -> np.ndarray:
    """Transpose of the sample-aligned bilinear upsample from Hs x Ws to G's grid."""
    Ht, Wt = G.shape
    scale = float(2 ** d)
    fy = np.clip(np.arange(Ht, dtype=np.float64) / scale, 0.0, Hs - 1.0)
    fx = np.clip(np.arange(Wt, dtype=np.float64) / scale, 0.0, Ws - 1.0)
    y0 = np.floor(fy).astype(np.int64)
    x0 = np.floor(fx).astype(np.int64)
    y1 = np.minimum(y0 + 1, Hs - 1)
    x1 = np.minimum(x0 + 1, Ws - 1)
    wy = (fy - y0)[:, None]
    wx = (fx - x0)[None, :]
    out = np.zeros((Hs, Ws))
    np.add.at(out, np.ix_(y0, x0), (1 - wy) * (1 - wx) * G)
    np.add.at(out, np.ix_(y0, x1), (1 - wy) * wx * G)
    np.add.at(out, np.ix_(y1, x0), wy * (1 - wx) * G)
    np.add.at(out, np.ix_(y1, x1), wy * wx * G)
    return out


def prior_chain_forward(C: np.ndarray, w: Sequence[float], Q: float, R: float,
                        p: OracleParams, H: int, W: int, c_max: int,
                        segs: Optional[Sequence[Optional[np.ndarray]]] = None) -> Dict:
    """S_t -> q_t -> pi_t for the whole clip, keeping everything the adjoint needs.
    C: [T][8][Hc][Wc]; segs[t] (optional) is the segmentation supplied at step t."""
    T = C.shape[0]
    w = np.asarray(w, dtype=np.float64)
    ring = border_mask(H, W, p.border)
    K, P = kalman_gains(T, Q, R)
    tape = {"S": [], "obs": [], "q": [], "f": [], "pi": [], "K": K, "P": P,
            "uses_pi": [], "ring": ring, "w": w, "Q": Q, "R": R, "c_max": c_max}
    prev = None
    for t in range(T):
        S = np.tensordot(w, C[t], axes=1)
        q, info = observation(S, p, H, W, c_max)
        if t == 0:
            f = None
            pi = q.copy()
            uses_pi = False
        else:
            seg = None if segs is None else segs[t]
            uses_pi = seg is None
            f = blur(prev if uses_pi else np.asarray(seg, dtype=np.float64))
            pi = f + K[t] * (q - f)
        pi[ring] = p.eps
        tape["S"].append(S)
        tape["obs"].append(info)
        tape["q"].append(q)
        tape["f"].append(f)
        tape["pi"].append(pi)
        tape["uses_pi"].append(uses_pi)
        prev = pi
    return tape


def prior_chain_backward(tape: Dict, C: np.ndarray, grad_pi: np.ndarray,
                         p: OracleParams, want_gS: bool = False):
    """Reverse sweep of the prior chain.

    nu_t = dl/dpi_t + (1 - K_{t+1}) G^T nut_{t+1} (when step t+1 read pi_t), nut_t = nu_t off
    the border ring; dL/dq_t = K_t nut_t; dL/dK_t = sum nut_t (q_t - f_t);
    dL/dS_t = up^T(dL/dq_t on unclamped pixels) / m - [x = x*] sum(g_s S_t) / m^2;
    dL/dw_k = sum_t sum_x dL/dS_t C_{k,t}; then the scalar sweep of K_t(P_{t-1}, Q, R).
    Returns (dL/dw, dL/dQ, dL/dR), and with want_gS also the list of dL/dS_t."""
    T = len(tape["pi"])
    K, P = tape["K"], tape["P"]
    Q, R = tape["Q"], tape["R"]
    ring = tape["ring"]
    c_max = tape["c_max"]
    Hc, Wc = tape["S"][0].shape
    grad_w = np.zeros(C.shape[1])
    gK = np.zeros(T)
    gS_all = [np.zeros((Hc, Wc)) for _ in range(T)]
    nut_next = None
    for t in range(T - 1, -1, -1):
        nu = np.array(grad_pi[t], dtype=np.float64)
        if t + 1 < T and tape["uses_pi"][t + 1]:
            nu = nu + (1.0 - K[t + 1]) * blur_adjoint(nut_next)
        nut = np.where(ring, 0.0, nu)
        gq = K[t] * nut if t > 0 else nut
        if t > 0:
            gK[t] = float((nut * (tape["q"][t] - tape["f"][t])).sum())
        info = tape["obs"][t]
        if not info["flat"]:
            gu = np.where(info["free"], gq, 0.0)
            gs = upsample_adjoint(gu, c_max, Hc, Wc)
            m = info["m"]
            S = tape["S"][t]
            gS = gs / m
            gS.flat[info["xstar"]] -= float((gs * S).sum()) / (m * m)
            grad_w += np.tensordot(C[t], gS, axes=([1, 2], [0, 1]))
            gS_all[t] = gS
        nut_next = nut
    # scalar sweep: K_t = a_t / (a_t + R), a_t = P_{t-1} + Q, P_t = R K_t, P_0 = R
    gQ, gR = 0.0, 0.0
    gP = 0.0
    for t in range(T - 1, 0, -1):
        g = gK[t] + R * gP
        gR += K[t] * gP
        a = P[t - 1] + Q
        ga = g * R / (a + R) ** 2
        gR -= g * a / (a + R) ** 2
        gQ += ga
        gP = ga
    gR += gP
    if want_gS:
        return grad_w, gQ, gR, gS_all
    return grad_w, gQ, gR


def _clip_loss(C, masks, w, Q, R, p, H, W, c_max, segs=None) -> float:
    tape = prior_chain_forward(C, w, Q, R, p, H, W, c_max, segs)
    return mse_mask_loss(np.stack(tape["pi"]), masks)[0]


def finite_difference_grad(C: np.ndarray, masks: np.ndarray, w: Sequence[float], Q: float,
                           R: float, p: OracleParams, H: int, W: int, c_max: int,
                           h: float = 1e-3, segs=None) -> Tuple[np.ndarray, float, float]:
    """Central differences of the clip loss: absolute step h on each w_k; relative step
    on Q and R (ln Q and ln R moved by +-h), converted back to d/dQ and d/dR."""
    w = np.asarray(w, dtype=np.float64)
    gw = np.zeros_like(w)
    for k in range(w.size):
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        gw[k] = (_clip_loss(C, masks, wp, Q, R, p, H, W, c_max, segs)
                 - _clip_loss(C, masks, wm, Q, R, p, H, W, c_max, segs)) / (2 * h)
    eh = np.exp(h)
    gQ = (_clip_loss(C, masks, w, Q * eh, R, p, H, W, c_max, segs)
          - _clip_loss(C, masks, w, Q / eh, R, p, H, W, c_max, segs)) / (2 * h) / Q
    gR = (_clip_loss(C, masks, w, Q, R * eh, p, H, W, c_max, segs)
          - _clip_loss(C, masks, w, Q, R / eh, p, H, W, c_max, segs)) / (2 * h) / R
    return gw, gQ, gR
