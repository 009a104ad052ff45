"""FP64 oracle, part 5: the colour likelihood of the t-links (Sections 4, 5, 7.3, 8.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy float64.

Section 4 gives the first likelihood term as psi_1(D | A_x) = -log p(C_x | A_x), with
p(C | A) a Gaussian mixture of M components over RGB fitted by the standard EM
algorithm; Section 5 fits it on every pixel, each sample weighted by the prior
p(A_x = 1); Section 8.1 takes M = 3.  Readings taken here:

* colours C = RGB / 255; full 3x3 covariances; the object mixture (label 1) weights
  pixel x by pi(x), the background mixture (label 0) by 1 - pi(x);
* initialisation (the paper ran k-means on the CPU; a discrete assignment would let
  FP32 and FP64 differ by whole pixels): weighted mean mu and covariance Sigma of the
  label's samples, leading eigenvector v of Sigma by power iteration (64 steps from
  (1, 1, 1) / sqrt 3, sign such that its largest-magnitude entry is positive), means
  mu + z_m sqrt(lambda) v with z_m evenly spaced in [-1, 1] (0 for M = 1), every
  covariance Sigma + reg I, weights 1 / M;
* a fixed number of EM iterations; the M-step adds reg I to every covariance;
* a component whose weighted count falls to at most 1e-12 of the label's total weight,
  or whose covariance is not positive definite (also at the start), gets weight 0 and
  keeps its mean and covariance (it no longer takes part); a label whose total weight is
  at most 1e-12 per pixel, or that has no component left, has no likelihood (psi_1 = 0
  for it);
* psi_1 is added to the unary costs: U0 += psi_1(C | A = 0), U1 += psi_1(C | A = 1).
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

LOG2PI = math.log(2.0 * math.pi)


def colours(rgb: np.ndarray) -> np.ndarray:
    """[N][3] samples in [0, 1] from uint8 RGB."""
    return np.asarray(rgb, dtype=np.float64).reshape(-1, 3) / 255.0


def weighted_moments(C: np.ndarray, w: np.ndarray) -> Tuple[float, np.ndarray, np.ndarray]:
    """Total weight, weighted mean and weighted (biased) covariance of the samples."""
    W0 = float(w.sum())
    mu = (w[:, None] * C).sum(axis=0) / W0
    D = C - mu
    S = (w[:, None, None] * D[:, :, None] * D[:, None, :]).sum(axis=0) / W0
    return W0, mu, S


def principal_axis(S: np.ndarray, iters: int = 64) -> Tuple[float, np.ndarray]:
    """Leading eigenpair of a symmetric 3x3 matrix by power iteration from (1,1,1)/sqrt 3;
    the sign puts the largest-magnitude entry positive (the first such entry on ties)."""
    v = np.ones(3) / math.sqrt(3.0)
    for _ in range(iters):
        u = S @ v
        n = math.sqrt(float(u @ u))
        if not n > 0.0:
            break
        v = u / n
    k = int(np.argmax(np.abs(v)))
    if v[k] < 0:
        v = -v
    return float(v @ S @ v), v


def init_mixture(C: np.ndarray, w: np.ndarray, M: int, reg: float) -> Dict:
    W0, mu, S = weighted_moments(C, w)
    lam, v = principal_axis(S)
    z = np.linspace(-1.0, 1.0, M) if M > 1 else np.zeros(1)
    s = math.sqrt(max(lam, 0.0))
    cov = S + reg * np.eye(3)
    alpha = np.full(M, 1.0 / M) if _usable(cov) else np.zeros(M)
    return {"alpha": alpha, "mu": mu[None, :] + z[:, None] * s * v[None, :],
            "cov": np.repeat(cov[None], M, axis=0)}


def _usable(cov: np.ndarray) -> bool:
    return bool(np.all(np.isfinite(cov))) and np.all(np.linalg.eigvalsh(cov) > 0.0)


def component_logpdf(C: np.ndarray, mix: Dict) -> np.ndarray:
    """[N][M] log(alpha_m N(c; mu_m, Sigma_m)); -inf for components of weight 0."""
    N, M = C.shape[0], mix["alpha"].size
    out = np.full((N, M), -np.inf)
    for m in range(M):
        a = mix["alpha"][m]
        if not a > 0.0:
            continue
        cov = mix["cov"][m]
        D = C - mix["mu"][m]
        P = np.linalg.inv(cov)
        q = np.einsum("ni,ij,nj->n", D, P, D)
        out[:, m] = math.log(a) - 0.5 * math.log(np.linalg.det(cov)) - 1.5 * LOG2PI - 0.5 * q
    return out


def log_likelihood(C: np.ndarray, mix: Dict) -> np.ndarray:
    """[N] log p(c) of the mixture (log-sum-exp over the components)."""
    lp = component_logpdf(C, mix)
    mx = lp.max(axis=1)
    return mx + np.log(np.exp(lp - mx[:, None]).sum(axis=1))


def em_step(C: np.ndarray, w: np.ndarray, mix: Dict, reg: float) -> Dict:
    """One EM iteration with sample weights w: responsibilities under the current
    mixture, then weighted counts, means and covariances (+ reg I)."""
    lp = component_logpdf(C, mix)
    mx = lp.max(axis=1)
    r = np.exp(lp - mx[:, None])
    r /= r.sum(axis=1)[:, None]
    W0 = float(w.sum())
    M = mix["alpha"].size
    Nm = (w[:, None] * r).sum(axis=0)
    out = {"alpha": np.zeros(M), "mu": mix["mu"].copy(), "cov": mix["cov"].copy()}
    for m in range(M):
        if not mix["alpha"][m] > 0.0 or not Nm[m] > 1e-12 * W0:
            continue
        wr = w * r[:, m]
        mu = (wr[:, None] * C).sum(axis=0) / Nm[m]
        D = C - mu
        cov = (wr[:, None, None] * D[:, :, None] * D[:, None, :]).sum(axis=0) / Nm[m] + reg * np.eye(3)
        if not _usable(cov):
            continue
        out["alpha"][m] = Nm[m]
        out["mu"][m] = mu
        out["cov"][m] = cov
    tot = out["alpha"].sum()
    if tot > 0:
        out["alpha"] /= tot
    return out


def fit_mixture(C: np.ndarray, w: np.ndarray, M: int, iters: int, reg: float):
    """Initial mixture, then `iters` EM steps.  Returns (mixture or None when the label's
    weight vanishes, [weighted log-likelihood of the samples under each mixture, from
    the initial one to the last])."""
    if not float(w.sum()) > 1e-12 * w.size:
        return None, []
    mix = init_mixture(C, w, M, reg)
    if not np.any(mix["alpha"] > 0.0):
        return mix, []
    hist = [float((w * log_likelihood(C, mix)).sum())]
    for _ in range(iters):
        mix = em_step(C, w, mix, reg)
        hist.append(float((w * log_likelihood(C, mix)).sum()))
    return mix, hist


def colour_likelihood(rgb: np.ndarray, prior: np.ndarray, M: int = 3, iters: int = 10, reg: float = 1e-4):
    """psi_1 of both labels, [2][H][W] (label 0 = background, label 1 = object), and the
    two fitted mixtures (None for a label without weight)."""
    H, W = np.asarray(prior).shape
    C = colours(rgb)
    pi = np.asarray(prior, dtype=np.float64).reshape(-1)
    psi = np.zeros((2, H * W))
    mixes: List = []
    for lab, w in ((0, 1.0 - pi), (1, pi)):
        mix, _ = fit_mixture(C, w, M, iters, reg)
        mixes.append(mix)
        if mix is not None and np.any(mix["alpha"] > 0.0):
            psi[lab] = -log_likelihood(C, mix)
    return psi.reshape(2, H, W), mixes
