"""CPU pins of the colour-likelihood oracle (oracle/gmm.py): uniform weights reduce to
the standard EM of scikit-learn's GaussianMixture from the same start; integer weights
equal unweighted EM on replicated samples; EM never lowers the weighted likelihood
(reg = 0); well-separated Gaussians are recovered; one component is the weighted
Gaussian in closed form; the power iteration finds numpy's leading eigenvector; a label
without weight has no likelihood.  Planted mistakes must turn a pin red."""
import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal
from sklearn.mixture import GaussianMixture

from oracle import gmm as Gm


def _blobs(rng, n, means, scales):
    k = len(means)
    lab = rng.integers(0, k, n)
    C = np.asarray(means)[lab] + rng.normal(size=(n, 3)) * np.asarray(scales)[lab][:, None]
    return C


def _sklearn(C, mix, iters, reg):
    g = GaussianMixture(n_components=mix["alpha"].size, covariance_type="full", reg_covar=reg, max_iter=iters,
                        tol=0.0, weights_init=mix["alpha"], means_init=mix["mu"],
                        precisions_init=np.linalg.inv(mix["cov"]), random_state=0)
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        g.fit(C)
    return g


@pytest.mark.parametrize("M,reg,seed", [(3, 1e-4, 0), (2, 1e-3, 1), (4, 1e-4, 2)])
def test_uniform_weights_equal_standard_em(M, reg, seed):
    rng = np.random.default_rng(seed)
    C = _blobs(rng, 3000, [[0.2, 0.3, 0.1], [0.6, 0.5, 0.4], [0.9, 0.2, 0.7]], [0.05, 0.08, 0.04])
    w = np.full(C.shape[0], 0.37)
    mix0 = Gm.init_mixture(C, w, M, reg)
    for iters in (1, 4):
        mix = mix0
        for _ in range(iters):
            mix = Gm.em_step(C, w, mix, reg)
        g = _sklearn(C, mix0, iters, reg)
        np.testing.assert_allclose(mix["alpha"], g.weights_, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(mix["mu"], g.means_, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(mix["cov"], g.covariances_, rtol=1e-8, atol=1e-13)


def test_integer_weights_equal_replicated_samples():
    rng = np.random.default_rng(5)
    C = _blobs(rng, 1500, [[0.1, 0.1, 0.8], [0.7, 0.6, 0.2]], [0.06, 0.1])
    w = rng.integers(0, 4, C.shape[0]).astype(np.float64)
    rep = np.repeat(C, w.astype(int), axis=0)
    mix0 = Gm.init_mixture(C, w, 3, 1e-4)
    mix = mix0
    for _ in range(3):
        mix = Gm.em_step(C, w, mix, 1e-4)
    g = _sklearn(rep, mix0, 3, 1e-4)
    np.testing.assert_allclose(mix["mu"], g.means_, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(mix["cov"], g.covariances_, rtol=1e-8, atol=1e-13)
    np.testing.assert_allclose(mix["alpha"], g.weights_, rtol=1e-9, atol=1e-12)
    # and the initial moments are those of the replicated set
    W0, mu, S = Gm.weighted_moments(C, w)
    assert W0 == rep.shape[0]
    np.testing.assert_allclose(mu, rep.mean(axis=0), rtol=1e-12)
    np.testing.assert_allclose(S, np.cov(rep.T, bias=True), rtol=1e-10, atol=1e-15)


def test_weighted_likelihood_never_decreases_without_regulariser():
    rng = np.random.default_rng(9)
    C = _blobs(rng, 4000, [[0.2, 0.2, 0.2], [0.5, 0.7, 0.3], [0.8, 0.4, 0.9]], [0.07, 0.05, 0.06])
    w = rng.random(C.shape[0])
    _, hist = Gm.fit_mixture(C, w, 3, 25, 0.0)
    d = np.diff(hist)
    assert np.all(d >= -1e-9 * abs(hist[-1])), d.min()
    assert hist[-1] > hist[0]


def test_separated_gaussians_are_recovered():
    rng = np.random.default_rng(11)
    means = np.array([[0.15, 0.2, 0.25], [0.5, 0.5, 0.5], [0.85, 0.8, 0.75]])
    C = _blobs(rng, 60000, means, [0.03, 0.03, 0.03])
    mix, _ = Gm.fit_mixture(C, np.ones(C.shape[0]), 3, 60, 1e-6)
    order = np.argsort(mix["mu"][:, 0])
    np.testing.assert_allclose(mix["mu"][order], means, atol=2e-3)
    np.testing.assert_allclose(mix["alpha"][order], [1 / 3] * 3, atol=0.02)
    for m in order:
        np.testing.assert_allclose(mix["cov"][m], 0.03 ** 2 * np.eye(3), atol=1e-4)


def test_single_component_is_the_weighted_gaussian():
    rng = np.random.default_rng(13)
    rgb = rng.integers(0, 256, (9, 11, 3)).astype(np.uint8)
    pi = rng.random((9, 11))
    psi, mixes = Gm.colour_likelihood(rgb, pi, M=1, iters=3, reg=1e-3)
    C = Gm.colours(rgb)
    for lab, w in ((0, 1.0 - pi.reshape(-1)), (1, pi.reshape(-1))):
        W0, mu, S = Gm.weighted_moments(C, w)
        ref = -multivariate_normal(mean=mu, cov=S + 1e-3 * np.eye(3)).logpdf(C)
        np.testing.assert_allclose(psi[lab].reshape(-1), ref, rtol=1e-10)


def test_power_iteration_finds_the_leading_eigenvector():
    rng = np.random.default_rng(17)
    for _ in range(5):
        A = rng.normal(size=(3, 3))
        S = A @ A.T + np.diag([0.5, 0.0, 0.0])
        vals, vecs = np.linalg.eigh(S)
        if vals[-1] < 1.5 * vals[-2]:
            continue
        lam, v = Gm.principal_axis(S)
        assert lam == pytest.approx(vals[-1], rel=1e-10)
        assert abs(abs(float(v @ vecs[:, -1])) - 1.0) < 1e-10
        assert v[np.argmax(np.abs(v))] > 0


def test_label_without_weight_has_no_likelihood():
    rgb = np.random.default_rng(1).integers(0, 256, (6, 7, 3)).astype(np.uint8)
    psi, mixes = Gm.colour_likelihood(rgb, np.zeros((6, 7)), M=3, iters=2)
    assert mixes[1] is None and np.all(psi[1] == 0.0)
    assert mixes[0] is not None and np.all(np.isfinite(psi[0]))


def test_initial_means_on_the_principal_axis():
    rng = np.random.default_rng(19)
    C = rng.random((500, 3)) * np.array([1.0, 0.1, 0.1])
    w = rng.random(500)
    mix = Gm.init_mixture(C, w, 3, 1e-4)
    W0, mu, S = Gm.weighted_moments(C, w)
    lam, v = Gm.principal_axis(S)
    np.testing.assert_allclose(mix["mu"][1], mu, rtol=1e-14)
    np.testing.assert_allclose(mix["mu"][2] - mu, math.sqrt(lam) * v, rtol=1e-12)
    np.testing.assert_allclose(mix["mu"][0] - mu, -math.sqrt(lam) * v, rtol=1e-12)
    assert np.all(mix["alpha"] == 1 / 3)


def test_planted_mistakes_fail_the_pins(monkeypatch):
    orig = Gm.em_step

    def unweighted(C, w, mix, reg):       # the M-step ignores the sample weights
        return orig(C, np.ones_like(w), mix, reg)
    monkeypatch.setattr(Gm, "em_step", unweighted)
    with pytest.raises(AssertionError):
        test_integer_weights_equal_replicated_samples()
    monkeypatch.undo()

    def no_reg(C, w, mix, reg):           # the regulariser dropped from the M-step
        return orig(C, w, mix, 0.0)
    monkeypatch.setattr(Gm, "em_step", no_reg)
    with pytest.raises(AssertionError):
        test_uniform_weights_equal_standard_em(3, 1e-3, 0)
    monkeypatch.undo()
    orig_lp = Gm.component_logpdf

    def no_alpha(C, mix):                 # responsibilities without the mixture weights
        m = dict(mix)
        m["alpha"] = np.where(mix["alpha"] > 0, 1.0, 0.0)
        return orig_lp(C, m)
    monkeypatch.setattr(Gm, "component_logpdf", no_alpha)
    with pytest.raises(AssertionError):
        test_uniform_weights_equal_standard_em(3, 1e-4, 0)
