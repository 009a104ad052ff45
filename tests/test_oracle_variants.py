"""CPU pins of the variants oracle (oracle/variants.py): the distance transform against
scipy's exact Euclidean distance transform and hand values, the f of Section 6 at known
distances, the manual prior of Section 4, the stochastic saliency map of Section 3 in
closed form, and the prior recursion with each variant on hand-checkable cases.  Each
planted mistake at the end must turn one of these pins red."""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle as O
from oracle import variants as V


@pytest.mark.parametrize("shape,density,seed", [((7, 5), 0.2, 0), ((16, 16), 0.05, 1), ((31, 9), 0.5, 2),
                                                ((1, 13), 0.3, 3), ((40, 57), 0.01, 4)])
def test_distance_matches_scipy_edt(shape, density, seed):
    rng = np.random.default_rng(seed)
    seg = (rng.random(shape) < density).astype(np.uint8)
    if not seg.any():
        seg[shape[0] // 2, shape[1] // 2] = 1
    ref = ndimage.distance_transform_edt(seg == 0) ** 2
    assert np.array_equal(V.distance_sq(seg), np.rint(ref))


def test_distance_hand_values_and_empty():
    seg = np.zeros((5, 7), np.uint8)
    seg[2, 3] = 1
    d2 = V.distance_sq(seg)
    assert d2[2, 3] == 0 and d2[0, 0] == 4 + 9 and d2[4, 6] == 4 + 9 and d2[2, 0] == 9 and d2[0, 3] == 4
    assert np.all(np.isinf(V.distance_sq(np.zeros((3, 4), np.uint8))))
    assert np.all(V.f_distance(np.zeros((3, 4), np.uint8), 2.0) == 0.0)


def test_f_distance_at_known_distances():
    seg = np.zeros((9, 9), np.uint8)
    seg[4, 4] = 1
    for sigma in (1.0, 2.0, 3.5):
        f = V.f_distance(seg, sigma)
        assert f[4, 4] == 1.0
        assert f[4, 5] == pytest.approx(math.exp(-1.0 / (2 * sigma * sigma)), rel=1e-15)
        assert f[3, 3] == pytest.approx(math.exp(-2.0 / (2 * sigma * sigma)), rel=1e-15)
        assert f[0, 1] == pytest.approx(math.exp(-25.0 / (2 * sigma * sigma)), rel=1e-15)


def test_manual_prior_codes():
    lab = np.array([[1, 0, 2], [255, 1, 0]], np.uint8)
    m = V.manual_prior(lab, 1e-4)
    assert m.tolist() == [[1.0, 1e-4, 0.5], [0.5, 1.0, 1e-4]]


def test_stochastic_saliency_closed_forms():
    rng = np.random.default_rng(7)
    Ss = [rng.random((6, 8)) for _ in range(5)]
    Qs, Rs = 2e-3, 5e-2
    mu, P = V.stochastic_saliency(Ss, Qs, Rs)
    assert np.array_equal(mu[0], Ss[0]) and P[0] == Rs
    K1 = (Rs + Qs) / (Rs + Qs + Rs)
    np.testing.assert_allclose(mu[1], Ss[0] + K1 * (Ss[1] - Ss[0]), rtol=1e-15, atol=1e-15)
    assert P[1] == pytest.approx(Rs * K1, rel=1e-15)
    # a constant map stays put; a vanishing observation variance follows S exactly
    c = [np.full((3, 3), 0.7)] * 4
    assert np.all(V.stochastic_saliency(c, Qs, Rs)[0] == 0.7)
    mu0, _ = V.stochastic_saliency(Ss, 1e-3, 1e-30)
    np.testing.assert_allclose(mu0, np.stack(Ss), rtol=1e-12, atol=1e-12)
    # steady state of the gain on a long run: K = P/R with P = (-Q + sqrt(Q^2 + 4QR)) / 2
    _, Pl = V.stochastic_saliency([np.zeros((1, 1))] * 400, Qs, Rs)
    assert Pl[-1] == pytest.approx((-Qs + math.sqrt(Qs * Qs + 4 * Qs * Rs)) / 2, rel=1e-12)


def test_default_variant_equals_prior_clip():
    rng = np.random.default_rng(3)
    qs = [np.clip(rng.random((12, 10)), 1e-4, 1 - 1e-4) for _ in range(4)]
    p = O.OracleParams(q=2e-3, r=3e-2)
    a, _, Ka = O.prior_clip(qs, p)
    b, _, Kb = V.prior_clip_variant(qs, p, f_mode=0)
    assert np.array_equal(Ka, Kb)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_distance_prior_by_hand():
    H, W = 11, 13
    p = O.OracleParams(q=1e-3, r=1e-1, border=1)
    q = np.full((H, W), 0.3)
    seg = np.zeros((H, W), np.uint8)
    seg[5, 6] = 1
    pis, fs, K = V.prior_clip_variant([q, q], p, f_mode=1, dt_sigma=2.0, segs=[None, seg])
    assert pis[1][5, 6] == pytest.approx(1.0 + K[1] * (0.3 - 1.0), rel=1e-15)
    f = math.exp(-1.0 / 8.0)
    assert pis[1][5, 7] == pytest.approx(f + K[1] * (0.3 - f), rel=1e-15)
    assert pis[1][0, 0] == p.eps and pis[1][H - 1, 4] == p.eps


def test_stand_in_threshold_is_strict():
    H, W = 9, 9
    p = O.OracleParams(border=0)
    q0 = np.full((H, W), 0.5)
    q0[4, 4] = 0.9
    pis, fs, _ = V.prior_clip_variant([q0, q0], p, f_mode=1, dt_sigma=1.0)
    # only the pixel above one half is object for the stand-in
    assert fs[1][4, 4] == 1.0 and fs[1][0, 0] == pytest.approx(math.exp(-32.0 / 2.0), rel=1e-15)


def test_manual_first_frame_then_blur():
    H, W = 8, 10
    p = O.OracleParams(border=1)
    lab = np.full((H, W), 2, np.uint8)
    lab[2:5, 3:7] = 1
    lab[0, :] = 0
    q = np.full((H, W), 0.25)
    pis, fs, K = V.prior_clip_variant([q, q], p, pi0=V.manual_prior(lab, p.eps))
    assert pis[0][0, 0] == p.eps and pis[0][3, 4] == 1.0 and pis[0][6, 1] == 0.5 and pis[0][6, 0] == 0.5
    f = O.blur(pis[0])
    ring = O.border_mask(H, W, 1)
    exp1 = f + K[1] * (q - f)
    exp1[ring] = p.eps
    np.testing.assert_allclose(pis[1], exp1, rtol=0, atol=0)


# -- planted mistakes: each variant of the oracle must fail one of the pins above
def _mistake_manhattan(seg):
    seg = np.asarray(seg) != 0
    H, W = seg.shape
    oy, ox = np.nonzero(seg)
    out = np.full((H, W), np.inf)
    for y in range(H):
        for x in range(W):
            if oy.size:
                out[y, x] = float(np.min((np.abs(oy - y) + np.abs(ox - x)) ** 2))
    return out


def test_planted_mistakes_fail_the_pins(monkeypatch):
    seg = np.zeros((5, 7), np.uint8)
    seg[2, 3] = 1
    monkeypatch.setattr(V, "distance_sq", _mistake_manhattan)
    with pytest.raises(AssertionError):
        test_distance_hand_values_and_empty()
    monkeypatch.undo()
    # f with sigma instead of sigma^2
    monkeypatch.setattr(V, "f_distance", lambda s, sg: np.exp(-V.distance_sq(s) / (2.0 * sg)))
    with pytest.raises(AssertionError):
        test_f_distance_at_known_distances()
    monkeypatch.undo()
    # stand-in with >= instead of >
    orig = V.prior_clip_variant

    def ge_variant(qs, p, f_mode=0, dt_sigma=2.0, segs=None, pi0=None):
        if f_mode == 1 and segs is None:
            segs = [None] + [None] * (len(qs) - 1)
            out, _, K = orig(qs[:1], p)
            prev = out[0]
            f = V.f_distance(prev >= 0.5, dt_sigma)
            pi = f + K[0] * 0 + O.kalman_gains(2, p.q, p.r)[0][1] * (qs[1] - f)
            return [prev, pi], [None, f], O.kalman_gains(2, p.q, p.r)[0]
        return orig(qs, p, f_mode, dt_sigma, segs, pi0)
    monkeypatch.setattr(V, "prior_clip_variant", ge_variant)
    with pytest.raises(AssertionError):
        test_stand_in_threshold_is_strict()
    monkeypatch.undo()
    # stochastic map started from zero instead of the first map
    monkeypatch.setattr(V, "stochastic_saliency",
                        lambda Ss, Qs, Rs: (np.stack([np.zeros_like(Ss[0])] + list(Ss[1:])), O.kalman_gains(len(Ss), Qs, Rs)[1]))
    with pytest.raises(AssertionError):
        test_stochastic_saliency_closed_forms()
