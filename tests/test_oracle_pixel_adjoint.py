"""CPU pins of the pixel-level adjoint oracle (oracle/pixel_adjoint.py): dot-product tests
of the pyramid-step and Gabor transposes, central differences of N(.), of the features, of
the whole saliency map and of the clip loss in random directions (real-valued frames, so
no kink lies within the step), central differences on a motion plateau (the sign band of
|D|), and planted mistakes that must turn a pin red."""
import numpy as np
import pytest

import oracle as O
from oracle import pixel_adjoint as PA
from oracle.saliency import CHANNELS, ORIENTATIONS_DEG, chromatic_mask


def _dot(a, b):
    return float(np.sum(a * b))


@pytest.mark.parametrize("H,W", [(7, 5), (16, 16), (13, 1), (1, 9), (2, 2), (21, 34)])
def test_reduce_adjoint_dot_product(H, W):
    rng = np.random.default_rng(H * 100 + W)
    X = rng.normal(size=(H, W))
    R = O.reduce_level(X)
    G = rng.normal(size=R.shape)
    assert _dot(R, G) == pytest.approx(_dot(X, PA.reduce_adjoint(G, H, W)), rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("H,W,theta", [(11, 9, 0.0), (20, 17, 45.0), (5, 3, 135.0), (14, 14, 90.0)])
def test_gabor_adjoint_dot_product(H, W, theta):
    rng = np.random.default_rng(int(theta) + H)
    h = O.gabor_kernel(theta)
    X = rng.normal(size=(H, W))
    G = rng.normal(size=(H, W))
    assert _dot(O.gabor(X, h), G) == pytest.approx(_dot(X, PA.gabor_adjoint(G, h)), rel=1e-12, abs=1e-12)


def _fd(f, x, v, h):
    return (f(x + h * v) - f(x - h * v)) / (2 * h)


@pytest.mark.parametrize("H,W,seed", [(13, 17, 0), (8, 8, 1), (30, 25, 2), (1, 12, 3)])
def test_normalise_vjp_matches_central_differences(H, W, seed):
    rng = np.random.default_rng(seed)
    X = rng.random((H, W))
    gN = rng.normal(size=(H, W))
    f = lambda Z: _dot(gN, O.normalise(Z))
    g = PA.normalise_vjp(X, gN)
    for _ in range(3):
        v = rng.normal(size=(H, W))
        assert _fd(f, X, v, 1e-7) == pytest.approx(_dot(g, v), rel=1e-6, abs=1e-9)


def _band_stats(rgb, prev, p, chrom):
    """Over every centre-surround pair and channel: the smallest |D| / scale above the sign
    band, and the number of positions at or below it whose D is not exactly zero."""
    _, _, inter = O.saliency(rgb, prev, p, want_intermediate=True, chrom=chrom)
    geo, base, orient = inter["geometry"], inter["base"], inter["orient"]
    maps = dict(base, **{n: orient[th] for n, th in zip(("O0", "O45", "O90", "O135"), ORIENTATIONS_DEG)})
    above, tiny = np.inf, 0
    for name in CHANNELS:
        for c, s in geo.pairs:
            D = maps[name][c] - O.upsample(maps[name][s], s - c, *geo.sizes[c])
            scale = max(np.abs(maps[name][c]).max(), np.abs(maps[name][s]).max())
            if scale == 0:
                continue
            r = np.abs(D) / scale
            above = min(above, float(r[r > PA.SIGN_BAND].min(initial=np.inf)))
            tiny += int(np.sum((r <= PA.SIGN_BAND) & (D != 0)))
    return above, tiny


def _real_frames(rng, T, H, W):
    base = rng.random((H, W, 3)) * 200 + 20
    return np.stack([np.clip(base + rng.normal(size=(H, W, 3)) * (8 + 4 * t), 0.5, 254.5) for t in range(T)])


def test_feature_vjp_matches_central_differences():
    rng = np.random.default_rng(5)
    fr = _real_frames(rng, 2, 9, 11)
    chrom = chromatic_mask(np.rint(fr[1]).astype(np.uint8))
    gs = {k: rng.normal(size=(9, 11)) for k in ("I", "RG", "BY", "M")}

    def f(x, prev):
        F = O.features(x, prev, -1, chrom)
        return sum(_dot(gs[k], F[k]) for k in gs)
    g, gp = PA.feature_vjp(fr[1], fr[0], chrom, gs["I"], gs["RG"], gs["BY"], gs["M"])
    for _ in range(3):
        v = rng.normal(size=fr[1].shape)
        assert _fd(lambda z: f(z, fr[0]), fr[1], v, 1e-5) == pytest.approx(_dot(g, v), rel=1e-7, abs=1e-12)
        assert _fd(lambda z: f(fr[1], z), fr[0], v, 1e-5) == pytest.approx(_dot(gp, v), rel=1e-7, abs=1e-12)


@pytest.mark.parametrize("H,W,seed,centers,deltas", [(40, 48, 3, (1, 2), (2, 3)), (36, 33, 1, (2,), (2, 3))])
def test_saliency_vjp_matches_central_differences(H, W, seed, centers, deltas):
    rng = np.random.default_rng(seed)
    p = O.OracleParams(centers=centers, deltas=deltas, weights=tuple(rng.random(8) + 0.5))
    fr = _real_frames(rng, 2, H, W)
    chrom = chromatic_mask(np.rint(fr[1]).astype(np.uint8))
    S0, _ = O.saliency(fr[1], fr[0], p, chrom=chrom)
    gS = rng.normal(size=S0.shape)
    # no centre-surround difference of these frames lies inside the sign band, so the
    # convention there does not enter and the exact derivative is the one to match
    assert _band_stats(fr[1], fr[0], p, chrom)[1] == 0
    g, gp = PA.saliency_vjp(fr[1], fr[0], gS, p, chrom)
    for _ in range(2):
        v = rng.normal(size=fr[1].shape)
        fd = _fd(lambda z: _dot(gS, O.saliency(z, fr[0], p, chrom=chrom)[0]), fr[1], v, 1e-4)
        assert fd == pytest.approx(_dot(g, v), rel=2e-6)
        fdp = _fd(lambda z: _dot(gS, O.saliency(fr[1], z, p, chrom=chrom)[0]), fr[0], v, 1e-4)
        assert fdp == pytest.approx(_dot(gp, v), rel=2e-6, abs=1e-12)


def test_clip_gradient_matches_central_differences():
    rng = np.random.default_rng(9)
    T, H, W = 3, 40, 48
    fr = _real_frames(rng, T, H, W)
    masks = np.zeros((T, H, W), np.uint8)
    masks[:, 12:26, 15:33] = 1
    p = O.OracleParams(q=2e-3, r=5e-2)
    # a few differences of these frames fall inside the sign band: the exact derivative
    loss, grad = PA.frame_gradients(fr, masks, p, sign_band=0.0)
    chroms = [chromatic_mask(fr[t]) for t in range(T)]
    for _ in range(2):
        v = rng.normal(size=fr.shape)
        # a step of 1e-5 (on the 0..255 scale) keeps the observation's clamp and the
        # argmax of S on one side for every pixel of this clip
        fd = _fd(lambda z: PA.clip_loss(z, masks, p, chroms), fr, v, 1e-5)
        assert fd == pytest.approx(_dot(grad, v), rel=1e-7)
    # every frame, including the last one, gets a gradient; the first also through motion
    assert all(np.abs(grad[t]).max() > 0 for t in range(T))


def _motion_pyramid_int(s_t, s_prev, top):
    """The motion map's pyramid in exact integers: level l holds 765 * 256^l * M_l (the
    binomial taps 1 4 6 4 1 in each direction, clamp-to-edge, even rows and columns)."""
    k = np.array([1, 4, 6, 4, 1], dtype=np.int64)
    Z = [np.abs(s_t.astype(np.int64) - s_prev.astype(np.int64))]
    for _ in range(top):
        X = Z[-1]
        H, W = X.shape
        ys, xs = np.arange(H), np.arange(W)
        B = np.zeros_like(X)
        for i in range(5):
            for j in range(5):
                B += k[i] * k[j] * X[np.ix_(np.clip(ys + i - 2, 0, H - 1), np.clip(xs + j - 2, 0, W - 1))]
        Z.append(B[::2, ::2])
    return Z


def _up_int(Z, d, Ht, Wt):
    """4^d times the sample-aligned bilinear up-sample of Z (exact: the weights are k / 2^d)."""
    Hs, Ws = Z.shape
    n = 1 << d

    def taps(m, size):
        i = np.arange(m)
        i0 = np.minimum(i >> d, size - 1)
        a = np.where((i >> d) >= size - 1, 0, i & (n - 1))
        return i0, np.minimum(i0 + 1, size - 1), a
    y0, y1, ay = taps(Ht, Hs)
    x0, x1, ax = taps(Wt, Ws)
    ay, ax = ay[:, None], ax[None, :]
    top = (n - ax) * Z[np.ix_(y0, x0)] + ax * Z[np.ix_(y0, x1)]
    bot = (n - ax) * Z[np.ix_(y1, x0)] + ax * Z[np.ix_(y1, x1)]
    return (n - ay) * top + ay * bot


def test_sign_band_against_exact_motion_differences():
    """A constant-colour object moving over a constant background makes the motion map a
    plateau: D = M(c) - up M(s) vanishes there in exact arithmetic, while the FP64 maps leave
    rounding residue of either sign.  The motion pyramid is exact in integers, so the sign of
    every D can be taken exactly: the band must cover every exact zero, and outside it the
    sign of the FP64 D must be the exact one."""
    from paper_1008_0502_amd import synth
    frames, _ = synth.Clip(synth.three_ellipse_spec(H=97, W=131, T=3, seed=2)).stack()
    p = O.OracleParams()
    _, _, inter = O.saliency(frames[2], frames[1], p, want_intermediate=True, chrom=chromatic_mask(frames[2]))
    geo, M = inter["geometry"], inter["base"]["M"]
    Z = _motion_pyramid_int(frames[2].astype(np.int64).sum(axis=2), frames[1].astype(np.int64).sum(axis=2), geo.top)
    zeros = residue = plain_wrong = 0
    for c, s in geo.pairs:
        d = s - c
        D = M[c] - O.upsample(M[s], d, *geo.sizes[c])
        Dx = Z[c] * (256 ** d) * (4 ** d) - _up_int(Z[s], d, *geo.sizes[c])
        band = PA.SIGN_BAND * max(np.abs(M[c]).max(), np.abs(M[s]).max())
        assert np.all(np.abs(D[Dx == 0]) <= band)
        out = np.abs(D) > band
        assert np.array_equal(np.sign(D[out]), np.sign(Dx[out]))
        zeros += int(np.sum(Dx == 0))
        residue += int(np.sum((Dx == 0) & (D != 0)))
        plain_wrong += int(np.sum(np.sign(D) != np.sign(Dx)))
    # the case the band is for: exact zeros that FP64 leaves nonzero, where sign(D) is noise
    assert zeros > 0 and residue > 0 and plain_wrong > 0


def test_planted_mistakes_fail_the_pins(monkeypatch):
    orig_n = PA.normalise_vjp

    def no_block_term(X, gN, flat_tol=1e-5, block=8):     # the block maxima's gradient dropped
        return orig_n(X, gN, flat_tol, max(X.shape) + 1)
    monkeypatch.setattr(PA, "normalise_vjp", no_block_term)
    with pytest.raises(AssertionError):
        test_normalise_vjp_matches_central_differences(13, 17, 0)
    monkeypatch.undo()
    # the pyramid transpose without the even-position insertion
    monkeypatch.setattr(PA, "reduce_adjoint", lambda G, Hf, Wf: O.adjoint.blur_adjoint(
        np.repeat(np.repeat(G, 2, 0), 2, 1)[:Hf, :Wf]) / 4.0)
    with pytest.raises(AssertionError):
        test_reduce_adjoint_dot_product(16, 16)
    monkeypatch.undo()
    orig_f = PA.feature_vjp

    def no_motion_to_prev(rgb, prev, chrom, gI, gRG, gBY, gM):   # motion never reaches frame t-1
        g, gp = orig_f(rgb, prev, chrom, gI, gRG, gBY, gM)
        return g, None if gp is None else 0 * gp
    monkeypatch.setattr(PA, "feature_vjp", no_motion_to_prev)
    with pytest.raises(AssertionError):
        test_feature_vjp_matches_central_differences()
    monkeypatch.undo()

    def no_norm_term(rgb, prev, chrom, gI, gRG, gBY, gM):          # r' = r / I taken as r
        return orig_f(rgb, prev, np.zeros_like(chrom), gI, gRG, gBY, gM)
    monkeypatch.setattr(PA, "feature_vjp", no_norm_term)
    with pytest.raises(AssertionError):
        test_feature_vjp_matches_central_differences()
