"""GPU parity of the minimum cut (sp_mincut) against the oracle (oracle/mincut.py): on
seeded float capacities the integer capacities, the maximum flow and the labelling (the
minimum cut with the largest object, unique) must agree bit for bit.  The closed loop
(each frame's cut fed back as the next frame's segmentation) is checked for validity on
every frame: the returned labelling is a minimum cut of the frame's own capacities."""
import sys

import numpy as np
import pytest

from oracle import mincut as MC
from paper_1008_0502_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def banner(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def _gpu_cut(unary, pairwise, scale):
    torch = _torch()
    from paper_1008_0502_amd.api import MinCut
    H, W = unary.shape[1:]
    mc = MinCut(H, W)
    lab, flow = mc.cut(torch.from_numpy(unary).cuda(), torch.from_numpy(pairwise).cuda(), scale)
    torch.cuda.synchronize()
    out = lab.cpu().numpy(), int(flow.cpu().item())
    mc.close()
    return out


def _compare(unary, pairwise, scale, label):
    lab, flow = _gpu_cut(unary, pairwise, scale)
    f_ref, lab_ref = MC.segment(unary, pairwise, scale)
    diff = int(np.sum(lab != lab_ref))
    print(f"[parity] {label}: flow {flow} vs {f_ref}, object {int(lab.sum())} px, labels differing {diff}", flush=True)
    assert flow == f_ref
    assert diff == 0


@pytest.mark.parametrize("H,W,seed", [(5, 7, 0), (17, 23, 1), (48, 64, 2), (97, 130, 3), (120, 160, 4)])
def test_integer_capacities(H, W, seed):
    banner(f"min cut, integer capacities {H}x{W}")
    rng = np.random.default_rng(seed)
    unary = rng.integers(0, 40, (2, H, W)).astype(np.float32)
    pairwise = rng.integers(0, 25, (4, H, W)).astype(np.float32)
    _compare(unary, pairwise, 1.0, f"int {H}x{W}")


def _blob_capacities(H, W, seed, T=1):
    """Unary costs of a soft object mask with noise and contrast-like n-links (seeded)."""
    frames, masks = synth.Clip(synth.single_ellipse_spec(H=H, W=W, T=T, seed=seed)).stack()
    rng = np.random.default_rng(seed)
    p = np.clip(0.15 + 0.7 * masks[0] + 0.3 * (rng.random((H, W)) - 0.5), 1e-4, 1 - 1e-4)
    unary = np.stack([-np.log1p(-p), -np.log(p)]).astype(np.float32)
    inten = frames[0].astype(np.float64).mean(axis=2) / 255.0
    pw = np.zeros((4, H, W))
    for d, (dy, dx) in enumerate(MC.DIRS):
        sh = np.full((H, W), np.nan)
        ys, yd = slice(0, H - dy), slice(dy, H)
        if dx >= 0:
            sh[ys, 0:W - dx] = inten[yd, dx:W]
        else:
            sh[ys, -dx:W] = inten[yd, 0:W + dx]
        w = np.exp(-8.0 * (inten - sh) ** 2) / np.hypot(dy, dx)
        pw[d] = np.where(np.isnan(sh), 0.0, w)
    return unary, pw.astype(np.float32)


@pytest.mark.parametrize("H,W,seed,scale", [(120, 160, 0, 256.0), (97, 131, 5, 100.0), (480, 640, 2, 256.0)])
def test_object_like_capacities(H, W, seed, scale):
    banner(f"min cut, object-like capacities {H}x{W} scale {scale}")
    unary, pw = _blob_capacities(H, W, seed)
    _compare(unary, pw, scale, f"blob {H}x{W}")


def test_random_float_capacities_and_edge_cases():
    banner("min cut: random floats, ties, no n-links, one row, one column")
    rng = np.random.default_rng(12)
    _compare(rng.random((2, 31, 45)).astype(np.float32) * 5, rng.random((4, 31, 45)).astype(np.float32), 64.0,
             "float 31x45")
    # every labelling ties: the whole frame is object
    _compare(np.full((2, 8, 9), 2.0, np.float32), np.zeros((4, 8, 9), np.float32), 1.0, "ties")
    _compare(rng.integers(0, 9, (2, 1, 37)).astype(np.float32), rng.integers(0, 5, (4, 1, 37)).astype(np.float32),
             1.0, "1x37")
    _compare(rng.integers(0, 9, (2, 41, 1)).astype(np.float32), rng.integers(0, 5, (4, 41, 1)).astype(np.float32),
             1.0, "41x1")
    _compare(rng.integers(0, 9, (2, 1, 1)).astype(np.float32), np.zeros((4, 1, 1), np.float32), 1.0, "1x1")


def test_closed_loop_cuts_are_minimum_cuts():
    torch = _torch()
    from paper_1008_0502_amd.api import Context, MinCut, Params
    banner("closed loop 160x120: saliency, prior from the previous cut, capacities, cut")
    frames, _ = synth.Clip(synth.single_ellipse_spec(H=120, W=160, T=6, seed=0)).stack()
    ctx = Context(120, 160, Params())
    mc = MinCut(120, 160)
    fr = torch.from_numpy(frames).cuda()
    seg = None
    for t in range(6):
        S, P = ctx.step(fr[t], fr[t - 1] if t else None, seg)
        U, PW, _ = ctx.mrf_weights(fr[t], P)
        lab, flow = mc.cut(U, PW, 256.0)
        torch.cuda.synchronize()
        # validity: the labels are the largest-object minimum cut of these capacities
        f_ref, lab_ref = MC.segment(U.cpu().numpy(), PW.cpu().numpy(), 256.0)
        l = lab.cpu().numpy()
        print(f"[loop] frame {t}: flow {int(flow.item())} object {int(l.sum())} px", flush=True)
        assert int(flow.item()) == f_ref and np.array_equal(l, lab_ref)
        seg = lab
    ctx.close()
    mc.close()
