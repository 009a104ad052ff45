"""GPU adjoint of the saliency -> Kalman -> prior chain vs the FP64 oracle.

Gradients of L = mean (prior - mask)^2 with respect to the 8 channel weights and the
Kalman variances Q, R.  Bar: per component |g - g_ref| / max(|g_ref|, 1e-3 |g_ref|_inf)
<= 1e-3 against both the oracle's analytic FP64 gradient and its FP64 central
differences (absolute step on w, relative step on Q and R).
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1008_0502_amd import synth

from _util import oracle_params

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def banner(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def grad_err(g, ref):
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return float(np.max(np.abs(g - ref) / scale))


def gpu_grad(frames, masks, pp, w, Q, R, segs=None):
    torch = _torch()
    from paper_1008_0502_amd.api import Context, Params
    import dataclasses
    T, H, W = frames.shape[:3]
    ctx = Context(H, W, dataclasses.replace(pp, record_tape=T, weights=tuple(w), q=Q, r=R))
    fr = torch.from_numpy(frames).cuda()
    mk = torch.from_numpy(masks).cuda()
    sg = None if segs is None else [None if s is None else torch.from_numpy(s).cuda() for s in segs]
    out = ctx.run_clip(fr, segs=sg)
    loss, grad = ctx.mse_mask_loss(out["pi"], mk)
    gw, gq, gr = ctx.saliency_backward(grad)
    torch.cuda.synchronize()
    res = (gw.cpu().numpy().astype(np.float64), float(gq.cpu()), float(gr.cpu()), float(loss.cpu()),
           out["pi"].cpu().numpy())
    ctx.close()
    return res


def oracle_grads(frames, masks, pp, w, Q, R, segs=None, fd=True):
    op = oracle_params(pp)
    T, H, W = frames.shape[:3]
    ref = O.run_clip(frames, op)
    geo = ref["geometry"]
    tape = O.prior_chain_forward(ref["C"], w, Q, R, op, H, W, geo.c_max, segs)
    L, g = O.mse_mask_loss(np.stack(tape["pi"]), masks)
    gw, gQ, gR = O.prior_chain_backward(tape, ref["C"], g, op)
    out = {"L": L, "gw": gw, "gQ": gQ, "gR": gR, "pi": np.stack(tape["pi"])}
    if fd:
        fw, fQ, fR = O.finite_difference_grad(ref["C"], masks, w, Q, R, op, H, W, geo.c_max, h=1e-3, segs=segs)
        out.update({"fw": fw, "fQ": fQ, "fR": fR})
    return out


def check(label, gpu, ref, tol=1e-3):
    gw, gq, gr, loss, pi = gpu
    full = np.concatenate([gw, [gq, gr]])
    an = np.concatenate([ref["gw"], [ref["gQ"], ref["gR"]]])
    e_an = grad_err(full, an)
    msg = f"[grad] {label}: loss gpu {loss:.6e} oracle {ref['L']:.6e}; vs analytic {e_an:.2e}"
    if "fw" in ref:
        fd = np.concatenate([ref["fw"], [ref["fQ"], ref["fR"]]])
        e_fd = grad_err(full, fd)
        msg += f"; vs FD {e_fd:.2e}"
    print(msg, flush=True)
    assert loss == pytest.approx(ref["L"], rel=1e-4)
    assert e_an <= tol, f"{label}: analytic gradient error {e_an:.3e}"
    if "fw" in ref:
        assert e_fd <= tol, f"{label}: FD gradient error {e_fd:.3e}"


def small_clip(H=64, W=80, T=10, seed=3):
    spec = synth.single_ellipse_spec(H=H, W=W, T=T, seed=seed)
    spec.axes = (9.0, 6.0)
    spec.speed = 1.5
    return synth.Clip(spec).stack()


def params(**kw):
    from paper_1008_0502_amd.api import Params
    return Params(**kw)


W8 = np.array([1.0, 0.8, 1.2, 0.9, 1.1, 0.7, 1.3, 1.0])


@pytest.mark.parametrize("Q,R", [(1e-3, 1e-1), (0.035 ** 2, 0.03 ** 2)])
def test_adjoint_small_clip(Q, R):
    banner(f"adjoint 64x80 x 10 frames, Q={Q:g} R={R:g}")
    frames, masks = small_clip()
    pp = params()
    gpu = gpu_grad(frames, masks, pp, W8, Q, R)
    ref = oracle_grads(frames, masks, pp, W8, Q, R)
    check("64x80", gpu, ref)
    # gauge: the prior does not change along w, so sum_k w_k dL/dw_k = 0
    gw = gpu[0]
    assert abs(float(np.dot(W8, gw))) <= 1e-3 * float(np.abs(W8).max() * np.abs(gw).max())


def test_adjoint_with_segmentation_feedback():
    banner("adjoint with the previous segmentation supplied at some steps")
    frames, masks = small_clip(T=8, seed=5)
    segs = [None, masks[0], None, None, masks[3], None, masks[5], None]
    pp = params()
    gpu = gpu_grad(frames, masks, pp, W8, 1e-3, 1e-1, segs=segs)
    ref = oracle_grads(frames, masks, pp, W8, 1e-3, 1e-1, segs=segs)
    check("seg-feedback", gpu, ref)


def test_adjoint_single_ellipse_clip():
    banner("adjoint 160x120 x 30 frames")
    frames, masks = synth.Clip(synth.single_ellipse_spec(T=30)).stack()
    pp = params()
    gpu = gpu_grad(frames, masks, pp, np.ones(8), 1e-3, 1e-1)
    ref = oracle_grads(frames, masks, pp, np.ones(8), 1e-3, 1e-1)
    check("160x120", gpu, ref)


def test_adjoint_640x480_sampled():
    banner("adjoint at 640x480, 6 frames, tape chunking over recompute streams")
    frames, masks = synth.Clip(synth.single_ellipse_spec(H=480, W=640, T=6, seed=2)).stack()
    pp = params()
    gpu = gpu_grad(frames, masks, pp, W8, 1e-3, 1e-1)
    ref = oracle_grads(frames, masks, pp, W8, 1e-3, 1e-1, fd=False)
    check("640x480", gpu, ref)


def test_adjoint_more_frames_than_a_recompute_chunk():
    banner("adjoint over 40 frames (two recompute chunks of 32)")
    frames, masks = small_clip(H=48, W=64, T=40, seed=8)
    pp = params()
    gpu = gpu_grad(frames, masks, pp, W8, 2e-3, 5e-2)
    ref = oracle_grads(frames, masks, pp, W8, 2e-3, 5e-2)
    check("40 frames", gpu, ref)


def test_autograd_function_fits_weights():
    banner("torch.autograd.Function wrapper: gradients and a few descent steps")
    torch = _torch()
    from paper_1008_0502_amd.api import Context, SaliencyPrior
    frames, masks = small_clip(T=8, seed=11)
    T, H, W = frames.shape[:3]
    ctx = Context(H, W, params(record_tape=T))
    fr = torch.from_numpy(frames).cuda()
    mk = torch.from_numpy(masks).cuda().float()
    w = torch.tensor(W8, dtype=torch.float32, device="cuda", requires_grad=True)
    q = torch.tensor(1e-3, dtype=torch.float64, requires_grad=True)
    r = torch.tensor(1e-1, dtype=torch.float64, requires_grad=True)
    pi = SaliencyPrior.apply(ctx, fr, w, q, r)
    loss = ((pi - mk) ** 2).mean()
    loss.backward()
    ref = oracle_grads(frames, masks, params(), W8, 1e-3, 1e-1, fd=False)
    full = np.concatenate([w.grad.cpu().numpy(), [float(q.grad), float(r.grad)]])
    an = np.concatenate([ref["gw"], [ref["gQ"], ref["gR"]]])
    e = grad_err(full, an)
    print(f"[grad] autograd wrapper vs oracle analytic: {e:.2e}", flush=True)
    assert e <= 1e-3
    # a few projected gradient steps on the weights lower the loss
    opt = torch.optim.SGD([w], lr=20.0)
    l0 = float(loss.detach())
    for _ in range(5):
        opt.zero_grad()
        pi = SaliencyPrior.apply(ctx, fr, w, q.detach(), r.detach())
        l = ((pi - mk) ** 2).mean()
        l.backward()
        opt.step()
        with torch.no_grad():
            w.clamp_(min=0.0)
    assert float(l.detach()) < l0
    ctx.close()


def test_autograd_backward_after_another_forward_raises():
    banner("autograd wrapper: a second forward on the same context invalidates the first graph's tape")
    torch = _torch()
    from paper_1008_0502_amd.api import Context, SaliencyPrior
    frames, masks = small_clip(T=4, seed=13)
    T, H, W = frames.shape[:3]
    ctx = Context(H, W, params(record_tape=T))
    fr = torch.from_numpy(frames).cuda()
    mk = torch.from_numpy(masks).cuda().float()
    w = torch.tensor(W8, dtype=torch.float32, device="cuda", requires_grad=True)
    q = torch.tensor(1e-3, dtype=torch.float64)
    r = torch.tensor(1e-1, dtype=torch.float64)
    pi1 = SaliencyPrior.apply(ctx, fr, w, q, r)
    pi2 = SaliencyPrior.apply(ctx, fr, w * 1.5, q, r)
    with pytest.raises(RuntimeError, match="tape"):
        ((pi1 - mk) ** 2).mean().backward()
    ((pi2 - mk) ** 2).mean().backward()          # the latest graph still differentiates
    assert w.grad is not None and torch.isfinite(w.grad).all()
    # set_weights after recorded steps: the C-ABI refuses the stale tape
    from paper_1008_0502_amd import SalpriorError
    ctx.run_clip(fr)
    ctx.set_weights(W8, 1e-3, 1e-1)
    with pytest.raises(SalpriorError):
        ctx.saliency_backward(torch.zeros((T, H, W), device="cuda"))
    ctx.close()
