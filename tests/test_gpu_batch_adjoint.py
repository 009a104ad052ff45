"""Batched forward + adjoint (every stream's tape recorded inside the graph-replayed
step, one launch per reverse step over all streams, conspicuity recomputed a few frames
of every stream per launch) against the single-stream adjoint and the FP64 oracle.

Bars: each stream's gradient equals the single-stream path's bit for bit (the same
kernels and reduction orders), and is within 1e-3 per component (relative to
max(|g|, 1e-3 |g|_inf)) of the oracle's analytic FP64 gradient and, where computed, of
its central differences."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_1008_0502_amd import synth

import _oracle_pool
from _util import oracle_params

pytestmark = pytest.mark.gpu

W8 = (1.0, 0.8, 1.2, 0.9, 1.1, 0.7, 1.3, 1.0)


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


def _pkw(pp):
    op = oracle_params(pp)
    return {k: getattr(op, k) for k in op.__dataclass_fields__}


def _clips(specs):
    torch = _torch()
    fr, mk = [], []
    for kind, H, W, T, seed in specs:
        f, m = synth.Clip(_oracle_pool._spec(kind, H, W, T, seed)).stack()
        fr.append(torch.from_numpy(f).cuda())
        mk.append(torch.from_numpy(m).cuda())
    return fr, mk


def batch_grads(specs, pp, T, autotune=False, per_launch=1):
    """Batched forward of T steps (per_launch steps per graph launch), per-stream loss and
    adjoint; host copies."""
    torch = _torch()
    from paper_1008_0502_amd.api import Batch
    fr, mk = _clips(specs)
    sizes = [(H, W) for _, H, W, _, _ in specs]
    b = Batch(sizes, dataclasses.replace(pp, record_tape=T))
    tabs = [Batch.pointer_table([f[t] for f in fr]) for t in range(T)]
    if autotune:
        print("[tune] " + b.autotune(tabs[0], steps=2).strip().replace("\n", "; "), flush=True)
    b.reset()
    for t0 in range(0, T, per_launch):
        if per_launch == 1:
            b.step(tabs[t0])
        else:
            b.steps(tabs[t0:t0 + per_launch])
    loss, grads = b.mse_mask_loss(mk, T)
    gw, gq, gr = b.backward(grads)
    torch.cuda.synchronize()
    out = {"loss": loss.cpu().numpy().astype(np.float64), "gw": gw.cpu().numpy().astype(np.float64),
           "gq": gq.cpu().numpy().astype(np.float64), "gr": gr.cpu().numpy().astype(np.float64),
           "pi": [b.tape_priors(i, T).cpu().numpy() for i in range(len(specs))]}
    b.close()
    return out, fr, mk


def plain_grads(frames, masks, pp, T):
    torch = _torch()
    from paper_1008_0502_amd.api import Context
    H, W = frames.shape[1:3]
    ctx = Context(H, W, dataclasses.replace(pp, record_tape=T))
    out = ctx.run_clip(frames[:T])
    loss, grad = ctx.mse_mask_loss(out["pi"], masks[:T].contiguous())
    gw, gq, gr = ctx.saliency_backward(grad)
    torch.cuda.synchronize()
    res = (gw.cpu().numpy().astype(np.float64), float(gq.cpu()), float(gr.cpu()), float(loss.cpu()),
           out["pi"].cpu().numpy())
    ctx.close()
    return res


def check_stream(i, got, plain, ref, label):
    gw, gq, gr = got["gw"][i], got["gq"][i], got["gr"][i]
    pw, pq, pr, pl, ppi = plain
    assert np.array_equal(got["pi"][i], ppi), f"{label}: stream {i} priors differ from the single-stream path"
    assert np.array_equal(gw, pw) and gq == pq and gr == pr, \
        f"{label}: stream {i} gradient differs from the single-stream path: {gw} {gq} {gr} vs {pw} {pq} {pr}"
    assert got["loss"][i] == pytest.approx(pl, rel=1e-6)
    if ref is None:
        return
    full = np.concatenate([gw, [gq, gr]])
    an = np.concatenate([ref["gw"], [ref["gQ"], ref["gR"]]])
    e_an = grad_err(full, an)
    msg = f"[grad] {label} stream {i}: loss {got['loss'][i]:.6e} oracle {ref['L']:.6e}; vs analytic {e_an:.2e}"
    assert got["loss"][i] == pytest.approx(ref["L"], rel=1e-4)
    assert e_an <= 1e-3, msg
    if "fw" in ref:
        e_fd = grad_err(full, np.concatenate([ref["fw"], [ref["fQ"], ref["fR"]]]))
        msg += f"; vs FD {e_fd:.2e}"
        assert e_fd <= 1e-3, msg
    print(msg, flush=True)


def test_batch_adjoint_mixed_sizes_two_chunks():
    # three streams of three sizes; 24 steps = a chunk of 22 frames per stream and a ragged one of 2
    T = 24
    specs = [("single", 64, 80, T, 3), ("single", 48, 64, T, 8), ("single", 120, 160, T, 0)]
    banner(f"batched fwd+bwd: 64x80, 48x64, 160x120 x {T} steps vs single-stream adjoint and oracle (FD)")
    from paper_1008_0502_amd.api import Params
    pp = Params(weights=W8, q=2e-3, r=5e-2)
    got, fr, mk = batch_grads(specs, pp, T)
    jobs = [(k, H, W, T, s, _pkw(pp), np.array(W8), 2e-3, 5e-2, True) for k, H, W, _, s in specs]
    refs = _oracle_pool.run(_oracle_pool.grad_job, jobs)
    for i in range(len(specs)):
        check_stream(i, got, plain_grads(fr[i], mk[i], pp, T), refs[i], "mixed")


def test_batch_adjoint_with_several_steps_per_launch():
    # the tape recorded by sp_batch_steps (4 + 4 + 2 steps) equals the one of single steps
    T = 10
    specs = [("single", 64, 80, T, 3), ("single", 48, 64, T, 8)]
    banner(f"batched fwd+bwd: 64x80, 48x64 x {T} steps, four steps per graph launch vs one")
    from paper_1008_0502_amd.api import Params
    pp = Params(weights=W8, q=2e-3, r=5e-2)
    one, _, _ = batch_grads(specs, pp, T)
    four, _, _ = batch_grads(specs, pp, T, per_launch=4)
    for key in ("loss", "gw", "gq", "gr"):
        assert np.array_equal(one[key], four[key]), key
    for i in range(len(specs)):
        assert np.array_equal(one["pi"][i], four["pi"][i]), i


def test_batch_adjoint_bench_shape():
    # the batched fwd+bwd benchmark's shape: 16 streams of 640x480 (autotuned launch shapes);
    # 6 steps = a chunk of 4 frames per stream and a ragged one of 2
    T = 6
    specs = [("single", 480, 640, T, 6000 + i) for i in range(16)]
    banner(f"batched fwd+bwd: 16 x 640x480 x {T} steps, autotuned; every stream vs single-stream, "
           "two vs the oracle")
    from paper_1008_0502_amd.api import Params
    pp = Params(weights=W8)
    got, fr, mk = batch_grads(specs, pp, T, autotune=True)
    picks = [0, 11]
    jobs = [("single", 480, 640, T, 6000 + i, _pkw(pp), np.array(W8), 1e-3, 1e-1, False) for i in picks]
    refs = dict(zip(picks, _oracle_pool.run(_oracle_pool.grad_job, jobs)))
    for i in range(16):
        check_stream(i, got, plain_grads(fr[i], mk[i], pp, T), refs.get(i), "16x640x480")


def test_batch_autograd_function_and_stale_tape():
    banner("BatchSaliencyPrior: shared-parameter gradient = sum of the streams' oracle gradients; "
           "a second forward invalidates the first graph")
    torch = _torch()
    from paper_1008_0502_amd import SalpriorError
    from paper_1008_0502_amd.api import Batch, BatchSaliencyPrior, Params
    T = 8
    specs = [("single", 64, 80, T, 11), ("single", 48, 64, T, 12)]
    fr, mk = _clips(specs)
    pp = Params(record_tape=T)
    b = Batch([(64, 80), (48, 64)], pp)
    tabs = [Batch.pointer_table([f[t] for f in fr]) for t in range(T)]
    w = torch.tensor(W8, dtype=torch.float32, device="cuda", requires_grad=True)
    q = torch.tensor(1e-3, dtype=torch.float64, requires_grad=True)
    r = torch.tensor(1e-1, dtype=torch.float64, requires_grad=True)
    pis = BatchSaliencyPrior.apply(b, tabs, w, q, r)
    loss = sum(((p - m.float()) ** 2).mean() for p, m in zip(pis, mk))
    loss.backward()
    jobs = [(k, H, W, T, s, _pkw(Params()), np.array(W8), 1e-3, 1e-1, False) for k, H, W, _, s in specs]
    refs = _oracle_pool.run(_oracle_pool.grad_job, jobs)
    an = sum(np.concatenate([r_["gw"], [r_["gQ"], r_["gR"]]]) for r_ in refs)
    full = np.concatenate([w.grad.cpu().numpy(), [float(q.grad), float(r.grad)]])
    e = grad_err(full, an)
    print(f"[grad] batched autograd wrapper vs summed oracle gradients: {e:.2e}", flush=True)
    assert e <= 1e-3
    # a second forward on the same batch: the first graph's backward must refuse
    pis1 = BatchSaliencyPrior.apply(b, tabs, w, q.detach(), r.detach())
    pis2 = BatchSaliencyPrior.apply(b, tabs, w * 1.5, q.detach(), r.detach())
    with pytest.raises(RuntimeError, match="tape"):
        sum(p.sum() for p in pis1).backward()
    sum(p.sum() for p in pis2).backward()
    # C-ABI guards: a step beyond the tape, a backward of the wrong length, stale weights
    with pytest.raises(SalpriorError):
        b.step(tabs[0])
    g0 = [torch.zeros((T - 1, H, W), device="cuda") for H, W in b.sizes]
    with pytest.raises(SalpriorError):
        b.backward(g0)
    b.set_weights(W8, 1e-3, 1e-1)
    with pytest.raises(SalpriorError):
        b.backward([torch.zeros((T, H, W), device="cuda") for H, W in b.sizes])
    b.close()
