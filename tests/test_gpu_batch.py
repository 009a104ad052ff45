"""Batched step (many streams of uneven size, one graph replay per step) vs the plain
per-stream calls: the same kernels on the same tiles, so results must be bitwise
equal, on every replay, with eager work and synchronisations between replays."""
import sys

import numpy as np
import pytest

from paper_1008_0502_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_batched_step_equals_plain_streams():
    print("\n[case] batch of 5 streams (160x120, 80x64, 320x240, 131x97, 120x160), 7 steps", flush=True)
    torch = _torch()
    from paper_1008_0502_amd.api import Batch, Context, Params
    sizes = [(120, 160), (64, 80), (240, 320), (97, 131), (120, 160)]
    T = 7
    clips = []
    for i, (H, W) in enumerate(sizes):
        spec = synth.single_ellipse_spec(H=H, W=W, T=T, seed=1000 + i)
        spec.axes = (min(15.0, W / 4), min(10.0, H / 4))
        f, _ = synth.Clip(spec).stack()
        clips.append(torch.from_numpy(f).cuda())
    pp = Params()
    # plain reference, stream by stream
    ref = []
    for (H, W), fr in zip(sizes, clips):
        ctx = Context(H, W, pp)
        ref.append(ctx.run_clip(fr)["pi"].cpu().numpy())
        ctx.close()
    b = Batch(sizes, pp)
    outs = [torch.empty((T, H, W), dtype=torch.float32, device="cuda") for (H, W) in sizes]
    for rep in range(2):
        b.reset()
        for t in range(T):
            rgb = Batch.pointer_table([fr[t] for fr in clips])
            dst = Batch.pointer_table([o[t] for o in outs])
            b.step(rgb, dst)
            # eager work and a synchronisation between replays
            junk = torch.ones(1000, device="cuda").sum()
            torch.cuda.synchronize()
            for i in range(len(sizes)):
                got = outs[i][t].cpu().numpy()
                assert np.array_equal(got, ref[i][t]), f"rep {rep} step {t} stream {i} differs"
    b.close()


def test_batch_of_one_large_stream_and_prior_pointer():
    print("\n[case] batch with a 1280x720 stream and a 160x120 stream, 3 steps", flush=True)
    torch = _torch()
    import ctypes
    from paper_1008_0502_amd.api import Batch, Context, Params
    sizes = [(720, 1280), (120, 160)]
    clips = [torch.from_numpy(synth.Clip(synth.single_ellipse_spec(H=H, W=W, T=3, seed=7 + i)).stack()[0]).cuda()
             for i, (H, W) in enumerate(sizes)]
    pp = Params()
    b = Batch(sizes, pp)
    for t in range(3):
        b.step(Batch.pointer_table([c[t] for c in clips]))
    torch.cuda.synchronize()
    ptr = ctypes.c_void_p()
    assert b.lib.sp_batch_prior(b._handle, 0, ctypes.byref(ptr)) == 0
    ctx = Context(720, 1280, pp)
    ref = ctx.run_clip(clips[0])["pi"][2]
    out = torch.empty_like(ref)
    # copy the batch's current prior of stream 0 with a device-to-device hipMemcpy
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    assert hip.hipMemcpy(out.data_ptr(), ptr.value, ref.numel() * 4, 3) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    ctx.close()
    b.close()


def _copy_from(ptr, like):
    import ctypes
    import torch
    out = torch.empty_like(like)
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    assert hip.hipMemcpy(out.data_ptr(), ptr, out.numel() * out.element_size(), 3) == 0
    return out


def test_batched_step_with_mrf_equals_fused_plain_step():
    print("\n[case] batch with MRF capacities (3 streams) vs the fused plain step, 4 steps", flush=True)
    torch = _torch()
    from paper_1008_0502_amd.api import Batch, Context, Params
    sizes = [(240, 320), (120, 160), (97, 131)]
    T = 4
    clips = []
    for i, (H, W) in enumerate(sizes):
        spec = synth.three_ellipse_spec(H=H, W=W, T=T, seed=40 + i)
        clips.append(torch.from_numpy(synth.Clip(spec).stack()[0]).cuda())
    pp = Params()
    ctxs = [Context(H, W, pp) for (H, W) in sizes]
    b = Batch(sizes, pp, mrf=True)
    for t in range(T):
        b.step(Batch.pointer_table([c[t] for c in clips]))
        torch.cuda.synchronize()
        for i, ((H, W), ctx) in enumerate(zip(sizes, ctxs)):
            g = ctx.geometry
            U = torch.empty((2, H, W), device="cuda")
            PW = torch.empty((4, H, W), device="cuda")
            B = torch.empty((1,), device="cuda")
            S, P = ctx.step(clips[i][t], clips[i][t - 1] if t else None, unary_out=U, pairwise_out=PW, beta_out=B)
            torch.cuda.synchronize()
            pS, pU, pPW, pB = b.output_pointers(i)
            assert torch.equal(_copy_from(pS, S), S), (t, i, "S")
            assert torch.equal(_copy_from(pU, U), U), (t, i, "unary")
            assert torch.equal(_copy_from(pPW, PW), PW), (t, i, "pairwise")
            assert torch.equal(_copy_from(pB, B), B), (t, i, "beta")
    for c in ctxs:
        c.close()
    b.close()


def test_autotuner_keeps_results_identical():
    print("\n[case] autotuned batch and context give the same priors as untuned ones", flush=True)
    torch = _torch()
    from paper_1008_0502_amd.api import Batch, Context, Params
    sizes = [(240, 320), (120, 160), (240, 320)]
    T = 3
    clips = [torch.from_numpy(synth.Clip(synth.single_ellipse_spec(H=H, W=W, T=T, seed=70 + i)).stack()[0]).cuda()
             for i, (H, W) in enumerate(sizes)]
    pp = Params()
    ref = []
    for (H, W), c in zip(sizes, clips):
        ctx = Context(H, W, pp)
        ref.append(ctx.run_clip(c)["pi"].cpu().numpy())
        ctx.close()
    b = Batch(sizes, pp)
    rep = b.autotune(Batch.pointer_table([c[0] for c in clips]), steps=2)
    print(rep, flush=True)
    assert "chosen" in rep
    outs = [torch.empty((T, H, W), device="cuda") for (H, W) in sizes]
    for t in range(T):
        b.step(Batch.pointer_table([c[t] for c in clips]), Batch.pointer_table([o[t] for o in outs]))
    torch.cuda.synchronize()
    for i in range(len(sizes)):
        got = outs[i].cpu().numpy()
        assert np.array_equal(got, ref[i]), (i, float(np.abs(got - ref[i]).max()))
    b.close()
    ctx = Context(240, 320, pp)
    print(ctx.autotune(clips[0][1], clips[0][0], steps=3), flush=True)
    got = ctx.run_clip(clips[0])["pi"].cpu().numpy()
    assert np.array_equal(got, ref[0]), float(np.abs(got - ref[0]).max())
    ctx.close()


def test_several_steps_per_graph_launch_equal_single_steps():
    print("\n[case] sp_batch_steps (3 steps, 3 more with other tables, then 2) vs sp_batch_step, 3 streams with MRF",
          flush=True)
    torch = _torch()
    import ctypes
    from paper_1008_0502_amd.api import Batch, Params
    sizes = [(240, 320), (120, 160), (97, 131)]
    T = 8
    clips = [torch.from_numpy(synth.Clip(synth.three_ellipse_spec(H=H, W=W, T=T, seed=90 + i)).stack()[0]).cuda()
             for i, (H, W) in enumerate(sizes)]
    tabs = [Batch.pointer_table([c[t] for c in clips]) for t in range(T)]
    pp = Params()
    multi = Batch(sizes, pp, mrf=True)
    single = Batch(sizes, pp, mrf=True)

    def state(b, i, H, W):
        ptr = ctypes.c_void_p()
        assert b.lib.sp_batch_prior(b._handle, i, ctypes.byref(ptr)) == 0
        like = torch.empty((H, W), device="cuda")
        pS, pU, pPW, pB = b.output_pointers(i)
        return [_copy_from(ptr.value, like), _copy_from(pU, torch.empty((2, H, W), device="cuda")),
                _copy_from(pPW, torch.empty((4, H, W), device="cuda")), _copy_from(pB, torch.empty((1,), device="cuda"))]

    for grp in ([0, 1, 2], [3, 4, 5], [6, 7]):
        multi.steps([tabs[k] for k in grp])
        for k in grp:
            single.step(tabs[k])
        torch.cuda.synchronize()
        for i, (H, W) in enumerate(sizes):
            for name, x, y in zip(("prior", "unary", "pairwise", "beta"), state(multi, i, H, W),
                                  state(single, i, H, W)):
                assert torch.equal(x, y), (grp, i, name)
    multi.close()
    single.close()


def test_new_variances_reach_a_reused_several_step_graph():
    print("\n[case] sp_batch_steps with the same tables before and after sp_batch_set_weights, 2 streams", flush=True)
    torch = _torch()
    import ctypes
    from paper_1008_0502_amd.api import Batch, Params
    sizes = [(120, 160), (97, 131)]
    clips = [torch.from_numpy(synth.Clip(synth.three_ellipse_spec(H=H, W=W, T=2, seed=140 + i)).stack()[0]).cuda()
             for i, (H, W) in enumerate(sizes)]
    tabs = [Batch.pointer_table([c[t] for c in clips]) for t in range(2)]
    pp = Params()
    multi, single, kept = (Batch(sizes, pp) for _ in range(3))

    def prior(b, i, H, W):
        ptr = ctypes.c_void_p()
        assert b.lib.sp_batch_prior(b._handle, i, ctypes.byref(ptr)) == 0
        return _copy_from(ptr.value, torch.empty((H, W), device="cuda"))

    multi.steps(tabs)
    kept.steps(tabs)
    for t in tabs:
        single.step(t)
    # the Kalman variances live in each step's first graph node; the same tables again must
    # still run with the new ones (the weights of the maps are changed as well)
    w2 = [1.0, 0.5, 0.5, 1.0, 0.25, 0.25, 0.25, 0.25]
    for b in (multi, single):
        b.set_weights(w2, 0.5 * pp.q + 1e-3, 4.0 * pp.r)
    multi.steps(tabs)
    kept.set_weights(list(pp.weights), pp.q, pp.r)
    kept.steps(tabs)
    for t in tabs:
        single.step(t)
    torch.cuda.synchronize()
    for i, (H, W) in enumerate(sizes):
        a, s, k = prior(multi, i, H, W), prior(single, i, H, W), prior(kept, i, H, W)
        assert torch.equal(a, s), i
        assert not torch.equal(a, k), i   # the change is visible at all
    for b in (multi, single, kept):
        b.close()
