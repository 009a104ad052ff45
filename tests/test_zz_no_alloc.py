"""GPU check of the allocation-free saliency entry point (sp_saliency_noalloc) through
the C-ABI: two calls in a row on one GPU, the second with a smaller frame, each against
saliency_forward of a context with the same parameters (the same kernels and launch
shapes, so the maps must agree bit for bit)."""
import ctypes
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


def _context_maps(torch, frames, pp):
    from paper_1008_0502_amd.api import Context
    H, W = frames.shape[1:3]
    ctx = Context(H, W, pp)
    S, C = ctx.saliency_forward(frames[1], frames[0], want_C=True)
    torch.cuda.synchronize()
    out = (S.cpu().numpy(), C.cpu().numpy(), ctx.geometry)
    ctx.close()
    return out


def test_noalloc_matches_saliency_forward_twice_smaller_second():
    torch = _torch()
    from paper_1008_0502_amd import _lib
    from paper_1008_0502_amd.api import Params
    lib = _lib.load()
    pp = Params()
    cases = [(480, 640, 11), (120, 160, 12)]
    for H, W, seed in cases:
        print(f"\n[case] sp_saliency_noalloc {H}x{W} seed {seed}", flush=True)
        sys.stdout.flush()
        fr, _ = synth.Clip(synth.single_ellipse_spec(H=H, W=W, T=2, seed=seed)).stack()
        frames = torch.from_numpy(fr).cuda()
        S_ref, C_ref, g = _context_maps(torch, frames, pp)
        # poison the outputs so a missing write shows
        S = torch.full((g.Hc, g.Wc), float("nan"), device="cuda")
        C = torch.full((8, g.Hc, g.Wc), float("nan"), device="cuda")
        cp = pp.to_c()
        rc = lib.sp_saliency_noalloc(ctypes.byref(cp), H, W, frames[1].data_ptr(), frames[0].data_ptr(),
                                     S.data_ptr(), C.data_ptr(), torch.cuda.current_stream().cuda_stream)
        _lib.check(rc, "sp_saliency_noalloc")
        torch.cuda.synchronize()
        s, c = S.cpu().numpy(), C.cpu().numpy()
        assert np.all(np.isfinite(s)) and np.all(np.isfinite(c))
        assert np.array_equal(s, S_ref), f"S differs at {H}x{W}: max {np.max(np.abs(s - S_ref))}"
        assert np.array_equal(c, C_ref), f"C differs at {H}x{W}: max {np.max(np.abs(c - C_ref))}"
        # first frame of a clip (no previous frame): the motion channel is zero
        S0 = torch.empty_like(S)
        rc = lib.sp_saliency_noalloc(ctypes.byref(cp), H, W, frames[0].data_ptr(), None, S0.data_ptr(), None,
                                     torch.cuda.current_stream().cuda_stream)
        _lib.check(rc, "sp_saliency_noalloc")
        from paper_1008_0502_amd.api import Context
        ctx = Context(H, W, pp)
        S0_ref, _ = ctx.saliency_forward(frames[0], None)
        torch.cuda.synchronize()
        assert np.array_equal(S0.cpu().numpy(), S0_ref.cpu().numpy())
        ctx.close()
