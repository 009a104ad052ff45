"""Batched step against the FP64 oracle at the benchmark's configuration, and every
launch-shape candidate of the autotuner against one another.

Bars (as for the plain calls): S, each conspicuity channel and the prior within 1e-4
peak-normalised per frame; unary and pairwise capacities stage-isolated (the oracle's
capacities of the GPU prior) within 1e-5; beta within 1e-6 relative.  Launch shapes
never change results, so every candidate must equal the reference bit for bit."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1008_0502_amd import synth

import _oracle_pool
from _util import oracle_params, peak_rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def banner(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def _pkw(pp):
    op = oracle_params(pp)
    return {k: getattr(op, k) for k in op.__dataclass_fields__}


def _copy(ptr, shape):
    import torch
    out = torch.empty(shape, dtype=torch.float32, device="cuda")
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    assert hip.hipMemcpy(out.data_ptr(), ptr, out.numel() * 4, 3) == 0
    return out.cpu().numpy()


def _run_batch(b, sizes, clips, T, geo):
    """Steps the batch over T frames; returns per stream the host copies of S, C, pi,
    unary, pairwise and beta of every step."""
    torch = _torch()
    outs = [{k: [] for k in ("S", "C", "pi", "unary", "pairwise", "beta")} for _ in sizes]
    for t in range(T):
        b.step(b.pointer_table([c[t] for c in clips]))
        torch.cuda.synchronize()
        for i, (H, W) in enumerate(sizes):
            Hc, Wc = geo[i]
            pS, pU, pPW, pB = b.output_pointers(i)
            prior = ctypes.c_void_p()
            assert b.lib.sp_batch_prior(b._handle, i, ctypes.byref(prior)) == 0
            outs[i]["S"].append(_copy(pS, (Hc, Wc)))
            outs[i]["C"].append(_copy(b.consp_pointer(i), (8, Hc, Wc)))
            outs[i]["pi"].append(_copy(prior.value, (H, W)))
            if pU is not None:
                outs[i]["unary"].append(_copy(pU, (2, H, W)))
                outs[i]["pairwise"].append(_copy(pPW, (4, H, W)))
                outs[i]["beta"].append(_copy(pB, (1,)))
    return [{k: np.stack(v) for k, v in o.items() if v} for o in outs]


def _geometry(sizes, pp):
    from paper_1008_0502_amd.api import Context
    geo = []
    for (H, W) in sizes:
        c = Context(H, W, pp)
        geo.append((c.geometry.Hc, c.geometry.Wc))
        c.close()
    return geo


def test_bench_batch_with_autotune_vs_oracle():
    sizes = [(480, 640)] * 16 + [(120, 160), (240, 320), (720, 1280)]
    seeds = [6000 + i for i in range(16)] + [7001, 7002, 7003]
    T = 4
    banner(f"batch of 16 x 640x480 + 160x120 + 320x240 + 1280x720 with MRF, autotuned, {T} steps vs oracle")
    torch = _torch()
    from paper_1008_0502_amd.api import Batch, Params
    pp = Params()
    clips = [torch.from_numpy(synth.Clip(synth.single_ellipse_spec(H=H, W=W, T=T, seed=s)).stack()[0]).cuda()
             for (H, W), s in zip(sizes, seeds)]
    geo = _geometry(sizes, pp)
    b = Batch(sizes, pp, mrf=True, consp=True)
    rep = b.autotune(b.pointer_table([c[0] for c in clips]), steps=3)
    print("[tune] " + rep.strip().replace("\n", "; "), flush=True)
    gpu = _run_batch(b, sizes, clips, T, geo)
    b.close()
    jobs = [("single", H, W, T, s, _pkw(pp)) for (H, W), s in zip(sizes, seeds)]
    print("[oracle] running the oracle on every stream in worker processes", flush=True)
    refs = _oracle_pool.run(_oracle_pool.clip_job, jobs)
    mjobs = [("single", H, W, T, s, _pkw(pp), g["pi"]) for (H, W), s, g in zip(sizes, seeds, gpu)]
    mrefs = _oracle_pool.run(_oracle_pool.mrf_job, mjobs)
    worst = {}
    for i, ((H, W), g, r, m) in enumerate(zip(sizes, gpu, refs, mrefs)):
        for t in range(T):
            errs = {"S": peak_rel_err(g["S"][t], r["S"][t]), "pi": peak_rel_err(g["pi"][t], r["pi"][t])}
            for k in range(8):
                errs[f"C{k}"] = peak_rel_err(g["C"][t][k], r["C"][t][k])
            errs["unary"] = peak_rel_err(g["unary"][t], m["unary"][t])
            errs["pairwise"] = peak_rel_err(g["pairwise"][t], m["pairwise"][t])
            for key, e in errs.items():
                worst[key] = max(worst.get(key, 0.0), e)
                bar = 1e-5 if key in ("unary", "pairwise") else TOL
                assert e <= bar, f"stream {i} ({H}x{W}) t={t}: {key} error {e:.3e} > {bar}"
            assert float(g["beta"][t][0]) == pytest.approx(m["beta"][t], rel=1e-6, abs=1e-30), (i, t)
    print("[parity] batch worst peak-normalised error per output: "
          + ", ".join(f"{k}={v:.2e}" for k, v in sorted(worst.items())), flush=True)


def test_every_launch_shape_candidate_is_bitwise_identical():
    sizes = [(480, 640), (480, 640), (240, 320)]
    seeds = [6100, 6101, 6102]
    T = 3
    banner("batch of 2 x 640x480 + 320x240 with MRF: 24 forced launch shapes, bitwise against one checked by the oracle")
    torch = _torch()
    from paper_1008_0502_amd.api import Batch, Context, Params
    pp = Params()
    clips = [torch.from_numpy(synth.Clip(synth.single_ellipse_spec(H=H, W=W, T=T, seed=s)).stack()[0]).cuda()
             for (H, W), s in zip(sizes, seeds)]
    geo = _geometry(sizes, pp)
    b = Batch(sizes, pp, mrf=True, consp=True)
    b.set_tune(32, False, 2)
    ref = _run_batch(b, sizes, clips, T, geo)
    r = _oracle_pool.run(_oracle_pool.clip_job, [("single", 480, 640, T, seeds[0], _pkw(pp))])[0]
    for t in range(T):
        for key in ("S", "pi"):
            e = peak_rel_err(ref[0][key][t], r[key][t])
            assert e <= TOL, (key, t, e)
        for k in range(8):
            assert peak_rel_err(ref[0]["C"][t][k], r["C"][t][k]) <= TOL, (k, t)
    for tw in (16, 32, 64):
        for xcd in (False, True):
            for nc in (1, 2, 4, 8):
                b.set_tune(tw, xcd, nc)
                b.reset()
                got = _run_batch(b, sizes, clips, T, geo)
                for i in range(len(sizes)):
                    for key, v in ref[i].items():
                        assert np.array_equal(got[i][key], v), f"tile {tw} xcd {xcd} nc {nc}: stream {i} {key}"
    b.close()
    # the plain context under forced shapes gives the same priors as the batch
    for tw, xcd, nc in ((16, True, 8), (64, False, 1), (32, True, 4)):
        ctx = Context(480, 640, pp)
        ctx.set_tune(tw, xcd, nc)
        out = ctx.run_clip(clips[0], with_mrf=True, want_C=True)
        torch.cuda.synchronize()
        assert np.array_equal(out["pi"].cpu().numpy(), ref[0]["pi"]), (tw, xcd, nc)
        assert np.array_equal(out["S"].cpu().numpy(), ref[0]["S"]), (tw, xcd, nc)
        assert np.array_equal(out["C"].cpu().numpy(), ref[0]["C"]), (tw, xcd, nc)
        ctx.close()
