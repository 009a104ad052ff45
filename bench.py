#!/usr/bin/env python3
"""Throughput of the saliency -> Kalman prior -> MRF weight path on one MI355X.

Prints ONE JSON line.  A step is one 640x480 frame (config-1 generator, seed 2) through
the whole forward path: saliency_forward + prior_update + mrf_weights, inputs resident
in HBM.  Beside the headline it reports, on the same GPU:
  * saliency + prior only (no MRF capacities),
  * fwd+bwd: a 120-frame clip forward with tape, masked-MSE loss and the adjoint,
  * batched: 16 streams of 640x480 per step (one graph replay), and the mixed batch of
    64 streams (16 each of 160x120, 320x240, 640x480, 1280x720),
  * the roofline of the dominant kernel, timed live with HIP events on its stream,
  * the FP64 CPU oracle on a bounded sample (cpu_baseline).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
H, W, T_CLIP = 480, 640, 120


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def alg_bytes(kind: str, g, launches: int) -> float:
    """Algorithmic bytes moved by ONE launch of a kernel kind (each input and output
    array counted once) for geometry g of the plain step; per-kernel formulas."""
    Hh, Ww = g.H, g.W
    px = Hh * Ww
    sizes = g.sizes
    used = sorted({c for c, _ in g.pairs} | {s for _, s in g.pairs})
    pxl = lambda l: sizes[l][0] * sizes[l][1]
    pc = pxl(g.c_max)
    if kind == "k_rgb":
        return 3.0 * px
    if kind == "k_feat":
        return 6.0 * px + 16.0 * pxl(1)
    if kind == "k_down":
        tot = sum(16.0 * pxl(l) + 16.0 * pxl(l + 1) for l in range(1, g.top))
        return tot / max(1, g.top - 1)
    if kind == "k_gabor":
        return sum(20.0 * pxl(l) for l in used)
    if kind == "k_csstats":
        return sum(32.0 * pxl(l) for l in used)
    if kind == "k_csapply":
        return sum(32.0 * pxl(l) for l in used) + 32.0 * pc
    if kind == "k_consp":
        return 36.0 * pc
    if kind == "k_smax":
        return 4.0 * pc
    if kind == "k_kalman":
        return 12.0 * px + 4.0 * pc
    if kind == "k_mrf":
        return 31.0 * px
    return float("nan")


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("sp_kernels.hip", "sp_internal.h"):
        with open(os.path.join(ROOT, "paper_1008_0502_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(frames_np, budget_s: float):
    """The FP64 oracle, as it stands, on the first frames of the same clip."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:
        limiter = None
    import oracle as O
    p = O.OracleParams()
    geo = O.geometry(H, W, p)
    t0 = time.perf_counter()
    n = 0
    qs = []
    prev_pi = None
    K, P = O.kalman_gains(frames_np.shape[0], p.q, p.r)
    ring = O.border_mask(H, W, p.border)
    while n < frames_np.shape[0]:
        S, C = O.saliency(frames_np[n], frames_np[n - 1] if n else None, p)
        q, _ = O.observation(S, p, H, W, geo.c_max)
        if n == 0:
            pi = q.copy()
        else:
            f = O.blur(prev_pi)
            pi = f + K[n] * (q - f)
        pi[ring] = p.eps
        O.mrf_weights(frames_np[n], pi, p)
        prev_pi = pi
        n += 1
        if time.perf_counter() - t0 >= budget_s and n >= 2:
            break
    dt = time.perf_counter() - t0
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    return {"value": n / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} frames of the 640x480 clip (config-1 generator, seed 2): saliency, observation, "
                      f"Kalman update and MRF capacities in FP64 NumPy, one thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--skip", default="", help="comma list of legs to skip: bwd,batched,mixed,cpu,profile")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(independent streams would shard one group per GPU with no communication).",
              file=sys.stderr)
        sys.exit(2)
    skip = set(s for s in args.skip.split(",") if s)

    import numpy as np
    import torch
    from paper_1008_0502_amd import synth
    from paper_1008_0502_amd.api import Batch, Context, Params, profile_enable, profile_read

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log("generating the 640x480 clip")
    clip = synth.Clip(synth.config1_spec(H=H, W=W, T=T_CLIP, seed=2))
    frames_np, masks_np = clip.stack()
    frames = torch.from_numpy(frames_np).to(dev)
    masks = torch.from_numpy(masks_np).to(dev)

    # ------------------------------------------------------------ plain step
    ctx = Context(H, W, Params())
    g = ctx.geometry
    lib, h = ctx.lib, ctx._handle
    S = torch.empty((g.Hc, g.Wc), dtype=torch.float32, device=dev)
    P = torch.empty((H, W), dtype=torch.float32, device=dev)
    U = torch.empty((2, H, W), dtype=torch.float32, device=dev)
    PW = torch.empty((4, H, W), dtype=torch.float32, device=dev)
    B = torch.empty((1,), dtype=torch.float32, device=dev)
    fp = [frames[t].data_ptr() for t in range(T_CLIP)]
    sp, pp, up, pwp, bp = S.data_ptr(), P.data_ptr(), U.data_ptr(), PW.data_ptr(), B.data_ptr()
    stream = torch.cuda.current_stream().cuda_stream
    lib.sp_set_stream(h, stream)

    def step(i, mrf=True):
        t = i % T_CLIP
        rc = lib.saliency_forward(h, fp[t], fp[t - 1] if t else None, sp, None)
        rc |= lib.prior_update(h, sp, None, pp)
        if mrf:
            rc |= lib.mrf_weights(h, fp[t], pp, up, pwp, bp)
        if rc:
            raise RuntimeError(lib.sp_last_error().decode())

    def timed(fn, n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            fn(i)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    log(f"plain step: warmup {args.warmup}, timed {args.steps}")
    timed(step, args.warmup)
    dt = timed(step, args.steps)
    ms_step = dt / args.steps * 1e3
    value = args.steps / dt
    dt2 = timed(lambda i: step(i, mrf=False), args.steps)
    fps_sp = args.steps / dt2

    roof = None
    kernels = {}
    if "profile" not in skip:
        nprof = min(args.steps, 200)
        profile_enable(ctx, True)
        timed(step, nprof)
        prof = profile_read(ctx)
        profile_enable(ctx, False)
        for name, (ms, cnt) in prof.items():
            kernels[name] = {"avg_us": ms / cnt * 1e3, "launches_per_step": cnt / nprof,
                             "us_per_step": ms / nprof * 1e3}
        dom = max(prof.items(), key=lambda kv: kv[1][0])[0]
        ms, cnt = prof[dom]
        avg_s = ms / cnt * 1e-3
        ab = alg_bytes(dom, g, cnt)
        achieved = ab / avg_s / 1e9
        traffic = None
        tfile = os.path.join(ROOT, "profiles", "traffic_640x480.json")
        if os.path.exists(tfile):
            try:
                tj = json.load(open(tfile))
                if tj.get("source_hash") == source_hash() and dom in tj.get("kernels", {}):
                    traffic = tj["kernels"][dom]["hbm_bytes_per_launch"]
            except Exception:
                traffic = None
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": dom,
                "alg_bytes_per_launch": ab, "avg_launch_us": round(avg_s * 1e6, 3)}
    log(f"plain: {value:.1f} frames/s ({ms_step:.4f} ms/frame); saliency+prior only {fps_sp:.1f}")

    # ------------------------------------------------------------ fwd + bwd (config 3)
    fb = None
    if "bwd" not in skip:
        tctx = Context(H, W, Params(record_tape=T_CLIP))
        th = tctx._handle
        lib.sp_set_stream(th, stream)
        Ps = torch.empty((T_CLIP, H, W), dtype=torch.float32, device=dev)
        Ss = torch.empty((T_CLIP, g.Hc, g.Wc), dtype=torch.float32, device=dev)
        loss = torch.empty((1,), dtype=torch.float32, device=dev)
        grad = torch.empty_like(Ps)
        gw = torch.empty(8, device=dev)
        gq = torch.empty(1, device=dev)
        gr = torch.empty(1, device=dev)

        def clip_fb(_):
            lib.sp_reset(th)
            for t in range(T_CLIP):
                rc = lib.saliency_forward(th, fp[t], fp[t - 1] if t else None, Ss[t].data_ptr(), None)
                rc |= lib.prior_update(th, Ss[t].data_ptr(), None, Ps[t].data_ptr())
                if rc:
                    raise RuntimeError(lib.sp_last_error().decode())
            rc = lib.sp_mse_mask_loss(th, Ps.data_ptr(), masks.data_ptr(), T_CLIP, loss.data_ptr(), grad.data_ptr())
            rc |= lib.saliency_backward(th, grad.data_ptr(), T_CLIP, gw.data_ptr(), gq.data_ptr(), gr.data_ptr())
            if rc:
                raise RuntimeError(lib.sp_last_error().decode())

        log("fwd+bwd clip")
        timed(clip_fb, 1)
        reps = 3
        dtb = timed(clip_fb, reps)
        fb = {"frames_per_s": reps * T_CLIP / dtb, "ms_per_clip": dtb / reps * 1e3, "clip_frames": T_CLIP,
              "loss": float(loss.item())}
        tctx.close()
        log(f"fwd+bwd: {fb['frames_per_s']:.1f} frames/s")

    # ------------------------------------------------------------ batched 16 x 640x480
    def run_batch(sizes, seeds, n_frames, steps, warm):
        bframes = []
        for (hh, ww), sd in zip(sizes, seeds):
            f, _ = synth.Clip(synth.config1_spec(H=hh, W=ww, T=n_frames, seed=sd)).stack()
            bframes.append(torch.from_numpy(f).to(dev))
        tables = [Batch.pointer_table([bf[t] for bf in bframes]) for t in range(n_frames)]
        bt = Batch(sizes, Params())
        fn = lambda i: bt.step(tables[i % n_frames])
        timed(fn, warm)
        dtx = timed(fn, steps)
        bt.close()
        return {"frames_per_s": len(sizes) * steps / dtx, "ms_per_step": dtx / steps * 1e3, "streams": len(sizes),
                "steps": steps}

    batched = mixed = None
    if "batched" not in skip:
        log("batched 16 x 640x480")
        batched = run_batch([(H, W)] * 16, [6000 + i for i in range(16)], 8, 60, 5)
        log(f"batched: {batched['frames_per_s']:.1f} frames/s")
    if "mixed" not in skip:
        log("batched 64 mixed streams")
        sizes = [(120, 160)] * 16 + [(240, 320)] * 16 + [(480, 640)] * 16 + [(720, 1280)] * 16
        mixed = run_batch(sizes, [1000 + i for i in range(64)], 4, 30, 3)
        mixed["mpx_per_s"] = sum(hh * ww for hh, ww in sizes) * mixed["frames_per_s"] / 64 / 1e6
        log(f"mixed: {mixed['frames_per_s']:.1f} frames/s")

    cpu = None
    if "cpu" not in skip:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(frames_np, args.cpu_seconds)

    out = {
        "metric": "frames/s saliency+Kalman prior at 640x480 (fwd, fwd+bwd, batched); HBM GB/s",
        "value": round(value, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "640x480 single stream, config-1 generator seed 2, 120-frame clip cycled; "
                               "per step saliency_forward + prior_update + mrf_weights",
                   "H": H, "W": W, "depth": g.depth, "pairs": g.pairs, "c_max": g.c_max,
                   "parallelism": "single GPU"},
        "fwd_saliency_prior_frames_per_s": round(fps_sp, 2),
        "fwd_bwd": fb,
        "batched_16x640x480": batched,
        "batched_mixed64": mixed,
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "source_hash": source_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
