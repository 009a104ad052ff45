#!/usr/bin/env python3
"""Throughput of the saliency -> Kalman prior -> MRF weight path on one MI355X.

Prints ONE JSON line.  A step is one replay of the batched step over 16 streams of
640x480 frames (single-ellipse generator, seeds 6000+i): every stream's saliency map, Kalman
prior and MRF capacities, each phase one launch over all streams, inputs resident in
HBM; value = frames per second over the 16 streams.  Beside the headline it reports, on
the same GPU:
  * plain: one 640x480 stream, one frame per sp_step call (and through the three
    separate calls, and saliency + prior only),
  * fwd+bwd: a 120-frame 640x480 clip forward with tape, masked-MSE loss and adjoint,
    on one stream and batched over 16 streams (the batched fwd+bwd workload),
  * the mixed batch of 64 streams (16 each of 160x120, 320x240, 640x480, 1280x720),
  * the roofline of the step's dominant kernel, timed live with HIP events,
  * the named single-stream workloads: the single ellipse at 160x120, the three
    ellipses at 320x240 with MRF capacities, the five ellipses at 1920x1080, and the
    single ellipse at 352x288, 480x384 and 640x512,
  * the FP64 CPU oracle on a bounded sample (cpu_baseline), single-threaded and with one
    process per stream.
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


def tail_source(g, lo=1, src=8192, alt=4096, hb=4096, vcap=8192):
    """Source level of the tail pyramid job (mirror of the library's rule)."""
    used = {c for c, _ in g.pairs} | {s for _, s in g.pairs}
    sz = lambda l: g.sizes[l][0] * g.sizes[l][1]
    for L0 in range(lo, g.top):
        ok = sz(L0) <= src
        for l in range(L0 + 1, g.top + 1):
            ok &= sz(l) <= (alt if (l - L0) % 2 else src)
            ok &= g.sizes[l - 1][0] * g.sizes[l][1] <= hb
            if l in used:
                ok &= 4 * sz(l) <= vcap
            if not ok:
                break
        if ok:
            return L0
    return g.top


def alg_bytes_per_stream(g, mrf: bool, prior_copy: bool):
    """Algorithmic bytes one step moves per stream, per kernel (each array read or
    written once), summed over that kernel's launches in the step."""
    px = g.H * g.W
    used = sorted({c for c, _ in g.pairs} | {s for _, s in g.pairs})
    pxl = lambda l: g.sizes[l][0] * g.sizes[l][1]
    pc = pxl(g.c_max)
    L0 = tail_source(g)
    mid = sum(16.0 * pxl(j) + 16.0 * pxl(j + 1) + (20.0 * pxl(j) if j in used else 0.0) for j in range(1, L0))
    tail = 0.0
    if L0 < g.top:
        tail += 16.0 * pxl(L0) + sum(16.0 * pxl(l) for l in range(L0 + 1, g.top + 1))
        tail += sum(4.0 * pxl(L0) + 16.0 * pxl(l) for l in used if l > L0)
    if L0 in used:
        tail += 20.0 * pxl(L0)
    lev = sum(32.0 * pxl(l) for l in used)
    npairs = len(g.pairs)
    return {
        "k_rgb": 3.0 * px,
        "k_feat": 6.0 * px + 16.0 * pxl(1) + (16.0 * px if mrf else 0.0),
        "k_pyr": mid,
        "k_pyr_tail": tail,
        "k_csstats": lev,
        "k_csapply": lev + 32.0 * pc,
        # reduced-map path (every centre at c_max or one level below): maps, partials and
        # reductions to c_max in one pass, then their normalised sum
        "k_csg": lev + 32.0 * npairs * pc,
        "k_csmix": 32.0 * npairs * pc + 32.0 * pc,
        "k_consp": 36.0 * pc,
        "k_kalman": 4.0 * pc + 8.0 * px + (4.0 * px if prior_copy else 0.0) + (8.0 * px if mrf else 0.0),
    }


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("sp_kernels.hip", "sp_gmm.hip", "sp_mincut.hip", "sp_pixadj.hip", "sp_device.h", "sp_internal.h",
              "sp_kernels.h",
              "sp_host.cpp"):
        with open(os.path.join(ROOT, "paper_1008_0502_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_info():
    """CPU model and the number of host threads this process may use."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


def _gen_clip(args):
    from paper_1008_0502_amd import synth
    kind, H, W, T, seed = args
    fn = {"single": synth.single_ellipse_spec, "three": synth.three_ellipse_spec,
          "five": synth.five_ellipse_spec}[kind]
    return synth.Clip(fn(H=H, W=W, T=T, seed=seed)).stack()


def gen_clips(jobs, workers=8):
    """Seeded clips drawn in worker processes (the generator holds no method arithmetic)."""
    import multiprocessing as mp
    if len(jobs) == 1:
        return [_gen_clip(jobs[0])]
    with mp.get_context("spawn").Pool(min(workers, len(jobs))) as pool:
        return pool.map(_gen_clip, jobs)


def _oracle_stream(args):
    """One stream of the oracle for the parallel baseline: frames of the clip until the
    deadline (saliency, observation, Kalman update), single-threaded; frames are drawn
    one at a time (a small share of the oracle's time per frame)."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except Exception:
        pass
    import oracle as O
    from paper_1008_0502_amd import synth
    H, W, T, seed, deadline = args
    clip = synth.Clip(synth.single_ellipse_spec(H=H, W=W, T=T, seed=seed))
    p = O.OracleParams()
    geo = O.geometry(H, W, p)
    K, _ = O.kalman_gains(T, p.q, p.r)
    ring = O.border_mask(H, W, p.border)
    n, prev, prev_rgb = 0, None, None
    while n < T and time.time() < deadline:
        rgb, _ = clip.frame(n)
        S, _ = O.saliency(rgb, prev_rgb, p)
        q, _ = O.observation(S, p, H, W, geo.c_max)
        if n == 0:
            pi = q.copy()
        else:
            f = O.blur(prev)
            pi = f + K[n] * (q - f)
        pi[ring] = p.eps
        prev, prev_rgb = pi, rgb
        n += 1
    return n


def _warm_oracle(_):
    import oracle  # noqa: F401
    from paper_1008_0502_amd import synth  # noqa: F401
    return os.getpid()


def cpu_baseline_parallel(streams: int, budget_s: float):
    """The oracle with one process per stream (16 streams of 640x480, seeds 6000+i) over
    min(streams, host threads) processes; frames finished by all processes in the budget."""
    import multiprocessing as mp
    _, nthreads = cpu_info()
    procs = max(1, min(streams, nthreads))
    with mp.get_context("spawn").Pool(procs) as pool:
        pool.map(_warm_oracle, range(procs))   # interpreter start and imports before the window
        t0 = time.time()
        jobs = [(H, W, T_CLIP, 6000 + i, t0 + budget_s) for i in range(streams)]
        counts = pool.map(_oracle_stream, jobs, chunksize=1)
        dt = time.time() - t0
    return {"value": sum(counts) / dt, "unit": "frames/s", "cores": procs, "kind": "oracle",
            "sample": f"{sum(counts)} frames over {streams} streams of 640x480 (single-ellipse generator, seeds "
                      f"6000+i): saliency, observation and Kalman update in FP64 NumPy, one single-threaded "
                      f"process per stream on {procs} processes, {dt:.1f} s"}


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
    model, nthreads = cpu_info()
    return {"value": n / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} frames of the 640x480 clip (single-ellipse generator, seed 2): saliency, observation, "
                      f"Kalman update and MRF capacities in FP64 NumPy, one thread, {dt:.1f} s",
            "cpu_model": model, "host_threads": nthreads}


CALIB = ((0, 512 << 20), (1, 96 << 20), (2, 16 << 20))   # (access form, bytes) of the calibration copies
VALU_ISSUE_PER_S = 256 * 2.4e9   # wave64 VALU instructions per second: one per CU per clock (no packed FP32)
KERNEL_KEYS = {"k_rgb": "k_rgb", "k_feat": "k_feat", "k_csstats": "k_csstats", "k_csfinal": "k_csfinal",
               "k_csapply": "k_csapply", "k_consp": "k_consp", "k_kalman": "k_kalman", "k_csg": "k_csg",
               "k_csg1": "k_csg", "k_csmix": "k_csmix", "k_calib": "k_calib"}


def _short_kernel(raw: str):
    import re
    short = re.sub(r"\(anonymous namespace\)::", "", raw)
    short = re.sub(r"\(.*\)$", "", short).replace("void ", "").replace(" ", "")
    if short.startswith("k_pyr<"):
        return "k_pyr_tail" if short.startswith("k_pyr<true") else "k_pyr"
    return KERNEL_KEYS.get(re.sub(r"<.*>$", "", short))


def _per_kernel(db: str, counter: str):
    """{kernel: [value per dispatch, in dispatch order]} of one counter of a rocprofv3 database."""
    import sqlite3
    con = sqlite3.connect(db)
    cur = con.cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(counters_collection)").fetchall()]
    order = " order by dispatch_id" if "dispatch_id" in cols else ""
    rows = cur.execute(f"select kernel_name, value from counters_collection where counter_name = ?{order}",
                       (counter,)).fetchall()
    out = {}
    for name, val in rows:
        key = _short_kernel(name)
        if key is not None:
            out.setdefault(key, []).append(float(val))
    return out


def _calib_factors(vals):
    """Scale factor (true bytes / counted bytes) of each calibration access form: the k_calib
    dispatches are told apart by their byte counts (disjoint ranges for factors 0.5..2)."""
    out = {}
    for mode, nbytes in CALIB:
        cands = [v for v in vals if 0.4 * nbytes <= v * 1024.0 <= 2.5 * nbytes]
        if cands:
            out[mode] = nbytes / (max(cands) * 1024.0)
    return out


def pmc_summarize(fetch_db: str, write_db: str, valu_db=None) -> None:
    """HBM traffic (and VALU instructions) per launch of each kernel of the batched step from
    rocprofv3 --pmc runs of --pmc-workload: FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    each scaled by what the counter reads for the library's own calibration copies of a
    known byte count; SQ_INSTS_VALU (wave instructions per dispatch) when given."""
    fetch = _per_kernel(fetch_db, "FETCH_SIZE")
    write = _per_kernel(write_db, "WRITE_SIZE")
    valu = _per_kernel(valu_db, "SQ_INSTS_VALU") if valu_db else {}
    kf = _calib_factors(fetch.get("k_calib", []))
    kw = _calib_factors(write.get("k_calib", []))
    forms = {0: "dword", 1: "dwordx4", 2: "global_load_lds dword"}
    fs, ws = kf.get(0, 1.0), kw.get(0, 1.0)
    kernels = {}
    for key in sorted(set(fetch) | set(write)):
        if key == "k_calib":
            continue
        f = fetch.get(key, [0.0])
        w = write.get(key, [0.0])
        fr = sum(f) / len(f) * 1024.0
        wr = sum(w) / len(w) * 1024.0
        rec = {"fetch_bytes_raw": fr, "write_bytes_raw": wr, "fetch_bytes_per_launch": fr * fs,
               "write_bytes_per_launch": wr * ws, "hbm_bytes_per_launch": fr * fs + wr * ws}
        if key in valu:
            v = valu[key]
            rec["valu_insts_per_launch"] = sum(v) / len(v)
        kernels[key] = rec
    out = {"source_hash": source_hash(), "workload": "batched step, 16 streams of 640x480, MRF on",
           "calibration": {"copies": {forms[m]: n for m, n in CALIB},
                           "fetch_scale": {forms[m]: v for m, v in kf.items()},
                           "write_scale": {forms[m]: v for m, v in kw.items()},
                           "applied": "dword"},
           "valu_issue_per_s": VALU_ISSUE_PER_S, "kernels": kernels}
    path = os.environ.get("SALPRIOR_TRAFFIC_OUT", os.path.join(ROOT, "profiles", "traffic_batched16_640x480.json"))
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def roofline_of(prof, bytes_per_step, n_steps, counters=True):
    """Roofline record of the kernel with the largest device time per step.  The counter
    traffic (taken on the batched workload) is attached only when counters is set."""
    dom = max(prof.items(), key=lambda kv: kv[1][0])[0]
    ms, cnt = prof[dom]
    avg_s = ms / cnt * 1e-3
    per_launch = bytes_per_step[dom] / (cnt / n_steps)
    achieved = per_launch / avg_s / 1e9
    traffic, valu = None, None
    tfile = os.path.join(ROOT, "profiles", "traffic_batched16_640x480.json")
    if counters and os.path.exists(tfile):
        try:
            tj = json.load(open(tfile))
            if tj.get("source_hash") == source_hash() and dom in tj.get("kernels", {}):
                rec = tj["kernels"][dom]
                traffic = rec["hbm_bytes_per_launch"]
                if "valu_insts_per_launch" in rec:
                    need = rec["valu_insts_per_launch"] / VALU_ISSUE_PER_S
                    valu = {"insts_per_launch": rec["valu_insts_per_launch"], "issue_s_at_peak": need,
                            "frac": round(need / avg_s, 4)}
        except Exception:
            traffic, valu = None, None
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "valu": valu, "kernel": dom,
            "alg_bytes_per_launch": per_launch, "avg_launch_us": round(avg_s * 1e6, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--skip", default="",
                    help="comma list of legs to skip: batched,plain,bwd,bwd_batched,mixed,configs,extras,cpu,cpu_par,"
                         "profile")
    ap.add_argument("--pmc-workload", action="store_true",
                    help="short run for rocprofv3 --pmc: a 256 MiB copy (calibration) then 5 batched steps")
    ap.add_argument("--pmc-summarize", nargs="+", metavar="DB",
                    help="write profiles/traffic_batched16_640x480.json from the rocprofv3 --pmc databases of "
                         "FETCH_SIZE, WRITE_SIZE and (optional) SQ_INSTS_VALU")
    args = ap.parse_args()
    if args.pmc_summarize:
        pmc_summarize(*args.pmc_summarize)
        return
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

    def timed(fn, n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            fn(i)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    if args.pmc_workload:
        from paper_1008_0502_amd import _lib
        lib = _lib.load()
        src = torch.ones(CALIB[0][1] // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for mode, nbytes in CALIB:
            _lib.check(lib.sp_calibration_copy(src.data_ptr(), dst.data_ptr(), nbytes, mode,
                                               torch.cuda.current_stream().cuda_stream), "sp_calibration_copy")
        torch.cuda.synchronize()
        del src, dst
        bf = [torch.from_numpy(synth.Clip(synth.single_ellipse_spec(H=H, W=W, T=2, seed=6000 + i)).stack()[0]).to(dev)
              for i in range(16)]
        tabs = [Batch.pointer_table([f[t] for f in bf]) for t in range(2)]
        b = Batch([(H, W)] * 16, Params(), mrf=True)
        # the launch shapes the autotuner picks for this workload (Kalman tile 40 x 64, XCD
        # order, two channels per across-scale workgroup), so the counters describe the timed run
        b.set_tune(64, True, 2)
        for i in range(5):
            b.step(tabs[i % 2])
        torch.cuda.synchronize()
        b.close()
        log("pmc workload done")
        return

    # ------------------------------------------------------------ headline: batched 16 x 640x480
    NS, NF = 16, 8
    value, ms_step, tune_report = None, None, ""
    roof, kernels, step_roof = None, {}, None
    g = Context(H, W, Params()).geometry
    if "batched" not in skip:   # skipped only to trace the other legs on their own
        log(f"generating {NS} streams x {NF} frames of 640x480")
        bframes = [torch.from_numpy(synth.Clip(synth.single_ellipse_spec(H=H, W=W, T=NF, seed=6000 + i)).stack()[0]).to(dev)
                   for i in range(NS)]
        tables = [Batch.pointer_table([bf[t] for bf in bframes]) for t in range(NF)]
        bt = Batch([(H, W)] * NS, Params(), mrf=True)
        tune_report = bt.autotune(tables[0], steps=5)
        log("autotune: " + tune_report.strip().replace("\n", "; "))
        bstep = lambda i: bt.step(tables[i % NF])

        def bsteps(k):
            # k steps: the clip's NF frame tables in one graph launch per NF steps
            # (sp_batch_steps), a remainder step by step
            for _ in range(k // NF):
                bt.steps(tables)
            for j in range(k % NF):
                bt.step(tables[j])

        log(f"batched step: warmup {args.warmup}, timed {args.steps}, {NF} steps per graph launch")
        timed(lambda _: bsteps(args.warmup), 1)
        dt = timed(lambda _: bsteps(args.steps), 1)
        ms_step = dt / args.steps * 1e3
        value = NS * args.steps / dt
        log(f"batched: {value:.1f} frames/s ({ms_step:.4f} ms/step)")
        if "profile" not in skip:
            nprof = min(args.steps, 100)
            profile_enable(bt, True)
            timed(bstep, nprof)
            prof = profile_read(bt)
            profile_enable(bt, False)
            per_stream = alg_bytes_per_stream(g, mrf=True, prior_copy=False)
            bytes_step = {k: NS * v for k, v in per_stream.items()}
            for name, (ms, cnt) in prof.items():
                kernels[name] = {"avg_us": round(ms / cnt * 1e3, 3), "launches_per_step": cnt / nprof,
                                 "us_per_step": round(ms / nprof * 1e3, 3),
                                 "alg_GBps": (round(bytes_step[name] / (ms / nprof * 1e-3) / 1e9, 2)
                                              if name in bytes_step else None)}
            roof = roofline_of(prof, bytes_step, nprof)
            # the whole step: algorithmic bytes of every kernel of the replay over the timed
            # step (the step's kernels run back to back, so this bounds the step as a whole)
            step_bytes = sum(bytes_step.get(name, 0.0) for name in prof)
            step_roof = {"bound": "hbm", "alg_bytes_per_step": step_bytes,
                         "achieved": round(step_bytes / (ms_step * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)}
        bt.close()

    # ------------------------------------------------------------ plain single stream, 640x480
    plain = None
    clip = synth.Clip(synth.single_ellipse_spec(H=H, W=W, T=T_CLIP, seed=2))
    frames_np, masks_np = clip.stack()
    frames = torch.from_numpy(frames_np).to(dev)
    masks = torch.from_numpy(masks_np).to(dev)
    stream = torch.cuda.current_stream().cuda_stream
    fp = [frames[t].data_ptr() for t in range(T_CLIP)]
    if "plain" not in skip:
        ctx = Context(H, W, Params())
        lib, h = ctx.lib, ctx._handle
        S = torch.empty((g.Hc, g.Wc), dtype=torch.float32, device=dev)
        P = torch.empty((H, W), dtype=torch.float32, device=dev)
        U = torch.empty((2, H, W), dtype=torch.float32, device=dev)
        PW = torch.empty((4, H, W), dtype=torch.float32, device=dev)
        B = torch.empty((1,), dtype=torch.float32, device=dev)
        sp, pp, up, pwp, bp = S.data_ptr(), P.data_ptr(), U.data_ptr(), PW.data_ptr(), B.data_ptr()
        lib.sp_set_stream(h, stream)

        def step(i, mrf=True):
            t = i % T_CLIP
            rc = lib.sp_step(h, fp[t], fp[t - 1] if t else None, None, sp, None, pp,
                             up if mrf else None, pwp if mrf else None, bp if mrf else None)
            if rc:
                raise RuntimeError(lib.sp_last_error().decode())

        def step_calls(i):
            t = i % T_CLIP
            rc = lib.saliency_forward(h, fp[t], fp[t - 1] if t else None, sp, None)
            rc |= lib.prior_update(h, sp, None, pp)
            rc |= lib.mrf_weights(h, fp[t], pp, up, pwp, bp)
            if rc:
                raise RuntimeError(lib.sp_last_error().decode())

        n = max(args.steps, 100)
        timed(step, args.warmup)
        d1 = timed(step, n)
        d2 = timed(lambda i: step(i, mrf=False), n)
        d3 = timed(step_calls, n)
        plain = {"frames_per_s": round(n / d1, 2), "ms_per_frame": round(d1 / n * 1e3, 5),
                 "saliency_prior_only_frames_per_s": round(n / d2, 2),
                 "three_calls_frames_per_s": round(n / d3, 2)}
        if "profile" not in skip:
            profile_enable(ctx, True)
            timed(step, 100)
            pr = profile_read(ctx)
            profile_enable(ctx, False)
            plain["kernels_us"] = {k: round(v[0] / v[1] * 1e3, 3) for k, v in pr.items()}
            pb = alg_bytes_per_stream(g, mrf=True, prior_copy=True)
            plain["roofline"] = roofline_of(pr, pb, 100, counters=False)
        ctx.close()
        log(f"plain: {plain['frames_per_s']} frames/s")

    # ------------------------------------------------------------ fwd + bwd, 640x480
    fb = None
    if "bwd" not in skip:
        tctx = Context(H, W, Params(record_tape=T_CLIP))
        lib, th = tctx.lib, tctx._handle
        lib.sp_set_stream(th, stream)
        Ps = torch.empty((T_CLIP, H, W), dtype=torch.float32, device=dev)
        Ss = torch.empty((T_CLIP, g.Hc, g.Wc), dtype=torch.float32, device=dev)
        loss = torch.empty((1,), dtype=torch.float32, device=dev)
        grad = torch.empty_like(Ps)
        gw, gq, gr = (torch.empty(8, device=dev), torch.empty(1, device=dev), torch.empty(1, device=dev))

        def clip_fb(_):
            lib.sp_reset(th)
            for t in range(T_CLIP):
                rc = lib.sp_step(th, fp[t], fp[t - 1] if t else None, None, Ss[t].data_ptr(), None,
                                 Ps[t].data_ptr(), None, None, None)
                if rc:
                    raise RuntimeError(lib.sp_last_error().decode())
            rc = lib.sp_mse_mask_loss(th, Ps.data_ptr(), masks.data_ptr(), T_CLIP, loss.data_ptr(), grad.data_ptr())
            rc |= lib.saliency_backward(th, grad.data_ptr(), T_CLIP, gw.data_ptr(), gq.data_ptr(), gr.data_ptr())
            if rc:
                raise RuntimeError(lib.sp_last_error().decode())

        timed(clip_fb, 1)
        reps = 3
        dtb = timed(clip_fb, reps)
        fb = {"frames_per_s": round(reps * T_CLIP / dtb, 2), "ms_per_clip": round(dtb / reps * 1e3, 4),
              "clip_frames": T_CLIP, "loss": float(loss.item())}
        tctx.close()
        log(f"fwd+bwd: {fb['frames_per_s']} frames/s")

    # ------------------------------------------------------------ batched fwd + bwd, 16 x 640x480 x 120
    fbb = None
    if "bwd_batched" not in skip:
        NB = 16
        log(f"generating {NB} clips of 640x480 x {T_CLIP} frames (seeds 6000+i)")
        clips = gen_clips([("single", H, W, T_CLIP, 6000 + i) for i in range(NB)])
        bfr = [torch.from_numpy(f).to(dev) for f, _ in clips]
        bmk = [torch.from_numpy(m).to(dev) for _, m in clips]
        del clips
        btabs = [Batch.pointer_table([f[t] for f in bfr]) for t in range(T_CLIP)]
        bb = Batch([(H, W)] * NB, Params(record_tape=T_CLIP))
        bb.autotune(btabs[0], steps=3)
        lib, bh = bb.lib, bb._handle
        from ctypes import c_void_p
        mptr = (c_void_p * NB)(*[m.data_ptr() for m in bmk])
        bgrad = [torch.empty((T_CLIP, H, W), dtype=torch.float32, device=dev) for _ in range(NB)]
        gptr = (c_void_p * NB)(*[x.data_ptr() for x in bgrad])
        bloss = torch.empty(NB, dtype=torch.float32, device=dev)
        bgw = torch.empty((NB, 8), dtype=torch.float32, device=dev)
        bgq = torch.empty(NB, dtype=torch.float32, device=dev)
        bgr = torch.empty(NB, dtype=torch.float32, device=dev)
        # the clip's frame tables, eight steps per graph launch (sp_batch_steps)
        tp = [(c_void_p * len(btabs[t0:t0 + 8]))(*[t.data_ptr() for t in btabs[t0:t0 + 8]])
              for t0 in range(0, T_CLIP, 8)]

        def batch_fwd(_):
            if lib.sp_batch_reset(bh):
                raise RuntimeError(lib.sp_last_error().decode())
            for arr in tp:
                if lib.sp_batch_steps(bh, len(arr), arr):
                    raise RuntimeError(lib.sp_last_error().decode())

        def batch_fb(_):
            batch_fwd(0)
            rc = lib.sp_batch_mse_mask_loss(bh, mptr, T_CLIP, bloss.data_ptr(), gptr)
            rc |= lib.sp_batch_backward(bh, gptr, T_CLIP, bgw.data_ptr(), bgq.data_ptr(), bgr.data_ptr())
            if rc:
                raise RuntimeError(lib.sp_last_error().decode())

        timed(batch_fb, 1)
        reps = 3
        dfb = timed(batch_fb, reps)
        dfw = timed(batch_fwd, reps)
        fbb = {"frames_per_s": round(reps * NB * T_CLIP / dfb, 2), "ms_per_clip_batch": round(dfb / reps * 1e3, 3),
               "forward_with_tape_frames_per_s": round(reps * NB * T_CLIP / dfw, 2),
               "streams": NB, "clip_frames": T_CLIP, "loss_mean": float(bloss.mean().item())}
        if "profile" not in skip:
            profile_enable(bb, True)
            timed(batch_fb, 1)
            pr = profile_read(bb)
            profile_enable(bb, False)
            fbb["kernels_ms_per_clip"] = {k: round(v[0], 3) for k, v in sorted(pr.items(), key=lambda kv: -kv[1][0])}
            fbb["launches_per_clip"] = {k: v[1] for k, v in pr.items()}
        bb.close()
        del bfr, bmk, bgrad, btabs
        torch.cuda.empty_cache()
        log(f"batched fwd+bwd: {fbb['frames_per_s']} frames/s")

    # ------------------------------------------------------------ mixed batch of 64 streams of four sizes
    mixed = None
    if "mixed" not in skip:
        sizes = [(120, 160)] * 16 + [(240, 320)] * 16 + [(480, 640)] * 16 + [(720, 1280)] * 16
        mf = [torch.from_numpy(synth.Clip(synth.single_ellipse_spec(H=hh, W=ww, T=4, seed=1000 + i)).stack()[0]).to(dev)
              for i, (hh, ww) in enumerate(sizes)]
        mtab = [Batch.pointer_table([f[t] for f in mf]) for t in range(4)]
        mb = Batch(sizes, Params())
        mb.autotune(mtab[0], steps=3)
        fn = lambda i: mb.step(mtab[i % 4])
        timed(fn, 3)
        steps = 30
        dtm = timed(fn, steps)
        mb.close()
        mixed = {"frames_per_s": round(64 * steps / dtm, 2), "ms_per_step": round(dtm / steps * 1e3, 4),
                 "mpx_per_s": round(sum(hh * ww for hh, ww in sizes) * steps / dtm / 1e6, 1), "streams": 64}
        log(f"mixed: {mixed['frames_per_s']} frames/s")

    # ------------------------------------------------------------ the named single-stream workloads
    configs = None
    if "configs" not in skip:
        configs = {}
        named = [
            ("single_ellipse_160x120_x30", "single", 120, 160, 30, 0, Params(), False, 300),
            ("three_ellipse_320x240_x300_mrf", "three", 240, 320, 300, 1,
             Params(depth=6, centers=(2, 3), deltas=(3, 4)), True, 300),
            ("five_ellipse_1920x1080", "five", 1080, 1920, 40, 5,
             Params(depth=9, centers=(2, 3, 4), deltas=(3, 4)), False, 1000),
            ("single_ellipse_352x288", "single", 288, 352, 30, 7, Params(), False, 300),
            ("single_ellipse_480x384", "single", 384, 480, 30, 7, Params(), False, 300),
            ("single_ellipse_640x512", "single", 512, 640, 30, 7, Params(), False, 300),
        ]
        log("generating the named clips")
        drawn = gen_clips([(k, hh, ww, tt, sd) for _, k, hh, ww, tt, sd, _, _, _ in named])
        for (name, kind, hh, ww, tt, sd, pp, mrf, nsteps), (fnp, _) in zip(named, drawn):
            fr = torch.from_numpy(fnp).to(dev)
            cx = Context(hh, ww, pp)
            gg = cx.geometry
            lib, ch = cx.lib, cx._handle
            lib.sp_set_stream(ch, stream)
            So = torch.empty((gg.Hc, gg.Wc), dtype=torch.float32, device=dev)
            Po = torch.empty((hh, ww), dtype=torch.float32, device=dev)
            Uo = torch.empty((2, hh, ww), dtype=torch.float32, device=dev) if mrf else None
            PWo = torch.empty((4, hh, ww), dtype=torch.float32, device=dev) if mrf else None
            Bo = torch.empty((1,), dtype=torch.float32, device=dev) if mrf else None
            fpp = [fr[t].data_ptr() for t in range(tt)]

            def cstep(i):
                t = i % tt
                if t == 0:
                    lib.sp_reset(ch)
                rc = lib.sp_step(ch, fpp[t], fpp[t - 1] if t else None, None, So.data_ptr(), None, Po.data_ptr(),
                                 Uo.data_ptr() if mrf else None, PWo.data_ptr() if mrf else None,
                                 Bo.data_ptr() if mrf else None)
                if rc:
                    raise RuntimeError(lib.sp_last_error().decode())

            timed(cstep, 20)
            dc = timed(cstep, nsteps)
            configs[name] = {"frames_per_s": round(nsteps / dc, 2), "ms_per_frame": round(dc / nsteps * 1e3, 5),
                             "H": hh, "W": ww, "depth": gg.depth, "pairs": gg.pairs, "mrf": mrf,
                             "distinct_frames": tt, "steps_timed": nsteps}
            cx.close()
            del fr
        log("configs: " + ", ".join(f"{k} {v['frames_per_s']}" for k, v in configs.items()))

    # ------------------------------------------------------------ beyond the step: prior variants, colour
    # likelihood, minimum cut (640x480 clip, seed 2; segmentations from the generator's masks)
    extras = None
    if "extras" not in skip:
        from paper_1008_0502_amd.api import MinCut
        extras = {}
        NT = 30
        px = H * W
        S = torch.empty((g.Hc, g.Wc), dtype=torch.float32, device=dev)
        P = torch.empty((H, W), dtype=torch.float32, device=dev)
        segp = [None] + [masks[t - 1].data_ptr() for t in range(1, NT)]
        for vname, vp in (("dt_prediction", Params(f_mode=1)), ("stochastic_map", Params(ssm_q=1e-3, ssm_r=1e-1)),
                          ("dt_prediction_and_stochastic_map", Params(f_mode=1, ssm_q=1e-3, ssm_r=1e-1))):
            cx = Context(H, W, vp)
            lib, ch = cx.lib, cx._handle
            lib.sp_set_stream(ch, stream)

            def vstep(i, lib=lib, ch=ch):
                t = i % NT
                if t == 0:
                    lib.sp_reset(ch)
                if lib.sp_step(ch, fp[t], fp[t - 1] if t else None, segp[t], S.data_ptr(), None, P.data_ptr(),
                               None, None, None):
                    raise RuntimeError(lib.sp_last_error().decode())

            timed(vstep, NT)
            nv = 300
            dv = timed(vstep, nv)
            rec = {"frames_per_s": round(nv / dv, 2), "ms_per_frame": round(dv / nv * 1e3, 5)}
            if "profile" not in skip:
                profile_enable(cx, True)
                timed(vstep, NT)
                pr = profile_read(cx)
                profile_enable(cx, False)
                if "k_dt" in pr:
                    ms, cnt = pr["k_dt"]
                    rec["k_dt_avg_us"] = round(ms / cnt * 1e3, 3)
                    rec["k_dt_alg_GBps"] = round(5.0 * px / (ms / cnt * 1e-3) / 1e9, 2)   # 1 B in, 4 B out per px
            extras[vname] = rec
            cx.close()
        # colour likelihood on the plain prior of frame 10
        cx = Context(H, W, Params())
        Pg = cx.run_clip(frames[:11])["pi"][10].contiguous()
        U0 = torch.zeros((2, H, W), dtype=torch.float32, device=dev)
        lib, ch = cx.lib, cx._handle
        lib.sp_set_stream(ch, stream)

        def gstep(_):
            if lib.sp_colour_likelihood(ch, fp[10], Pg.data_ptr(), U0.data_ptr(), None):
                raise RuntimeError(lib.sp_last_error().decode())

        timed(gstep, 5)
        ng = 50
        dg = timed(gstep, ng)
        rec = {"calls_per_s": round(ng / dg, 2), "ms_per_call": round(dg / ng * 1e3, 4), "components": 3,
               "em_iterations": 10}
        if "profile" not in skip:
            profile_enable(cx, True)
            timed(gstep, 10)
            pr = profile_read(cx)
            profile_enable(cx, False)
            per_px = {"k_gmm_acc": 7.0, "k_gmm_psi": 19.0}   # RGB + prior read; RGB read + U0, U1 read and written
            rec["kernels"] = {k: {"avg_us": round(v[0] / v[1] * 1e3, 3), "launches_per_call": v[1] / 10,
                                  "alg_GBps": (round(per_px[k] * px / (v[0] / v[1] * 1e-3) / 1e9, 2)
                                               if k in per_px else None)} for k, v in pr.items()}
        extras["colour_likelihood"] = rec
        cx.close()
        # minimum cut: the closed loop (each cut is the next frame's segmentation) and the cut alone
        cx = Context(H, W, Params())
        mc = MinCut(H, W)
        lib, ch = cx.lib, cx._handle
        lib.sp_set_stream(ch, stream)
        Uc = torch.empty((2, H, W), dtype=torch.float32, device=dev)
        PWc = torch.empty((4, H, W), dtype=torch.float32, device=dev)
        Bc = torch.empty((1,), dtype=torch.float32, device=dev)
        lab = [torch.zeros((H, W), dtype=torch.uint8, device=dev) for _ in range(2)]
        flow = torch.empty((1,), dtype=torch.int64, device=dev)
        cut_s = [0.0]

        def loop_step(i):
            t = i % NT
            if t == 0:
                lib.sp_reset(ch)
            seg = lab[(t + 1) % 2].data_ptr() if t else None
            if lib.sp_step(ch, fp[t], fp[t - 1] if t else None, seg, S.data_ptr(), None, P.data_ptr(),
                           Uc.data_ptr(), PWc.data_ptr(), Bc.data_ptr()):
                raise RuntimeError(lib.sp_last_error().decode())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mc.cut(Uc, PWc, 256.0, lab[t % 2], flow)
            torch.cuda.synchronize()
            cut_s[0] += time.perf_counter() - t0

        timed(loop_step, 5)
        cut_s[0] = 0.0
        nl = NT
        dl = timed(loop_step, nl)
        extras["min_cut_closed_loop"] = {"frames_per_s": round(nl / dl, 2), "ms_per_frame": round(dl / nl * 1e3, 4),
                                         "cut_ms_per_frame": round(cut_s[0] / nl * 1e3, 4), "scale": 256.0,
                                         "object_px_last": int(lab[(nl - 1) % 2].sum().item())}
        mc.close()
        cx.close()
        # pixel-level adjoint: dL/d frames of an 8-frame clip, after the adjoint of the weights
        # (each call recomputes every frame's maps, then runs the adjoint kernels per frame)
        TP = 8
        cx = Context(H, W, Params(record_tape=TP))
        out = cx.run_clip(frames[:TP])
        _, gpi = cx.mse_mask_loss(out["pi"], masks[:TP])
        cx.saliency_backward(gpi)
        lib, ch = cx.lib, cx._handle
        lib.sp_set_stream(ch, stream)
        GF = torch.empty((TP, H, W, 3), dtype=torch.float32, device=dev)

        def pstep(_):
            if lib.saliency_backward_frames(ch, frames.data_ptr(), TP, GF.data_ptr()):
                raise RuntimeError(lib.sp_last_error().decode())

        timed(pstep, 2)
        npa = 20
        dpa = timed(pstep, npa)
        rec = {"clip_frames": TP, "ms_per_clip": round(dpa / npa * 1e3, 4),
               "frames_per_s": round(npa * TP / dpa, 2)}
        if "profile" not in skip:
            profile_enable(cx, True)
            timed(pstep, 3)
            pr = profile_read(cx)
            profile_enable(cx, False)
            rec["ms_per_clip_by_kind"] = {k: round(v[0] / 3, 4) for k, v in pr.items()}
        extras["pixel_adjoint"] = rec
        cx.close()
        log("extras: " + json.dumps(extras))

    cpu = None
    if "cpu" not in skip:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(frames_np, args.cpu_seconds)
        if "cpu_par" not in skip:
            log("cpu baseline (oracle), one process per stream")
            cpu["parallel"] = cpu_baseline_parallel(16, args.cpu_seconds)

    out = {
        "metric": "frames/s saliency+Kalman prior at 640x480 (fwd, fwd+bwd, batched); HBM GB/s",
        "value": None if value is None else round(value, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None if ms_step is None else round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched step: 16 streams of 640x480 (single-ellipse generator, seeds 6000+i, 8 frames "
                               "cycled), every stream's saliency map, Kalman prior and MRF capacities each step, "
                               "eight steps per graph launch",
                   "streams": NS, "H": H, "W": W, "depth": g.depth, "pairs": g.pairs, "c_max": g.c_max,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "step_roofline": step_roof,
        "kernels": kernels,
        "autotune": tune_report.strip().splitlines(),
        "plain_640x480": plain,
        "fwd_bwd_640x480": fb,
        "fwd_bwd_batched16_640x480": fbb,
        "configs": configs,
        "batched_mixed64": mixed,
        "beyond_the_step_640x480": extras,
        "cpu_baseline": cpu,
        "source_hash": source_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
