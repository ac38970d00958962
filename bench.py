#!/usr/bin/env python3
"""Benchmark of region-adaptive DP pixelization on one MI355X.

A step is one pass of the whole hot path over one batch already resident in
HBM: plan (mask classification + store scan), forward (exact cell sums,
Laplace noise, clip, compact store) with the reconstruction fused in.

Default workload: 64 RGB 1920x1080 frames, 8-rectangle foreground masks,
simple cells b=32 / eps=1.0, complex subcells s_b=8 / eps=0.3, m=16.
Reported beside it: the same kernels launched once per frame, the uneven
mixed-resolution batch (256 frames, one launch per layout group, graph-replayed),
and the CPU oracle on a bounded sample.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2511_04261_amd", "csrc", "dppix_kernels.hip")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_forward_region_1080p_x64_counters.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _code_only(text: str) -> str:
    """C/C++ source without comments and blank lines (the code the compiler sees)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())


def kernel_source_hash(root: str = ROOT) -> str:
    """Hash of the device code (kernels and the headers they include), so that
    a counter summary is only trusted for the kernels it was taken from."""
    h = hashlib.sha256()
    for name in ("dppix_kernels.hip", "dppix_internal.h", "dppix_tiles.h"):
        with open(os.path.join(root, "paper_2511_04261_amd", "csrc", name), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def read_traffic(bytes_per_launch_alg: float):
    """HBM bytes per forward launch from the committed rocprofv3 counter
    summary, scaled by the copy-kernel calibration; None when the kernels
    changed since the counters were taken."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    kv = {}
    with open(COUNTERS_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        fetch = float(kv["fetch_kib_per_dispatch"]) * 1024.0 * float(kv["fetch_scale"])
        write = float(kv["write_kib_per_dispatch"]) * 1024.0 * float(kv["write_scale"])
    except (KeyError, ValueError):
        return None
    return fetch + write


def build_batch(frames_s, dev, persistent=0, threads=0, host_render=False, frames=None):
    import torch
    import paper_2511_04261_amd as dp
    if frames is None:
        frames = [dp.FrameParams.from_spec(s) for s in frames_s]
    plan = dp.Plan(frames, device=dev, threads=threads, persistent=persistent)
    if host_render:
        # byte-identical frames rendered on the host and copied over (no
        # device kernels besides the library's, e.g. under a counter profiler)
        imgs, masks = [], []
        for i, s in enumerate(frames_s):
            imgs.append(torch.from_numpy(s.image).to(dev))
            masks.append(torch.from_numpy(s.mask).to(dev))
            s.drop_host()
            if i % 16 == 15:
                log("inputs: %d of %d frames on the device" % (i + 1, len(frames_s)))
    else:
        imgs = [s.image_torch(dev) for s in frames_s]
        masks = [s.mask_torch(dev) for s in frames_s]
    outs = [torch.empty_like(t) for t in imgs]
    return plan, imgs, masks, outs


def store_bytes(plan):
    """Bytes of the compact store written by one forward (from the device counts)."""
    counts = plan.counts.cpu().numpy()
    tot = 0
    for fp, fi, c in zip(plan.frames, plan.info, counts):
        tot += 4 * fp.channels * (int(c[0]) + fi.n * fi.n * int(c[1])) + fi.grid_rows * fi.grid_cols
    return tot


def alg_bytes(plan):
    """Algorithmic HBM bytes of one step: image + mask read, reconstruction
    and store written (each byte once; padding never counted)."""
    px = sum(fp.height * fp.width * fp.channels for fp in plan.frames)
    mask = sum(fp.height * fp.width for fp in plan.frames)
    st = store_bytes(plan)
    return dict(image=px, mask=mask, recon=px, store=st, forward=2 * px + st, step=2 * px + mask + st)


def time_steps(step_fn, warmup, steps):
    import torch
    for _ in range(warmup):
        step_fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step_fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def warm_up(call, ms=30.0):
    """Untimed launches until about `ms` of GPU time has passed: after the
    host has kept the GPU idle (building inputs), its clocks take some 10 ms
    of load to settle, and work timed before that reads several per cent
    slow."""
    import torch
    t0 = time.perf_counter()
    while True:
        for _ in range(4):
            call()
        torch.cuda.synchronize()
        if (time.perf_counter() - t0) * 1e3 >= ms:
            return


def time_launches(call, n, stream):
    """Average duration of one launch: n back-to-back launches of the same
    call between two HIP events on the stream the kernels run on, after a
    warm-up."""
    import torch
    warm_up(call)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(n):
        call()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / n


def run_batched(frames_s, dev, warmup, steps, graph=False, threads=0, persistent=0, frames=None,
                compare=False):
    """Steps of plan + forward over one batch: replays of a captured HIP graph
    (graph=True) or the two C-ABI calls issued back to back on the stream; with
    compare=True the other form is timed too (other_step_ms)."""
    import torch
    plan, imgs, masks, outs = build_batch(frames_s, dev, persistent=persistent, threads=threads, frames=frames)
    stream = torch.cuda.current_stream()
    plan_call, fwd_call = plan.bound_calls(masks, imgs, outs, stream)
    g = plan.graph(masks, imgs, outs, stream) if (graph or compare) else None

    def step_graph():
        g.launch(stream)

    def step_calls():
        plan_call()
        fwd_call()

    # the step time (plan + forward per step); then each kernel's launch time
    dt = time_steps(step_graph if graph else step_calls, warmup, steps)
    other = None
    if compare:
        other = 1e3 * time_steps(step_calls if graph else step_graph, warmup, steps) / steps
    fwd_ms = time_launches(fwd_call, max(steps, 10), stream)
    plan_ms = time_launches(plan_call, max(steps, 10), stream)
    ab = alg_bytes(plan)
    return dict(plan=plan, seconds=dt, step_ms=1e3 * dt / steps, fwd_ms=fwd_ms, plan_ms=plan_ms, bytes=ab,
                pixels=sum(fp.height * fp.width for fp in plan.frames), other_step_ms=other)


def autotune_batch(frames_s, dev):
    """Tile shapes and workgroup size for the batch from the project's
    autotuner, timing whole candidate configurations of this batch (one
    workgroup per tile; tile rows of about 1-4 KB or the library's choice;
    0 / 128 / 256 lanes)."""
    import torch
    import paper_2511_04261_amd as dp
    from paper_2511_04261_amd.autotune import Autotuner
    t0 = time.perf_counter()
    imgs = [s.image_torch(dev) for s in frames_s]
    masks = [s.mask_torch(dev) for s in frames_s]
    tuner = Autotuner(dev, cache_path=None, reps=5, threads=(0, 128, 256), launch_modes=(0,))
    tuned, info = tuner.tune_whole_batch([dp.FrameParams.from_spec(s) for s in frames_s], imgs, masks)
    del imgs, masks
    torch.cuda.empty_cache()
    launch = dict(threads=info["threads"], persistent=info["persistent"])
    return tuned, launch, dict(seconds=round(time.perf_counter() - t0, 1), tile_bytes=info["tile_bytes"],
                               threads=info["threads"], candidates=len(info["tried"]),
                               ms_best=round(info["ms"], 4),
                               ms_library_default=round(min(r["ms"] for r in info["tried"] if r["tile_bytes"] == 0
                                                            and r["threads"] == 0), 4))


def run_per_frame(frames_s, dev, warmup, steps):
    """The same kernels launched once per frame (one plan per frame)."""
    import torch
    per = [build_batch([s], dev, persistent=False) for s in frames_s]
    stream = torch.cuda.current_stream()

    calls = [p[0].bound_calls(p[2], p[1], p[3], stream) for p in per]

    def step():
        for plan_call, fwd_call in calls:
            plan_call()
            fwd_call()

    dt = time_steps(step, warmup, steps)
    px = sum(s.height * s.width for s in frames_s)
    b = sum(alg_bytes(p[0])["step"] for p in per)
    return dict(seconds=dt, step_ms=1e3 * dt / steps, pixels=px, bytes=b)


def run_single_frame(dev, calls=200):
    """One 256x256 grayscale frame, b = 16, m = 16, eps = 0.5, no mask: the
    latency of one plan + forward (GPU time from HIP events over back-to-back
    calls, and host wall time per call including the launch)."""
    import torch
    import paper_2511_04261_amd as dp
    from paper_2511_04261_amd import synth
    img = torch.from_numpy(synth.single_gray()[:, :, 0].copy()).to(dev)
    out = torch.empty_like(img)
    plan = dp.Plan([dp.FrameParams(256, 256, 1, dp.U8_HWC, b=16, sb=16, m=16, eps_bg=0.5, seed=0)], device=dev)
    stream = torch.cuda.current_stream()
    pc, fc = plan.bound_calls(None, [img], [out], stream)

    def call():
        pc()
        fc()

    gpu_ms = time_launches(call, calls, stream)
    t0 = time.perf_counter()
    for _ in range(calls):
        call()
        torch.cuda.synchronize()
    wall_ms = 1e3 * (time.perf_counter() - t0) / calls
    plan.close()
    return dict(us_per_frame_gpu=round(1e3 * gpu_ms, 2), us_per_call_synchronous=round(1e3 * wall_ms, 2),
                frame="256x256x1", b=16, m=16, eps=0.5)


def run_autograd_batch(dev, reps=20):
    """32 x 3 x 512 x 512 fp32 frames with rectangle masks, b_fg = 8,
    b_bg = 16, m = 8, eps_fg = 0.5, eps_bg = 1.0: forward (with the clip
    flags the adjoint needs) and adjoint, algorithmic GB/s of each."""
    import torch
    import paper_2511_04261_amd as dp
    from paper_2511_04261_amd import synth
    x, masks, w = synth.autograd_batch()
    B, C, H, W = x.shape
    tx = torch.from_numpy(x).to(dev)
    tm = [torch.from_numpy(m).to(dev) for m in masks]
    gy = torch.from_numpy(w).to(dev)
    y = torch.empty_like(tx)
    gx = torch.empty_like(tx)
    frames = [dp.FrameParams(H, W, C, dp.F32_CHW, b=16, sb=8, m=8, eps_bg=1.0, eps_fg=0.5, tau=1, seed=4,
                             frame_index=i) for i in range(B)]
    plan = dp.Plan(frames, device=dev)
    clip = plan.clip_buffers()
    scratch = torch.empty(max(plan.sizes.grad_scratch_bytes, 256), dtype=torch.uint8, device=dev)
    xs, ys = [tx[i] for i in range(B)], [y[i] for i in range(B)]
    gys, gxs = [gy[i] for i in range(B)], [gx[i] for i in range(B)]
    stream = torch.cuda.current_stream()
    plan_call, fwd_call = plan.bound_calls(tm, xs, ys, stream, clip=clip)
    bwd_call = plan.bound_backward(gys, gxs, clip, scratch, stream)
    plan_call()
    fwd_ms = time_launches(fwd_call, reps, stream)
    bwd_ms = time_launches(bwd_call, reps, stream)
    nbytes = 4 * tx.numel()
    st = store_bytes(plan)
    plan.close()
    return dict(shape="32x3x512x512 fp32", forward_ms=round(fwd_ms, 4), backward_ms=round(bwd_ms, 4),
                forward_gbs=round((2 * nbytes + st) / (fwd_ms * 1e-3) / 1e9, 1),
                backward_gbs=round((2 * nbytes + st) / (bwd_ms * 1e-3) / 1e9, 1))


SERVE_PARAMS = dict(b=32, sb=8, m=16, eps_bg=1.0, eps_fg=0.3, tau=1)


def run_serving(dev, seconds, cap_bytes=8 << 30):
    """16 camera streams (8 x 1080p, 6 x 768x576, 2 x 2160p), Poisson 30 Hz
    each, replayed in real time through the continuous-batching server."""
    from paper_2511_04261_amd.serving import (GpuBackend, MemoryLedger, Scheduler, camera_streams, latency_stats,
                                              serve_streams)
    be = GpuBackend(dev)
    warm = camera_streams(duration_s=1.0, pool=2, device=dev, seed=999)
    serve_streams(warm, Scheduler(be, MemoryLedger(cap_bytes)), SERVE_PARAMS)
    streams = camera_streams(duration_s=seconds, pool=8, device=dev)
    sch = Scheduler(be, MemoryLedger(cap_bytes), max_batch=64, max_inflight=2)
    t0 = time.perf_counter()
    done = serve_streams(streams, sch, SERVE_PARAMS)
    wall = time.perf_counter() - t0
    st = latency_stats(done)
    ok = [r for r in done if r.error is None]
    px = sum(r.height * r.width for r in ok)
    return dict(p50_ms=round(st.get("p50_ms", float("nan")), 3), p99_ms=round(st.get("p99_ms", float("nan")), 3),
                max_ms=round(st.get("max_ms", float("nan")), 3), frames=len(ok), rejected=len(sch.rejected),
                megapixels_per_s=round(px / wall / 1e6, 1), seconds=round(wall, 2), streams=len(streams),
                batches=sch.batches, mean_batch=round(sum(sch.batch_sizes) / max(1, len(sch.batch_sizes)), 2),
                peak_admitted_bytes=sch.ledger.peak)


def counters_run(frames_s, dev, launches=3, copy_bytes=1 << 30):
    """Short run for rocprofv3 --pmc: one plain device copy of known size
    (the calibration of FETCH_SIZE / WRITE_SIZE), then a few plan + forward
    launches of the headline workload."""
    import torch
    # a converting copy int32 -> uint8 is an elementwise kernel that reads
    # 4 bytes and writes 1 byte per element (a same-dtype copy_() would be a
    # runtime memcpy that the counters do not see)
    n = copy_bytes // 4
    src = torch.ones(n, dtype=torch.int32, device=dev)
    dst = torch.empty(n, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    log("counters run: calibration buffers ready")
    dst.copy_(src)
    torch.cuda.synchronize()
    log("counters run: calibration kernel done")
    del src, dst
    plan, imgs, masks, outs = build_batch(frames_s, dev, host_render=True)
    torch.cuda.synchronize()
    log("counters run: batch ready")
    for i in range(launches):
        plan.plan(masks)
        plan.forward(imgs, out=outs)
        torch.cuda.synchronize()
        log("counters run: launch %d done" % i)
    ab = alg_bytes(plan)
    log("counters run: calibration copy %d -> %d bytes; forward alg bytes %d per launch" % (4 * n, n, ab["forward"]))
    print(json.dumps({"copy_read_bytes": 4 * n, "copy_write_bytes": n, "forward_alg_bytes": ab["forward"],
                      "kernel_source_sha256_16": kernel_source_hash()}), flush=True)


def cpu_baseline(frames_s, budget_s=15.0, dev=None):
    """The oracle as it stands, single-threaded, on a bounded sample of the
    same workload: whole frames until about budget_s of CPU work."""
    import oracle
    oracle.build()
    dt = 0.0
    done = px = passes = 0
    while dt < budget_s and passes < 8:
        passes += 1
        for s in frames_s:
            # inputs rendered on the device and copied back (byte-identical), not timed
            img = s.image_torch(dev).cpu().numpy() if dev is not None else s.image
            mask = s.mask
            t1 = time.perf_counter()
            oracle.forward(img, mask, oracle.Params(s.height, s.width, s.channels, b=s.b, sb=s.sb, m=s.m,
                                                    eps_simple=s.eps_simple, eps_complex=s.eps_complex, tau=s.tau,
                                                    seed=s.seed, frame_index=s.frame_index))
            dt += time.perf_counter() - t1
            done += 1
            px += s.height * s.width
            s.drop_host()
            if dt > budget_s:
                break
    return dict(value=round(px / dt / 1e6, 3), unit="megapixels/s", cores=1, kind="oracle",
                sample="%d frame passes over the %d-frame batch (%dx%d RGB, masks, same parameters), "
                       "single thread, %.1f s of oracle time" % (
                           done, len(frames_s), frames_s[0].width, frames_s[0].height, dt))


def cpu_worker(frames_s, k, procs, budget_s):
    """One worker of the parallel oracle baseline: frames k, k+procs, ...
    rendered on the host (untimed), then the oracle over them until about
    budget_s of oracle time.  Prints one JSON line."""
    import oracle
    mine = frames_s[k::procs]
    inputs = [(s.image, s.mask) for s in mine]
    dt, px, done = 0.0, 0, 0
    while dt < budget_s:
        for s, (img, mask) in zip(mine, inputs):
            t1 = time.perf_counter()
            oracle.forward(img, mask, oracle.Params(s.height, s.width, s.channels, b=s.b, sb=s.sb, m=s.m,
                                                    eps_simple=s.eps_simple, eps_complex=s.eps_complex, tau=s.tau,
                                                    seed=s.seed, frame_index=s.frame_index))
            dt += time.perf_counter() - t1
            px += s.height * s.width
            done += 1
    print(json.dumps({"px": px, "seconds": dt, "frames": done}), flush=True)


def cpu_baseline_parallel(n_frames, budget_s=10.0):
    """The same oracle, one process per host core (at most 16), frames
    distributed round-robin: the all-cores reference.  Workers are child
    processes that never touch the GPU."""
    import subprocess
    import oracle
    oracle.build()
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    procs = max(1, min(16, cores, n_frames))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", "--cpu-procs", str(procs),
           "--cpu-budget", str(budget_s), "--frames", str(n_frames)]
    env = dict(os.environ, OMP_NUM_THREADS="1", HIP_VISIBLE_DEVICES="")
    workers = [subprocess.Popen(cmd + ["--cpu-index", str(k)], stdout=subprocess.PIPE, env=env, text=True)
               for k in range(procs)]
    rate, frames, seconds = 0.0, 0, 0.0
    for w in workers:
        out, _ = w.communicate()
        if w.returncode != 0:
            raise RuntimeError("CPU oracle worker failed with status %d" % w.returncode)
        r = json.loads(out.strip().splitlines()[-1])
        rate += r["px"] / r["seconds"]
        frames += r["frames"]
        seconds = max(seconds, r["seconds"])
    return dict(value=round(rate / 1e6, 3), unit="megapixels/s", cores=procs, kind="oracle",
                sample="%d processes, one per host core, over the %d-frame batch (frames round-robin, host-rendered, "
                       "untimed); %d frame passes, about %.1f s of oracle time each" % (procs, n_frames, frames,
                                                                                      seconds))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 200 untimed steps (about 40 ms of GPU work) bring the clocks to their
    # steady state before the timed steps start
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-extra", action="store_true", help="only the headline workload")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="seconds of camera-stream arrivals for the latency leg (0 skips it)")
    ap.add_argument("--counters", action="store_true", help="short run for rocprofv3 --pmc")
    ap.add_argument("--cpu-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-index", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-procs", type=int, default=1, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-budget", type=float, default=10.0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the method shards by frame with no collective, "
              "so --gpus N>1 is not run here", file=sys.stderr)
        sys.exit(2)

    if args.cpu_worker:
        from paper_2511_04261_amd import synth
        cpu_worker(synth.region_batch(args.frames), args.cpu_index, args.cpu_procs, args.cpu_budget)
        return

    import torch
    from paper_2511_04261_amd import synth
    dev = torch.device("cuda:0")
    log("bench: generating %d RGB 1080p frames" % args.frames)
    frames_s = synth.region_batch(args.frames)
    if args.counters:
        counters_run(frames_s, dev)
        return

    log("bench: batched region-adaptive 1080p")
    res = run_batched(frames_s, dev, args.warmup, args.steps, graph=False, threads=args.threads, compare=True)
    mp = res["pixels"] * args.steps / res["seconds"] / 1e6
    ab = res["bytes"]
    fwd_gbs = ab["forward"] / (res["fwd_ms"] * 1e-3) / 1e9
    step_gbs = ab["step"] / (res["step_ms"] * 1e-3) / 1e9
    traffic = read_traffic(ab["forward"])
    out = {
        "metric": "megapixels/sec + % HBM roofline (batched vs per-frame); p50/p99 frame latency",
        "value": round(mp, 1),
        "unit": "megapixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["step_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "region-adaptive DP pixelization, %d RGB 1920x1080 uint8 frames, 8-rectangle "
                               "masks (~15%% cover), b=32 eps=1.0 simple / s_b=8 eps=0.3 complex, m=16, "
                               "plan+forward with fused reconstruction, one launch each for the whole batch, the "
                               "two C-ABI calls back to back on one stream" % args.frames,
                   "frames": args.frames, "resolution": "1920x1080x3", "b_bg": 32, "b_fg": 8, "m": 16,
                   "eps_bg": 1.0, "eps_fg": 0.3},
        "roofline": {"bound": "hbm", "achieved": round(fwd_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(fwd_gbs / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "kernel": "k_forward_u8<3>", "alg_bytes_per_launch": ab["forward"],
                     "avg_launch_ms": round(res["fwd_ms"], 4),
                     "timing": "HIP events around back-to-back launches on the library stream"},
        "plan_kernel": {"kernel": "k_plan + k_scan_prefix (one dp_pix_plan call)",
                        "avg_launch_ms": round(res["plan_ms"], 4),
                        "alg_bytes_per_launch": ab["mask"],
                        "gbs": round(ab["mask"] / (res["plan_ms"] * 1e-3) / 1e9, 1)},
        "step_gbs_algorithmic": round(step_gbs, 1),
        "step_frac_hbm": round(step_gbs / HBM_PEAK_GBS, 4),
        "graph_replayed_ms_per_step": None if res["other_step_ms"] is None else round(res["other_step_ms"], 4),
    }
    if not args.skip_extra:
        log("bench: per-frame launches")
        pf = run_per_frame(frames_s, dev, 10, max(3, min(args.steps, 50)))
        pf_gbs = pf["bytes"] / (pf["step_ms"] * 1e-3) / 1e9
        out["per_frame"] = {"value": round(pf["pixels"] / (pf["step_ms"] * 1e-3) / 1e6, 1), "unit": "megapixels/s",
                            "ms_per_step": round(pf["step_ms"], 3), "frac_hbm": round(pf_gbs / HBM_PEAK_GBS, 4)}
        del res
        torch.cuda.empty_cache()
        log("bench: uneven mixed-resolution batch (256 frames): autotuning its tile shapes")
        ub = synth.uneven_batch(256)
        tuned, launch, tinfo = autotune_batch(ub, dev)
        torch.cuda.empty_cache()
        log("bench: uneven batch, autotuned tiles (%.1f s of tuning) and default tiles" % tinfo["seconds"])
        u_steps = max(5, min(args.steps, 50))
        for key, kw in (("uneven_batch", dict(frames=tuned, **launch)),
                        ("uneven_batch_default_tiles", dict(threads=args.threads))):
            ur = run_batched(ub, dev, 15, u_steps, graph=True, **kw)
            u_gbs = ur["bytes"]["step"] / (ur["step_ms"] * 1e-3) / 1e9
            uf_gbs = ur["bytes"]["forward"] / (ur["fwd_ms"] * 1e-3) / 1e9
            out[key] = {"value": round(ur["pixels"] / (ur["step_ms"] * 1e-3) / 1e6, 1),
                        "unit": "megapixels/s", "ms_per_step": round(ur["step_ms"], 3),
                        "frames": 256, "gigapixels": round(ur["pixels"] / 1e9, 3),
                        "step_frac_hbm": round(u_gbs / HBM_PEAK_GBS, 4),
                        "forward_frac_hbm": round(uf_gbs / HBM_PEAK_GBS, 4)}
            if key == "uneven_batch":
                out[key]["autotune"] = tinfo
            del ur
            torch.cuda.empty_cache()
        del ub
    if not args.skip_extra:
        log("bench: single 256x256 frame latency")
        out["single_frame"] = run_single_frame(dev)
        log("bench: fp32 autograd batch (forward + adjoint)")
        out["autograd_batch"] = run_autograd_batch(dev)
        torch.cuda.empty_cache()
    if args.serve_seconds > 0 and not args.skip_extra:
        log("bench: serving %.0f s of 16 camera streams" % args.serve_seconds)
        out["serving"] = run_serving(dev, args.serve_seconds)
        out["p50_ms"] = out["serving"]["p50_ms"]
        out["p99_ms"] = out["serving"]["p99_ms"]
        torch.cuda.empty_cache()
    if not args.skip_cpu:
        log("bench: CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(frames_s, dev=dev)
        log("bench: CPU oracle sample on all host cores")
        out["cpu_baseline_all_cores"] = cpu_baseline_parallel(args.frames)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
