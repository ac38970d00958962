#!/usr/bin/env python3
"""Benchmark of region-adaptive DP pixelization on one MI355X.

A step is one pass of the whole hot path over one batch already resident in
HBM: plan (mask classification + store scan), forward (exact cell sums,
Laplace noise, clip, compact store) with the reconstruction fused in.

Headline workload: the uneven batch, 256 RGB frames with resolutions drawn
from {768x576, 1920x1080, 3840x2160, 6000x4000}, per-frame b in {16, 32},
s_b in {4, 8} and budgets, 8-rectangle foreground masks, tile shapes from the
autotuner, plan + forward captured once in a HIP graph and replayed per step.
Reported beside it: the 64-frame 1080p batch, both batches with the same
kernels launched once per frame, every other kernel of the library on its own,
the HBM ceilings of the streaming probes (linear and tile-shaped copies), the
single-frame latency, the fp32 autograd batch, the serving loop at the camera
rate and under heavier load, and the CPU oracle on a bounded sample.

Prints ONE JSON line.  Other modes (each prints its own line and exits):
--counters (short run for rocprofv3 --pmc), --class-batch, --kernel-legs
(profiling runs), --ceilings, --sweep-b (time against the cell size),
--serve-only, --dump-inputs.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_forward_uneven_x256_counters.txt")
#: untimed GPU work before each timed region: after the host has kept the GPU
#: idle (building inputs), its clocks take some 10 ms of load to settle
CLOCK_WARMUP_MS = 30.0
UNEVEN_FRAMES = 256
#: CPU share of one GPU on the MI355X machines (processes of the all-cores oracle)
CPU_SHARE = 16


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _code_only(text: str) -> str:
    """C/C++ source without comments and blank lines (the code the compiler sees)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())


def kernel_source_hash(root: str = ROOT) -> str:
    """Hash of the library's code (kernels, their headers, and the host side
    that lays out tiles and their order), so that a counter summary is only
    trusted for the build it was taken from."""
    h = hashlib.sha256()
    for name in ("dppix_kernels.hip", "dppix_internal.h", "dppix_tiles.h", "dppix_api.hip"):
        with open(os.path.join(root, "paper_2511_04261_amd", "csrc", name), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def launch_signature(plan) -> str:
    """Hash of what decides the forward's launches besides the kernels: every
    frame's geometry and tile width, and the workgroup size / launch mode."""
    h = hashlib.sha256()
    for fp, fi in zip(plan.frames, plan.info):
        h.update(("%d,%d,%d,%d,%d,%d;" % (fp.height, fp.width, fp.channels, fp.b, fp.sb or fp.b,
                                          fi.tile_cells)).encode())
    h.update(("threads=%d,persistent=%d" % (plan.threads, plan.persistent)).encode())
    return h.hexdigest()[:16]


def read_counters(path: str = COUNTERS_FILE) -> dict:
    kv = {}
    if not os.path.exists(path):
        return kv
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def read_traffic(plan):
    """HBM bytes per forward launch (average over the call's launches) from
    the committed rocprofv3 counter summary, scaled by the copy-kernel
    calibration; None when the kernels or the launch shapes changed since the
    counters were taken."""
    kv = read_counters()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if kv.get("launch_signature") != launch_signature(plan):
        return None
    try:
        fetch = float(kv["fetch_kib_per_dispatch"]) * 1024.0 * float(kv["fetch_scale"])
        write = float(kv["write_kib_per_dispatch"]) * 1024.0 * float(kv["write_scale"])
    except (KeyError, ValueError):
        return None
    return fetch + write


def load_inputs(frames_s, dev, inputs_dir=None, host_render=False):
    """Device images and masks of a batch: rendered on the device (default),
    on the host (byte-identical; no device kernels besides the library's, e.g.
    under a counter profiler), or loaded from files that --dump-inputs wrote."""
    import numpy as np
    import torch
    imgs, masks = [], []
    for i, s in enumerate(frames_s):
        if inputs_dir is not None:
            img = np.load(os.path.join(inputs_dir, "f%03d_img.npy" % i))
            mk = np.load(os.path.join(inputs_dir, "f%03d_mask.npy" % i))
            imgs.append(torch.from_numpy(img).to(dev))
            masks.append(torch.from_numpy(mk).to(dev))
        elif host_render:
            imgs.append(torch.from_numpy(s.image).to(dev))
            masks.append(torch.from_numpy(s.mask).to(dev))
            s.drop_host()
        else:
            imgs.append(s.image_torch(dev))
            masks.append(s.mask_torch(dev))
        if (inputs_dir is not None or host_render) and i % 32 == 31:
            log("inputs: %d of %d frames on the device" % (i + 1, len(frames_s)))
    return imgs, masks


def make_plan(frames_s, dev, frames=None, threads=0, persistent=0):
    import paper_2511_04261_amd as dp
    if frames is None:
        frames = [dp.FrameParams.from_spec(s) for s in frames_s]
    return dp.Plan(frames, device=dev, threads=threads, persistent=persistent)


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
    cells = sum(fi.grid_rows * fi.grid_cols for fi in plan.info)
    st = store_bytes(plan)
    return dict(image=px, mask=mask, recon=px, store=st, cells=cells, forward=2 * px + st, step=2 * px + mask + st,
                plan=mask + cells)


def warm_up(call, ms=CLOCK_WARMUP_MS):
    """Untimed calls until about `ms` of wall time has passed with the GPU busy."""
    import torch
    t0 = time.perf_counter()
    while True:
        for _ in range(4):
            call()
        torch.cuda.synchronize()
        if (time.perf_counter() - t0) * 1e3 >= ms:
            return


def time_steps(step_fn, warmup, steps):
    """Wall time of `steps` steps: `warmup` untimed steps, then about
    CLOCK_WARMUP_MS of untimed steps, then the timed steps bracketed by
    device synchronisation on both sides."""
    import torch
    for _ in range(warmup):
        step_fn()
    warm_up(step_fn)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step_fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def time_launches(call, n, stream):
    """Average duration of one call: n back-to-back calls between two HIP
    events on the stream the kernels run on, after a warm-up."""
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


def frac(nbytes, ms):
    gbs = nbytes / (ms * 1e-3) / 1e9
    return round(gbs, 1), round(gbs / HBM_PEAK_GBS, 4)


def run_batched(plan, imgs, masks, outs, warmup, steps, graph=False, compare=False):
    """Steps of plan + forward over one batch: replays of a captured HIP graph
    (graph=True) or the two C-ABI calls issued back to back on the stream; with
    compare=True the other form is timed too (other_step_ms)."""
    import torch
    stream = torch.cuda.current_stream()
    plan_call, fwd_call = plan.bound_calls(masks, imgs, outs, stream)
    g = plan.graph(masks, imgs, outs, stream) if (graph or compare) else None

    def step_graph():
        g.launch(stream)

    def step_calls():
        plan_call()
        fwd_call()

    dt = time_steps(step_graph if graph else step_calls, warmup, steps)
    other = None
    if compare:
        other = 1e3 * time_steps(step_calls if graph else step_graph, warmup, steps) / steps
    fwd_ms = time_launches(fwd_call, max(steps, 10), stream)
    plan_ms = time_launches(plan_call, max(steps, 10), stream)
    ab = alg_bytes(plan)
    if g is not None:
        g.close()
    return dict(seconds=dt, step_ms=1e3 * dt / steps, fwd_ms=fwd_ms, plan_ms=plan_ms, bytes=ab,
                pixels=sum(fp.height * fp.width for fp in plan.frames), other_step_ms=other,
                launches=int(plan.sizes.forward_launches))


def workload_key(frames) -> str:
    """Hash of a batch's frame parameters (the key of a tuning cache file)."""
    h = hashlib.sha256()
    for fp in frames:
        h.update(repr((fp.height, fp.width, fp.channels, fp.b, fp.sb, fp.m, fp.eps_bg, fp.eps_fg, fp.tau)).encode())
    return h.hexdigest()[:16]


def tuned_uneven(ub, dev, cache_path=None):
    """Tile shapes and launch shape of the uneven batch from the project's
    autotuner (whole-batch candidates timed on this batch), or from a cache
    file an earlier run on the same device wrote."""
    import torch
    import paper_2511_04261_amd as dp
    from paper_2511_04261_amd.autotune import Autotuner, with_tile_bytes
    frames = [dp.FrameParams.from_spec(s) for s in ub]
    key = workload_key(frames)
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            c = json.load(f)
        if c.get("workload") == key:
            log("bench: tile shapes from %s" % cache_path)
            c["info"]["from_cache"] = True
            return with_tile_bytes(frames, c["tile_bytes"]), dict(threads=c["threads"],
                                                                  persistent=c["persistent"]), c["info"]
    t0 = time.perf_counter()
    imgs, masks = load_inputs(ub, dev)
    tuner = Autotuner(dev, cache_path=None, reps=5, threads=(0, 128, 256), launch_modes=(0,))
    tuned, info = tuner.tune_whole_batch(frames, imgs, masks)
    del imgs, masks
    torch.cuda.empty_cache()
    summary = dict(seconds=round(time.perf_counter() - t0, 1), tile_bytes=info["tile_bytes"],
                   threads=info["threads"], candidates=len(info["tried"]), ms_best=round(info["ms"], 4),
                   ms_library_default=round(min(r["ms"] for r in info["tried"] if r["tile_bytes"] == 0
                                                and r["threads"] == 0), 4))
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(dict(workload=key, tile_bytes=info["tile_bytes"], threads=info["threads"],
                           persistent=info["persistent"], info=summary), f)
    return tuned, dict(threads=info["threads"], persistent=info["persistent"]), summary


def run_per_frame(frames_s, imgs, masks, outs, dev, warmup, steps, frames=None):
    """The same kernels launched once per frame (one plan per frame, the
    batch's own device buffers)."""
    import torch
    stream = torch.cuda.current_stream()
    plans = [make_plan([s], dev, None if frames is None else [frames[i]]) for i, s in enumerate(frames_s)]
    calls = [p.bound_calls([masks[i]], [imgs[i]], [outs[i]], stream) for i, p in enumerate(plans)]

    def step():
        for plan_call, fwd_call in calls:
            plan_call()
            fwd_call()

    dt = time_steps(step, warmup, steps)
    px = sum(s.height * s.width for s in frames_s)
    b = sum(alg_bytes(p)["step"] for p in plans)
    for p in plans:
        p.close()
    step_ms = 1e3 * dt / steps
    _, fr = frac(b, step_ms)
    return {"value": round(px / (step_ms * 1e-3) / 1e6, 1), "unit": "megapixels/s", "ms_per_step": round(step_ms, 3),
            "frac_hbm": fr, "frames": len(frames_s)}


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


def kernel_entry(name, ms, nbytes, launches=1, note=None):
    gbs, fr = frac(nbytes, ms)
    e = {"kernel": name, "avg_call_ms": round(ms, 4), "launches_per_call": launches, "alg_bytes_per_call": nbytes,
         "gbs": gbs, "frac_hbm": fr}
    if note:
        e["bytes"] = note
    return e


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
    counts = plan.counts.cpu().numpy()
    stats = sum(fp.channels * (int(c[0]) + fi.n * fi.n * int(c[1])) for fp, fi, c in zip(frames, plan.info, counts))
    cells = sum(fi.grid_rows * fi.grid_cols for fi in plan.info)
    # forward: frames read, reconstruction written, statistics (4 B) and
    # their clip bytes (1 B) written, flags read
    fwd_bytes = 2 * nbytes + 5 * stats + cells
    # adjoint: grad_out read, grad_in written, clip bytes read and statistic
    # gradients written (5 B per statistic), flags read and cell indices
    # written (5 B per cell); the border pass's re-reads are not counted
    bwd_bytes = 2 * nbytes + 5 * stats + 5 * cells
    plan.close()
    return dict(shape="32x3x512x512 fp32", forward_ms=round(fwd_ms, 4), backward_ms=round(bwd_ms, 4),
                forward_gbs=frac(fwd_bytes, fwd_ms)[0], backward_gbs=frac(bwd_bytes, bwd_ms)[0],
                forward=kernel_entry("k_forward_f32<3>", fwd_ms, fwd_bytes,
                                     note="frames read and written (4 B/value), 5 B per statistic, 1 B per cell"),
                backward=kernel_entry("k_backward_reduce + k_backward_mirror", bwd_ms, bwd_bytes, launches=2,
                                      note="grad_out read + grad_in written (4 B/value), 5 B per statistic, "
                                           "5 B per cell"))


def run_kernel_legs(plan, imgs, masks, outs, reps=20):
    """The library's other kernels on the 1080p batch, each call timed with
    HIP events over back-to-back calls: the plan on its own, standalone
    reconstruction, Sobel complexity labels, on-device MSE/SSIM."""
    import torch
    stream = torch.cuda.current_stream()
    plan.plan(masks)
    plan.forward(imgs, out=outs)
    ab = alg_bytes(plan)
    rec = plan.bound_reconstruct(outs, stream)
    rec_ms = time_launches(rec, reps, stream)
    edge_out = [torch.empty_like(m) for m in masks]
    edge_ms = time_launches(lambda: plan.edge_masks(imgs, 24, out=edge_out), reps, stream)
    labels_ms = time_launches(lambda: plan.plan_labels(imgs, 24), reps, stream)
    plan.plan(masks)
    met_ms = time_launches(lambda: plan.metrics(imgs, outs), reps, stream)
    plan_call, _ = plan.bound_calls(masks, imgs, outs, stream)
    plan_ms = time_launches(plan_call, reps, stream)
    return {
        "plan": kernel_entry("k_plan + k_scan_prefix", plan_ms, ab["plan"], launches=2,
                             note="mask read (1 B/px), flags written (1 B/cell)"),
        "reconstruct_u8": kernel_entry("k_reconstruct_u8<3>", rec_ms, ab["recon"] + ab["store"],
                                       note="store read (statistics + flags), frames written (3 B/px)"),
        "edge_mask": kernel_entry("k_edge_mask<3>", edge_ms, ab["image"] + ab["mask"],
                                  note="frames read (3 B/px), mask written (1 B/px)"),
        "plan_labels": kernel_entry("k_plan_labels + k_scan_prefix", labels_ms, ab["image"] + ab["cells"],
                                    launches=2, note="frames read (3 B/px), flags written (1 B/cell); "
                                                     "replaces edge_mask followed by plan"),
        "metrics": kernel_entry("k_metrics<3>", met_ms, 2 * ab["image"],
                                note="frame and reconstruction read (3 + 3 B/px)"),
    }


SERVE_PARAMS = dict(b=32, sb=8, m=16, eps_bg=1.0, eps_fg=0.3, tau=1)


def run_serving(dev, seconds, rate_scale=1.0, cap_bytes=8 << 30):
    """16 camera streams (8 x 1080p, 6 x 768x576, 2 x 2160p), Poisson arrivals
    at rate_scale x 30 Hz each, replayed in real time through the
    continuous-batching server."""
    from paper_2511_04261_amd.serving import (GpuBackend, MemoryLedger, Scheduler, camera_streams, latency_stats,
                                              serve_streams)
    be = GpuBackend(dev)
    warm = camera_streams(duration_s=1.0, pool=2, device=dev, seed=999)
    serve_streams(warm, Scheduler(be, MemoryLedger(cap_bytes)), SERVE_PARAMS)
    streams = camera_streams(duration_s=seconds, rate_hz=30.0 * rate_scale, pool=8, device=dev)
    sch = Scheduler(be, MemoryLedger(cap_bytes), max_batch=64, max_inflight=2)
    t0 = time.perf_counter()
    done = serve_streams(streams, sch, SERVE_PARAMS)
    wall = time.perf_counter() - t0
    st = latency_stats(done)
    ok = [r for r in done if r.error is None]
    px = sum(r.height * r.width for r in ok)
    offered = sum(s.height * s.width * len(s.arrivals) for s in streams)
    return dict(rate_hz_per_stream=30.0 * rate_scale, offered_megapixels_per_s=round(offered / seconds / 1e6, 1),
                p50_ms=round(st.get("p50_ms", float("nan")), 3), p99_ms=round(st.get("p99_ms", float("nan")), 3),
                max_ms=round(st.get("max_ms", float("nan")), 3), frames=len(ok), rejected=len(sch.rejected),
                megapixels_per_s=round(px / wall / 1e6, 1), seconds=round(wall, 2), streams=len(streams),
                batches=sch.batches, mean_batch=round(sum(sch.batch_sizes) / max(1, len(sch.batch_sizes)), 2),
                peak_admitted_bytes=sch.ledger.peak, plans_built=be.plans_built, plan_cache_hits=be.plan_hits,
                split_ms={k[len("split_"):]: round(v, 3) for k, v in st.items() if k.startswith("split_")})


def counters_run(ub, dev, inputs_dir=None, tune_cache=None, launches=3, copy_bytes=1 << 30):
    """Short run for rocprofv3 --pmc: one plain device copy of known size
    (the calibration of FETCH_SIZE / WRITE_SIZE), then a few plan + forward
    launches of the headline workload with the tile shapes the headline runs."""
    import torch
    if tune_cache is None or not os.path.exists(tune_cache):
        raise SystemExit("--counters needs --tune-cache with the headline run's tile shapes")
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
    tuned, launch, _ = tuned_uneven(ub, dev, tune_cache)
    plan = make_plan(ub, dev, tuned, **launch)
    imgs, masks = load_inputs(ub, dev, inputs_dir=inputs_dir, host_render=inputs_dir is None)
    outs = [torch.empty_like(t) for t in imgs]
    torch.cuda.synchronize()
    log("counters run: batch ready")
    for i in range(launches):
        plan.plan(masks)
        plan.forward(imgs, out=outs)
        torch.cuda.synchronize()
        log("counters run: launch %d done" % i)
    ab = alg_bytes(plan)
    log("counters run: calibration copy %d -> %d bytes; forward alg bytes %d per call" % (4 * n, n, ab["forward"]))
    print(json.dumps({"copy_read_bytes": 4 * n, "copy_write_bytes": n, "forward_alg_bytes": ab["forward"],
                      "forward_launches": int(plan.sizes.forward_launches),
                      "kernel_source_sha256_16": kernel_source_hash(),
                      "launch_signature": launch_signature(plan)}), flush=True)


def class_batch_run(spec, dev, launches=5):
    """Profiling run over a batch of one class, "HxW:b:s_b:frames" (RGB,
    8-rectangle masks, eps 1.0 / 0.3, m 16): frames rendered on the host, then
    a few plan + forward launches, one JSON line with the algorithmic bytes."""
    import torch
    from paper_2511_04261_amd import synth
    hw, b, sb, n = spec.split(":")
    H, W = (int(v) for v in hw.split("x"))
    frames_s = synth.region_batch(int(n), height=H, width=W, b=int(b), sb=int(sb))
    plan = make_plan(frames_s, dev)
    imgs, masks = load_inputs(frames_s, dev, host_render=True)
    outs = [torch.empty_like(t) for t in imgs]
    torch.cuda.synchronize()
    log("class batch %s: inputs ready" % spec)
    for i in range(launches):
        plan.plan(masks)
        plan.forward(imgs, out=outs)
        torch.cuda.synchronize()
    ab = alg_bytes(plan)
    log("class batch %s: %d launches done" % (spec, launches))
    print(json.dumps({"class_batch": spec, "forward_alg_bytes": ab["forward"], "plan_alg_bytes": ab["plan"],
                      "forward_launches": int(plan.sizes.forward_launches),
                      "kernel_source_sha256_16": kernel_source_hash()}), flush=True)


def ceilings_run(dev, reps=20):
    """Practical HBM ceilings of this machine, from the streaming probes
    (libdppix_probes.so, hand-written 16-byte non-temporal accesses): a linear
    copy, read and write of 1 GiB, and copies in the forward's tile shape --
    a workgroup reads a whole tile, waits at a barrier, then writes it -- over
    64 frames of 1088 rows x 5760 bytes cut into 32-row x 1920-byte tiles (the
    64-frame 1080p batch at b = 32), and over 5 frames of 4000 rows x 18000
    bytes (6000-pixel RGB rows, not a whole number of 128-byte lines) cut
    into 16-row and 32-row x 2016-byte tiles."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2511_04261_amd", "libdppix_probes.so"))
    lib.dppix_probe_stream.restype = ctypes.c_int
    lib.dppix_probe_stream.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_uint32, ctypes.c_void_p]
    lib.dppix_probe_tiles.restype = ctypes.c_int
    lib.dppix_probe_tiles.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_void_p]
    stream = torch.cuda.current_stream()
    sh = ctypes.c_void_p(stream.cuda_stream)

    def checked(rc):
        if rc != 0:
            raise RuntimeError("probe launch failed: hipError %d" % rc)

    out = {}
    n = 1 << 30
    a = torch.full((n,), 1, dtype=torch.uint8, device=dev)     # every 16-byte word xors to 0
    b = torch.empty(n, dtype=torch.uint8, device=dev)
    for name, mode, moved in (("copy", 0, 2 * n), ("read", 1, n), ("write", 2, n)):
        ms = time_launches(lambda: checked(lib.dppix_probe_stream(mode, a.data_ptr(), b.data_ptr(), n, 0xFFFFFFFF,
                                                                  sh)), reps, stream)
        gbs, fr = frac(moved, ms)
        out["stream_" + name] = dict(bytes=moved, ms=round(ms, 4), gbs=gbs, frac_hbm=fr)
        log("ceilings: %s %s" % (name, out["stream_" + name]))
    del a, b
    torch.cuda.empty_cache()
    for name, frames, rows, pitch, tile_rows, tile_bytes in (("tiles_1080p_x64_b32", 64, 1088, 5760, 32, 1920),
                                                            ("tiles_6000_x5_b16", 5, 4000, 18000, 16, 2016),
                                                            ("tiles_6000_x5_b32", 5, 4000, 18000, 32, 2016)):
        fb = rows * pitch
        a = torch.full((frames * fb,), 1, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        ms = time_launches(lambda: checked(lib.dppix_probe_tiles(a.data_ptr(), b.data_ptr(), frames, fb, pitch, rows,
                                                                 pitch, tile_rows, tile_bytes, sh)), reps, stream)
        moved = 2 * frames * fb
        gbs, fr = frac(moved, ms)
        out[name] = dict(frames=frames, rows=rows, pitch=pitch, tile_rows=tile_rows, tile_bytes=tile_bytes,
                         bytes=moved, ms=round(ms, 4), gbs=gbs, frac_hbm=fr)
        log("ceilings: %s %s" % (name, out[name]))
        del a, b
        torch.cuda.empty_cache()
    return out


def kernel_legs_run(dev, reps=3):
    """Profiling run of the standalone kernels (plan, reconstruction, Sobel
    labels as a mask and in the plan, metrics) on the 64-frame 1080p batch:
    inputs rendered on the host, a few calls of each, one JSON line with the
    per-call times and the kernel source hash."""
    import torch
    from paper_2511_04261_amd import synth
    c2 = synth.region_batch(64)
    plan = make_plan(c2, dev)
    imgs, masks = load_inputs(c2, dev, host_render=True)
    outs = [torch.empty_like(t) for t in imgs]
    torch.cuda.synchronize()
    log("kernel legs: inputs ready")
    legs = run_kernel_legs(plan, imgs, masks, outs, reps=reps)
    plan.close()
    print(json.dumps({"kernel_legs": legs, "kernel_source_sha256_16": kernel_source_hash()}), flush=True)


SWEEP_B = (2, 4, 8, 12, 16, 20, 32)


def sweep_b_run(dev, steps=20):
    """Step time against the cell size b (Sec. VII's timing against block
    size, in shape): 64 RGB 1920x1080 frames and 300 RGB 768x576 frames (about
    the same pixel count), s_b = b / 2 (1 at b = 2), 8-rectangle masks,
    eps 1.0 / 0.3, m 16, default tiles, plan + forward replayed from a HIP
    graph.  Frames whose sides b does not divide are padded virtually, so a
    bandwidth-bound pass should give about the same rate at every b."""
    import torch
    from paper_2511_04261_amd import synth
    rows = []
    for (H, W, n) in ((1080, 1920, 64), (576, 768, 300)):
        for b in SWEEP_B:
            sb = max(1, b // 2)
            frames_s = synth.region_batch(n, height=H, width=W, b=b, sb=sb)
            plan = make_plan(frames_s, dev)
            imgs, masks = load_inputs(frames_s, dev)
            outs = [torch.empty_like(t) for t in imgs]
            r = run_batched(plan, imgs, masks, outs, 5, steps, graph=True)
            ab = r["bytes"]
            row = dict(frame="%dx%d" % (W, H), frames=n, b=b, s_b=sb, step_ms=round(r["step_ms"], 4),
                       megapixels_per_s=round(r["pixels"] / (r["step_ms"] * 1e-3) / 1e6, 1),
                       step_frac_hbm=frac(ab["step"], r["step_ms"])[1], forward_ms=round(r["fwd_ms"], 4),
                       forward_frac_hbm=frac(ab["forward"], r["fwd_ms"])[1], plan_ms=round(r["plan_ms"], 4))
            log("sweep b: %s" % row)
            rows.append(row)
            plan.close()
            del plan, imgs, masks, outs
            torch.cuda.empty_cache()
    print(json.dumps({"sweep_b": rows, "kernel_source_sha256_16": kernel_source_hash()}), flush=True)


def dump_inputs(ub, dev, path):
    """Render the batch on the device and save it as .npy files (for the
    counter runs, which must not launch the rendering kernels)."""
    import numpy as np
    os.makedirs(path, exist_ok=True)
    for i, s in enumerate(ub):
        np.save(os.path.join(path, "f%03d_img.npy" % i), s.image_torch(dev).cpu().numpy())
        np.save(os.path.join(path, "f%03d_mask.npy" % i), s.mask_torch(dev).cpu().numpy())
        if i % 32 == 31:
            log("dump: %d of %d frames written" % (i + 1, len(ub)))


def _oracle_params(s):
    import oracle
    return oracle.Params(s.height, s.width, s.channels, b=s.b, sb=s.sb, m=s.m, eps_simple=s.eps_simple,
                         eps_complex=s.eps_complex, tau=s.tau, seed=s.seed, frame_index=s.frame_index)


def cpu_baseline(frames_s, budget_s=15.0, dev=None):
    """The oracle as it stands, single-threaded, on a bounded sample of the
    headline workload: its frames in batch order until about budget_s of
    oracle time."""
    import oracle
    oracle.build()
    dt = 0.0
    done = px = 0
    for s in frames_s:
        # inputs rendered on the device and copied back (byte-identical), not timed
        img = s.image_torch(dev).cpu().numpy() if dev is not None else s.image
        mask = s.mask
        t1 = time.perf_counter()
        oracle.forward(img, mask, _oracle_params(s))
        dt += time.perf_counter() - t1
        done += 1
        px += s.height * s.width
        s.drop_host()
        if dt > budget_s:
            break
    return dict(value=round(px / dt / 1e6, 3), unit="megapixels/s", cores=1, kind="oracle",
                sample="the first %d frames of the %d-frame uneven batch (%.2f gigapixels, same parameters), "
                       "single thread, %.1f s of oracle time" % (done, len(frames_s), px / 1e9, dt))


def cpu_worker(frames_s, k, procs, budget_s):
    """One worker of the parallel oracle baseline: frames k, k+procs, ...
    rendered on the host (untimed), then the oracle over them until about
    budget_s of oracle time.  Prints one JSON line."""
    import oracle
    mine = frames_s[k::procs]
    dt, px, done = 0.0, 0, 0
    while dt < budget_s:
        for s in mine:
            img, mask = s.image, s.mask
            t1 = time.perf_counter()
            oracle.forward(img, mask, _oracle_params(s))
            dt += time.perf_counter() - t1
            px += s.height * s.width
            done += 1
            if dt >= budget_s:
                break
    print(json.dumps({"px": px, "seconds": dt, "frames": done}), flush=True)


def cpu_baseline_parallel(n_frames, budget_s=10.0):
    """The same oracle, one single-threaded process per core of the host's
    share for this GPU (the affinity mask, at most CPU_SHARE cores), frames
    distributed round-robin.  Workers are child processes that never touch
    the GPU."""
    import subprocess
    import oracle
    oracle.build()
    nproc = os.cpu_count() or 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = nproc
    procs = max(1, min(CPU_SHARE, affinity, n_frames))
    log("bench: oracle on %d processes (nproc %d, affinity %d cores, share %d)" % (procs, nproc, affinity,
                                                                                  CPU_SHARE))
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
    return dict(value=round(rate / 1e6, 3), unit="megapixels/s", cores=procs, nproc=nproc, affinity_cores=affinity,
                kind="oracle",
                sample="%d single-threaded processes (one per core of the %d-core affinity mask, at most %d, the CPU "
                       "share of one GPU) over the %d-frame uneven batch, frames round-robin, host-rendered "
                       "(untimed); %d frame passes, about %.1f s of oracle time each" % (
                           procs, affinity, CPU_SHARE, n_frames, frames, seconds))


def headline_entry(out, res, plan, tinfo, launch, warmup):
    ab = res["bytes"]
    launches = res["launches"]
    fwd_gbs, fwd_frac = frac(ab["forward"], res["fwd_ms"])
    step_gbs, step_frac = frac(ab["step"], res["step_ms"])
    traffic = read_traffic(plan)
    out.update({
        "value": round(res["pixels"] / (res["step_ms"] * 1e-3) / 1e6, 1),
        "ms_per_step": round(res["step_ms"], 4),
        "config": {"workload": "region-adaptive DP pixelization, uneven batch of %d RGB uint8 frames, resolutions "
                               "uniform over 768x576 / 1920x1080 / 3840x2160 / 6000x4000, per frame b in {16, 32}, "
                               "s_b in {4, 8}, eps_simple ~ U[0.5, 2], eps_complex ~ U[0.1, 0.5], m=16, "
                               "8-rectangle masks (~15%% cover), tiles from the autotuner, plan + forward with fused "
                               "reconstruction captured in one HIP graph and replayed per step" % len(plan.frames),
                   "frames": len(plan.frames), "gigapixels": round(res["pixels"] / 1e9, 4),
                   "tile_bytes": tinfo.get("tile_bytes"), "threads": launch["threads"],
                   "persistent": launch["persistent"]},
        "roofline": {"bound": "hbm", "achieved": fwd_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fwd_frac,
                     "traffic": None if traffic is None else round(traffic),
                     "kernel": "k_forward_u8<3>", "launches_per_call": launches,
                     "alg_bytes_per_launch": round(ab["forward"] / launches),
                     "avg_launch_ms": round(res["fwd_ms"] / launches, 4),
                     "timing": "HIP events around back-to-back dp_pix_forward calls on the library stream; a call "
                               "is one launch per group of frames sharing a workgroup size, and per-launch figures "
                               "are the call's divided by its launches"},
        "plan_kernel": {"kernel": "k_plan + k_scan_prefix, or k_plan + k_scan_tiles + k_scan_frames (one dp_pix_plan call)",
                        "avg_call_ms": round(res["plan_ms"], 4), "alg_bytes_per_call": ab["plan"],
                        "gbs": frac(ab["plan"], res["plan_ms"])[0]},
        "step_gbs_algorithmic": step_gbs,
        "step_frac_hbm": step_frac,
        "calls_ms_per_step": None if res["other_step_ms"] is None else round(res["other_step_ms"], 4),
        "autotune": tinfo,
        "clock_warmup": "%d warm-up steps, then about %.0f ms of untimed steps, before the timed steps" % (
            warmup, CLOCK_WARMUP_MS),
    })


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--frames", type=int, default=UNEVEN_FRAMES)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-extra", action="store_true", help="only the headline workload")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="seconds of camera-stream arrivals for the latency leg (0 skips it)")
    ap.add_argument("--load-seconds", type=float, default=20.0,
                    help="seconds of arrivals for each heavier-load serving leg (0 skips them)")
    ap.add_argument("--tune-cache", default=None, help="JSON file of the uneven batch's tuned tile shapes")
    ap.add_argument("--counters", action="store_true", help="short run for rocprofv3 --pmc")
    ap.add_argument("--inputs", default=None, help="directory of .npy inputs from --dump-inputs")
    ap.add_argument("--dump-inputs", default=None, help="write the uneven batch's inputs here and exit")
    ap.add_argument("--class-batch", default=None, help="profiling run over one class, HxW:b:s_b:frames")
    ap.add_argument("--sweep-b", action="store_true", help="step time against the cell size b, then exit")
    ap.add_argument("--ceilings", action="store_true", help="the streaming probes' HBM ceilings, then exit")
    ap.add_argument("--kernel-legs", action="store_true",
                    help="profiling run of the standalone kernels on the 64-frame 1080p batch (host-rendered inputs)")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the serving leg (--serve-seconds of camera streams), then exit")
    ap.add_argument("--cpu-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-index", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-procs", type=int, default=1, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-budget", type=float, default=10.0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the method shards by frame with no collective, "
              "so --gpus N>1 is not run here", file=sys.stderr)
        sys.exit(2)

    from paper_2511_04261_amd import synth
    if args.cpu_worker:
        cpu_worker(synth.uneven_batch(args.frames), args.cpu_index, args.cpu_procs, args.cpu_budget)
        return

    import torch
    dev = torch.device("cuda:0")
    if args.class_batch:
        class_batch_run(args.class_batch, dev)
        return
    if args.sweep_b:
        sweep_b_run(dev)
        return
    if args.kernel_legs:
        kernel_legs_run(dev)
        return
    if args.ceilings:
        print(json.dumps({"ceilings": ceilings_run(dev)}), flush=True)
        return
    if args.serve_only:
        log("bench: serving %.0f s of 16 camera streams" % args.serve_seconds)
        print(json.dumps({"serving": run_serving(dev, args.serve_seconds)}), flush=True)
        return
    log("bench: uneven batch of %d frames" % args.frames)
    ub = synth.uneven_batch(args.frames)
    if args.dump_inputs:
        dump_inputs(ub, dev, args.dump_inputs)
        return
    if args.counters:
        counters_run(ub, dev, args.inputs, args.tune_cache)
        return

    log("bench: tile shapes of the uneven batch")
    tuned, launch, tinfo = tuned_uneven(ub, dev, args.tune_cache)
    plan = make_plan(ub, dev, tuned, **launch)
    imgs, masks = load_inputs(ub, dev)
    outs = [torch.empty_like(t) for t in imgs]
    log("bench: uneven batch, graph-replayed steps")
    res = run_batched(plan, imgs, masks, outs, args.warmup, args.steps, graph=True, compare=True)
    out = {
        "metric": "megapixels/sec + % HBM roofline (batched vs per-frame); p50/p99 frame latency",
        "value": None, "unit": "megapixels/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
    }
    headline_entry(out, res, plan, tinfo, launch, args.warmup)
    if not args.skip_extra:
        log("bench: uneven batch, per-frame launches")
        out["per_frame"] = run_per_frame(ub, imgs, masks, outs, dev, 2, max(3, min(args.steps, 10)), frames=tuned)
    plan.close()
    del plan, imgs, masks, outs, res
    torch.cuda.empty_cache()

    if not args.skip_extra:
        log("bench: 64-frame 1080p batch")
        c2 = synth.region_batch(64)
        p2 = make_plan(c2, dev)
        i2, m2 = load_inputs(c2, dev)
        o2 = [torch.empty_like(t) for t in i2]
        r2 = run_batched(p2, i2, m2, o2, args.warmup, max(args.steps, 50), graph=True, compare=True)
        ab = r2["bytes"]
        fg, ff = frac(ab["forward"], r2["fwd_ms"])
        _, sf = frac(ab["step"], r2["step_ms"])
        out["region_1080p_x64"] = {
            "value": round(r2["pixels"] / (r2["step_ms"] * 1e-3) / 1e6, 1), "unit": "megapixels/s",
            "ms_per_step": round(r2["step_ms"], 4), "calls_ms_per_step": round(r2["other_step_ms"], 4),
            "step_frac_hbm": sf, "forward": {"kernel": "k_forward_u8<3>", "avg_launch_ms": round(r2["fwd_ms"], 4),
                                             "alg_bytes_per_launch": ab["forward"], "gbs": fg, "frac_hbm": ff},
            "config": "64 RGB 1920x1080 frames, b=32 eps=1.0 simple / s_b=8 eps=0.3 complex, m=16, 8-rectangle "
                      "masks (~15% cover), default tiles, graph-replayed"}
        log("bench: 1080p batch, per-frame launches")
        out["region_1080p_x64"]["per_frame"] = run_per_frame(c2, i2, m2, o2, dev, 3, max(3, min(args.steps, 20)))
        log("bench: standalone kernels on the 1080p batch")
        out["kernels"] = run_kernel_legs(p2, i2, m2, o2)
        p2.close()
        del p2, i2, m2, o2, r2
        torch.cuda.empty_cache()
        log("bench: HBM ceilings of the streaming probes")
        out["ceilings"] = ceilings_run(dev)
        log("bench: single 256x256 frame latency")
        out["single_frame"] = run_single_frame(dev)
        log("bench: fp32 autograd batch (forward + adjoint)")
        ag = run_autograd_batch(dev)
        out["kernels"]["forward_f32"] = ag.pop("forward")
        out["kernels"]["backward_f32"] = ag.pop("backward")
        out["autograd_batch"] = ag
        torch.cuda.empty_cache()
    if args.serve_seconds > 0 and not args.skip_extra:
        log("bench: serving %.0f s of 16 camera streams" % args.serve_seconds)
        out["serving"] = run_serving(dev, args.serve_seconds)
        out["p50_ms"] = out["serving"]["p50_ms"]
        out["p99_ms"] = out["serving"]["p99_ms"]
        torch.cuda.empty_cache()
        if args.load_seconds > 0:
            out["serving_load"] = []
            for scale in (4.0, 8.0):
                log("bench: serving %.0f s of 16 streams at %.0fx the camera rate" % (args.load_seconds, scale))
                out["serving_load"].append(run_serving(dev, args.load_seconds, rate_scale=scale))
                torch.cuda.empty_cache()
    if not args.skip_cpu:
        log("bench: CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(ub, dev=dev)
        log("bench: CPU oracle sample on all host cores")
        out["cpu_baseline_all_cores"] = cpu_baseline_parallel(args.frames)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
