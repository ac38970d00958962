"""Continuous-batching server for many camera streams (not in the paper; the
paper motivates real-time use but times one frame at a time).

Requests (one frame of one stream) arrive at any time.  The scheduler admits
them while the device-memory ledger has room, starts each admitted frame's
host-to-device copy at once on a copy stream, and launches every admitted,
copied frame as one batch (one plan, one forward launch) as soon as fewer
than ``max_inflight`` batches are on the GPU — so frames that arrive while a
batch runs are copied during it and join the next one.  Each frame keeps its
own Philox counter (its stream and its sequence number in it), so its result
is the same alone or in any mix; streams differ in the counter's high bits,
so no two frames of any streams share noise (``StreamCounters``, which also
saves and restores the counters so that resumed streams continue them).
Completions, admissions and launches are ROCTx ranges (``markers``), so a
marker trace shows the loop's host phases beside its kernels.

The scheduler is host logic over a small backend interface; ``GpuBackend``
drives libdppix, and the tests drive the same scheduler with a CPU backend.
"""
from __future__ import annotations

import collections
import ctypes
import gc
import math
import time
from dataclasses import dataclass, field
from typing import Any, Deque, Dict, List, Optional

import numpy as np

from .markers import marker_range
from .store_codec import privacy_ledger


@dataclass
class Request:
    rid: int
    stream: int
    frame_index: int
    height: int
    width: int
    channels: int
    b: int
    sb: int
    m: int
    eps_bg: float
    eps_fg: float
    tau: int
    seed: int
    image: Any = None            # host uint8 (H, W, C) (numpy or pinned torch)
    mask: Any = None             # host uint8 (H, W) or None
    arrival: float = 0.0
    admitted: Optional[float] = None
    launched: Optional[float] = None
    done: Optional[float] = None
    result: Optional[dict] = None
    error: Optional[str] = None
    nbytes: int = 0
    state: Any = None            # backend bookkeeping
    timing: Optional[dict] = None  # backend's split of the in-flight time (ms)

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class MemoryLedger:
    """Device bytes held by admitted, unfinished requests."""

    def __init__(self, cap_bytes: int):
        self.cap = int(cap_bytes)
        self.used = 0
        self.peak = 0

    def try_reserve(self, n: int) -> bool:
        if self.used + n > self.cap:
            return False
        self.used += n
        self.peak = max(self.peak, self.used)
        return True

    def release(self, n: int):
        self.used -= n
        assert self.used >= 0


class Scheduler:
    """Admission by memory, continuous batching, completion polling."""

    def __init__(self, backend, ledger: MemoryLedger, max_batch: int = 64, max_inflight: int = 2,
                 max_queue: int = 4096, clock=time.perf_counter, on_done=None):
        """on_done(request), if given, runs for every finished request right
        after its result is set (e.g. to hand the result on and drop it)."""
        self.backend = backend
        self.on_done = on_done
        self.ledger = ledger
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.max_queue = max_queue
        self.clock = clock
        self.queue: Deque[Request] = collections.deque()     # waiting for memory
        self.admitted: List[Request] = []                     # copying / ready, not launched
        self.inflight: Deque[Any] = collections.deque()       # (handle, [requests])
        self.finished: List[Request] = []
        self.rejected: List[Request] = []
        self.batches = 0
        self.batch_sizes: List[int] = []

    # -- intake ------------------------------------------------------------
    def offer(self, req: Request):
        err = self.backend.validate(req)
        if err is not None:
            req.error = err
            req.done = self.clock()
            self.rejected.append(req)
            return
        req.nbytes = self.backend.request_bytes(req)
        if req.nbytes > self.ledger.cap:
            req.error = "request needs %d bytes, above the memory cap %d" % (req.nbytes, self.ledger.cap)
            req.done = self.clock()
            self.rejected.append(req)
            return
        if len(self.queue) >= self.max_queue:
            req.error = "queue full"
            req.done = self.clock()
            self.rejected.append(req)
            return
        self.queue.append(req)

    # -- one turn of the loop ----------------------------------------------
    def pump(self) -> int:
        """Admit, launch, complete; returns how many requests changed state."""
        moved = 0
        # completions first: they free memory for admissions
        while self.inflight and self.backend.poll(self.inflight[0][0]):
            handle, reqs = self.inflight.popleft()
            now = self.clock()
            with marker_range("dppix.serve.collect[%d]" % len(reqs)):
                results = self.backend.collect(handle)
            for r, res in zip(reqs, results):
                r.result = res
                r.done = now
                self.ledger.release(r.nbytes)
                self.backend.release(r)
                self.finished.append(r)
                if self.on_done is not None:
                    self.on_done(r)
                moved += 1
        # admissions in arrival order; a request that does not fit blocks the
        # ones behind it (no overtaking, so per-stream order holds)
        while self.queue and self.ledger.try_reserve(self.queue[0].nbytes):
            r = self.queue.popleft()
            r.admitted = self.clock()
            with marker_range("dppix.serve.admit"):
                self.backend.admit(r)
            self.admitted.append(r)
            moved += 1
        # launch everything admitted (up to max_batch) when a batch slot is free
        if self.admitted and len(self.inflight) < self.max_inflight:
            batch = self.admitted[: self.max_batch]
            self.admitted = self.admitted[self.max_batch:]
            now = self.clock()
            for r in batch:
                r.launched = now
            try:
                with marker_range("dppix.serve.launch[%d]" % len(batch)):
                    handle = self.backend.launch(batch)
                self.inflight.append((handle, batch))
                self.batches += 1
                self.batch_sizes.append(len(batch))
            except Exception:
                # isolate the request that fails: relaunch each one alone
                for r in batch:
                    try:
                        with marker_range("dppix.serve.launch[1]"):
                            handle = self.backend.launch([r])
                        self.inflight.append((handle, [r]))
                        self.batches += 1
                        self.batch_sizes.append(1)
                    except Exception as e:  # this request alone is bad
                        r.error = "%s: %s" % (type(e).__name__, e)
                        r.done = self.clock()
                        self.ledger.release(r.nbytes)
                        self.backend.release(r)
                        self.rejected.append(r)
            moved += len(batch)
        return moved

    def idle(self) -> bool:
        return not self.queue and not self.admitted and not self.inflight

    def drain(self, timeout_s: float = 60.0):
        t0 = self.clock()
        while not self.idle():
            if self.pump() == 0:
                time.sleep(1e-4)
            if self.clock() - t0 > timeout_s:
                raise TimeoutError("scheduler did not drain")


def latency_stats(reqs: List[Request]) -> Dict[str, float]:
    """Percentiles of arrival -> result latency over the requests that
    finished, and where that time went: waiting for memory (arrival ->
    admitted), waiting for a batch slot while the frame's copy runs (admitted
    -> launched), in flight (launched -> done), and the backend's own split of
    the in-flight time when it records one (``Request.timing``)."""
    ok = [r for r in reqs if r.latency is not None and r.error is None]
    lat = np.array([r.latency for r in ok])
    if lat.size == 0:
        return dict(n=0)
    out = dict(n=int(lat.size), p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
               max_ms=float(lat.max() * 1e3), mean_ms=float(lat.mean() * 1e3))
    parts = {"queue": [r.admitted - r.arrival for r in ok if r.admitted is not None],
             "wait_launch": [r.launched - r.admitted for r in ok if r.launched is not None and r.admitted is not None],
             "in_flight": [r.done - r.launched for r in ok if r.launched is not None]}
    for name, vals in parts.items():
        if vals:
            v = np.asarray(vals) * 1e3
            out["split_%s_mean_ms" % name] = float(v.mean())
            out["split_%s_p99_ms" % name] = float(np.percentile(v, 99))
    keys = sorted({k for r in ok if r.timing for k in r.timing})
    for k in keys:
        v = np.asarray([r.timing[k] for r in ok if r.timing and k in r.timing])
        out["split_%s_mean_ms" % k] = float(v.mean())
        out["split_%s_p99_ms" % k] = float(np.percentile(v, 99))
    return out


# ---------------------------------------------------------------------------
# GPU backend over libdppix
# ---------------------------------------------------------------------------
class GpuBackend:
    """Frames are copied host->device on a copy stream at admission; a batch
    waits for its copies on the compute stream, runs plan + forward (optionally
    with the fused reconstruction), and its store is copied back on the copy
    stream into pinned host memory.

    Plans stay bound on the device and are reused: a batch is ordered by
    frame geometry, and its plan is looked up by the sequence of geometries
    (frames of one geometry are interchangeable in a plan).  The frames'
    Philox counters reach the kernels through the store's noise array (one
    pinned upload of 16 bytes per frame), so a cached plan serves any frames
    of its composition.  Each plan keeps a few stores, one per batch in
    flight."""

    MAX_PLANS = 512

    def __init__(self, device=None, reconstruct: bool = False, persistent: int = 0):
        import torch
        import paper_2511_04261_amd as dp
        self.torch = torch
        self.dp = dp
        self.device = torch.device(device if device is not None else "cuda:0")
        self.reconstruct = reconstruct
        self.persistent = persistent
        self.copy_stream = torch.cuda.Stream(self.device)
        self.compute_stream = torch.cuda.Stream(self.device)
        self._pool: Dict[tuple, List[Any]] = collections.defaultdict(list)
        self._plans: "collections.OrderedDict[tuple, dict]" = collections.OrderedDict()
        self.plans_built = 0
        self.plan_hits = 0

    def frame_params(self, r: Request):
        return self.dp.FrameParams(r.height, r.width, r.channels, self.dp.U8_HWC, r.b, r.sb, r.m, r.eps_bg,
                                   r.eps_fg, r.tau, self.dp.PAD_SYMMETRIC, r.seed, r.frame_index)

    @staticmethod
    def geometry_key(r: Request) -> tuple:
        """Everything of a frame that its plan depends on (not its counter)."""
        return (r.height, r.width, r.channels, r.b, r.sb, r.m, r.eps_bg, r.eps_fg, r.tau)

    def validate(self, r: Request) -> Optional[str]:
        lib = self.dp._lib.load()
        d = (self.dp._lib.FrameDesc * 1)(self.frame_params(r).desc())
        h = ctypes.c_void_p()
        st = lib.dp_pix_plan_create(d, 1, ctypes.byref(h))
        if st != 0:
            return lib.dp_pix_last_error().decode(errors="replace")
        lib.dp_pix_plan_destroy(h)
        if r.image is None or tuple(r.image.shape[:2]) != (r.height, r.width):
            return "image does not match the request geometry"
        return None

    def request_bytes(self, r: Request) -> int:
        n = r.b // r.sb
        cells = -(-r.height // r.b) * -(-r.width // r.b)
        img = r.height * r.width * r.channels
        store = 4 * cells * r.channels * (1 + n * n) + cells
        return img + r.height * r.width + store + (img if self.reconstruct else 0)

    def _buf(self, shape, dtype):
        lst = self._pool[(shape, dtype)]
        if lst:
            return lst.pop()
        return self.torch.empty(shape, dtype=dtype, device=self.device)

    def admit(self, r: Request):
        torch = self.torch
        img = self._buf(tuple(r.image.shape), torch.uint8)
        mk = None if r.mask is None else self._buf(tuple(r.mask.shape), torch.uint8)
        with torch.cuda.stream(self.copy_stream):
            src = r.image if isinstance(r.image, torch.Tensor) else torch.from_numpy(r.image)
            img.copy_(src, non_blocking=True)
            if mk is not None:
                msrc = r.mask if isinstance(r.mask, torch.Tensor) else torch.from_numpy(r.mask)
                mk.copy_(msrc, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
        r.state = dict(img=img, mask=mk, ev=ev)

    def _plan_for(self, keys: tuple, reqs: List[Request]) -> dict:
        """The cached plan of this composition (built and bound on a miss)."""
        ent = self._plans.get(keys)
        if ent is not None:
            self._plans.move_to_end(keys)
            self.plan_hits += 1
            return ent
        plan = self.dp.Plan([self.frame_params(r) for r in reqs], device=self.device, persistent=self.persistent,
                            default_store=False)
        ent = dict(plan=plan, free=[])
        self._plans[keys] = ent
        self.plans_built += 1
        while len(self._plans) > self.MAX_PLANS:
            _, old = self._plans.popitem(last=False)
            old["plan"].close()
        return ent

    def _store_for(self, ent: dict) -> dict:
        """A store of the plan that no batch in flight uses, with its device
        table and the pinned host buffer that fills it: per frame the noise
        counters (seed, frame_index), then the image, mask and output pointer
        arrays the kernels read (one host-to-device copy per batch)."""
        if ent["free"]:
            return ent["free"].pop()
        torch = self.torch
        n = len(ent["plan"].frames)
        table = torch.zeros(5 * n, dtype=torch.int64, device=self.device)
        return dict(store=ent["plan"].new_store(noise=table[: 2 * n].view(n, 2)), table=table,
                    host=torch.zeros(5 * n, dtype=torch.int64).pin_memory())

    def launch(self, batch: List[Request]):
        torch = self.torch
        t_host = time.perf_counter()
        order = sorted(range(len(batch)), key=lambda i: self.geometry_key(batch[i]))
        reqs = [batch[i] for i in order]
        keys = tuple(self.geometry_key(r) for r in reqs)
        ent = self._plan_for(keys, reqs)
        plan = ent["plan"]
        st = self._store_for(ent)
        n = len(reqs)
        ht = st["host"].numpy().view(np.uint64)
        outs = [self._buf(tuple(r.state["img"].shape), torch.uint8) for r in reqs] if self.reconstruct else None
        any_mask = False
        for i, r in enumerate(reqs):
            ht[2 * i] = r.seed & (2**64 - 1)
            ht[2 * i + 1] = r.frame_index & (2**64 - 1)
            ht[2 * n + i] = r.state["img"].data_ptr()
            mk = r.state["mask"]
            ht[3 * n + i] = 0 if mk is None else mk.data_ptr()
            any_mask = any_mask or mk is not None
            ht[4 * n + i] = 0 if outs is None else outs[i].data_ptr()
        lib, h, sc = plan.lib, plan.handle, ctypes.byref(st["store"].c)
        base = st["table"].data_ptr()
        imgs_p = ctypes.c_void_p(base + 8 * 2 * n)
        masks_p = ctypes.c_void_p(base + 8 * 3 * n) if any_mask else None
        outs_p = ctypes.c_void_p(base + 8 * 4 * n) if outs is not None else None
        with torch.cuda.stream(self.compute_stream):
            for r in reqs:
                self.compute_stream.wait_event(r.state["ev"])
            start = torch.cuda.Event(enable_timing=True)
            start.record(self.compute_stream)
            st["table"].copy_(st["host"], non_blocking=True)
            sh = ctypes.c_void_p(self.compute_stream.cuda_stream)
            self.dp._lib.check(lib.dp_pix_plan(h, masks_p, sc, sh))
            self.dp._lib.check(lib.dp_pix_forward(h, imgs_p, sc, None, None, outs_p, sh))
            done = torch.cuda.Event(enable_timing=True)
            done.record(self.compute_stream)
        # store back to pinned host memory on the copy stream
        store = st["store"]
        with torch.cuda.stream(self.copy_stream):
            self.copy_stream.wait_event(done)
            host = dict(counts=store.counts.to("cpu", non_blocking=True), bg=store.bg.to("cpu", non_blocking=True),
                        fg=store.fg.to("cpu", non_blocking=True), flags=store.flags.to("cpu", non_blocking=True))
            if outs is not None:
                host["recon"] = [o.to("cpu", non_blocking=True) for o in outs]
            fin = torch.cuda.Event(enable_timing=True)
            fin.record(self.copy_stream)
        host_ms = (time.perf_counter() - t_host) * 1e3
        return dict(ent=ent, st=st, host=host, start=start, done=done, fin=fin, outs=outs, order=order,
                    host_ms=host_ms, batch=batch)

    def poll(self, handle) -> bool:
        return handle["fin"].query()

    def collect(self, handle) -> List[dict]:
        plan, host = handle["ent"]["plan"], handle["host"]
        counts = host["counts"].numpy()
        bg, fg, flags = host["bg"].numpy(), host["fg"].numpy(), host["flags"].numpy()
        timing = dict(host_launch=handle["host_ms"], gpu=handle["start"].elapsed_time(handle["done"]),
                      d2h=handle["done"].elapsed_time(handle["fin"]))
        res: List[Optional[dict]] = [None] * len(handle["order"])
        for f, (fp, fi) in enumerate(zip(plan.frames, plan.info)):
            nb, nf, ob, of = (int(x) for x in counts[f])
            C, nn = fp.channels, fi.n * fi.n
            d = dict(flags=flags[fi.cell_offset: fi.cell_offset + fi.grid_rows * fi.grid_cols].reshape(
                fi.grid_rows, fi.grid_cols).copy(), bg=bg[ob: ob + nb * C].reshape(nb, C).copy(),
                fg=fg[of: of + nf * nn * C].reshape(nf, nn, C).copy(), counts=(nb, nf))
            if "recon" in host:
                d["recon"] = host["recon"][f].numpy()
            # the request's own parameters: a cached plan's frame records keep
            # the counters of the batch it was built for
            r = handle["batch"][handle["order"][f]]
            d["ledger"] = dict(privacy_ledger(C, r.m, r.eps_bg, r.eps_fg), frame_index=r.frame_index)
            res[handle["order"][f]] = d
        for r in handle["batch"]:
            r.timing = dict(timing)
        if handle["outs"] is not None:
            for o in handle["outs"]:
                self._pool[(tuple(o.shape), self.torch.uint8)].append(o)
        handle["ent"]["free"].append(handle["st"])
        return res

    def release(self, r: Request):
        st = r.state or {}
        if st.get("img") is not None:
            self._pool[(tuple(st["img"].shape), self.torch.uint8)].append(st["img"])
        if st.get("mask") is not None:
            self._pool[(tuple(st["mask"].shape), self.torch.uint8)].append(st["mask"])
        r.state = None


# ---------------------------------------------------------------------------
# Camera-stream workload
# ---------------------------------------------------------------------------
@dataclass
class StreamSpec:
    stream: int
    height: int
    width: int
    arrivals: np.ndarray
    pool_images: list = field(default_factory=list)   # pinned host frames, cycled
    pool_masks: list = field(default_factory=list)


def camera_streams(duration_s: float = 60.0, rate_hz: float = 30.0, seed: int = 1004, pool: int = 8,
                   mix=None, device=None, pinned: bool = True):
    """16 streams (8 x 1080p, 6 x 768x576, 2 x 2160p) with Poisson arrivals;
    each stream cycles a pool of rendered frames with moving-rectangle masks."""
    import torch
    from . import synth
    mix = mix if mix is not None else synth.STREAM_MIX
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    sid = 0
    dev = device if device is not None else ("cuda:0" if torch.cuda.is_available() else "cpu")
    for (h, w, count) in mix:
        for _ in range(count):
            arr = synth.poisson_arrivals(rng, rate_hz, duration_s)
            ramps = [synth.draw_ramp(rng) for _ in range(3)]
            mover = synth.MovingRects(rng, h, w)
            imgs, masks = [], []
            base = synth.render_image_torch(ramps, h, w, dev)
            for k in range(pool):
                img = torch.roll(base, shifts=3 * k, dims=1).cpu()
                mk = synth.paint_mask_torch(mover.step(), h, w, dev).cpu()
                if pinned and torch.cuda.is_available():
                    img, mk = img.pin_memory(), mk.pin_memory()
                imgs.append(img)
                masks.append(mk)
            out.append(StreamSpec(sid, h, w, arr, imgs, masks))
            sid += 1
    return out


class StreamCounters:
    """Philox frame counters of camera streams.  Frame k of stream s is
    drawn with counter words 2-3 = (s << 40) | k under one key (the seed), so
    no two frames of any streams share a counter: two frames released with
    the same noise would give away the exact difference of their true cell
    means.  The state (seed and each stream's next k) can be saved and
    restored, so a resumed stream continues its counter instead of reusing
    one."""

    STREAM_SHIFT = 40

    def __init__(self, seed: int, next_index: Optional[Dict[int, int]] = None):
        self.seed = int(seed)
        self.next_index: Dict[int, int] = {int(k): int(v) for k, v in (next_index or {}).items()}

    def frame_index(self, stream: int, k: int) -> int:
        if not (0 <= stream < (1 << (64 - self.STREAM_SHIFT)) and 0 <= k < (1 << self.STREAM_SHIFT)):
            raise ValueError("stream %d / frame %d outside the counter range" % (stream, k))
        return (int(stream) << self.STREAM_SHIFT) | int(k)

    def take(self, stream: int) -> int:
        """The next frame of `stream`: its counter, advancing the stream."""
        k = self.next_index.get(int(stream), 0)
        self.next_index[int(stream)] = k + 1
        return self.frame_index(stream, k)

    def state(self) -> dict:
        return {"seed": self.seed, "next": {str(s): n for s, n in sorted(self.next_index.items())}}

    @classmethod
    def from_state(cls, state: dict) -> "StreamCounters":
        return cls(state["seed"], {int(s): int(n) for s, n in state["next"].items()})

    def save(self, path: str):
        import json
        import os
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(self.state(), f)
        os.replace(tmp, path)

    @classmethod
    def load(cls, path: str) -> "StreamCounters":
        import json
        with open(path) as f:
            return cls.from_state(json.load(f))


def serve_streams(streams, scheduler: Scheduler, params: dict, duration_s: Optional[float] = None,
                  seed: int = 4, keep_results: bool = False, clock=time.perf_counter,
                  counters: Optional[StreamCounters] = None, freeze_gc: bool = True):
    """Replay the streams' arrivals in real time through the scheduler.
    params: b, sb, m, eps_bg, eps_fg, tau.  Each frame's Philox counter comes
    from `counters` (a fresh StreamCounters(seed) by default), which the
    caller can save to resume the streams later.  Returns the finished
    requests.

    freeze_gc: a full (generation 2) collection walks every tracked object of
    the process — several hundred thousand once torch is imported — and
    stalls the loop for tens of milliseconds, which every frame queued behind
    it sees as latency.  The loop therefore moves the objects that exist when
    it starts to the collector's permanent generation (gc.freeze) and
    releases them when it ends; objects made by the loop are collected as
    usual.  A caller that has frozen objects itself keeps control: the loop
    then leaves the collector as it finds it."""
    counters = counters if counters is not None else StreamCounters(seed)
    own_freeze = freeze_gc and gc.get_freeze_count() == 0
    # without keep_results a result is dropped as soon as its frame finishes,
    # so a long replay holds no stores on the host
    hook = scheduler.on_done
    if not keep_results:
        def drop(r, prev=hook):
            if prev is not None:
                prev(r)
            r.result = None
        scheduler.on_done = drop
    if own_freeze:
        gc.collect()
        gc.freeze()
    try:
        return _serve_loop(streams, scheduler, params, duration_s, clock, counters)
    finally:
        scheduler.on_done = hook
        if own_freeze:
            gc.unfreeze()


def _serve_loop(streams, scheduler, params, duration_s, clock, counters):
    events = []
    for s in streams:
        for k, t in enumerate(s.arrivals):
            if duration_s is None or t < duration_s:
                events.append((float(t), s.stream, k))
    events.sort()
    by_id = {s.stream: s for s in streams}
    t0 = clock()
    i = rid = 0
    while i < len(events) or not scheduler.idle():
        now = clock() - t0
        while i < len(events) and events[i][0] <= now:
            t, sid, k = events[i]
            s = by_id[sid]
            r = Request(rid, sid, counters.take(sid), s.height, s.width, 3, params["b"], params["sb"], params["m"],
                        params["eps_bg"], params["eps_fg"], params["tau"], counters.seed,
                        image=s.pool_images[k % len(s.pool_images)], mask=s.pool_masks[k % len(s.pool_masks)],
                        arrival=t0 + t)
            scheduler.offer(r)
            rid += 1
            i += 1
        if scheduler.pump() == 0:
            nxt = events[i][0] - (clock() - t0) if i < len(events) else 0.0
            time.sleep(min(max(nxt, 0.0), 2e-4))
    return scheduler.finished
