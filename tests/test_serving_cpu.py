"""Serving scheduler on the CPU: admission by memory, continuous batching,
failure isolation and ordering, with the oracle as a fake backend."""
import math

import numpy as np
import pytest

import oracle
from paper_2511_04261_amd import synth
from paper_2511_04261_amd.serving import MemoryLedger, Request, Scheduler, StreamCounters, latency_stats


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3
        return self.t


class CpuBackend:
    """Runs the oracle per request; a batch completes after `polls` polls."""

    def __init__(self, polls=2, explode_on=None):
        self.polls = polls
        self.explode_on = explode_on or set()
        self.launches = []

    @staticmethod
    def params(r):
        return oracle.Params(r.height, r.width, r.channels, b=r.b, sb=r.sb, m=r.m, eps_simple=r.eps_bg,
                             eps_complex=r.eps_fg, tau=r.tau, seed=r.seed, frame_index=r.frame_index)

    def validate(self, r):
        try:
            self.params(r).geometry()
        except ValueError as e:
            return str(e)
        if r.image is None or r.image.shape[:2] != (r.height, r.width):
            return "image does not match the request geometry"
        return None

    def request_bytes(self, r):
        return r.height * r.width * (r.channels + 1)

    def admit(self, r):
        r.state = "admitted"

    def launch(self, batch):
        if any(r.rid in self.explode_on for r in batch):
            raise RuntimeError("backend failure on request %s" % [r.rid for r in batch if r.rid in self.explode_on])
        self.launches.append([r.rid for r in batch])
        res = [oracle.forward(r.image, r.mask, self.params(r)) for r in batch]
        return {"left": self.polls, "res": res}

    def poll(self, h):
        h["left"] -= 1
        return h["left"] <= 0

    def collect(self, h):
        return h["res"]

    def release(self, r):
        r.state = None


def make_requests(n, streams=3, H=24, W=40, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    counters = StreamCounters(9)
    for i in range(n):
        s = i % streams
        img = synth.gradient_image(rng, H, W, 3)
        mk = synth.rect_mask(rng, H, W, n_rects=2, rect_frac=0.05, cover=(0.05, 0.3))
        reqs.append(Request(i, s, counters.take(s), H, W, 3, 8, 4, 4, 1.0, 0.5, 1, counters.seed, image=img, mask=mk,
                            arrival=0.0))
    return reqs


def run(sched, reqs, per_pump=1):
    i = 0
    while i < len(reqs) or not sched.idle():
        for _ in range(per_pump):
            if i < len(reqs):
                sched.offer(reqs[i])
                i += 1
        sched.pump()


def test_every_request_gets_its_own_result_in_stream_order():
    be = CpuBackend()
    sch = Scheduler(be, MemoryLedger(10**9), max_batch=8, max_inflight=2, clock=FakeClock())
    reqs = make_requests(30)
    run(sch, reqs, per_pump=3)
    assert len(sch.finished) == 30 and not sch.rejected
    for r in reqs:
        alone = oracle.forward(r.image, r.mask, CpuBackend.params(r))
        assert np.array_equal(r.result["bg"], alone["bg"]) and np.array_equal(r.result["fg"], alone["fg"])
    for s in range(3):
        order = [r.frame_index for r in sch.finished if r.stream == s]
        assert order == sorted(order)


def test_continuous_batching_joins_arrivals_during_flight():
    be = CpuBackend(polls=4)
    sch = Scheduler(be, MemoryLedger(10**9), max_batch=64, max_inflight=1, clock=FakeClock())
    reqs = make_requests(24)
    run(sch, reqs, per_pump=1)
    # first batch launches at once with one request; later ones collect what
    # arrived while the previous batch was in flight
    assert sch.batch_sizes[0] == 1
    assert max(sch.batch_sizes) >= 3
    assert sum(sch.batch_sizes) == 24


def test_memory_cap_queues_and_bounds_peak():
    be = CpuBackend(polls=3)
    need = 24 * 40 * 4
    led = MemoryLedger(3 * need)
    sch = Scheduler(be, led, max_batch=64, max_inflight=4, clock=FakeClock())
    reqs = make_requests(20)
    run(sch, reqs, per_pump=5)
    assert len(sch.finished) == 20
    assert led.peak <= 3 * need and led.used == 0
    assert max(sch.batch_sizes) <= 3


def test_request_above_cap_and_malformed_fail_alone():
    be = CpuBackend()
    sch = Scheduler(be, MemoryLedger(24 * 40 * 4 * 4), clock=FakeClock())
    reqs = make_requests(6)
    big = Request(100, 0, 99, 400, 400, 3, 8, 4, 4, 1.0, 0.5, 1, 9, image=np.zeros((400, 400, 3), np.uint8))
    bad = Request(101, 1, 98, 24, 40, 3, 8, 3, 4, 1.0, 0.5, 1, 9, image=np.zeros((24, 40, 3), np.uint8))
    mism = Request(102, 2, 97, 24, 40, 3, 8, 4, 4, 1.0, 0.5, 1, 9, image=np.zeros((10, 10, 3), np.uint8))
    run(sch, reqs[:3] + [big, bad, mism] + reqs[3:], per_pump=2)
    assert {r.rid for r in sch.rejected} == {100, 101, 102}
    assert "cap" in big.error and mism.error
    assert len(sch.finished) == 6 and all(r.error is None for r in sch.finished)


def test_backend_failure_in_a_batch_is_isolated():
    be = CpuBackend(explode_on={4})
    sch = Scheduler(be, MemoryLedger(10**9), max_batch=8, max_inflight=1, clock=FakeClock())
    reqs = make_requests(10)
    for r in reqs:
        sch.offer(r)
    sch.drain()
    assert [r.rid for r in sch.rejected] == [4]
    assert "backend failure" in reqs[4].error
    assert len(sch.finished) == 9
    assert sch.ledger.used == 0


def test_queue_limit_rejects():
    be = CpuBackend()
    sch = Scheduler(be, MemoryLedger(1), max_queue=2, clock=FakeClock())  # nothing fits... except rejection
    reqs = make_requests(3)
    for r in reqs:
        sch.offer(r)
    assert all("cap" in r.error for r in sch.rejected)


def test_latency_stats():
    rs = []
    for i, lat in enumerate([0.001 * k for k in range(1, 101)]):
        r = Request(i, 0, i, 1, 1, 1, 1, 1, 1, 1.0, 1.0, 1, 0, arrival=0.0)
        r.done = lat
        rs.append(r)
    st = latency_stats(rs)
    assert st["n"] == 100 and abs(st["p50_ms"] - 50.5) < 1e-9 and abs(st["p99_ms"] - 99.01) < 1e-9


def test_latency_split():
    """The split of each latency: memory wait, launch wait, in flight, and
    the backend's own timing keys, each with mean and p99."""
    rs = []
    for i in range(10):
        r = Request(i, 0, i, 1, 1, 1, 1, 1, 1, 1.0, 1.0, 1, 0, arrival=0.0)
        r.admitted, r.launched, r.done = 0.001 * i, 0.002 * i, 0.004 * i
        r.timing = dict(gpu=0.5, d2h=float(i))
        rs.append(r)
    st = latency_stats(rs)
    assert abs(st["split_queue_mean_ms"] - 4.5) < 1e-9
    assert abs(st["split_wait_launch_mean_ms"] - 4.5) < 1e-9
    assert abs(st["split_in_flight_mean_ms"] - 9.0) < 1e-9
    assert st["split_gpu_mean_ms"] == 0.5 and st["split_gpu_p99_ms"] == 0.5
    assert abs(st["split_d2h_p99_ms"] - np.percentile(np.arange(10.0), 99)) < 1e-9


def test_stream_counters_unique_and_resumable(tmp_path):
    """Every (stream, frame) gets its own Philox counter; a saved and
    restored counter state continues each stream where it stopped."""
    a = StreamCounters(7)
    seen = [a.take(s) for _ in range(50) for s in (0, 1, 5)]
    path = str(tmp_path / "counters.json")
    a.save(path)
    b = StreamCounters.load(path)
    assert b.state() == a.state() and b.seed == 7
    more = [b.take(s) for _ in range(50) for s in (0, 1, 5, 6)]
    whole = StreamCounters(7)
    ref = [whole.take(s) for _ in range(50) for s in (0, 1, 5)] + [whole.take(s) for _ in range(50) for s in (0, 1, 5, 6)]
    assert seen + more == ref
    assert len(set(seen + more)) == len(seen) + len(more)
    assert a.frame_index(0, 3) == 3 and a.frame_index(2, 3) == (2 << 40) | 3
    with pytest.raises(ValueError):
        a.frame_index(0, 1 << 40)
    with pytest.raises(ValueError):
        a.frame_index(1 << 24, 0)


def test_identical_frames_of_two_streams_get_independent_noise():
    """The same image sent as frame 0 of two streams: each release has its
    own noise (equal noise would give away the difference of true means)."""
    rng = np.random.Generator(np.random.PCG64(3))
    img = synth.gradient_image(rng, 32, 48, 3)
    counters = StreamCounters(11)
    outs = []
    for stream in (0, 1):
        p = oracle.Params(32, 48, 3, b=8, sb=8, m=4, eps_simple=1.0, eps_complex=1.0, seed=counters.seed,
                          frame_index=counters.take(stream))
        outs.append(oracle.forward(img, None, p)["bg"])
    assert outs[0].shape == outs[1].shape
    assert (outs[0] == outs[1]).mean() < 0.01


def _tiny_streams(rng, n_streams=2, frames=3, H=24, W=40):
    from paper_2511_04261_amd.serving import StreamSpec
    out = []
    for s in range(n_streams):
        imgs = [synth.gradient_image(rng, H, W, 3) for _ in range(2)]
        masks = [synth.rect_mask(rng, H, W, n_rects=2, rect_frac=0.05, cover=(0.05, 0.3)) for _ in range(2)]
        out.append(StreamSpec(s, H, W, np.arange(frames) * 2e-3, imgs, masks))
    return out


def test_serve_streams_freezes_the_collector_only_for_its_loop():
    import gc

    from paper_2511_04261_amd.serving import serve_streams
    rng = np.random.Generator(np.random.PCG64(5))
    streams = _tiny_streams(rng)
    params = dict(b=8, sb=4, m=4, eps_bg=1.0, eps_fg=0.5, tau=1)
    seen = []

    class Probe(CpuBackend):
        def launch(self, batch):
            seen.append(gc.get_freeze_count())
            return super().launch(batch)

    assert gc.get_freeze_count() == 0
    done = serve_streams(streams, Scheduler(Probe(), MemoryLedger(1 << 20), clock=FakeClock()), params,
                         keep_results=True, clock=FakeClock())
    assert gc.get_freeze_count() == 0 and seen and min(seen) > 0
    assert len(done) == 6 and all(r.error is None for r in done)
    for r in done:
        s = streams[r.stream]
        k = r.frame_index & ((1 << StreamCounters.STREAM_SHIFT) - 1)
        want = oracle.forward(s.pool_images[k % 2], s.pool_masks[k % 2], CpuBackend.params(r))
        np.testing.assert_array_equal(r.result["bg"], want["bg"])
    # a caller that froze objects itself keeps them frozen
    gc.freeze()
    try:
        before = gc.get_freeze_count()
        serve_streams(_tiny_streams(rng), Scheduler(CpuBackend(), MemoryLedger(1 << 20), clock=FakeClock()), params,
                      clock=FakeClock())
        assert gc.get_freeze_count() == before
    finally:
        gc.unfreeze()
    # and the switch turns it off
    seen.clear()
    serve_streams(_tiny_streams(rng), Scheduler(Probe(), MemoryLedger(1 << 20), clock=FakeClock()), params,
                  clock=FakeClock(), freeze_gc=False)
    assert seen and max(seen) == 0


def test_on_done_hook_sees_results_and_replay_drops_them():
    from paper_2511_04261_amd.serving import serve_streams
    rng = np.random.Generator(np.random.PCG64(6))
    params = dict(b=8, sb=4, m=4, eps_bg=1.0, eps_fg=0.5, tau=1)
    seen = []
    sch = Scheduler(CpuBackend(), MemoryLedger(1 << 20), clock=FakeClock(),
                    on_done=lambda r: seen.append((r.rid, r.result is not None)))
    done = serve_streams(_tiny_streams(rng), sch, params, clock=FakeClock())
    assert len(seen) == len(done) == 6 and all(has for _, has in seen)
    assert all(r.result is None and r.done is not None for r in done)
    assert sch.on_done is not None and sch.on_done.__name__ == "<lambda>"   # the caller's hook is restored
    kept = serve_streams(_tiny_streams(rng), Scheduler(CpuBackend(), MemoryLedger(1 << 20), clock=FakeClock()), params,
                         keep_results=True, clock=FakeClock())
    assert all(r.result is not None for r in kept)


def test_stream_that_stops_sending_does_not_hold_back_the_others():
    """One stream sends two frames and goes silent; the other streams keep
    arriving.  Every frame sent is served with its own result, in per-stream
    order, nothing waits for the silent stream, and its saved counter state
    resumes it after the two frames it did send."""
    from paper_2511_04261_amd.serving import StreamSpec, serve_streams
    rng = np.random.Generator(np.random.PCG64(8))
    streams = _tiny_streams(rng, n_streams=3, frames=6)
    s = streams[1]
    streams[1] = StreamSpec(s.stream, s.height, s.width, s.arrivals[:2], s.pool_images, s.pool_masks)
    params = dict(b=8, sb=4, m=4, eps_bg=1.0, eps_fg=0.5, tau=1)
    counters = StreamCounters(12)
    done = serve_streams(streams, Scheduler(CpuBackend(), MemoryLedger(1 << 20), clock=FakeClock()), params,
                         keep_results=True, clock=FakeClock(), counters=counters)
    assert len(done) == 6 + 2 + 6 and all(r.error is None and r.result is not None for r in done)
    for sid, n in ((0, 6), (1, 2), (2, 6)):
        mine = [r for r in done if r.stream == sid]
        assert len(mine) == n
        seq = [r.frame_index & ((1 << StreamCounters.STREAM_SHIFT) - 1) for r in mine]
        assert seq == sorted(seq) == list(range(n))
    # the silent stream resumes after the frames it sent
    restored = StreamCounters.from_state(counters.state())
    assert restored.take(1) & ((1 << StreamCounters.STREAM_SHIFT) - 1) == 2
    assert restored.take(0) & ((1 << StreamCounters.STREAM_SHIFT) - 1) == 6
