"""GPU tests of batching, graphs, tuning, the autograd layer and serving,
each against the oracle or against the plain eager path (bitwise)."""
import math
import sys

import numpy as np
import pytest

import oracle
from tests.helpers import compare_frame, oracle_params, chw_to_hwc, run_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

dp = pytest.importorskip("paper_2511_04261_amd")
from paper_2511_04261_amd import synth  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _store_equal(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("flags", "bg", "fg")) and tuple(a["counts"]) == tuple(b["counts"])


def test_graph_replays_match_eager(dev):
    """Replay several times with eager work and new frame contents between
    replays; every replay equals the eager plan + forward on the same data."""
    say("case: graph replay")
    specs = synth.region_batch(6, height=270, width=480)
    frames = [dp.FrameParams.from_spec(s) for s in specs]
    plan = dp.Plan(frames, device=dev, persistent=True)
    imgs = [s.image_torch(dev) for s in specs]
    masks = [s.mask_torch(dev) for s in specs]
    outs = [torch.empty_like(t) for t in imgs]
    g = plan.graph(masks, imgs, outs)
    ref = dp.Plan(frames, device=dev, persistent=False)
    rng = np.random.Generator(np.random.PCG64(77))
    for rep in range(4):
        if rep:
            for t, m in zip(imgs, masks):     # new contents, same buffers (eager torch work in between)
                t.copy_(torch.randint(0, 256, t.shape, dtype=torch.uint8, device=dev))
                m.copy_(synth.paint_mask_torch(synth.draw_rects(rng, 270, 480), 270, 480, dev))
        g.launch()
        torch.cuda.synchronize()
        got = plan.store_host()
        got_out = [o.cpu().numpy() for o in outs]
        ro = [torch.empty_like(t) for t in imgs]
        ref.plan(masks)
        ref.forward(imgs, out=ro)
        torch.cuda.synchronize()
        want = ref.store_host()
        for i in range(len(frames)):
            assert _store_equal(got[i], want[i]), (rep, i)
            assert np.array_equal(got_out[i], ro[i].cpu().numpy()), (rep, i)
    g.close()


def test_autotuned_shapes_are_bitwise_identical(dev, tmp_path):
    say("case: autotune")
    from paper_2511_04261_amd.autotune import Autotuner
    specs = synth.region_batch(3, height=300, width=500)
    frames = [dp.FrameParams.from_spec(s) for s in specs]
    tuner = Autotuner(dev, cache_path=str(tmp_path / "cache.json"), min_pixels=2e6, reps=2)
    tuned, launch = tuner.tune_batch(frames)
    assert (tmp_path / "cache.json").exists()
    imgs = [s.image_torch(dev) for s in specs]
    masks = [s.mask_torch(dev) for s in specs]
    a = dp.Plan(frames, device=dev)
    b = dp.Plan(tuned, device=dev, **launch)
    oa = [torch.empty_like(t) for t in imgs]
    ob = [torch.empty_like(t) for t in imgs]
    for p, o in ((a, oa), (b, ob)):
        p.plan(masks)
        p.forward(imgs, out=o)
    torch.cuda.synchronize()
    for x, y in zip(a.store_host(), b.store_host()):
        assert _store_equal(x, y)
    for x, y in zip(oa, ob):
        assert torch.equal(x, y)


def test_whole_batch_autotune_is_bitwise_identical(dev):
    """tune_whole_batch times candidate tile widths and workgroup sizes on the
    batch itself; whatever it picks gives the same store and output bit for
    bit as the library's defaults."""
    say("case: whole-batch autotune")
    from paper_2511_04261_amd.autotune import Autotuner
    specs = synth.region_batch(2, height=300, width=500) + synth.region_batch(2, height=200, width=700, b=16, sb=4)
    frames = [dp.FrameParams.from_spec(s) for s in specs]
    imgs = [s.image_torch(dev) for s in specs]
    masks = [s.mask_torch(dev) for s in specs]
    tuner = Autotuner(dev, cache_path=None, reps=2, threads=(0, 128), launch_modes=(0, 1))
    tuned, info = tuner.tune_whole_batch(frames, imgs, masks, tile_bytes=(0, 1024, 4096))
    assert len(info["tried"]) == 3 * 2 * 2 and abs(info["ms"] - min(t["ms"] for t in info["tried"])) < 1e-4
    a = dp.Plan(frames, device=dev)
    b = dp.Plan(tuned, device=dev, threads=info["threads"], persistent=info["persistent"])
    oa = [torch.empty_like(t) for t in imgs]
    ob = [torch.empty_like(t) for t in imgs]
    for p, o in ((a, oa), (b, ob)):
        p.plan(masks)
        p.forward(imgs, out=o)
    torch.cuda.synchronize()
    for x, y in zip(a.store_host(), b.store_host()):
        assert _store_equal(x, y)
    for x, y in zip(oa, ob):
        assert torch.equal(x, y)


def test_uneven_batch_full_size_sampled(dev):
    """256 frames of 768x576 .. 6000x4000, per-frame grids and budgets, one
    graph-replayed launch in the benchmark's configuration (one workgroup per
    tile); one frame of every (resolution, b, s_b) class present checked in
    full against the oracle (the classes decide the tile shapes and which
    launch group, 128 or 256 lanes, a frame runs in), all frames for store
    invariants."""
    say("case: uneven 256-frame batch")
    specs = synth.uneven_batch(256)
    frames = [dp.FrameParams.from_spec(s) for s in specs]
    plan = dp.Plan(frames, device=dev)
    imgs = [s.image_torch(dev) for s in specs]
    masks = [s.mask_torch(dev) for s in specs]
    outs = [torch.empty_like(t) for t in imgs]
    g = plan.graph(masks, imgs, outs)
    g.launch()
    g.launch()
    torch.cuda.synchronize()
    store = plan.store_host()
    ob = of = 0
    for i, (fp, fi, st) in enumerate(zip(frames, plan.info, store)):
        nb, nf = st["counts"]
        assert nb + nf == fi.grid_rows * fi.grid_cols and nf == int(st["flags"].sum())
        assert st["offsets"] == (ob, of)
        ob += nb * 3
        of += nf * fi.n * fi.n * 3
    seen = set()
    for i, s in enumerate(specs):
        if (s.height, s.width, s.b, s.sb) in seen:
            continue
        seen.add((s.height, s.width, s.b, s.sb))
        say("  oracle on frame", i, s.height, s.width, s.b, s.sb)
        img = imgs[i].cpu().numpy()
        want = oracle.forward(img, s.mask, oracle_params(frames[i]))
        compare_frame(store[i], want, outs[i].cpu().numpy(), "frame %d" % i)
        s.drop_host()
    assert len(seen) == 16      # every class of 4 resolutions x b in {16, 32} x s_b in {4, 8} occurs
    g.close()


def test_autograd_layer_matches_oracle(dev):
    """DPPixFn through the autograd engine: y and dL/dx against the oracle for
    3x64x64 crops (no padding) and 3x61x57 (mirror multiplicity)."""
    for (H, W) in [(64, 64), (61, 57)]:
        say("case: autograd", H, W)
        r = np.random.Generator(np.random.PCG64(H))
        x = synth.uniform_f32(r, (2, 3, H, W))
        masks = [synth.rect_mask(r, H, W, n_rects=2, rect_frac=0.1, cover=(0.05, 0.5)) for _ in range(2)]
        w = r.standard_normal((2, 3, H, W)).astype(np.float32)
        layer = dp.DPPixLayer(b=16, sb=8, m=8, eps_bg=1.0, eps_fg=0.5, tau=1, seed=3)
        tx = torch.from_numpy(x).to(dev).requires_grad_(True)
        tm = [torch.from_numpy(m).to(dev) for m in masks]
        y = layer(tx, tm)
        (y * torch.from_numpy(w).to(dev)).sum().backward()
        for i in range(2):
            fp = dp.FrameParams(H, W, 3, dp.F32_CHW, b=16, sb=8, m=8, eps_bg=1.0, eps_fg=0.5, tau=1, seed=3,
                                frame_index=i)
            p = oracle_params(fp)
            want = oracle.forward(chw_to_hwc(x[i]), masks[i], p)
            assert np.abs(chw_to_hwc(y[i].detach().cpu().numpy()) - want["recon_f32"]).max() <= 1e-3
            gw = oracle.backward(chw_to_hwc(x[i]).astype(np.float64), masks[i], chw_to_hwc(w[i]).astype(np.float64), p)
            got = chw_to_hwc(tx.grad[i].cpu().numpy())
            assert np.abs(got - gw).max() <= 1e-5


def test_autograd_full_batch_and_fd(dev):
    """32x3x512x512 fp32, b_fg=8 / b_bg=16, m=8, eps 0.5 / 1.0: forward and
    backward on the GPU; two images against the oracle gradient; central
    differences of the GPU forward (piecewise linear, h=0.5) at sampled pixels."""
    say("case: autograd 32x3x512x512")
    x, masks, w = synth.autograd_batch()
    layer = dp.DPPixLayer(b=16, sb=8, m=8, eps_bg=1.0, eps_fg=0.5, tau=1, seed=5)
    tx = torch.from_numpy(x).to(dev).requires_grad_(True)
    tm = [torch.from_numpy(m).to(dev) for m in masks]
    tw = torch.from_numpy(w).to(dev)
    y = layer(tx, tm)
    (y * tw).sum().backward()
    torch.cuda.synchronize()
    for i in (0, 31):
        fp = dp.FrameParams(512, 512, 3, dp.F32_CHW, b=16, sb=8, m=8, eps_bg=1.0, eps_fg=0.5, tau=1, seed=5,
                            frame_index=i)
        gw = oracle.backward(chw_to_hwc(x[i]).astype(np.float64), masks[i], chw_to_hwc(w[i]).astype(np.float64),
                             oracle_params(fp))
        assert np.abs(chw_to_hwc(tx.grad[i].cpu().numpy()) - gw).max() <= 1e-5
    r = np.random.Generator(np.random.PCG64(8))
    h = 0.5
    with torch.no_grad():
        for _ in range(6):
            i, c, yy, xx = int(r.integers(0, 32)), int(r.integers(0, 3)), int(r.integers(0, 512)), int(r.integers(0, 512))
            xp = tx.detach().clone()
            xp[i, c, yy, xx] += h
            xm = tx.detach().clone()
            xm[i, c, yy, xx] -= h
            fd = ((layer(xp, tm) * tw).sum(dtype=torch.float64) - (layer(xm, tm) * tw).sum(dtype=torch.float64)) / (2 * h)
            assert abs(fd.item() - tx.grad[i, c, yy, xx].item()) <= 2e-3 + 1e-3 * abs(tx.grad[i, c, yy, xx].item())


def test_serving_alone_equals_mix(dev):
    """Frames served from 16 mixed-resolution streams (continuous batching,
    memory admission) give the same store bit for bit as each frame alone,
    and served frames of every resolution equal the oracle's release of the
    same frame with the same counter."""
    say("case: serving alone vs mix")
    from paper_2511_04261_amd.serving import GpuBackend, MemoryLedger, Scheduler, camera_streams, serve_streams
    streams = camera_streams(duration_s=1.5, pool=3, device=dev)
    params = dict(b=32, sb=8, m=16, eps_bg=1.0, eps_fg=0.3, tau=1)
    be = GpuBackend(dev)
    sch = Scheduler(be, MemoryLedger(4 << 30), max_batch=64, max_inflight=2)
    done = serve_streams(streams, sch, params, keep_results=True)
    assert not sch.rejected and len(done) > 100
    assert max(sch.batch_sizes) > 1
    for q in done:
        # every served frame carries its privacy ledger (Thm. 1: max of the
        # region budgets per channel value, C times that per whole pixel)
        led = q.result["ledger"]
        assert (led["eps_bg"], led["eps_fg"], led["eps_frame"], led["eps_pixel"], led["m"]) == (1.0, 0.3, 1.0, 3.0, 16)
        assert led["frame_index"] == q.frame_index
    r = np.random.Generator(np.random.PCG64(5))
    for k in r.choice(len(done), size=12, replace=False):
        q = done[int(k)]
        fp = be.frame_params(q)
        plan = dp.Plan([fp], device=dev)
        plan.plan([q.mask.to(dev)])
        plan.forward([q.image.to(dev)])
        torch.cuda.synchronize()
        alone = plan.store_host()[0]
        assert _store_equal(q.result, alone), (q.rid, q.stream, q.frame_index)
    by_res = {}
    for q in done:
        by_res.setdefault((q.height, q.width), []).append(q)
    assert len(by_res) == 3
    for (H, W), qs in sorted(by_res.items()):
        for q in (qs[0], qs[len(qs) // 2], qs[-1]):
            say("  oracle on served frame", q.rid, H, W, q.frame_index)
            want = oracle.forward(q.image.numpy(), q.mask.numpy(), oracle_params(be.frame_params(q)))
            compare_frame(q.result, want, None, "served frame %d" % q.rid)


@pytest.mark.parametrize("H,W,C,b,sb,T,pad", [(75, 97, 3, 16, 4, 60, 0), (270, 480, 3, 32, 8, 40, 0),
                                              (33, 40, 1, 8, 2, 30, 1), (1080, 1920, 3, 32, 8, 48, 0),
                                              (5, 3, 3, 8, 4, 10, 0), (45, 70, 3, 16, 4, 40, 2)])
def test_edge_mask_label_matches_oracle(dev, H, W, C, b, sb, T, pad):
    """Sobel complexity labels bit-exact against the oracle, then the whole
    path driven by them against the oracle driven by the oracle's labels."""
    say("case: edge mask", H, W, C, b, sb, T, pad)
    r = np.random.Generator(np.random.PCG64(H * W))
    img = synth.gradient_image(r, H, W, C)
    img[H // 4: H // 2, W // 5: W // 2] = 250          # a bright block: strong edges
    fp = dp.FrameParams(H, W, C, dp.U8_HWC, b=b, sb=sb, m=16, eps_bg=1.0, eps_fg=0.3, tau=4, pad_mode=pad, seed=6)
    plan = dp.Plan([fp], device=dev)
    ti = torch.from_numpy(img).to(dev)
    masks = plan.edge_masks([ti], T)
    out = torch.empty_like(ti)
    plan.plan(masks)
    plan.forward([ti], out=[out])
    torch.cuda.synchronize()
    want_mask = oracle.edge_mask(img, T, pad)
    assert np.array_equal(masks[0].cpu().numpy(), want_mask)
    want = oracle.forward(img, want_mask, oracle_params(fp))
    compare_frame(plan.store_host()[0], want, out.cpu().numpy(), "edge-labelled")



@pytest.mark.parametrize("case", ["1100 tiny frames, mixed C and n", "1100 tiny frames, one C and n",
                                  "300 frames, 38400 tiles"])
def test_scan_many_frames_store_offsets(dev, case):
    """Both scans of the complex counts: the per-frame workgroups with a
    frame-level pass (mixed C or n, or more than 16384 tiles; here with more
    frames than one workgroup's lanes, so that pass loops) and the one where
    each workgroup adds up the counts of all earlier frames itself (one C and
    n, few tiles).  Store offsets are the running sums of every frame's counts
    in batch order, and sampled frames (first, last and random ones) equal the
    oracle."""
    say("case: scan", case)
    r = np.random.Generator(np.random.PCG64(len(case)))
    frames, imgs, masks = [], [], []
    if case.startswith("1100"):
        mixed = "mixed" in case
        for i in range(1100):
            H, W = int(r.integers(1, 41)), int(r.integers(1, 71))
            C = int(r.choice([1, 3])) if mixed else 3
            b = int(r.choice([4, 8]))
            sb = int(r.choice([s for s in (1, 2, 4, 8) if b % s == 0])) if mixed else b // 2
            frames.append(dp.FrameParams(H, W, C, dp.U8_HWC, b=b, sb=sb, m=4, eps_bg=1.0, eps_fg=0.5, tau=1,
                                         pad_mode=int(r.integers(0, 3)), seed=9, frame_index=i))
            imgs.append(r.integers(0, 256, (H, W, C), dtype=np.uint8))
            masks.append((r.random((H, W)) < 0.3).astype(np.uint8))
    else:
        for i in range(300):
            frames.append(dp.FrameParams(256, 64, 1, dp.U8_HWC, b=2, sb=1, m=2, eps_bg=1.0, eps_fg=0.5, tau=2,
                                         seed=10, frame_index=i))
            imgs.append(r.integers(0, 256, (256, 64, 1), dtype=np.uint8))
            masks.append((r.random((256, 64)) < 0.4).astype(np.uint8))
    res = run_gpu(frames, imgs, masks, dev, reconstruct=False)
    ob = of = 0
    for fp, fi, st in zip(frames, res["info"], res["store"]):
        nb, nf = st["counts"]
        assert nb + nf == fi.grid_rows * fi.grid_cols and nf == int(st["flags"].sum())
        assert st["offsets"] == (ob, of)
        ob += nb * fp.channels
        of += nf * fi.n * fi.n * fp.channels
    picks = {0, len(frames) - 1} | {int(k) for k in r.choice(len(frames), size=8, replace=False)}
    for i in sorted(picks):
        want = oracle.forward(imgs[i], masks[i], oracle_params(frames[i]))
        compare_frame(res["store"][i], want, res["fused"][i], "frame %d" % i)


def test_two_plans_on_two_streams_overlap(dev):
    """Two plans issued alternately on two streams, so that their launches
    can overlap on the device: each plan's workspace (tickets, counters,
    tables) is its own, and every round's stores and reconstructions equal
    those of each plan run alone."""
    say("case: two plans, two streams")
    runs = []
    for specs in (synth.region_batch(6, height=270, width=480, seed=3), synth.uneven_batch(12, seed=8)):
        plan = dp.Plan([dp.FrameParams.from_spec(s) for s in specs], device=dev)
        imgs = [s.image_torch(dev) for s in specs]
        masks = [s.mask_torch(dev) for s in specs]
        runs.append((plan, imgs, masks, [torch.empty_like(t) for t in imgs]))
    alone = []
    for plan, imgs, masks, outs in runs:
        plan.plan(masks)
        plan.forward(imgs, out=outs)
        torch.cuda.synchronize()
        alone.append((plan.store_host(), [o.cpu().numpy() for o in outs]))
    streams = [torch.cuda.Stream(dev), torch.cuda.Stream(dev)]
    for rnd in range(4):
        for _, _, _, outs in runs:
            for o in outs:
                o.zero_()
        torch.cuda.synchronize()
        for (plan, imgs, masks, outs), st in zip(runs, streams):
            plan.plan(masks, stream=st)
        for (plan, imgs, masks, outs), st in zip(runs, streams):
            plan.forward(imgs, out=outs, stream=st)
        torch.cuda.synchronize()
        for (plan, _, _, outs), (store, recon) in zip(runs, alone):
            got = plan.store_host()
            assert all(_store_equal(a, b) for a, b in zip(got, store)), rnd
            assert all(np.array_equal(o.cpu().numpy(), w) for o, w in zip(outs, recon)), rnd
    for plan, *_ in runs:
        plan.close()
