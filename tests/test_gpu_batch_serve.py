"""Batched and served forms: every frame's result equals the same frame
reconstructed alone, bit for bit (the per-pixel computation does not depend on
which frames share a launch), across graph replays and under budget pressure."""
import sys
import time

import numpy as np
import pytest

import oracle
from synth import configs
from synth.scene import EdgeScene
from parity_utils import compare

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make_frames(n, seed0=4100):
    """Small mixed frames: sizes, sensor counts, exposure sets and orders vary."""
    rng = np.random.default_rng(seed0)
    frames = []
    for i in range(n):
        w, h = [(96, 64), (64, 64), (80, 48)][i % 3]
        ns = 2 + (i % 3)
        exps = [1.0]
        for _ in range(ns - 1):
            exps.append(exps[-1] * 2.0 ** -int(rng.integers(2, 7)))
        from synth import rig as R
        sensors = R.random_rig(ns, w, h, exps, 2.0, 0.3, seed0 + i, **configs.NOISE)
        scene = EdgeScene(w, h, seed0 + i, n_lines=6)
        raws = configs.capture_all(scene, sensors, seed0 + i)
        order = 1 + (i % 2)
        params = configs.lpa_params(w, h, order, [1.0, 2.0, 3.0, 4.0])
        frames.append((sensors, raws, params))
    return frames


def alone(torch, ctx, rig, raws_dev, params):
    out = torch.empty((params["out_h"], params["out_w"], 3), dtype=torch.float32, device="cuda")
    smap = torch.empty((params["out_h"], params["out_w"], 3), dtype=torch.uint8, device="cuda")
    rig.reconstruct(raws_dev, params, out, smap)
    torch.cuda.synchronize()
    return out.cpu().numpy(), smap.cpu().numpy()


@pytest.mark.parametrize("storage", ["fused", "fp16"])
def test_batch_equals_alone_across_replays(torch_mod, storage):
    torch = torch_mod
    from paper_1308_4908_amd import Context, Rig

    ctx = Context(0)
    frames = make_frames(7)
    rigs, devs, params, refs = [], [], [], []
    for sensors, raws, p in frames:
        p = dict(p, storage=storage)
        rig = Rig(ctx, sensors)
        dev = [torch.from_numpy(r).cuda() for r in raws]
        rigs.append(rig)
        devs.append(dev)
        params.append(p)
        refs.append(alone(torch, ctx, rig, dev, p))
    # the first frame also against the oracle, to anchor the comparison
    if storage == "fused":
        s0, r0, p0 = frames[0]
        st = compare(refs[0][0], refs[0][1], oracle.reconstruct(s0, r0, p0, want_fits=True), s0, p0["order"])
        _say(f"[gpu] batch anchor frame vs oracle {st}")
    for rep in range(3):
        outs = [torch.full((p["out_h"], p["out_w"], 3), float(rep), device="cuda") for p in params]
        maps = [torch.zeros((p["out_h"], p["out_w"], 3), dtype=torch.uint8, device="cuda") for p in params]
        _say(f"[gpu] batch replay {rep} storage={storage}")
        ctx.reconstruct_batch(rigs, devs, params, outs, maps)
        torch.cuda.synchronize()
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda").sum().item()
        assert np.isfinite(x)
        for i in range(len(frames)):
            assert np.array_equal(outs[i].cpu().numpy(), refs[i][0], equal_nan=True), f"frame {i} replay {rep}"
            assert np.array_equal(maps[i].cpu().numpy(), refs[i][1]), f"frame {i} replay {rep}"
    for r in rigs:
        r.close()
    ctx.close()


@pytest.mark.parametrize("storage", ["fp16", "fp32"])
def test_batch_prepass_rows_unaligned_and_ragged(torch_mod, storage):
    """The batch pre-pass converts 8 samples per lane with 16-byte loads where
    both planes' rows are 16-byte aligned, and one at a time elsewhere and past
    the last group of 8.  Frames of odd widths, raw rows contiguous (unaligned
    pitch) or views into a wider buffer (aligned pitch, ragged tail), uint16
    and float DN: each batched frame equals its per-frame result bit for bit
    (the per-frame pre-pass converts one sample per lane)."""
    torch = torch_mod
    from paper_1308_4908_amd import Context, Rig
    from synth import rig as R

    ctx = Context(0)
    specs = [(93, 61, 2, False), (77, 50, 3, True), (93, 61, 4, True), (61, 37, 2, False)]
    for dt in (np.uint16, np.float32):
        rigs, devs, params, refs = [], [], [], []
        for k, (w, h, ns, padded) in enumerate(specs):
            seed = 4700 + k
            exps = [1.0, 1 / 8, 1 / 64, 1 / 4][:ns]
            sensors = R.random_rig(ns, w, h, exps, 2.0, 0.3, seed, **configs.NOISE)
            raws = configs.capture_all(EdgeScene(w, h, seed, n_lines=6), sensors, seed)
            dev = []
            for r in raws:
                r = r.astype(dt)
                if padded:  # a view into rows of 96 samples: aligned pitch, ragged tail
                    buf = np.zeros((h, 96), dt)
                    buf[:, :w] = r
                    dev.append(torch.from_numpy(buf).cuda()[:, :w])
                else:
                    dev.append(torch.from_numpy(np.ascontiguousarray(r)).cuda())
            p = configs.lpa_params(w, h, 1 + (k % 2), [1.0, 2.0, 3.0], storage=storage)
            rig = Rig(ctx, sensors)
            rigs.append(rig)
            devs.append(dev)
            params.append(p)
            refs.append(alone(torch, ctx, rig, dev, p))
        outs = [torch.full((p["out_h"], p["out_w"], 3), -3.0, device="cuda") for p in params]
        maps = [torch.zeros((p["out_h"], p["out_w"], 3), dtype=torch.uint8, device="cuda") for p in params]
        _say(f"[gpu] batch pre-pass storage={storage} raw {np.dtype(dt).name}")
        ctx.reconstruct_batch(rigs, devs, params, outs, maps)
        torch.cuda.synchronize()
        for i in range(len(specs)):
            assert np.array_equal(outs[i].cpu().numpy(), refs[i][0], equal_nan=True), f"frame {i} {np.dtype(dt).name}"
            assert np.array_equal(maps[i].cpu().numpy(), refs[i][1]), f"frame {i} map"
        for rig in rigs:
            rig.close()
    torch.cuda.synchronize()
    ctx.close()


def test_batch_refit_blocks_sliced_over_xcds(torch_mod):
    """The batch refit gives each of the 8 XCDs an eighth of every frame's
    32x32 output blocks (uneven slices: 12 to 80 blocks per frame, frames with
    and without refits).  Every batched frame equals its per-frame result bit
    for bit, and the FP64-refit counts match, with hundreds of refit outputs
    per frame."""
    torch = torch_mod
    from paper_1308_4908_amd import Context, Rig
    from synth import rig as R

    ctx = Context(0)
    specs = [(320, 200, 4), (256, 256, 3), (200, 320, 2), (130, 90, 3), (300, 140, 4)]
    rigs, devs, params, refs, counts = [], [], [], [], []
    for k, (w, h, ns) in enumerate(specs):
        seed = 4800 + k
        sensors = R.random_rig(ns, w, h, [1.0, 1 / 16, 1 / 128, 1 / 4][:ns], 2.0, 0.3, seed, **configs.NOISE)
        raws = configs.capture_all(EdgeScene(w, h, seed, n_lines=8), sensors, seed)
        dev = [torch.from_numpy(r).cuda() for r in raws]
        p = configs.lpa_params(w, h, 2 - (k % 2), [1.0, 2.0, 3.0, 4.0])
        if k == 3:
            p = dict(p, value_tol=-1.0)  # no accuracy target: no refit blocks for this frame
        rig = Rig(ctx, sensors)
        st = torch.zeros(2, dtype=torch.int64, device="cuda")
        out = torch.empty((h, w, 3), device="cuda")
        smap = torch.empty((h, w, 3), dtype=torch.uint8, device="cuda")
        rig.reconstruct(dev, p, out, smap, stats=st)
        torch.cuda.synchronize()
        rigs.append(rig)
        devs.append(dev)
        params.append(p)
        refs.append((out.cpu().numpy(), smap.cpu().numpy()))
        counts.append(st.cpu().numpy())
    assert sum(int(c[0]) for c in counts) > 1000
    outs = [torch.full((p["out_h"], p["out_w"], 3), -5.0, device="cuda") for p in params]
    maps = [torch.zeros((p["out_h"], p["out_w"], 3), dtype=torch.uint8, device="cuda") for p in params]
    stats = [torch.full((2,), -1, dtype=torch.int64, device="cuda") for _ in params]
    _say(f"[gpu] batch refit over XCD slices, fp64 counts {[int(c[0]) for c in counts]}")
    ctx.reconstruct_batch(rigs, devs, params, outs, maps, stats=stats)
    torch.cuda.synchronize()
    for i in range(len(specs)):
        assert np.array_equal(outs[i].cpu().numpy(), refs[i][0], equal_nan=True), f"frame {i}"
        assert np.array_equal(maps[i].cpu().numpy(), refs[i][1]), f"frame {i} map"
        assert np.array_equal(stats[i].cpu().numpy(), counts[i]), f"frame {i} counts"
    for rig in rigs:
        rig.close()
    torch.cuda.synchronize()
    ctx.close()


def test_batch_graph_reused_across_lds_sizes(torch_mod):
    """Consecutive batches of frames that need different LDS sizes (2- and
    4-sensor frames) replay each slot's graph with its kernel nodes updated:
    10 launches over the 4 slots, every frame equal to its result alone."""
    torch = torch_mod
    from paper_1308_4908_amd import Context, Rig

    ctx = Context(0)
    frames = make_frames(6, seed0=4300)
    sets = [[0, 3], [2, 5], [1, 4]]  # 2 sensors, 4 sensors, 3 sensors
    rigs, devs, params, refs = [], [], [], []
    for sensors, raws, p in frames:
        rig = Rig(ctx, sensors)
        dev = [torch.from_numpy(r).cuda() for r in raws]
        rigs.append(rig)
        devs.append(dev)
        params.append(p)
        refs.append(alone(torch, ctx, rig, dev, p))
    for launch in range(10):
        sel = sets[launch % 3]
        outs = [torch.full((params[i]["out_h"], params[i]["out_w"], 3), -1.0, device="cuda") for i in sel]
        maps = [torch.zeros((params[i]["out_h"], params[i]["out_w"], 3), dtype=torch.uint8, device="cuda")
                for i in sel]
        _say(f"[gpu] batch launch {launch}: frames {sel}")
        ctx.reconstruct_batch([rigs[i] for i in sel], [devs[i] for i in sel], [params[i] for i in sel], outs, maps)
        torch.cuda.synchronize()
        for k, i in enumerate(sel):
            assert np.array_equal(outs[k].cpu().numpy(), refs[i][0], equal_nan=True), f"frame {i} launch {launch}"
            assert np.array_equal(maps[k].cpu().numpy(), refs[i][1]), f"frame {i} launch {launch}"
    for r in rigs:
        r.close()
    ctx.close()


def test_injected_failure_fails_pending_and_context_recreates(torch_mod, monkeypatch):
    """LPA_TEST_FAIL_AFTER=2 (the serving loop's second batch launch fails
    from the host, no GPU work enqueued): the first frame completes, every
    later ticket ends with LPA_ERR_DEVICE, submissions are refused, and a new
    context on the device reconstructs as before."""
    torch = torch_mod
    from paper_1308_4908_amd import Context, LpaError, Rig, lpa

    frames = make_frames(3, seed0=4400)
    sensors, raws, p = frames[0]
    monkeypatch.setenv("LPA_TEST_FAIL_AFTER", "2")
    ctx = Context(0)
    monkeypatch.delenv("LPA_TEST_FAIL_AFTER")
    rig = Rig(ctx, sensors)
    dev = [torch.from_numpy(r).cuda() for r in raws]
    ref = alone(torch, ctx, rig, dev, p)
    outs = [torch.full((p["out_h"], p["out_w"], 3), -1.0, device="cuda") for _ in range(5)]
    torch.cuda.synchronize()
    _say("[gpu] injected serving failure: first batch")
    t0 = rig.submit(dev, p, outs[0])
    ctx.drain()
    r0 = ctx.poll(t0)
    assert r0.status == lpa.OK
    assert np.array_equal(outs[0].cpu().numpy(), ref[0], equal_nan=True)
    _say("[gpu] injected serving failure: later batches")
    # the loop may fail the context while these are submitted: then the
    # submission itself is refused with the same status
    tickets = []
    for o in outs[1:]:
        try:
            tickets.append(rig.submit(dev, p, o))
        except LpaError as e:
            assert e.status == lpa.ERR_DEVICE
    assert tickets
    with pytest.raises(LpaError):
        ctx.drain()
    for t in tickets:
        assert ctx.poll(t).status == lpa.ERR_DEVICE
    with pytest.raises(LpaError) as e:
        rig.submit(dev, p, outs[1])
    assert e.value.status == lpa.ERR_DEVICE
    assert "LPA_TEST_FAIL_AFTER" in str(e.value)
    ctx.close()
    _say("[gpu] injected serving failure: new context")
    ctx2 = Context(0)
    rig2 = Rig(ctx2, sensors)
    assert np.array_equal(alone(torch, ctx2, rig2, dev, p)[0], ref[0], equal_nan=True)
    rig2.close()
    ctx2.close()


def _serve(torch, ctx, items, host_pinned=True):
    """Submit items = [(rig, raws_np, params)] as fast as possible; returns outputs and results."""
    outs, tickets, hosts = [], [], []
    for rig, raws, p in items:
        if host_pinned:
            hs = [torch.from_numpy(r).pin_memory() for r in raws]
        else:
            hs = [np.ascontiguousarray(r) for r in raws]
        hosts.append(hs)
        out = torch.full((p["out_h"], p["out_w"], 3), -1.0, device="cuda")
        smap = torch.zeros((p["out_h"], p["out_w"], 3), dtype=torch.uint8, device="cuda")
        outs.append((out, smap))
        # the library's streams are not ordered after torch's: the fills must be done
        torch.cuda.synchronize()
        t = None
        while t is None:
            t = rig.submit(hs, p, out, smap, arrival_ns=0, host=True)
        tickets.append(t)
    ctx.drain()
    res = [ctx.poll(t) for t in tickets]
    torch.cuda.synchronize()
    return [(o.cpu().numpy(), m.cpu().numpy()) for o, m in outs], res


def test_serving_results_equal_alone(torch_mod):
    torch = torch_mod
    from paper_1308_4908_amd import Context, Rig, lpa

    ctx = Context(0)
    frames = make_frames(9, seed0=4200)
    items, refs = [], []
    for k, (sensors, raws, p) in enumerate(frames * 2):
        p = dict(p, storage=["fused", "fp16"][k % 2])
        rig = Rig(ctx, sensors)
        refs.append(alone(torch, ctx, rig, [torch.from_numpy(r).cuda() for r in raws], p))
        items.append((rig, raws, p))
    _say(f"[gpu] serving {len(items)} mixed frames (pinned host input)")
    got, res = _serve(torch, ctx, items, host_pinned=True)
    sizes = []
    for i, (g, r) in enumerate(zip(got, res)):
        assert r.status == lpa.OK, i
        assert r.t_arrival_ns <= r.t_admit_ns <= r.t_start_ns <= r.t_done_ns
        sizes.append(r.batch_size)
        assert np.array_equal(g[0], refs[i][0], equal_nan=True), f"frame {i}"
        assert np.array_equal(g[1], refs[i][1]), f"frame {i}"
    _say(f"  batch sizes {sizes}")
    _say("[gpu] serving with pageable host input")
    got, res = _serve(torch, ctx, items[:5], host_pinned=False)
    for i, (g, r) in enumerate(zip(got, res)):
        assert r.status == lpa.OK
        assert np.array_equal(g[0], refs[i][0], equal_nan=True)
    for it in items:
        it[0].close()
    ctx.close()


def test_serving_under_tight_budget(torch_mod):
    """A budget that holds about two frames: frames queue for admission and all
    complete correctly."""
    torch = torch_mod
    from paper_1308_4908_amd import Context, Rig, lpa

    frames = make_frames(6, seed0=4300)
    sizes = [sum((r.nbytes + 255) // 256 * 256 for r in raws) for _, raws, _ in frames]
    budget = int(2.5 * max(sizes)) + 4096
    ctx = Context(0, hbm_budget_bytes=budget)
    items, refs = [], []
    for sensors, raws, p in frames:
        rig = Rig(ctx, sensors)
        refs.append(alone(torch, ctx, rig, [torch.from_numpy(r).cuda() for r in raws], p))
        items.append((rig, raws, p))
    _say("[gpu] serving under a two-frame budget")
    got, res = _serve(torch, ctx, items)
    for i, (g, r) in enumerate(zip(got, res)):
        assert r.status == lpa.OK
        # frames in one launch were admitted together, so they fit the budget together
        assert r.batch_size <= budget // min(sizes)
        assert np.array_equal(g[0], refs[i][0], equal_nan=True)
    # a frame larger than the whole budget is rejected with OOM (terminal), not hung
    small_ctx = Context(0, hbm_budget_bytes=1024)
    sensors, raws, p = frames[0]
    rig = Rig(small_ctx, sensors)
    out = torch.empty((p["out_h"], p["out_w"], 3), device="cuda")
    t = rig.submit([torch.from_numpy(r).pin_memory() for r in raws], p, out, host=True)
    small_ctx.drain()
    assert small_ctx.poll(t).status == lpa.ERR_OOM
    rig.close()
    small_ctx.close()
    for it in items:
        it[0].close()
    ctx.close()


def test_autotune_keeps_results_and_persists(torch_mod, tmp_path):
    """The tuner only changes the launch shape: tuned output is bit-identical;
    its choices round-trip through the JSON file."""
    torch = torch_mod
    from paper_1308_4908_amd import Context, Rig

    sensors, raws, p = make_frames(2, seed0=4400)[1]  # an order-2 frame
    assert p["order"] == 2
    ctx = Context(0)
    rig = Rig(ctx, sensors)
    dev = [torch.from_numpy(r).cuda() for r in raws]
    ref = alone(torch, ctx, rig, dev, p)
    out = torch.empty((p["out_h"], p["out_w"], 3), device="cuda")
    _say("[gpu] autotune")
    res = rig.autotune(dev, p, out, reps=2)
    assert res.n_candidates == 8 and res.tile_w * res.tile_h == 256
    got = alone(torch, ctx, rig, dev, p)
    assert np.array_equal(got[0], ref[0], equal_nan=True) and np.array_equal(got[1], ref[1])
    path = str(tmp_path / "tune.json")
    ctx.tuner_save(path)
    ctx2 = Context(0)
    ctx2.tuner_load(path)
    rig2 = Rig(ctx2, sensors)
    got2 = alone(torch, ctx2, rig2, dev, p)
    assert np.array_equal(got2[0], ref[0], equal_nan=True)
    text = open(path).read()
    assert f'"tile_w": {res.tile_w}' in text
    rig2.close()
    ctx2.close()
    rig.close()
    ctx.close()
