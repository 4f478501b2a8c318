"""Temporal LPA on the GPU (lpa_reconstruct_temporal) against the oracle's
temporal reconstruction (readings T1-T4 in oracle/lpa_oracle.h), through the
C ABI, with the metric and gates of parity_utils.

  * a static scene over 3 noisy frames of 2 sensors, order 2, ICI over three
    spatio-temporal scales, a ragged 72 x 56 frame: every output;
  * a scene moving by 0.6 px per frame (frames captured through shifted
    sensor maps, reconstructed through the rig's own): every output;
  * 4 sensors x 2 frames of 384^2 (every staged sensor slot used): sampled
    outputs, borders and the ragged tail included;
  * one frame, or h_t = 0 over several, equals lpa_reconstruct bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import configs, rig as R
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


@pytest.fixture(scope="module")
def ctx(torch_mod):
    from paper_1308_4908_amd import Context

    c = Context(0)
    yield c
    torch_mod.cuda.synchronize()
    c.close()


def _run(torch, ctx, sensors, frames, params, temporal=True):
    from paper_1308_4908_amd import Rig

    rig = Rig(ctx, sensors)
    dev = [[torch.from_numpy(np.ascontiguousarray(r)).cuda() for r in fr] for fr in frames]
    H, W = params["out_h"], params["out_w"]
    out = torch.full((H, W, 3), -12345.0, device="cuda")
    smap = torch.full((H, W, 3), 0xEE, dtype=torch.uint8, device="cuda")
    sd = torch.full((H, W, 3), -1.0, device="cuda")
    stats = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    if temporal:
        rig.reconstruct_temporal(dev, params, out, smap, sd_map=sd, stats=stats)
    else:
        rig.reconstruct(dev[0], params, out, smap, sd_map=sd, stats=stats)
    torch.cuda.synchronize()
    res = out.cpu().numpy(), smap.cpu().numpy(), sd.cpu().numpy(), stats.cpu().numpy()
    rig.close()
    return res


def _static_case(seed, size, n_sensors, n_times):
    sensors = R.random_rig(n_sensors, size, size, [1.0, 1 / 8, 1 / 64, 1 / 4][:n_sensors], 1.5, 0.2, seed,
                           **configs.NOISE)
    scene = EdgeScene(size, size, seed, n_lines=max(4, size // 16))
    frames = [[R.capture(scene, s, (seed, t, i)) for i, s in enumerate(sensors)] for t in range(n_times)]
    return sensors, frames


def test_static_scene_full_frame(torch_mod, ctx):
    sensors, frames = _static_case(7100, 80, 2, 3)
    params = configs.lpa_params(72, 56, 2, [1.0, 2.0, 3.0], out_affine=[1, 0, 4, 0, 1, 12],
                                h_t=[0.25, 1.0, 4.0])
    _say("[gpu] temporal static 2 sensors x 3 frames, 72x56")
    rgb, smap, sd, stats = _run(torch_mod, ctx, sensors, frames, params)
    assert not np.any(rgb == -12345.0) and not np.any(smap == 0xEE)
    orc = oracle.reconstruct_temporal(sensors, frames, params, want_fits=True)
    st = compare(rgb.reshape(-1, 3), smap.reshape(-1, 3), orc, sensors, 2, gpu_sd=sd.reshape(-1, 3))
    _say(f"  stats {st}; fp64 outputs {stats[0]}")
    assert st["agree_frac"] > 0.999
    assert stats[1] == np.count_nonzero(smap == 0xFF)


def test_moving_scene_full_frame(torch_mod, ctx):
    size = 80
    sensors = R.random_rig(2, size, size, [1.0, 1 / 16], 1.5, 0.2, 7200, **configs.NOISE)
    scene = EdgeScene(size, size, 7200, n_lines=6)
    frames = []
    for t in range(3):
        # the scene at time -t sits 0.6 t px to the left: capture through shifted maps
        moved = [dict(s, affine=[*s["affine"][:2], s["affine"][2] + 0.6 * t, *s["affine"][3:]]) for s in sensors]
        frames.append([R.capture(scene, s, (7200, t, i)) for i, s in enumerate(moved)])
    params = configs.lpa_params(64, 64, 1, [1.0, 2.0, 3.0], out_affine=[1, 0, 8, 0, 1, 8], h_t=[0.5, 2.0, 8.0])
    _say("[gpu] temporal moving scene 2 sensors x 3 frames, 64x64, order 1")
    rgb, smap, sd, stats = _run(torch_mod, ctx, sensors, frames, params)
    orc = oracle.reconstruct_temporal(sensors, frames, params, want_fits=True)
    st = compare(rgb.reshape(-1, 3), smap.reshape(-1, 3), orc, sensors, 1, gpu_sd=sd.reshape(-1, 3))
    _say(f"  stats {st}")
    assert st["agree_frac"] > 0.999


def test_every_staged_slot_sampled(torch_mod, ctx):
    sensors, frames = _static_case(7300, 384, 4, 2)
    params = configs.lpa_params(384, 384, 2, [1.0, 2.0, 3.0, 4.0], h_t=[0.5, 1.0, 2.0, 4.0])
    _say("[gpu] temporal 4 sensors x 2 frames, 384^2, sampled")
    rgb, smap, sd, stats = _run(torch_mod, ctx, sensors, frames, params)
    rng = np.random.default_rng(73)
    u = np.concatenate([rng.integers(0, 384, 1500), np.arange(0, 384, 7), np.full(20, 383)])
    v = np.concatenate([rng.integers(0, 384, 1500), np.full(55, 0), np.arange(364, 384)])
    pix = np.stack([u, v], 1).astype(np.int32)
    orc = oracle.reconstruct_temporal(sensors, frames, params, pixels=pix, want_fits=True)
    st = compare(rgb[v, u], smap[v, u], orc, sensors, 2, gpu_sd=sd[v, u])
    _say(f"  stats {st}; fp64 outputs {stats[0]}")
    assert st["agree_frac"] > 0.999


@pytest.mark.parametrize("n_times", [1, 3])
def test_single_frame_is_spatial(torch_mod, ctx, n_times):
    sensors, frames = _static_case(7400, 96, 2, 3)
    params = configs.lpa_params(88, 70, 2, [1.0, 2.0, 4.0], h_t=[0.0, 0.0, 0.0])
    _say(f"[gpu] temporal n_times={n_times}, h_t=0 vs spatial")
    a = _run(torch_mod, ctx, sensors, frames[:n_times], params)
    b = _run(torch_mod, ctx, sensors, frames[:1], params, temporal=False)
    assert np.array_equal(a[0], b[0], equal_nan=True)
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2], equal_nan=True)
    assert np.array_equal(a[3], b[3])


def test_refused_forms(torch_mod, ctx):
    from paper_1308_4908_amd import LpaError, Rig, lpa

    sensors, frames = _static_case(7500, 32, 2, 3)
    rig = Rig(ctx, sensors)
    dev = [[torch_mod.from_numpy(np.ascontiguousarray(r)).cuda() for r in fr] for fr in frames]
    out = torch_mod.full((32, 32, 3), 7.0, device="cuda")
    base = configs.lpa_params(32, 32, 1, [2.0], h_t=[1.0])
    cases = [
        (dev, dict(base, storage="fp16"), lpa.ERR_UNSUPPORTED),        # raw frames only
        (dev, dict(base, mode="calpa"), lpa.ERR_UNSUPPORTED),          # isotropic windows only
        (dev * 2, base, lpa.ERR_UNSUPPORTED),                          # 6 frames x 2 sensors > 8 staged
        (dev, dict(base, h_t=[0.1]), lpa.ERR_INVALID_ARG),             # oldest frame's factor would underflow
        (dev, dict(base, h_t=[-1.0]), lpa.ERR_INVALID_ARG),
    ]
    for fr, prm, status in cases:
        with pytest.raises(LpaError) as e:
            rig.reconstruct_temporal(fr, prm, out)
        assert e.value.status == status
    torch_mod.cuda.synchronize()
    assert torch_mod.all(out == 7.0)
    rig.close()
