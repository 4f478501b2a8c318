"""Per-pixel calibration frames (Sec. 6: bias frame, photo-response
non-uniformity, readout variance, saturation frame; defect mask) through the
C ABI, against the FP64 oracle fed the same frames (float32 values)."""
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


def frames(sensor, seed, defects=0.01, low_sat=0.05):
    """Random calibration frames for one sensor, as float32 values (what the
    library stores), returned as float64 for the oracle."""
    rng = np.random.default_rng(seed)
    shape = (sensor["height"], sensor["width"])
    sat = np.full(shape, 4095.0)
    sat[rng.random(shape) < low_sat] = 2500.0
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    return {"bias": f32(rng.uniform(55.0, 75.0, shape)), "prnu": f32(rng.uniform(0.85, 1.15, shape)),
            "read_var": f32(rng.uniform(4.0, 20.0, shape)), "sat": f32(sat),
            "defect": (rng.random(shape) < defects).astype(np.uint8)}


def calibrated(sensors, seed):
    return [dict(s, calib=frames(s, seed + i)) for i, s in enumerate(sensors)]


def run(torch, ctx, sensors, raws, params, plain=False, steer=None):
    """Returns (rgb, scale map, sd map); with steer = [] (CALPA) the steering
    matrices the GPU used are appended to it."""
    from paper_1308_4908_amd import Rig

    rig = Rig(ctx, sensors)
    dev = [torch.from_numpy(np.ascontiguousarray(r)).cuda() for r in raws]
    H, W = params["out_h"], params["out_w"]
    out = torch.full((H, W, 3), -12345.0, device="cuda")
    smap = torch.full((H, W, 3), 0xEE, dtype=torch.uint8, device="cuda")
    sd = torch.full((H, W, 3), -1.0, device="cuda")
    st = torch.full((H, W, 4), -7.0, device="cuda") if steer is not None else None
    rig.reconstruct(dev, params, out, smap, plain=plain, sd_map=sd, steer_map=st)
    torch.cuda.synchronize()
    res = out.cpu().numpy(), smap.cpu().numpy(), sd.cpu().numpy()
    if steer is not None:
        steer.append(st.cpu().numpy().reshape(-1, 4)[:, :3].astype(np.float64))
    rig.close()
    return res


def test_full_frame_vs_oracle(torch_mod, ctx):
    """3 x 96^2 rotated rig with random frames, order 2 and ICI: every pixel."""
    base = R.random_rig(3, 96, 96, [1.0, 1 / 8, 1 / 64], 1.5, 0.2, 8100, **configs.NOISE)
    sensors = calibrated(base, 8100)
    raws = configs.capture_all(EdgeScene(96, 96, 8100, n_lines=10), base, 8100)
    params = configs.lpa_params(96, 96, 2, [1.0, 2.0, 3.0])
    _say("[gpu] calibration frames, full frame")
    rgb, smap, sd = run(torch_mod, ctx, sensors, raws, params)
    orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
    st = compare(rgb, smap, orc, sensors, 2, gpu_sd=sd)
    _say(f"  stats {st}")
    assert st["agree_frac"] > 0.999
    # the frames matter: the scalar model gives a different reconstruction
    plain = oracle.reconstruct(base, raws, params)
    assert np.nanmax(np.abs(plain["rgb"] - orc["rgb"]) / np.maximum(np.abs(orc["rgb"]), 2.0)) > 1e-2


def test_plain_form_equals_fused_and_fp16(torch_mod, ctx):
    """The pre-pass decodes with the same frames (bit-identical); FP16 storage
    of 12-bit raw values is lossless, so it is bit-identical too and meets the
    value gate against the oracle."""
    base = R.random_rig(3, 64, 64, [1.0, 1 / 8, 1 / 64], 1.5, 0.2, 8200, **configs.NOISE)
    sensors = calibrated(base, 8200)
    raws = configs.capture_all(EdgeScene(64, 64, 8200, n_lines=8), base, 8200)
    params = configs.lpa_params(64, 64, 1, [1.5, 3.0])
    _say("[gpu] calibration frames, plain / fused / fp16")
    a = run(torch_mod, ctx, sensors, raws, params)
    b = run(torch_mod, ctx, sensors, raws, params, plain=True)
    assert np.array_equal(a[0], b[0], equal_nan=True) and np.array_equal(a[1], b[1])
    c = run(torch_mod, ctx, sensors, raws, dict(params, storage="fp16"))
    assert np.array_equal(a[0], c[0], equal_nan=True) and np.array_equal(a[1], c[1])
    orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
    st = compare(c[0], c[1], orc, sensors, 1)
    _say(f"  fp16 vs oracle {st}")
    assert st["agree_frac"] > 0.999


def test_constant_scene_closed_form(torch_mod, ctx):
    """y_i = b_i + g n a_i f with integer b_i and a_i on a 2^-10 grid, so every
    raw value is exact in FP32 (float DN, no noise).  The oracle returns f
    exactly (closed form); the GPU is held to the conditioning-aware gates
    against it (its per-sample radiance carries one FP32 rounding of
    1 / (g n a_i))."""
    base = R.random_rig(3, 64, 64, [1.0, 1 / 4, 1 / 16], 1.5, 0.3, 8300, **configs.NOISE)
    sensors, raws = [], []
    f = 640.0
    for i, s in enumerate(base):
        fr = frames(s, 8300 + i)
        fr["bias"] = np.round(fr["bias"])
        fr["prnu"] = np.round(fr["prnu"] * 1024.0) / 1024.0
        sensors.append(dict(s, calib=fr))
        y = fr["bias"] + s["gain"] * s["exposure"] * fr["prnu"] * f
        assert np.array_equal(y.astype(np.float32).astype(np.float64), y)
        raws.append(y.astype(np.float32))
    params = configs.lpa_params(48, 48, 2, [1.5, 3.0], out_affine=[1, 0, 8, 0, 1, 8])
    _say("[gpu] calibration frames, constant scene")
    rgb, smap, sd = run(torch_mod, ctx, sensors, raws, params)
    orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
    ok = ~np.isnan(orc["rgb"])
    assert ok.mean() > 0.99
    np.testing.assert_allclose(orc["rgb"][ok], f, rtol=1e-12)
    st = compare(rgb, smap, orc, sensors, 2, gpu_sd=sd)
    _say(f"  stats {st}")
    assert st["agree_frac"] > 0.999
    assert np.median(np.abs(rgb[np.isfinite(rgb)] - f)) / f < 1e-6  # a few FP32 ulps


def test_batch_and_serving_equal_alone(torch_mod, ctx):
    """Batches and served frames read the rig's resident frames: results are
    bit-identical to the frame reconstructed alone."""
    from paper_1308_4908_amd import Rig

    torch = torch_mod
    base = R.random_rig(3, 80, 48, [1.0, 1 / 8, 1 / 64], 1.5, 0.2, 8400, **configs.NOISE)
    sensors = calibrated(base, 8400)
    raws = configs.capture_all(EdgeScene(80, 48, 8400, n_lines=6), base, 8400)
    params = configs.lpa_params(80, 48, 2, [1.0, 2.0, 3.0, 4.0])
    _say("[gpu] calibration frames, batch and serving")
    alone = run(torch, ctx, sensors, raws, params)
    rig = Rig(ctx, sensors)
    dev = [torch.from_numpy(r).cuda() for r in raws]
    outs = [torch.full((48, 80, 3), -1.0, device="cuda") for _ in range(3)]
    ctx.reconstruct_batch([rig] * 3, [dev] * 3, [params] * 3, outs)
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(o.cpu().numpy(), alone[0], equal_nan=True)
    out = torch.full((48, 80, 3), -1.0, device="cuda")
    torch.cuda.synchronize()  # the library's streams are not ordered after torch's
    t = None
    while t is None:
        t = rig.submit([torch.from_numpy(r).pin_memory() for r in raws], params, out, host=True)
    ctx.drain()
    from paper_1308_4908_amd import lpa

    assert ctx.poll(t).status == lpa.OK
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), alone[0], equal_nan=True)
    rig.close()


def test_precomputed_weights_with_frames(torch_mod, ctx):
    """The pre-computed-weight path stages samples with the same decode."""
    base = R.random_rig(4, 64, 64, [1.0, 1 / 4, 1 / 16, 1 / 64], 2.0, 0.0, 8500, **configs.NOISE)
    sensors = calibrated(base, 8500)
    raws = configs.capture_all(EdgeScene(64, 64, 8500, n_lines=8), base, 8500)
    params = configs.lpa_params(64, 64, 2, [1.0, 2.0, 3.0], precomputed_weights=True)
    _say("[gpu] calibration frames, pre-computed weights")
    rgb, smap, sd = run(torch_mod, ctx, sensors, raws, params)
    orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
    st = compare(rgb, smap, orc, sensors, 2, gpu_sd=sd)
    _say(f"  stats {st}")
    assert st["agree_frac"] > 0.999


def test_invalid_frames_rejected(torch_mod, ctx):
    from paper_1308_4908_amd import LpaError, Rig, lpa

    base = R.random_rig(1, 32, 24, [1.0], 1.0, 0.0, 8600, **configs.NOISE)[0]
    shape = (24, 32)
    for bad in ({"prnu": np.zeros(shape)}, {"prnu": np.full(shape, np.inf)}, {"read_var": np.zeros(shape)},
                {"bias": np.full(shape, np.nan)}, {"sat": np.full(shape, np.nan)}):
        with pytest.raises(LpaError) as e:
            Rig(ctx, [dict(base, calib=bad)])
        assert e.value.status == lpa.ERR_INVALID_ARG


def test_calpa_with_frames(torch_mod, ctx):
    """CALPA's three passes decode with the frames too: the end-to-end chain
    against the oracle's chain on the same frames (each value within the gate
    of the oracle's chain or of its last stage run on the GPU's steering)."""
    base = R.random_rig(3, 64, 64, [1.0, 1 / 8, 1 / 64], 1.5, 0.2, 8700, **configs.NOISE)
    sensors = calibrated(base, 8700)
    raws = configs.capture_all(EdgeScene(64, 64, 8700, n_lines=8), base, 8700)
    adapt = {"alpha": 0.2, "lambda1": 1.0, "lambda2": 0.001, "grad_radius": 2.0, "grad_order": 1,
             "grad_halfwin": 2, "max_stretch": 2.0}
    params = configs.lpa_params(64, 64, 2, [1.0, 2.0, 3.0], mode="calpa", adapt=adapt)
    _say("[gpu] calibration frames, CALPA")
    cg = []
    rgb, smap, sd = run(torch_mod, ctx, sensors, raws, params, steer=cg)
    orc = oracle.reconstruct_adaptive(sensors, raws, params, adapt, want_fits=True, want_stages=True)
    assert np.abs(cg[0] - orc["C"]).max() < 1e-5 * np.abs(orc["C"]).max()
    # the steering difference's effect, measured by the oracle's last stage on the GPU's matrices
    orc_g = oracle.reconstruct_steered(sensors, raws, params, cg[0], want_fits=True)
    st = compare(rgb, smap, orc, sensors, 2, gpu_sd=sd, alt_orc=orc_g)
    _say(f"  stats {st}")
    assert st["agree_frac"] > 0.999
