"""Parity at the limits of the C ABI: the most sensors (8) and window radii (8)
a rig and a call take, with radii wide enough that the staged tile falls back
to 16 x 8, 8 x 8, 8 x 4 and 4 x 4 output pixels (fewer lanes than a wave at
the smallest); green windows of another size (kappa_G != 1, Sec. 5.5) and
explicit window parameters h on the general kernel; windows no tile can stage
refused with the output untouched.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import configs, rig as R
from synth.scene import EdgeScene
from parity_utils import compare

pytestmark = pytest.mark.gpu

OUT_AFFINE = [1, 0, 18.5, 0, 1, 20.25]  # 29 x 21 output inside 64 x 64 sensors


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


def run(torch, ctx, sensors, raws, params, plain=False):
    from paper_1308_4908_amd import Rig

    rig = Rig(ctx, sensors)
    dev = [torch.from_numpy(np.ascontiguousarray(r)).cuda() for r in raws]
    H, W = params["out_h"], params["out_w"]
    out = torch.full((H, W, 3), -12345.0, device="cuda")
    smap = torch.full((H, W, 3), 0xEE, dtype=torch.uint8, device="cuda")
    sd = torch.full((H, W, 3), -1.0, device="cuda")
    rig.reconstruct(dev, params, out, smap, plain=plain, sd_map=sd)
    torch.cuda.synchronize()
    res = out.cpu().numpy(), smap.cpu().numpy(), sd.cpu().numpy()
    rig.close()
    return res


def eight_sensor_rig(seed):
    return R.random_rig(8, 64, 64, [2.0 ** -k for k in range(8)], 2.0, 0.3, seed, **configs.NOISE)


# Largest radius -> the tile the launch falls back to for 8 sensors (LDS of the
# staged regions: 16 x 16 needs more than 64 KiB from r = 4 on).
@pytest.mark.parametrize("r_max,tile", [(4.0, "16x8"), (7.0, "8x8"), (8.0, "8x4"), (9.5, "4x4")])
def test_most_sensors_and_scales(torch_mod, ctx, r_max, tile):
    """8 sensors (exposures 2^0 .. 2^-7), 8 radii from 1 to r_max, order 2 with
    ICI, ragged 29 x 21 output: every pixel against the oracle, and the plain
    FP32 form (pre-pass planes) bit-identical to the fused one."""
    sensors = eight_sensor_rig(9100)
    raws = configs.capture_all(EdgeScene(64, 64, 9100, n_lines=8), sensors, 9100)
    params = configs.lpa_params(29, 21, 2, list(np.linspace(1.0, r_max, 8)), out_affine=OUT_AFFINE)
    _say(f"[gpu] 8 sensors, 8 radii up to {r_max} (tile {tile})")
    rgb, smap, sd = run(torch_mod, ctx, sensors, raws, params)
    orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
    st = compare(rgb, smap, orc, sensors, 2, gpu_sd=sd)
    _say(f"  stats {st}")
    assert st["agree_frac"] > 0.999
    assert np.isfinite(rgb).mean() > 0.99
    assert len(np.unique(smap & 0x0F)) > 2  # ICI picks among several radii
    plain = run(torch_mod, ctx, sensors, raws, params, plain=True)
    assert np.array_equal(plain[0], rgb, equal_nan=True) and np.array_equal(plain[1], smap)


@pytest.mark.parametrize("kappa", [0.75, 1.3])
def test_green_window_ratio(torch_mod, ctx, kappa):
    """Green windows kappa_G times the red/blue ones (radius r kappa_G, window
    parameter h kappa_G^2) on a rotated 4-sensor rig: every pixel."""
    sensors = R.random_rig(4, 64, 64, [1.0, 1 / 4, 1 / 16, 1 / 64], 2.0, 0.3, 9200, **configs.NOISE)
    raws = configs.capture_all(EdgeScene(64, 64, 9200, n_lines=8), sensors, 9200)
    params = configs.lpa_params(37, 23, 2, [1.0, 2.0, 3.0], out_affine=[1, 0, 12.5, 0, 1, 20.25],
                                green_ratio=kappa)
    _say(f"[gpu] green window ratio {kappa}")
    rgb, smap, sd = run(torch_mod, ctx, sensors, raws, params)
    orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
    st = compare(rgb, smap, orc, sensors, 2, gpu_sd=sd)
    _say(f"  stats {st}")
    assert st["agree_frac"] > 0.999
    # the green channel's result depends on kappa, the red and blue do not
    ref = oracle.reconstruct(sensors, raws, dict(params, green_ratio=1.0))
    assert np.array_equal(ref["rgb"][..., 0], orc["rgb"][..., 0], equal_nan=True)
    assert not np.array_equal(ref["rgb"][..., 1], orc["rgb"][..., 1], equal_nan=True)


def test_explicit_window_parameters(torch_mod, ctx):
    """Window parameters h given per radius (wider and narrower than the
    default 2 r^2 / 9), order 1 and order 2 with ICI."""
    sensors = configs.full_rig(seed=9300, size=64)
    raws = configs.capture_all(EdgeScene(64, 64, 9300, n_lines=8), sensors, 9300)
    for order in (1, 2):
        params = configs.lpa_params(37, 23, order, [1.5, 2.5, 4.0], out_affine=[1, 0, 12.5, 0, 1, 20.25],
                                    h=[0.3, 2.5, 2.0])
        _say(f"[gpu] explicit window parameters, order {order}")
        rgb, smap, sd = run(torch_mod, ctx, sensors, raws, params)
        orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
        st = compare(rgb, smap, orc, sensors, order, gpu_sd=sd)
        _say(f"  stats {st}")
        assert st["agree_frac"] > 0.999
        default = oracle.reconstruct(sensors, raws, dict(params, h=[0.0] * 3))
        assert not np.array_equal(default["rgb"], orc["rgb"], equal_nan=True)


def test_windows_too_wide_refused(torch_mod, ctx):
    """A window no tile can stage (8 sensors, r = 10: more than 64 KiB at 4 x 4)
    and one wider than 240 sensor pixels are refused as unsupported before
    anything is enqueued; the output keeps its contents."""
    from paper_1308_4908_amd import LpaError, Rig, lpa

    torch = torch_mod
    sensors = eight_sensor_rig(9400)
    raws = configs.capture_all(EdgeScene(64, 64, 9400, n_lines=4), sensors, 9400)
    rig = Rig(ctx, sensors)
    dev = [torch.from_numpy(r).cuda() for r in raws]
    out = torch.full((21, 29, 3), 7.0, device="cuda")
    _say("[gpu] windows too wide")
    for radii, plain in (([2.0, 10.0], False), ([2.0, 10.0], True), ([130.0], False)):
        p = configs.lpa_params(29, 21, 2, radii, out_affine=OUT_AFFINE)
        with pytest.raises(LpaError) as e:
            rig.reconstruct(dev, p, out, plain=plain)
        assert e.value.status == lpa.ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
    rig.close()
