"""Pre-computed window weights (Sec. 8: the paper's fast path for registered
sensors), through the C ABI, against the FP64 oracle.

Rigs whose sensor maps and output map are translations get their window
weights and monomials from per-parity tables instead of computing them per
sample.  The estimator is unchanged, so the oracle and the metric and
tolerances of ``parity_utils`` apply as they are; noise-free scenes pin the
scale maps bit for bit.  Everything else (rotated rigs, scaled output maps,
CALPA, batches, serving, the tuner) must refuse the flag with
LPA_ERR_UNSUPPORTED and leave the output untouched.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import configs, rig as R
from synth.scene import EdgeScene, PolynomialScene, StepScene
from parity_utils import compare, firm_mask, fp16_round_dn

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


def run(torch, ctx, sensors, raws, params, stencil=True, plain=False, rig=None):
    from paper_1308_4908_amd import Rig

    own = rig is None
    rig = rig or Rig(ctx, sensors)
    dev = [torch.from_numpy(np.ascontiguousarray(r)).cuda() for r in raws]
    H, W = params["out_h"], params["out_w"]
    out = torch.full((H, W, 3), -12345.0, device="cuda")
    smap = torch.full((H, W, 3), 0xEE, dtype=torch.uint8, device="cuda")
    sd = torch.full((H, W, 3), -1.0, device="cuda")
    rig.reconstruct(dev, dict(params, precomputed_weights=stencil), out, smap, plain=plain, sd_map=sd)
    torch.cuda.synchronize()
    res = out.cpu().numpy(), smap.cpu().numpy(), sd.cpu().numpy()
    if own:
        rig.close()
    return res


def translation_rig(n, size, seed):
    return R.random_rig(n, size, size, [1.0, 1 / 4, 1 / 16, 1 / 64][:n], 2.0, 0.0, seed, **configs.NOISE)


@pytest.mark.parametrize("order,radii,storage", [(2, [1.0, 2.0, 3.0, 4.0], "fused"), (1, [2.0], "fp32"),
                                                 (0, [1.5, 3.0], "fused"), (1, [1.0, 2.5], "fused")])
def test_full_frame_vs_oracle(torch_mod, ctx, order, radii, storage):
    """4 x 96^2 translation-only rig, every output pixel (6 x 6 tiles)."""
    sensors = translation_rig(4, 96, 7000 + order)
    scene = EdgeScene(96, 96, 7000 + order, n_lines=10)
    raws = configs.capture_all(scene, sensors, 7000 + order)
    params = configs.lpa_params(96, 96, order, radii, storage=storage)
    _say(f"[gpu] stencil full frame order={order} radii={radii} storage={storage}")
    rgb, smap, sd = run(torch_mod, ctx, sensors, raws, params)
    orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
    st = compare(rgb, smap, orc, sensors, order, gpu_sd=sd)
    _say(f"  stats {st}")
    assert st["agree_frac"] > 0.999


def test_ragged_translated_output_green_ratio(torch_mod, ctx):
    """Ragged 37 x 23 grid whose output map is a fractional translation, three
    sensors, smaller green windows (kappa_G = 2^-1/4), order 2 with ICI."""
    sensors = translation_rig(3, 64, 7100)
    scene = EdgeScene(64, 64, 7100, n_lines=8)
    raws = configs.capture_all(scene, sensors, 7100)
    params = configs.lpa_params(37, 23, 2, [1.5, 3.0], out_affine=[1.0, 0.0, 20.5, 0.0, 1.0, 30.25],
                                green_ratio=2 ** -0.25)
    _say("[gpu] stencil ragged, translated output, green ratio")
    rgb, smap, sd = run(torch_mod, ctx, sensors, raws, params)
    orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
    st = compare(rgb, smap, orc, sensors, 2, gpu_sd=sd)
    _say(f"  stats {st}")
    assert st["agree_frac"] > 0.999
    assert not np.any(rgb == -12345.0)


def test_noise_free_polynomial_exact(torch_mod, ctx):
    """Noise-free quadratic radiance (float DN): the order-2 estimate is the
    field value and ICI keeps the largest valid radius: scale maps equal the
    oracle's bit for bit."""
    rng = np.random.default_rng(15)
    coeffs = np.zeros((3, 6))
    coeffs[:, 0] = rng.uniform(500, 900, 3)
    coeffs[:, 1:3] = rng.uniform(-4, 4, (3, 2))
    coeffs[:, 3:6] = rng.uniform(-0.02, 0.02, (3, 3))
    scene = PolynomialScene(coeffs)
    sensors = translation_rig(4, 64, 7200)
    raws = [R.capture_noise_free(scene, s) for s in sensors]
    params = configs.lpa_params(40, 40, 2, [1.0, 2.0, 3.0, 4.0], out_affine=[1, 0, 12, 0, 1, 12])
    _say("[gpu] stencil noise-free polynomial")
    rgb, smap, _ = run(torch_mod, ctx, sensors, raws, params)
    orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
    u, v = np.meshgrid(np.arange(40.0) + 12, np.arange(40.0) + 12)
    truth = np.stack([scene.radiance(u, v, c) for c in range(3)], -1)
    np.testing.assert_allclose(rgb, truth, rtol=2e-5)
    assert firm_mask(orc, 2, sensors).mean() > 0.7
    assert np.array_equal(smap.reshape(-1, 3), orc["scale_map"])


def test_noise_free_step_edge_ici_exact(torch_mod, ctx):
    """Axis-aligned step edge, integer-translated sensors, noise-free: every
    oracle decision is firm, and the scale map must match it everywhere."""
    scene = StepScene(20.0, 300.0, 3000.0)
    sensors = [R.make_sensor(48, 48, [1, 0, t[0], 0, 1, t[1]], e)
               for t, e in (((0, 0), 1.0), ((1, 0), 0.25), ((0, 1), 1 / 16), ((1, 1), 1 / 64))]
    raws = [R.capture_noise_free(scene, s) for s in sensors]
    params = configs.lpa_params(32, 32, 2, [1.0, 2.0, 3.0, 4.0], out_affine=[1, 0, 6, 0, 1, 6])
    _say("[gpu] stencil noise-free step edge")
    rgb, smap, _ = run(torch_mod, ctx, sensors, raws, params)
    orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
    assert firm_mask(orc, 2, sensors).all()
    assert np.array_equal(smap.reshape(-1, 3), orc["scale_map"])
    compare(rgb, smap, orc, sensors, 2)


def test_fp16_storage(torch_mod, ctx):
    """FP16 storage against the oracle fed the same FP16-rounded samples."""
    sensors = translation_rig(4, 96, 7300)
    scene = EdgeScene(96, 96, 7300, n_lines=10)
    raws = configs.capture_all(scene, sensors, 7300)
    params = configs.lpa_params(96, 96, 2, [1.0, 2.0, 3.0, 4.0], storage="fp16")
    _say("[gpu] stencil fp16 storage")
    rgb, smap, _ = run(torch_mod, ctx, sensors, raws, params)
    conv = [fp16_round_dn(r, s) for r, s in zip(raws, sensors)]
    orc16 = oracle.reconstruct([c[1] for c in conv], [c[0] for c in conv], params, want_fits=True)
    st = compare(rgb, smap, orc16, sensors, 2)
    _say(f"  vs fp16-fed oracle {st}")
    assert st["agree_frac"] > 0.999


def test_agrees_with_general_path_and_plain_form(torch_mod, ctx):
    """Same frame through the general kernel: the same firm decisions and
    values within both paths' tolerance; the plain form (FP32 planes) of the
    pre-computed path equals its fused form bit for bit."""
    sensors = translation_rig(4, 96, 7400)
    scene = EdgeScene(96, 96, 7400, n_lines=10)
    raws = configs.capture_all(scene, sensors, 7400)
    params = configs.lpa_params(96, 96, 2, [1.0, 2.0, 3.0, 4.0])
    _say("[gpu] stencil vs general path")
    a, ma, _ = run(torch_mod, ctx, sensors, raws, params, stencil=True)
    b, mb, _ = run(torch_mod, ctx, sensors, raws, params, stencil=False)
    p, mp, _ = run(torch_mod, ctx, sensors, raws, params, stencil=True, plain=True)
    assert np.array_equal(a, p, equal_nan=True) and np.array_equal(ma, mp)
    orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
    firm = firm_mask(orc, 2, sensors).reshape(96, 96, 3)
    assert np.array_equal(ma[firm], mb[firm])
    both = firm & np.isfinite(a) & np.isfinite(b)
    rel = np.abs(a[both] - b[both]) / np.maximum(np.abs(b[both]), 2.0)
    _say(f"  stencil vs general: max rel {rel.max():.2e}, median {np.median(rel):.2e}")
    assert np.median(rel) < 1e-5


def test_tables_cached_per_parameter_class(torch_mod, ctx):
    """One rig, three parameter classes in turn (the first again last): each
    result equals that of a fresh rig (a table built for that class alone)."""
    from paper_1308_4908_amd import Rig

    sensors = translation_rig(3, 64, 7500)
    scene = EdgeScene(64, 64, 7500, n_lines=6)
    raws = configs.capture_all(scene, sensors, 7500)
    classes = [configs.lpa_params(64, 64, 2, [1.0, 2.0, 3.0]),
               configs.lpa_params(64, 64, 1, [2.0], out_affine=[1, 0, 0.5, 0, 1, -0.25]),
               configs.lpa_params(64, 64, 2, [1.5, 3.0], green_ratio=0.9)]
    _say("[gpu] stencil table cache")
    fresh = [run(torch_mod, ctx, sensors, raws, p) for p in classes]
    rig = Rig(ctx, sensors)
    for i in (0, 1, 2, 0):
        got = run(torch_mod, ctx, sensors, raws, classes[i], rig=rig)
        assert np.array_equal(got[0], fresh[i][0], equal_nan=True), i
        assert np.array_equal(got[1], fresh[i][1]), i
    rig.close()


def test_full_size_sampled(torch_mod, ctx):
    """4 x 2048^2 aligned rig, order 2, ICI {1,2,3,4} (the benchmark's
    pre-computed-weight leg): sampled pixels against the oracle."""
    from test_gpu_parity import sample_pixels

    sensors, scene, params = configs.aligned()
    _say("[gpu] generating 4 x 2048^2 aligned frame")
    raws = configs.capture_all(scene, sensors, 2000)
    _say("[gpu] stencil full-size run")
    rgb, smap, sd = run(torch_mod, ctx, sensors, raws, params)
    pix = sample_pixels(2048, 2048, 1500, 78)
    orc = oracle.reconstruct(sensors, raws, params, pixels=pix, want_fits=True)
    st = compare(rgb[pix[:, 1], pix[:, 0]], smap[pix[:, 1], pix[:, 0]], orc, sensors, 2,
                 gpu_sd=sd[pix[:, 1], pix[:, 0]])
    _say(f"  stats {st}")
    assert st["agree_frac"] > 0.999
    assert not np.any(rgb == -12345.0)
    assert not np.any(smap == 0xEE)


def test_refused_where_not_applicable(torch_mod, ctx):
    from paper_1308_4908_amd import LpaError, Rig, lpa

    sensors = translation_rig(3, 32, 7600)
    scene = EdgeScene(32, 32, 7600, n_lines=4)
    raws = configs.capture_all(scene, sensors, 7600)
    p = configs.lpa_params(32, 32, 2, [1.0, 2.0], precomputed_weights=True)
    dev = [torch_mod.from_numpy(r).cuda() for r in raws]
    out = torch_mod.full((32, 32, 3), 7.0, device="cuda")
    _say("[gpu] stencil refusals")

    def refused(fn, status=lpa.ERR_UNSUPPORTED):
        with pytest.raises(LpaError) as e:
            fn()
        assert e.value.status == status

    rig = Rig(ctx, sensors)
    # output map with a scale, or rotated
    refused(lambda: rig.reconstruct(dev, dict(p, out_affine=[0.5, 0, 0, 0, 0.5, 0]), out))
    refused(lambda: rig.reconstruct(dev, dict(p, out_affine=[0.0, -1.0, 31.0, 1.0, 0.0, 0.0]), out))
    # CALPA
    refused(lambda: rig.reconstruct(dev, dict(p, mode="calpa", adapt={}), out))
    # batches, serving, tuning
    refused(lambda: ctx.reconstruct_batch([rig], [dev], [p], [out]))
    refused(lambda: rig.submit([torch_mod.from_numpy(r) for r in raws], p, out, host=True))
    refused(lambda: rig.autotune(dev, p, out, reps=1))
    rig.close()
    # a rotated sensor
    rot = [dict(sensors[0], affine=R.rotation_affine(32, 32, 0.5, 0.3, 0.2))] + sensors[1:]
    rig2 = Rig(ctx, rot)
    refused(lambda: rig2.reconstruct(dev, p, out))
    rig2.close()
    torch_mod.cuda.synchronize()
    assert torch_mod.all(out == 7.0)


@pytest.mark.parametrize("cfa", ["GRBG", "BGGR"])
def test_other_cfa_layouts_and_odd_sizes(torch_mod, ctx, cfa):
    """The tables take each sensor's sub-lattice parities from its CFA; odd
    sensor and output sizes leave ragged tiles on both axes."""
    sensors = [dict(s, cfa=cfa) for s in translation_rig(3, 77, 7700)]
    sensors = [dict(s, height=59) for s in sensors]
    scene = EdgeScene(77, 59, 7700, n_lines=8)
    raws = configs.capture_all(scene, sensors, 7700)
    params = configs.lpa_params(75, 57, 2, [1.0, 2.0, 3.0], out_affine=[1, 0, 1.0, 0, 1, 1.0])
    _say(f"[gpu] stencil cfa={cfa} odd sizes")
    rgb, smap, sd = run(torch_mod, ctx, sensors, raws, params)
    orc = oracle.reconstruct(sensors, raws, params, want_fits=True)
    st = compare(rgb, smap, orc, sensors, 2, gpu_sd=sd)
    _say(f"  stats {st}")
    assert st["agree_frac"] > 0.999
