"""Adaptive anisotropic LPA with colour-channel correlation (CALPA, Sec. 5.4,
5.5) on the GPU, stage by stage against the FP64 oracle:

1. gradient pass: the G-channel gradient of every output pixel against the
   oracle's gradients (the pass accumulates in FP64: only its FP32 inputs differ);
2. steering pass: the steering matrices against the oracle's steering of the
   GPU's own gradient plane (identical inputs: FP64 arithmetic on both sides,
   FP32 storage);
3. steered fit: values, codes and standard deviations against the oracle's
   steered reconstruction fed the GPU's steering matrices, with the same metric
   and tolerances as the isotropic fit (``parity_utils``).

Plus: with the stretch bound at 1 every steering matrix is the identity and
CALPA reproduces LPA bit for bit; batches, serving and the tuner refuse CALPA.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import configs
from synth.scene import EdgeScene
from parity_utils import compare, floor_of

pytestmark = pytest.mark.gpu

ADAPT = {"alpha": 0.2, "lambda1": 1.0, "lambda2": 0.001, "grad_radius": 2.0, "grad_order": 1,
         "grad_halfwin": 2, "max_stretch": 2.0}


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


def _case(size=96, seed=2300, order=2, w=None, h=None, out_affine=None):
    sensors = configs.full_rig(seed=seed, size=size)
    scene = EdgeScene(size, size, seed, n_lines=12)
    raws = configs.capture_all(scene, sensors, seed)
    w = w or size
    h = h or size
    p = configs.lpa_params(w, h, order, [1.0, 2.0, 3.0, 4.0], out_affine=out_affine, mode="calpa",
                           adapt=dict(ADAPT))
    return sensors, raws, p


def run_calpa(torch, ctx, sensors, raws, p, plain=False):
    from paper_1308_4908_amd import Rig

    rig = Rig(ctx, sensors)
    dev = [torch.from_numpy(np.ascontiguousarray(r)).cuda() for r in raws]
    H, W = p["out_h"], p["out_w"]
    out = torch.full((H, W, 3), -12345.0, device="cuda")
    smap = torch.full((H, W, 3), 0xEE, dtype=torch.uint8, device="cuda")
    sd = torch.full((H, W, 3), -1.0, device="cuda")
    grad = torch.full((H, W, 2), -7.0, device="cuda")
    steer = torch.full((H, W, 4), -7.0, device="cuda")
    rig.reconstruct(dev, p, out, smap, plain=plain, sd_map=sd, grad_map=grad, steer_map=steer)
    torch.cuda.synchronize()
    res = {k: t.cpu().numpy() for k, t in (("rgb", out), ("map", smap), ("sd", sd), ("grad", grad),
                                          ("steer", steer))}
    rig.close()
    return res


@pytest.mark.parametrize("case", ["square", "ragged"])
def test_calpa_stages_match_oracle(torch_mod, ctx, case):
    if case == "square":
        sensors, raws, p = _case()
    else:
        sensors, raws, p = _case(w=37, h=23, out_affine=[1.0, 0.0, 20.5, 0.0, 1.0, 30.25])
    _say(f"[gpu] calpa stages case={case}")
    g = run_calpa(torch_mod, ctx, sensors, raws, p)
    H, W = p["out_h"], p["out_w"]
    adapt = p["adapt"]

    # 1. gradients
    og, ovalid = oracle.gradients(sensors, raws, p, adapt)
    gg = g["grad"].reshape(-1, 2).astype(np.float64)
    gvalid = np.any(gg != 0.0, axis=1)
    mismatch = np.mean(gvalid != (ovalid != 0))
    both = gvalid & (ovalid != 0)
    floor = floor_of(sensors) / 2.0  # one DN per reference pixel over the fit's half-width
    err = np.abs(gg[both] - og[both]).max(axis=1) / (np.abs(og[both]).max(axis=1) + floor)
    _say(f"  gradients: validity mismatch {mismatch:.4f}, rel err median {np.median(err):.2e} "
         f"p99.9 {np.quantile(err, 0.999):.2e}")
    # FP64 accumulation on both sides: only the FP32 inputs (sample values,
    # offsets, window weights) differ
    assert mismatch < 0.001
    assert err.max() < 1e-4

    # 2. steering from the GPU's gradient plane
    C = oracle.steering(p, adapt, g["grad"].astype(np.float64))
    gs = g["steer"].reshape(-1, 4)
    assert np.all(gs[:, 3] == 0.0)
    np.testing.assert_allclose(gs[:, :3], C, rtol=2e-6, atol=2e-6 * np.abs(C).max())

    # 3. steered fit fed the GPU's steering matrices
    Cg = gs[:, :3].astype(np.float64)
    orc = oracle.reconstruct_steered(sensors, raws, p, Cg, want_fits=True)
    st = compare(g["rgb"], g["map"], orc, sensors, p["order"], gpu_sd=g["sd"])
    _say(f"  steered fit {st}")
    assert st["agree_frac"] > 0.999
    # the windows really are anisotropic
    lam = np.linalg.eigvalsh(np.stack([np.stack([Cg[:, 0], Cg[:, 1]], -1), np.stack([Cg[:, 1], Cg[:, 2]], -1)], -2))
    assert (lam[:, 1] / lam[:, 0]).max() > 4.0


def test_calpa_end_to_end_matches_oracle(torch_mod, ctx):
    """The whole chain against the oracle's own chain (its FP64 gradients and
    steering).  The gradient pass accumulates in FP64, so the two chains'
    steering matrices agree to a few 1e-6 (asserted); what that difference
    does to a value is measured by the oracle's own last stage run on the
    GPU's steering matrices, and each value must meet the gate against one of
    the two oracle results (its decisions against the oracle's own chain)."""
    sensors, raws, p = _case(size=64, seed=2400)
    _say("[gpu] calpa end to end")
    g = run_calpa(torch_mod, ctx, sensors, raws, p)
    orc = oracle.reconstruct_adaptive(sensors, raws, p, p["adapt"], want_fits=True, want_stages=True)
    Cg = g["steer"].reshape(-1, 4)[:, :3].astype(np.float64)
    assert np.abs(Cg - orc["C"]).max() < 1e-5 * np.abs(orc["C"]).max()
    orc_g = oracle.reconstruct_steered(sensors, raws, p, Cg, want_fits=True)
    st = compare(g["rgb"], g["map"], orc, sensors, p["order"], gpu_sd=g["sd"], alt_orc=orc_g)
    _say(f"  end to end {st}")
    assert st["agree_frac"] > 0.999


def test_calpa_with_unit_stretch_is_lpa(torch_mod, ctx):
    """max_stretch = 1 clamps both eigenvalues to 1: C = I exactly, and the
    steered fit reproduces the isotropic one bit for bit."""
    sensors, raws, p = _case(size=64, seed=2500)
    p["adapt"]["max_stretch"] = 1.0
    _say("[gpu] calpa with unit stretch vs lpa")
    g = run_calpa(torch_mod, ctx, sensors, raws, p)
    assert np.all(g["steer"][..., 0] == 1.0) and np.all(g["steer"][..., 1] == 0.0) and np.all(g["steer"][..., 2] == 1.0)
    from paper_1308_4908_amd import Rig

    rig = Rig(ctx, sensors)
    dev = [torch_mod.from_numpy(r).cuda() for r in raws]
    out = torch_mod.empty((64, 64, 3), device="cuda")
    smap = torch_mod.empty((64, 64, 3), dtype=torch_mod.uint8, device="cuda")
    lp = dict(p, mode="lpa")
    lp.pop("adapt")
    rig.reconstruct(dev, lp, out, smap)
    torch_mod.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), g["rgb"], equal_nan=True)
    assert np.array_equal(smap.cpu().numpy(), g["map"])
    rig.close()


def test_calpa_plain_and_fp16_forms(torch_mod, ctx):
    """Every storage form runs the three passes: the plain form (FP32 planes)
    equals the fused one bit for bit; FP16 storage stays within its rounding."""
    sensors, raws, p = _case(size=48, seed=2600)
    _say("[gpu] calpa plain / fp16")
    a = run_calpa(torch_mod, ctx, sensors, raws, p)
    b = run_calpa(torch_mod, ctx, sensors, raws, p, plain=True)
    assert np.array_equal(a["rgb"], b["rgb"], equal_nan=True)
    assert np.array_equal(a["steer"], b["steer"])
    c = run_calpa(torch_mod, ctx, sensors, raws, dict(p, storage="fp16"))
    fin = np.isfinite(a["rgb"]) & np.isfinite(c["rgb"])
    rel = np.abs(c["rgb"][fin] - a["rgb"][fin]) / np.maximum(np.abs(a["rgb"][fin]), floor_of(sensors))
    assert np.median(rel) < 1e-3


def test_calpa_refused_where_unsupported(torch_mod, ctx):
    from paper_1308_4908_amd import Rig, lpa

    sensors, raws, p = _case(size=32, seed=2700)
    rig = Rig(ctx, sensors)
    dev = [torch_mod.from_numpy(r).cuda() for r in raws]
    out = torch_mod.empty((32, 32, 3), device="cuda")
    with pytest.raises(lpa.LpaError) as e:
        ctx.reconstruct_batch([rig], [dev], [p], [out])
    assert e.value.status == lpa.ERR_UNSUPPORTED
    with pytest.raises(lpa.LpaError) as e:
        rig.autotune(dev, p, out, reps=1)
    assert e.value.status == lpa.ERR_UNSUPPORTED
    with pytest.raises(lpa.LpaError) as e:
        rig.submit([torch_mod.from_numpy(r) for r in raws], p, out, host=True)
    assert e.value.status == lpa.ERR_UNSUPPORTED
    bad = dict(p, adapt=dict(p["adapt"], max_stretch=0.5))
    with pytest.raises(lpa.LpaError) as e:
        rig.reconstruct(dev, bad, out)
    assert e.value.status == lpa.ERR_INVALID_ARG
    rig.close()
