"""The five synthetic workloads (rig, scene, LPA parameters), seeded.

small      3 x 256^2 raw, exposures 1, 1/8, 1/64, +-1.5 px / +-0.2 deg, order 1,
           one radius 2, output 256^2 identity, FP32 storage.
full       4 x 2048^2 raw, exposures 1, 1/4, 1/16, 1/64, +-2 px / +-0.3 deg,
           order 2, ICI radii {1,2,3,4}, Gamma 2, output 2048^2 identity.
resampled  the small rig, output 4096^2 with X = (u + 1/2)/16 - 1/2, FP16 storage.
batch      64 frames of mixed size / sensor count / order (see batch_frames).
served     8 cameras, fixed rig per camera (see camera_rigs).
aligned    the full workload's rig without rotation (translation-only sensor
           maps), for the pre-computed-weight form.

Noise for all: gain 0.5 DN/e-, readout sigma 3 DN, black 64, saturation 4095,
12-bit RGGB.  These stand in for the paper's four-sensor KAI-04050 rig
(2336 x 1752, 12 bit, exposures a few f-stops apart, misregistration of a few
pixels and fractions of a degree); its scenes and captured video are not
available.
"""
from __future__ import annotations

import numpy as np

from . import rig as _rig
from .scene import EdgeScene

NOISE = dict(gain=0.5, read_sigma=3.0, black_level=64.0, saturation=4095.0, bit_depth=12, cfa="RGGB")


def lpa_params(out_w, out_h, order, radii, out_affine=None, gamma=2.0, storage="fused", **kw):
    p = {
        "out_w": int(out_w), "out_h": int(out_h),
        "out_affine": list(out_affine) if out_affine is not None else _rig.identity_output(out_w, out_h),
        "order": int(order), "radii": [float(r) for r in radii], "h": [0.0] * len(radii),
        "gamma": float(gamma), "green_ratio": 1.0, "tau_inv": 1e-5, "tau_fp64": 1e-3,
        "storage": storage,
    }
    p.update(kw)
    return p


def small_rig(seed=1000, size=256):
    return _rig.random_rig(3, size, size, [1.0, 1.0 / 8, 1.0 / 64], 1.5, 0.2, seed, **NOISE)


def full_rig(seed=2000, size=2048):
    return _rig.random_rig(4, size, size, [1.0, 1.0 / 4, 1.0 / 16, 1.0 / 64], 2.0, 0.3, seed, **NOISE)


def aligned_rig(seed=2000, size=2048, n_sensors=4):
    """The full rig's exposures and translations without rotation (registered
    sensors, e.g. behind a beam splitter): every sensor map is a translation."""
    return _rig.random_rig(n_sensors, size, size, [1.0, 1.0 / 4, 1.0 / 16, 1.0 / 64][:n_sensors], 2.0, 0.0, seed,
                           **NOISE)


def aligned(seed=2000, size=2048, storage="fused"):
    """(sensors, scene, params) of the 4-sensor order-2 ICI workload on the aligned rig."""
    sensors = aligned_rig(seed, size)
    scene = EdgeScene(size, size, seed)
    return sensors, scene, lpa_params(size, size, 2, [1.0, 2.0, 3.0, 4.0], storage=storage)


def small(seed=1000, size=256):
    """(sensors, scene, params) of the small single-scale order-1 workload."""
    sensors = small_rig(seed, size)
    scene = EdgeScene(size, size, seed)
    return sensors, scene, lpa_params(size, size, 1, [2.0])


def full(seed=2000, size=2048, storage="fused"):
    """(sensors, scene, params) of the 4-sensor order-2 ICI workload."""
    sensors = full_rig(seed, size)
    scene = EdgeScene(size, size, seed)
    return sensors, scene, lpa_params(size, size, 2, [1.0, 2.0, 3.0, 4.0], storage=storage)


def resampled(seed=3000, size=256, scale=16):
    sensors = small_rig(seed, size)
    scene = EdgeScene(size, size, seed)
    return sensors, scene, lpa_params(size * scale, size * scale, 1, [2.0],
                                      out_affine=_rig.resample_output(scale), storage="fp16")


def capture_all(scene, sensors, seed):
    return [_rig.capture(scene, s, (seed, i)) for i, s in enumerate(sensors)]


BATCH_SIZES = [(1280, 720), (1920, 1080), (2048, 2048)]


def batch_frame_spec(frame: int, base_seed=4000):
    """Spec of frame `frame` of the mixed batch: size, sensor count, exposure set, order."""
    rng = np.random.default_rng(np.random.SeedSequence([base_seed + frame, 7]))
    w, h = BATCH_SIZES[int(rng.integers(0, 3))]
    ns = int(rng.integers(2, 5))
    exps = [1.0]
    for _ in range(ns - 1):
        exps.append(exps[-1] * 2.0 ** -int(rng.integers(2, 7)))
    order = int(rng.integers(1, 3))
    return {"width": w, "height": h, "n_sensors": ns, "exposures": exps, "order": order,
            "seed": base_seed + frame}


def batch_frame(frame: int, base_seed=4000, storage="fp32", scene_seed=None):
    spec = batch_frame_spec(frame, base_seed)
    sensors = _rig.random_rig(spec["n_sensors"], spec["width"], spec["height"], spec["exposures"],
                              2.0, 0.3, spec["seed"], **NOISE)
    scene = EdgeScene(spec["width"], spec["height"], spec["seed"] if scene_seed is None else scene_seed)
    params = lpa_params(spec["width"], spec["height"], spec["order"], [1.0, 2.0, 3.0, 4.0],
                        storage=storage)
    return sensors, scene, params


CAMERA_SIZES = [(1920, 1080), (2048, 2048)]


def camera_spec(camera: int):
    seed = 5000 + 100 * camera
    rng = np.random.default_rng(np.random.SeedSequence([seed, 9]))
    w, h = CAMERA_SIZES[int(rng.integers(0, 2))]
    ns = int(rng.integers(3, 5))
    exps = [1.0]
    for _ in range(ns - 1):
        exps.append(exps[-1] * 2.0 ** -int(rng.integers(2, 7)))
    return {"width": w, "height": h, "n_sensors": ns, "exposures": exps, "seed": seed}


def camera_rig(camera: int):
    spec = camera_spec(camera)
    sensors = _rig.random_rig(spec["n_sensors"], spec["width"], spec["height"], spec["exposures"],
                              2.0, 0.3, spec["seed"], **NOISE)
    params = lpa_params(spec["width"], spec["height"], 2, [1.0, 2.0, 3.0, 4.0], storage="fp16")
    return sensors, params, spec


def poisson_arrivals(camera: int, rate_hz: float = 30.0, duration_s: float = 60.0):
    """Arrival times (seconds) of a Poisson process: exponential gaps with mean 1/rate."""
    rng = np.random.default_rng(np.random.SeedSequence([5000 + 100 * camera, 11]))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            return np.asarray(out)
        out.append(t)
