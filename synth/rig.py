"""Seeded synthetic multi-sensor rigs and raw captures.

The forward image-formation model: N_s sensors see one scene through a common
lens; sensor s samples the scene at X = T_s(x) through a Bayer CFA with
exposure scale n_s, collects Poisson photo-electrons, applies gain g_s, adds
Gaussian readout noise and a black level, rounds and clips to the ADC range.
This is the model the reconstruction inverts; nothing here performs any of the
reconstruction's arithmetic.

A sensor is described by a plain dict with keys
  width, height, cfa ('RGGB' | 'BGGR' | 'GRBG' | 'GBRG'), affine (6 floats:
  X = a0 x + a1 y + a2, Y = a3 x + a4 y + a5 for pixel centre (x = col, y = row)),
  exposure, gain [DN/e-], read_sigma [DN], black_level [DN], saturation [DN],
  bit_depth.
"""
from __future__ import annotations

import math

import numpy as np

# Colour (0 R, 1 G, 2 B) of the 2x2 CFA cell, indexed [row parity][col parity].
_CFA_LAYOUT = {
    "RGGB": ((0, 1), (1, 2)),
    "BGGR": ((2, 1), (1, 0)),
    "GRBG": ((1, 0), (2, 1)),
    "GBRG": ((1, 2), (0, 1)),
}


def cfa_channels(cfa: str, height: int, width: int) -> np.ndarray:
    lay = np.asarray(_CFA_LAYOUT[cfa], np.int64)
    rows = np.arange(height)[:, None] & 1
    cols = np.arange(width)[None, :] & 1
    return lay[rows, cols]


def rotation_affine(width: int, height: int, theta_deg: float, tx: float, ty: float):
    """Rotation by theta about the sensor centre followed by a translation."""
    th = math.radians(theta_deg)
    c, s = math.cos(th), math.sin(th)
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    return [c, -s, cx - (c * cx - s * cy) + tx, s, c, cy - (s * cx + c * cy) + ty]


def make_sensor(width, height, affine, exposure, gain=0.5, read_sigma=3.0, black_level=64.0,
                saturation=4095.0, bit_depth=12, cfa="RGGB") -> dict:
    return {
        "width": int(width), "height": int(height), "cfa": cfa,
        "affine": [float(a) for a in affine], "exposure": float(exposure), "gain": float(gain),
        "read_sigma": float(read_sigma), "black_level": float(black_level),
        "saturation": float(saturation), "bit_depth": int(bit_depth),
    }


def random_rig(n_sensors, width, height, exposures, max_shift, max_rot_deg, seed, **noise):
    """Sensors misregistered by uniform translation in [-max_shift, max_shift]^2 and
    rotation in [-max_rot_deg, max_rot_deg] about the sensor centre."""
    rig = []
    for s in range(n_sensors):
        rng = np.random.default_rng(np.random.SeedSequence([int(seed), 1, s]))
        tx, ty = rng.uniform(-max_shift, max_shift, 2)
        th = rng.uniform(-max_rot_deg, max_rot_deg)
        rig.append(make_sensor(width, height, rotation_affine(width, height, th, tx, ty),
                               exposures[s], **noise))
    return rig


def sample_positions(sensor: dict, rows=None):
    """Reference-plane positions (X, Y) of every pixel centre (or of a row range)."""
    h, w = sensor["height"], sensor["width"]
    r0, r1 = (0, h) if rows is None else rows
    y, x = np.mgrid[r0:r1, 0:w].astype(np.float64)
    a = sensor["affine"]
    return a[0] * x + a[1] * y + a[2], a[3] * x + a[4] * y + a[5]


def _channel_radiance(scene, sensor, rows):
    X, Y = sample_positions(sensor, rows)
    ch = cfa_channels(sensor["cfa"], sensor["height"], sensor["width"])[rows[0]:rows[1]]
    return scene.radiance(X, Y, ch)


def capture(scene, sensor: dict, seed, chunk_rows: int = 256) -> np.ndarray:
    """Noisy raw frame (uint16): e ~ Poisson(n f), y = round(g e + N(0, s_r^2) + b),
    clipped to [0, 2^bits - 1]."""
    h, w = sensor["height"], sensor["width"]
    out = np.empty((h, w), np.uint16)
    key = [int(k) for k in (seed if isinstance(seed, (tuple, list)) else (seed,))]
    rng = np.random.default_rng(np.random.SeedSequence(key + [2]))
    top = 2 ** sensor["bit_depth"] - 1
    for r0 in range(0, h, chunk_rows):
        r1 = min(h, r0 + chunk_rows)
        f = _channel_radiance(scene, sensor, (r0, r1))
        e = rng.poisson(sensor["exposure"] * f)
        y = sensor["gain"] * e + rng.normal(0.0, sensor["read_sigma"], e.shape) + sensor["black_level"]
        out[r0:r1] = np.clip(np.floor(y + 0.5), 0, top).astype(np.uint16)
    return out


def capture_noise_free(scene, sensor: dict) -> np.ndarray:
    """Noise-free frame as float32 DN: y = g n f + b (values >= saturation are
    left as they are; the reconstruction masks them)."""
    h = sensor["height"]
    f = _channel_radiance(scene, sensor, (0, h))
    return (sensor["gain"] * sensor["exposure"] * f + sensor["black_level"]).astype(np.float32)


def capture_noise_free_f64(scene, sensor: dict) -> np.ndarray:
    """As capture_noise_free, in float64 (for oracle-only exactness pins)."""
    h = sensor["height"]
    f = _channel_radiance(scene, sensor, (0, h))
    return sensor["gain"] * sensor["exposure"] * f + sensor["black_level"]


def identity_output(width: int, height: int) -> list:
    return [1.0, 0.0, 0.0, 0.0, 1.0, 0.0]


def resample_output(scale: float) -> list:
    """Centre-aligned resampling: output pixel (u, v) sits at ((u + 1/2) / scale - 1/2, ...)."""
    return [1.0 / scale, 0.0, 0.5 / scale - 0.5, 0.0, 1.0 / scale, 0.5 / scale - 0.5]


def capture_float_noisy(scene, sensor: dict, seed) -> np.ndarray:
    """Noisy frame without ADC rounding or clipping (float64 DN):
    y = g Poisson(n f) + N(0, s_r^2) + b.  Used for Monte-Carlo checks of the
    noise model, where quantisation would add a variance the model omits."""
    key = [int(k) for k in (seed if isinstance(seed, (tuple, list)) else (seed,))]
    rng = np.random.default_rng(np.random.SeedSequence(key + [3]))
    h = sensor["height"]
    f = _channel_radiance(scene, sensor, (0, h))
    e = rng.poisson(sensor["exposure"] * f)
    return sensor["gain"] * e + rng.normal(0.0, sensor["read_sigma"], e.shape) + sensor["black_level"]
