"""Pins of the oracle's temporal LPA (readings T1-T4 in oracle/lpa_oracle.h;
Sec. 9 names the extension of the supports to time as future work).

  * one frame, or any number of frames with h_t = 0, is the spatial
    reconstruction bit for bit;
  * K copies of one frame: the moments scale by sum_t K_t, so every fit's C0
    and pivot ratio equal the spatial ones, its support is K times larger and
    its variance scales by (sum_t K_t^2) / (sum_t K_t)^2 (closed form);
  * distinct frames: every fit equals a brute-force weighted least squares
    (numpy lstsq / pinv) on the pooled sample set with weights
    K_s(d) K_t(t) / sigma^2;
  * the box scan equals the exhaustive scan.
"""
import math

import numpy as np
import pytest

import oracle
from synth import rig as R
from synth.scene import EdgeScene


def _rig(seed, size=14, n=2):
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n):
        th = rng.uniform(-1.0, 1.0)
        tx, ty = rng.uniform(-1.0, 1.0, 2)
        out.append(R.make_sensor(size, size, R.rotation_affine(size, size, th, tx, ty), [1.0, 1 / 8, 1 / 64][s],
                                 gain=0.5, read_sigma=3.0, black_level=64.0, saturation=4095.0))
    return out


def _params(size, order, radii, h_t, **kw):
    p = {"out_w": size, "out_h": size, "out_affine": [1, 0, 0, 0, 1, 0], "order": order,
         "radii": list(radii), "h": [0.0] * len(radii), "gamma": 2.0, "green_ratio": 1.0, "tau_inv": 1e-5,
         "h_t": list(h_t)}
    p.update(kw)
    return p


def _frames(sensors, scene, n_times, seed):
    return [[R.capture(scene, s, (seed, t, i)) for i, s in enumerate(sensors)] for t in range(n_times)]


PIX = np.array([[4, 5], [6, 6], [7, 4], [5, 8], [9, 9]], np.int32)


@pytest.mark.parametrize("order", [0, 1, 2])
def test_single_frame_and_zero_temporal_scale_are_spatial(order):
    sensors = _rig(300 + order)
    scene = EdgeScene(14, 14, 31 + order, n_lines=3)
    frames = _frames(sensors, scene, 3, 5)
    params = _params(14, order, [1.5, 2.5], [0.0, 0.0])
    ref = oracle.reconstruct(sensors, frames[0], params, want_fits=True)
    for fr in (frames[:1], frames):
        got = oracle.reconstruct_temporal(sensors, fr, params, want_fits=True)
        assert np.array_equal(got["rgb"], ref["rgb"], equal_nan=True)
        assert np.array_equal(got["scale_map"], ref["scale_map"])
        for f in ("yhat", "var", "rho", "n"):
            assert np.array_equal(got["fits"][f], ref["fits"][f], equal_nan=True)


@pytest.mark.parametrize("order", [0, 1, 2])
def test_repeated_frame_scales_the_moments(order):
    sensors = _rig(310 + order)
    scene = EdgeScene(14, 14, 41 + order, n_lines=3)
    frame = _frames(sensors, scene, 1, 6)[0]
    K = 4
    h_t = [1.5, 6.0]
    params = _params(14, order, [1.5, 2.5], h_t)
    ref = oracle.reconstruct(sensors, frame, params, pixels=PIX, want_fits=True)
    got = oracle.reconstruct_temporal(sensors, [frame] * K, params, pixels=PIX, want_fits=True)
    for m, ht in enumerate(h_t):
        kt = np.exp(-np.arange(K) ** 2 / ht)
        ratio = np.sum(kt * kt) / np.sum(kt) ** 2
        for o in range(order + 1):
            a, b = got["fits"][:, :, m, o], ref["fits"][:, :, m, o]
            assert np.array_equal(a["n"], K * b["n"])
            ok = b["valid"] == 1
            assert np.array_equal(a["valid"][ok], b["valid"][ok])
            np.testing.assert_allclose(a["yhat"][ok], b["yhat"][ok], rtol=1e-10, atol=1e-9)
            np.testing.assert_allclose(a["rho"][ok], b["rho"][ok], rtol=1e-9)
            np.testing.assert_allclose(a["var"][ok], b["var"][ok] * ratio, rtol=1e-9)


def _pooled_support(sensors, frames, X, Y, c, r, h, h_t):
    rows = []
    for t, raws in enumerate(frames):
        kt = 1.0 if t == 0 else (math.exp(-t * t / h_t) if h_t > 0 else 0.0)
        if kt == 0.0:
            continue
        for s, raw in zip(sensors, raws):
            chan = R.cfa_channels(s["cfa"], s["height"], s["width"])
            Xs, Ys = R.sample_positions(s)
            d2 = (Xs - X) ** 2 + (Ys - Y) ** 2
            ok = (chan == c) & (raw < s["saturation"]) & (d2 < r * r)
            for yy, xx in zip(*np.nonzero(ok)):
                g, e = s["gain"], s["exposure"]
                fh = (float(raw[yy, xx]) - s["black_level"]) / (g * e)
                var = (g * g * e * max(fh, 0.0) + s["read_sigma"] ** 2) / (g * g * e * e)
                k = (math.exp(-d2[yy, xx] / h) - math.exp(-r * r / h)) * kt
                rows.append((Xs[yy, xx] - X, Ys[yy, xx] - Y, fh, var, k))
    return np.array(rows)


@pytest.mark.parametrize("order", [0, 1, 2])
def test_bruteforce_pooled_lstsq(order):
    sensors = _rig(320 + order)
    scene = EdgeScene(14, 14, 51 + order, n_lines=3)
    frames = _frames(sensors, scene, 3, 7)
    radii, h_t = [2.0, 3.0], [0.8, 3.0]
    params = _params(14, order, radii, h_t)
    res = oracle.reconstruct_temporal(sensors, frames, params, pixels=PIX, want_fits=True)
    n = {0: 1, 1: 3, 2: 6}[order]
    checked = 0
    for p, (u, v) in enumerate(PIX):
        for c in range(3):
            for m, r in enumerate(radii):
                S = _pooled_support(sensors, frames, float(u), float(v), c, r, 2 * r * r / 9, h_t[m])
                fit = res["fits"][p, c, m, order]
                assert fit["n"] == len(S)
                if not fit["valid"]:
                    continue
                dx, dy, fh, var, k = S.T
                Phi = np.stack([np.ones_like(dx), dx, dy, dx * dx, dx * dy, dy * dy], 1)[:, :n]
                sw = np.sqrt(k / var)
                C, *_ = np.linalg.lstsq(Phi * sw[:, None], fh * sw, rcond=None)
                a = np.linalg.pinv(Phi * sw[:, None])[0] * sw
                assert fit["yhat"] == pytest.approx(C[0], rel=1e-9, abs=1e-9)
                assert fit["var"] == pytest.approx(np.sum(a * a * var), rel=1e-8)
                checked += 1
    assert checked >= 15


def test_box_scan_equals_exhaustive_scan():
    sensors = _rig(330)
    scene = EdgeScene(14, 14, 61, n_lines=3)
    frames = _frames(sensors, scene, 3, 8)
    params = _params(14, 2, [1.0, 2.0, 3.0], [0.5, 2.0, 8.0])
    a = oracle.reconstruct_temporal(sensors, frames, params, want_fits=True)
    b = oracle.reconstruct_temporal(sensors, frames, params, want_fits=True, exhaustive=True)
    assert np.array_equal(a["rgb"], b["rgb"], equal_nan=True)
    assert np.array_equal(a["fits"]["n"], b["fits"]["n"])
