"""Pins of the oracle's per-pixel calibration frames (Sec. 6: bias frame b_i,
photo-response non-uniformity a_i, per-pixel readout variance, saturation
frame; plus a defect mask).  Each pin is fixed by something other than the
oracle's own formula:

- frames holding the sensor's scalars reproduce the scalar model exactly;
- a noise-free constant scene captured through random per-pixel a_i and b_i
  (non-square sensors, so transposed indexing fails) gives f at every order
  and scale (closed form);
- Monte Carlo of the forward model (Poisson photo-electrons through a_i,
  Gaussian readout with per-pixel variance) against the variance estimate at
  the true signal;
- a sample at its saturation-frame level, a sample flagged in the defect mask
  and a sample above the scalar saturation are excluded alike (three routes
  to one support set).
"""
import numpy as np
import pytest

import oracle
from synth import configs, rig as R



def _sensor(w, h, affine, exposure, calib=None):
    s = R.make_sensor(w, h, affine, exposure)
    if calib is not None:
        s["calib"] = calib
    return s


def _rig(n=3, w=40, h=56, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        th = rng.uniform(-3, 3)
        tx, ty = rng.uniform(-1.5, 1.5, 2)
        out.append(_sensor(w, h, R.rotation_affine(w, h, th, tx, ty), [1.0, 0.25, 1 / 16][i]))
    return out


def _params(w, h, order, radii):
    return configs.lpa_params(w - 8, h - 8, order, radii, out_affine=[1, 0, 4, 0, 1, 4])


def test_uniform_frames_equal_scalars():
    sensors = _rig()
    rng = np.random.default_rng(3)
    raws = [np.round(rng.uniform(60, 4200, (56, 40))) for _ in sensors]
    p = _params(40, 56, 2, [1.5, 3.0])
    ref = oracle.reconstruct(sensors, raws, p)
    cal = [dict(s, calib={"bias": np.full((56, 40), s["black_level"]), "prnu": np.ones((56, 40)),
                          "read_var": np.full((56, 40), s["read_sigma"] ** 2),
                          "sat": np.full((56, 40), s["saturation"]), "defect": np.zeros((56, 40), np.uint8)})
           for s in sensors]
    got = oracle.reconstruct(cal, raws, p)
    assert np.array_equal(got["rgb"], ref["rgb"], equal_nan=True)
    assert np.array_equal(got["scale_map"], ref["scale_map"])


@pytest.mark.parametrize("order", [0, 1, 2])
def test_constant_scene_through_per_pixel_frames(order):
    """y_i = b_i + g t a_i n f: every sample's radiance estimate is f, so every
    valid fit returns f (non-square sensors: a transposed index breaks it)."""
    sensors = _rig(seed=21)
    rng = np.random.default_rng(22)
    f = 700.0
    cal, raws = [], []
    for s in sensors:
        a = rng.uniform(0.8, 1.25, (56, 40))
        b = rng.uniform(40, 90, (56, 40))
        y = b + s["gain"] * s["exposure"] * a * f
        cal.append(dict(s, calib={"bias": b, "prnu": a}))
        raws.append(y)
    p = _params(40, 56, order, [1.5, 2.5])
    got = oracle.reconstruct(cal, raws, p)
    ok = ~np.isnan(got["rgb"])
    assert ok.mean() > 0.99
    np.testing.assert_allclose(got["rgb"][ok], f, rtol=1e-11)
    # the same raw values read with the scalar model are not constant
    plain = oracle.reconstruct(sensors, raws, p)["rgb"]
    assert np.nanmax(np.abs(plain - f)) > 10.0


def test_variance_model_monte_carlo():
    """Forward model per pixel: e ~ Poisson(t a_i n f), y = g e + N(0, rv_i) + b_i.
    The empirical variance of the radiance estimate matches the oracle's
    variance estimate at the mean value, pixel by pixel (a_i and rv_i vary)."""
    rng = np.random.default_rng(5)
    w, h = 4, 2
    a = np.array([[0.7, 1.0, 1.3, 0.9], [1.1, 0.8, 1.2, 1.0]])
    rv = np.array([[100.0, 9.0, 400.0, 25.0], [1.0, 250.0, 64.0, 9.0]])
    b = np.array([[60.0, 64.0, 70.0, 55.0], [64.0, 80.0, 50.0, 62.0]])
    s = _sensor(w, h, [1, 0, 0, 0, 1, 0], 0.25, calib={"bias": b, "prnu": a, "read_var": rv})
    f = 180.0
    n_draw = 20000
    for iy in range(h):
        for ix in range(w):
            e = rng.poisson(s["exposure"] * a[iy, ix] * f, n_draw)
            y = s["gain"] * e + rng.normal(0.0, np.sqrt(rv[iy, ix]), n_draw) + b[iy, ix]
            _, fh, _ = oracle.sample_radiance_at(s, ix, iy, y)  # the oracle's own estimate per draw
            assert abs(np.mean(fh) / f - 1.0) < 5 * np.std(fh) / f / np.sqrt(n_draw)
            y_mean = s["gain"] * s["exposure"] * a[iy, ix] * f + b[iy, ix]
            ok, fm, var_model = oracle.sample_radiance_at(s, ix, iy, y_mean)
            assert ok and abs(fm - f) < 1e-9
            # chi-square band: relative standard error of a sample variance is sqrt(2/n)
            assert abs(np.var(fh) / var_model - 1.0) < 5 * np.sqrt(2.0 / n_draw), (ix, iy)


def test_saturation_frame_defects_and_scalar_saturation_agree():
    """Three ways to exclude the same samples give the same reconstruction."""
    sensors = _rig(seed=31)
    rng = np.random.default_rng(32)
    raws = [np.round(rng.uniform(100, 3000, (56, 40))) for _ in sensors]
    hit = [rng.random((56, 40)) < 0.1 for _ in sensors]
    p = _params(40, 56, 1, [1.5, 2.5])
    via_sat = oracle.reconstruct([dict(s, calib={"sat": np.where(m, r, 4095.0)})
                                  for s, m, r in zip(sensors, hit, raws)], raws, p)
    via_defect = oracle.reconstruct([dict(s, calib={"defect": m.astype(np.uint8)}) for s, m in zip(sensors, hit)],
                                    raws, p)
    via_scalar = oracle.reconstruct(sensors, [np.where(m, 4095.0, r) for m, r in zip(hit, raws)], p)
    for other in (via_defect, via_scalar):
        assert np.array_equal(via_sat["rgb"], other["rgb"], equal_nan=True)
        assert np.array_equal(via_sat["scale_map"], other["scale_map"])
    # and it is not the unmasked reconstruction
    plain = oracle.reconstruct(sensors, raws, p)
    assert not np.array_equal(plain["rgb"], via_sat["rgb"], equal_nan=True)


def test_invalid_frames_rejected():
    s = _rig(n=1)[0]
    raws = [np.full((56, 40), 500.0)]
    p = _params(40, 56, 0, [2.0])
    for bad in ({"prnu": np.zeros((56, 40))}, {"read_var": np.full((56, 40), -1.0)},
                {"bias": np.full((56, 40), np.nan)}):
        with pytest.raises(ValueError):
            oracle.reconstruct([dict(s, calib=bad)], raws, p)
