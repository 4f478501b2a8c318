"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names the passage or property it pins.  None of them re-types the
oracle's own formulas as the expected value: expectations come from closed
forms, invariants, an independent least-squares routine (SVD), a textbook
demosaicing routine, Monte-Carlo statistics of the forward model, or worked
examples under tests/golden/.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
from synth import rig as R
from synth.scene import PolynomialScene, StepScene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _params(out_w, out_h, order, radii, out_affine=None, **kw):
    p = {"out_w": out_w, "out_h": out_h,
         "out_affine": out_affine or [1.0, 0.0, 0.0, 0.0, 1.0, 0.0],
         "order": order, "radii": list(radii), "gamma": 2.0, "green_ratio": 1.0, "tau_inv": 1e-5}
    p.update(kw)
    return p


def _affine(rng, scale_jitter=0.0, max_rot=3.0, max_shift=2.0):
    th = math.radians(rng.uniform(-max_rot, max_rot))
    sx, sy = 1.0 + rng.uniform(-scale_jitter, scale_jitter, 2)
    shear = rng.uniform(-scale_jitter, scale_jitter)
    c, s = math.cos(th), math.sin(th)
    A = np.array([[c, -s], [s, c]]) @ np.array([[sx, shear], [0.0, sy]])
    t = rng.uniform(-max_shift, max_shift, 2)
    return [A[0, 0], A[0, 1], t[0], A[1, 0], A[1, 1], t[1]]


def _sensor(w, h, affine, exposure, **kw):
    d = dict(gain=0.5, read_sigma=3.0, black_level=64.0, saturation=1e300, bit_depth=12, cfa="RGGB")
    d.update(kw)
    return R.make_sensor(w, h, affine, exposure, **d)


# --------------------------------------------------------------------------
# Polynomial reproduction (Sec. 5.1 / eq. wlsqe): an order-M fit reproduces any
# field of degree <= M exactly, for any positive weights and full-rank normal
# matrix.  Pins the basis, the transforms, the moment assembly and the solve.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("order", [0, 1, 2])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_polynomial_reproduction(order, seed):
    rng = np.random.default_rng(seed)
    coeffs = np.zeros((3, 6))
    nterm = {0: 1, 1: 3, 2: 6}[order]
    coeffs[:, 0] = rng.uniform(200, 400, 3)
    coeffs[:, 1:nterm] = rng.uniform(-3, 3, (3, nterm - 1)) / np.array([1, 1, 20, 20, 20])[: nterm - 1]
    scene = PolynomialScene(coeffs)
    size = 28
    sensors = [_sensor(size, size, _affine(rng, 0.05), e) for e in (1.0, 0.25, 1 / 16)]
    raws = [R.capture_noise_free_f64(scene, s) for s in sensors]
    out_aff = _affine(rng, 0.1, max_rot=10.0, max_shift=0.5)
    out_aff[2] += 8.0
    out_aff[5] += 8.0
    params = _params(10, 10, order, [2.5, 3.5])
    params["out_affine"] = out_aff
    res = oracle.reconstruct(sensors, raws, params, want_fits=True)
    u, v = np.meshgrid(np.arange(10.0), np.arange(10.0))
    X = out_aff[0] * u + out_aff[1] * v + out_aff[2]
    Y = out_aff[3] * u + out_aff[4] * v + out_aff[5]
    truth = np.stack([scene.radiance(X, Y, c) for c in range(3)], -1).reshape(-1, 3)
    assert np.all(res["scale_map"] >> 4 == order), "every pixel must be valid at the full order"
    np.testing.assert_allclose(res["rgb"], truth, rtol=1e-10, atol=0)
    if order >= 1:
        # C1 is the gradient of the field at X_j (Sec. 5.1) for every scale.
        c = coeffs
        gx = c[:, 1][None, :] + 2 * c[:, 3][None, :] * X.reshape(-1, 1) + c[:, 4][None, :] * Y.reshape(-1, 1)
        gy = c[:, 2][None, :] + c[:, 4][None, :] * X.reshape(-1, 1) + 2 * c[:, 5][None, :] * Y.reshape(-1, 1)
        fits = res["fits"][:, :, :, order]
        for m in range(2):
            np.testing.assert_allclose(fits["c1x"][:, :, m], gx, rtol=1e-8, atol=1e-9)
            np.testing.assert_allclose(fits["c1y"][:, :, m], gy, rtol=1e-8, atol=1e-9)


# --------------------------------------------------------------------------
# Constant scene through the uint16 path (Sec. 6 eq. Efsi): with g n_s f an
# integer for every sensor, the radiance estimate of every unmasked sample is
# exactly f, so the reconstruction is f at every order and scale, including
# where the brightest sensor saturates (masked, end of Sec. 6.1).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k,order", [(20, 0), (20, 1), (20, 2), (64, 1), (64, 2)])
def test_constant_scene_exact(k, order):
    f = 128.0 * k  # n = 1, 1/8, 1/64 and g = 0.5 give y - b = 64k, 8k, k
    rng = np.random.default_rng(7)
    sensors = [R.make_sensor(24, 24, _affine(rng, 0.0, 0.2, 1.5), e, saturation=4095.0)
               for e in (1.0, 1 / 8, 1 / 64)]
    raws = []
    for s in sensors:
        y = np.full((24, 24), s["black_level"] + s["gain"] * s["exposure"] * f)
        raws.append(np.clip(np.floor(y + 0.5), 0, 4095).astype(np.uint16))
    if k == 64:
        assert raws[0].min() == 4095  # the brightest sensor is fully saturated
    params = _params(12, 12, order, [2.0, 3.0], out_affine=[1, 0, 6, 0, 1, 6])
    res = oracle.reconstruct(sensors, raws, params)
    assert np.all(res["scale_map"] >> 4 == order)
    np.testing.assert_allclose(res["rgb"], f, rtol=1e-13)


# --------------------------------------------------------------------------
# Brute force with an independent least-squares routine: per (pixel, channel,
# scale) the support set is rebuilt here and C = argmin ||sqrt(W)(Phi C - f)||
# is solved by SVD (numpy lstsq); the variance of C0 is sum_k a_k^2 sigma_k^2
# with a = e0^T pinv(sqrt(W) Phi) sqrt(W).  Pins the normal-equation assembly,
# equilibration, Cholesky solve and the sandwich variance.
# --------------------------------------------------------------------------
def _support(sensors, raws, X, Y, c, r, h):
    rows = []
    for s, raw in zip(sensors, raws):
        chan = R.cfa_channels(s["cfa"], s["height"], s["width"])
        Xs, Ys = R.sample_positions(s)
        ok = (chan == c) & (raw < s["saturation"])
        d2 = (Xs - X) ** 2 + (Ys - Y) ** 2
        ok &= d2 < r * r
        for yy, xx in zip(*np.nonzero(ok)):
            g, e = s["gain"], s["exposure"]
            fh = (float(raw[yy, xx]) - s["black_level"]) / (g * e)
            var = (g * g * e * max(fh, 0.0) + s["read_sigma"] ** 2) / (g * g * e * e)
            k = math.exp(-d2[yy, xx] / h) - math.exp(-r * r / h)
            rows.append((Xs[yy, xx] - X, Ys[yy, xx] - Y, fh, var, k))
    return np.array(rows)


@pytest.mark.parametrize("order", [0, 1, 2])
def test_bruteforce_lstsq(order):
    rng = np.random.default_rng(11 + order)
    size = 12
    sensors = [_sensor(size, size, _affine(rng, 0.0, 1.0, 1.0), e, saturation=4095.0)
               for e in (1.0, 1 / 8)]
    from synth.scene import EdgeScene
    scene = EdgeScene(size, size, 5 + order, n_lines=3)
    raws = [R.capture(scene, s, (99, i)) for i, s in enumerate(sensors)]
    radii = [2.0, 3.0]
    params = _params(size, size, order, radii)
    pix = np.array([[4, 5], [6, 6], [7, 4], [5, 8]], np.int32)
    res = oracle.reconstruct(sensors, raws, params, pixels=pix, want_fits=True)
    n = {0: 1, 1: 3, 2: 6}[order]
    checked = 0
    for p, (u, v) in enumerate(pix):
        for c in range(3):
            for m, r in enumerate(radii):
                S = _support(sensors, raws, float(u), float(v), c, r, 2 * r * r / 9)
                fit = res["fits"][p, c, m, order]
                assert fit["n"] == len(S)
                if len(S) < n:
                    assert not fit["valid"]
                    continue
                dx, dy, fh, var, k = S.T
                Phi = np.stack([np.ones_like(dx), dx, dy, dx * dx, dx * dy, dy * dy], 1)[:, :n]
                sw = np.sqrt(k / var)
                C, *_ = np.linalg.lstsq(Phi * sw[:, None], fh * sw, rcond=None)
                a = np.linalg.pinv(Phi * sw[:, None])[0] * sw
                v_ref = np.sum(a * a * var)
                # smallest pivot of the Jacobi-equilibrated normal matrix (numpy Cholesky)
                A = (Phi * (k / var)[:, None]).T @ Phi
                dsc = 1.0 / np.sqrt(np.diag(A))
                try:
                    rho_ref = np.min(np.diag(np.linalg.cholesky(A * np.outer(dsc, dsc))) ** 2)
                except np.linalg.LinAlgError:
                    rho_ref = 0.0
                assert fit["rho"] == pytest.approx(rho_ref, rel=1e-6, abs=1e-9)
                if not fit["valid"]:
                    continue
                assert fit["yhat"] == pytest.approx(C[0], rel=1e-9, abs=1e-9)
                assert fit["var"] == pytest.approx(v_ref, rel=1e-8)
                checked += 1
    assert checked >= 12


# --------------------------------------------------------------------------
# Rounding-sensitivity diagnostics of a fit (Sec. 5.2, eq. (wlsqe) solved
# from moment sums), pinned by experiment rather than by their formulas:
#   l1f    = sum_k |a_k f_k| with a = e0^T pinv(sqrt(W) Phi) sqrt(W), the
#            equivalent-kernel weights from numpy's pseudo-inverse;
#   sens_y = the first-order change of C0 when every term of every moment sum
#            of A and b moves by a relative eps with the worst signs: the
#            perturbed systems are re-solved with numpy (central difference),
#            and random sign patterns must stay within eps sens_y;
#   sens_v = an upper bound of the same experiment on the variance g^T B g
#            (terms of A and B perturbed), attained for order 0.
# --------------------------------------------------------------------------
def _perturbed_terms(S, n):
    dx, dy, fh, var, k = S.T
    Phi = np.stack([np.ones_like(dx), dx, dy, dx * dx, dx * dy, dy * dy], 1)[:, :n]
    w = k / var
    tA = w[:, None, None] * Phi[:, :, None] * Phi[:, None, :]      # terms of A (k, i, j)
    tB = (k * k / var)[:, None, None] * Phi[:, :, None] * Phi[:, None, :]
    tb = (w * fh)[:, None] * Phi                                   # terms of b (k, i)
    return Phi, w, fh, tA, tB, tb


def _c0(tA, tb, dA, db):
    A = np.sum(tA * (1 + dA), 0)
    b = np.sum(tb * (1 + db), 0)
    return np.linalg.solve(A, b)[0]


def _var(tA, tB, dA, dB):
    A = np.sum(tA * (1 + dA), 0)
    B = np.sum(tB * (1 + dB), 0)
    g = np.linalg.solve(A, np.eye(A.shape[0])[0])
    return g @ B @ g


@pytest.mark.parametrize("order", [0, 1, 2])
def test_rounding_sensitivities(order):
    rng = np.random.default_rng(71 + order)
    size = 12
    sensors = [_sensor(size, size, _affine(rng, 0.0, 1.0, 1.0), e, saturation=4095.0) for e in (1.0, 1 / 8)]
    from synth.scene import EdgeScene
    scene = EdgeScene(size, size, 9 + order, n_lines=3)
    raws = [R.capture(scene, s, (77, i)) for i, s in enumerate(sensors)]
    radii = [2.0, 3.0]
    params = _params(size, size, order, radii)
    pix = np.array([[4, 5], [6, 6], [7, 4], [5, 7]], np.int32)
    res = oracle.reconstruct(sensors, raws, params, pixels=pix, want_fits=True)
    n = {0: 1, 1: 3, 2: 6}[order]
    eps = 1e-6
    checked = 0
    for p, (u, v) in enumerate(pix):
        for c in range(3):
            for m, r in enumerate(radii):
                fit = res["fits"][p, c, m, order]
                if not fit["valid"] or fit["rho"] < 1e-3:
                    continue
                S = _support(sensors, raws, float(u), float(v), c, r, 2 * r * r / 9)
                Phi, w, fh, tA, tB, tb = _perturbed_terms(S, n)
                sw = np.sqrt(w)
                a = np.linalg.pinv(Phi * sw[:, None])[0] * sw
                assert fit["l1f"] == pytest.approx(np.sum(np.abs(a * fh)), rel=1e-8)
                A = np.sum(tA, 0)
                g = np.linalg.solve(A, np.eye(n)[0])
                C = np.linalg.solve(A, np.sum(tb, 0))
                # C0: worst signs raise C0 by eps sens_y to first order
                db = np.sign(g[None, :] * tb)
                dA = -np.sign(g[None, :, None] * tA * C[None, None, :])
                slope = (_c0(tA, tb, eps * dA, eps * db) - _c0(tA, tb, -eps * dA, -eps * db)) / (2 * eps)
                assert slope == pytest.approx(fit["sens_y"], rel=1e-5)
                for _ in range(8):
                    rA = rng.choice([-1.0, 1.0], tA.shape)
                    rb = rng.choice([-1.0, 1.0], tb.shape)
                    dev = abs(_c0(tA, tb, eps * rA, eps * rb) - fit["yhat"]) / eps
                    assert dev <= fit["sens_y"] * (1 + 1e-4) + 1e-9 * abs(fit["yhat"]) / eps
                # variance: the worst signs of the exact first-order change
                Bm = np.sum(tB, 0)
                h = np.linalg.solve(A.T, Bm @ g)
                dB = np.sign(g[None, :, None] * tB * g[None, None, :])
                dA = -np.sign(h[None, :, None] * tA * g[None, None, :])
                slope_v = (_var(tA, tB, eps * dA, eps * dB) - _var(tA, tB, -eps * dA, -eps * dB)) / (2 * eps)
                assert slope_v <= fit["sens_v"] * (1 + 1e-5)
                if order == 0:
                    assert slope_v == pytest.approx(fit["sens_v"], rel=1e-5)
                else:
                    assert slope_v >= 0.05 * fit["sens_v"]
                checked += 1
    assert checked >= 8


# --------------------------------------------------------------------------
# Bilinear demosaicing special case: one aligned sensor, identity output,
# M = 0, r = 1.5 for R/B and r_G = 1.2 (kappa_G = 0.8), equal noise variances.
# The supports are then exactly the bilinear-interpolation neighbourhoods
# (distance 1 and sqrt 2 for R/B; distance 1 for G) with equal weights per
# distance class only within one class, so the estimate is the textbook
# bilinear demosaic.  Pins CFA handling and the pixel-centre convention.
# --------------------------------------------------------------------------
def test_bilinear_demosaic_special_case():
    rng = np.random.default_rng(3)
    size = 16
    s = _sensor(size, size, [1, 0, 0, 0, 1, 0], 1.0, gain=1.0, read_sigma=1e6, black_level=0.0)
    raw = rng.uniform(100.0, 1000.0, (size, size))
    params = _params(size, size, 0, [1.5], green_ratio=0.8)
    res = oracle.reconstruct([s], [raw], params)
    rgb = res["rgb"].reshape(size, size, 3)
    chan = R.cfa_channels("RGGB", size, size)
    k_rb = np.array([[1, 2, 1], [2, 4, 2], [1, 2, 1]]) / 4.0
    k_g = np.array([[0, 1, 0], [1, 4, 1], [0, 1, 0]]) / 4.0
    ref = np.stack([
        ndimage.convolve(raw * (chan == 0), k_rb, mode="constant"),
        ndimage.convolve(raw * (chan == 1), k_g, mode="constant"),
        ndimage.convolve(raw * (chan == 2), k_rb, mode="constant"),
    ], -1)
    inner = (slice(2, -2), slice(2, -2))
    np.testing.assert_allclose(rgb[inner], ref[inner], rtol=1e-9)


# --------------------------------------------------------------------------
# Window form (Sec. 5.3.1, reading R2): in the continuous limit the order-0
# estimate of f = c + (X - X_j)^2 is c + <dx^2> with
# <dx^2> = 1/2 * int K rho^3 / int K rho over the disc, and for
# K = exp(-rho^2/h) - exp(-r^2/h):
#   int_0^r K rho  drho = h/2 (1 - e) - r^2 e / 2,
#   int_0^r K rho^3 drho = h^2/2 (1 - e (1 + r^2/h)) - r^4 e / 4,   e = exp(-r^2/h).
# A dense aligned sensor (spacing 1/8) approximates the integral.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("h_given", [0.0, 0.4, 1.5])
def test_window_second_moment_closed_form(h_given):
    """h_given = 0 selects the default 2 r^2 / 9; the closed form holds for any h."""
    r = 2.0
    h = h_given if h_given > 0 else 2 * r * r / 9
    e = math.exp(-r * r / h)
    i1 = h / 2 * (1 - e) - r * r * e / 2
    i3 = h * h / 2 * (1 - e * (1 + r * r / h)) - r ** 4 * e / 4
    expected = 0.5 * i3 / i1
    step = 1.0 / 16
    n = 96
    X0 = Y0 = (n - 1) * step / 2 + 1e-3  # off-lattice centre
    s = _sensor(n, n, [step, 0, 0, 0, step, 0], 1.0, gain=1.0, read_sigma=1e6, black_level=0.0)
    y, x = np.mgrid[0:n, 0:n] * step
    c0 = 5000.0
    raw = c0 + (x - X0) ** 2
    params = _params(1, 1, 0, [r], out_affine=[0, 0, X0, 0, 0, Y0], h=[h_given])
    res = oracle.reconstruct([s], [raw], params)
    got = res["rgb"][0] - c0
    # discretisation error at spacing 1/16 is well below 1%; the plausible
    # mistakes (no truncation, h^2 for h, 2h for h) move the value by >= 7%.
    np.testing.assert_allclose(got, expected, rtol=0.01)


# --------------------------------------------------------------------------
# Invariants: sensor order, rigid motion of the whole rig and output grid, and
# pointwise consistency of arbitrary output maps.
# --------------------------------------------------------------------------
def _noisy_rig(seed, size=20, n=3):
    rng = np.random.default_rng(seed)
    sensors = [R.make_sensor(size, size, _affine(rng, 0.02, 2.0, 1.5), e)
               for e in (1.0, 1 / 8, 1 / 64)[:n]]
    from synth.scene import EdgeScene
    scene = EdgeScene(size, size, seed, n_lines=4)
    raws = [R.capture(scene, s, (seed, i)) for i, s in enumerate(sensors)]
    return sensors, raws


@pytest.mark.parametrize("order", [1, 2])
def test_sensor_order_invariance(order):
    sensors, raws = _noisy_rig(21)
    params = _params(20, 20, order, [1.5, 2.5, 3.5])
    a = oracle.reconstruct(sensors, raws, params)
    perm = [2, 0, 1]
    b = oracle.reconstruct([sensors[i] for i in perm], [raws[i] for i in perm], params)
    # summation order changes; FP64 rounding times the condition number of the
    # order-2 normal matrices (pivot ratios down to 1e-5) stays below 1e-9
    np.testing.assert_allclose(a["rgb"], b["rgb"], rtol=1e-9, atol=1e-9, equal_nan=True)
    firm = a["margin"] > 1e-6
    assert np.array_equal(a["scale_map"][firm], b["scale_map"][firm])


def _moved(aff, th_deg, t):
    th = math.radians(th_deg)
    Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    A = np.array([[aff[0], aff[1]], [aff[3], aff[4]]])
    b = np.array([aff[2], aff[5]])
    A2, b2 = Rm @ A, Rm @ b + np.asarray(t)
    return [A2[0, 0], A2[0, 1], b2[0], A2[1, 0], A2[1, 1], b2[1]]


@pytest.mark.parametrize("order", [0, 1, 2])
def test_rigid_motion_invariance(order):
    """A rotation + translation applied to every T_s and to the output map leaves
    each fit (support, C0, its variance) unchanged: distances are preserved and
    the polynomial space is closed under rotation.  The validity threshold is
    taken on the Jacobi-equilibrated pivot, which is not rotation invariant, so
    per-fit values are compared where both runs call the fit valid; under a
    half-turn (axes negated) the equilibrated pivots are identical too, and the
    whole output must match."""
    sensors, raws = _noisy_rig(22)
    params = _params(20, 20, order, [2.0, 3.0])
    a = oracle.reconstruct(sensors, raws, params, want_fits=True)
    for th, exact in ((33.0, False), (180.0, True)):
        t = (123.25, -47.5)
        moved = [dict(s, affine=_moved(s["affine"], th, t)) for s in sensors]
        b = oracle.reconstruct(moved, raws, dict(params, out_affine=_moved(params["out_affine"], th, t)),
                               want_fits=True)
        fa, fb = a["fits"], b["fits"]
        assert np.array_equal(fa["n"], fb["n"])
        both = (fa["valid"] == 1) & (fb["valid"] == 1)
        assert both.sum() > 0.5 * (fa["valid"] == 1).sum()
        # FP64 rounding of the moved coordinates (ulp ~3e-14 near 150) moves the
        # weights; the effect on C0 and on its variance scales with the data
        # range (radiance up to ~1e4 here) and with the conditioning of the
        # fit: allow 1e-10 / rho of that (a real mistake moves values by O(1)).
        rho = np.minimum(fa["rho"], fb["rho"])[both]
        tol = 1e-10 / rho
        sd = np.sqrt(fa["var"][both])
        for key, scale in (("yhat", np.maximum(np.maximum(np.abs(fa["yhat"][both]), sd), 1e3)),
                           ("var", fa["var"][both])):
            x, y = fa[key][both], fb[key][both]
            assert np.all(np.abs(x - y) <= tol * scale), key
        if exact:
            np.testing.assert_allclose(fa["rho"], fb["rho"], rtol=1e-6, atol=1e-8)  # rank-deficient supports: rounding-level pivots
            firm = a["margin"] > 1e-6
            assert np.array_equal(a["scale_map"][firm], b["scale_map"][firm])
            np.testing.assert_allclose(a["rgb"][firm], b["rgb"][firm], rtol=1e-8, atol=1e-8)


def test_pointwise_consistency_of_output_maps():
    sensors, raws = _noisy_rig(23)
    fine = _params(64, 64, 1, [2.0], out_affine=R.resample_output(4.0))
    a = oracle.reconstruct(sensors, raws, fine)
    # a 16x16 grid of unit spacing whose pixels coincide with every 4th fine pixel
    # shifted by 2: fine (u, v) = (4i + 2, 4j + 2) -> X = (4i + 2.5)/4 - 1/2 = i + 1/8
    coarse = _params(16, 16, 1, [2.0], out_affine=[1, 0, 0.125, 0, 1, 0.125])
    b = oracle.reconstruct(sensors, raws, coarse)
    fa = a["rgb"].reshape(64, 64, 3)[2::4, 2::4]
    np.testing.assert_allclose(fa.reshape(-1, 3), b["rgb"], rtol=1e-13, atol=1e-10, equal_nan=True)


def test_bounding_box_matches_exhaustive_scan():
    sensors, raws = _noisy_rig(24)
    params = _params(20, 20, 2, [1.0, 2.0, 3.0, 4.0])
    a = oracle.reconstruct(sensors, raws, params, want_fits=True)
    b = oracle.reconstruct(sensors, raws, params, want_fits=True, exhaustive=True)
    assert np.array_equal(a["rgb"], b["rgb"], equal_nan=True)
    assert np.array_equal(a["fits"]["n"], b["fits"]["n"])


# --------------------------------------------------------------------------
# Noise model (Sec. 6, 6.1): Monte-Carlo of the forward model.  The radiance
# estimate is unbiased and its variance is (g^2 n f + Var r)/(g n)^2; the
# oracle's variance estimate evaluated at the mean digital value must match
# the empirical variance.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("f,exposure", [(3.0, 1.0), (500.0, 0.25), (4000.0, 1 / 16)])
def test_noise_model_monte_carlo(f, exposure):
    s = R.make_sensor(400, 400, [1, 0, 0, 0, 1, 0], exposure, saturation=1e300)
    scene = PolynomialScene(np.tile([f, 0, 0, 0, 0, 0], (3, 1)))
    y = R.capture_float_noisy(scene, s, 5).ravel()  # 160000 independent samples
    fh = np.empty_like(y)
    for i in range(0, y.size, 1):
        if i >= 4000:
            break
        fh[i] = oracle.sample_radiance(s, y[i])[1]
    g, b = s["gain"], s["black_level"]
    fh_all = (y - b) / (g * exposure)
    np.testing.assert_allclose(fh[:4000], fh_all[:4000], rtol=1e-12)
    ok, _, var_model = oracle.sample_radiance(s, g * exposure * f + b)
    assert ok
    assert abs(fh_all.mean() - f) < 5 * math.sqrt(var_model / fh_all.size)
    assert fh_all.var() == pytest.approx(var_model, rel=0.02)
    assert not oracle.sample_radiance(s | {"saturation": 100.0}, 100.0)[0]
    assert oracle.sample_radiance(s | {"saturation": 100.0}, 99.0)[0]


def test_estimate_variance_monte_carlo():
    """The sandwich variance v = e0^T A^-1 B A^-1 e0 of the chosen fit matches the
    empirical variance of the estimate over independent captures (readout-
    dominated noise so the weights barely depend on the noise)."""
    rng = np.random.default_rng(9)
    sensors = [R.make_sensor(14, 14, _affine(rng, 0.0, 0.5, 1.0), e, read_sigma=40.0,
                             saturation=1e300) for e in (1.0, 0.5)]
    scene = PolynomialScene(np.tile([300.0, 4.0, -3.0, 0, 0, 0], (3, 1)))
    params = _params(1, 1, 1, [2.5], out_affine=[0, 0, 7.3, 0, 0, 6.6])
    vals, vs = [], []
    for t in range(3000):
        raws = [R.capture_float_noisy(scene, s, (t, i)) for i, s in enumerate(sensors)]
        res = oracle.reconstruct(sensors, raws, params, want_fits=True)
        vals.append(res["rgb"][0])
        vs.append(res["fits"][0, :, 0, 1]["var"])
    vals, vs = np.array(vals), np.array(vs)
    emp = vals.var(0)
    # relative standard error of a sample variance over 3000 draws is ~2.6%
    np.testing.assert_allclose(emp, vs.mean(0), rtol=0.1)


# --------------------------------------------------------------------------
# Saturation-boundary bias (Sec. 5.3, fig. polyfit): on a linear ramp where the
# brighter sensor saturates for X beyond a threshold, an order-1 fit is exact
# everywhere while an order-0 fit is biased next to the saturation boundary.
# --------------------------------------------------------------------------
def test_saturation_boundary_order_effect():
    size = 40
    ramp = PolynomialScene(np.tile([2000.0, 150.0, 0, 0, 0, 0], (3, 1)))
    aligned = [1, 0, 0, 0, 1, 0]
    bright = _sensor(size, size, aligned, 1.0, read_sigma=2.0, saturation=64 + 0.5 * 2000 + 0.5 * 150 * 20.5)
    dim = _sensor(size, size, aligned, 1 / 16, read_sigma=2.0)
    raws = [R.capture_noise_free_f64(ramp, s) for s in (bright, dim)]
    res = {}
    for order in (0, 1):
        out = oracle.reconstruct([bright, dim], raws, _params(size, size, order, [3.0]))
        res[order] = out["rgb"].reshape(size, size, 3)
    u = np.arange(size, dtype=np.float64)
    truth = (2000.0 + 150.0 * u)[None, :, None]
    inner = (slice(5, -5), slice(5, -5))
    err1 = np.abs(res[1] - truth)[inner] / truth[:, 5:-5]
    err0 = np.abs(res[0] - truth)[inner] / truth[:, 5:-5]
    assert err1.max() < 1e-10
    cols = np.arange(5, size - 5)
    near = np.abs(cols - 20.5) < 3
    far = np.abs(cols - 20.5) > 8
    bias_near = err0[:, near].max()
    bias_far = err0[:, far].max()
    # away from the boundary the order-0 fit is only mildly biased (the shot-noise
    # weights vary along the ramp); next to it the bias is an order larger
    assert bias_near > 1e-2
    assert bias_near > 8 * bias_far


# --------------------------------------------------------------------------
# ICI (reading R8): worked examples, and the closed form on noise-free
# polynomial scenes, where every scale estimates the same value so the
# intersection never empties and the largest valid scale is chosen.
# --------------------------------------------------------------------------
def test_ici_worked_examples():
    with open(os.path.join(GOLDEN, "ici_worked_examples.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        k, mu, gap = oracle.ici_select(c["yhat"], c["var"], c["valid"], c["gamma"])
        assert k == c["chosen"], c["name"]
        want = math.inf if c["margin"] == "inf" else c["margin"]
        assert mu == pytest.approx(want), c["name"]
        want = math.inf if c["gap"] == "inf" else c["gap"]
        assert gap == pytest.approx(want), c["name"]


@pytest.mark.parametrize("order", [1, 2])
def test_ici_picks_largest_valid_scale_on_polynomials(order):
    rng = np.random.default_rng(40 + order)
    coeffs = np.zeros((3, 6))
    coeffs[:, 0] = 800.0
    coeffs[:, 1:3] = rng.uniform(-5, 5, (3, 2))
    if order == 2:
        coeffs[:, 3:6] = rng.uniform(-0.05, 0.05, (3, 3))
    scene = PolynomialScene(coeffs)
    sensors = [_sensor(30, 30, _affine(rng, 0.0, 0.3, 2.0), e) for e in (1.0, 0.25, 1 / 16, 1 / 64)]
    raws = [R.capture_noise_free_f64(scene, s) for s in sensors]
    params = _params(12, 12, order, [1.0, 2.0, 3.0, 4.0], out_affine=[1, 0, 9, 0, 1, 9])
    res = oracle.reconstruct(sensors, raws, params, want_fits=True)
    valid = res["fits"]["valid"][:, :, :, order]
    largest = 3 - np.argmax(valid[:, :, ::-1], axis=2)
    assert np.all(valid.any(axis=2))
    assert np.array_equal(res["scale_map"] & 0xF, largest.astype(np.uint8))


def test_order_fallback_and_no_data():
    """Order fallback (reading R9): with a single radius-1 window most R/B
    supports have too few samples for the 6-term fit, so the chosen order drops;
    the value then equals a direct fit at that order.  A pixel with no sample
    at all gives NaN and the NO_DATA code."""
    sensors, raws = _noisy_rig(25)
    p2 = _params(20, 20, 2, [1.2])
    a = oracle.reconstruct(sensors, raws, p2)
    orders = a["scale_map"] >> 4
    assert (orders < 2).any()
    for o in (0, 1):
        direct = oracle.reconstruct(sensors, raws, _params(20, 20, o, [1.2]))
        sel = (orders == o) & (a["scale_map"] != 0xFF)
        np.testing.assert_array_equal(a["rgb"][sel], direct["rgb"][sel])
    far = oracle.reconstruct(sensors, raws, _params(1, 1, 1, [2.0], out_affine=[0, 0, 500.0, 0, 0, 500.0]))
    assert np.all(np.isnan(far["rgb"])) and np.all(far["scale_map"] == 0xFF)


def test_gain_calibration_relation_on_generator():
    """Sec. 6.2: (Var y - Var b) / (E y - E b) = g on flat fields; a check that
    the synthetic forward model carries the paper's noise model."""
    s = R.make_sensor(300, 300, [1, 0, 0, 0, 1, 0], 1.0, saturation=1e300)
    flat = R.capture_float_noisy(PolynomialScene(np.tile([2000.0, 0, 0, 0, 0, 0], (3, 1))), s, 1)
    dark = R.capture_float_noisy(PolynomialScene(np.zeros((3, 6))), s, 2)
    g_est = (flat.var() - dark.var()) / (flat.mean() - dark.mean())
    assert g_est == pytest.approx(s["gain"], rel=0.02)


def test_cfa_patterns():
    # RGGB, BGGR, GRBG, GBRG read row-major from pixel (0, 0) (Sec. 3, Bayer CFA)
    want = {"RGGB": [0, 1, 1, 2], "BGGR": [2, 1, 1, 0], "GRBG": [1, 0, 2, 1], "GBRG": [1, 2, 0, 1]}
    for name, seq in want.items():
        got = [oracle.cfa_channel(name, x, y) for (y, x) in [(0, 0), (0, 1), (1, 0), (1, 1)]]
        assert got == seq, name
        assert oracle.cfa_channel(name, 4, 6) == seq[0]
