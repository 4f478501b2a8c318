"""Pins of the oracle's adaptive anisotropic LPA with colour-channel
correlation (CALPA, Sec. 5.4 and 5.5).

Expectations come from closed-form special cases of the steering matrix, an
independent SVD (numpy), polynomial reproduction, rotation equivariance,
the exhaustive sample scan, and the geometric property the section states
(windows elongated along edges) -- not from the oracle's own formulas.
"""
import math

import numpy as np
import pytest

import oracle
from synth import configs, rig as R
from synth.scene import EdgeScene, PolynomialScene

WIDE = {"max_stretch": 100.0}  # clamp far outside the values these pins produce


def _params(out_w, out_h, order, radii, **kw):
    p = {"out_w": out_w, "out_h": out_h, "out_affine": [1.0, 0.0, 0.0, 0.0, 1.0, 0.0],
         "order": order, "radii": list(radii), "gamma": 2.0, "green_ratio": 1.0, "tau_inv": 1e-5}
    p.update(kw)
    return p


def _sensor(w, h, affine, exposure):
    return R.make_sensor(w, h, affine, exposure, gain=0.5, read_sigma=3.0, black_level=64.0,
                         saturation=1e300, bit_depth=12, cfa="RGGB")


def _small_case(seed=2100, size=48):
    sensors = configs.full_rig(seed=seed, size=size)
    scene = EdgeScene(size, size, seed, n_lines=8)
    raws = configs.capture_all(scene, sensors, seed)
    return sensors, raws, _params(size, size, 2, [1.0, 2.0, 3.0, 4.0])


def _eig_sorted(C):
    """Eigen-decomposition of symmetric 2x2 matrices given as (n, 3) rows."""
    M = np.stack([np.stack([C[:, 0], C[:, 1]], -1), np.stack([C[:, 1], C[:, 2]], -1)], -2)
    w, V = np.linalg.eigh(M)  # ascending
    return w, V


# --------------------------------------------------------------------------
# With C = I the steered window is the isotropic one (Sec. 5.4 with
# H = hI): bit-identical to the plain reconstruction; so is CALPA with the
# stretch bound at 1 (every eigenvalue clamped to 1).
# --------------------------------------------------------------------------
def test_identity_steering_reduces_to_lpa():
    sensors, raws, p = _small_case()
    iso = oracle.reconstruct(sensors, raws, p, want_fits=True)
    n = p["out_w"] * p["out_h"]
    st = oracle.reconstruct_steered(sensors, raws, p, np.tile([1.0, 0.0, 1.0], (n, 1)), want_fits=True)
    assert np.array_equal(st["rgb"], iso["rgb"], equal_nan=True)
    assert np.array_equal(st["scale_map"], iso["scale_map"])
    assert np.array_equal(st["fits"]["var"], iso["fits"]["var"], equal_nan=True)
    ad = oracle.reconstruct_adaptive(sensors, raws, p, {"max_stretch": 1.0, "alpha": 0.3})
    assert np.array_equal(ad["rgb"], iso["rgb"], equal_nan=True)


# --------------------------------------------------------------------------
# Steering special cases (Sec. 5.4 definitions of sigma and gamma):
#  - no gradient anywhere: sigma = 1, gamma = (l2 / M)^alpha, C = gamma I,
#    with M = 25 inside the grid and 9 at a corner (q = 2);
#  - one gradient g0 everywhere: G has rank 1, s1 = sqrt(M)|g0|, s2 = 0, so
#    sigma = s1 / l1 + 1 and (alpha = 0) C has eigenvalue sigma along g0
#    and 1/sigma across it.
# --------------------------------------------------------------------------
def test_steering_zero_gradients_closed_form():
    p = _params(9, 7, 1, [2.0])
    a = dict(WIDE, alpha=0.5, lambda2=0.001, grad_halfwin=2)
    C = oracle.steering(p, a, np.zeros((7, 9, 2)))
    C = C.reshape(7, 9, 3)
    inner = math.sqrt(0.001 / 25.0)
    corner = math.sqrt(0.001 / 9.0)
    np.testing.assert_allclose(C[3, 4], [inner, 0.0, inner], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(C[0, 0], [corner, 0.0, corner], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(C[6, 8], [corner, 0.0, corner], rtol=1e-12, atol=1e-15)


def test_steering_rank_one_closed_form():
    p = _params(9, 9, 1, [2.0])
    plane = np.zeros((9, 9, 2))
    plane[...] = [3.0, 4.0]
    a = dict(WIDE, alpha=0.0, lambda1=1.0, grad_halfwin=2)
    C = oracle.steering(p, a, plane).reshape(9, 9, 3)
    sigma = 5.0 * 5.0 + 1.0  # sqrt(25) * |g0| / l1 + 1
    w, V = _eig_sorted(C[4, 4][None])
    np.testing.assert_allclose(w[0], [1.0 / sigma, sigma], rtol=1e-12)
    along_g0 = np.abs(V[0][:, 1] @ np.array([0.6, 0.8]))
    assert along_g0 > 1 - 1e-12


# --------------------------------------------------------------------------
# The singular values and the second right singular vector of the stacked
# gradient matrix (Sec. 5.4) against numpy's SVD, on random gradient fields;
# the steering matrix's smaller eigenvalue lies along that vector (window
# elongated along the edge) and det C = gamma^2 when nothing is clamped.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_steering_against_numpy_svd(seed):
    rng = np.random.default_rng(seed)
    H, W, q = 8, 11, 2
    base = rng.normal(size=2)
    plane = base + 0.4 * rng.normal(size=(H, W, 2))
    p = _params(W, H, 1, [2.0])
    a = dict(WIDE, alpha=0.3, lambda1=0.5, lambda2=0.01, grad_halfwin=q)
    C, diag = oracle.steering(p, a, plane, want_diag=True)
    w, V = _eig_sorted(C)
    for v in range(H):
        for u in range(W):
            k = v * W + u
            rows = plane[max(0, v - q): v + q + 1, max(0, u - q): u + q + 1].reshape(-1, 2)
            _, s, Vt = np.linalg.svd(rows, full_matrices=False)
            np.testing.assert_allclose(diag[k, :2], s, rtol=1e-10)
            v2 = Vt[1]
            # theta = arctan(v1 / v2) of the second right singular vector
            assert abs(math.tan(diag[k, 2]) - v2[0] / v2[1]) < 1e-8 * (1 + abs(v2[0] / v2[1]))
            # the window's long axis (smaller eigenvalue of C) is v
            assert abs(V[k][:, 0] @ v2) > 1 - 1e-9
            gamma = diag[k, 4]
            assert abs(w[k, 0] * w[k, 1] - gamma * gamma) < 1e-10 * gamma * gamma


# --------------------------------------------------------------------------
# Rotating the gradient plane by 90 degrees (grid and vectors) rotates every
# steering matrix: C'(rotated pixel) = R C R^T.
# --------------------------------------------------------------------------
def test_steering_rotation_equivariance():
    rng = np.random.default_rng(7)
    H, W = 6, 9
    plane = rng.normal(size=(H, W, 2)) * [2.0, 0.5]
    a = dict(alpha=0.2, lambda1=0.3, lambda2=0.01, grad_halfwin=1, max_stretch=3.0)
    C = oracle.steering(_params(W, H, 1, [2.0]), a, plane).reshape(H, W, 3)
    # pixel (u, v) -> (H - 1 - v, u); vector (x, y) -> (-y, x)
    rot = np.zeros((W, H, 2))
    for v in range(H):
        for u in range(W):
            gx, gy = plane[v, u]
            rot[u, H - 1 - v] = [-gy, gx]
    C2 = oracle.steering(_params(H, W, 1, [2.0]), a, rot).reshape(W, H, 3)
    Rm = np.array([[0.0, -1.0], [1.0, 0.0]])
    for v in range(H):
        for u in range(W):
            c = C[v, u]
            M = Rm @ np.array([[c[0], c[1]], [c[1], c[2]]]) @ Rm.T
            np.testing.assert_allclose(C2[u, H - 1 - v], [M[0, 0], M[0, 1], M[1, 1]], rtol=1e-9, atol=1e-12)


# --------------------------------------------------------------------------
# Stage 1 (Sec. 5.4 first step, Sec. 5.5 G channel): on a noise-free field
# whose G channel is linear (R and B differ), the gradient of every pixel is
# exactly the G field's gradient, at orders 1 and 2; a quadratic G field at
# order 2 gives its gradient at X_j.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("grad_order", [1, 2])
def test_gradients_reproduce_green_field(grad_order):
    coeffs = np.array([[300.0, -2.0, 1.0, 0, 0, 0],
                       [250.0, 1.5, -0.75, 0.01 if grad_order == 2 else 0, -0.02 if grad_order == 2 else 0,
                        0.015 if grad_order == 2 else 0],
                       [200.0, 0.5, 2.0, 0, 0, 0]])
    scene = PolynomialScene(coeffs)
    rng = np.random.default_rng(3)
    sensors = [_sensor(30, 30, [math.cos(0.05), -math.sin(0.05), rng.uniform(-1, 1),
                                math.sin(0.05), math.cos(0.05), rng.uniform(-1, 1)], e) for e in (1.0, 0.25)]
    raws = [R.capture_noise_free_f64(scene, s) for s in sensors]
    p = _params(12, 12, 2, [2.0], out_affine=[1.0, 0.0, 8.0, 0.0, 1.0, 9.0])
    g, valid = oracle.gradients(sensors, raws, p, {"grad_order": grad_order, "grad_radius": 2.5})
    assert valid.all()
    u, v = np.meshgrid(np.arange(12.0), np.arange(12.0))
    X = (u + 8.0).ravel()
    Y = (v + 9.0).ravel()
    c = coeffs[1]
    np.testing.assert_allclose(g[:, 0], c[1] + 2 * c[3] * X + c[4] * Y, rtol=1e-8, atol=1e-9)
    np.testing.assert_allclose(g[:, 1], c[2] + c[4] * X + 2 * c[5] * Y, rtol=1e-8, atol=1e-9)


# --------------------------------------------------------------------------
# CALPA reproduces any field of degree <= M exactly (Sec. 5.1: the weighted
# fit is exact whatever the window), with steering matrices far from I.
# --------------------------------------------------------------------------
def test_calpa_reproduces_polynomials():
    rng = np.random.default_rng(11)
    coeffs = np.zeros((3, 6))
    coeffs[:, 0] = rng.uniform(200, 400, 3)
    coeffs[:, 1:] = rng.uniform(-3, 3, (3, 5)) / np.array([1, 1, 20, 20, 20])
    scene = PolynomialScene(coeffs)
    sensors = [_sensor(34, 34, [math.cos(t), -math.sin(t), dx, math.sin(t), math.cos(t), dy], e)
               for t, dx, dy, e in ((0.0, 0.0, 0.0, 1.0), (0.04, 0.7, -0.4, 0.25), (-0.03, -0.3, 0.6, 1 / 16))]
    raws = [R.capture_noise_free_f64(scene, s) for s in sensors]
    p = _params(14, 14, 2, [2.5, 3.5], out_affine=[1.0, 0.0, 10.0, 0.0, 1.0, 10.0])
    out = oracle.reconstruct_adaptive(sensors, raws, p, {"alpha": 0.0, "max_stretch": 1.6}, want_stages=True)
    w, _ = _eig_sorted(out["C"])
    assert (w[:, 1] / w[:, 0]).max() > 2.0, "the gradients must make the windows anisotropic"
    u, v = np.meshgrid(np.arange(14.0), np.arange(14.0))
    X, Y = (u + 10.0).ravel(), (v + 10.0).ravel()
    truth = np.stack([scene.radiance(X, Y, c) for c in range(3)], -1)
    assert np.all(out["scale_map"] >> 4 == 2)
    np.testing.assert_allclose(out["rgb"], truth, rtol=1e-10, atol=0)


# --------------------------------------------------------------------------
# Steered supports: the ellipse's bounding box against a scan of every sample.
# --------------------------------------------------------------------------
def test_steered_box_matches_exhaustive_scan():
    sensors, raws, p = _small_case(seed=2200, size=32)
    rng = np.random.default_rng(5)
    n = p["out_w"] * p["out_h"]
    th = rng.uniform(0, math.pi, n)
    la, lb = rng.uniform(0.25, 4.0, n), rng.uniform(0.25, 4.0, n)
    c, s = np.cos(th), np.sin(th)
    C = np.stack([la * c * c + lb * s * s, (la - lb) * c * s, la * s * s + lb * c * c], -1)
    a = oracle.reconstruct_steered(sensors, raws, p, C, want_fits=True)
    b = oracle.reconstruct_steered(sensors, raws, p, C, want_fits=True, exhaustive=True)
    assert np.array_equal(a["fits"]["n"], b["fits"]["n"])
    assert np.array_equal(a["rgb"], b["rgb"], equal_nan=True)


# --------------------------------------------------------------------------
# Orientation (Sec. 5.4: "elongated along edges"): beside a straight oblique
# step edge, the steering matrix's larger eigenvalue (the window's short axis)
# lies along the edge normal; and a window so steered keeps the estimate
# closer to the step than the isotropic one.
# --------------------------------------------------------------------------
class _ObliqueStep:
    def __init__(self, normal, offset, lo, hi):
        self.n = np.asarray(normal, float) / np.linalg.norm(normal)
        self.offset, self.lo, self.hi = offset, lo, hi

    def radiance(self, X, Y, channel):
        X, Y = np.asarray(X, float), np.asarray(Y, float)
        return np.where(self.n[0] * X + self.n[1] * Y < self.offset, self.lo, self.hi)


@pytest.mark.parametrize("angle", [0.0, 0.5, 1.2])
def test_orientation_and_sharpening_on_oblique_edge(angle):
    normal = (math.cos(angle), math.sin(angle))
    scene = _ObliqueStep(normal, normal[0] * 20.3 + normal[1] * 20.3, 50.0, 800.0)
    sensors = [_sensor(44, 44, [1.0, 0.0, 0.0, 0.0, 1.0, 0.0], 1.0),
               _sensor(44, 44, [1.0, 0.0, 0.5, 0.0, 1.0, 0.5], 0.5)]
    raws = [R.capture_noise_free_f64(scene, s) for s in sensors]
    p = _params(20, 20, 1, [2.0], out_affine=[1.0, 0.0, 11.0, 0.0, 1.0, 11.0])
    a = {"alpha": 0.0, "max_stretch": 2.0, "grad_radius": 1.5}
    out = oracle.reconstruct_adaptive(sensors, raws, p, a, want_stages=True)
    iso = oracle.reconstruct(sensors, raws, p)
    u, v = np.meshgrid(np.arange(20.0), np.arange(20.0))
    X, Y = (u + 11.0).ravel(), (v + 11.0).ravel()
    dist = normal[0] * X + normal[1] * Y - scene.offset
    near = (np.abs(dist) > 0.3) & (np.abs(dist) < 1.6)
    w, V = _eig_sorted(out["C"][near])
    across = np.abs(V[:, :, 1] @ np.asarray(normal))  # eigenvector of the larger eigenvalue
    assert np.median(across) > 0.98
    truth = scene.radiance(X, Y, 1)
    err_c = np.abs(out["rgb"][near, 1] - truth[near])
    err_i = np.abs(iso["rgb"][near, 1] - truth[near])
    assert err_c.mean() < 0.8 * err_i.mean()
