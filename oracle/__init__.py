"""Plain FP64 CPU oracle for LPA + ICI HDR reconstruction (arXiv 1308.4908).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  This module marshals numpy arrays
into the C oracle (``lpa_oracle.c``); every step of the method is computed
there, in FP64, single-threaded.  It shares no code with the GPU library.

Rig and parameter descriptions are plain dicts (see ``synth.rig``):
sensor keys  width, height, cfa, affine(6), exposure, gain, read_sigma,
             black_level, saturation; optional calib: per-pixel frames
             (height x width) bias, prnu, read_var, sat, defect (Sec. 6)
param keys   out_w, out_h, out_affine(6), order, radii, h (optional), gamma,
             green_ratio, tau_inv; for CALPA the adapt dict (reconstruct_adaptive)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lpa_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblpa_oracle.so")
# A test that checks the pins catch planted mistakes points this at a mutated build.
_OVERRIDE = os.environ.get("LPA_ORACLE_LIB_OVERRIDE")
_lib = None

CFA = {"RGGB": 0, "BGGR": 1, "GRBG": 2, "GBRG": 3}
MAX_SCALES = 8


class _Sensor(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("cfa", ctypes.c_int32),
        ("affine", ctypes.c_double * 6),
        ("exposure", ctypes.c_double),
        ("gain", ctypes.c_double),
        ("read_sigma", ctypes.c_double),
        ("black_level", ctypes.c_double),
        ("saturation", ctypes.c_double),
        ("bias", ctypes.c_void_p),
        ("prnu", ctypes.c_void_p),
        ("read_var", ctypes.c_void_p),
        ("sat", ctypes.c_void_p),
        ("defect", ctypes.c_void_p),
    ]


class _Params(ctypes.Structure):
    _fields_ = [
        ("out_w", ctypes.c_int32),
        ("out_h", ctypes.c_int32),
        ("out_affine", ctypes.c_double * 6),
        ("order", ctypes.c_int32),
        ("n_scales", ctypes.c_int32),
        ("radii", ctypes.c_double * MAX_SCALES),
        ("h", ctypes.c_double * MAX_SCALES),
        ("gamma", ctypes.c_double),
        ("green_ratio", ctypes.c_double),
        ("tau_inv", ctypes.c_double),
        ("exhaustive", ctypes.c_int32),
    ]


class _Fit(ctypes.Structure):
    _fields_ = [
        ("yhat", ctypes.c_double),
        ("var", ctypes.c_double),
        ("rho", ctypes.c_double),
        ("c1x", ctypes.c_double),
        ("c1y", ctypes.c_double),
        ("l1f", ctypes.c_double),
        ("sens_y", ctypes.c_double),
        ("sens_v", ctypes.c_double),
        ("n", ctypes.c_int32),
        ("valid", ctypes.c_int32),
    ]


class _Adapt(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_double),
        ("lambda1", ctypes.c_double),
        ("lambda2", ctypes.c_double),
        ("grad_radius", ctypes.c_double),
        ("grad_h", ctypes.c_double),
        ("max_stretch", ctypes.c_double),
        ("grad_order", ctypes.c_int32),
        ("grad_halfwin", ctypes.c_int32),
    ]


# Adaptive (CALPA) parameters: the paper's regularisers (Sec. 5.4) and the
# readings R20..R22 (analysis window, stretch bound, gradient fit).
ADAPT_DEFAULTS = {"alpha": 0.005, "lambda1": 1.0, "lambda2": 0.001, "grad_radius": 2.0, "grad_h": 0.0,
                  "max_stretch": 2.0, "grad_order": 1, "grad_halfwin": 2}


FIT_DTYPE = np.dtype(
    [("yhat", "f8"), ("var", "f8"), ("rho", "f8"), ("c1x", "f8"), ("c1y", "f8"), ("l1f", "f8"),
     ("sens_y", "f8"), ("sens_v", "f8"),
     ("n", "i4"), ("valid", "i4")],
    align=True,
)
assert FIT_DTYPE.itemsize == ctypes.sizeof(_Fit)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict IEEE FP64: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-Wall",
             "-Wextra", "-o", tmp, _SRC, "-lm"],
            check=True,
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if _OVERRIDE:
            lib = ctypes.CDLL(_OVERRIDE)
        else:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build()
            lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_reconstruct.restype = ctypes.c_int
        lib.orc_reconstruct.argtypes = [
            ctypes.POINTER(_Sensor), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
            ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ]
        lib.orc_reconstruct_steered.restype = ctypes.c_int
        lib.orc_reconstruct_steered.argtypes = [
            ctypes.POINTER(_Sensor), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
            ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ]
        lib.orc_gradients.restype = ctypes.c_int
        lib.orc_gradients.argtypes = [
            ctypes.POINTER(_Sensor), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
            ctypes.POINTER(_Params), ctypes.POINTER(_Adapt), ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p,
        ]
        lib.orc_steering.restype = ctypes.c_int
        lib.orc_steering.argtypes = [
            ctypes.POINTER(_Params), ctypes.POINTER(_Adapt), ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
        ]
        lib.orc_reconstruct_temporal.restype = ctypes.c_int
        lib.orc_reconstruct_temporal.argtypes = [
            ctypes.POINTER(_Sensor), ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
            ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ]
        lib.orc_sample_radiance.restype = ctypes.c_int
        lib.orc_sample_radiance.argtypes = [
            ctypes.POINTER(_Sensor), ctypes.c_double, ctypes.POINTER(ctypes.c_double),
            ctypes.POINTER(ctypes.c_double),
        ]
        lib.orc_sample_radiance_at.restype = ctypes.c_int
        lib.orc_sample_radiance_at.argtypes = [
            ctypes.POINTER(_Sensor), ctypes.c_int64, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
            ctypes.POINTER(ctypes.c_double),
        ]
        lib.orc_cfa_channel.restype = ctypes.c_int
        lib.orc_cfa_channel.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        lib.orc_ici_select.restype = ctypes.c_int
        lib.orc_ici_select.argtypes = [
            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
        ]
        _lib = lib
    return _lib


def _sensor_struct(d: dict) -> _Sensor:
    s = _Sensor()
    s.width = int(d["width"])
    s.height = int(d["height"])
    cfa = d.get("cfa", "RGGB")
    s.cfa = CFA[cfa] if isinstance(cfa, str) else int(cfa)
    for i, a in enumerate(d["affine"]):
        s.affine[i] = float(a)
    s.exposure = float(d["exposure"])
    s.gain = float(d["gain"])
    s.read_sigma = float(d["read_sigma"])
    s.black_level = float(d["black_level"])
    s.saturation = float(d["saturation"])
    # optional per-pixel calibration frames (kept alive on the struct)
    keep = []
    calib = d.get("calib") or {}
    for name in ("bias", "prnu", "read_var", "sat"):
        if calib.get(name) is not None:
            a = np.ascontiguousarray(np.asarray(calib[name], dtype=np.float64).reshape(s.height, s.width))
            keep.append(a)
            setattr(s, name, a.ctypes.data)
    if calib.get("defect") is not None:
        a = np.ascontiguousarray(np.asarray(calib["defect"], dtype=np.uint8).reshape(s.height, s.width))
        keep.append(a)
        s.defect = a.ctypes.data
    s._keep = keep
    return s


def _params_struct(p: dict, exhaustive: bool) -> _Params:
    q = _Params()
    q.out_w = int(p["out_w"])
    q.out_h = int(p["out_h"])
    for i, a in enumerate(p["out_affine"]):
        q.out_affine[i] = float(a)
    q.order = int(p["order"])
    radii = list(p["radii"])
    q.n_scales = len(radii)
    hs = list(p.get("h") or [0.0] * len(radii))
    for i, r in enumerate(radii):
        q.radii[i] = float(r)
        q.h[i] = float(hs[i])
    q.gamma = float(p.get("gamma", 2.0))
    q.green_ratio = float(p.get("green_ratio", 1.0))
    q.tau_inv = float(p.get("tau_inv", 1e-5))
    q.exhaustive = 1 if exhaustive else 0
    return q


def reconstruct(sensors, raws, params, pixels=None, want_fits=False, exhaustive=False):
    """Run the oracle.

    sensors : list of sensor dicts; raws : list of 2-D arrays (DN values, any
    numeric dtype; converted exactly to float64); params : parameter dict;
    pixels : optional (n, 2) int array of (u, v) output pixels (default: the
    whole grid, row-major).  Returns a dict with ``rgb`` (n, 3) float64,
    ``scale_map`` (n, 3) uint8, ``margin`` (n, 3), ``gap`` (n, 3) and, if asked, ``fits``
    (n, 3, n_scales, 3) structured array (see FIT_DTYPE).
    """
    lib = _load()
    ns = len(sensors)
    structs = [_sensor_struct(d) for d in sensors]  # hold the calibration frames during the call
    sens = (_Sensor * ns)(*structs)
    planes = [np.ascontiguousarray(np.asarray(r), dtype=np.float64) for r in raws]
    for d, pl in zip(sensors, planes):
        if pl.shape != (int(d["height"]), int(d["width"])):
            raise ValueError(f"raw plane shape {pl.shape} does not match sensor {d['height']}x{d['width']}")
    ptrs = (ctypes.c_void_p * ns)(*[pl.ctypes.data for pl in planes])
    prm = _params_struct(params, exhaustive)
    if pixels is None:
        n = prm.out_w * prm.out_h
        pix_ptr = None
        pix = None
    else:
        pix = np.ascontiguousarray(np.asarray(pixels, dtype=np.int32).reshape(-1, 2))
        n = pix.shape[0]
        pix_ptr = pix.ctypes.data
    rgb = np.empty((n, 3), np.float64)
    smap = np.empty((n, 3), np.uint8)
    margin = np.empty((n, 3), np.float64)
    gap = np.empty((n, 3), np.float64)
    fits = np.zeros((n, 3, prm.n_scales, 3), FIT_DTYPE) if want_fits else None
    rc = lib.orc_reconstruct(
        sens, ns, ptrs, ctypes.byref(prm), pix_ptr, n, rgb.ctypes.data, smap.ctypes.data,
        margin.ctypes.data, gap.ctypes.data, fits.ctypes.data if fits is not None else None,
    )
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (code {rc})")
    out = {"rgb": rgb, "scale_map": smap, "margin": margin, "gap": gap}
    if fits is not None:
        out["fits"] = fits
    return out


def reconstruct_temporal(sensors, frames, params, pixels=None, want_fits=False, exhaustive=False):
    """Temporal LPA (readings T1-T4 in lpa_oracle.h): frames[t] is the list of
    the sensors' raw planes at time -t (frames[0] the output's frame);
    params["h_t"] gives one temporal scale per radius (0: only t = 0).
    Returns the same dict as reconstruct()."""
    lib = _load()
    ns = len(sensors)
    nt = len(frames)
    structs = [_sensor_struct(d) for d in sensors]
    sens = (_Sensor * ns)(*structs)
    planes = []
    for fr in frames:
        if len(fr) != ns:
            raise ValueError("every frame holds one raw plane per sensor")
        for d, r in zip(sensors, fr):
            pl = np.ascontiguousarray(np.asarray(r), dtype=np.float64)
            if pl.shape != (int(d["height"]), int(d["width"])):
                raise ValueError(f"raw plane shape {pl.shape} does not match sensor {d['height']}x{d['width']}")
            planes.append(pl)
    ptrs = (ctypes.c_void_p * (ns * nt))(*[pl.ctypes.data for pl in planes])
    prm = _params_struct(params, exhaustive)
    ht = np.ascontiguousarray(np.asarray(params["h_t"], dtype=np.float64).reshape(-1))
    if ht.size != prm.n_scales:
        raise ValueError("h_t needs one temporal scale per radius")
    if pixels is None:
        n = prm.out_w * prm.out_h
        pix_ptr = None
    else:
        pix = np.ascontiguousarray(np.asarray(pixels, dtype=np.int32).reshape(-1, 2))
        n = pix.shape[0]
        pix_ptr = pix.ctypes.data
    rgb = np.empty((n, 3), np.float64)
    smap = np.empty((n, 3), np.uint8)
    margin = np.empty((n, 3), np.float64)
    gap = np.empty((n, 3), np.float64)
    fits = np.zeros((n, 3, prm.n_scales, 3), FIT_DTYPE) if want_fits else None
    rc = lib.orc_reconstruct_temporal(
        sens, ns, nt, ptrs, ctypes.byref(prm), ht.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), pix_ptr, n,
        rgb.ctypes.data, smap.ctypes.data, margin.ctypes.data, gap.ctypes.data,
        fits.ctypes.data if fits is not None else None,
    )
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (code {rc})")
    out = {"rgb": rgb, "scale_map": smap, "margin": margin, "gap": gap}
    if fits is not None:
        out["fits"] = fits
    return out


def sample_radiance_at(sensor: dict, x: int, row: int, y):
    """(usable, f_hat, var_hat) of digital value(s) y at sensor pixel (x, row),
    with the sensor's calibration frames.  y may be an array (then arrays)."""
    lib = _load()
    s = _sensor_struct(sensor)
    i = int(row) * int(sensor["width"]) + int(x)
    ys = np.atleast_1d(np.asarray(y, dtype=np.float64))
    ok = np.empty(ys.shape, bool)
    fh = np.empty(ys.shape)
    vh = np.empty(ys.shape)
    f = ctypes.c_double()
    v = ctypes.c_double()
    for k, yk in enumerate(ys):
        ok[k] = bool(lib.orc_sample_radiance_at(ctypes.byref(s), i, float(yk), ctypes.byref(f), ctypes.byref(v)))
        fh[k], vh[k] = f.value, v.value
    if np.ndim(y) == 0:
        return bool(ok[0]), float(fh[0]), float(vh[0])
    return ok, fh, vh


def sample_radiance(sensor: dict, y: float):
    """(usable, f_hat, var_hat) of one digital value y on a sensor."""
    lib = _load()
    s = _sensor_struct(sensor)
    f = ctypes.c_double()
    v = ctypes.c_double()
    ok = lib.orc_sample_radiance(ctypes.byref(s), float(y), ctypes.byref(f), ctypes.byref(v))
    return bool(ok), f.value, v.value


def cfa_channel(cfa, x: int, y: int) -> int:
    lib = _load()
    return lib.orc_cfa_channel(CFA[cfa] if isinstance(cfa, str) else int(cfa), int(x), int(y))


def ici_select(yhat, var, valid, gamma: float = 2.0):
    """The ICI rule on given per-scale estimates: (chosen index or -1, margin, gap)."""
    lib = _load()
    y = np.ascontiguousarray(yhat, np.float64)
    v = np.ascontiguousarray(var, np.float64)
    ok = np.ascontiguousarray(valid, np.int32)
    mu = ctypes.c_double()
    gp = ctypes.c_double()
    k = lib.orc_ici_select(len(y), y.ctypes.data, v.ctypes.data, ok.ctypes.data, float(gamma),
                           ctypes.byref(mu), ctypes.byref(gp))
    return k, mu.value, gp.value


def _adapt_struct(a: dict | None) -> _Adapt:
    d = dict(ADAPT_DEFAULTS, **(a or {}))
    q = _Adapt()
    for k in ("alpha", "lambda1", "lambda2", "grad_radius", "grad_h", "max_stretch"):
        setattr(q, k, float(d[k]))
    q.grad_order = int(d["grad_order"])
    q.grad_halfwin = int(d["grad_halfwin"])
    return q


def _pixels(params, pixels):
    if pixels is None:
        return None, int(params["out_w"]) * int(params["out_h"])
    pix = np.ascontiguousarray(np.asarray(pixels, dtype=np.int32).reshape(-1, 2))
    return pix, pix.shape[0]


def gradients(sensors, raws, params, adapt=None, pixels=None, exhaustive=False):
    """Stage 1 of CALPA (Sec. 5.4, 5.5): G-channel gradients of an isotropic
    fit at the listed pixels (default: the whole grid).  Returns (grad (n, 2),
    valid (n,)); invalid fits give a zero gradient."""
    lib = _load()
    ns = len(sensors)
    structs = [_sensor_struct(d) for d in sensors]  # hold the calibration frames during the call
    sens = (_Sensor * ns)(*structs)
    planes = [np.ascontiguousarray(np.asarray(r), dtype=np.float64) for r in raws]
    ptrs = (ctypes.c_void_p * ns)(*[pl.ctypes.data for pl in planes])
    prm = _params_struct(params, exhaustive)
    ad = _adapt_struct(adapt)
    pix, n = _pixels(params, pixels)
    grad = np.zeros((n, 2), np.float64)
    valid = np.zeros(n, np.int32)
    rc = lib.orc_gradients(sens, ns, ptrs, ctypes.byref(prm), ctypes.byref(ad),
                           pix.ctypes.data if pix is not None else None, n, grad.ctypes.data, valid.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (code {rc})")
    return grad, valid


def steering(params, adapt, grad_plane, pixels=None, want_diag=False):
    """Stage 2 of CALPA (Sec. 5.4): steering matrices (n, 3) = (cxx, cxy, cyy)
    from a gradient plane of shape (out_h, out_w, 2); optionally the
    diagnostics (n, 5) = (s1, s2, theta, sigma, gamma)."""
    lib = _load()
    prm = _params_struct(params, False)
    ad = _adapt_struct(adapt)
    g = np.ascontiguousarray(np.asarray(grad_plane, np.float64))
    if g.shape != (int(params["out_h"]), int(params["out_w"]), 2):
        raise ValueError(f"gradient plane shape {g.shape} does not match the output grid")
    pix, n = _pixels(params, pixels)
    C = np.zeros((n, 3), np.float64)
    diag = np.zeros((n, 5), np.float64) if want_diag else None
    rc = lib.orc_steering(ctypes.byref(prm), ctypes.byref(ad), g.ctypes.data,
                          pix.ctypes.data if pix is not None else None, n, C.ctypes.data,
                          diag.ctypes.data if diag is not None else None)
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (code {rc})")
    return (C, diag) if want_diag else C


def reconstruct_steered(sensors, raws, params, C, pixels=None, want_fits=False, exhaustive=False):
    """Stage 3 of CALPA: LPA-ICI with the window exp(-d'Cd/h) (C: (n, 3) per
    listed pixel).  Returns the same dict as reconstruct()."""
    lib = _load()
    ns = len(sensors)
    structs = [_sensor_struct(d) for d in sensors]  # hold the calibration frames during the call
    sens = (_Sensor * ns)(*structs)
    planes = [np.ascontiguousarray(np.asarray(r), dtype=np.float64) for r in raws]
    ptrs = (ctypes.c_void_p * ns)(*[pl.ctypes.data for pl in planes])
    prm = _params_struct(params, exhaustive)
    pix, n = _pixels(params, pixels)
    Cm = np.ascontiguousarray(np.asarray(C, np.float64).reshape(n, 3))
    rgb = np.empty((n, 3), np.float64)
    smap = np.empty((n, 3), np.uint8)
    margin = np.empty((n, 3), np.float64)
    gap = np.empty((n, 3), np.float64)
    fits = np.zeros((n, 3, prm.n_scales, 3), FIT_DTYPE) if want_fits else None
    rc = lib.orc_reconstruct_steered(
        sens, ns, ptrs, ctypes.byref(prm), Cm.ctypes.data, pix.ctypes.data if pix is not None else None, n,
        rgb.ctypes.data, smap.ctypes.data, margin.ctypes.data, gap.ctypes.data,
        fits.ctypes.data if fits is not None else None,
    )
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (code {rc})")
    out = {"rgb": rgb, "scale_map": smap, "margin": margin, "gap": gap}
    if fits is not None:
        out["fits"] = fits
    return out


def neighbourhood(params, adapt, pixels):
    """Output pixels whose gradients the steering of the listed pixels reads."""
    q = int(dict(ADAPT_DEFAULTS, **(adapt or {}))["grad_halfwin"])
    W, H = int(params["out_w"]), int(params["out_h"])
    pix = np.asarray(pixels, np.int64).reshape(-1, 2)
    need = np.zeros((H, W), bool)
    for b in range(-q, q + 1):
        for a in range(-q, q + 1):
            u = np.clip(pix[:, 0] + a, 0, W - 1)
            v = np.clip(pix[:, 1] + b, 0, H - 1)
            need[v, u] = True
    v, u = np.nonzero(need)
    return np.stack([u, v], 1).astype(np.int32)


def reconstruct_adaptive(sensors, raws, params, adapt=None, pixels=None, want_fits=False, want_stages=False):
    """CALPA end to end (Sec. 5.4, 5.5): gradients at every pixel the listed
    pixels' analysis windows read, steering matrices, steered reconstruction."""
    W, H = int(params["out_w"]), int(params["out_h"])
    if pixels is None:
        v, u = np.mgrid[0:H, 0:W]
        pix = np.stack([u.ravel(), v.ravel()], 1).astype(np.int32)
    else:
        pix = np.asarray(pixels, np.int32).reshape(-1, 2)
    need = neighbourhood(params, adapt, pix)
    g, _ = gradients(sensors, raws, params, adapt, pixels=need)
    plane = np.zeros((H, W, 2), np.float64)
    plane[need[:, 1], need[:, 0]] = g
    C = steering(params, adapt, plane, pixels=pix)
    out = reconstruct_steered(sensors, raws, params, C, pixels=pix, want_fits=want_fits)
    if want_stages:
        out["grad_plane"] = plane
        out["C"] = C
    return out
