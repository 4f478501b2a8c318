"""Helpers for comparing the HIP path with the FP64 oracle.

Error metric (per output pixel and channel):
    e = |y_gpu - y_oracle| / max(|y_oracle|, f_floor),  f_floor = 1 / (g n_max),
i.e. relative error floored at one digital number of the most exposed sensor.

Value gate (compare): the GPU value is held against the oracle's fit at the
GPU's (order, radius) choice.
  * pivot ratio of that oracle fit >= tau_fp64 = 1e-3:  e <= 1e-4;
  * pivot ratio in [tau_inv, tau_fp64) (the FP64-fallback band):
    e <= max(1e-4, 2 kappa 1e-6) with kappa = 1 / rho, the perturbation bound
    of a fit whose moments carry 1e-6 relative error.
The library recomputes from FP64 moments every output whose FP32 rounding
bound could exceed 1e-4 and every fit below tau_fp64, so both bands are met by
construction; each band's count above 1e-4 and its maximum are reported.
FP16 storage of raw values of up to 12 bits is lossless, so the FP16 form is
held to the same gate; deeper ADCs are compared with an oracle fed the same
FP16-rounded samples (fp16_round_dn) at that gate, and with the exact oracle
at 2e-3 where the storage rounding cannot move the value further.

Decisions (which radius and order) are integers decided in floating point,
on FP32 moments for well-conditioned fits.  To first order a relative
perturbation eps of every moment term moves C0 by at most eps * sens_y, where
the oracle reports for each fit
    sens_y = |g|' |b|abs + |g|' |A|abs |C|      (g = A^-1 e0, C the coefficients,
                                                 |.|abs = sums of absolute terms),
so an interval end the ICI rule compares may move by max(1e-4 scale,
64 u sens_y) plus gamma times the sd bound (tol_value, tol_sd_rel).  Where the
oracle's decision is firm (firm_mask: every validity test away from tau by a
factor 10, every ICI gap wider than twice what the arithmetic can move an
interval end) the GPU must make the same decision.  Elsewhere either decision
is correct to within rounding.

The standard deviation of C0 (which sets the ICI intervals) is checked to
max(1e-3, 32 u sens_v / var) relative, sens_v being the same first-order
condition of the variance (half of it for the square root).
"""
from __future__ import annotations

import numpy as np

TAU_INV = 1e-5
TAU_FP64 = 1e-3
VALUE_TOL = 1e-4
U32 = 2.0 ** -24
# Standard deviation of the output (square root of the ICI variance): from the
# moments for well-conditioned fits, from a positive-term second pass over the
# samples below a pivot of 1e-2; either way a few u / rho relative.
SD_TOL = 1e-3
MARGIN_TIE = 1e-2
RHO_BAND = 10.0


def floor_of(sensors) -> float:
    return 1.0 / max(s["gain"] * s["exposure"] for s in sensors)


def tol_value(fits, floor):
    """How far the FP32 arithmetic may move C0 of a fit that decides an ICI
    step (an interval end; see the module docstring)."""
    return np.maximum(1e-4 * np.maximum(np.abs(fits["yhat"]), floor), 64 * U32 * fits["sens_y"])


def tol_sd_rel(fits):
    """Relative tolerance on the standard deviation of each fit's C0."""
    var = fits["var"]
    ok = np.isfinite(var) & (var > 0)
    rel = np.divide(32 * U32 * fits["sens_v"], var, out=np.full(var.shape, np.inf), where=ok)
    return np.maximum(SD_TOL, rel)


def firm_mask(orc: dict, order: int, sensors=None, gamma: float = 2.0, tau: float = TAU_INV) -> np.ndarray:
    """(n, 3) bool: the oracle's decisions are away from every threshold by more
    than the GPU arithmetic can move them.

    Validity: every fit with enough samples has its pivot ratio outside
    [tau / 10, 10 tau] (FP32 moments carry ~1e-6 absolute error in rho).
    ICI: the smallest gap |U - L| of the steps taken exceeds twice the largest
    uncertainty of an interval end among the valid radii, where an end moves by
    the C0 tolerance plus gamma times the sd tolerance."""
    fits = orc["fits"]  # (n, 3, S, 3)
    rho = fits["rho"][..., : order + 1]
    nb = np.array([1, 3, 6])[: order + 1]
    enough = fits["n"][..., : order + 1] >= nb
    near = enough & (rho > tau / RHO_BAND) & (rho < tau * RHO_BAND)
    firm = ~near.any(axis=(2, 3))
    floor = floor_of(sensors) if sensors is not None else 1.0
    f = fits[..., : order + 1]
    valid = f["valid"] == 1
    sd = np.sqrt(np.where(valid, np.maximum(f["var"], 0.0), 0.0))
    with np.errstate(invalid="ignore", over="ignore"):
        unc = np.where(valid, tol_value(f, floor) + gamma * tol_sd_rel(f) * sd, 0.0)
    code = orc["scale_map"]
    o_used = np.where(code == 0xFF, 0, code >> 4).astype(int)
    unc_used = np.take_along_axis(unc.max(axis=2), o_used[..., None], axis=2)[..., 0]
    gap = orc["gap"]
    firm &= ~(gap <= 2 * unc_used)
    return firm


def compare(gpu_rgb, gpu_map, orc: dict, sensors, order: int, f16_exact: bool = False,
            extra_tol: float = 0.0, gpu_sd=None, sd_tol: float = SD_TOL, alt_orc: dict | None = None):
    """Returns a dict of statistics; raises AssertionError on a parity failure.

    alt_orc: a second oracle run on other inputs (the exact samples where `orc`
    saw FP16-rounded ones); a value may then meet the gate against either (the
    FP64 refit of an output reads the raw frame, the FP32 pass the stored
    samples)."""
    y_o = orc["rgb"]
    map_o = orc["scale_map"]
    fits = orc["fits"]
    n = y_o.shape[0]
    gpu_rgb = np.asarray(gpu_rgb, np.float64).reshape(n, 3)
    gpu_map = np.asarray(gpu_map).reshape(n, 3)
    firm = firm_mask(orc, order, sensors)
    nan_o = np.isnan(y_o)
    nan_g = np.isnan(gpu_rgb)
    # NO_DATA must agree wherever the oracle is firm
    assert np.array_equal(nan_o[firm], nan_g[firm]), "NaN (no valid fit) masks differ"
    dif = np.nonzero(firm & (map_o != gpu_map))
    if dif[0].size:
        p, c = dif[0][0], dif[1][0]
        f = fits[p, c]
        detail = "; ".join(
            f"m{m}o{o}: y={f[m, o]['yhat']:.6g} sd={np.sqrt(max(f[m, o]['var'], 0)):.4g} rho={f[m, o]['rho']:.2e} "
            f"n={f[m, o]['n']} ok={f[m, o]['valid']}" for m in range(f.shape[0]) for o in range(order + 1))
        raise AssertionError(
            f"decisions differ at {dif[0].size} firm entries; first pixel {p} ch {c}: gpu code "
            f"{gpu_map[p, c]:#x} value {gpu_rgb[p, c]!r}, oracle code {map_o[p, c]:#x} margin "
            f"{orc['margin'][p, c]:.3g}; {detail}")
    # value to compare against: oracle fit at the GPU's (order, radius)
    ref = y_o.copy()
    rho = np.ones_like(y_o)
    sens = np.zeros_like(y_o)
    idx = np.nonzero(gpu_map != 0xFF)
    o_g = (gpu_map[idx] >> 4).astype(int)
    m_g = (gpu_map[idx] & 0xF).astype(int)
    chosen = fits[idx[0], idx[1], m_g, o_g]
    ref[idx] = chosen["yhat"]
    rho[idx] = chosen["rho"]
    sens[idx] = chosen["sens_y"]
    both = ~np.isnan(ref) & ~nan_g
    fl = floor_of(sensors)
    scale = np.maximum(np.abs(ref), fl)
    err = np.abs(gpu_rgb - ref) / scale
    if alt_orc is not None:
        alt = alt_orc["rgb"].copy()
        alt[idx] = alt_orc["fits"][idx[0], idx[1], m_g, o_g]["yhat"]
        with np.errstate(invalid="ignore"):
            err = np.fmin(err, np.abs(gpu_rgb - alt) / np.maximum(np.abs(alt), fl))
    hi = rho >= TAU_FP64
    with np.errstate(divide="ignore"):
        band_tol = np.maximum(VALUE_TOL, 2e-6 / np.maximum(rho, 1e-300))
    tol_rel = np.where(hi, VALUE_TOL, band_tol) + extra_tol
    bad = both & (err > tol_rel)
    if bad.any():
        i = np.argmax(np.where(bad, err / tol_rel, -1).ravel())
        p, c = np.unravel_index(i, err.shape)
        raise AssertionError(
            f"{np.count_nonzero(bad)} values outside tolerance ({np.count_nonzero(bad & hi)} with rho >= tau_fp64); "
            f"worst pixel {p} ch {c}: gpu {gpu_rgb[p, c]!r} oracle {ref[p, c]!r} e={err[p, c]:.3e} "
            f"rho={rho[p, c]:.3e} sens_y={sens[p, c]:.3e} code={gpu_map[p, c]}")
    # a GPU NaN where the oracle has a value (or vice versa) is allowed only off-firm
    mism = (nan_g != np.isnan(ref)) & ~firm
    sd_stats = {}
    if gpu_sd is not None:
        sd_g = np.asarray(gpu_sd, np.float64).reshape(n, 3)
        sd_o = np.full_like(y_o, np.nan)
        sd_o[idx] = np.sqrt(np.maximum(chosen["var"], 0.0))
        lim_all = np.full_like(y_o, sd_tol)
        lim_all[idx] = tol_sd_rel(chosen)
        okv = both & (sd_o > 0)
        esd = np.abs(sd_g[okv] - sd_o[okv]) / sd_o[okv]
        if esd.size:
            sd_stats = {"sd_err_max": float(esd.max()), "sd_err_p50": float(np.median(esd))}
            lim = lim_all[okv]
            if np.any(esd > lim):
                k = np.argmax(esd / lim)
                raise AssertionError(f"standard deviation off by {esd[k]:.3e} (relative) at rho={rho[okv][k]:.3e} "
                                     f"gpu {sd_g[okv][k]!r} oracle {sd_o[okv][k]!r}")
        assert np.all(np.isnan(sd_g[nan_g])), "sd must be NaN where there is no value"
    e_ok = err[both]
    cond = (np.abs(gpu_rgb - ref) / np.maximum(U32 * sens, 1e-300))[both]
    hb, lb = both & hi, both & ~hi
    return {
        "above_1e-4_rho_ge_tau64": int(np.count_nonzero(err[hb] > VALUE_TOL)),
        "err_max_rho_ge_tau64": float(err[hb].max()) if hb.any() else 0.0,
        "n_rho_lt_tau64": int(np.count_nonzero(lb)),
        "above_1e-4_rho_lt_tau64": int(np.count_nonzero(err[lb] > VALUE_TOL)),
        "err_max_rho_lt_tau64": float(err[lb].max()) if lb.any() else 0.0,
        **sd_stats,
        "agree_frac": float(np.mean(map_o == gpu_map)),
        "above_1e-4": int(np.count_nonzero(e_ok > 1e-4)),
        "err_over_u_sens_max": float(cond.max()) if cond.size else 0.0,
        "n": int(n * 3), "firm_frac": float(firm.mean()), "nan": int(nan_o.sum()),
        "decision_mismatch_unfirm": int(np.count_nonzero(map_o != gpu_map)),
        "nan_mismatch_unfirm": int(mism.sum()),
        "err_max": float(e_ok.max()) if e_ok.size else 0.0,
        "err_p50": float(np.median(e_ok)) if e_ok.size else 0.0,
        "err_p999": float(np.quantile(e_ok, 0.999)) if e_ok.size else 0.0,
    }


def fp16_offset(sensor: dict) -> float:
    """Offset of the FP16 storage form: 2^(bits-1) for ADCs of up to 12 bits
    (every raw value is then stored exactly), the black level beyond."""
    bits = sensor.get("bit_depth", 12)
    return 2.0 ** (bits - 1) if bits <= 12 else float(np.float32(sensor["black_level"]))


def fp16_round_dn(raw_u16: np.ndarray, sensor: dict):
    """Input for an oracle that sees exactly what the FP16 storage form stores.

    Returns (dn, sensor'): dn = o + fp16((y - o) 2^-B) 2^B (round-to-nearest-
    even, o = fp16_offset), +Inf where the raw sample is saturated, and
    sensor' = sensor with the saturation test moved to +Inf, so masking follows
    the raw value exactly as the pre-pass does."""
    o = fp16_offset(sensor)
    scale = 2.0 ** sensor.get("bit_depth", 12)
    y = raw_u16.astype(np.float64)
    v = ((y - o) / scale).astype(np.float16).astype(np.float64)
    dn = np.where(y >= sensor["saturation"], np.inf, o + v * scale)
    return dn, dict(sensor, saturation=1e300)
