"""Benchmark: HDR output Mpixel/s of LPA + ICI reconstruction on one MI355X.

Workload (one step = one reconstruction of one frame, the whole hot path):
4 sensors x 2048 x 2048 raw uint16 (12-bit RGGB), exposures 1, 1/4, 1/16,
1/64, misregistration +-2 px / +-0.3 deg, Poisson-Gaussian noise, order-2 LPA
with ICI over radii {1, 2, 3, 4}, Gamma = 2, 2048 x 2048 RGB float32 output.
Synthetic seeded scene (random step edges + smooth gradients, radiance
log-uniform over [1e-2, 1e4]); inputs are resident in HBM before timing.
A frame is the fit launch plus the FP64 refit launch of the outputs whose
FP32 rounding bound exceeds 1e-4.

Reported: the optimised form (raw samples decoded straight into LDS by the
fit kernel, tuned tile) as `value`; the plain per-frame FP32 form (FP32
pre-pass planes + fixed 16x16 tile) beside it; the roofline of the fit kernel
from its own launch durations (HIP events around each fit launch, on the
launch stream); the FP64 oracle on a bounded band of the same frame on the
host cores (one core, and every core of the process's share).  More legs:
the small frame (3 x 256^2, order 1, one radius), the FP16-storage resample
of the small rig to 4096^2, CALPA, calibration frames, pre-computed weights
on a registered rig, temporal LPA over the current and previous frame, a batch of 64 mixed frames in one persistent graph
launch (checked bit-for-bit against the same frames one plain launch each),
and a served run of 8 cameras with Poisson arrivals at 30 fps each (60 s by
default) reporting p50 / p99 frame latency.  Batched and served frames are
cut from the full capture (random even crop offsets, random subsets of 2-4 of
its sensors, so random exposure sets drawn from its four exposures): new
captures of that size take tens of seconds each on the host.

Every leg also reports the fraction of outputs recomputed in FP64 and, when
the oracle leg runs, the error of sampled outputs against the FP64 oracle:
    e = |y_gpu - y_oracle| / max(|y_oracle|, 1 / (g n_max))
with y_oracle the oracle's fit at the GPU's (order, radius) choice, split by
the pivot ratio of that fit (>= 1e-3: gate 1e-4; below: max(1e-4, 2e-6 / rho)),
plus the error against the oracle's own ICI result and the fraction of equal
decisions.  The oracle runs only inside the oracle leg, after the GPU legs.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--serve-seconds S]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3  # 256 CU x 4 SIMD x 16 lanes x 2 (packed) x 2 (FMA) x 2.4 GHz
HBM_TBPS = 8.0
RADII = [1.0, 2.0, 3.0, 4.0]
VALUE_GATE = 1e-4
TAU_FP64 = 1e-3
# host threads for the all-core oracle figure: the process's CPU share, at most 16
MAX_ORACLE_THREADS = 16

# Algorithmic FLOP per unit of work for an order-2 (n = 6) fit with ICI,
# counting FMA = 2 and mul/add/exp/rcp = 1:
FLOP_PER_SAMPLE = 19          # transform 8, |d|^2 3, quadratic basis 3, radiance 1, inverse variance 4
FLOP_PER_SAMPLE_SCALE = 111   # window 3, weight 1, basis products 5, A 42, b 12, ICI B 48
FLOP_PER_SOLVE = 294          # 6x6 equilibrated Cholesky + C0 + variance
# With pre-computed window weights the window, weight and basis products come
# from the tables: per sample the radiance and inverse variance (5), per
# sample-radius update w f and K w (2) and the 36 moment FMAs (72).
FLOP_PER_SAMPLE_STENCIL = 5
FLOP_PER_SAMPLE_SCALE_STENCIL = 74
# A steered window's test d^T C d takes two more operations than |d|^2.
FLOP_PER_SAMPLE_SCALE_STEER = FLOP_PER_SAMPLE_SCALE + 2

# The paper's own timings (Sec. 8), for context only: order-0 LPA with one
# fixed window, 4 sensors to a 2336 x 1752 output on a GeForce GTX 680, at
# 26 fps with pre-computed window weights and 7 fps with per-pixel weights.
PAPER_CONTEXT = {
    "source": "Sec. 8, CUDA implementation", "hardware": "NVIDIA GeForce GTX 680",
    "workload": "order-0 LPA, one fixed window, 4 sensors, 2336x1752 output",
    "fps_precomputed_weights": 26, "mpix_s_precomputed_weights": round(26 * 2336 * 1752 / 1e6, 1),
    "fps_per_pixel_weights": 7, "mpix_s_per_pixel_weights": round(7 * 2336 * 1752 / 1e6, 1),
    "note": "not this workload (order 2 with ICI over four radii here); no timing of order 1 or 2 or of ICI is given",
}


def algorithmic_flops(raws, sensors, n_pixels: int):
    """Per-frame algorithmic FLOPs: expected in-disc unmasked samples per output
    pixel (pi r^2 per sensor, times the sensor's unmasked fraction) times the
    per-unit costs, plus one solve per (channel, radius)."""
    import numpy as np

    unmasked = [float(np.mean(r < s["saturation"])) for r, s in zip(raws, sensors)]
    samples = sum(unmasked) * math.pi * RADII[-1] ** 2
    updates = sum(unmasked) * math.pi * sum(r * r for r in RADII)
    per_px = FLOP_PER_SAMPLE * samples + FLOP_PER_SAMPLE_SCALE * updates + FLOP_PER_SOLVE * 3 * len(RADII)
    return per_px * n_pixels, per_px, samples, updates


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("lpa_kernels.hip", "lpa_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1308_4908_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    e = d.get(kernel)
    if not e or e.get("kernel_source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def host_threads() -> tuple[int, int]:
    """(threads used for the all-core oracle figure, CPUs the process may run on)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    return max(1, min(MAX_ORACLE_THREADS, avail)), avail


# ---------------------------------------------------------------------------
# GPU side: legs record sampled outputs; the oracle leg checks them later.
# ---------------------------------------------------------------------------

def sample_pixels(w: int, h: int, n: int, seed: int):
    """n distinct output pixels (u, v), uniformly at random (all of them if n >= w h)."""
    import numpy as np

    if n >= w * h:
        v, u = np.mgrid[0:h, 0:w]
        return np.stack([u.ravel(), v.ravel()], 1).astype(np.int32)
    rng = np.random.default_rng(seed)
    idx = rng.choice(w * h, size=n, replace=False)
    return np.stack([idx % w, idx // w], 1).astype(np.int32)


def gather(torch, t, pix):
    """Values of an (H, W, C) device tensor at pixels (u, v), as numpy (n, C)."""
    idx_v = torch.from_numpy(pix[:, 1].astype("int64")).to(t.device)
    idx_u = torch.from_numpy(pix[:, 0].astype("int64")).to(t.device)
    return t[idx_v, idx_u].cpu().numpy()


class Check:
    """Sampled GPU outputs of one leg, checked against the oracle in the oracle leg."""

    def __init__(self, leg: dict, sensors, raws, params, pix, rgb, smap, steer=None, frames=None):
        self.leg, self.sensors, self.raws, self.params = leg, sensors, raws, params
        self.pix, self.rgb, self.smap, self.steer = pix, rgb, smap, steer
        self.frames = frames  # temporal legs: the raw planes of every frame (frames[0] is raws)


def frame_counts(stats, n_px: int) -> dict:
    s = stats.cpu().numpy()
    return {"fp64_outputs": int(s[0]), "fp64_frac": round(int(s[0]) / (3 * n_px), 6), "no_fit_outputs": int(s[1])}


def cut_frame(sensors, raws, keep, w, h, x0=0, y0=0):
    """A smaller frame cut from the capture: sensors `keep`, the w x h window
    at (x0, y0) (even, so the CFA phase is kept) of each plane, the affines
    shifted to the window's pixel coordinates."""
    ss, rr = [], []
    for i in keep:
        a = list(sensors[i]["affine"])
        a[2] += a[0] * x0 + a[1] * y0
        a[5] += a[3] * x0 + a[4] * y0
        ss.append(dict(sensors[i], width=w, height=h, affine=a))
        rr.append(raws[i][y0:y0 + h, x0:x0 + w])
    return ss, rr


def random_cut(rng, sensors, raws, w, h, n_sensors):
    """Random even crop offset and a random subset of n_sensors of the capture's sensors."""
    full = raws[0].shape
    x0 = 2 * int(rng.integers(0, (full[1] - w) // 2 + 1))
    y0 = 2 * int(rng.integers(0, (full[0] - h) // 2 + 1))
    keep = sorted(int(k) for k in rng.choice(len(sensors), size=n_sensors, replace=False))
    ss, rr = cut_frame(sensors, raws, keep, w, h, x0, y0)
    # the output grid follows the window: output pixel (u, v) sits at reference (u + x0, v + y0)
    return ss, rr, [1.0, 0.0, float(x0), 0.0, 1.0, float(y0)], keep


BATCH_SHAPES = [(1280, 720), (1920, 1080), (2048, 2048)]


def batch_leg(torch, ctx, Rig, sensors, raws, configs, n_frames, storage, checks, reps=3):
    """n_frames mixed frames in one persistent launch vs one plain launch each;
    every batched output must equal its plain per-frame output bit for bit."""
    import numpy as np

    rng = np.random.default_rng(4000)
    frames = []
    for i in range(n_frames):
        w, h = BATCH_SHAPES[int(rng.integers(0, 3))]
        ns = int(rng.integers(2, 5))
        order = int(rng.integers(1, 3))
        ss, rr, oa, keep = random_cut(rng, sensors, raws, w, h, ns)
        rig = Rig(ctx, ss)
        dev = [torch.from_numpy(np.ascontiguousarray(r)).cuda() for r in rr]
        p = configs.lpa_params(w, h, order, RADII, out_affine=oa, storage=storage)
        out = torch.empty((h, w, 3), device="cuda")
        smap = torch.empty((h, w, 3), dtype=torch.uint8, device="cuda")
        st = torch.zeros(2, dtype=torch.int64, device="cuda")
        frames.append((rig, dev, p, out, smap, st, ss, rr, [sensors[k]["exposure"] for k in keep]))
    n_px = sum(f[2]["out_w"] * f[2]["out_h"] for f in frames)
    rigs = [f[0] for f in frames]
    devs = [f[1] for f in frames]
    ps = [f[2] for f in frames]
    outs = [f[3] for f in frames]
    maps = [f[4] for f in frames]
    stats = [f[5] for f in frames]
    ctx.reconstruct_batch(rigs, devs, ps, outs, maps, stats=stats)  # builds the graph; counts and maps once
    torch.cuda.synchronize()
    fp64 = sum(int(s[0]) for s in (t.cpu().numpy() for t in stats))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.reconstruct_batch(rigs, devs, ps, outs)
    e1.record()
    torch.cuda.synchronize()
    ms_batch = e0.elapsed_time(e1) / reps
    batched = [(o.clone(), m.clone()) for o, m in zip(outs, maps)]
    for rig, dev, p, out, smap, *_ in frames:
        rig.reconstruct(dev, p, out, smap, plain=True)
    torch.cuda.synchronize()
    e0.record()
    for rig, dev, p, out, *_ in frames:
        rig.reconstruct(dev, p, out, plain=True)
    e1.record()
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1)
    same = 0
    for (bo, bm), out, smap in zip(batched, outs, maps):
        if torch.equal(bo.view(torch.int32), out.view(torch.int32)) and torch.equal(bm, smap):
            same += 1
    res = {"frames": n_frames, "mpix": round(n_px / 1e6, 2), "storage": storage,
           "batched_mpix_s": round(n_px / (ms_batch * 1e-3) / 1e6, 3), "batch_ms": round(ms_batch, 3),
           "plain_per_frame_mpix_s": round(n_px / (ms_plain * 1e-3) / 1e6, 3),
           "speedup": round(ms_plain / ms_batch, 3),
           "frames_bit_identical_to_per_frame": same,
           "fp64_frac": round(fp64 / (3 * n_px), 6),
           "exposure_sets": sorted({tuple(f[8]) for f in frames}).__len__(),
           "accuracy": None}
    # a few frames for the oracle check
    for k in (0, n_frames // 3, 2 * n_frames // 3):
        _, _, p, _, _, _, ss, rr, _ = frames[k]
        pix = sample_pixels(p["out_w"], p["out_h"], 1024, 4100 + k)
        checks.append(Check(res, ss, rr, p, pix, gather(torch, batched[k][0], pix), gather(torch, batched[k][1], pix)))
    del batched
    for r in rigs:
        r.close()
    return res


def serve_leg(torch, ctx, Rig, sensors, raws, configs, seconds, checks=None, n_cameras=8, rate=30.0):
    """Cameras with Poisson arrivals; frames submitted from pinned host memory."""
    import numpy as np

    cams = []
    for c in range(n_cameras):
        spec = configs.camera_spec(c)
        w, h = spec["width"], spec["height"]
        rng = np.random.default_rng(np.random.SeedSequence([spec["seed"], 13]))
        ss, rr, oa, _ = random_cut(rng, sensors, raws, w, h, spec["n_sensors"])
        rig = Rig(ctx, ss)
        host = [torch.from_numpy(np.ascontiguousarray(r)).pin_memory() for r in rr]
        p = configs.lpa_params(w, h, 2, RADII, out_affine=oa, storage="fp16")
        outs = [torch.empty((h, w, 3), device="cuda") for _ in range(6)]
        maps = [torch.empty((h, w, 3), dtype=torch.uint8, device="cuda") for _ in range(6)]
        arr = configs.poisson_arrivals(c, rate, seconds)
        cams.append((rig, host, p, outs, arr, maps, ss, rr))
    events = sorted((t, c) for c, cam in enumerate(cams) for t in cam[4])
    tickets = []
    t0 = time.monotonic_ns()
    k = [0] * n_cameras
    for t, c in events:
        due = t0 + int(t * 1e9)
        while True:
            now = time.monotonic_ns()
            if now >= due:
                break
            time.sleep(min(0.0005, (due - now) / 1e9))
        rig, host, p, outs, _, maps, _, _ = cams[c]
        out = outs[k[c] % len(outs)]
        smap = maps[k[c] % len(maps)]
        k[c] += 1
        tk = None
        while tk is None:
            tk = rig.submit(host, p, out, smap, arrival_ns=due, host=True)
        tickets.append((tk, p["out_w"] * p["out_h"]))
    ctx.drain()
    t_end = time.monotonic_ns()
    lat, px, done_last, fp64, n_out = [], 0, t0, 0, 0
    for tk, npx in tickets:
        r = ctx.poll(tk)
        if r.status == 0:
            lat.append((r.t_done_ns - r.t_arrival_ns) / 1e6)
            px += npx
            done_last = max(done_last, r.t_done_ns)
            fp64 += int(r.n_fp64)
            n_out += 3 * npx
    lat = np.asarray(lat)
    res = {"cameras": n_cameras, "seconds": seconds, "frames": len(tickets), "completed": int(lat.size),
           "served_mpix_s": round(px / ((done_last - t0) / 1e9) / 1e6, 2),
           "latency_p50_ms": round(float(np.percentile(lat, 50)), 3),
           "latency_p99_ms": round(float(np.percentile(lat, 99)), 3),
           "latency_max_ms": round(float(lat.max()), 3), "drain_ms": round((t_end - t0) / 1e6 - seconds * 1e3, 1),
           "fp64_frac": round(fp64 / max(n_out, 1), 6), "accuracy": None}
    if checks is not None:
        # every frame of a camera is the same capture: check the camera's last output
        for c in (0, n_cameras // 2):
            rig, host, p, outs, _, maps, ss, rr = cams[c]
            last = (k[c] - 1) % len(outs)
            pix = sample_pixels(p["out_w"], p["out_h"], 1024, 5100 + c)
            checks.append(Check(res, ss, rr, p, pix, gather(torch, outs[last], pix), gather(torch, maps[last], pix)))
    for cam in cams:
        cam[0].close()
    return res


# ---------------------------------------------------------------------------
# Oracle leg: the CPU baseline, and the accuracy of every leg's samples.
# ---------------------------------------------------------------------------

def run_oracle(oracle, sensors, raws64, params, pix, threads, want_fits=False, steer=None, frames64=None):
    """The oracle on the listed pixels, chunks spread over host threads (the
    oracle is reentrant and the C call releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    n_chunks = max(1, min(len(pix) // 256, 4 * threads))
    chunks = np.array_split(np.arange(len(pix)), n_chunks)

    def one(ix):
        if frames64 is not None:
            return oracle.reconstruct_temporal(sensors, frames64, params, pixels=pix[ix], want_fits=want_fits)
        if steer is not None:
            return oracle.reconstruct_steered(sensors, raws64, params, steer[ix], pixels=pix[ix], want_fits=want_fits)
        return oracle.reconstruct(sensors, raws64, params, pixels=pix[ix], want_fits=want_fits)

    if threads == 1 or n_chunks == 1:
        parts = [one(ix) for ix in chunks]
    else:
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(one, chunks))
    out = {k: np.concatenate([p[k] for p in parts]) for k in ("rgb", "scale_map")}
    if want_fits:
        out["fits"] = np.concatenate([p["fits"] for p in parts])
    return out


def accuracy(orc, rgb, smap, sensors) -> dict:
    """Error statistics of sampled GPU outputs against the oracle (see the module docstring)."""
    import numpy as np

    floor = 1.0 / max(s["gain"] * s["exposure"] for s in sensors)
    y_o, map_o, fits = orc["rgb"], orc["scale_map"], orc["fits"]
    g = np.asarray(rgb, np.float64).reshape(y_o.shape)
    gm = np.asarray(smap).reshape(y_o.shape)
    ref = y_o.copy()
    rho = np.ones_like(y_o)
    idx = np.nonzero(gm != 0xFF)
    chosen = fits[idx[0], idx[1], (gm[idx] & 0xF).astype(int), (gm[idx] >> 4).astype(int)]
    ref[idx] = chosen["yhat"]
    rho[idx] = chosen["rho"]
    both = ~np.isnan(ref) & ~np.isnan(g)
    err = np.where(both, np.abs(g - ref) / np.maximum(np.abs(ref), floor), 0.0)
    hi = both & (rho >= TAU_FP64)
    lo = both & (rho < TAU_FP64)
    with np.errstate(divide="ignore"):
        lo_gate = np.maximum(VALUE_GATE, 2e-6 / np.maximum(rho, 1e-300))
    both_f = ~np.isnan(y_o) & ~np.isnan(g)
    err_f = np.abs(g - y_o)[both_f] / np.maximum(np.abs(y_o[both_f]), floor)
    e = err[both]
    return {
        "values": int(g.size), "compared": int(both.sum()),
        "err_max": float(e.max()) if e.size else 0.0,
        "err_p50": float(np.median(e)) if e.size else 0.0,
        "err_p999": float(np.quantile(e, 0.999)) if e.size else 0.0,
        "above_1e-4_rho_ge_1e-3": int(np.count_nonzero(err[hi] > VALUE_GATE)),
        "err_max_rho_ge_1e-3": float(err[hi].max()) if hi.any() else 0.0,
        "n_rho_lt_1e-3": int(lo.sum()),
        "err_max_rho_lt_1e-3": float(err[lo].max()) if lo.any() else 0.0,
        "above_band_gate_rho_lt_1e-3": int(np.count_nonzero(err[lo] > lo_gate[lo])),
        "decisions_equal_frac": float(np.mean(map_o == gm)),
        "no_fit_mismatch": int(np.count_nonzero(np.isnan(y_o) != np.isnan(g))),
        "err_vs_oracle_ici_result_max": float(err_f.max()) if err_f.size else 0.0,
        "err_vs_oracle_ici_result_p999": float(np.quantile(err_f, 0.999)) if err_f.size else 0.0,
        "gate_met": bool(np.count_nonzero(err[hi] > VALUE_GATE) == 0 and
                         np.count_nonzero(err[lo] > lo_gate[lo]) == 0),
    }


def oracle_leg(sensors, raws, params, rows: int, checks, threads: int, avail: int, all_core_rows: int):
    """The FP64 oracle timed single-threaded on a band of `rows` output rows,
    then on `all_core_rows` rows over `threads` host threads; then every leg's
    sampled outputs against it."""
    import numpy as np

    import oracle

    raws64 = [np.ascontiguousarray(r, dtype=np.float64) for r in raws]
    w = params["out_w"]

    def band(n_rows):
        v0 = params["out_h"] // 2 - n_rows // 2
        u, v = np.meshgrid(np.arange(w), np.arange(v0, v0 + n_rows))
        return np.stack([u.ravel(), v.ravel()], 1).astype(np.int32)

    pix = band(rows)
    t0 = time.perf_counter()
    oracle.reconstruct(sensors, raws64, params, pixels=pix)
    dt = time.perf_counter() - t0
    pix_a = band(all_core_rows)
    t0 = time.perf_counter()
    run_oracle(oracle, sensors, raws64, params, pix_a, threads)
    dt_a = time.perf_counter() - t0
    base = {"value": round(pix.shape[0] / dt / 1e6, 5), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows} rows x {w} px ({pix.shape[0]} output pixels) of the same frame, "
                      f"{dt:.1f} s single-threaded FP64",
            "cpu_model": cpu_model(),
            "all_core": {"value": round(pix_a.shape[0] / dt_a / 1e6, 5), "unit": "Mpixel/s", "threads": threads,
                         "cpus_available": avail,
                         "sample": f"{all_core_rows} rows x {w} px ({pix_a.shape[0]} output pixels), {dt_a:.1f} s, "
                                   f"{threads} threads over row chunks"}}
    t0 = time.perf_counter()
    by_leg = {}
    for ck in checks:
        r64 = [np.ascontiguousarray(r, dtype=np.float64) for r in ck.raws]
        f64 = None
        if ck.frames is not None:
            f64 = [r64] + [[np.ascontiguousarray(r, dtype=np.float64) for r in fr] for fr in ck.frames[1:]]
        orc = run_oracle(oracle, ck.sensors, r64, ck.params, ck.pix, threads, want_fits=True, steer=ck.steer,
                         frames64=f64)
        by_leg.setdefault(id(ck.leg), (ck.leg, []))[1].append((orc, ck))
    for leg, items in by_leg.values():
        # pool the leg's samples (several frames for batched and served legs)
        rgb = np.concatenate([c.rgb.reshape(-1, 3) for _, c in items])
        smap = np.concatenate([c.smap.reshape(-1, 3) for _, c in items])
        orc = {k: np.concatenate([o[k] for o, _ in items]) for k in ("rgb", "scale_map", "fits")}
        floor_sensors = [s for _, c in items for s in c.sensors]
        acc = accuracy(orc, rgb, smap, floor_sensors)
        acc["sample"] = f"{len(items)} frame(s), {rgb.shape[0]} random output pixels"
        leg["accuracy"] = acc
    base["accuracy_check_s"] = round(time.perf_counter() - t0, 1)
    return base


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--cpu-rows", type=int, default=160)
    ap.add_argument("--cpu-rows-all-core", type=int, default=640)
    ap.add_argument("--samples", type=int, default=16384, help="sampled output pixels of the headline frame")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-calpa", action="store_true")
    ap.add_argument("--no-precomputed", action="store_true")
    ap.add_argument("--no-calib", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--no-resample", action="store_true")
    ap.add_argument("--no-temporal", action="store_true")
    ap.add_argument("--batch-frames", type=int, default=64)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this size (HBM counter calibration)")
    ap.add_argument("--peak-probe", action="store_true",
                    help="only run the FMA issue-rate probe (vector-ALU ceiling without packed FP32)")
    args = ap.parse_args()
    if args.peak_probe:
        import subprocess

        probe = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1308_4908_amd", "peak_probe")
        if not os.path.exists(probe):
            sys.exit(f"{probe} is not built; run __graft_entry__.build() first")
        sys.exit(subprocess.run([probe]).returncode)
    if args.copy_probe_mib:
        import torch

        n = args.copy_probe_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU (--gpus 1): frames and output row bands shard across GPUs without "
              "collectives, but that form is not run here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1308_4908_amd import Context, Rig
    from synth import configs

    def say(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    size = args.size
    sensors, scene, params = configs.full(size=size)
    say(f"generating {len(sensors)} x {size}^2 synthetic frame")
    raws = configs.capture_all(scene, sensors, 2000)
    n_px = params["out_w"] * params["out_h"]
    flops, flop_px, samples_px, updates_px = algorithmic_flops(raws, sensors, n_px)
    checks = []

    ctx = Context(0)
    rig = Rig(ctx, sensors)
    dev = [torch.from_numpy(r).cuda() for r in raws]
    out = torch.empty((params["out_h"], params["out_w"], 3), dtype=torch.float32, device="cuda")
    smap = torch.empty((params["out_h"], params["out_w"], 3), dtype=torch.uint8, device="cuda")
    stats = torch.zeros(2, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(plain: bool, steps: int, warmup: int, prm=None, rig_=None, dev_=None, out_=None, kernels=False):
        prm = params if prm is None else prm
        rig_ = rig if rig_ is None else rig_
        dev_ = dev if dev_ is None else dev_
        out_ = out if out_ is None else out_
        for _ in range(warmup):
            rig_.reconstruct(dev_, prm, out_, plain=plain)
        torch.cuda.synchronize()
        if kernels:
            ctx.set_kernel_timing(True)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        evs[0].record(stream)
        for i in range(steps):
            rig_.reconstruct(dev_, prm, out_, plain=plain)
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = None
        if kernels:
            kt = ctx.kernel_times()
            ctx.set_kernel_timing(False)
        per = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
        return sum(per) / steps, wall, per, kt

    def one_pass(prm, rig_, dev_, out_, smap_, plain=False, steer=None):
        """One untimed reconstruction with the scale map and the FP64 counts."""
        st = torch.zeros(2, dtype=torch.int64, device="cuda")
        rig_.reconstruct(dev_, prm, out_, smap_, plain=plain, stats=st, steer_map=steer)
        torch.cuda.synchronize()
        return st

    say("tuning the launch shape for this frame class")
    tr = rig.autotune(dev, params, out, reps=3)
    tuned = {"tile": f"{tr.tile_w}x{tr.tile_h}", "waves_per_simd_budget": 4 if tr.occupancy == 4 else 3,
             "candidates": tr.n_candidates, "ms_best": round(tr.ms_best, 4), "ms_default": round(tr.ms_default, 4)}
    say("timing the optimised form")
    ms, wall, per, kt = timed(False, args.steps, args.warmup, kernels=True)
    value = n_px / (ms * 1e-3) / 1e6
    head = {"accuracy": None}
    head.update(frame_counts(one_pass(params, rig, dev, out, smap), n_px))
    pix_h = sample_pixels(params["out_w"], params["out_h"], args.samples, 2100)
    head_rgb, head_map = gather(torch, out, pix_h), gather(torch, smap, pix_h)
    checks.append(Check(head, sensors, raws, params, pix_h, head_rgb, head_map))
    plain = None
    if not args.no_plain:
        say("timing the plain FP32 form")
        ms_p, _, _, _ = timed(True, max(3, args.steps // 2), 1)
        one_pass(params, rig, dev, out, smap, plain=True)
        p_rgb, p_map = gather(torch, out, pix_h), gather(torch, smap, pix_h)
        plain = {"value": round(n_px / (ms_p * 1e-3) / 1e6, 3), "unit": "Mpixel/s", "ms_per_frame": round(ms_p, 4),
                 "form": "FP32 pre-pass planes + fit, fixed 16x16 tile",
                 "samples_bit_identical_to_optimised": bool(
                     np.array_equal(p_rgb.view(np.int32), head_rgb.view(np.int32)) and np.array_equal(p_map, head_map))}
    small = None
    if not args.no_small:
        # the small frame: 3 x 256^2, order 1, one radius 2, 256^2 output
        s_sensors, s_scene, s_params = configs.small()
        s_raws = configs.capture_all(s_scene, s_sensors, 1000)
        s_rig = Rig(ctx, s_sensors)
        s_dev = [torch.from_numpy(r).cuda() for r in s_raws]
        s_out = torch.empty((256, 256, 3), device="cuda")
        s_map = torch.empty((256, 256, 3), dtype=torch.uint8, device="cuda")
        say("timing the small frame (3 x 256^2, order 1, one radius)")
        ms_s, _, _, _ = timed(False, 50, 5, s_params, s_rig, s_dev, s_out)
        small = {"workload": "3 x 256x256 raw uint16 12-bit RGGB, exposures 1, 1/8, 1/64, +-1.5 px / +-0.2 deg, "
                             "order-1 LPA, one radius 2, 256x256 RGB fp32 output",
                 "value": round(256 * 256 / (ms_s * 1e-3) / 1e6, 3), "unit": "Mpixel/s", "ms_per_frame": round(ms_s, 4),
                 "accuracy": None}
        small.update(frame_counts(one_pass(s_params, s_rig, s_dev, s_out, s_map), 256 * 256))
        pix = sample_pixels(256, 256, 256 * 256, 0)
        checks.append(Check(small, s_sensors, s_raws, s_params, pix, gather(torch, s_out, pix), gather(torch, s_map, pix)))
        s_rig.close()
        del s_dev, s_out, s_map
    resample = None
    if not args.no_resample:
        # the small rig resampled to 4096^2, samples stored as FP16 normalised radiance
        r_sensors, r_scene, r_params = configs.resampled()
        r_raws = configs.capture_all(r_scene, r_sensors, 3000)
        r_rig = Rig(ctx, r_sensors)
        r_dev = [torch.from_numpy(r).cuda() for r in r_raws]
        H, W = r_params["out_h"], r_params["out_w"]
        r_out = torch.empty((H, W, 3), device="cuda")
        r_map = torch.empty((H, W, 3), dtype=torch.uint8, device="cuda")
        say("timing the FP16-storage resample (3 x 256^2 -> 4096^2)")
        ms_r, _, _, _ = timed(False, 10, 2, r_params, r_rig, r_dev, r_out)
        resample = {"workload": "3 x 256x256 raw uint16 12-bit (the small rig), output 4096x4096 "
                                "(X = (u + 1/2)/16 - 1/2), order-1 LPA radius 2, FP16 normalised radiance storage "
                                "(pre-pass), FP32 moments, FP64 solves and refits where flagged",
                    "value": round(H * W / (ms_r * 1e-3) / 1e6, 3), "unit": "Mpixel/s",
                    "ms_per_frame": round(ms_r, 4), "accuracy": None}
        resample.update(frame_counts(one_pass(r_params, r_rig, r_dev, r_out, r_map), H * W))
        pix = sample_pixels(W, H, 8192, 3100)
        checks.append(Check(resample, r_sensors, r_raws, r_params, pix, gather(torch, r_out, pix),
                            gather(torch, r_map, pix)))
        r_rig.close()
        del r_dev, r_out, r_map
    calpa = None
    if not args.no_calpa:
        # adaptive anisotropic LPA (Sec. 5.4-5.5): the paper's regularisers and
        # structure sensitivity, gradient fit at radius 2 (order 1), 5x5
        # gradient analysis window, eigenvalues of C within [1/4, 4]
        adapt = {"alpha": 0.005, "lambda1": 1.0, "lambda2": 0.001, "grad_radius": 2.0, "grad_order": 1,
                 "grad_halfwin": 2, "max_stretch": 2.0}
        pc = dict(params, mode="calpa", adapt=adapt)
        say("timing CALPA (gradient, steering and steered-fit passes)")
        ms_c, _, _, kt_c = timed(False, max(3, args.steps // 2), 1, pc, kernels=True)
        calpa = {"value": round(n_px / (ms_c * 1e-3) / 1e6, 3), "unit": "Mpixel/s", "ms_per_frame": round(ms_c, 4),
                 "vs_lpa": round(ms_c / ms, 3), "params": adapt,
                 "steered_fit_ms_per_launch": round(kt_c.fit_ms / max(kt_c.n_fit, 1), 4),
                 "form": "G gradient pass + steering pass + steered fit (+ FP64 refit), 16x16 tiles",
                 "accuracy": None}
        steer = torch.empty((params["out_h"], params["out_w"], 4), device="cuda")
        calpa.update(frame_counts(one_pass(pc, rig, dev, out, smap, steer=steer), n_px))
        # the steered fit's algorithmic work: the ellipse d^T C d < r^2 holds
        # pi r^2 / sqrt(det C) of a sensor's pixels, so samples and updates
        # scale by the frame's mean 1 / sqrt(det C)
        det = steer[..., 0].double() * steer[..., 2].double() - steer[..., 1].double() ** 2
        area = float(torch.mean(torch.rsqrt(det)).item())
        c_flop_px = (FLOP_PER_SAMPLE * samples_px * area + FLOP_PER_SAMPLE_SCALE_STEER * updates_px * area +
                     FLOP_PER_SOLVE * 3 * len(RADII))
        c_ms_k = kt_c.fit_ms / max(kt_c.n_fit, 1)
        c_ach = c_flop_px * n_px / (c_ms_k * 1e-3) / 1e12
        calpa["roofline"] = {"bound": "alu", "kernel": "fit_kernel_steer<order 2, ICI, raw uint16>",
                             "achieved": round(c_ach, 3), "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                             "frac": round(c_ach / PEAK_FP32_VECTOR_TFLOPS, 4), "flop_per_pixel": round(c_flop_px, 1),
                             "mean_window_area_vs_isotropic": round(area, 4), "kernel_ms_per_launch": round(c_ms_k, 4)}
        pix = sample_pixels(params["out_w"], params["out_h"], 4096, 2200)
        c_steer = gather(torch, steer, pix)[:, :3].astype(np.float64)
        checks.append(Check(calpa, sensors, raws, pc, pix, gather(torch, out, pix), gather(torch, smap, pix),
                            steer=c_steer))
        calpa["accuracy_note"] = "steered fit against the oracle's steered fit on the GPU's steering matrices"
        del steer
    calib = None
    if not args.no_calib:
        # per-pixel calibration frames (Sec. 6) on every sensor of the same
        # frame: bias frame, non-uniformity, readout variance, saturation frame
        # and 0.1 % defects, drawn at random around the scalar model
        rng = np.random.default_rng(6000)
        c_sensors = []
        for s in sensors:
            shape = (s["height"], s["width"])
            c_sensors.append(dict(s, calib={
                "bias": rng.uniform(60.0, 68.0, shape), "prnu": rng.uniform(0.95, 1.05, shape),
                "read_var": rng.uniform(7.0, 11.0, shape), "sat": np.full(shape, s["saturation"]),
                "defect": (rng.random(shape) < 1e-3).astype(np.uint8)}))
        say("timing with per-pixel calibration frames")
        c_rig = Rig(ctx, c_sensors)
        ms_cal, _, _, _ = timed(False, max(3, args.steps // 2), 1, None, c_rig, dev)
        calib = {"value": round(n_px / (ms_cal * 1e-3) / 1e6, 3), "unit": "Mpixel/s", "ms_per_frame": round(ms_cal, 4),
                 "vs_scalar_model": round(ms_cal / ms, 3),
                 "form": "same frame and launch with a resident (b_i, a_i, Var r_i, saturation_i) plane per "
                         "sensor read during staging (16 B per staged sample)", "accuracy": None}
        calib.update(frame_counts(one_pass(params, c_rig, dev, out, smap), n_px))
        pix = sample_pixels(params["out_w"], params["out_h"], 4096, 2300)
        checks.append(Check(calib, c_sensors, raws, params, pix, gather(torch, out, pix), gather(torch, smap, pix)))
        c_rig.close()
    pre = None
    if not args.no_precomputed:
        # the paper's fast path for registered sensors (Sec. 8): the same
        # workload on the rig without rotation, general kernel vs pre-computed
        # window weights
        say("generating the aligned (translation-only) frame")
        a_sensors, a_scene, a_params = configs.aligned(size=size)
        a_raws = configs.capture_all(a_scene, a_sensors, 2000)
        a_rig = Rig(ctx, a_sensors)
        a_dev = [torch.from_numpy(r).cuda() for r in a_raws]
        say("timing pre-computed weights vs the general kernel")
        ms_g, _, _, _ = timed(False, max(3, args.steps // 2), 1, a_params, a_rig, a_dev)
        sp = dict(a_params, precomputed_weights=True)
        ms_s, _, _, kt_s = timed(False, max(3, args.steps // 2), 2, sp, a_rig, a_dev, kernels=True)
        _, _, a_samples, a_updates = algorithmic_flops(a_raws, a_sensors, n_px)
        s_flop_px = (FLOP_PER_SAMPLE_STENCIL * a_samples + FLOP_PER_SAMPLE_SCALE_STENCIL * a_updates +
                     FLOP_PER_SOLVE * 3 * len(RADII))
        s_ms_k = kt_s.fit_ms / max(kt_s.n_fit, 1)
        s_ach = s_flop_px * n_px / (s_ms_k * 1e-3) / 1e12
        pre = {"workload": f"aligned rig: {len(a_sensors)} x {size}x{size} raw uint16, translation-only sensor maps, "
                           "same exposures, noise and LPA parameters", "value": round(n_px / (ms_s * 1e-3) / 1e6, 3),
               "unit": "Mpixel/s", "ms_per_frame": round(ms_s, 4), "general_kernel_ms_same_frame": round(ms_g, 4),
               "speedup_vs_general": round(ms_g / ms_s, 3),
               "form": "fit_kernel_stencil (per-parity tables of K x monomials, scalar loads), 16x16 tiles",
               "roofline": {"bound": "alu", "achieved": round(s_ach, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                            "unit": "TFLOP/s", "frac": round(s_ach / PEAK_FP32_VECTOR_TFLOPS, 4),
                            "flop_per_pixel": round(s_flop_px, 1), "kernel_ms_per_launch": round(s_ms_k, 4)},
               "accuracy": None}
        pre.update(frame_counts(one_pass(sp, a_rig, a_dev, out, smap), n_px))
        pix = sample_pixels(params["out_w"], params["out_h"], 4096, 2400)
        checks.append(Check(pre, a_sensors, a_raws, sp, pix, gather(torch, out, pix), gather(torch, smap, pix)))
        a_rig.close()
        del a_dev
    temporal = None
    if not args.no_temporal:
        # temporal LPA over the current and the previous frame of the same
        # static scene (new noise): 4 sensors x 2 frames = 8 staged sensors,
        # one temporal scale per radius
        say("generating the previous frame for the temporal leg")
        prev = configs.capture_all(scene, sensors, 2001)
        t_dev = [dev, [torch.from_numpy(r).cuda() for r in prev]]
        tp = dict(params, h_t=[0.5, 1.0, 2.0, 4.0])
        say("timing temporal LPA (4 sensors x 2 frames)")
        for _ in range(2):
            rig.reconstruct_temporal(t_dev, tp, out)
        torch.cuda.synchronize()
        n_t = max(3, args.steps // 2)
        ctx.set_kernel_timing(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n_t):
            rig.reconstruct_temporal(t_dev, tp, out)
        e1.record(stream)
        torch.cuda.synchronize()
        kt_t = ctx.kernel_times()
        ctx.set_kernel_timing(False)
        ms_t = e0.elapsed_time(e1) / n_t
        t_flops, t_flop_px, _, t_updates = algorithmic_flops(raws + prev, sensors + sensors, n_px)
        t_flops += t_updates * n_px  # the temporal factor: one product per update
        t_ms_k = kt_t.fit_ms / max(kt_t.n_fit, 1)
        t_ach = t_flops / (t_ms_k * 1e-3) / 1e12
        temporal = {"workload": f"the headline rig over 2 frames (current + previous, same static scene, new noise): "
                                f"4 sensors x 2 x {size}x{size} raw uint16, h_t = 0.5/1/2/4 frames^2 per radius",
                    "value": round(n_px / (ms_t * 1e-3) / 1e6, 3), "unit": "Mpixel/s", "ms_per_frame": round(ms_t, 4),
                    "vs_single_frame": round(ms_t / ms, 3),
                    "form": "fit_kernel_temporal (every frame's sensors staged as sensors of their own) + FP64 refit",
                    "roofline": {"bound": "alu", "achieved": round(t_ach, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                                 "unit": "TFLOP/s", "frac": round(t_ach / PEAK_FP32_VECTOR_TFLOPS, 4),
                                 "flop_per_pixel": round(t_flops / n_px, 1), "kernel_ms_per_launch": round(t_ms_k, 4)},
                    "accuracy": None}
        st = torch.zeros(2, dtype=torch.int64, device="cuda")
        rig.reconstruct_temporal(t_dev, tp, out, smap, stats=st)
        torch.cuda.synchronize()
        temporal.update(frame_counts(st, n_px))
        pix = sample_pixels(params["out_w"], params["out_h"], 4096, 2500)
        checks.append(Check(temporal, sensors, raws, tp, pix, gather(torch, out, pix), gather(torch, smap, pix),
                            frames=[raws, prev]))
        del t_dev
    fit_ms = kt.fit_ms / max(kt.n_fit, 1)
    refit_ms = kt.refit_ms / max(kt.n_refit, 1) if kt.n_refit else 0.0
    achieved = flops / (fit_ms * 1e-3) / 1e12
    traffic = measured_traffic("fit_kernel<2,ICI,RAW_U16>")
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4), "traffic": traffic,
            "kernel": "fit_kernel<order 2, ICI, raw uint16>",
            "kernel_ms_per_launch": round(fit_ms, 4), "launches_timed": int(kt.n_fit),
            "flop_per_launch": round(flops), "flop_per_pixel": round(flop_px, 1),
            "samples_per_pixel": round(samples_px, 2), "sample_scale_updates_per_pixel": round(updates_px, 2)}
    refit = {"kernel": "refit_kernel<order 2, isotropic, uint16> (FP64 from the raw frame)", "ms_per_launch": round(refit_ms, 4),
             "launches_timed": int(kt.n_refit), "outputs_per_frame": head["fp64_outputs"],
             "frac_of_outputs": head["fp64_frac"]}
    batched = None
    if args.batch_frames > 0 and size == 2048:
        batched = {}
        for st in ("fused", "fp16"):
            say(f"batched leg ({args.batch_frames} mixed frames, {st})")
            batched[st] = batch_leg(torch, ctx, Rig, sensors, raws, configs, args.batch_frames, st, checks)
    served = None
    if args.serve_seconds > 0 and size == 2048:
        # untimed warm-up: the first batches of each capacity class build their graphs
        say("served leg warm-up (1 s, 8 cameras)")
        serve_leg(torch, ctx, Rig, sensors, raws, configs, 1.0)
        say(f"served leg ({args.serve_seconds} s, 8 cameras)")
        served = serve_leg(torch, ctx, Rig, sensors, raws, configs, args.serve_seconds, checks)
        served["warmup_s"] = 1.0
    cpu = None
    if not args.no_cpu:
        threads, avail = host_threads()
        say(f"oracle leg: FP64 oracle on a band (1 and {threads} threads), then the legs' samples")
        cpu = oracle_leg(sensors, raws, params, args.cpu_rows, checks, threads, avail, args.cpu_rows_all_core)
    line = {
        "metric": "HDR output Mpixel/s at 4 Mpix order-2 ICI vs plain FP32; p99 frame latency",
        "value": round(value, 3), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"4 x {size}x{size} raw uint16 12-bit RGGB, exposures 1/1/4/1/16/1/64, "
                               f"order-2 LPA, ICI radii {{1,2,3,4}} Gamma 2, {size}x{size} RGB fp32 output",
                   "form": "fused raw decode + fit, tuned launch shape, then the FP64 refit launch",
                   "frames_per_step": 1, "tuned": tuned},
        "headline": head,
        "plain_fp32": plain,
        "small": small,
        "resample_fp16": resample,
        "calpa": calpa,
        "precomputed_weights": pre,
        "calibration_frames": calib,
        "temporal": temporal,
        "speedup_vs_plain": round(value / plain["value"], 3) if plain else None,
        "roofline": roof,
        "refit": refit,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
        "batched": batched,
        "served": served,
        "wall_s_timed": round(wall, 3),
        "ms_per_step_min": round(min(per), 4), "ms_per_step_max": round(max(per), 4),
    }
    print(json.dumps(line))
    rig.close()
    ctx.close()


if __name__ == "__main__":
    main()
