"""Python binding of liblpa.so (the C ABI in include/lpa.h).

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels behind the C ABI.  torch is used for device memory and streams.  The
module refuses to work without the built library (there is no fallback).

Low level: the C functions under their own names (``lpa_create_ctx`` ...),
called with ctypes structures.  High level: ``Context`` and ``Rig``.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblpa.so")

MAX_SENSORS = 8
MAX_SCALES = 8

OK, NOT_READY, AGAIN = 0, 1, 2
ERR_INVALID_ARG, ERR_OOM, ERR_DEVICE, ERR_UNSUPPORTED, ERR_INTERNAL = -1, -2, -3, -4, -5
CFA = {"RGGB": 0, "BGGR": 1, "GRBG": 2, "GBRG": 3}
DTYPE_U16, DTYPE_F32 = 0, 1
MEM_DEVICE, MEM_HOST = 0, 1
STORE = {"fused": 0, "fp32": 1, "fp16": 2}
FLAG_NO_FP64_FALLBACK = 0x1
FLAG_PRECOMPUTED_WEIGHTS = 0x2
MODE = {"lpa": 0, "calpa": 1}


class LpaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lpa status {status}: {msg}")
        self.status = status


class Calib(ctypes.Structure):
    _fields_ = [("bias", ctypes.c_void_p), ("prnu", ctypes.c_void_p), ("read_var", ctypes.c_void_p),
                ("saturation", ctypes.c_void_p), ("defect", ctypes.c_void_p)]


class SensorDesc(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("cfa", ctypes.c_int32),
        ("bit_depth", ctypes.c_int32), ("affine", ctypes.c_double * 6), ("exposure", ctypes.c_double),
        ("gain", ctypes.c_double), ("read_sigma", ctypes.c_double), ("black_level", ctypes.c_double),
        ("saturation", ctypes.c_double), ("calib", ctypes.POINTER(Calib)),
    ]


class RigDesc(ctypes.Structure):
    _fields_ = [("n_sensors", ctypes.c_int32), ("sensors", ctypes.POINTER(SensorDesc))]


class Params(ctypes.Structure):
    _fields_ = [
        ("out_w", ctypes.c_int32), ("out_h", ctypes.c_int32), ("out_affine", ctypes.c_double * 6),
        ("order", ctypes.c_int32), ("n_scales", ctypes.c_int32),
        ("radii", ctypes.c_double * MAX_SCALES), ("h", ctypes.c_double * MAX_SCALES),
        ("gamma", ctypes.c_double), ("green_ratio", ctypes.c_double), ("storage", ctypes.c_int32),
        ("tau_inv", ctypes.c_double), ("tau_fp64", ctypes.c_double), ("flags", ctypes.c_uint32),
        ("mode", ctypes.c_int32), ("grad_order", ctypes.c_int32), ("grad_halfwin", ctypes.c_int32),
        ("pad_", ctypes.c_int32), ("alpha", ctypes.c_double), ("lambda1", ctypes.c_double),
        ("lambda2", ctypes.c_double), ("grad_radius", ctypes.c_double), ("grad_h", ctypes.c_double),
        ("max_stretch", ctypes.c_double), ("value_tol", ctypes.c_double),
        ("h_t", ctypes.c_double * MAX_SCALES),
    ]


class Frame(ctypes.Structure):
    _fields_ = [
        ("n_sensors", ctypes.c_int32), ("raw", ctypes.c_void_p * MAX_SENSORS),
        ("row_pitch_bytes", ctypes.c_int64 * MAX_SENSORS), ("dtype", ctypes.c_int32),
        ("memory", ctypes.c_int32),
    ]


class Output(ctypes.Structure):
    _fields_ = [
        ("rgb", ctypes.c_void_p), ("row_pitch_bytes", ctypes.c_int64),
        ("scale_map", ctypes.c_void_p), ("scale_map_pitch", ctypes.c_int64),
        ("sd_map", ctypes.c_void_p), ("sd_map_pitch", ctypes.c_int64),
        ("grad_map", ctypes.c_void_p), ("grad_map_pitch", ctypes.c_int64),
        ("steer_map", ctypes.c_void_p), ("steer_map_pitch", ctypes.c_int64),
        ("stats", ctypes.c_void_p),
    ]


class TuneResult(ctypes.Structure):
    _fields_ = [
        ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("occupancy", ctypes.c_int32),
        ("n_candidates", ctypes.c_int32), ("ms_best", ctypes.c_double), ("ms_default", ctypes.c_double),
    ]


class KernelTime(ctypes.Structure):
    _fields_ = [("fit_ms", ctypes.c_double), ("refit_ms", ctypes.c_double), ("n_fit", ctypes.c_int64),
                ("n_refit", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("batch_size", ctypes.c_int32), ("t_arrival_ns", ctypes.c_int64),
        ("t_admit_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
        ("n_fp64", ctypes.c_uint64), ("n_invalid", ctypes.c_uint64),
    ]


_lib = None
_lock = threading.Lock()

# Every symbol the header declares, with its ctypes signature.
SIGNATURES = {
    "lpa_create_ctx": (ctypes.c_int32, [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]),
    "lpa_destroy_ctx": (ctypes.c_int32, [ctypes.c_void_p]),
    "lpa_create_rig": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(RigDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "lpa_destroy_rig": (ctypes.c_int32, [ctypes.c_void_p]),
    "lpa_reconstruct": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Frame), ctypes.POINTER(Params),
                                         ctypes.POINTER(Output), ctypes.c_void_p]),
    "lpa_reconstruct_plain": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Frame), ctypes.POINTER(Params),
                                               ctypes.POINTER(Output), ctypes.c_void_p]),
    "lpa_reconstruct_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Frame), ctypes.POINTER(Params),
                                                 ctypes.POINTER(Output), ctypes.c_void_p]),
    "lpa_reconstruct_batch": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                               ctypes.POINTER(Frame), ctypes.POINTER(Params),
                                               ctypes.POINTER(Output), ctypes.c_void_p]),
    "lpa_submit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Frame), ctypes.POINTER(Params),
                                    ctypes.POINTER(Output), ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)]),
    "lpa_poll": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Result)]),
    "lpa_drain": (ctypes.c_int32, [ctypes.c_void_p]),
    "lpa_autotune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Frame), ctypes.POINTER(Params),
                                      ctypes.POINTER(Output), ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.POINTER(TuneResult)]),
    "lpa_tuner_save": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_char_p]),
    "lpa_tuner_load": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_char_p]),
    "lpa_reconstruct_temporal": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Frame), ctypes.c_int32,
                                                  ctypes.POINTER(Params), ctypes.POINTER(Output), ctypes.c_void_p]),
    "lpa_set_kernel_timing": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "lpa_kernel_times": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(KernelTime)]),
    "lpa_last_error": (ctypes.c_char_p, []),
}


def load(path: str | None = None):
    """Load liblpa.so (raises if it is missing: there is no fallback path)."""
    global _lib
    with _lock:
        if _lib is None:
            p = path or LIB_PATH
            if not os.path.exists(p):
                raise ImportError(f"{p} is not built; run __graft_entry__.build() first")
            lib = ctypes.CDLL(p)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def last_error() -> str:
    return load().lpa_last_error().decode(errors="replace")


def check(status: int, ok=(OK,)) -> int:
    if status not in ok:
        raise LpaError(status, last_error())
    return status


def _c(name):
    def call(*args):
        return getattr(load(), name)(*args)
    call.__name__ = name
    return call


lpa_create_ctx = _c("lpa_create_ctx")
lpa_destroy_ctx = _c("lpa_destroy_ctx")
lpa_create_rig = _c("lpa_create_rig")
lpa_destroy_rig = _c("lpa_destroy_rig")
lpa_reconstruct = _c("lpa_reconstruct")
lpa_reconstruct_plain = _c("lpa_reconstruct_plain")
lpa_reconstruct_batch = _c("lpa_reconstruct_batch")
lpa_reconstruct_noalloc = _c("lpa_reconstruct_noalloc")
lpa_submit = _c("lpa_submit")
lpa_poll = _c("lpa_poll")
lpa_drain = _c("lpa_drain")
lpa_autotune = _c("lpa_autotune")
lpa_tuner_save = _c("lpa_tuner_save")
lpa_tuner_load = _c("lpa_tuner_load")
lpa_reconstruct_temporal = _c("lpa_reconstruct_temporal")
lpa_set_kernel_timing = _c("lpa_set_kernel_timing")
lpa_kernel_times = _c("lpa_kernel_times")
lpa_last_error = _c("lpa_last_error")


# ---------------------------------------------------------------------------
# Marshalling helpers (plain dicts -> structures)
# ---------------------------------------------------------------------------
def sensor_desc(d: dict) -> SensorDesc:
    s = SensorDesc()
    s.width, s.height = int(d["width"]), int(d["height"])
    cfa = d.get("cfa", "RGGB")
    s.cfa = CFA[cfa] if isinstance(cfa, str) else int(cfa)
    s.bit_depth = int(d.get("bit_depth", 12))
    for i, a in enumerate(d["affine"]):
        s.affine[i] = float(a)
    s.exposure, s.gain = float(d["exposure"]), float(d["gain"])
    s.read_sigma, s.black_level = float(d["read_sigma"]), float(d["black_level"])
    s.saturation = float(d["saturation"])
    cal = d.get("calib")
    if cal:
        # per-pixel frames as float32 (uint8 defects), kept alive with the struct
        # until lpa_create_rig has copied them
        import numpy as np

        c = Calib()
        keep = []
        shape = (s.height, s.width)
        for name, key in (("bias", "bias"), ("prnu", "prnu"), ("read_var", "read_var"), ("saturation", "sat")):
            if cal.get(key) is not None:
                a = np.ascontiguousarray(np.asarray(cal[key], dtype=np.float32).reshape(shape))
                keep.append(a)
                setattr(c, name, a.ctypes.data)
        if cal.get("defect") is not None:
            a = np.ascontiguousarray(np.asarray(cal["defect"], dtype=np.uint8).reshape(shape))
            keep.append(a)
            c.defect = a.ctypes.data
        keep.append(c)
        s.calib = ctypes.pointer(c)
        s._keep = keep
    return s


def params_struct(p: dict) -> Params:
    q = Params()
    q.out_w, q.out_h = int(p["out_w"]), int(p["out_h"])
    for i, a in enumerate(p["out_affine"]):
        q.out_affine[i] = float(a)
    q.order = int(p["order"])
    radii = list(p["radii"])
    q.n_scales = len(radii)
    hs = list(p.get("h") or [])
    if len(hs) != len(radii):
        if any(hs):
            raise ValueError("h must give one value per radius")
        hs = [0.0] * len(radii)
    if len(radii) > MAX_SCALES:
        raise ValueError(f"at most {MAX_SCALES} radii")
    for i, r in enumerate(radii):
        q.radii[i] = float(r)
        q.h[i] = float(hs[i])
    q.gamma = float(p.get("gamma", 2.0))
    q.green_ratio = float(p.get("green_ratio", 1.0))
    st = p.get("storage", "fused")
    q.storage = STORE[st] if isinstance(st, str) else int(st)
    q.tau_inv = float(p.get("tau_inv", 0.0))
    q.tau_fp64 = float(p.get("tau_fp64", 0.0))
    q.flags = int(p.get("flags", 0)) | (FLAG_PRECOMPUTED_WEIGHTS if p.get("precomputed_weights") else 0)
    mode = p.get("mode", "lpa")
    q.mode = MODE[mode] if isinstance(mode, str) else int(mode)
    ad = p.get("adapt") or {}
    q.alpha = float(ad.get("alpha", 0.005))
    q.lambda1 = float(ad.get("lambda1", 1.0))
    q.lambda2 = float(ad.get("lambda2", 0.001))
    q.grad_radius = float(ad.get("grad_radius", 0.0))
    q.grad_h = float(ad.get("grad_h", 0.0))
    q.max_stretch = float(ad.get("max_stretch", 0.0))
    q.grad_order = int(ad.get("grad_order", 0))
    q.grad_halfwin = int(ad.get("grad_halfwin", 2))
    q.value_tol = float(p.get("value_tol", 0.0))
    hts = list(p.get("h_t") or [])
    if hts and len(hts) != len(radii):
        raise ValueError("h_t must give one value per radius")
    for i, ht in enumerate(hts):
        q.h_t[i] = float(ht)
    return q


def frame_struct(raws: Sequence, on_device: bool = True) -> Frame:
    """raws: torch tensors (uint16 or float32, 2-D, row-contiguous) or numpy arrays (host)."""
    import torch

    f = Frame()
    f.n_sensors = len(raws)
    dtypes = set()
    for i, r in enumerate(raws):
        if isinstance(r, torch.Tensor):
            if r.dim() != 2 or r.stride(1) != 1:
                raise ValueError("raw planes must be 2-D with contiguous rows")
            dtypes.add(r.dtype)
            f.raw[i] = r.data_ptr()
            f.row_pitch_bytes[i] = r.stride(0) * r.element_size()
        else:
            import numpy as np

            a = r
            if a.ndim != 2 or a.strides[1] != a.itemsize:
                raise ValueError("raw planes must be 2-D with contiguous rows")
            dtypes.add(torch.uint16 if a.dtype == np.uint16 else torch.float32)
            f.raw[i] = a.ctypes.data
            f.row_pitch_bytes[i] = a.strides[0]
    if len(dtypes) != 1:
        raise ValueError("all raw planes of a frame must share a dtype")
    dt = dtypes.pop()
    if dt == torch.uint16:
        f.dtype = DTYPE_U16
    elif dt == torch.float32:
        f.dtype = DTYPE_F32
    else:
        raise ValueError(f"raw dtype {dt} unsupported (uint16 or float32)")
    f.memory = MEM_DEVICE if on_device else MEM_HOST
    return f


def output_struct(rgb, scale_map=None, sd_map=None, grad_map=None, steer_map=None, stats=None) -> Output:
    """stats: optional int64 device tensor of 2 elements (FP64-valued and
    no-data output counts, written by the library)."""
    o = Output()
    if stats is not None:
        if stats.numel() != 2 or stats.element_size() != 8 or not stats.is_contiguous():
            raise ValueError("stats must be a contiguous 2-element 64-bit tensor")
        o.stats = stats.data_ptr()
    if rgb.dim() != 3 or rgb.shape[2] != 3 or rgb.stride(2) != 1 or rgb.stride(1) != 3:
        raise ValueError("rgb must be (H, W, 3) float32 with interleaved pixels")
    o.rgb = rgb.data_ptr()
    o.row_pitch_bytes = rgb.stride(0) * 4
    if scale_map is not None:
        if scale_map.dim() != 3 or scale_map.stride(2) != 1 or scale_map.stride(1) != 3:
            raise ValueError("scale_map must be (H, W, 3) uint8 with interleaved pixels")
        o.scale_map = scale_map.data_ptr()
        o.scale_map_pitch = scale_map.stride(0)
    if sd_map is not None:
        if sd_map.dim() != 3 or sd_map.stride(2) != 1 or sd_map.stride(1) != 3:
            raise ValueError("sd_map must be (H, W, 3) float32 with interleaved pixels")
        o.sd_map = sd_map.data_ptr()
        o.sd_map_pitch = sd_map.stride(0) * 4
    if grad_map is not None:
        if grad_map.dim() != 3 or grad_map.shape[2] != 2 or grad_map.stride(2) != 1 or grad_map.stride(1) != 2:
            raise ValueError("grad_map must be (H, W, 2) float32 with interleaved pixels")
        o.grad_map = grad_map.data_ptr()
        o.grad_map_pitch = grad_map.stride(0) * 4
    if steer_map is not None:
        if steer_map.dim() != 3 or steer_map.shape[2] != 4 or steer_map.stride(2) != 1 or steer_map.stride(1) != 4:
            raise ValueError("steer_map must be (H, W, 4) float32 with interleaved pixels")
        o.steer_map = steer_map.data_ptr()
        o.steer_map_pitch = steer_map.stride(0) * 4
    return o


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Context:
    """A library context on one device (owns streams, tables, scheduler)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        import weakref

        h = ctypes.c_void_p()
        check(lpa_create_ctx(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
        self.handle = h
        self.device = device
        self._rigs = weakref.WeakSet()

    def close(self):
        if self.handle:
            # the C context destroys its live rigs; mark their handles dead first
            for r in list(self._rigs):
                r.handle = None
            check(lpa_destroy_ctx(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reconstruct_batch(self, rigs, frames_raws, params_list, outs, maps=None, stream=None, stats=None):
        n = len(rigs)
        rig_arr = (ctypes.c_void_p * n)(*[r.handle.value for r in rigs])
        fr = (Frame * n)(*[frame_struct(r) for r in frames_raws])
        pr = (Params * n)(*[params_struct(p) for p in params_list])
        maps = maps or [None] * n
        stats = stats or [None] * n
        ou = (Output * n)(*[output_struct(o, m, stats=s) for o, m, s in zip(outs, maps, stats)])
        check(lpa_reconstruct_batch(self.handle, n, rig_arr, fr, pr, ou, _stream_handle(stream)))

    def tuner_save(self, path: str):
        check(lpa_tuner_save(self.handle, path.encode()))

    def tuner_load(self, path: str):
        check(lpa_tuner_load(self.handle, path.encode()))

    def poll(self, ticket: int) -> Result:
        r = Result()
        check(lpa_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(r)), ok=(OK, NOT_READY))
        return r

    def drain(self):
        check(lpa_drain(self.handle))

    def set_kernel_timing(self, on: bool):
        check(lpa_set_kernel_timing(self.handle, 1 if on else 0))

    def kernel_times(self) -> KernelTime:
        t = KernelTime()
        check(lpa_kernel_times(self.handle, ctypes.byref(t)))
        return t


class Rig:
    """A camera rig: sensor calibration and noise constants resident on the device."""

    def __init__(self, ctx: Context, sensors: Sequence[dict]):
        descs = [sensor_desc(d) for d in sensors]  # holds any calibration frames until the rig has copied them
        arr = (SensorDesc * len(sensors))(*descs)
        desc = RigDesc(len(sensors), arr)
        h = ctypes.c_void_p()
        check(lpa_create_rig(ctx.handle, ctypes.byref(desc), ctypes.byref(h)))
        self.handle = h
        self.ctx = ctx
        self.sensors = [dict(d) for d in sensors]
        ctx._rigs.add(self)

    def close(self):
        if self.handle and self.ctx.handle:
            check(lpa_destroy_rig(self.handle))
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reconstruct(self, raws, params: dict, out, scale_map=None, stream=None, plain: bool = False,
                    sd_map=None, grad_map=None, steer_map=None, stats=None, noalloc: bool = False):
        """plain: the plain per-frame FP32 form; noalloc: the allocation-free
        entry point (fused LPA, static scratch)."""
        fr = frame_struct(raws)
        pr = params_struct(params)
        ou = output_struct(out, scale_map, sd_map, grad_map, steer_map, stats)
        fn = lpa_reconstruct_plain if plain else (lpa_reconstruct_noalloc if noalloc else lpa_reconstruct)
        check(fn(self.handle, ctypes.byref(fr), ctypes.byref(pr), ctypes.byref(ou), _stream_handle(stream)))

    def reconstruct_temporal(self, frames, params: dict, out, scale_map=None, stream=None, sd_map=None,
                             stats=None):
        """Temporal LPA: frames[t] holds the sensors' raw planes at time -t
        (frames[0] is reconstructed); params["h_t"] one temporal scale per radius."""
        n = len(frames)
        fr = (Frame * n)(*[frame_struct(f) for f in frames])
        pr = params_struct(params)
        ou = output_struct(out, scale_map, sd_map, stats=stats)
        check(lpa_reconstruct_temporal(self.handle, fr, n, ctypes.byref(pr), ctypes.byref(ou),
                                       _stream_handle(stream)))

    def autotune(self, raws, params: dict, out, reps: int = 3, stream=None) -> TuneResult:
        """Time every launch-shape candidate on this frame; keep the fastest for its class."""
        fr = frame_struct(raws)
        pr = params_struct(params)
        ou = output_struct(out)
        res = TuneResult()
        check(lpa_autotune(self.handle, ctypes.byref(fr), ctypes.byref(pr), ctypes.byref(ou),
                           _stream_handle(stream), int(reps), ctypes.byref(res)))
        return res

    def submit(self, raws, params: dict, out, scale_map=None, arrival_ns: int = 0, host: bool = False):
        fr = frame_struct(raws, on_device=not host)
        pr = params_struct(params)
        ou = output_struct(out, scale_map)
        t = ctypes.c_uint64()
        st = lpa_submit(self.handle, ctypes.byref(fr), ctypes.byref(pr), ctypes.byref(ou), int(arrival_ns),
                        ctypes.byref(t))
        check(st, ok=(OK, AGAIN))
        return None if st == AGAIN else t.value
