"""The Python binding marshals plain dicts and arrays into the C ABI structs
faithfully (CPU only: nothing is launched)."""
import ctypes
import os

import numpy as np
import pytest
import torch

from paper_1308_4908_amd import lpa
from synth import configs
from synth import rig as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_params_struct_fields():
    p = configs.lpa_params(640, 480, 2, [1.0, 2.0, 3.0, 4.0], out_affine=[0.5, 0, 1, 0, 0.5, 2], storage="fp16",
                           gamma=2.5, green_ratio=0.8, flags=lpa.FLAG_NO_FP64_FALLBACK)
    q = lpa.params_struct(p)
    assert (q.out_w, q.out_h, q.order, q.n_scales) == (640, 480, 2, 4)
    assert list(q.radii)[:4] == [1.0, 2.0, 3.0, 4.0] and list(q.h)[:4] == [0.0] * 4
    assert list(q.out_affine) == [0.5, 0, 1, 0, 0.5, 2]
    assert q.storage == lpa.STORE["fp16"] and q.gamma == 2.5 and q.green_ratio == 0.8
    assert q.flags == lpa.FLAG_NO_FP64_FALLBACK


def test_params_h_handling():
    p = configs.lpa_params(8, 8, 1, [1.0, 2.0])
    p["h"] = [0.0]  # all-default shorter list is padded
    assert list(lpa.params_struct(p).h)[:2] == [0.0, 0.0]
    p["h"] = [0.3]  # explicit values must match the radii
    with pytest.raises(ValueError):
        lpa.params_struct(p)
    p["h"] = [0.3, 0.9]
    assert list(lpa.params_struct(p).h)[:2] == [0.3, 0.9]
    with pytest.raises(ValueError):
        lpa.params_struct(configs.lpa_params(8, 8, 1, [float(r) for r in range(1, 10)]))


def test_sensor_desc_fields():
    s = configs.small_rig()[1]
    d = lpa.sensor_desc(s)
    assert (d.width, d.height, d.cfa, d.bit_depth) == (256, 256, lpa.CFA["RGGB"], 12)
    assert list(d.affine) == s["affine"]
    assert (d.exposure, d.gain, d.read_sigma, d.black_level, d.saturation) == (1 / 8, 0.5, 3.0, 64.0, 4095.0)


def test_frame_struct_host_and_pitch():
    a = np.zeros((10, 12), np.uint16)
    b = np.zeros((16, 20), np.uint16)[:10, :12]  # a view with a wider row pitch
    f = lpa.frame_struct([a, b], on_device=False)
    assert f.n_sensors == 2 and f.dtype == lpa.DTYPE_U16 and f.memory == lpa.MEM_HOST
    assert f.row_pitch_bytes[0] == 24 and f.row_pitch_bytes[1] == 40
    assert f.raw[0] == a.ctypes.data
    with pytest.raises(ValueError):
        lpa.frame_struct([a, np.zeros((10, 12), np.float32)], on_device=False)  # mixed dtypes
    with pytest.raises(ValueError):
        lpa.frame_struct([np.zeros((10, 12), np.uint16)[:, ::2]], on_device=False)  # strided columns
    t = torch.zeros((4, 6), dtype=torch.float32)
    f2 = lpa.frame_struct([t])
    assert f2.dtype == lpa.DTYPE_F32 and f2.row_pitch_bytes[0] == 24


def test_output_struct_checks_layout():
    out = torch.zeros((5, 7, 3), dtype=torch.float32)
    o = lpa.output_struct(out, torch.zeros((5, 7, 3), dtype=torch.uint8), torch.zeros((5, 7, 3)))
    assert o.row_pitch_bytes == 7 * 12 and o.scale_map_pitch == 21 and o.sd_map_pitch == 7 * 12
    with pytest.raises(ValueError):
        lpa.output_struct(torch.zeros((5, 7, 4)))
    with pytest.raises(ValueError):
        lpa.output_struct(torch.zeros((5, 3, 7)).permute(0, 2, 1))


def test_missing_library_fails_loudly(tmp_path):
    """There is no fallback path: loading a library that is not built raises."""
    import subprocess
    import sys

    code = ("from paper_1308_4908_amd import lpa\n"
            f"lpa.LIB_PATH = {str(tmp_path / 'liblpa.so')!r}\n"
            "try:\n    lpa.load()\nexcept ImportError as e:\n    print('raised', e)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert "raised" in r.stdout and "not built" in r.stdout


def test_sensor_calibration_frames_marshalled():
    """Per-pixel frames are passed as float32 planes (uint8 defects) of the
    sensor's shape; absent frames stay NULL."""
    import ctypes

    import numpy as np

    s = dict(R.make_sensor(4, 3, [1, 0, 0, 0, 1, 0], 1.0),
             calib={"bias": np.full((3, 4), 60.0), "defect": np.eye(3, 4, dtype=np.uint8)})
    d = lpa.sensor_desc(s)
    c = d.calib.contents
    bias = np.ctypeslib.as_array(ctypes.cast(c.bias, ctypes.POINTER(ctypes.c_float)), shape=(12,))
    assert np.all(bias == 60.0)
    defect = np.ctypeslib.as_array(ctypes.cast(c.defect, ctypes.POINTER(ctypes.c_uint8)), shape=(12,))
    assert defect.reshape(3, 4)[1, 1] == 1 and defect.sum() == 3
    assert not c.prnu and not c.read_var and not c.saturation
    assert not lpa.sensor_desc(R.make_sensor(4, 3, [1, 0, 0, 0, 1, 0], 1.0)).calib


def test_bench_refuses_several_gpus():
    import subprocess
    import sys

    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_bench_traffic_only_for_the_profiled_source(monkeypatch):
    """The benchmark reports the counter-measured HBM traffic only while the
    kernel sources hash to the value the counters were taken on."""
    import sys

    sys.path.insert(0, ROOT)
    import bench

    import json

    key = "fit_kernel<2,ICI,RAW_U16>"
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[key]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["kernel_source_hash"])
    got = bench.measured_traffic(key)
    assert got == rec["bytes_per_launch"] > 0  # counters taken on these sources are reported
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.measured_traffic(key) is None  # and never for other sources
