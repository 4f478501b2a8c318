"""The C-ABI library builds, loads and exports every symbol include/lpa.h
declares (no GPU needed: nothing here computes)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpa.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:lpa_status|const char\*)\s+(lpa_\w+)\s*\(", text, re.M)))


def test_header_declares_core_calls():
    names = declared_functions()
    for must in ("lpa_create_rig", "lpa_reconstruct", "lpa_submit", "lpa_poll", "lpa_create_ctx",
                 "lpa_destroy_ctx", "lpa_destroy_rig", "lpa_last_error", "lpa_reconstruct_batch"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1308_4908_amd import lpa

    lib = lpa.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in lpa.SIGNATURES, f"binding lacks {name}"


def test_struct_layouts_match_header():
    """Sizes of the ABI structs computed by the C compiler equal the ctypes mirrors."""
    import subprocess
    import tempfile

    from paper_1308_4908_amd import lpa

    src = '#include "lpa.h"\n#include <stdio.h>\nint main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n",' \
          'sizeof(lpa_sensor_desc),sizeof(lpa_rig_desc),sizeof(lpa_params),sizeof(lpa_frame),' \
          'sizeof(lpa_output),sizeof(lpa_result),sizeof(lpa_tune_result),sizeof(lpa_calib));return 0;}\n'
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "s")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        sizes = [int(x) for x in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    mine = [ctypes.sizeof(t) for t in (lpa.SensorDesc, lpa.RigDesc, lpa.Params, lpa.Frame, lpa.Output, lpa.Result,
                                       lpa.TuneResult, lpa.Calib)]
    assert sizes == mine


def test_no_device_is_a_clean_error():
    """Without a GPU, creating a context fails with a status and a message (no crash)."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1308_4908_amd import lpa

    h = ctypes.c_void_p()
    st = lpa.lpa_create_ctx(0, 0, ctypes.byref(h))
    assert st == lpa.ERR_DEVICE
    assert lpa.last_error()


def test_null_arguments_are_rejected_without_a_device():
    from paper_1308_4908_amd import lpa

    assert lpa.lpa_create_ctx(0, 0, None) == lpa.ERR_INVALID_ARG
    assert lpa.lpa_destroy_ctx(None) == lpa.ERR_INVALID_ARG
    assert lpa.lpa_destroy_rig(None) == lpa.ERR_INVALID_ARG
    assert lpa.lpa_create_rig(None, None, None) == lpa.ERR_INVALID_ARG
    assert lpa.lpa_reconstruct(None, None, None, None, None) == lpa.ERR_INVALID_ARG
    assert lpa.lpa_poll(None, 0, None) == lpa.ERR_INVALID_ARG
    assert lpa.lpa_autotune(None, None, None, None, None, 1, None) == lpa.ERR_INVALID_ARG
    assert lpa.lpa_tuner_save(None, None) == lpa.ERR_INVALID_ARG
    assert lpa.lpa_tuner_load(None, None) == lpa.ERR_INVALID_ARG
