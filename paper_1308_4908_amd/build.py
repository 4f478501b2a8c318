"""Build liblpa.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

All HIP code is compiled with packed-FP32 instructions disabled and with
floating-point contraction limited to single expressions, so every kernel that
inlines the per-pixel fit produces bit-identical results.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblpa.so")
PEAK_PROBE = os.path.join(HERE, "peak_probe")  # vector-ALU ceiling measurement (bench.py --peak-probe)
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["lpa_kernels.hip", "lpa_api.cpp", "lpa_batch.cpp", "lpa_serve.cpp", "lpa_tune.cpp", "lpa_stencil.cpp",
           "lpa_noalloc.cpp"]
ARCH = os.environ.get("LPA_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=on", "-Wall", "-Wno-unused-result",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = ["hipcc", *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    if not src.endswith(".hip"):
        cmd.insert(1, "-xhip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    r = subprocess.run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
                        "-lpthread"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    r = subprocess.run(["hipcc", *COMMON, "-o", PEAK_PROBE + ".tmp", os.path.join(CSRC, "peak_probe.hip")],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on peak_probe.hip:\n{r.stderr}")
    os.replace(PEAK_PROBE + ".tmp", PEAK_PROBE)
    if verbose:
        print(f"built {LIB} and {PEAK_PROBE}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
