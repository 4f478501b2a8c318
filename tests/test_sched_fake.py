"""The serving scheduler's policy (paper_1308_4908_amd/csrc/lpa_sched.hpp,
the SchedCore that lpa_serve.cpp drives the device with) on the CPU, against
a fake executor (tests/sched_fake.cpp), built with ThreadSanitizer and with
AddressSanitizer + UndefinedBehaviorSanitizer.

Scenarios (each checks the contract listed in sched_fake.cpp):
  * mixed       4 client threads, 1600 frames of two batch keys, random
                sizes, frames that can never fit (LPA_ERR_OOM) and failed
                copies, concurrent polling;
  * fail        the 5th launch fails as a device error would: every ticket
                ends, those not launched with LPA_ERR_DEVICE, nothing is
                launched afterwards and the budget is returned;
  * queue_full  a stalled device: the admission queue reports LPA_AGAIN at
                1024 waiting frames, and everything accepted completes once
                the device runs again.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "sched_fake.cpp")
SCENARIOS = ["mixed", "fail", "queue_full"]

SANITIZERS = {
    "tsan": (["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1 exitcode=66 second_deadlock_stack=1"}),
    "asan": (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
             {"ASAN_OPTIONS": "detect_leaks=1 halt_on_error=1 exitcode=66"}),
}


@pytest.fixture(scope="module", params=sorted(SANITIZERS))
def fake_bin(request, tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    flags, env = SANITIZERS[request.param]
    out = str(tmp_path_factory.mktemp("sched") / f"sched_fake_{request.param}")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror", *flags,
           "-I", os.path.join(ROOT, "include"), SRC, "-o", out, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return request.param, out, env


@pytest.mark.parametrize("scenario", SCENARIOS)
@pytest.mark.parametrize("seed", [1, 2])
def test_scheduler_policy(fake_bin, scenario, seed):
    name, exe, env = fake_bin
    r = subprocess.run([exe, scenario, str(seed)], capture_output=True, text=True, timeout=240,
                       env={**os.environ, **env})
    report = (r.stdout + r.stderr)[-6000:]
    assert r.returncode == 0, f"{name} {scenario} seed {seed}:\n{report}"
    assert f"ok {scenario}" in r.stdout
    assert "Sanitizer" not in r.stderr, report
