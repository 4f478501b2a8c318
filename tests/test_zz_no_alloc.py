"""The allocation-free entry point (lpa_reconstruct_noalloc) against
lpa_reconstruct through the C ABI: same kernels and launch shape, so the
values, codes, standard deviations and output counts must be identical, on
two calls in a row (the second on a smaller frame, reusing the static scratch
that the first left behind)."""
import sys

import numpy as np
import pytest

from synth import configs
from synth.scene import EdgeScene

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(torch, rig, dev, params, noalloc):
    H, W = params["out_h"], params["out_w"]
    out = torch.full((H, W, 3), -12345.0, device="cuda")
    smap = torch.full((H, W, 3), 0xEE, dtype=torch.uint8, device="cuda")
    sd = torch.full((H, W, 3), -1.0, device="cuda")
    stats = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    rig.reconstruct(dev, params, out, smap, sd_map=sd, stats=stats, noalloc=noalloc)
    torch.cuda.synchronize()
    return out.cpu().numpy(), smap.cpu().numpy(), sd.cpu().numpy(), stats.cpu().numpy()


def test_noalloc_equals_reconstruct_twice(torch_mod):
    from paper_1308_4908_amd import Context, LpaError, Rig, lpa

    ctx = Context(0)
    sensors = configs.full_rig(seed=2600, size=192)
    scene = EdgeScene(192, 192, 2600, n_lines=14)
    raws = configs.capture_all(scene, sensors, 2600)
    rig = Rig(ctx, sensors)
    dev = [torch_mod.from_numpy(r).cuda() for r in raws]
    # a 192 x 176 frame (ragged tiles), then a smaller 100 x 61 one at an offset
    cases = [configs.lpa_params(192, 176, 2, [1.0, 2.0, 3.0, 4.0]),
             configs.lpa_params(100, 61, 2, [1.0, 2.0, 3.0, 4.0], out_affine=[1, 0, 40.5, 0, 1, 70.25])]
    for i, params in enumerate(cases):
        _say(f"[gpu] noalloc call {i}: {params['out_w']}x{params['out_h']}")
        a = _run(torch_mod, rig, dev, params, noalloc=True)
        b = _run(torch_mod, rig, dev, params, noalloc=False)
        assert np.array_equal(a[0], b[0], equal_nan=True)
        assert np.array_equal(a[1], b[1])
        assert np.array_equal(a[2], b[2], equal_nan=True)
        assert np.array_equal(a[3], b[3])
        assert not np.any(a[0] == -12345.0) and not np.any(a[1] == 0xEE)
        _say(f"  identical; outputs refitted in FP64: {a[3][0]}, without a valid fit: {a[3][1]}")
        assert a[3][0] > 0  # the static scratch carried refit marks
    # outputs beyond the static scratch are refused before anything is enqueued
    big = configs.lpa_params(4096, 4096, 2, [1.0, 2.0])
    out = torch_mod.full((4096, 4096, 3), 7.0, device="cuda")
    with pytest.raises(LpaError) as e:
        rig.reconstruct(dev, big, out, noalloc=True)
    assert e.value.status == lpa.ERR_UNSUPPORTED
    # and forms that need other scratch
    with pytest.raises(LpaError) as e:
        rig.reconstruct(dev, dict(cases[1], storage="fp16"), torch_mod.empty((61, 100, 3), device="cuda"),
                        noalloc=True)
    assert e.value.status == lpa.ERR_UNSUPPORTED
    torch_mod.cuda.synchronize()
    assert torch_mod.all(out == 7.0)
    rig.close()
    ctx.close()
