"""The render entry point that allocates nothing, against g4d_render."""
import sys

import numpy as np
import pytest
import torch

import scenegen
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_render_noalloc_matches_render_on_two_calls():
    """g4d_render_noalloc through the C ABI gives the images of g4d_render
    bit for bit (same kernels, same inputs), on two calls in a row, the second
    with a smaller input (fewer primitives, fewer and smaller views) whose
    scratch holds the first call's leftovers; inputs beyond its limits are a
    capacity error, after which both entry points still work."""
    from paper_2310_10642_amd import g4d
    _say("[no-allocation render]")
    wl = scenegen.bench_workload(1)           # 300k primitives, one 1352x1014 view
    big = wl.scene
    small = scenegen.random_scene(61, 20000, sh_degree=3, t_order=2)
    cases = [("300k x 1 view 1352x1014", big, wl.cameras, [float(x) for x in wl.times]),
             ("20k x 2 views 200x150 / 96x64", small,
              [scenegen.look_at_camera((1.0, 0.4, 3.4), 200, 150), scenegen.look_at_camera((-0.8, 0.1, 3.6), 96, 64)],
              [0.31, 0.77])]
    r = None
    for name, scene, cams, times in cases:
        r, _ = PT.gpu_setup(scene)
        ref = [x.clone() for x in r.render(cams, times)]
        out = tuple(torch.full_like(x, float("nan")) for x in ref)
        r.render_noalloc(cams, times, out)
        torch.cuda.synchronize()
        for a, b in zip(ref, out):
            assert torch.equal(a, b), name
        # without the depth and alpha planes
        out2 = (torch.full_like(ref[0], float("nan")), None, None)
        r.render_noalloc(cams, times, out2)
        torch.cuda.synchronize()
        assert torch.equal(out2[0], ref[0]), name
        _say(f"  {name}: identical")
        with pytest.raises(g4d.G4DError) as ei:     # no state for a backward
            r.backward(torch.zeros_like(ref[0]))
        assert ei.value.status == g4d.G4D_ESTATE
    # beyond the pixel limit: 1920 x 1080 + 200 x 150 > 2^21 pixels
    cams = [scenegen.look_at_camera((0.0, 0.2, 3.5), 1920, 1080), scenegen.look_at_camera((0.5, 0.2, 3.5), 200, 150)]
    assert 1920 * 1080 + 200 * 150 > 2 ** 21
    outs = (torch.empty(3 * (1920 * 1080 + 200 * 150), device="cuda"), None, None)
    with pytest.raises(g4d.G4DError) as ei:
        r.render_noalloc(cams, [0.5, 0.5], outs)
    assert ei.value.status == g4d.G4D_ECAPACITY
    name, scene, cams, times = cases[1]
    ref = r.render(cams, times)
    out = tuple(torch.empty_like(x) for x in ref)
    r.render_noalloc(cams, times, out)
    torch.cuda.synchronize()
    for a, b in zip(ref, out):
        assert torch.equal(a, b)
