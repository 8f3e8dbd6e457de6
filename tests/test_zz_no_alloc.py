"""gsr_render_noalloc (the entry point for callers that cannot allocate)
against gsr_render on the same inputs: two calls in a row, the second with a
smaller scene and image, so the second reuses the fixed workspace the first
left behind.  The same kernels run on both paths, so every output must agree
bit for bit."""
import numpy as np
import pytest
import torch

from paper_2402_00525_amd import synth

from gpu_util import say

pytestmark = pytest.mark.gpu


def _host(fr):
    return {k: getattr(fr, k).cpu().numpy().copy() for k in ("rgb", "depth", "count", "T")}


def _check_same(a, b):
    for k in ("rgb", "depth", "T"):
        np.testing.assert_array_equal(a[k].view(np.uint32), b[k].view(np.uint32), err_msg=k)
    np.testing.assert_array_equal(a["count"], b["count"])


def test_noalloc_matches_render_twice():
    from paper_2402_00525_amd import gsr
    assert torch.cuda.is_available()
    cases = [
        ("20k mixture, 1920x1080", synth.subsample(synth.mixture_scene(200_000, seed=1), 20_000),
         synth.orbit_camera(1920, 1080, view=3)),
        ("1500 uniform, 200x120", synth.uniform_scene(1500, seed=21, sh_degree=2), synth.orbit_camera(200, 120, view=11)),
    ]
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    for name, sc, cam in cases:
        say("case: no-alloc render,", name)
        ds = gsr.DeviceScene.from_host(sc)
        ref = _host(gsr.Renderer(entries_hint=64 * sc.n).render(ds, cam, gsr.config()))
        status.zero_()
        fr = gsr.render_noalloc(ds, cam, gsr.config(), status=status)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        got = _host(fr)
        _check_same(got, ref)
        assert got["count"].max() > 0


def test_noalloc_refuses_what_does_not_fit():
    from paper_2402_00525_amd import gsr
    sc = synth.uniform_scene(600_000, seed=0, sh_degree=0)   # per-Gaussian regions alone exceed 64 MiB
    ds = gsr.DeviceScene.from_host(sc)
    with pytest.raises(gsr.GsrError) as e:
        gsr.render_noalloc(ds, synth.orbit_camera(1920, 1080, view=0), gsr.config())
    assert e.value.code == gsr.GSR_ECAPACITY
