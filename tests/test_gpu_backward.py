"""GPU backward (gsr_render_backward and the autograd Function) against the
oracle's float32 backward, which is itself pinned by float64 finite
differences (test_oracle_backward.py).  Atomic additions make the GPU sums
order-dependent, so the comparison is to a tolerance derived from float32
rounding of sums of a few hundred terms."""
import numpy as np
import pytest
import torch

import oracle
from paper_2402_00525_amd import synth

from gpu_util import say

pytestmark = pytest.mark.gpu

PARAMS = ("means", "scales", "rots", "opacities", "sh")


@pytest.fixture(scope="module", autouse=True)
def _setup(oracle_lib):
    assert torch.cuda.is_available()
    return oracle_lib


def _compare(gpu, ref, rtol=2e-3):
    for name in PARAMS:
        a, b = gpu[name].astype(np.float64), ref[name].astype(np.float64)
        scale = np.abs(b).max() + 1e-30
        err = np.abs(a - b)
        bad = err > rtol * scale + rtol * np.abs(b)
        assert not bad.any(), (name, err.max() / scale, int(bad.sum()))


def _gpu_grads(scene, cam, dL, head=4, sort_prefix=0):
    from paper_2402_00525_amd import gsr
    ds = gsr.DeviceScene.from_host(scene)
    r = gsr.Renderer(entries_hint=max(1 << 16, 64 * scene.n))
    cfg = gsr.config(head=head, sort_prefix=sort_prefix)
    fr = r.render(ds, cam, cfg)
    g = gsr.render_backward(r, ds, cam, cfg, fr, torch.from_numpy(np.ascontiguousarray(dL, np.float32)).cuda())
    torch.cuda.synchronize()
    return fr.rgb.cpu().numpy(), {k: v.cpu().numpy() for k, v in g.items()}


@pytest.mark.parametrize("case", ["fd64", "small", "mixture720", "small_prefix16"])
def test_backward_matches_oracle(case):
    if case == "fd64":
        scene, cam = synth.uniform_scene(64, seed=5, sh_degree=3), synth.front_camera(32, 32)
    elif case.startswith("small"):
        scene, cam = synth.uniform_scene(2000, seed=0, sh_degree=1), synth.orbit_camera(128, 96, 2)
    else:
        scene, cam = synth.subsample(synth.mixture_scene(100_000, seed=3), 10_000), synth.orbit_camera(1280, 720, 7)
    say("case: backward", case)
    target = synth.random_target(cam.H, cam.W, seed=4)
    rgb_o, _, _ = oracle.backward(scene, cam, np.zeros((3, cam.H, cam.W), np.float32), "f32")
    dL = (np.sign(rgb_o - target) / rgb_o.size).astype(np.float32)
    rgb_r, g_ref, _ = oracle.backward(scene, cam, dL, "f32")
    rgb_g, g_gpu = _gpu_grads(scene, cam, dL, sort_prefix=16 if case.endswith("prefix16") else 0)
    np.testing.assert_array_equal(rgb_g.view(np.uint32), rgb_r.view(np.uint32))
    _compare(g_gpu, g_ref)


def test_autograd_function_l1_loss():
    from paper_2402_00525_amd import gsr
    scene, cam = synth.uniform_scene(64, seed=5, sh_degree=3), synth.front_camera(32, 32)
    say("case: autograd")
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(scene, k))).cuda().requires_grad_(True) for k in PARAMS}
    target = torch.from_numpy(synth.random_target(cam.H, cam.W, seed=4)).cuda()
    rgb, depth, count, T = gsr.render(t["means"], t["scales"], t["rots"], t["opacities"], t["sh"], cam)
    loss = (rgb - target).abs().mean()
    loss.backward()
    dL = (torch.sign(rgb.detach() - target) / rgb.numel()).cpu().numpy().astype(np.float32)
    _, g_ref, _ = oracle.backward(scene, cam, dL, "f32")
    _compare({k: t[k].grad.cpu().numpy() for k in PARAMS}, g_ref)
    assert not depth.requires_grad and not T.requires_grad
