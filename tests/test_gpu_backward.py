"""GPU backward (gsr_render_backward and the autograd Function) against the
oracle, per element (Sec. 3.5).

The 2D gradients the render accumulates (atomics, per-tile LDS slots for the
first 512 list ranks and global atomics beyond) are compared with the float64
oracle's sums within a rounding bound derived from each sum's own terms; the
parameter gradients with the float64 chain rule applied to the GPU's own 2D
gradients, within the spread of float32 evaluations of that chain (see
grad_check.py).  The oracle's backward is itself pinned by float64 finite
differences (test_oracle_backward.py)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2402_00525_amd import synth

from gpu_util import say
from grad_check import PARAMS, check_grad2d, check_params, grad2d_tolerance, propagated_tolerance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup(oracle_lib):
    assert torch.cuda.is_available()
    return oracle_lib


def _gpu_grads(scene, cam, dL, head=4, sort_prefix=0):
    from paper_2402_00525_amd import gsr
    ds = gsr.DeviceScene.from_host(scene)
    r = gsr.Renderer(entries_hint=max(1 << 16, 64 * scene.n))
    cfg = gsr.config(head=head, sort_prefix=sort_prefix)
    fr = r.render(ds, cam, cfg)
    g = gsr.render_backward(r, ds, cam, cfg, fr, torch.from_numpy(np.ascontiguousarray(dL, np.float32)).cuda())
    torch.cuda.synchronize()
    g2 = r.region(scene.n, cam, "grad2d", torch.float32, 9 * scene.n).view(scene.n, 9).cpu().numpy().copy()
    lists = r.tile_lists(scene.n, cam)
    return fr.rgb.cpu().numpy(), {k: v.cpu().numpy() for k, v in g.items()}, g2, lists


def _l1_dL(scene, cam, head=4):
    target = synth.random_target(cam.H, cam.W, seed=4)
    rgb_o, _, _ = oracle.backward(scene, cam, np.zeros((3, cam.H, cam.W), np.float32), "f32", head=head)
    return (np.sign(rgb_o - target) / rgb_o.size).astype(np.float32)


def _faint_scene():
    sc = synth.uniform_scene(30_000, seed=3, sh_degree=1)
    sc.opacities[:] = (sc.opacities * 0.02).astype(np.float32)
    return sc, synth.front_camera(64, 48)


def _blends_at_deep_ranks(scene, cam, slots=512):
    """Blends (pixel, Gaussian) whose Gaussian sits at list rank >= slots in
    its tile's sorted list (oracle)."""
    fr = oracle.frame(scene, cam, max_k=256)
    assert fr.count.max() < 256
    tiles_x = (cam.W + 15) // 16
    n = 0
    for t in range(fr.ranges.shape[0]):
        lo, hi = (int(v) for v in fr.ranges[t])
        rank = {int(v): i for i, v in enumerate(fr.values[lo:hi])}
        ty, tx = divmod(t, tiles_x)
        ids = fr.blend_ids[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16].reshape(-1)
        n += sum(1 for i in ids[ids >= 0] if rank[int(i)] >= slots)
    return n


CASES = ["fd64", "small", "mixture720", "small_prefix16", "small_head8", "small_head2", "long_lists"]


@pytest.mark.parametrize("case", CASES)
def test_backward_matches_oracle(case):
    head, prefix = 4, 0
    if case == "fd64":
        scene, cam = synth.uniform_scene(64, seed=5, sh_degree=3), synth.front_camera(32, 32)
    elif case.startswith("small"):
        scene, cam = synth.uniform_scene(2000, seed=0, sh_degree=1), synth.orbit_camera(128, 96, 2)
        prefix = 16 if case.endswith("prefix16") else 0
        head = 8 if case.endswith("head8") else (2 if case.endswith("head2") else 4)
    elif case == "long_lists":
        # faint Gaussians keep pixels alive deep into lists of thousands of
        # entries: blends at list ranks beyond the 512 LDS gradient slots
        # take the global atomics
        scene, cam = _faint_scene()
        prefix = 256
    else:
        scene, cam = synth.subsample(synth.mixture_scene(100_000, seed=3), 10_000), synth.orbit_camera(1280, 720, 7)
    say("case: backward", case)
    dL = _l1_dL(scene, cam, head)
    rgb_r, _, _ = oracle.backward(scene, cam, dL, "f32", head=head)
    g2_ref, bound, nterms = oracle.grad2d(scene, cam, dL, head=head)
    count_max = int(oracle.frame(scene, cam, head=head, want_entries=False).count.max())
    rgb_g, g_gpu, g2_gpu, lists = _gpu_grads(scene, cam, dL, head=head, sort_prefix=prefix)
    np.testing.assert_array_equal(rgb_g.view(np.uint32), rgb_r.view(np.uint32))
    if case == "long_lists":
        assert int(lists["tile_flag"].max()) > 1024 and _blends_at_deep_ranks(scene, cam) > 1000
    w2 = check_grad2d(g2_gpu, g2_ref, bound, nterms, count_max)
    wp = check_params(g_gpu, scene, cam, g2_gpu)
    say("  worst err/tol: 2D %.3g, params %s" % (w2, {k: round(v, 3) for k, v in wp.items()}))


def test_autograd_function_l1_loss():
    """The autograd Function's gradients equal a direct C-ABI backward of the
    same loss, up to the freedom atomics leave (both runs are within the 2D
    rounding bound of the exact sums, so they differ by at most twice its
    image through the chain rule)."""
    from paper_2402_00525_amd import gsr
    scene, cam = synth.uniform_scene(64, seed=5, sh_degree=3), synth.front_camera(32, 32)
    say("case: autograd")
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(scene, k))).cuda().requires_grad_(True) for k in PARAMS}
    target = torch.from_numpy(synth.random_target(cam.H, cam.W, seed=4)).cuda()
    rgb, depth, count, T = gsr.render(t["means"], t["scales"], t["rots"], t["opacities"], t["sh"], cam)
    loss = (rgb - target).abs().mean()
    loss.backward()
    dL = (torch.sign(rgb.detach() - target) / rgb.numel()).cpu().numpy().astype(np.float32)
    _, g_direct, g2_direct, _ = _gpu_grads(scene, cam, dL)
    g2_ref, bound, nterms = oracle.grad2d(scene, cam, dL)
    count_max = int(count.max().item())
    check_grad2d(g2_direct, g2_ref, bound, nterms, count_max)
    prop = propagated_tolerance(scene, cam, grad2d_tolerance(bound, nterms, count_max))
    for k in PARAMS:
        a, b = t[k].grad.cpu().numpy().astype(np.float64), g_direct[k].astype(np.float64)
        tol = 2 * prop[k] + 1e-9 * (np.abs(b).max() + 1e-300)
        assert np.all(np.abs(a - b) <= tol), k
    assert not depth.requires_grad and not T.requires_grad


def test_backward_refuses_a_workspace_of_another_forward():
    """The forward leaves a fingerprint of its scene, camera and configuration
    in the workspace; a backward with other arguments adds nothing, returns
    zero gradients and sets the mismatch bit (checked on the device)."""
    from paper_2402_00525_amd import gsr
    scene, cam = synth.uniform_scene(2000, seed=0, sh_degree=1), synth.orbit_camera(128, 96, 2)
    other_cam = synth.orbit_camera(128, 96, 3)
    say("case: backward fingerprint")
    ds = gsr.DeviceScene.from_host(scene)
    r = gsr.Renderer(entries_hint=1 << 17)
    cfg = gsr.config()
    fr = r.render(ds, cam, cfg)
    dL = torch.full((3, cam.H, cam.W), 1e-3, device="cuda")
    ok = gsr.render_backward(r, ds, cam, cfg, fr, dL)             # same arguments: no mismatch
    assert any(float(v.abs().max()) > 0 for v in ok.values())
    for bad_cam, bad_cfg in ((other_cam, cfg), (cam, gsr.config(head=8)), (cam, gsr.config(sort_prefix=64))):
        with pytest.raises(gsr.GsrError):
            gsr.render_backward(r, ds, bad_cam, bad_cfg, fr, dL)
        r.status.zero_()
        g = gsr.render_backward(r, ds, bad_cam, bad_cfg, fr, dL, check=False)
        torch.cuda.synchronize()
        assert int(r.status.item()) & gsr.STATUS_MISMATCH
        assert all(float(v.abs().max()) == 0 for v in g.values())
