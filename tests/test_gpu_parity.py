"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact: per-Gaussian records, tile counts, sorted (tile, depth) keys and
Gaussian ids, tile ranges, per-pixel blend counts and blend order.  Images:
within 1e-4 absolute per float32 channel (the arithmetic is specified to be
identical, so they are expected to match exactly; the bound is the contract).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2402_00525_amd import synth

from gpu_util import (assert_images_close, assert_records_equal, assert_sorted_equal, gpu_frame, say)

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _setup(oracle_lib):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2402_00525_amd import gsr
    gsr.lib()
    return oracle_lib


def test_device_arithmetic_matches_host():
    from paper_2402_00525_amd import gsr
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.uniform(-90, 10, 20000), rng.uniform(1, 1e6, 5000), rng.standard_normal(5000) * 1e-3,
                        np.array([0.0, -0.0, 1.0, -80.0, -80.5, 0.5, 1.5, 2.5, -2.5])]).astype(np.float32)
    b = rng.uniform(-5, 5, a.size).astype(np.float32)
    b[b == 0] = 1.0
    out = gsr.probe_math(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()).cpu().numpy()
    with np.errstate(all="ignore"):
        np.testing.assert_array_equal(out[0].view(np.uint32), (a / b).view(np.uint32))
        sq = np.sqrt(a)
        ok = a >= 0
        np.testing.assert_array_equal(out[1][ok].view(np.uint32), sq[ok].view(np.uint32))
        np.testing.assert_array_equal(out[4], np.rint(a))
        np.testing.assert_array_equal(out[5].view(np.uint32), (a * b + a).view(np.uint32))
    e = np.array([oracle.exp32(x) for x in a], np.float32)
    np.testing.assert_array_equal(out[2].view(np.uint32), e.view(np.uint32))
    big = a >= 1
    l = np.array([oracle.ln32(x) for x in a[big]], np.float32)
    np.testing.assert_array_equal(out[3][big].view(np.uint32), l.view(np.uint32))


@pytest.mark.parametrize("mode", [oracle.MODE_HIER, oracle.MODE_GLOBAL])
def test_small_scene_bit_exact(mode):
    sc, cam = synth.workload_small()
    say("case: small scene mode", mode)
    o = oracle.frame(sc, cam, mode=mode, max_k=64)
    g = gpu_frame(sc, cam, mode=mode, max_k=64)
    assert_records_equal(g, o)
    assert_sorted_equal(g, o)
    assert_images_close(g, o, TOL)
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
    # the arithmetic is the same, so the images agree bit for bit
    np.testing.assert_array_equal(g["rgb"].view(np.uint32), o.rgb.view(np.uint32))


@pytest.mark.parametrize("mode,prefix,head", [(oracle.MODE_HIER, 0, 4), (oracle.MODE_HIER, 64, 4),
                                              (oracle.MODE_GLOBAL, 0, 4), (oracle.MODE_HIER, 0, 2),
                                              (oracle.MODE_HIER, 0, 8), (oracle.MODE_HIER, 0, 12)])
def test_small_image_whole_lists(mode, prefix, head):
    """Below 512 tiles the default sorts every tile's whole list before one
    render pass (no prefix), and the hierarchical render loads its splats
    ahead (heads up to 8); an explicit prefix keeps the prefix pass and the
    fallback.  All give the oracle's lists and blend order."""
    from paper_2402_00525_amd import gsr
    sc = synth.subsample(synth.mixture_scene(100_000, seed=3), 30_000)
    cam = synth.orbit_camera(256, 256, 11)
    assert gsr.lib().gsr_default_prefix(256, 256, mode) == 0
    say("case: 256x256, mode", mode, "prefix", prefix, "head", head)
    o = oracle.frame(sc, cam, mode=mode, head=head, max_k=64)
    g = gpu_frame(sc, cam, mode=mode, head=head, max_k=64, sort_prefix=prefix)
    L = g["lists"]
    nonempty = int((np.diff(L["ranges"], axis=1) > 0).sum())
    if prefix == 0:
        assert L["fallback_tiles"] == nonempty and L["fallback_entries"] == len(g["keys"])
    else:
        assert 0 < L["fallback_tiles"] < nonempty
    assert_sorted_equal(g, o)
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
    np.testing.assert_array_equal(g["rgb"].view(np.uint32), o.rgb.view(np.uint32))
    np.testing.assert_array_equal(g["count"], o.count)


@pytest.mark.parametrize("head", [1, 2, 3, 6, 8, 12, 16, 20, 24])
def test_head_sizes_bit_exact(head):
    sc, cam = synth.workload_small()
    cam = synth.orbit_camera(128, 96, view=5)
    say("case: head", head)
    o = oracle.frame(sc, cam, mode=oracle.MODE_HIER, head=head, max_k=48)
    g = gpu_frame(sc, cam, mode=oracle.MODE_HIER, head=head, max_k=48)
    assert_sorted_equal(g, o)
    assert_images_close(g, o, TOL)
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)


@pytest.mark.parametrize("W,H", [(200, 120), (33, 17), (16, 16), (1, 1), (250, 9)])
def test_ragged_images(W, H):
    sc = synth.uniform_scene(1500, seed=21, sh_degree=2)
    cam = synth.orbit_camera(W, H, view=11)
    say("case: ragged", W, H)
    for mode in (oracle.MODE_HIER, oracle.MODE_GLOBAL):
        o = oracle.frame(sc, cam, mode=mode, max_k=32)
        g = gpu_frame(sc, cam, mode=mode, max_k=32)
        assert_records_equal(g, o)
        assert_sorted_equal(g, o)
        assert_images_close(g, o, TOL)
        np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)


def test_mixture_scene_1080p_subsample_bit_exact():
    full = synth.mixture_scene(200_000, seed=1)
    sc = synth.subsample(full, 20_000)
    cam = synth.orbit_camera(1920, 1080, view=3)
    say("case: 20k mixture at 1080p")
    o = oracle.frame(sc, cam, mode=oracle.MODE_HIER, max_k=16)
    g = gpu_frame(sc, cam, mode=oracle.MODE_HIER, max_k=16)
    assert_records_equal(g, o)
    assert_sorted_equal(g, o)
    assert_images_close(g, o, TOL)
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)


def test_two_grouping_passes_4k_bit_exact():
    """3840x2160 has 32400 tiles: after the 5 bits of grouped duplication the
    remaining 10 tile bits take two radix passes."""
    from paper_2402_00525_amd import gsr
    assert gsr.lib().gsr_group_passes(3840, 2160) == 2
    sc = synth.subsample(synth.mixture_scene(100_000, seed=5), 6000)
    cam = synth.orbit_camera(3840, 2160, view=12)
    say("case: 6k mixture at 3840x2160 (two grouping passes)")
    o = oracle.frame(sc, cam, mode=oracle.MODE_HIER, max_k=8)
    g = gpu_frame(sc, cam, mode=oracle.MODE_HIER, max_k=8)
    assert_records_equal(g, o)
    assert_sorted_equal(g, o)
    assert_images_close(g, o, TOL)
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)


@pytest.mark.parametrize("prefix", [1, 16, 100, 4096, 16384])
def test_prefix_fallback_bit_exact(prefix):
    """Short sorted prefixes force many tiles through the fallback sort; the
    blend order and images stay those of the full sort."""
    sc, cam = synth.workload_small()
    say("case: sort prefix", prefix)
    o = oracle.frame(sc, cam, mode=oracle.MODE_HIER, max_k=48)
    g = gpu_frame(sc, cam, mode=oracle.MODE_HIER, max_k=48, sort_prefix=prefix)
    assert_sorted_equal(g, o)
    if prefix <= 16:
        assert g["lists"]["fallback_entries"] > 0
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
    np.testing.assert_array_equal(g["rgb"].view(np.uint32), o.rgb.view(np.uint32))
    np.testing.assert_array_equal(g["count"], o.count)


@pytest.mark.parametrize("mode,K,prefix", [(oracle.MODE_GLOBAL, 4, 1), (oracle.MODE_GLOBAL, 4, 16),
                                           (oracle.MODE_GLOBAL, 4, 100), (oracle.MODE_WINDOW, 4, 16),
                                           (oracle.MODE_WINDOW, 16, 100)])
def test_prefix_fallback_3dgs_lists_bit_exact(mode, K, prefix):
    """The 3DGS order and the resort window take the same prefix pass and
    fallback: short prefixes flag tiles, which are rendered again from their
    whole sorted lists; blend order and images are those of the full sort."""
    sc, cam = synth.workload_small()
    say("case: 3DGS lists, mode", mode, "K", K, "prefix", prefix)
    o = oracle.frame(sc, cam, mode=mode, head=K, max_k=48)
    g = gpu_frame(sc, cam, mode=mode, head=K, max_k=48, sort_prefix=prefix)
    assert_sorted_equal(g, o)
    if prefix <= 16:
        assert g["lists"]["fallback_entries"] > 0
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
    np.testing.assert_array_equal(g["rgb"].view(np.uint32), o.rgb.view(np.uint32))
    np.testing.assert_array_equal(g["count"], o.count)


@pytest.mark.parametrize("n,longest", [(30_000, 4096), (100_000, 16384)])
def test_prefix_fallback_long_lists(n, longest):
    """Faint Gaussians keep pixels alive past every prefix, so whole lists of
    more than 4096 entries are sorted by the fallback: in LDS up to 16384
    entries, by radix passes beyond."""
    sc = synth.uniform_scene(n, seed=3, sh_degree=0)
    sc.opacities[:] = (sc.opacities * 0.02).astype(np.float32)
    cam = synth.front_camera(64, 48)
    say("case: long fallback lists", n)
    o = oracle.frame(sc, cam, mode=oracle.MODE_HIER, max_k=64)
    g = gpu_frame(sc, cam, mode=oracle.MODE_HIER, max_k=64, sort_prefix=256)
    assert np.diff(o.ranges, axis=1).max() > longest
    assert_sorted_equal(g, o)
    flag = g["lists"]["tile_flag"]
    assert flag.max() > longest
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
    np.testing.assert_array_equal(g["rgb"].view(np.uint32), o.rgb.view(np.uint32))
    np.testing.assert_array_equal(g["count"], o.count)


def test_fallback_one_depth_layer():
    """A layer of faint Gaussians at one distance from the camera puts more
    than 8192 entries of a tile into one depth bin (bits 16..30 of the depth
    key): the fallback sorts that bin's chunk by radix passes over the id and
    depth bits instead of in LDS."""
    n = 40_000
    rng = np.random.default_rng(11)
    means = np.zeros((n, 3), np.float32)
    means[:, :2] = rng.uniform(-0.08, 0.08, (n, 2)).astype(np.float32)
    scales = np.full((n, 3), 0.01, np.float32)
    rots = np.tile(np.array([1.0, 0.0, 0.0, 0.0], np.float32), (n, 1))
    opac = np.full(n, 0.02, np.float32)
    sh = rng.uniform(0.0, 1.0, (n, 1, 3)).astype(np.float32)
    sc = synth.Scene(means, scales, rots, opac, sh, 0)
    cam = synth.front_camera(32, 32)
    say("case: fallback, one depth layer")
    o = oracle.frame(sc, cam, mode=oracle.MODE_HIER, max_k=64)
    base = np.uint64(0xBB800000)
    deepest_bin = 0
    for lo, hi in o.ranges.astype(np.int64):
        d = o.keys[lo:hi] & np.uint64(0xffffffff)
        b = (d[d >= base] - base) >> np.uint64(16)
        if b.size:
            deepest_bin = max(deepest_bin, int(np.bincount(b.astype(np.int64)).max()))
    assert deepest_bin > 8192, deepest_bin
    g = gpu_frame(sc, cam, mode=oracle.MODE_HIER, max_k=64, sort_prefix=256)
    assert g["lists"]["fallback_entries"] > 8192
    assert_sorted_equal(g, o)
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
    np.testing.assert_array_equal(g["rgb"].view(np.uint32), o.rgb.view(np.uint32))
    np.testing.assert_array_equal(g["count"], o.count)


@pytest.mark.parametrize("K", [1, 4, 8, 16, 24])
def test_window_mode_bit_exact(K):
    """Per-ray resorting window (Sec. 3.3) over the 3DGS lists."""
    sc, _ = synth.workload_small()
    cam = synth.orbit_camera(144, 100, view=9)
    say("case: window", K)
    o = oracle.frame(sc, cam, mode=oracle.MODE_WINDOW, head=K, max_k=64)
    g = gpu_frame(sc, cam, mode=oracle.MODE_WINDOW, head=K, max_k=64)
    assert_records_equal(g, o)
    assert_sorted_equal(g, o)
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
    assert_images_close(g, o, TOL)
    np.testing.assert_array_equal(g["rgb"].view(np.uint32), o.rgb.view(np.uint32))


@pytest.mark.parametrize("mode,K", [(oracle.MODE_HIER, 4), (oracle.MODE_HIER, 1), (oracle.MODE_GLOBAL, 4),
                                    (oracle.MODE_WINDOW, 4), (oracle.MODE_WINDOW, 16), (oracle.MODE_FULL, 4)])
def test_sort_error_bit_exact(mode, K):
    """Per-pixel sort error (Sec. 3.3, Table sortcost) through
    gsr_render_sort_error equals the oracle's, in every mode; zero for the
    full per-pixel sort."""
    from paper_2402_00525_amd import gsr
    sc = synth.subsample(synth.mixture_scene(100_000, seed=1), 8000)
    cam = synth.orbit_camera(320, 180, view=3)
    say("case: sort error mode", mode, "K", K)
    o = oracle.frame(sc, cam, mode=mode, head=K)
    ds = gsr.DeviceScene.from_host(sc)
    r = gsr.Renderer(entries_hint=1 << 18)
    out, delta = r.render_sort_error(ds, cam, gsr.config(mode=mode, head=K))
    d = delta.cpu().numpy()
    np.testing.assert_array_equal(out.count.cpu().numpy(), o.count)
    np.testing.assert_array_equal(d.view(np.uint32), o.delta.view(np.uint32))
    if mode == oracle.MODE_FULL:
        assert d.max() == 0.0
    else:
        assert d.max() > 0.0


def test_window_mode_mixture_1080p():
    sc = synth.subsample(synth.mixture_scene(200_000, seed=1), 20_000)
    cam = synth.orbit_camera(1920, 1080, view=21)
    say("case: window 16, 20k mixture at 1080p")
    o = oracle.frame(sc, cam, mode=oracle.MODE_WINDOW, head=16, max_k=16)
    g = gpu_frame(sc, cam, mode=oracle.MODE_WINDOW, head=16, max_k=16)
    assert_sorted_equal(g, o)
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
    assert_images_close(g, o, TOL)


@pytest.mark.parametrize("flags", [1, 2, 4, 7])
def test_ablations_bit_exact(flags):
    """Table performance_ablation (B) no tile depth, (D) no tile culling,
    (E) no hierarchical culling, and all three."""
    sc, _ = synth.workload_small()
    cam = synth.orbit_camera(160, 112, view=13)
    say("case: ablation flags", flags)
    o = oracle.frame(sc, cam, mode=oracle.MODE_HIER, max_k=48, flags=flags)
    g = gpu_frame(sc, cam, mode=oracle.MODE_HIER, max_k=48, flags=flags)
    assert_records_equal(g, o)
    assert_sorted_equal(g, o)
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
    np.testing.assert_array_equal(g["rgb"].view(np.uint32), o.rgb.view(np.uint32))
    assert_images_close(g, o, TOL)


@pytest.mark.parametrize("case", ["small", "mixture"])
def test_tile_centre_depth_bit_exact(case):
    """The 3DGS order with naive per-tile depth (Sec. 3.3, Fig. pertiledepth):
    keys along each tile's centre ray, entries, blend order, image and
    per-pixel sort error equal the oracle's."""
    from paper_2402_00525_amd import gsr
    if case == "small":
        sc, _ = synth.workload_small()
        cam = synth.orbit_camera(160, 112, view=13)
    else:
        sc = synth.subsample(synth.mixture_scene(100_000, seed=1), 8000)
        cam = synth.orbit_camera(320, 180, view=3)
    say("case: tile-centre depth", case)
    o = oracle.frame(sc, cam, mode=oracle.MODE_GLOBAL, max_k=48, flags=oracle.TILE_CENTRE_DEPTH)
    g = gpu_frame(sc, cam, mode=oracle.MODE_GLOBAL, max_k=48, flags=gsr.TILE_CENTRE_DEPTH)
    assert_records_equal(g, o)
    assert_sorted_equal(g, o)
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
    np.testing.assert_array_equal(g["rgb"].view(np.uint32), o.rgb.view(np.uint32))
    assert_images_close(g, o, TOL)
    ds = gsr.DeviceScene.from_host(sc)
    r = gsr.Renderer(entries_hint=1 << 18)
    out, delta = r.render_sort_error(ds, cam, gsr.config(mode=oracle.MODE_GLOBAL, flags=gsr.TILE_CENTRE_DEPTH))
    np.testing.assert_array_equal(delta.cpu().numpy().view(np.uint32), o.delta.view(np.uint32))


def _big_gaussian_scene():
    sc = synth.uniform_scene(1500, seed=31, sh_degree=1)
    rng = np.random.default_rng(31)
    big = rng.choice(sc.n, 60, replace=False)
    sc.scales[big] = rng.uniform(0.15, 0.5, (60, 3)).astype(np.float32)
    return sc


@pytest.mark.parametrize("lb", [0, 1, 16, 32, 48, 64, 65, 100, 1000, 1 << 30])
def test_load_balancing_threshold_changes_nothing(lb):
    """(C) and the threshold sweep: masked, serial and cooperative work
    classes give the same entries and images."""
    sc = _big_gaussian_scene()
    cam = synth.front_camera(320, 240)
    say("case: lb threshold", lb)
    for mode in (oracle.MODE_HIER, oracle.MODE_GLOBAL):
        o = oracle.frame(sc, cam, mode=mode, max_k=32)
        g = gpu_frame(sc, cam, mode=mode, max_k=32, lb_threshold=lb)
        r = o.rect.astype(np.int64)
        area = (r[:, 2] - r[:, 0] + 1) * (r[:, 3] - r[:, 1] + 1)
        assert area[o.touched > 0].max() > 64          # every work class occurs
        assert_records_equal(g, o)
        assert_sorted_equal(g, o)
        np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
        assert_images_close(g, o, TOL)


@pytest.mark.parametrize("case", ["small", "ragged", "mixture"])
def test_full_sort_bit_exact(case):
    """The full per-pixel sort (Sec. 3.2) against the oracle's brute force
    over every Gaussian."""
    if case == "small":
        sc, cam = synth.workload_small()
    elif case == "ragged":
        sc, cam = synth.uniform_scene(1500, seed=21, sh_degree=2), synth.orbit_camera(200, 120, view=11)
    else:
        sc, cam = synth.subsample(synth.mixture_scene(100_000, seed=3), 3000), synth.orbit_camera(480, 270, 7)
    say("case: full sort", case)
    o = oracle.frame(sc, cam, mode=oracle.MODE_FULL, max_k=128)
    g = gpu_frame(sc, cam, mode=oracle.MODE_FULL, max_k=128)
    assert o.count.max() < 128
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
    np.testing.assert_array_equal(g["count"], o.count)
    np.testing.assert_array_equal(g["rgb"].view(np.uint32), o.rgb.view(np.uint32))
    assert_images_close(g, o, TOL)


def test_render_work_counts_are_consistent():
    """gsr_render_work renders the same image and counts one blend per
    blended Gaussian, at most one keyed entry per test at every level."""
    from paper_2402_00525_amd import gsr
    sc = synth.subsample(synth.mixture_scene(100_000, seed=1), 20_000)
    cam = synth.orbit_camera(640, 360, view=4)
    say("case: render work counts")
    ds = gsr.DeviceScene.from_host(sc)
    r = gsr.Renderer(entries_hint=64 * sc.n)
    ref = r.render(ds, cam)
    ref = {k: getattr(ref, k).cpu().numpy().copy() for k in ("rgb", "count", "T")}
    fr, w = r.render_work(ds, cam)
    np.testing.assert_array_equal(fr.rgb.cpu().numpy().view(np.uint32), ref["rgb"].view(np.uint32))
    np.testing.assert_array_equal(fr.count.cpu().numpy(), ref["count"])
    assert w["blends"] == int(ref["count"].astype(np.int64).sum())
    for lvl in ("tail", "mid", "head"):
        assert 0 < w[lvl + "_keyed"] <= w[lvl + "_tests"], w
    assert w["mid_tests"] <= 4 * w["tail_keyed"] and w["head_tests"] <= 4 * w["mid_keyed"], w
    with pytest.raises(gsr.GsrError):
        r.render_work(ds, cam, gsr.config(head=8))


def test_edge_cases_empty_culled_nan():
    from paper_2402_00525_amd import gsr
    cam = synth.front_camera(64, 48)
    say("case: empty scene")
    empty = synth.Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), np.zeros((0, 4), np.float32),
                        np.zeros((0,), np.float32), np.zeros((0, 1, 3), np.float32), 0)
    ds = gsr.DeviceScene.from_host(empty)
    r = gsr.Renderer(entries_hint=16)
    out = r.render(ds, cam, gsr.config(bg=(0.25, 0.5, 0.75)))
    rgb = out.rgb.cpu().numpy()
    assert np.all(rgb[0] == 0.25) and np.all(rgb[2] == 0.75)
    assert np.all(out.count.cpu().numpy() == 0) and np.all(out.T.cpu().numpy() == 1.0)
    say("case: culled / NaN / zero quaternion")
    sc = synth.uniform_scene(300, seed=9)
    sc.means[0] = [0, 0, -10]          # behind the camera
    sc.means[1, 0] = np.nan            # NaN parameter
    sc.scales[2, 1] = 0.0              # zero scale
    sc.rots[3] = 0.0                   # zero quaternion -> identity
    sc.opacities[4] = 0.001            # below 1/255
    sc.opacities[5] = np.inf
    o = oracle.frame(sc, cam, mode=oracle.MODE_HIER, max_k=16)
    g = gpu_frame(sc, cam, mode=oracle.MODE_HIER, max_k=16)
    assert o.touched[[0, 1, 2, 4, 5]].sum() == 0
    assert_records_equal(g, o)
    assert_sorted_equal(g, o)
    assert_images_close(g, o, TOL)
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)


def test_deterministic_repeat():
    """Outputs, tile ranges and sorted tile lists repeat exactly (the order of
    entries inside a tile of the grouped buffer is not specified)."""
    sc, cam = synth.workload_small()
    a = gpu_frame(sc, cam, max_k=16)
    b = gpu_frame(sc, cam, max_k=16)
    for k in ("rgb", "depth", "T", "count", "blend_ids", "ranges"):
        np.testing.assert_array_equal(a[k], b[k])
    oa, ob = np.lexsort((a["values"], a["keys"])), np.lexsort((b["values"], b["keys"]))
    np.testing.assert_array_equal(a["keys"][oa], b["keys"][ob])
    np.testing.assert_array_equal(a["values"][oa], b["values"][ob])
    for k in ("pre_vals", "pre_len"):
        np.testing.assert_array_equal(a["lists"][k], b["lists"][k])


def test_overflow_grows_workspace():
    from paper_2402_00525_amd import gsr
    sc, cam = synth.workload_small()
    say("case: overflow")
    ds = gsr.DeviceScene.from_host(sc)
    r = gsr.Renderer(entries_hint=100)           # far too small: status bit, then re-plan
    out = r.render(ds, cam, gsr.config(), max_k=8)
    o = oracle.frame(sc, cam, mode=oracle.MODE_HIER, max_k=8)
    np.testing.assert_array_equal(out.blend_ids.cpu().numpy(), o.blend_ids)


def test_truncated_prefix_walks_whole_batches_only():
    """A prefix of 40 entries ends in a partial batch.  Rendered as it is, the
    tail's first pop after that batch would terminate every pixel with blend
    orders that differ from the whole list's (the premise is checked on the
    CPU in test_prefix_cases.py), and the tile would not be flagged.  The
    render must stop at the last whole batch, flag the tile, and give the
    whole list's result."""
    from micro_scenes import PREFIX_M, cam16, prefix_partial_batch_scene
    sc, _ = prefix_partial_batch_scene()
    cam = cam16()
    say("case: truncated prefix ending in a partial batch")
    o = oracle.frame(sc, cam, mode=oracle.MODE_HIER, max_k=16)
    g = gpu_frame(sc, cam, mode=oracle.MODE_HIER, max_k=16, sort_prefix=PREFIX_M)
    L = g["lists"]
    assert L["fallback_tiles"] == 1 and int(L["tile_flag"][0]) == 64
    assert_sorted_equal(g, o)
    np.testing.assert_array_equal(g["blend_ids"], o.blend_ids)
    np.testing.assert_array_equal(g["count"], o.count)
    np.testing.assert_array_equal(g["rgb"].view(np.uint32), o.rgb.view(np.uint32))


def _bench_tile_mask(cam, flag, seed, n_random=24):
    """Tiles to check on a benchmark frame: every tile the prefix pass
    flagged, eight tiles of the bottom (partial) tile row, and a seeded
    random sample."""
    tx, ty = (cam.W + 15) // 16, (cam.H + 15) // 16
    rng = np.random.default_rng(seed)
    mask = np.zeros(tx * ty, np.uint8)
    mask[np.nonzero(flag)[0]] = 1
    mask[(ty - 1) * tx + rng.choice(tx, 8, replace=False)] = 1
    mask[rng.choice(tx * ty, n_random, replace=False)] = 1
    return mask


@pytest.mark.parametrize("n,seed,view,W,H", [(3_000_000, 2, 5, 1920, 1080), (3_000_000, 2, 24, 1920, 1080),
                                           (1_000_000, 1, 0, 1920, 1080), (1_000_000, 1, 3, 512, 512)])
def test_benchmark_frames_on_sampled_tiles(n, seed, view, W, H):
    """The benchmarked frames themselves (mixture scenes of 3M and 1M
    Gaussians at 1920x1080, orbit views; and a 512x512 view of the 1M scene,
    whose default prefix is 8192) in the launch configuration the
    benchmark times: per-Gaussian records and tile counts of every Gaussian,
    the ranges of every tile, and on a sample of tiles (all flagged tiles,
    part of the partial bottom row, random ones) the sorted lists, per-pixel
    blend order and images, bit for bit against the oracle rendering only
    those tiles."""
    from paper_2402_00525_amd import gsr
    sc = synth.mixture_scene(n, seed=seed)
    cam = synth.orbit_camera(W, H, view)
    say("case: benchmark frame, %d Gaussians, seed %d, view %d, %dx%d" % (n, seed, view, W, H))
    ds = gsr.DeviceScene.from_host(sc)
    r = gsr.Renderer(entries_hint=32 * n)
    plain = r.render(ds, cam, gsr.config())                 # the benchmarked kernels
    torch.cuda.synchronize()
    img = {k: getattr(plain, k).cpu().numpy().copy() for k in ("rgb", "depth", "count", "T")}
    lists = r.tile_lists(n, cam)
    rec = {k: v.cpu().numpy() for k, v in r.records(n, cam).items()}
    dbg = r.render(ds, cam, gsr.config(), max_k=16)         # same frame, with blend-id lists
    torch.cuda.synchronize()
    bids = dbg.blend_ids.cpu().numpy()
    flag = lists["tile_flag"].view(np.uint32)
    mask = _bench_tile_mask(cam, flag, seed=view)
    say("  flagged tiles %d, checked tiles %d" % (int((flag > 0).sum()), int(mask.sum())))
    o = oracle.frame(sc, cam, mode=oracle.MODE_HIER, max_k=16, tile_mask=mask)
    np.testing.assert_array_equal(rec["touched"], o.touched)
    for k in ("xy", "conic_o", "sw", "zd"):
        np.testing.assert_array_equal(rec[k].view(np.uint32), getattr(o, k).view(np.uint32))
    np.testing.assert_array_equal(lists["ranges"].view(np.uint32), o.ranges)
    ov = o.values.view(np.uint32)
    pre, plen = lists["pre_vals"].view(np.uint32), lists["pre_len"]
    tx = (cam.W + 15) // 16
    pix = np.zeros((cam.H, cam.W), bool)
    for t in np.nonzero(mask)[0]:
        rb, re = (int(v) for v in o.ranges[t])
        c = int(plen[t])
        if flag[t]:
            assert c == re - rb
        else:
            assert c <= min(re - rb, gsr.lib().gsr_default_prefix(W, H, gsr.MODE_HIER))
        np.testing.assert_array_equal(pre[rb:rb + c], ov[rb:rb + c])
        y0, x0 = (t // tx) * 16, (t % tx) * 16
        pix[y0:y0 + 16, x0:x0 + 16] = True
    np.testing.assert_array_equal(bids[pix], o.blend_ids[pix])
    np.testing.assert_array_equal(img["count"][pix], o.count[pix])
    np.testing.assert_array_equal(img["rgb"][:, pix].view(np.uint32), o.rgb[:, pix].view(np.uint32))
    for k in ("depth", "T"):
        np.testing.assert_array_equal(img[k][pix].view(np.uint32), getattr(o, k)[pix].view(np.uint32))
    np.testing.assert_array_equal(dbg.rgb.cpu().numpy().view(np.uint32), img["rgb"].view(np.uint32))
