"""Batched persistent rendering (gsr_batch_*): every view of a batch equals
the single-view render of that view bit for bit (and the oracle's image), for
every schedule the autotuner may pick, eagerly and through HIP-graph replay."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2402_00525_amd import synth

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup(oracle_lib):
    assert torch.cuda.is_available()
    return oracle_lib


def small_batch():
    scenes = [synth.uniform_scene(2000, seed=0, sh_degree=0),
              synth.subsample(synth.mixture_scene(100_000, seed=1), 20_000),
              synth.uniform_scene(1500, seed=21, sh_degree=2)]
    views = [(0, synth.front_camera(128, 128)), (1, synth.orbit_camera(256, 256, 3)),
             (1, synth.sphere_camera(200, 120, 40.0, -20.0)), (2, synth.orbit_camera(33, 17, 11)),
             (0, synth.orbit_camera(64, 48, 7)), (1, synth.sphere_camera(512, 512, 200.0, 50.0)),
             (2, synth.front_camera(96, 96)), (1, synth.orbit_camera(1280, 720, 29))]
    return scenes, views


def _frames_np(frames):
    return [{k: getattr(f, k).cpu().numpy().copy() for k in ("rgb", "depth", "count", "T")} for f in frames]


def _single(scenes, views):
    from paper_2402_00525_amd import gsr
    out = []
    dss = [gsr.DeviceScene.from_host(s) for s in scenes]
    for si, cam in views:
        r = gsr.Renderer(entries_hint=64 * scenes[si].n)
        f = r.render(dss[si], cam)
        out.append({k: getattr(f, k).cpu().numpy().copy() for k in ("rgb", "depth", "count", "T")})
    return out


def _assert_same(a, b):
    for x, y in zip(a, b):
        for k in ("rgb", "depth", "T"):
            np.testing.assert_array_equal(x[k].view(np.uint32), y[k].view(np.uint32))
        np.testing.assert_array_equal(x["count"], y["count"])


def _batch(scenes, views, **kw):
    from paper_2402_00525_amd import gsr
    dss = [gsr.DeviceScene.from_host(s) for s in scenes]
    return gsr.BatchRenderer(dss, views, **kw), dss


def test_batch_equals_single_views_and_oracle():
    scenes, views = small_batch()
    say("case: batch vs single views")
    b, _ = _batch(scenes, views)
    frames = b.render()
    torch.cuda.synchronize()
    got = _frames_np(frames)
    _assert_same(got, _single(scenes, views))
    for k in (0, 3):
        si, cam = views[k]
        o = oracle.frame(scenes[si], cam, mode=oracle.MODE_HIER)
        np.testing.assert_array_equal(got[k]["rgb"].view(np.uint32), o.rgb.view(np.uint32))
        np.testing.assert_array_equal(got[k]["count"], o.count)


def test_batch_schedules_do_not_change_results():
    from paper_2402_00525_amd import gsr
    scenes, views = small_batch()
    say("case: schedules")
    b, _ = _batch(scenes, views)
    ref = _frames_np(b.render())
    for w, c, lb in [(1, 0, 1), (3, 1, 64), (2, 0, 1000), (8, 1, 0)]:
        b.set_schedule(gsr.schedule(w, c, lb))
        _assert_same(_frames_np(b.render()), ref)


def test_batch_graph_replays_match_eager():
    scenes, views = small_batch()
    say("case: graph replay")
    b, _ = _batch(scenes, views)
    eager = _frames_np(b.render())
    b.capture()
    scratch = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        for f in b.frames:                       # eager work between replays
            f.rgb.zero_()
            f.count.fill_(-7)
        scratch.mul_(1.5).add_(1.0)
        torch.cuda.synchronize()
        b.status.zero_()
        b.replay()
        torch.cuda.synchronize()
        assert int(b.status.item()) == 0
        _assert_same(_frames_np(b.frames), eager)


def test_batch_autotune_and_cache(tmp_path):
    scenes, views = small_batch()
    say("case: autotune")
    b, _ = _batch(scenes, views)
    ref = _frames_np(b.render())
    cache = str(tmp_path / "gsr_tune.txt")
    best, ms = b.tune(cache_path=cache, repeats=1)
    assert 1 <= best.wgs_per_cu <= 3 and best.cost_order in (0, 1) and best.lb_threshold in (32, 64, 128)
    assert ms > 0 and os.path.exists(cache)
    line = open(cache).read().split()
    assert int(line[1]) == best.wgs_per_cu
    best2, ms2 = b.tune(cache_path=cache, repeats=1)     # read back, no timing
    assert (best2.wgs_per_cu, best2.cost_order, best2.lb_threshold) == (best.wgs_per_cu, best.cost_order,
                                                                       best.lb_threshold)
    _assert_same(_frames_np(b.render()), ref)
    # A damaged cache line for this batch (a schedule set_schedule would
    # refuse) is ignored: the batch is tuned again and a valid line appended.
    bad = str(tmp_path / "gsr_tune_bad.txt")
    with open(bad, "w") as f:
        f.write("%s 99 1 64 0.5\n%s 2 7 64 0.5\n%s 2 1 -5 0.5\n" % (line[0], line[0], line[0]))
    best3, ms3 = b.tune(cache_path=bad, repeats=1)
    assert 1 <= best3.wgs_per_cu <= 3 and best3.cost_order in (0, 1) and best3.lb_threshold in (32, 64, 128)
    assert len(open(bad).read().splitlines()) == 4
    _assert_same(_frames_np(b.render()), ref)


def test_batch_prefix_fallback_matches():
    from paper_2402_00525_amd import gsr
    scenes, views = small_batch()
    say("case: batch sort prefix 16")
    b, _ = _batch(scenes, views, cfg=gsr.config(sort_prefix=16))
    got = _frames_np(b.render())
    torch.cuda.synchronize()
    c = b.counters().cpu().numpy()
    assert c[5] > 0 and c[6] > 0          # fallback entries and tiles
    _assert_same(got, _single(scenes, views))


def test_batch_overflow_replans():
    scenes, views = small_batch()
    say("case: batch overflow")
    b, _ = _batch(scenes, views, entries_hint=1000)
    got = _frames_np(b.render())
    assert b.capacity() > 1000
    _assert_same(got, _single(scenes, views))


def test_batch_fewer_tiles_than_work_queues():
    # 1 + 6 tiles: most of the eight per-XCD queues hold nothing, and with a
    # prefix of 16 the flagged pass lists only a few tiles.
    from paper_2402_00525_amd import gsr
    scenes = [synth.uniform_scene(2000, seed=0, sh_degree=0), synth.uniform_scene(1500, seed=21, sh_degree=2)]
    views = [(0, synth.front_camera(16, 16)), (1, synth.orbit_camera(33, 17, 11))]
    ref = _single(scenes, views)
    for prefix in (0, 16):
        say("case: 7-tile batch, prefix %d" % prefix)
        b, _ = _batch(scenes, views, cfg=gsr.config(sort_prefix=prefix))
        for w in (1, 8):
            b.set_schedule(gsr.schedule(w, 1, 64))
            _assert_same(_frames_np(b.render()), ref)
        if prefix:
            assert int(b.counters()[6].item()) > 0


def test_batch_truncated_prefix_walks_whole_batches_only():
    # The constructed tile whose 40-entry prefix ends in a partial batch (see
    # test_prefix_cases.py), among other views of a batch.
    from micro_scenes import PREFIX_M, cam16, prefix_partial_batch_scene
    from paper_2402_00525_amd import gsr
    sc, _ = prefix_partial_batch_scene()
    scenes = [sc, synth.uniform_scene(2000, seed=0, sh_degree=0)]
    views = [(0, cam16()), (1, synth.front_camera(64, 64)), (0, cam16())]
    say("case: batch, truncated prefix ending in a partial batch")
    b, _ = _batch(scenes, views, cfg=gsr.config(sort_prefix=PREFIX_M))
    got = _frames_np(b.render())
    o = oracle.frame(sc, cam16(), mode=oracle.MODE_HIER)
    for k in (0, 2):
        np.testing.assert_array_equal(got[k]["rgb"].view(np.uint32), o.rgb.view(np.uint32))
        np.testing.assert_array_equal(got[k]["count"], o.count)
