#!/usr/bin/env python3
"""Benchmark of the sorted Gaussian-splatting frame on one MI355X.

A step is one whole frame of the hot path -- preprocess, prefix sum and
duplication, radix sort and tile ranges, hierarchical render -- for one view
of a 60-view orbit around a synthetic 3M-Gaussian scene (degree-3 SH) at
1920x1080, with the scene resident in HBM.  Prints ONE JSON line.

Timing: W untimed frames, then K frames bracketed by torch.cuda.synchronize(),
spread evenly over the orbit's views (all of them when K equals their number);
stage and kernel durations come from HIP events recorded on the render stream
at the stage boundaries and around every radix-scatter launch.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ms/frame @1080p fwd & fwd+bwd; batched views/s; achieved HBM GB/s"
HBM_PEAK_GBS = 8000.0
# fp32 vector peak without packed FP32 (which this build does not use): 256
# CUs x 64 lanes x 2 flops per fused multiply-add x 2.4 GHz.
ALU_PEAK_TFLOPS = 78.6
WORKLOADS = {
    "3m_1080p": dict(n=3_000_000, seed=2, W=1920, H=1080),
    "1m_1080p": dict(n=1_000_000, seed=1, W=1920, H=1080),
    "small": dict(n=2000, seed=0, W=128, H=128),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Source files that define each timed kernel; a change to any of them voids
# the HBM byte counts taken for it (the profile stores their hash).
KERNEL_SOURCES = {
    "k_preprocess": ("frame.hip", "gsr_device.h", "gsr_internal.h"),
    "k_duplicate": ("frame.hip", "gsr_device.h", "gsr_internal.h"),
    "k_radix_scatter": ("sort.hip", "gsr_internal.h"),
    "k_tile_prefix": ("tile_sort.hip", "gsr_internal.h"),
    "k_render_hier1": ("render.hip", "gsr_device.h", "gsr_internal.h"),
}
PROFILE = os.path.join(ROOT, "profiles", "frame_3m_1080p_hier.md")


def kernel_source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2402_00525_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel, workload):
    """HBM bytes of one launch from the committed counter profile, or None
    when there is none or the kernel's sources changed since it was taken."""
    try:
        with open(PROFILE) as f:
            for ln in f:
                p = ln.split()
                if len(p) == 5 and p[0] == "traffic" and p[1] == kernel and p[2] == workload:
                    return int(p[3]) if p[4] == kernel_source_hash(kernel) else None
    except OSError:
        pass
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="3m_1080p", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-global", action="store_true", help="skip timing the 3DGS global order alongside")
    ap.add_argument("--views", type=int, default=60, help="orbit views to cycle through (60 = full orbit)")
    ap.add_argument("--sort-prefix", type=int, default=0,
                    help="entries per tile sorted up front in the hierarchical mode (0 = library default)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched measurement (128 views of 9 scenes, one HIP-graph launch)")
    ap.add_argument("--no-fwd-bwd", action="store_true",
                    help="skip the forward+backward measurement (500k Gaussians, 1280x720, L1 loss)")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the sweep of the other renderers (resort windows, head sizes, ablations, "
                         "load-balancing thresholds, full per-pixel sort)")
    ap.add_argument("--no-sort-error", action="store_true",
                    help="skip the per-ray sort error of every renderer (two orbit views)")
    ap.add_argument("--no-rotation", action="store_true",
                    help="skip the pure-rotation popping sweep (views 0/15/30/45; yaw, pitch, roll of +-0.5/2/5 "
                         "degrees and a 180-degree roll)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (reference for HBM byte counters)")
    ap.add_argument("--gather-calibration-mib", type=int, default=0,
                    help="run one gather of this many MiB of 64-byte rows at random row indices first (reference "
                         "for HBM byte counters of gather-heavy kernels)")
    return ap.parse_args()


def make_events(n):
    import torch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    for e in evs:
        e.record()
    torch.cuda.synchronize()
    return evs, (C.c_void_p * n)(*[e.cuda_event for e in evs])


def timed_view(i, steps, n_views):
    """Orbit view of timed frame i: the timed frames spread evenly over the
    whole orbit (every view once when steps equals the number of views)."""
    return (i * n_views) // steps if steps <= n_views else i % n_views


def time_frames(r, ds, cams, cfg, steps, warmup, passes):
    """Render warmup + steps frames; returns per-frame stage/kernel times (ms)."""
    import torch
    from paper_2402_00525_amd import gsr
    W, H = cams[0].W, cams[0].H
    out = gsr.Frame(H, W, "cuda")
    for i in range(warmup):
        r.render_async(ds, cams[i % len(cams)], cfg, out)
    nev = 9 + 2 * passes
    frames = [make_events(nev) for _ in range(steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    r.status.zero_()
    torch.cuda.synchronize()
    start.record()
    for i in range(steps):
        r.render_async(ds, cams[timed_view(i, steps, len(cams))], cfg, out, events=frames[i][1])
    end.record()
    torch.cuda.synchronize()
    if int(r.status.item()) != 0:
        raise RuntimeError("tile entries overflowed the planned workspace during timing")
    total = start.elapsed_time(end)
    stages, scatter, kernels = [], [], []
    for evs, _ in frames:
        stages.append([evs[k].elapsed_time(evs[k + 1]) for k in range(4)])
        scatter.append([evs[5 + 2 * p].elapsed_time(evs[6 + 2 * p]) for p in range(passes)])
        k0 = 5 + 2 * passes    # per-tile ordering launch, then the first render launch
        kernels.append([evs[k0].elapsed_time(evs[k0 + 1]), evs[k0 + 2].elapsed_time(evs[k0 + 3])])
    return total / steps, stages, scatter, kernels


def time_simple(r, ds, cams, cfg, steps, warmup):
    """ms per frame over `steps` frames after `warmup` untimed ones."""
    import torch
    from paper_2402_00525_amd import gsr
    out = gsr.Frame(cams[0].H, cams[0].W, "cuda")
    for i in range(warmup):
        r.render_async(ds, cams[i % len(cams)], cfg, out)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    r.status.zero_()
    torch.cuda.synchronize()
    start.record()
    for i in range(steps):
        r.render_async(ds, cams[timed_view(i, steps, len(cams))], cfg, out)
    end.record()
    torch.cuda.synchronize()
    if int(r.status.item()) != 0:
        raise RuntimeError("tile entries overflowed the planned workspace during timing")
    return start.elapsed_time(end) / steps


def mode_sweep(ds, cams, n, sort_prefix):
    """The other renderers on the same scene and views: the per-ray resort
    window over the 3DGS list (Sec. 3.3), the hierarchical render with larger
    heads, the ablations of Table performance_ablation -- (B) no tile-depth
    adjustment, (C) no load balancing, (D) no tile culling, (E) no
    hierarchical culling --, a load-balancing threshold sweep, the 3DGS order
    keyed along each tile's centre ray (Fig. pertiledepth), and the full
    per-pixel sort (Sec. 3.2).  Each: plan over the views, 2 untimed frames,
    then one timed frame per view."""
    import torch
    from paper_2402_00525_amd import gsr
    H = gsr.MODE_HIER
    cases = [("window_K%d" % k, dict(mode=gsr.MODE_WINDOW, head=k)) for k in (4, 8, 16, 24)]
    cases += [("hier_K%d" % k, dict(mode=H, head=k)) for k in (4, 8, 16, 24)]
    cases += [("ablation_B_no_tile_depth", dict(mode=H, flags=gsr.ABLATE_TILE_DEPTH)),
              ("ablation_C_no_load_balancing", dict(mode=H, lb_threshold=gsr.NO_LOAD_BALANCE)),
              ("ablation_D_no_tile_culling", dict(mode=H, flags=gsr.ABLATE_TILE_CULL)),
              ("ablation_E_no_hier_culling", dict(mode=H, flags=gsr.ABLATE_HIER_CULL)),
              ("ablation_BCDE", dict(mode=H, lb_threshold=gsr.NO_LOAD_BALANCE,
                                     flags=gsr.ABLATE_TILE_DEPTH | gsr.ABLATE_TILE_CULL | gsr.ABLATE_HIER_CULL))]
    cases += [("lb_threshold_%d" % t, dict(mode=H, lb_threshold=t)) for t in (1, 4, 16, 32, 128, 256)]
    cases += [("global_tile_centre_depth", dict(mode=gsr.MODE_GLOBAL, flags=gsr.TILE_CENTRE_DEPTH))]
    cases += [("full_sort", dict(mode=gsr.MODE_FULL))]
    res = {}
    for name, kw in cases:
        if kw["mode"] in (H, gsr.MODE_FULL):
            kw["sort_prefix"] = sort_prefix
        cfg = gsr.config(**kw)
        r = gsr.Renderer(entries_hint=40 * n)
        emax, _ = plan(r, ds, cams, cfg)
        ms = time_simple(r, ds, cams, cfg, len(cams), 2)
        res[name] = {"ms_per_frame": round(ms, 4), "entries_max": int(emax)}
        log("mode %s: %.3f ms/frame (entries max %d)" % (name, ms, emax))
        del r
        torch.cuda.empty_cache()
    return res


def sort_errors(ds, cams, n):
    """Per-ray sort error (Sec. 3.3, the measure of Table sortcost) of every
    renderer on the given views: the maximum over pixels and the mean over
    pixels of each pixel's sum of out-of-order t_opt differences between
    consecutive blends (0 for the full per-pixel sort)."""
    import torch
    from paper_2402_00525_amd import gsr
    cases = [("global_3dgs", dict(mode=gsr.MODE_GLOBAL)),
             ("global_tile_centre_depth", dict(mode=gsr.MODE_GLOBAL, flags=gsr.TILE_CENTRE_DEPTH))]
    cases += [("window_K%d" % k, dict(mode=gsr.MODE_WINDOW, head=k)) for k in (4, 8, 16, 24)]
    cases += [("hier_K%d" % k, dict(mode=gsr.MODE_HIER, head=k)) for k in (4, 8, 16, 24)]
    cases += [("full_sort", dict(mode=gsr.MODE_FULL))]
    res = {}
    for name, kw in cases:
        r = gsr.Renderer(entries_hint=60 * n)
        dmax, dsum, pix = 0.0, 0.0, 0
        for cam in cams:
            _, d = r.render_sort_error(ds, cam, gsr.config(**kw))
            dmax = max(dmax, float(d.max()))
            dsum += float(d.double().sum())
            pix += d.numel()
        res[name] = {"delta_max": round(dmax, 4), "delta_avg": round(dsum / pix, 5)}
        log("sort error %s: %s" % (name, res[name]))
        del r
        torch.cuda.empty_cache()
    return res


ROTATION_VIEWS = (0, 15, 30, 45)
ROTATION_ANGLES = (-5.0, -2.0, -0.5, 0.5, 2.0, 5.0)


def rotation_sweep(ds, n, W, H):
    """Popping under pure camera rotation (Sec. 1 and Sec. 3).  At orbit views
    0, 15, 30 and 45 the camera turns about its centre by yaw, pitch and roll
    of +-0.5, +-2 and +-5 degrees, and rolls by 180 degrees.  The full
    per-pixel sort orders each pixel by t_opt along its own ray, which depends
    on the ray alone, so an order equal to it cannot pop.  For each renderer
    and angle this reports, averaged over the four views, the fraction of
    pixels whose first 16 blends differ from the full sort's and the per-ray
    sort error; for the 180-degree roll, which maps pixel (i, j) to
    (W-1-i, H-1-j) with the same world ray, the fraction of pixels whose first
    16 blends differ between the two views."""
    import torch
    from paper_2402_00525_amd import gsr, synth
    K = 16
    rend = {"hier_K4": dict(mode=gsr.MODE_HIER), "global_3dgs": dict(mode=gsr.MODE_GLOBAL),
            "window_K16": dict(mode=gsr.MODE_WINDOW, head=16)}
    rs = {k: gsr.Renderer(entries_hint=60 * n) for k in list(rend) + ["full_sort"]}
    cfgs = {k: gsr.config(**v) for k, v in rend.items()}
    cfgs["full_sort"] = gsr.config(mode=gsr.MODE_FULL)
    acc = {k: {} for k in rend}
    flips = {k: [] for k in cfgs}
    for v in ROTATION_VIEWS:
        base = synth.orbit_camera(W, H, v)
        rots = [("%s%+g" % (ax, a), synth.rotate_camera(base, **{ax + "_deg": a}))
                for ax in ("yaw", "pitch", "roll") for a in ROTATION_ANGLES]
        for name, cam in [("none", base)] + rots:
            full = rs["full_sort"].render(ds, cam, cfgs["full_sort"], max_k=K).blend_ids
            for k, cfg in ((k, cfgs[k]) for k in rend):
                ids = rs[k].render(ds, cam, cfg, max_k=K).blend_ids
                mis = float((ids != full).any(dim=-1).float().mean())
                _, d = rs[k].render_sort_error(ds, cam, cfg)
                a = acc[k].setdefault(name, [0.0, 0.0, 0.0])
                a[0] += mis / len(ROTATION_VIEWS)
                a[1] += float(d.double().mean()) / len(ROTATION_VIEWS)
                a[2] = max(a[2], float(d.max()))
        rolled = synth.roll_180(base)
        for k, cfg in cfgs.items():
            a = rs[k].render(ds, base, cfg, max_k=K).blend_ids
            b = rs[k].render(ds, rolled, cfg, max_k=K).blend_ids.flip(0).flip(1)
            flips[k].append(float((a != b).any(dim=-1).float().mean()))
        log("rotation sweep: view %d done" % v)
    res = {}
    for k in cfgs:
        e = {"roll180_pixels_changed": round(mean(flips[k]), 6)}
        if k in acc:
            e["vs_full_sort"] = {name: {"pixels_differing": round(a[0], 5), "delta_avg": round(a[1], 5),
                                        "delta_max": round(a[2], 4)} for name, a in acc[k].items()}
        res[k] = e
        log("rotation %s: roll180 %.5f" % (k, e["roll180_pixels_changed"]))
    del rs
    torch.cuda.empty_cache()
    return {"views": list(ROTATION_VIEWS), "angles_deg": list(ROTATION_ANGLES), "first_blends_compared": K,
            "results": res}


def plan(r, ds, cams, cfg):
    """Render every view once (untimed, with the overflow check) and size the
    workspace for the largest frame plus 5%."""
    import torch
    n = ds.n
    emax, consumed = 0, []
    for cam in cams:
        r.render(ds, cam, cfg)
        emax = max(emax, r.counter(n, cam, 0))
        consumed.append(r.counter(n, cam, 1))
    r.plan(n, cams[0].W, cams[0].H, int(emax * 1.05) + 1024)
    torch.cuda.synchronize()
    return emax, consumed


def mean(x):
    return sum(x) / max(1, len(x))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.lower().startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, cam, E):
    """The oracle on a bounded sample of the same frame: every per-Gaussian
    stage and the full sort, but the render on 1 tile in 256; the render time
    is scaled to the whole image."""
    import numpy as np
    import oracle
    tiles = ((cam.W + 15) // 16) * ((cam.H + 15) // 16)
    mask = np.zeros(tiles, np.uint8)
    mask[::256] = 1
    t0 = time.time()
    r = oracle.frame(scene, cam, mode=oracle.MODE_HIER, tile_mask=mask, want_entries=False, capacity=E + 1024)
    wall = time.time() - t0
    pre, dup, srt, ren = r.stats["ms"]
    est = pre + dup + srt + ren * tiles / int(mask.sum())
    return {"value": round(est, 1), "unit": "ms/frame", "cores": int(r.stats["threads"]), "kind": "oracle",
            "cpu": cpu_model(),
            "sample": "one %dx%d frame of the same scene: all %d Gaussians preprocessed, duplicated and sorted "
                      "(%d entries), hierarchical render on %d of %d tiles scaled to the full image; %.1f s wall"
                      % (cam.W, cam.H, scene.n, r.stats["entries"], int(mask.sum()), tiles, wall),
            "stages_ms": {"preprocess": round(pre, 1), "duplicate": round(dup, 1), "sort": round(srt, 1),
                          "render_scaled": round(ren * tiles / int(mask.sum()), 1)}}


def fwd_bwd(steps, warmup):
    """Forward + L1-loss gradient + backward on 500k mixture Gaussians at
    1280x720 (target: a seeded random image); returns ms per training step."""
    import torch
    from paper_2402_00525_amd import gsr, synth
    scene = synth.mixture_scene(500_000, seed=3)
    cams = [synth.orbit_camera(1280, 720, v) for v in range(0, 60, 6)]
    target = torch.from_numpy(synth.random_target(720, 1280, seed=4)).cuda()
    ds = gsr.DeviceScene.from_host(scene)
    cfg = gsr.config()
    r = gsr.Renderer(entries_hint=40 * scene.n)
    plan(r, ds, cams, cfg)
    out = gsr.Frame(720, 1280, "cuda")
    grads = {k: torch.empty_like(getattr(ds, k)) for k in ("means", "scales", "rots", "opacities", "sh")}

    def step(cam, evs=None):
        if evs is not None:
            evs[0].record()
        r.render_async(ds, cam, cfg, out)
        if evs is not None:
            evs[1].record()
        dL = torch.sign(out.rgb - target) / out.rgb.numel()
        g = gsr.render_backward(r, ds, cam, cfg, out, dL, check=False)
        if evs is not None:
            evs[2].record()
        return g

    for i in range(warmup):
        step(cams[i % len(cams)])
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    r.status.zero_()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for i in range(steps):
        step(cams[(warmup + i) % len(cams)], evs[i])
    t1.record()
    torch.cuda.synchronize()
    if int(r.status.item()) != 0:
        raise RuntimeError("overflow or workspace mismatch during fwd+bwd timing")
    fwd = mean([e[0].elapsed_time(e[1]) for e in evs])
    bwd = mean([e[1].elapsed_time(e[2]) for e in evs])
    return {"ms_per_step": round(t0.elapsed_time(t1) / steps, 4), "forward_ms": round(fwd, 4),
            "loss_and_backward_ms": round(bwd, 4),
            "workload": "500000-Gaussian mixture scene (SH degree 3), 1280x720, 10 orbit views, L1 loss to a "
                        "seeded random target, gradients for means/scales/rotations/opacities/SH"}


def single_view_reference(dss, views, steps):
    """The batch's views rendered one at a time through the plain single-view
    renderer (gsr_render): ms for all views, mean of `steps` passes after one
    planning pass."""
    import torch
    from paper_2402_00525_amd import gsr
    cfg = gsr.config()
    r = gsr.Renderer(entries_hint=1 << 20)
    outs = [gsr.Frame(c.H, c.W, "cuda") for _, c in views]
    emax = 0
    for s, c in views:
        r.render(dss[s], c, cfg)
        emax = max(emax, r.counter(dss[s].n, c, 0))
    nmax = max(d.n for d in dss)
    Wm, Hm = max(c.W for _, c in views), max(c.H for _, c in views)
    r.plan(nmax, Wm, Hm, int(emax * 1.05) + 1024)
    for (s, c), o in zip(views, outs):
        r.render_async(dss[s], c, cfg, o)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    r.status.zero_()
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        for (s, c), o in zip(views, outs):
            r.render_async(dss[s], c, cfg, o)
    t1.record()
    torch.cuda.synchronize()
    if int(r.status.item()) != 0:
        raise RuntimeError("overflow during the single-view reference of the batch")
    ms = t0.elapsed_time(t1) / steps
    log("batch views one at a time: %.2f ms for %d views" % (ms, len(views)))
    del r, outs
    torch.cuda.empty_cache()
    return ms


def batched(steps):
    """128 views (64 of the 1M-Gaussian scene, 8 each of 8 scenes with N
    log-uniform in [1e5, 2e6]) at resolutions drawn from 256^2, 512^2,
    1280x720 and 1920x1080, rendered by one captured HIP graph; the schedule is
    chosen by the autotuner first.  Returns views/s."""
    import torch
    from paper_2402_00525_amd import gsr, synth
    t0 = time.time()
    scenes, views = synth.batch_workload()
    log("batch workload generated in %.1fs (%d scenes, %d views)" % (time.time() - t0, len(scenes), len(views)))
    dss = [gsr.DeviceScene.from_host(s) for s in scenes]
    b = gsr.BatchRenderer(dss, views)
    b.render()
    torch.cuda.synchronize()
    E = b.entries()
    cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), "gsr_batch_schedule.txt")
    sched, tune_ms = b.tune(cache_path=cache, repeats=2)
    b.capture()
    b.replay()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.status.zero_()
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        b.replay()
    t1.record()
    torch.cuda.synchronize()
    if int(b.status.item()) != 0:
        raise RuntimeError("overflow during batched timing")
    ms = t0.elapsed_time(t1) / steps
    single_ms = single_view_reference(dss, views, steps=2)
    res = {"views_per_s": round(len(views) / (ms * 1e-3), 1), "ms_per_batch": round(ms, 3), "views": len(views),
           "single_view": {"views_per_s": round(len(views) / (single_ms * 1e-3), 1),
                           "ms_per_batch": round(single_ms, 3),
                           "how": "the same views rendered one after another through gsr_render (one workspace, "
                                  "one stream, no host synchronisation between views)"},
           "scenes": len(scenes), "gaussians": [s.n for s in scenes], "entries": int(E),
           "schedule": {"wgs_per_cu": sched.wgs_per_cu, "cost_order": sched.cost_order,
                        "lb_threshold": sched.lb_threshold},
           "workload": "64 views of the 1M-Gaussian scene + 8 views each of 8 scenes (N log-uniform in [1e5, 2e6]); "
                       "resolutions uniform over 256^2, 512^2, 1280x720, 1920x1080; one HIP graph per batch"}
    del b, dss
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build renders on one GPU only (the multi-GPU sharding is a design note); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2402_00525_amd import gsr, synth

    wl = WORKLOADS[args.workload]
    t0 = time.time()
    if args.workload == "small":
        scene, cam0 = synth.workload_small()
        cams = [cam0]
    else:
        scene = synth.mixture_scene(wl["n"], seed=wl["seed"])
        cams = [synth.orbit_camera(wl["W"], wl["H"], v) for v in range(0, 60, max(1, 60 // args.views))]
    log("scene generated in %.1fs" % (time.time() - t0))
    if args.copy_calibration_mib:
        src = torch.ones(args.copy_calibration_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d MiB read + %d MiB written" % (args.copy_calibration_mib, args.copy_calibration_mib))
        del src, dst
    if args.gather_calibration_mib:
        # rows of 16 float32 (64 bytes, the size of a packed splat) from a table
        # four times larger, at seeded random indices: reads the index array
        # and the gathered rows, writes the rows
        rows = args.gather_calibration_mib << 14
        table = torch.ones((4 * rows, 16), dtype=torch.float32, device="cuda")
        g = torch.Generator(device="cpu").manual_seed(0)
        idx = torch.randint(0, 4 * rows, (rows,), generator=g).cuda()
        out = torch.index_select(table, 0, idx)
        torch.cuda.synchronize()
        log("gather calibration: %d MiB of 64-byte rows gathered (+ %d MiB of int64 indices), %d MiB written" %
            (args.gather_calibration_mib, args.gather_calibration_mib // 8, args.gather_calibration_mib))
        del table, idx, out
    ds = gsr.DeviceScene.from_host(scene)
    n, W, H = scene.n, cams[0].W, cams[0].H
    P = W * H
    ksh = (scene.sh_degree + 1) ** 2

    results = {}
    for label, mode in (("hier", gsr.MODE_HIER), ("global", gsr.MODE_GLOBAL)):
        if label == "global" and args.no_global:
            continue
        cfg = gsr.config(mode=mode, sort_prefix=args.sort_prefix if mode == gsr.MODE_HIER else 0)
        passes = (gsr.lib().gsr_group_passes(W, H) if mode == gsr.MODE_HIER else gsr.lib().gsr_sort_passes(W, H))
        r = gsr.Renderer(entries_hint=40 * n)
        emax, consumed = plan(r, ds, cams, cfg)
        ms, stages, scatter, kernels = time_frames(r, ds, cams, cfg, args.steps, args.warmup, passes)
        # entries of the timed views (every view was rendered once while planning)
        views = [timed_view(i, args.steps, len(cams)) for i in range(args.steps)]
        E_views, cons_views, fb_views = [], [], []
        for v in sorted(set(views)):
            r.render(ds, cams[v], cfg)
            E_views.append(r.counter(n, cams[v], 0))
            cons_views.append(r.counter(n, cams[v], 1))
            fb_views.append(r.counter(n, cams[v], 5))
        results[label] = dict(ms=ms, stages=[mean([s[k] for s in stages]) for k in range(4)],
                              scatter=mean([mean(s) for s in scatter]) if passes else 0.0, E=mean(E_views),
                              consumed=mean(cons_views), fallback=mean(fb_views), emax=emax, passes=passes,
                              order_ms=mean([k[0] for k in kernels]), render_ms=mean([k[1] for k in kernels]))
        log("%s: %.3f ms/frame, stages %s, scatter %.3f ms/launch x %d, ordering %.3f ms, render %.3f ms, E %.0f, "
            "consumed %.0f, fallback entries %.0f" %
            (label, ms, ["%.3f" % x for x in results[label]["stages"]], results[label]["scatter"], passes,
             results[label]["order_ms"], results[label]["render_ms"], results[label]["E"], results[label]["consumed"],
             results[label]["fallback"]))
        del r
        torch.cuda.empty_cache()

    h = results["hier"]
    # Render work model: counted evaluations of one timed view x flops per
    # evaluation of the formulas (cull test: Algorithm 1 18, exponent 11, exp
    # 19, opacity 1; t_opt 26; pixel alpha 31; blend 14).
    r = gsr.Renderer(entries_hint=40 * n)
    r.plan(n, W, H, int(h["emax"] * 1.05) + 1024)
    timed = sorted(set(timed_view(i, args.steps, len(cams)) for i in range(args.steps)))
    works = [r.render_work(ds, cams[v], gsr.config(mode=gsr.MODE_HIER, sort_prefix=args.sort_prefix))[1]
             for v in timed]
    work = {k: int(round(mean([w[k] for w in works]))) for k in works[0]}
    del r
    torch.cuda.empty_cache()
    render_flops = (49.0 * (work["tail_tests"] + work["mid_tests"]) + 26.0 * (work["tail_keyed"] + work["mid_keyed"])
                    + 31.0 * work["head_tests"] + 26.0 * work["head_keyed"] + 14.0 * work["blends"])
    # Kernels of a hierarchical frame: (ms per frame, ms per launch, algorithmic HBM bytes per launch).
    pre_bytes = n * (44 + 12 * ksh) + n * 116          # inputs; records: splat 64, colour 16, zd 8, rect 16,
                                                       # kept-tile count 4 and mask 8
    dup_bytes = n * 108 + 12.0 * h["E"]                # records of every Gaussian; one key + id per entry
    cands = {
        "k_preprocess": (h["stages"][0], h["stages"][0], pre_bytes),
        "k_duplicate": (h["stages"][1], h["stages"][1], dup_bytes),
        "k_radix_scatter": (h["scatter"] * h["passes"], h["scatter"], 24.0 * h["E"]),
        "k_tile_prefix": (h["order_ms"], h["order_ms"], 16.0 * h["E"]),
        "k_render_hier1": (h["render_ms"], h["render_ms"], 80.0 * h["consumed"] + 24.0 * P),
    }
    kernels = {k: {"ms_per_frame": round(v[0], 4), "GBs": round(v[2] / (v[1] * 1e-3) / 1e9, 1)}
               for k, v in cands.items() if v[1] > 0}
    kernels["k_render_hier1"]["TFLOPs"] = round(render_flops / (h["render_ms"] * 1e-3) / 1e12, 3)
    dom = max(cands, key=lambda k: cands[k][0])
    per_frame, dur, nbytes = cands[dom]
    if dom == "k_render_hier1":
        # On-chip bound (LDS queues, VALU): the roofline is the vector ALU's.
        achieved = render_flops / (dur * 1e-3) / 1e12
        roofline = {"kernel": dom, "bound": "alu", "achieved": round(achieved, 3), "peak": ALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TFLOPS, 4),
                    "traffic": profiled_traffic(dom, args.workload),
                    "algorithmic_flops_per_launch": int(render_flops), "avg_launch_ms": round(dur, 4),
                    "work": work}
    else:
        achieved = nbytes / (dur * 1e-3) / 1e9
        roofline = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": profiled_traffic(dom, args.workload),
                    "algorithmic_bytes_per_launch": int(nbytes), "avg_launch_ms": round(dur, 4)}
    frame_bytes = pre_bytes + dup_bytes + h["passes"] * 32.0 * h["E"] + 16.0 * h["E"] + 80.0 * h["consumed"] \
        + 24.0 * P
    line = {
        "metric": METRIC, "value": round(h["ms"], 4), "unit": "ms/frame", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(h["ms"], 4), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": ("%d-Gaussian uniform scene (SH degree %d), %dx%d, one camera at distance 3, "
                                "hierarchical resort 64/8/4" % (n, scene.sh_degree, W, H)) if args.workload == "small"
                   else ("%d-Gaussian mixture scene (SH degree %d), %dx%d, 60-view orbit, hierarchical resort "
                         "64/8/4" % (n, scene.sh_degree, W, H)),
                   "gaussians": n, "width": W, "height": H, "views": len(cams), "head": 4},
        "stages_ms": {k: round(v, 4) for k, v in zip(("preprocess", "duplicate", "sort", "render"), h["stages"])},
        "entries": int(h["E"]), "entries_consumed": int(h["consumed"]), "fallback_entries": int(h["fallback"]),
        "frame_hbm_GBs": round(frame_bytes / (h["ms"] * 1e-3) / 1e9, 1),
        "roofline": roofline,
        "kernels": kernels,
    }
    if "global" in results:
        g = results["global"]
        line["global_order"] = {"ms_per_frame": round(g["ms"], 4), "entries": int(g["E"]),
                                "stages_ms": {k: round(v, 4) for k, v in
                                              zip(("preprocess", "duplicate", "sort", "render"), g["stages"])}}
    if not args.no_modes:
        log("mode sweep ...")
        line["modes"] = {"views": list(range(0, len(cams), 6)),
                         "results": mode_sweep(ds, cams[::6], n, args.sort_prefix)}
    if not args.no_sort_error:
        log("sort error ...")
        sel = [0, len(cams) // 2] if len(cams) > 1 else [0]
        line["sort_error"] = {"views": sel, "results": sort_errors(ds, [cams[v] for v in sel], n)}
    if not args.no_rotation and args.workload != "small":
        log("rotation sweep ...")
        line["rotation"] = rotation_sweep(ds, n, W, H)
    if not args.no_batch and args.workload != "small":
        log("batched ...")
        line["batched"] = batched(5)
        log("batched: %s" % line["batched"])
    if not args.no_fwd_bwd and args.workload != "small":
        log("forward+backward ...")
        line["fwd_bwd"] = fwd_bwd(max(5, args.steps // 2), 3)
        log("fwd+bwd: %s" % line["fwd_bwd"])
    if not args.no_cpu_baseline and args.workload != "small":
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(scene, cams[timed_view(0, args.steps, len(cams))], int(h["emax"]))
    elif not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(scene, cams[0], int(h["emax"]))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
