"""Helpers for the GPU tests: run a frame through the C ABI and fetch every
intermediate to host numpy arrays."""
import sys

import numpy as np
import torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_frame(scene, cam, mode=1, head=4, max_k=0, entries_hint=None, renderer=None):
    from paper_2402_00525_amd import gsr
    ds = gsr.DeviceScene.from_host(scene)
    r = renderer or gsr.Renderer(entries_hint=entries_hint or max(1 << 16, 64 * scene.n))
    cfg = gsr.config(mode=mode, head=head)
    out = r.render(ds, cam, cfg, max_k=max_k)
    torch.cuda.synchronize()
    n = scene.n
    rec = {k: v.cpu().numpy() for k, v in r.records(n, cam).items()} if n > 0 else {}
    keys, vals, ranges = r.sorted_entries(n, cam)
    res = dict(rgb=out.rgb.cpu().numpy(), depth=out.depth.cpu().numpy(), count=out.count.cpu().numpy(),
               T=out.T.cpu().numpy(), keys=keys.cpu().numpy().view(np.uint64), values=vals.cpu().numpy().view(np.uint32),
               ranges=ranges.cpu().numpy().view(np.uint32), consumed=r.counter(n, cam, 1), **rec)
    if max_k > 0:
        res["blend_ids"] = out.blend_ids.cpu().numpy()
    return res


def assert_records_equal(g, o):
    np.testing.assert_array_equal(g["touched"], o.touched)
    vis = o.touched >= 0
    np.testing.assert_array_equal(g["xy"][vis].view(np.uint32), o.xy[vis].view(np.uint32))
    np.testing.assert_array_equal(g["conic_o"].view(np.uint32), o.conic_o.view(np.uint32))
    np.testing.assert_array_equal(g["sw"].view(np.uint32), o.sw.view(np.uint32))
    np.testing.assert_array_equal(g["zd"].view(np.uint32), o.zd.view(np.uint32))
    np.testing.assert_array_equal(g["rect"], o.rect)


def assert_sorted_equal(g, o):
    assert len(g["keys"]) == len(o.keys), (len(g["keys"]), len(o.keys))
    np.testing.assert_array_equal(g["keys"], o.keys)
    np.testing.assert_array_equal(g["values"], o.values)
    np.testing.assert_array_equal(g["ranges"], o.ranges)


def assert_images_close(g, o, tol=1e-4, mask=None):
    sel = (slice(None),) if mask is None else (mask,)
    for name in ("rgb", "depth", "T"):
        a, b = g[name], getattr(o, name)
        if name == "rgb":
            a = a[:, mask] if mask is not None else a
            b = b[:, mask] if mask is not None else b
        elif mask is not None:
            a, b = a[mask], b[mask]
        d = np.abs(a.astype(np.float64) - b.astype(np.float64))
        assert d.max() <= tol, (name, d.max())
    a, b = g["count"], o.count
    if mask is not None:
        a, b = a[mask], b[mask]
    np.testing.assert_array_equal(a, b)
