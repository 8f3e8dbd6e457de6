"""Helpers for the GPU tests: run a frame through the C ABI and fetch every
intermediate to host numpy arrays."""
import sys

import numpy as np
import torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_frame(scene, cam, mode=1, head=4, max_k=0, entries_hint=None, renderer=None, sort_prefix=0, flags=0,
              lb_threshold=64):
    from paper_2402_00525_amd import gsr
    ds = gsr.DeviceScene.from_host(scene)
    r = renderer or gsr.Renderer(entries_hint=entries_hint or max(1 << 16, 64 * scene.n))
    cfg = gsr.config(mode=mode, head=head, sort_prefix=sort_prefix, flags=flags, lb_threshold=lb_threshold)
    out = r.render(ds, cam, cfg, max_k=max_k)
    torch.cuda.synchronize()
    n = scene.n
    rec = {k: v.cpu().numpy() for k, v in r.records(n, cam).items()} if n > 0 else {}
    keys, vals, ranges = r.sorted_entries(n, cam)
    res = dict(rgb=out.rgb.cpu().numpy(), depth=out.depth.cpu().numpy(), count=out.count.cpu().numpy(),
               T=out.T.cpu().numpy(), keys=keys.cpu().numpy().view(np.uint64), values=vals.cpu().numpy().view(np.uint32),
               ranges=ranges.cpu().numpy().view(np.uint32), consumed=r.counter(n, cam, 1), **rec)
    res["mode"] = mode
    res["flags"] = flags
    res["sort_prefix"] = sort_prefix or gsr.lib().gsr_default_prefix(cam.W, cam.H, mode)
    res["lists"] = r.tile_lists(n, cam)
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
    if g.get("mode", 0) in (1, 2) and not (g.get("flags", 0) & 2):
        # Hierarchical lists: the GPU bounds a Gaussian by its alpha ellipse's
        # box, inside the oracle's lambda_max square; exact culling keeps the
        # same tiles either way (touched is equal above).
        gr, orr = g["rect"][vis], o.rect[vis]
        live = o.touched[vis] > 0
        assert np.all(gr[live, :2] >= orr[live, :2]) and np.all(gr[live, 2:] <= orr[live, 2:])
    else:
        np.testing.assert_array_equal(g["rect"], o.rect)
    # the renderer's packed copy holds the same bits, and ln(eps_O / opacity)
    pk = g["splat"]
    ref = np.concatenate([o.xy, o.conic_o, o.sw[:, :9]], axis=1)
    live = o.conic_o[:, 3] > 0
    ref[~live] = 0.0
    np.testing.assert_array_equal(pk[:, :15].view(np.uint32), ref.view(np.uint32))
    lt = np.log((1.0 / 255.0) / o.conic_o[live, 3].astype(np.float64))
    np.testing.assert_allclose(pk[live, 15], lt, rtol=0, atol=2e-6)
    assert np.all(pk[~live, 15] == 0.0)


def assert_sorted_equal(g, o):
    """Every order (its own keys: t_opt through x^ in the hierarchical
    order, view depth in the global one): the entries grouped by tile are the
    oracle's (as a set per tile, in any order inside a tile), every tile's
    sorted prefix is the start of the oracle's sorted list, and every tile
    that took the fallback has the oracle's whole sorted list."""
    assert len(g["keys"]) == len(o.keys), (len(g["keys"]), len(o.keys))
    np.testing.assert_array_equal(g["ranges"], o.ranges)
    L = g["lists"]
    ov = o.values.view(np.uint32)
    flag = L["tile_flag"].view(np.uint32)
    if L["fallback_entries"] == 0:
        k, v = g["keys"], g["values"]
        tile = k >> np.uint64(32)
        assert np.all(np.diff(tile.astype(np.int64)) >= 0)
        order = np.lexsort((v, k))
        np.testing.assert_array_equal(k[order], o.keys)
        np.testing.assert_array_equal(v[order], ov)
    M = g["sort_prefix"]
    pre, plen = L["pre_vals"].view(np.uint32), L["pre_len"]
    rng = L["ranges"]
    assert int(flag.astype(np.int64).sum()) == L["fallback_entries"]
    assert int((flag > 0).sum()) == L["fallback_tiles"]
    for t in range(len(rng)):
        rb, re = int(rng[t, 0]), int(rng[t, 1])
        n, c = re - rb, int(plen[t])
        if flag[t]:
            assert flag[t] == n and c == n, (t, n, c)
        else:
            assert c <= min(n, M) and (n > M or c == n), (t, n, c)
        np.testing.assert_array_equal(pre[rb:rb + c], ov[rb:rb + c])


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
