"""The C-ABI library loads, exports every function the header declares, and
its host-only entry points (workspace planning, configuration checks) behave
as documented.  No kernel is launched here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsr.h")


@pytest.fixture(scope="module")
def L():
    from paper_2402_00525_amd import gsr
    if not os.path.exists(gsr.LIB_PATH):
        from paper_2402_00525_amd import build
        build.build()
    return gsr


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function(L):
    names = declared_functions()
    assert "gsr_render" in names and len(names) >= 8
    lib = C.CDLL(L.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(L.EXPORTS) <= set(names)


def test_version_and_default_config(L):
    assert b"gfx950" in L.lib().gsr_version()
    c = L.config()
    assert (c.mode, c.batch, c.tail, c.pop, c.mid, c.mid_batch, c.head, c.lb_threshold) == (1, 32, 64, 16, 8, 4, 4, 64)
    assert c.sort_prefix == 0
    assert L.lib().gsr_check_config(C.byref(c)) == 0
    for m in (1, 100, 4096, 16384):
        c.sort_prefix = m
        assert L.lib().gsr_check_config(C.byref(c)) == 0
    c.sort_prefix = 16385
    assert L.lib().gsr_check_config(C.byref(c)) == -1
    c.sort_prefix = 0
    for f in (1, 2, 4, 7):                                # ablations of the hierarchical mode
        c.flags = f
        assert L.lib().gsr_check_config(C.byref(c)) == 0
    c.mode = L.MODE_GLOBAL
    assert L.lib().gsr_check_config(C.byref(c)) == -1    # ablations need GSR_MODE_HIER
    c.flags = L.TILE_CENTRE_DEPTH                         # naive per-tile depth of the 3DGS order
    assert L.lib().gsr_check_config(C.byref(c)) == 0
    for m in (L.MODE_HIER, L.MODE_WINDOW, L.MODE_FULL):
        c.mode = m
        assert L.lib().gsr_check_config(C.byref(c)) == -1
    c.mode = L.MODE_GLOBAL
    c.flags = L.TILE_CENTRE_DEPTH | 1
    assert L.lib().gsr_check_config(C.byref(c)) == -1
    c.flags = 0
    c.mode = L.MODE_WINDOW                                # per-ray window of `head` samples
    for K, code in ((1, 0), (24, 0), (25, -4), (0, -1)):
        c.head = K
        assert L.lib().gsr_check_config(C.byref(c)) == code


@pytest.mark.parametrize("field,value,code", [
    ("tail", 48, -1), ("tail", 96, -4), ("mid", 6, -1), ("mid", 12, -4), ("head", 0, -1), ("head", 25, -4),
    ("mode", 7, -1), ("mode", -1, -1), ("flags", 8, -1), ("flags", 16, -1), ("lb_threshold", -1, -1), ("sort_prefix", -1, -1),
    ("sort_prefix", 16385, -1)])
def test_config_validation(L, field, value, code):
    # Sec. 3.4: tail = 32n+32, mid = 4m+4, head >= 1; only the built sizes run.
    c = L.config()
    setattr(c, field, value)
    assert L.lib().gsr_check_config(C.byref(c)) == code
    assert len(L.lib().gsr_last_error()) > 0


def test_workspace_planning_roundtrip(L):
    for n, W, H, E in [(2000, 128, 128, 10000), (1_000_000, 1920, 1080, 30_000_000), (0, 16, 16, 1), (5, 1, 1, 7)]:
        nbytes = L.workspace_bytes(n, W, H, E)
        lay = L.layout(n, W, H, nbytes)
        assert lay.entry_capacity >= E
        assert lay.total_bytes <= nbytes
        offs = sorted([lay.splat, lay.colour, lay.zd, lay.rect, lay.touched, lay.offsets, lay.keys,
                       lay.values, lay.ranges, lay.counters])
        assert all(o % 256 == 0 for o in offs)
        assert len(set(offs)) == len(offs) or n == 0


def test_workspace_errors(L):
    assert L.lib().gsr_workspace_bytes(-1, 16, 16, 10) == 0
    assert L.lib().gsr_workspace_bytes(10, 0, 16, 10) == 0
    with pytest.raises(L.GsrError) as e:
        L.layout(1000, 64, 64, 1024)
    assert e.value.code == L.GSR_ECAPACITY


def _batch_structs(L, sizes):
    from paper_2402_00525_amd import gsr
    scenes = (gsr.CScene * 2)()
    for k, n in enumerate((1000, 500)):
        scenes[k].n, scenes[k].sh_degree = n, 3
        for f in ("means", "scales", "rots", "opacities", "sh"):
            setattr(scenes[k], f, 0x1000)       # never dereferenced by the host functions
    views = (gsr.CView * len(sizes))()
    for k, (W, H) in enumerate(sizes):
        views[k].scene = k % 2
        views[k].cam.W, views[k].cam.H, views[k].cam.fx, views[k].cam.fy = W, H, 100.0, 100.0
        views[k].rgb = views[k].depth = views[k].count = views[k].T = 0x1000
    return scenes, views


def test_batch_workspace_planning(L):
    from paper_2402_00525_amd import gsr
    B = gsr._blib()
    scenes, views = _batch_structs(L, [(256, 256), (1920, 1080), (33, 17)])
    small = B.gsr_batch_workspace_bytes(scenes, 2, views, 3, 1000)
    big = B.gsr_batch_workspace_bytes(scenes, 2, views, 3, 10_000_000)
    assert 0 < small < big
    assert big - small >= 24 * (10_000_000 - 1000)      # two key and two value buffers
    assert B.gsr_batch_workspace_bytes(scenes, 2, views, 3, 0) == 0
    views[1].scene = 5                                    # out-of-range scene index
    assert B.gsr_batch_workspace_bytes(scenes, 2, views, 3, 1000) == 0
    s = gsr.schedule()
    assert (s.wgs_per_cu, s.cost_order, s.lb_threshold) == (2, 1, 64)


def test_sort_pass_count(L):
    # global order: grouping over every tile bit, digits of at most 9 bits
    assert L.lib().gsr_sort_passes(1920, 1080) == 2      # 8160 tiles -> 13 bits
    assert L.lib().gsr_sort_passes(128, 128) == 1        # 64 tiles -> 6 bits
    assert L.lib().gsr_sort_passes(16, 16) == 0          # 1 tile
    # grouping by tile: duplication buckets the low 5 tile bits, radix passes the rest
    assert L.lib().gsr_group_passes(1920, 1080) == 1     # 13 bits
    assert L.lib().gsr_group_passes(80, 64) == 0         # 20 tiles, 5 bits
    assert L.lib().gsr_group_passes(128, 128) == 1       # 6 bits
    assert L.lib().gsr_group_passes(7680, 4320) == 2     # 129600 tiles, 17 bits
    assert L.lib().gsr_group_passes(16, 16) == 0
    assert L.lib().gsr_group_passes(0, 16) < 0


def test_default_prefix_by_image_size(L):
    # about 2^23 sorted entries per frame (2^25 for the 3DGS lists), a power
    # of two between 1024 (4096) and 8192; below 512 tiles 0 (whole lists sorted up front)
    f = L.lib().gsr_default_prefix
    assert f(1920, 1080, L.MODE_HIER) == 1024
    assert f(1280, 720, L.MODE_HIER) == 2048
    assert f(512, 512, L.MODE_HIER) == 8192
    assert f(256, 256, L.MODE_HIER) == 0
    assert f(128, 128, L.MODE_HIER) == 0 and f(368, 352, L.MODE_HIER) == 0 and f(368, 368, L.MODE_HIER) == 8192
    assert f(3840, 2160, L.MODE_HIER) == 1024
    assert f(1920, 1080, L.MODE_GLOBAL) == 4096
    assert f(512, 512, L.MODE_WINDOW) == 8192
    assert f(256, 256, L.MODE_WINDOW) == 0
    assert f(0, 10, L.MODE_HIER) < 0 and f(10, 10, 9) < 0
