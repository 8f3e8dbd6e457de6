"""ctypes front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

The oracle (``gsr_oracle.cpp``) is a plain CPU statement of the sorted
Gaussian-splatting frame.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module; the product library in
``paper_2402_00525_amd`` never does.  It shares no code with the HIP path: its
inputs come from ``paper_2402_00525_amd.synth`` (input drawing only).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gsr_oracle.cpp")
LIB = os.path.join(HERE, "libgsr_oracle.so")

MODE_GLOBAL, MODE_HIER, MODE_FULL, MODE_WINDOW = 0, 1, 2, 3

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with plain IEEE float semantics (no contraction, no fast math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


class OCam(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("center", C.c_float * 3),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("znear", C.c_float), ("W", C.c_int32), ("H", C.c_int32)]


class OCfg(C.Structure):
    _fields_ = [("mode", C.c_int32), ("batch", C.c_int32), ("tail", C.c_int32), ("pop", C.c_int32),
                ("mid", C.c_int32), ("mid_batch", C.c_int32), ("head", C.c_int32), ("bg", C.c_float * 3),
                ("flags", C.c_int32)]


class OFrameOut(C.Structure):
    _fields_ = [("xy", C.c_void_p), ("conic_o", C.c_void_p), ("sw", C.c_void_p), ("zd", C.c_void_p),
                ("rect", C.c_void_p), ("touched", C.c_void_p), ("keys", C.c_void_p),
                ("values", C.c_void_p), ("capacity", C.c_int64), ("n_entries", C.c_int64),
                ("ranges", C.c_void_p), ("rgb", C.c_void_p), ("depth", C.c_void_p),
                ("count", C.c_void_p), ("T", C.c_void_p), ("blend_ids", C.c_void_p),
                ("max_k", C.c_int32), ("delta", C.c_void_p), ("stats", C.c_int64 * 12), ("tile_mask", C.c_void_p),
                ("ms", C.c_double * 4), ("threads", C.c_int32), ("signature", C.c_uint64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        L.oracle_frame_f32.restype = C.c_int
        L.oracle_frame_f64.restype = C.c_int
        L.oracle_exp_f32.restype = C.c_float
        L.oracle_exp_f32.argtypes = [C.c_float]
        L.oracle_ln_f32.restype = C.c_float
        L.oracle_ln_f32.argtypes = [C.c_float]
        L.oracle_sh_basis.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_void_p]
        L.oracle_sh_basis_f32.argtypes = [C.c_int, C.c_float, C.c_float, C.c_float, C.c_void_p]
        L.oracle_alg1.argtypes = [C.c_double] * 9 + [C.c_void_p]
        L.oracle_topt_f64.argtypes = [C.c_void_p] * 7
        L.oracle_topt_f64.restype = C.c_int
        L.oracle_ray_f64.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_void_p]
        L.oracle_ray_f32.argtypes = [C.c_void_p, C.c_float, C.c_float, C.c_void_p]
        L.oracle_backward_f64.restype = C.c_int
        L.oracle_backward_f32.restype = C.c_int
        L.oracle_grad2d_f64.restype = C.c_int
        L.oracle_chain_f64.restype = C.c_int
        L.oracle_chain_f32.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def ocam(cam) -> OCam:
    c = OCam()
    for i in range(9):
        c.R[i] = float(cam.R.reshape(-1)[i])
    for i in range(3):
        c.t[i] = float(cam.t[i])
        c.center[i] = float(cam.center[i])
    c.fx, c.fy, c.cx, c.cy, c.znear = cam.fx, cam.fy, cam.cx, cam.cy, cam.znear
    c.W, c.H = cam.W, cam.H
    return c


# Ablations of the hierarchical mode (see the C++ source): no tile-depth
# adjustment, no tile-based culling, no culling at the 4x4 / 2x2 levels.
ABL_TILE_DEPTH, ABL_TILE_CULL, ABL_HIER_CULL = 1, 2, 4
TILE_CENTRE_DEPTH = 8  # global order keyed along each tile's centre ray (Sec. 3.3)


def ocfg(mode=MODE_HIER, head=4, tail=64, mid=8, batch=32, pop=16, mid_batch=4, bg=(0.0, 0.0, 0.0),
         flags=0) -> OCfg:
    f = OCfg()
    f.mode, f.batch, f.tail, f.pop, f.mid, f.mid_batch, f.head = mode, batch, tail, pop, mid, mid_batch, head
    f.flags = flags
    for i in range(3):
        f.bg[i] = bg[i]
    return f


@dataclass
class FrameResult:
    xy: np.ndarray
    conic_o: np.ndarray
    sw: np.ndarray
    zd: np.ndarray
    rect: np.ndarray
    touched: np.ndarray
    keys: np.ndarray
    values: np.ndarray
    ranges: np.ndarray
    rgb: np.ndarray
    depth: np.ndarray
    count: np.ndarray
    T: np.ndarray
    blend_ids: np.ndarray | None
    delta: np.ndarray
    stats: dict


def _scene_arrays(scene):
    return [np.ascontiguousarray(a, dtype=np.float32) for a in
            (scene.means, scene.scales, scene.rots, scene.opacities, scene.sh)]


def frame(scene, cam, mode=MODE_HIER, head=4, max_k=0, precision="f32", tile_mask=None, capacity=None,
          want_entries=True, **cfgkw) -> FrameResult:
    """Run the whole frame on the CPU and return every intermediate.  With
    ``tile_mask`` (uint8 per tile) only those tiles are rendered; per-Gaussian
    records and the sorted entries are always complete."""
    L = lib()
    n = scene.n
    arrs = _scene_arrays(scene)
    H, W = cam.H, cam.W
    tiles = ((W + 15) // 16) * ((H + 15) // 16)
    dt = np.float32 if precision == "f32" else np.float64
    xy = np.zeros((n, 2), np.float32)
    conic_o = np.zeros((n, 4), np.float32)
    sw = np.zeros((n, 12), np.float32)
    zd = np.zeros((n, 2), np.float32)
    rect = np.zeros((n, 4), np.int32)
    touched = np.zeros(n, np.int32)
    ranges = np.zeros((tiles, 2), np.uint32)
    rgb = np.zeros((3, H, W), dt)
    depth = np.zeros((H, W), dt)
    count = np.zeros((H, W), np.int32)
    T = np.zeros((H, W), dt)
    delta = np.zeros((H, W), np.float32)
    bids = np.zeros((H, W, max_k), np.int32) if max_k > 0 else None
    cap = int(capacity) if capacity is not None else 64 * n + 4096
    for attempt in range(2):
        keys = np.empty(max(cap, 1), np.uint64) if want_entries else None
        values = np.empty(max(cap, 1), np.uint32) if want_entries else None
        o = OFrameOut()
        o.xy, o.conic_o, o.sw, o.zd, o.rect, o.touched = map(_p, (xy, conic_o, sw, zd, rect, touched))
        o.keys, o.values, o.capacity = _p(keys), _p(values), cap
        o.ranges, o.count, o.delta = _p(ranges), _p(count), _p(delta)
        o.blend_ids, o.max_k = _p(bids), max_k
        mask = None if tile_mask is None else np.ascontiguousarray(tile_mask, dtype=np.uint8)
        o.tile_mask = _p(mask)
        oc, of = ocam(cam), ocfg(mode=mode, head=head, **cfgkw)
        if precision == "f32":
            o.rgb, o.depth, o.T = _p(rgb), _p(depth), _p(T)
            rc = L.oracle_frame_f32(C.c_int(n), C.c_int(scene.sh_degree), *map(_p, arrs), C.byref(oc), C.byref(of), C.byref(o))
        else:
            rc = L.oracle_frame_f64(C.c_int(n), C.c_int(scene.sh_degree), *map(_p, arrs), C.byref(oc), C.byref(of), C.byref(o),
                                    _p(rgb), _p(depth), _p(T))
        if rc == -2:
            cap = int(o.n_entries)
            continue
        if rc != 0:
            raise RuntimeError("oracle failed: %d" % rc)
        break
    E = int(o.n_entries)
    st = list(o.stats)
    stats = dict(tail_in=st[0], mid_in=st[1], head_in=st[2], blends=st[3], max_tail=st[4], max_mid=st[5],
                 max_head=st[6], min_tail_after_pop=st[7], entries=st[8], ms=list(o.ms), threads=int(o.threads),
                 signature=int(o.signature))
    if want_entries:
        keys, values = keys[:E], values[:E]
    return FrameResult(xy, conic_o, sw, zd, rect, touched, keys, values, ranges, rgb, depth, count, T,
                       bids, delta, stats)


def exp32(x: float) -> np.float32:
    return np.float32(lib().oracle_exp_f32(float(x)))


def ln32(x: float) -> np.float32:
    return np.float32(lib().oracle_ln_f32(float(x)))


def sh_basis(deg, d, precision="f64"):
    if precision == "f64":
        b = np.zeros(16, np.float64)
        lib().oracle_sh_basis(deg, float(d[0]), float(d[1]), float(d[2]), _p(b))
    else:
        b = np.zeros(16, np.float32)
        lib().oracle_sh_basis_f32(deg, float(d[0]), float(d[1]), float(d[2]), _p(b))
    return b[: (deg + 1) ** 2]


def alg1(mean, conic, box):
    out = np.zeros(2, np.float64)
    lib().oracle_alg1(*[float(v) for v in mean], *[float(v) for v in conic], *[float(v) for v in box], _p(out))
    return out


def topt(mu, s, q, cam, d):
    """t_opt (double) of a Gaussian along unit direction d from the camera centre."""
    mu, s, q = (np.ascontiguousarray(a, dtype=np.float32) for a in (mu, s, q))
    d = np.ascontiguousarray(d, dtype=np.float64)
    t = np.zeros(1, np.float64)
    sinv = np.zeros(6, np.float64)
    oc = ocam(cam)
    rc = lib().oracle_topt_f64(_p(mu), _p(s), _p(q), C.byref(oc), _p(d), _p(t), _p(sinv))
    if rc != 0:
        raise ValueError("Gaussian culled")
    return float(t[0]), sinv


def ray(cam, u, v, precision="f64"):
    oc = ocam(cam)
    if precision == "f64":
        d = np.zeros(3, np.float64)
        lib().oracle_ray_f64(C.byref(oc), float(u), float(v), _p(d))
    else:
        d = np.zeros(3, np.float32)
        lib().oracle_ray_f32(C.byref(oc), float(u), float(v), _p(d))
    return d


def backward(scene, cam, dL_drgb, precision="f64", head=4, mode=MODE_HIER, bg=(0.0, 0.0, 0.0)):
    """Forward + backward of one frame (Sec. 3.5): returns the image, the
    gradients of sum(dL_drgb * rgb) with respect to every Gaussian parameter,
    and the decision signature of the frame."""
    L = lib()
    n, K = scene.n, (scene.sh_degree + 1) ** 2
    dt = np.float64 if precision == "f64" else np.float32
    dL = np.ascontiguousarray(dL_drgb, dtype=dt)
    g = dict(means=np.zeros((n, 3), dt), scales=np.zeros((n, 3), dt), rots=np.zeros((n, 4), dt),
             opacities=np.zeros(n, dt), sh=np.zeros((n, K, 3), dt))
    rgb = np.zeros((3, cam.H, cam.W), dt)
    sig = np.zeros(1, np.uint64)
    oc, of = ocam(cam), ocfg(mode=mode, head=head, bg=bg)
    fn = L.oracle_backward_f64 if precision == "f64" else L.oracle_backward_f32
    rc = fn(C.c_int(n), C.c_int(scene.sh_degree), *map(_p, _scene_arrays(scene)), C.byref(oc), C.byref(of), _p(dL),
            _p(g["means"]), _p(g["scales"]), _p(g["rots"]), _p(g["opacities"]), _p(g["sh"]), _p(rgb), _p(sig))
    if rc != 0:
        raise RuntimeError("oracle backward failed: %d" % rc)
    return rgb, g, int(sig[0])


GRAD2D_NAMES = ("mean_x", "mean_y", "conic_a", "conic_b", "conic_c", "opacity", "r", "g", "b")


def grad2d(scene, cam, dL_drgb, head=4, mode=MODE_HIER, bg=(0.0, 0.0, 0.0)):
    """Float64 gradients of sum(dL_drgb * rgb) with respect to every
    Gaussian's 2D quantities [N,9] (GRAD2D_NAMES order), a bound [N,9] on the
    magnitudes each is summed from, and the number of blends [N]."""
    L = lib()
    n = scene.n
    g2 = np.zeros((n, 9), np.float64)
    bd = np.zeros((n, 9), np.float64)
    nt = np.zeros(n, np.int32)
    dL = np.ascontiguousarray(dL_drgb, dtype=np.float64)
    oc, of = ocam(cam), ocfg(mode=mode, head=head, bg=bg)
    rc = L.oracle_grad2d_f64(C.c_int(n), C.c_int(scene.sh_degree), *map(_p, _scene_arrays(scene)), C.byref(oc),
                             C.byref(of), _p(dL), _p(g2), _p(bd), _p(nt))
    if rc != 0:
        raise RuntimeError("oracle grad2d failed: %d" % rc)
    return g2, bd, nt


def chain(scene, cam, g2, mode=MODE_HIER, precision="f64"):
    """Parameter gradients from given 2D gradients g2 [N,9], computed in
    float64 (or in float32 arithmetic with ``precision="f32"``)."""
    L = lib()
    n, K = scene.n, (scene.sh_degree + 1) ** 2
    g = dict(means=np.zeros((n, 3)), scales=np.zeros((n, 3)), rots=np.zeros((n, 4)), opacities=np.zeros(n),
             sh=np.zeros((n, K, 3)))
    g2 = np.ascontiguousarray(g2, dtype=np.float64)
    oc, of = ocam(cam), ocfg(mode=mode)
    fn = L.oracle_chain_f64 if precision == "f64" else L.oracle_chain_f32
    rc = fn(C.c_int(n), C.c_int(scene.sh_degree), *map(_p, _scene_arrays(scene)), C.byref(oc), C.byref(of),
            _p(g2), _p(g["means"]), _p(g["scales"]), _p(g["rots"]), _p(g["opacities"]), _p(g["sh"]))
    if rc != 0:
        raise RuntimeError("oracle chain failed: %d" % rc)
    return g
