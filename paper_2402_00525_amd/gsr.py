"""Python binding of ``libgsr.so`` (the C ABI declared in ``include/gsr.h``).

Argument marshalling only: every step of a frame runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  If the
library is missing the binding raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsr.so")

GSR_OK, GSR_EINVAL, GSR_ECAPACITY, GSR_EDEVICE, GSR_EUNSUPPORTED = 0, -1, -2, -3, -4
MODE_GLOBAL, MODE_HIER, MODE_FULL, MODE_WINDOW = 0, 1, 2, 3
# Ablations of the hierarchical mode (gsr_config.flags) and the load-balancing
# threshold that turns load balancing off.
ABLATE_TILE_DEPTH, ABLATE_TILE_CULL, ABLATE_HIER_CULL = 1, 2, 4
TILE_CENTRE_DEPTH = 8
NO_LOAD_BALANCE = 1 << 30
STATUS_OVERFLOW = 1
STATUS_MISMATCH = 2


class GsrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("gsr error %d: %s" % (code, msg))
        self.code = code


class CScene(C.Structure):
    _fields_ = [("n", C.c_int32), ("sh_degree", C.c_int32), ("means", C.c_void_p), ("scales", C.c_void_p),
                ("rots", C.c_void_p), ("opacities", C.c_void_p), ("sh", C.c_void_p)]


class CCamera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("center", C.c_float * 3), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float), ("znear", C.c_float),
                ("W", C.c_int32), ("H", C.c_int32)]


class CConfig(C.Structure):
    _fields_ = [("mode", C.c_int32), ("batch", C.c_int32), ("tail", C.c_int32), ("pop", C.c_int32),
                ("mid", C.c_int32), ("mid_batch", C.c_int32), ("head", C.c_int32), ("lb_threshold", C.c_int32),
                ("bg", C.c_float * 3), ("flags", C.c_uint32), ("sort_prefix", C.c_int32)]


class CLayout(C.Structure):
    _fields_ = [(name, C.c_int64) for name in
                ("splat", "colour", "zd", "rect", "touched", "kmask", "offsets", "dup_hist", "grad2d", "keys",
                 "values",
                 "ranges", "counters", "pre_vals", "pre_len", "tile_flag", "entry_capacity", "total_bytes")]


_lib = None

EXPORTS = ("gsr_workspace_bytes", "gsr_workspace_layout", "gsr_default_config", "gsr_check_config",
           "gsr_render", "gsr_render_debug", "gsr_render_sort_error", "gsr_render_backward", "gsr_render_staged",
           "gsr_render_work", "gsr_render_noalloc",
           "gsr_sort_passes", "gsr_group_passes", "gsr_default_prefix",
           "gsr_probe_math",
           "gsr_last_error", "gsr_version")


def lib():
    """Load ``libgsr.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgsr.so is not built; run python -m paper_2402_00525_amd.build")
        L = C.CDLL(LIB_PATH)
        L.gsr_workspace_bytes.restype = C.c_size_t
        L.gsr_workspace_bytes.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_int64]
        L.gsr_workspace_layout.restype = C.c_int
        L.gsr_workspace_layout.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_size_t, C.POINTER(CLayout)]
        L.gsr_default_config.argtypes = [C.POINTER(CConfig)]
        L.gsr_check_config.argtypes = [C.POINTER(CConfig)]
        L.gsr_check_config.restype = C.c_int
        L.gsr_render.restype = C.c_int
        L.gsr_render.argtypes = [C.POINTER(CScene), C.POINTER(CCamera), C.POINTER(CConfig), C.c_void_p, C.c_size_t,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.gsr_render_debug.restype = C.c_int
        L.gsr_render_debug.argtypes = [C.POINTER(CScene), C.POINTER(CCamera), C.POINTER(CConfig), C.c_void_p,
                                       C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_int32, C.c_void_p, C.c_void_p]
        L.gsr_render_sort_error.restype = C.c_int
        L.gsr_render_sort_error.argtypes = [C.POINTER(CScene), C.POINTER(CCamera), C.POINTER(CConfig), C.c_void_p,
                                            C.c_size_t] + [C.c_void_p] * 7
        L.gsr_render_backward.restype = C.c_int
        L.gsr_render_backward.argtypes = [C.POINTER(CScene), C.POINTER(CCamera), C.POINTER(CConfig), C.c_void_p,
                                          C.c_size_t] + [C.c_void_p] * 10
        L.gsr_render_work.restype = C.c_int
        L.gsr_render_work.argtypes = [C.POINTER(CScene), C.POINTER(CCamera), C.POINTER(CConfig), C.c_void_p,
                                      C.c_size_t] + [C.c_void_p] * 6 + [C.c_void_p]
        L.gsr_render_staged.restype = C.c_int
        L.gsr_render_staged.argtypes = [C.POINTER(CScene), C.POINTER(CCamera), C.POINTER(CConfig), C.c_void_p,
                                        C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_int32]
        L.gsr_render_noalloc.restype = C.c_int
        L.gsr_render_noalloc.argtypes = [C.POINTER(CScene), C.POINTER(CCamera), C.POINTER(CConfig)] + [C.c_void_p] * 6
        L.gsr_sort_passes.restype = C.c_int
        L.gsr_sort_passes.argtypes = [C.c_int32, C.c_int32]
        L.gsr_group_passes.restype = C.c_int
        L.gsr_group_passes.argtypes = [C.c_int32, C.c_int32]
        L.gsr_default_prefix.restype = C.c_int
        L.gsr_default_prefix.argtypes = [C.c_int32, C.c_int32, C.c_int32]
        L.gsr_probe_math.restype = C.c_int
        L.gsr_probe_math.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.gsr_last_error.restype = C.c_char_p
        L.gsr_version.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != GSR_OK:
        raise GsrError(rc, lib().gsr_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def config(mode=MODE_HIER, head=4, lb_threshold=64, bg=(0.0, 0.0, 0.0), sort_prefix=0, flags=0) -> CConfig:
    c = CConfig()
    lib().gsr_default_config(C.byref(c))
    c.mode, c.head, c.lb_threshold, c.sort_prefix, c.flags = mode, head, lb_threshold, sort_prefix, flags
    for i in range(3):
        c.bg[i] = bg[i]
    return c


def camera(cam) -> CCamera:
    """Convert any object with R, t, center, fx, fy, cx, cy, W, H, znear."""
    c = CCamera()
    R = [float(v) for v in cam.R.reshape(-1)]
    for i in range(9):
        c.R[i] = R[i]
    for i in range(3):
        c.t[i] = float(cam.t[i])
        c.center[i] = float(cam.center[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.znear = float(getattr(cam, "znear", 0.2))
    c.W, c.H = int(cam.W), int(cam.H)
    return c


@dataclass
class DeviceScene:
    """Gaussian parameters resident on the GPU (float32, contiguous)."""
    means: torch.Tensor
    scales: torch.Tensor
    rots: torch.Tensor
    opacities: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @staticmethod
    def from_host(scene, device="cuda") -> "DeviceScene":
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)
        return DeviceScene(f(scene.means), f(scene.scales), f(scene.rots), f(scene.opacities), f(scene.sh),
                           int(scene.sh_degree))

    def c_struct(self) -> CScene:
        s = CScene()
        s.n, s.sh_degree = self.n, self.sh_degree
        s.means, s.scales, s.rots = self.means.data_ptr(), self.scales.data_ptr(), self.rots.data_ptr()
        s.opacities, s.sh = self.opacities.data_ptr(), self.sh.data_ptr()
        return s


def workspace_bytes(n, W, H, entries_max) -> int:
    b = lib().gsr_workspace_bytes(n, W, H, entries_max)
    if b == 0:
        raise GsrError(GSR_EINVAL, "bad workspace request")
    return int(b)


def layout(n, W, H, ws_bytes) -> CLayout:
    L = CLayout()
    _check(lib().gsr_workspace_layout(n, W, H, ws_bytes, C.byref(L)))
    return L


class Frame:
    """Outputs of one render plus a view of the workspace it used."""

    def __init__(self, H, W, device, max_k=0):
        self.rgb = torch.empty((3, H, W), dtype=torch.float32, device=device)
        self.depth = torch.empty((H, W), dtype=torch.float32, device=device)
        self.count = torch.empty((H, W), dtype=torch.int32, device=device)
        self.T = torch.empty((H, W), dtype=torch.float32, device=device)
        self.blend_ids = torch.empty((H, W, max_k), dtype=torch.int32, device=device) if max_k > 0 else None


class Renderer:
    """Holds a workspace and renders frames into it.

    ``render`` checks the device status word after the frame (one host
    synchronisation) and grows the workspace when the tile entries overflowed;
    ``render_async`` enqueues without any host synchronisation.
    """

    def __init__(self, device="cuda", entries_hint: int = 1 << 20):
        self.device = torch.device(device)
        self.entries_hint = int(entries_hint)
        self.ws = None
        self.ws_key = None
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)

    def plan(self, n, W, H, entries):
        nbytes = workspace_bytes(n, W, H, max(1, int(entries)))
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ws_key = (n, W, H)
        return self.ws

    def render_async(self, scene: DeviceScene, cam, cfg: CConfig, out: Frame, max_k: int = 0, events=None):
        """Enqueue one frame.  ``events``: optional ctypes array of hipEvent_t
        handles recorded at the stage boundaries (see gsr_render_staged)."""
        if self.ws is None:
            self.plan(scene.n, cam.W, cam.H, self.entries_hint)
        sc, cc = scene.c_struct(), camera(cam)
        if events is not None:
            rc = lib().gsr_render_staged(C.byref(sc), C.byref(cc), C.byref(cfg), _ptr(self.ws), self.ws.numel(),
                                         _ptr(out.rgb), _ptr(out.depth), _ptr(out.count), _ptr(out.T),
                                         _ptr(self.status), _stream(), events, len(events))
        elif max_k > 0:
            rc = lib().gsr_render_debug(C.byref(sc), C.byref(cc), C.byref(cfg), _ptr(self.ws), self.ws.numel(),
                                        _ptr(out.rgb), _ptr(out.depth), _ptr(out.count), _ptr(out.T),
                                        _ptr(out.blend_ids), max_k, _ptr(self.status), _stream())
        else:
            rc = lib().gsr_render(C.byref(sc), C.byref(cc), C.byref(cfg), _ptr(self.ws), self.ws.numel(),
                                  _ptr(out.rgb), _ptr(out.depth), _ptr(out.count), _ptr(out.T), _ptr(self.status),
                                  _stream())
        _check(rc)
        return out

    WORK_NAMES = ("tail_tests", "tail_keyed", "mid_tests", "mid_keyed", "head_tests", "head_keyed", "blends")

    def render_work(self, scene: DeviceScene, cam, cfg: CConfig | None = None):
        """Render once with the render's work counters (gsr_render_work);
        returns (frame, dict of counts).  Synchronises."""
        cfg = cfg or config()
        out = Frame(cam.H, cam.W, self.device)
        work = torch.zeros(len(self.WORK_NAMES), dtype=torch.int64, device=self.device)
        if self.ws is None:
            self.plan(scene.n, cam.W, cam.H, self.entries_hint)
        sc, cc = scene.c_struct(), camera(cam)
        _check(lib().gsr_render_work(C.byref(sc), C.byref(cc), C.byref(cfg), _ptr(self.ws), self.ws.numel(),
                                     _ptr(out.rgb), _ptr(out.depth), _ptr(out.count), _ptr(out.T), _ptr(self.status),
                                     _ptr(work), _stream()))
        torch.cuda.synchronize()
        if int(self.status.item()) != 0:
            raise GsrError(GSR_ECAPACITY, "tile entries overflowed the workspace")
        return out, dict(zip(self.WORK_NAMES, work.cpu().tolist()))

    def render_sort_error(self, scene: DeviceScene, cam, cfg: CConfig | None = None):
        """Render once with each pixel's sort error (gsr_render_sort_error);
        returns (frame, sort_error [H,W] float32 tensor).  Synchronises."""
        cfg = cfg or config()
        out = Frame(cam.H, cam.W, self.device)
        delta = torch.empty((cam.H, cam.W), dtype=torch.float32, device=self.device)
        if self.ws is None:
            self.plan(scene.n, cam.W, cam.H, self.entries_hint)
        sc, cc = scene.c_struct(), camera(cam)
        self.status.zero_()
        _check(lib().gsr_render_sort_error(C.byref(sc), C.byref(cc), C.byref(cfg), _ptr(self.ws), self.ws.numel(),
                                           _ptr(out.rgb), _ptr(out.depth), _ptr(out.count), _ptr(out.T),
                                           _ptr(delta), _ptr(self.status), _stream()))
        torch.cuda.synchronize()
        if int(self.status.item()) != 0:
            raise GsrError(GSR_ECAPACITY, "tile entries overflowed the workspace")
        return out, delta

    def render(self, scene: DeviceScene, cam, cfg: CConfig | None = None, max_k: int = 0) -> Frame:
        cfg = cfg or config()
        out = Frame(cam.H, cam.W, self.device, max_k)
        if self.ws is None:
            self.plan(scene.n, cam.W, cam.H, self.entries_hint)
        for _ in range(4):
            self.status.zero_()
            self.render_async(scene, cam, cfg, out, max_k)
            st = int(self.status.item())
            if not (st & STATUS_OVERFLOW):
                return out
            need = self.counter(scene.n, cam, 3) & 0xffffffff
            self.plan(scene.n, cam.W, cam.H, max(int(need * 1.05) + 1024, 2 * self.capacity(scene.n, cam)))
        raise GsrError(GSR_ECAPACITY, "tile entries keep overflowing the workspace")

    # ----- workspace inspection (debugging / tests) -----
    def capacity(self, n, cam) -> int:
        return int(layout(n, cam.W, cam.H, self.ws.numel()).entry_capacity)

    def region(self, n, cam, name, dtype, count):
        L = layout(n, cam.W, cam.H, self.ws.numel())
        off = getattr(L, name)
        nbytes = count * torch.tensor([], dtype=dtype).element_size()
        return self.ws[off:off + nbytes].view(dtype)

    def counter(self, n, cam, k):
        """counters[k]: 0 entries, 1 entries consumed by the renderer, 3 entries
        needed, 5 entries and 6 number of the tiles that took the fallback."""
        c = self.region(n, cam, "counters", torch.int32, 8)
        return int(c[k].item())

    def records(self, n, cam):
        """Per-Gaussian records of the last frame (device tensors): the packed
        splat and colour as stored, and views of them by quantity -- xy (2D
        mean), conic_o (a, b, c, opacity), sw (Sigma^-1, w, rgb)."""
        splat = self.region(n, cam, "splat", torch.float32, 16 * n).view(n, 16)
        colour = self.region(n, cam, "colour", torch.float32, 4 * n).view(n, 4)
        return dict(
            xy=splat[:, 0:2],
            conic_o=splat[:, 2:6],
            sw=torch.cat([splat[:, 6:15], colour[:, 0:3]], dim=1),
            splat=splat,
            colour=colour,
            zd=self.region(n, cam, "zd", torch.float32, 2 * n).view(n, 2),
            rect=self.region(n, cam, "rect", torch.int32, 4 * n).view(n, 4),
            touched=self.region(n, cam, "touched", torch.int32, n),
        )

    def sorted_entries(self, n, cam):
        E = self.counter(n, cam, 0)
        keys = self.region(n, cam, "keys", torch.int64, E)
        vals = self.region(n, cam, "values", torch.int32, E)
        tiles = ((cam.W + 15) // 16) * ((cam.H + 15) // 16)
        ranges = self.region(n, cam, "ranges", torch.int32, 2 * tiles).view(tiles, 2)
        return keys, vals, ranges

    def tile_lists(self, n, cam):
        """Per-tile sorted ids of the last frame (a prefix, or the whole list
        for tiles that took the fallback) as host numpy arrays; pre_vals is
        indexed by range start."""
        E = self.counter(n, cam, 0)
        F = self.counter(n, cam, 5)
        tiles = ((cam.W + 15) // 16) * ((cam.H + 15) // 16)
        get = lambda name, dt, cnt: self.region(n, cam, name, dt, cnt).cpu().numpy().copy()
        return dict(ranges=get("ranges", torch.int32, 2 * tiles).reshape(tiles, 2),
                    pre_vals=get("pre_vals", torch.int32, E), pre_len=get("pre_len", torch.int32, tiles),
                    tile_flag=get("tile_flag", torch.int32, tiles), fallback_entries=F,
                    fallback_tiles=self.counter(n, cam, 6))


NOALLOC_BYTES = 64 << 20  # GSR_NOALLOC_BYTES


def render_noalloc(scene: DeviceScene, cam, cfg: CConfig | None = None, out: Frame | None = None,
                   status: torch.Tensor | None = None) -> Frame:
    """gsr_render_noalloc: one frame in the library's fixed per-GPU workspace
    (no device allocation by the library).  Enqueues only; the caller reads
    ``status`` (bit 0: entries overflowed the fixed workspace)."""
    cfg = cfg or config()
    dev = scene.means.device
    out = out or Frame(cam.H, cam.W, dev)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    sc, cc = scene.c_struct(), camera(cam)
    _check(lib().gsr_render_noalloc(C.byref(sc), C.byref(cc), C.byref(cfg), _ptr(out.rgb), _ptr(out.depth),
                                    _ptr(out.count), _ptr(out.T), _ptr(status), _stream()))
    return out


def probe_math(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    n = a.numel()
    out = torch.empty(6 * n, dtype=torch.float32, device=a.device)
    _check(lib().gsr_probe_math(_ptr(a), _ptr(b), n, _ptr(out), _stream()))
    return out.view(6, n)


# ---------------------------------------------------------------------------
# Differentiable rendering (torch.autograd.Function over gsr_render /
# gsr_render_backward).
# ---------------------------------------------------------------------------
_ENTRY_HINTS = {}


def _sh_degree(sh: torch.Tensor) -> int:
    k = int(sh.shape[1])
    d = {1: 0, 4: 1, 9: 2, 16: 3}.get(k)
    if d is None:
        raise GsrError(GSR_EINVAL, "sh must be [N,(d+1)^2,3] with d in 0..3")
    return d


class RenderFunction(torch.autograd.Function):
    """rgb = render(means, scales, rots, opacities, sh) for one camera, with
    the hierarchical per-pixel order; the backward re-runs the same order front
    to back inside the library.  depth, count and T are returned without
    gradients."""

    @staticmethod
    def forward(ctx, means, scales, rots, opacities, sh, cam, cfg):
        ds = DeviceScene(means.detach().contiguous(), scales.detach().contiguous(), rots.detach().contiguous(),
                         opacities.detach().contiguous(), sh.detach().contiguous(), _sh_degree(sh))
        key = (ds.n, int(cam.W), int(cam.H))
        # every call gets its own workspace: the backward needs it untouched
        r = Renderer(device=means.device, entries_hint=_ENTRY_HINTS.get(key, max(1 << 16, 32 * ds.n)))
        out = r.render(ds, cam, cfg)
        _ENTRY_HINTS[key] = int(1.2 * r.counter(ds.n, cam, 0)) + 1024
        ctx.state = (r, ds, cam, cfg, out)
        ctx.mark_non_differentiable(out.depth, out.count, out.T)
        return out.rgb, out.depth, out.count, out.T

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_count, g_T):
        r, ds, cam, cfg, out = ctx.state
        g_rgb = g_rgb.contiguous() if g_rgb is not None else torch.zeros_like(out.rgb)
        dm, dsc, drt = torch.empty_like(ds.means), torch.empty_like(ds.scales), torch.empty_like(ds.rots)
        dop, dsh = torch.empty_like(ds.opacities), torch.empty_like(ds.sh)
        sc, cc = ds.c_struct(), camera(cam)
        # The workspace is this Function's own, untouched since the forward,
        # so the fingerprint check cannot fail here; no synchronisation.
        _check(lib().gsr_render_backward(C.byref(sc), C.byref(cc), C.byref(cfg), _ptr(r.ws), r.ws.numel(),
                                         _ptr(g_rgb), _ptr(out.rgb), _ptr(out.T), _ptr(dm), _ptr(dsc), _ptr(drt),
                                         _ptr(dop), _ptr(dsh), _ptr(r.status), _stream()))
        ctx.state = None
        return dm, dsc, drt, dop, dsh, None, None


def render(means, scales, rots, opacities, sh, cam, cfg: CConfig | None = None):
    """Differentiable render of one view: returns (rgb [3,H,W], depth, count, T)."""
    return RenderFunction.apply(means, scales, rots, opacities, sh, cam, cfg or config())


def render_backward(renderer: Renderer, scene: DeviceScene, cam, cfg: CConfig, frame: Frame, dL_drgb,
                    check: bool = True):
    """Gradients of a frame rendered with ``renderer.render`` (direct C-ABI
    call).  With ``check`` the call clears the renderer's status word,
    synchronises once and raises if the renderer's workspace does not hold
    the forward of this scene, camera and configuration (the library then
    returns zero gradients); without it nothing waits and a mismatch only
    sets bit 1 of the status word."""
    grads = dict(means=torch.empty_like(scene.means), scales=torch.empty_like(scene.scales),
                 rots=torch.empty_like(scene.rots), opacities=torch.empty_like(scene.opacities),
                 sh=torch.empty_like(scene.sh))
    sc, cc = scene.c_struct(), camera(cam)
    if check:
        renderer.status.zero_()
    _check(lib().gsr_render_backward(C.byref(sc), C.byref(cc), C.byref(cfg), _ptr(renderer.ws), renderer.ws.numel(),
                                     _ptr(dL_drgb.contiguous()), _ptr(frame.rgb), _ptr(frame.T), _ptr(grads["means"]),
                                     _ptr(grads["scales"]), _ptr(grads["rots"]), _ptr(grads["opacities"]),
                                     _ptr(grads["sh"]), _ptr(renderer.status), _stream()))
    if check and int(renderer.status.item()) & STATUS_MISMATCH:
        raise GsrError(GSR_EINVAL, "the workspace does not hold the forward of this scene, camera and configuration")
    return grads


# ---------------------------------------------------------------------------
# Batched rendering (gsr_batch_*)
# ---------------------------------------------------------------------------
class CView(C.Structure):
    _fields_ = [("scene", C.c_int32), ("cam", CCamera), ("rgb", C.c_void_p), ("depth", C.c_void_p),
                ("count", C.c_void_p), ("T", C.c_void_p)]


class CSchedule(C.Structure):
    _fields_ = [("wgs_per_cu", C.c_int32), ("cost_order", C.c_int32), ("lb_threshold", C.c_int32)]


_BATCH_FNS = {
    "gsr_batch_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int64]),
    "gsr_default_schedule": (None, [C.c_void_p]),
    "gsr_batch_create": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_size_t, C.c_void_p]),
    "gsr_batch_render": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_batch_set_schedule": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gsr_batch_get_schedule": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gsr_batch_tune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_char_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "gsr_batch_records": (C.c_int64, [C.c_void_p]),
    "gsr_batch_tiles": (C.c_int64, [C.c_void_p]),
    "gsr_batch_entry_capacity": (C.c_int64, [C.c_void_p]),
    "gsr_batch_counters_offset": (C.c_int64, [C.c_void_p]),
    "gsr_batch_destroy": (None, [C.c_void_p]),
}
EXPORTS = EXPORTS + tuple(_BATCH_FNS)


def _blib():
    L = lib()
    if not getattr(L, "_batch_ready", False):
        for name, (res, args) in _BATCH_FNS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        L._batch_ready = True
    return L


def schedule(wgs_per_cu=None, cost_order=None, lb_threshold=None) -> CSchedule:
    s = CSchedule()
    _blib().gsr_default_schedule(C.byref(s))
    if wgs_per_cu is not None:
        s.wgs_per_cu = wgs_per_cu
    if cost_order is not None:
        s.cost_order = cost_order
    if lb_threshold is not None:
        s.lb_threshold = lb_threshold
    return s


class BatchRenderer:
    """Many views of several scenes rendered by one launch sequence
    (gsr_batch_render), optionally captured once into a HIP graph and replayed.

    scenes: list of DeviceScene; views: list of (scene index, camera)."""

    def __init__(self, scenes, views, cfg: CConfig | None = None, sched: CSchedule | None = None,
                 entries_hint: int | None = None, device="cuda"):
        self.device = torch.device(device)
        self.scenes = scenes
        self.cfg = cfg or config()
        self.sched = sched
        self.frames = [Frame(cam.H, cam.W, self.device) for _, cam in views]
        self.cscenes = (CScene * len(scenes))(*[s.c_struct() for s in scenes])
        self.cviews = (CView * len(views))()
        for k, (si, cam) in enumerate(views):
            f = self.frames[k]
            self.cviews[k].scene = si
            self.cviews[k].cam = camera(cam)
            self.cviews[k].rgb, self.cviews[k].depth = f.rgb.data_ptr(), f.depth.data_ptr()
            self.cviews[k].count, self.cviews[k].T = f.count.data_ptr(), f.T.data_ptr()
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.handle = None
        self.ws = None
        self.graph = None
        records = sum(scenes[si].n for si, _ in views)
        self._plan(entries_hint or min((1 << 31) - 1, 16 * records + (1 << 20)))

    def _plan(self, entries):
        L = _blib()
        self.close_plan()
        nbytes = L.gsr_batch_workspace_bytes(self.cscenes, len(self.cscenes), self.cviews, len(self.cviews),
                                             int(entries))
        if nbytes == 0:
            raise GsrError(GSR_EINVAL, L.gsr_last_error().decode())
        self.ws = None
        torch.cuda.empty_cache()
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(L.gsr_batch_create(self.cscenes, len(self.cscenes), self.cviews, len(self.cviews), C.byref(self.cfg),
                                  C.byref(self.sched) if self.sched is not None else None, _ptr(self.ws), nbytes,
                                  C.byref(h)))
        self.handle = h
        self.graph = None

    def close_plan(self):
        if self.handle is not None:
            _blib().gsr_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close_plan()
        except Exception:
            pass

    @property
    def n_views(self):
        return len(self.frames)

    def counters(self):
        off = _blib().gsr_batch_counters_offset(self.handle)
        return self.ws[off:off + 32].view(torch.int32)

    def capacity(self):
        return int(_blib().gsr_batch_entry_capacity(self.handle))

    def render_async(self):
        """Enqueue the batch (no synchronisation)."""
        _check(_blib().gsr_batch_render(self.handle, _ptr(self.status), _stream()))

    def render(self):
        """Render with the overflow check; grows the workspace until the entries fit."""
        for _ in range(8):
            self.status.zero_()
            self.render_async()
            if int(self.status.item()) & STATUS_OVERFLOW == 0:
                return self.frames
            need = int(self.counters()[3].item()) & 0xffffffff
            if need >= (1 << 31) - 1:
                raise GsrError(GSR_ECAPACITY, "batch needs more than 2^31 entries")
            self._plan(min((1 << 31) - 1, int(need * 1.05) + 1024))
        raise GsrError(GSR_ECAPACITY, "batch entries keep overflowing")

    def entries(self) -> int:
        return int(self.counters()[0].item())

    def tune(self, cache_path=None, repeats=3):
        best, ms = CSchedule(), C.c_float()
        self.status.zero_()
        _check(_blib().gsr_batch_tune(self.handle, _ptr(self.status), _stream(),
                                      cache_path.encode() if cache_path else None, repeats, C.byref(best),
                                      C.byref(ms)))
        self.sched = best
        self.graph = None
        return best, ms.value

    def set_schedule(self, sched: CSchedule):
        _check(_blib().gsr_batch_set_schedule(self.handle, C.byref(sched)))
        self.sched = sched
        self.graph = None

    def get_schedule(self) -> CSchedule:
        s = CSchedule()
        _check(_blib().gsr_batch_get_schedule(self.handle, C.byref(s)))
        return s

    def capture(self):
        """Capture one gsr_batch_render into a HIP graph (torch.cuda.CUDAGraph)."""
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.render_async()
        torch.cuda.synchronize()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
