"""Seeded synthetic scenes and cameras.

This module only draws inputs: Gaussian parameters and camera poses.  It holds
none of the rasterizer's arithmetic and is the single source of inputs for both
the HIP path and the CPU oracle.  Everything is drawn in float64 with
``numpy.random.Generator(PCG64(seed))`` and rounded to float32 once.

The paper evaluates on trained captures (Mip-NeRF 360, Deep Blending, Tanks &
Temples; Sec. 4) that are not available here.  The scenes below stand in for
them with the shapes of the paper's workloads: millions of anisotropic
Gaussians with degree-3 SH colour, rendered at 1920x1080 (Sec. 4.3).

Camera convention: world->camera rotation ``R`` (row-major 3x3), translation
``t`` with ``p_cam = R p_world + t``, camera centre ``center = -R^T t``.  The
camera looks along +z, x points right and y points down.  Pixel (i, j) has
its centre at image coordinates (i, j); the principal point is the image
centre ((W-1)/2, (H-1)/2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SH_COEFFS = {0: 1, 1: 4, 2: 9, 3: 16}


@dataclass
class Scene:
    means: np.ndarray      # [N,3] f32
    scales: np.ndarray     # [N,3] f32, activated (> 0)
    rots: np.ndarray       # [N,4] f32, quaternion (w, x, y, z), not normalised
    opacities: np.ndarray  # [N]   f32, activated, in [0, 1]
    sh: np.ndarray         # [N,(d+1)^2,3] f32
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])


@dataclass
class Camera:
    R: np.ndarray       # [3,3] f32 world->camera
    t: np.ndarray       # [3] f32
    center: np.ndarray  # [3] f32 camera centre in world space
    fx: float
    fy: float
    cx: float
    cy: float
    W: int
    H: int
    znear: float = 0.2


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _random_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def uniform_scene(n: int = 2000, seed: int = 0, sh_degree: int = 0) -> Scene:
    """Centres U[-1,1]^3, log-uniform scales in [0.01, 0.1] per axis, random unit
    quaternions, opacity U[0.05, 0.99].  At degree 0 the DC coefficient is drawn
    U[-sqrt(pi), sqrt(pi)], which maps to a base colour in [0, 1]; higher
    coefficients (degree > 0) are N(0, 0.2^2)."""
    rng = _rng(seed)
    means = rng.uniform(-1.0, 1.0, (n, 3))
    scales = np.exp(rng.uniform(math.log(0.01), math.log(0.1), (n, 3)))
    rots = _random_quats(rng, n)
    opac = rng.uniform(0.05, 0.99, n)
    k = SH_COEFFS[sh_degree]
    sh = np.empty((n, k, 3))
    sh[:, 0, :] = rng.uniform(-math.sqrt(math.pi), math.sqrt(math.pi), (n, 3))
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.2, (n, k - 1, 3))
    return Scene(_f32(means), _f32(scales), _f32(rots), _f32(opac), _f32(sh), sh_degree)


def mixture_scene(n: int, seed: int, sh_degree: int = 3, components: int = 64,
                  scale_median: float = 0.02, scale_sigma: float = 0.5) -> Scene:
    """Outdoor-capture-like density: centres from a ``components``-way Gaussian
    mixture (weights Dirichlet(1), component means U[-1,1]^3, per-axis component
    std log-uniform in [0.05, 0.3]); log-normal scales with median
    ``scale_median`` and log-std ``scale_sigma``; opacity Beta(2,2); SH
    coefficients N(0, 0.2^2) for every band including DC."""
    rng = _rng(seed)
    w = rng.dirichlet(np.ones(components))
    cmeans = rng.uniform(-1.0, 1.0, (components, 3))
    cstd = np.exp(rng.uniform(math.log(0.05), math.log(0.3), (components, 3)))
    comp = rng.choice(components, size=n, p=w)
    means = cmeans[comp] + cstd[comp] * rng.standard_normal((n, 3))
    scales = scale_median * np.exp(scale_sigma * rng.standard_normal((n, 3)))
    rots = _random_quats(rng, n)
    opac = rng.beta(2.0, 2.0, n)
    k = SH_COEFFS[sh_degree]
    sh = rng.normal(0.0, 0.2, (n, k, 3))
    return Scene(_f32(means), _f32(scales), _f32(rots), _f32(opac), _f32(sh), sh_degree)


def look_at(position, target=(0.0, 0.0, 0.0), up=(0.0, -1.0, 0.0)):
    """World->camera rotation (rows: right, down, forward) and translation."""
    c = np.asarray(position, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - c
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ c
    return R, t, c


def pinhole(W: int, H: int, fov_x_deg: float, R, t, center, znear: float = 0.2) -> Camera:
    """Pinhole camera with horizontal field of view ``fov_x_deg`` and square pixels."""
    fx = (W / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(R=_f32(R), t=_f32(t), center=_f32(center), fx=float(np.float32(fx)),
                  fy=float(np.float32(fx)), cx=float(np.float32((W - 1) / 2.0)),
                  cy=float(np.float32((H - 1) / 2.0)), W=int(W), H=int(H), znear=znear)


def camera_with_pose(W, H, fov_x_deg, R, center, znear: float = 0.2) -> Camera:
    """Camera from a world->camera rotation and a centre (t = -R c in float64)."""
    R = np.asarray(R, dtype=np.float64)
    c = np.asarray(center, dtype=np.float64)
    return pinhole(W, H, fov_x_deg, R, -R @ c, c, znear)


def front_camera(W: int = 128, H: int = 128, fov_x_deg: float = 60.0, dist: float = 3.0) -> Camera:
    """Camera at (0, 0, -dist) looking along +z at the origin (R = I)."""
    R, t, c = look_at((0.0, 0.0, -dist))
    return pinhole(W, H, fov_x_deg, R, t, c)


def orbit_camera(W: int, H: int, view: int, n_views: int = 60, elevation_deg: float = 20.0,
                 radius: float = 3.0, fov_x_deg: float = 60.0) -> Camera:
    """View ``view`` of an orbit about the origin: azimuth steps of 360/n_views
    degrees, fixed elevation above the horizontal plane (world up is -y)."""
    az = math.radians(360.0 * view / n_views)
    el = math.radians(elevation_deg)
    pos = (radius * math.cos(el) * math.sin(az), -radius * math.sin(el),
           -radius * math.cos(el) * math.cos(az))
    R, t, c = look_at(pos)
    return pinhole(W, H, fov_x_deg, R, t, c)


def rotate_camera(cam: Camera, yaw_deg: float = 0.0, pitch_deg: float = 0.0,
                  roll_deg: float = 0.0) -> Camera:
    """Pure rotation about the camera centre (the centre stays bit-identical).
    Yaw turns about the camera y axis, pitch about x, roll about z."""
    def rot(axis, ang):
        c, s = math.cos(ang), math.sin(ang)
        if axis == 0:
            return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
        if axis == 1:
            return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
        return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
    Q = rot(2, math.radians(roll_deg)) @ rot(0, math.radians(pitch_deg)) @ rot(1, math.radians(yaw_deg))
    R = Q @ cam.R.astype(np.float64)
    c = cam.center.astype(np.float64)
    out = Camera(R=_f32(R), t=_f32(-R @ c), center=cam.center.copy(), fx=cam.fx, fy=cam.fy,
                 cx=cam.cx, cy=cam.cy, W=cam.W, H=cam.H, znear=cam.znear)
    return out


def roll_180(cam: Camera) -> Camera:
    """Exact 180 degree roll about the optical axis: negates the first two rows of R
    (exact in float32) and keeps the centre, so pixel (i, j) maps to
    (W-1-i, H-1-j) with bit-identical world rays."""
    R = cam.R.copy()
    R[0] = -R[0]
    R[1] = -R[1]
    t = cam.t.copy()
    t[0] = -t[0]
    t[1] = -t[1]
    return Camera(R=R, t=t, center=cam.center.copy(), fx=cam.fx, fy=cam.fy, cx=cam.cx,
                  cy=cam.cy, W=cam.W, H=cam.H, znear=cam.znear)


# ----------------------------------------------------------------------------
# Named workloads (sizes of the paper's evaluation, Sec. 4.3, on synthetic data)
# ----------------------------------------------------------------------------

def workload_small():
    """2k uniform Gaussians, degree 0, one 128x128 camera at distance 3."""
    return uniform_scene(2000, seed=0, sh_degree=0), front_camera(128, 128)


def workload_1080p(n: int = 1_000_000, seed: int = 1, view: int = 0):
    """Mixture scene with degree-3 SH at 1920x1080, view ``view`` of a 60-view orbit."""
    return mixture_scene(n, seed), orbit_camera(1920, 1080, view)


def workload_720p(n: int = 500_000, seed: int = 3, view: int = 0):
    return mixture_scene(n, seed), orbit_camera(1280, 720, view)


def random_target(H: int, W: int, seed: int = 4) -> np.ndarray:
    """Seeded target image U[0,1]^{3,H,W} for the L1 loss of the backward pass."""
    return _f32(_rng(seed).uniform(0.0, 1.0, (3, H, W)))


def subsample(scene: Scene, n: int, seed: int = 123) -> Scene:
    """Deterministic subset of ``n`` Gaussians (same distribution, fewer points)."""
    idx = np.sort(_rng(seed).choice(scene.n, size=n, replace=False))
    return Scene(scene.means[idx].copy(), scene.scales[idx].copy(), scene.rots[idx].copy(),
                 scene.opacities[idx].copy(), scene.sh[idx].copy(), scene.sh_degree)


BATCH_RESOLUTIONS = ((256, 256), (512, 512), (1280, 720), (1920, 1080))


def sphere_camera(W: int, H: int, azimuth_deg: float, elevation_deg: float, radius: float = 3.0,
                  fov_x_deg: float = 60.0) -> Camera:
    az, el = math.radians(azimuth_deg), math.radians(elevation_deg)
    pos = (radius * math.cos(el) * math.sin(az), -radius * math.sin(el), -radius * math.cos(el) * math.cos(az))
    R, t, c = look_at(pos)
    return pinhole(W, H, fov_x_deg, R, t, c)


def batch_views(n_views: int, rng: np.random.Generator, scene_index: int):
    """Cameras with resolutions drawn uniformly from 256^2, 512^2, 1280x720,
    1920x1080 and poses uniform on the radius-3 sphere about the origin with
    elevation in [-30, 60] degrees."""
    out = []
    for _ in range(n_views):
        W, H = BATCH_RESOLUTIONS[int(rng.integers(0, len(BATCH_RESOLUTIONS)))]
        az = float(rng.uniform(0.0, 360.0))
        # uniform on the sphere band: sin(elevation) uniform
        el = math.degrees(math.asin(rng.uniform(math.sin(math.radians(-30.0)), math.sin(math.radians(60.0)))))
        out.append((scene_index, sphere_camera(W, H, az, el)))
    return out


def batch_workload(scale: float = 1.0, seed: int = 6, views_a: int = 64, views_b: int = 8, n_b: int = 8):
    """One 1M-Gaussian mixture scene (the 1080p scene, seed 1) seen by 64
    cameras, plus 8 scenes with N log-uniform in [1e5, 2e6] (seeds 7..14), 8
    cameras each.  ``scale`` shrinks every scene for tests."""
    rng = _rng(seed)
    scenes = [mixture_scene(max(1, int(1_000_000 * scale)), seed=1)]
    views = batch_views(views_a, rng, 0)
    for k in range(n_b):
        n = int(math.exp(rng.uniform(math.log(1e5), math.log(2e6))) * scale)
        scenes.append(mixture_scene(max(1, n), seed=7 + k))
        views += batch_views(views_b, rng, k + 1)
    return scenes, views
