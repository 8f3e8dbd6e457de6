"""Hand-placed micro-scenes of isotropic Gaussians seen by a 16x16 camera.

Inputs only: the camera sits at the origin looking along +z (R = I) with
fx = fy = 8 and principal point (7.5, 7.5), so the ray through image point
(u, v) is along (a(u), a(v), 1) with a(u) = (u - 7.5) / 8.  For isotropic
Gaussians t_opt = d . (mu - o) along a unit ray d (Sec. 3.2), so along the ray
through (u, v) the depth order of Gaussians is the order of
e(m; u, v) = m_z + a(u) m_x + a(v) m_y with m = mu - o.
"""
import numpy as np

from paper_2402_00525_amd import synth


def cam16():
    return synth.Camera(R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32), center=np.zeros(3, np.float32),
                        fx=8.0, fy=8.0, cx=7.5, cy=7.5, W=16, H=16)


def a_of(u):
    return (u - 7.5) / 8.0


def e_of(m, u, v):
    return m[2] + a_of(u) * m[0] + a_of(v) * m[1]


def scene_of(gauss):
    """gauss: list of (mean, scale, opacity); isotropic, SH degree 0, grey."""
    n = len(gauss)
    means = np.array([g[0] for g in gauss], np.float32)
    scales = np.array([[g[1]] * 3 for g in gauss], np.float32)
    rots = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1))
    opac = np.array([g[2] for g in gauss], np.float32)
    sh = np.zeros((n, 1, 3), np.float32)
    return synth.Scene(means, scales, rots, opac, sh, 0)


def blend_seq(blend_ids, u, v):
    ids = blend_ids[v, u]
    return [int(i) for i in ids[ids >= 0]]


# ---------------------------------------------------------------------------
# A truncated per-tile prefix whose last batch is partial.
# ---------------------------------------------------------------------------
PREFIX_M = 40          # sorted prefix length that cuts the tile's list at 40
PREFIX_X = 40          # list position (and id) of the late, near-to-one-corner Gaussian


def prefix_partial_batch_scene():
    """One tile, 64 entries.  B_0..B_62 sit on the optical axis at depths
    4 + 0.05 k (k < 40) and 4.05 + 0.05 k (k >= 40): large (scale 8) and
    nearly opaque (0.99), so every pixel has alpha >= 0.79 for each of them
    and terminates after at most 6 blends.  X (|m| = 6.0, between B_39 = 5.95
    and B_40 = 6.05, so list position 40) is off axis towards +x +y: along the
    rays of the top-left sub-tile (a <= -0.56) its e = 5.29 + 4 a is at most
    3.05, nearer than every B.  Depths 0.05 apart fall into different bins of
    any histogram of 128 bins per octave (bin width <= 4/128 in [4, 8)), so a
    prefix of 40 entries ends exactly before X.

    Rendered from the first 40 entries only, batch 1 is partial (8 entries)
    and the tail's first pop after it terminates every pixel; the full list
    brings X in batch 1, and the first pop of the top-left sub-tile carries X
    to its pixels first: their blend orders differ."""
    gs = []
    for k in range(63):
        zk = 4.0 + 0.05 * k + (0.05 if k >= 40 else 0.0)
        gs.append(([0.0, 0.0, zk], 8.0, 0.99))
    M = 2.0
    mz = float(np.sqrt(36.0 - 2 * M * M))
    gs.insert(PREFIX_X, ([M, M, mz], 4.0, 0.99))
    ids = np.arange(64)
    # ids: B_k keeps id k for k < 40, X has id 40, B_k has id k + 1 for k >= 40
    return scene_of(gs), ids
