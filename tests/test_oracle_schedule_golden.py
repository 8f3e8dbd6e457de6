"""Hand-derived goldens of the hierarchical resorting schedule.

The queue schedule of Sec. 3.4 (Fig. pipeline: a 4x4 tail queue of 64 fed in
batches of 32 and popped 16 at a time, 2x2 mid queues of 8 fed in runs of 4
and popped 4 at a time, a per-pixel head of K) and the k-buffer rule of
Sec. 3.3 (insert, and blend the nearest sample when the buffer overflows)
fix which Gaussian every pixel blends when.  Nothing in the paper prints such
a sequence, so the expected sequences below are derived by hand, step by
step in the comments, from micro-scenes whose depth orders are known in
closed form.  The oracle only has to reproduce them.

Closed form used for every order.  All Gaussians are isotropic (equal scales,
identity rotation), so Eq. dopt gives t_opt = d . (mu - o) for a unit ray d
(Sec. 3.2).  The camera sits at the origin looking along +z (R = I), with
fx = fy = 8 and principal point (7.5, 7.5) on a 16x16 image: the ray through
image point (u, v) is d = (a(u), a(v), 1) / |(a(u), a(v), 1)| with
a(u) = (u - 7.5) / 8.  Every Gaussian seen along that ray shares the factor
1 / |d|, so the order along it is the order of

    e(m; u, v) = m_z + a(u) m_x + a(v) m_y,      m = mu - o.

The levels use these rays (the reading of Sec. 3.4 also taken by the oracle):
the 4x4 tail keys along the sub-tile centre ray, the 2x2 mid keys along the
quad centre ray, the head along the pixel ray, and the tile list along the
ray through the Gaussian's maximum point in the tile (its 2D mean, when that
lies inside the tile: then t = |m|).

"Axis" Gaussians A_k sit on the optical axis at depth z_k = 4 + 0.01 k: their
e is z_k along every ray, so every level sees them in index order.  Each
scene adds one or two special Gaussians whose e differs from level to level.
Every designed e is at least 0.005 away from the nearest z_k, far beyond
float32 rounding.  Most scenes look at sub-tile (8..11, 8..11) of the image: its
centre ray is at (9.5, 9.5), a(9.5) = 0.25; quad (8..9, 8..9) has its centre
at (8.5, 8.5), a = 0.125; quad (10..11, 10..11) at (10.5, 10.5), a = 0.375;
pixel (8, 8) has a = 0.0625 and pixel (10, 10) a = 0.3125.
"""
import numpy as np
import pytest

import oracle
from micro_scenes import cam16, e_of, scene_of

Z0, DZ = 4.0, 0.01


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def z(k):
    return Z0 + DZ * k


def axis(k):
    # large and faint: seen by every pixel of the tile with alpha in
    # [0.02, 0.1], so no pixel terminates within 40 blends (0.9^40 > 1e-4)
    return ([0.0, 0.0, z(k)], 3.0, 0.1)


def blends_at(fr, u, v):
    ids = fr.blend_ids[v, u]
    return [int(i) for i in ids[ids >= 0]]


def test_late_entry_reaches_the_head_through_the_mid_window():
    """Scene X, default queues (64/8/4).  A_0..A_38 (ids 0..38) and X (id 39)
    at m = (1.6, 1.6, 2.885).  Pixel (10, 10) in quad (10..11, 10..11).

    e of X: sub-tile 2.885 + 0.5*1.6 = 3.685 (before every A), quad
    2.885 + 0.75*1.6 = 4.085 (between A_8 = 4.08 and A_9 = 4.09), pixel
    2.885 + 0.625*1.6 = 3.885 (before every A).  List: |m_X| = 3.67 < 4, so X
    is entry 0 and the A's follow in index order.

    Tail of the sub-tile: batch 0 (X, A_0..A_30) -> [X, A_0..A_30]; batch 1
    (A_31..A_38) -> 40 > 32, pop 16 = [X, A_0..A_14]; the end of the list
    drains [A_15..A_30] and [A_31..A_38].
    Mid of the quad, first chunk in runs of 4:
      [X, A0, A1, A2] -> [A0, A1, A2, X]                 (4, no pop)
      [A3..A6]  -> [A0..A6, X] (8)      -> pop A0..A3, keep [A4, A5, A6, X]
      [A7..A10] -> [A4..A8, X, A9, A10] -> pop A4..A7, keep [A8, X, A9, A10]
      [A11..A14] -> [A8, X, A9..A14]    -> pop A8, X, A9, A10
    Later chunks hold A's only and leave in index order.  Arrivals at the
    pixel's head: A0..A8, X, A9..A38.
    Head (K = 4): A0..A3 fill it; A4..A8 each blend the front (A0..A4),
    leaving [A5..A8]; X arrives, is the nearest of the five and is blended;
    then each arrival blends the front, and the end drains the rest.
    Blend order: A0..A4, X, A5..A38.

    Mutations this pins: keying the mid level along the sub-tile ray (X
    leaves the mid first: X, A0, ...); evicting the front before inserting
    (A0..A5, X, ...); keying the head along the quad ray (A0..A8, X, ...).
    """
    X = 39
    mX = (1.6, 1.6, 2.885)
    assert e_of(mX, 9.5, 9.5) < z(0) - 0.3
    assert z(8) + 0.004 < e_of(mX, 10.5, 10.5) < z(9) - 0.004
    assert e_of(mX, 10, 10) < z(0) - 0.1
    assert np.linalg.norm(mX) < z(0) - 0.3
    sc = scene_of([axis(k) for k in range(39)] + [(list(mX), 0.5, 0.5)])
    fr = oracle.frame(sc, cam16(), mode=oracle.MODE_HIER, head=4, max_k=48)
    expect = [0, 1, 2, 3, 4, X] + list(range(5, 39))
    assert blends_at(fr, 10, 10) == expect


def test_entry_held_in_the_tail_reaches_the_head_late():
    """Scene Y, default queues (64/8/4).  A_0..A_38 (ids 0..38) and Y (id 39)
    at m = (1.6, 1.6, 3.405).  Pixel (8, 8) in quad (8..9, 8..9).

    e of Y: sub-tile 3.405 + 0.5*1.6 = 4.205 (between A_20 and A_21), quad
    3.405 + 0.25*1.6 = 3.805 (before every A), pixel 3.405 + 0.125*1.6 =
    3.605 (before every A).  List: |m_Y| = 4.088, so Y is entry 9 (after
    A_0..A_8); it is in batch 0 either way.

    Tail: batch 0 -> [A0..A20, Y, A21..A30]; batch 1 (A31..A38) -> 40 > 32,
    pop 16 = [A0..A15]; the end drains [A16..A20, Y, A21..A30], then
    [A31..A38].
    Mid of the quad: the first chunk leaves in order (pops A0..A3, A4..A7,
    A8..A11, keeps [A12..A15]).  Second chunk:
      [A16..A19]         -> pop A12..A15, keep [A16..A19]
      [A20, Y, A21, A22] -> [Y, A16..A22] (8) -> pop Y, A16, A17, A18
    and A's in order after that.  Arrivals: A0..A15, Y, A16..A38.
    Head (K = 4): A0..A3 fill it; A4..A15 blend A0..A11, leaving [A12..A15];
    Y is the nearest and is blended at once; then A12..A38 in order.
    Blend order: A0..A11, Y, A12..A38.

    Mutation this pins: keying the tail along the quad or the pixel ray (Y
    would be in the first pop and blended first).
    """
    Y = 39
    mY = (1.6, 1.6, 3.405)
    assert z(20) + 0.004 < e_of(mY, 9.5, 9.5) < z(21) - 0.004
    assert e_of(mY, 8.5, 8.5) < z(0) - 0.1
    assert e_of(mY, 8, 8) < z(0) - 0.3
    assert z(8) < np.linalg.norm(mY) < z(9)
    sc = scene_of([axis(k) for k in range(39)] + [(list(mY), 1.0, 0.5)])
    fr = oracle.frame(sc, cam16(), mode=oracle.MODE_HIER, head=4, max_k=48)
    expect = list(range(0, 12)) + [Y] + list(range(12, 39))
    assert blends_at(fr, 8, 8) == expect


def test_head_inserts_before_it_evicts():
    """Scene Z, head K = 2 (tail and mid queues at their defaults).  A_0, A_1
    (ids 0, 1) and Z (id 2) at m = (0.8, 0.8, 3.815).  Pixel (8, 8).

    e of Z: sub-tile 3.815 + 0.4 = 4.215, quad 3.815 + 0.2 = 4.015 (between
    A_1 = 4.01 and A_2), pixel 3.815 + 0.1 = 3.915 (before A_0).
    Three entries: the tail never pops during the list; the end drains all
    three to the mid, which sorts them by the quad ray as [A0, A1, Z] and,
    holding no more than 4, drains them to the head in that order.
    Head (K = 2), the k-buffer rule (insert, then blend the nearest when more
    than K are held): A0, A1 fill it; Z is inserted in front, three are held,
    Z is blended; the end blends A0, A1.  Blend order: Z, A0, A1.
    Evicting the front before inserting would blend A0, then Z, A1.
    """
    mZ = (0.8, 0.8, 3.815)
    assert z(1) + 0.004 < e_of(mZ, 8.5, 8.5) < z(2) - 0.004
    assert e_of(mZ, 8, 8) < z(0) - 0.08
    sc = scene_of([axis(0), axis(1), (list(mZ), 0.5, 0.5)])
    fr = oracle.frame(sc, cam16(), mode=oracle.MODE_HIER, head=2, max_k=8)
    assert blends_at(fr, 8, 8) == [2, 0, 1]
    # With room for all three the head blends the pixel-ray order.
    fr4 = oracle.frame(sc, cam16(), mode=oracle.MODE_HIER, head=4, max_k=8)
    assert blends_at(fr4, 8, 8) == [2, 0, 1]


def test_quad_culling_frees_a_mid_slot():
    """Scene C/W, default queues (64/8/4).  A_0..A_13 (ids 0..13), C (id 14)
    and W (id 15).  Pixel (8, 8) in quad (8..9, 8..9).

    C: m = (0.875, 0.875, 2), tiny (scale 0.01), opacity 0.9: its 2D mean is
    (11, 11), the corner of the sub-tile's pixel-centre hull, so the sub-tile
    keeps it (alpha 0.9 there), while the quad's hull [8, 9]^2 is 2*sqrt(2)
    pixels away, where the dilated footprint (variance about 0.3 px^2) gives
    exp(-13) * 0.9 < 1/255: the quad culls it.  e of C: sub-tile 2.44,
    quad 2.22 (before every other Gaussian).
    W: m = (0.8, 0.8, 3.705): e sub-tile 4.105 (between A_10 and A_11), quad
    3.905 and pixel 3.805 (before every A).
    Sixteen entries at the sub-tile: the end of the list drains one chunk of
    16 in sub-tile order: [C, A0, A1, A2 | A3..A6 | A7..A10 | W, A11..A13].
    Mid of the quad, C culled:
      [C, A0, A1, A2] -> [A0, A1, A2]       (3)
      [A3..A6]        -> 7, pop A0..A3,   keep [A4, A5, A6]
      [A7..A10]       -> 7, pop A4..A7,   keep [A8, A9, A10]
      [W, A11..A13]   -> [W, A8..A13] (7), pop W, A8, A9, A10
    then A11..A13.  Arrivals: A0..A7, W, A8..A13.
    Head (K = 4): A4..A7 blend A0..A3, leaving [A4..A7]; W is blended at
    once; then A4..A13.  Blend order: A0..A3, W, A4..A13.
    Culling the quad against the sub-tile's hull instead would keep C in the
    mid queue: [C, A0, A1, A2] fills it, the second run pops C, A0, A1, A2,
    and W then arrives after A0..A6: blend order A0..A2, W, A3..A13.
    """
    W_, C_ = 15, 14
    mC, mW = (0.875, 0.875, 2.0), (0.8, 0.8, 3.705)
    assert abs(8 * mC[0] / mC[2] + 7.5 - 11.0) < 1e-6
    assert e_of(mC, 9.5, 9.5) < z(0) - 1 and e_of(mC, 8.5, 8.5) < z(0) - 1
    assert z(10) + 0.004 < e_of(mW, 9.5, 9.5) < z(11) - 0.004
    assert e_of(mW, 8.5, 8.5) < z(0) - 0.09 and e_of(mW, 8, 8) < z(0) - 0.19
    sc = scene_of([axis(k) for k in range(14)] + [(list(mC), 0.01, 0.9), (list(mW), 0.5, 0.5)])
    fr = oracle.frame(sc, cam16(), mode=oracle.MODE_HIER, head=4, max_k=32)
    assert blends_at(fr, 8, 8) == [0, 1, 2, 3, W_] + list(range(4, 14))
    # C is blended where its own quad sees it, and nowhere in quad (8..9, 8..9)
    assert C_ in blends_at(fr, 11, 11)
    assert all(C_ not in blends_at(fr, u, v) for u in (8, 9) for v in (8, 9))


def test_tail_pops_only_above_its_threshold():
    """Scene V, default queues (64/8/4).  A_0..A_38 (ids 0..38) and V (id 39)
    at m = (1, 1, 4.2), large (scale 3).  Sub-tile (0..3, 0..3), centre ray
    a = -0.75; pixel (1, 1) in quad (0..1, 0..1).

    e of V: sub-tile 4.2 - 1.5 = 2.7, quad (a = -0.875) 2.45, pixel
    (a = -0.8125) 2.575: nearest of all at every level of this sub-tile.
    List: |m_V| = 4.43 > z_38 = 4.38, so V is the last entry (batch 1).
    Tail: batch 0 (A0..A31) -> 32 entries, not more than 64 - 32: no pop.
    Batch 1 (A32..A38, V) -> [V, A0..A38] (40) -> pop 16 = [V, A0..A14].
    Mid: [V, A0, A1, A2] fills it; the next run pops V, A0, A1, A2; the head
    holds them, and the next arrival (A3) blends V.  Everything after
    leaves every level in index order.  Blend order: V, A0..A38.
    Popping already at 32 would send A0..A15 from batch 0 and V only at the
    end of the list: V would be blended after A0..A7.
    """
    V = 39
    mV = (1.0, 1.0, 4.2)
    assert e_of(mV, 1.5, 1.5) < z(0) - 1 and e_of(mV, 0.5, 0.5) < z(0) - 1 and e_of(mV, 1, 1) < z(0) - 1
    assert np.linalg.norm(mV) > z(38) + 0.04
    sc = scene_of([axis(k) for k in range(39)] + [(list(mV), 3.0, 0.5)])
    fr = oracle.frame(sc, cam16(), mode=oracle.MODE_HIER, head=4, max_k=48)
    assert blends_at(fr, 1, 1) == [V] + list(range(39))


def test_tail_pops_after_every_batch_that_overfills_it():
    """Scene U, default queues (64/8/4).  A_0..A_71 (ids 0..71) and U (id 72)
    at m = (1, 1, 4.6), large (scale 3).  Sub-tile (0..3, 0..3); pixel (1, 1)
    in quad (0..1, 0..1).

    e of U: sub-tile 4.6 - 1.5 = 3.1, quad 4.6 - 1.75 = 2.85, pixel
    4.6 - 1.625 = 2.975: nearest of all at every level.  List: |m_U| = 4.81 >
    z_71 = 4.71, so U is the last entry (batch 2).
    Tail: batch 0 (A0..A31) -> 32, no pop.  Batch 1 (A32..A63) -> 64: pop
    [A0..A15], pop [A16..A31], 32 left.  Batch 2 (A64..A71, U) -> 41: pop
    [U, A32..A46], 25 left; the end drains [A47..A62] and [A63..A71].
    Mid: the first two chunks leave every run in index order; after them
    A0..A27 have gone to the head and [A28..A31] wait.  The run [U, A32, A33,
    A34] makes [U, A28..A34]: pop U, A28, A29, A30.  Head arrivals: A0..A27,
    U, A28..A71.  Head (K = 4): when U arrives it holds [A24..A27] (A0..A23
    blended); U is inserted at the front and blended at once.
    Blend order: A0..A23, U, A24..A71.
    A tail that never popped during the list would drain U first (U, A0..);
    one that popped already at 32 would send A0..A47 before U.
    """
    U = 72
    mU = (1.0, 1.0, 4.6)
    assert e_of(mU, 1.5, 1.5) < z(0) - 0.5 and e_of(mU, 0.5, 0.5) < z(0) - 0.5 and e_of(mU, 1, 1) < z(0) - 0.5
    assert np.linalg.norm(mU) > z(71) + 0.04
    sc = scene_of([axis(k) for k in range(72)] + [(list(mU), 3.0, 0.5)])
    fr = oracle.frame(sc, cam16(), mode=oracle.MODE_HIER, head=4, max_k=80)
    assert blends_at(fr, 1, 1) == list(range(24)) + [U] + list(range(24, 72))
