"""CPU premises of the GPU parity cases built around the per-tile sorted
prefix (the GPU side is in test_gpu_parity.py): the constructed scene must
really exercise what the GPU case is meant to catch."""
import copy

import numpy as np
import pytest

import oracle
from micro_scenes import PREFIX_M, PREFIX_X, blend_seq, cam16, prefix_partial_batch_scene


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def test_prefix_partial_batch_scene_premise():
    sc, _ = prefix_partial_batch_scene()
    cam = cam16()
    full = oracle.frame(sc, cam, mode=oracle.MODE_HIER, max_k=16)
    E = len(full.keys)
    assert E == 64 and PREFIX_M < E and PREFIX_M % 32 != 0
    assert int(full.values[PREFIX_X]) == PREFIX_X
    # Depths 0.05 apart or more: a histogram of 128 bins per octave (bin width
    # at most 4/128 in [4, 8)) separates every entry, so a prefix of M entries
    # is exactly the first M of the sorted list.
    depth = np.sort(full.keys & np.uint64(0xffffffff)).astype(np.uint32)
    t = np.where(depth >= 2 ** 31, depth & 0x7fffffff, ~depth).astype(np.uint32).view(np.float32)
    assert t.min() >= 4.0 and t.max() < 8.0 and np.diff(np.sort(t)).min() > 4.0 / 128
    # The first M entries alone (the rest made invisible; ids, ranks and keys
    # unchanged): every pixel terminates within the blends the tail's first
    # pop after the partial batch 1 feeds (at most 8 per pixel), ...
    red_sc = copy.deepcopy(sc)
    keep = np.zeros(sc.n, bool)
    keep[full.values[:PREFIX_M]] = True
    red_sc.opacities = np.where(keep, sc.opacities, 0).astype(np.float32)
    red = oracle.frame(red_sc, cam, mode=oracle.MODE_HIER, max_k=16)
    assert red.count.max() <= 7 and red.count.min() >= 1
    # ... and the blend orders differ from those of the whole list: X reaches
    # the top-left pixels first only when its batch is complete.
    assert blend_seq(full.blend_ids, 0, 0)[0] == PREFIX_X
    assert PREFIX_X not in blend_seq(red.blend_ids, 0, 0)
    assert np.any(red.blend_ids != full.blend_ids)
