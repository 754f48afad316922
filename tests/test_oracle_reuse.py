"""Pins of the temporal-reuse classification (Sec. "Temporal Reuse": a later
frame re-shades only newly visible triangles and triangles that were partially
visible, some vertex with max(|x|, |y|) >= w, in the key frame).

Checked against an independent numpy evaluation of the definition on orbit
frames, and on hand-built cases at the exact boundary.
"""
import numpy as np

import oracle
from synth import scenes


def _numpy_flags(pos, tri, M, key_vis, vis):
    M = np.asarray(M, np.float32).reshape(4, 4)
    p = np.asarray(pos, np.float32)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    clip = [((M[i, 0] * x + M[i, 1] * y) + M[i, 2] * z) + M[i, 3] for i in range(4)]
    part_v = np.maximum(np.abs(clip[0]), np.abs(clip[1])) >= clip[3]
    partial = part_v[tri].any(1)
    reuse = (key_vis == 1) & ~partial
    return np.where(vis == 1, np.where(reuse, 1, 2), 0).astype(np.uint8)


def test_matches_numpy_on_orbit():
    key = scenes.orbit_frame(10)
    for k in (11, 14, 19):
        f = scenes.orbit_frame(k)
        flags, n = oracle.reuse_flags(f.positions, f.indices, key.view_proj, key.visible,
                                      f.visible)
        ref = _numpy_flags(f.positions, f.indices, key.view_proj, key.visible, f.visible)
        assert np.array_equal(flags, ref)
        assert n == int((ref == 1).sum())
        # a nearby frame reuses most of what it sees, and shades something
        seen = int((ref > 0).sum())
        assert 0 < n < seen


def test_same_frame_reuses_everything_fully_on_screen():
    f = scenes.grid_frame(4)
    flags, n = oracle.reuse_flags(f.positions, f.indices, f.view_proj, f.visible, f.visible)
    assert ((flags == 0) == (f.visible == 0)).all()
    ref = _numpy_flags(f.positions, f.indices, f.view_proj, f.visible, f.visible)
    assert np.array_equal(flags, ref)


def test_boundary_cases():
    # identity view_proj: clip = (x, y, z, 1); w = 1
    M = np.eye(4, dtype=np.float32).ravel()
    pos = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 0.5, 0.0],    # inside
                    [1.0, 0.0, 0.0],                                        # |x| == w
                    [0.0, -1.5, 0.0]], np.float32)                          # outside
    tri = np.array([[0, 1, 2],    # fully inside, key visible -> reuse
                    [0, 1, 3],    # vertex on the boundary -> partial -> shade
                    [0, 2, 4],    # vertex outside -> shade
                    [0, 1, 2],    # inside but newly visible -> shade
                    [0, 1, 2]],   # not visible now -> 0
                   np.int32)
    key_vis = np.array([1, 1, 1, 0, 1], np.uint8)
    vis = np.array([1, 1, 1, 1, 0], np.uint8)
    flags, n = oracle.reuse_flags(pos, tri, M, key_vis, vis)
    assert flags.tolist() == [1, 2, 2, 2, 0]
    assert n == 1
