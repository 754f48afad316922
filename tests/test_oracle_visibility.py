"""Pins of the visibility oracle (App. "Detecting Visible Triangles": depth
pre-pass, then a "less or equal" test of every triangle's samples).

The oracle is checked against (1) the scene generator's own visible sets,
computed by an independent vectorized float64 implementation of the same
reading, and (2) hand-built scenes whose answer is known by construction:
facing, frustum, occlusion, the conservative rule for triangles that cover no
sample, and near-plane crossing.
"""
import numpy as np
import pytest

import oracle
from synth import scenes


def _vis(f, coarse=None):
    return oracle.visibility(f.positions, f.indices, f.view_proj, f.eye, f.near, f.width,
                             f.height, f.coarse if coarse is None else coarse)


@pytest.mark.parametrize("seed", [0, 5, 11])
def test_matches_generator_grid(seed):
    f = scenes.grid_frame(seed)
    assert np.array_equal(_vis(f), f.visible)


@pytest.mark.parametrize("frame", [0, 40, 85])
def test_matches_generator_orbit(frame):
    f = scenes.orbit_frame(frame)
    assert np.array_equal(_vis(f), f.visible)


def test_matches_generator_city_coarse():
    f = scenes.city_frame(9)
    v = _vis(f)
    assert f.coarse == 8
    assert np.array_equal(v, f.visible)
    # the depth test only removes candidates, and it removes some
    cand = _vis(f, coarse=0)
    assert (v <= cand).all() and cand.sum() > v.sum() + 1000


# ---------------------------------------------------------------------------
# hand-built scenes: camera at the origin looking down -z, 64x64 viewport
# ---------------------------------------------------------------------------
def _camera(W=64, H=64, near=0.1):
    return scenes.make_camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), W, H, near, 100.0, up=(0, 1, 0))


def _quad(z, half, cx=0.0, cy=0.0):
    """Two triangles facing +z (towards the camera at the origin)."""
    p = np.array([[cx - half, cy - half, z], [cx + half, cy - half, z],
                  [cx + half, cy + half, z], [cx - half, cy + half, z]], np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return p, t


def _scene(*parts):
    pos, tri, off = [], [], 0
    for p, t in parts:
        pos.append(p)
        tri.append(t + off)
        off += p.shape[0]
    return np.concatenate(pos), np.concatenate(tri)


def _run(pos, tri, cam, coarse):
    return oracle.visibility(pos, tri, cam.view_proj, cam.eye, cam.near, cam.width, cam.height,
                             coarse)


def test_facing_and_frustum():
    cam = _camera()
    front = _quad(-2.0, 0.5)
    back = (front[0], front[1][:, ::-1].copy())          # same place, wound away
    behind = _quad(+2.0, 0.5)                             # behind the camera
    aside = _quad(-2.0, 0.2, cx=50.0)                     # far outside the right plane
    pos, tri = _scene(front, back, behind, aside)
    v = _run(pos, tri, cam, 0)
    assert v.tolist() == [1, 1, 0, 0, 0, 0, 0, 0]


@pytest.mark.parametrize("coarse", [1, 2])
def test_occluded_quad_is_culled(coarse):
    cam = _camera()
    near_q = _quad(-2.0, 1.0)      # covers the middle of the view
    far_q = _quad(-5.0, 1.0)       # smaller on screen, entirely behind near_q
    pos, tri = _scene(near_q, far_q)
    assert _run(pos, tri, cam, 0).tolist() == [1, 1, 1, 1]
    assert _run(pos, tri, cam, coarse).tolist() == [1, 1, 0, 0]


def test_partly_hidden_quad_stays():
    cam = _camera()
    pos, tri = _scene(_quad(-2.0, 0.3), _quad(-5.0, 3.0))
    assert _run(pos, tri, cam, 1).tolist() == [1, 1, 1, 1]


def test_sub_sample_triangle_is_kept():
    # covers no sample centre of the coarse buffer: cannot be proven hidden
    cam = _camera()
    occ = _quad(-2.0, 1.0)
    tiny = (np.array([[0.001, 0.001, -5.0], [0.004, 0.001, -5.0], [0.001, 0.004, -5.0]],
                     np.float32), np.array([[0, 1, 2]], np.int32))
    pos, tri = _scene(occ, tiny)
    assert _run(pos, tri, cam, 8).tolist() == [1, 1, 1]


def test_near_crossing_triangle_is_kept():
    # front-facing, inside the side planes, one vertex in front of the near
    # plane: it never writes or fails the depth test
    cam = _camera(near=0.1)
    occ = _quad(-2.0, 1.0)
    cross = (np.array([[-0.02, -0.02, -0.05], [0.3, -0.3, -6.0], [0.3, 0.3, -6.0]], np.float32),
             np.array([[0, 1, 2]], np.int32))
    pos, tri = _scene(occ, cross)
    v = _run(pos, tri, cam, 1)
    assert v.tolist() == [1, 1, 1]


def test_equal_depth_passes():
    # the same quad twice: "less or equal" keeps both copies
    cam = _camera()
    pos, tri = _scene(_quad(-3.0, 1.0), _quad(-3.0, 1.0))
    assert _run(pos, tri, cam, 1).tolist() == [1, 1, 1, 1]
