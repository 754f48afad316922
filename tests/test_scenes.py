"""Seeded input generator: determinism, sizes and the visible-set rules."""
import numpy as np

from synth import scenes


def test_grid_frame_deterministic_and_sized():
    a, b = scenes.grid_frame(7), scenes.grid_frame(7)
    assert a.digest() == b.digest()
    assert a.num_triangles == 8192 and a.num_vertices == 4225
    assert scenes.grid_frame(8).digest() != a.digest()
    assert 0 < int(a.visible.sum()) < a.num_triangles


def test_orbit_frame_sizes():
    f = scenes.orbit_frame(0)
    assert f.num_triangles == 20480 + 100 * 300 + 100 * 360
    assert f.indices.min() >= 0 and f.indices.max() < f.num_vertices


def test_visible_set_rules():
    f = scenes.orbit_frame(3)
    p = f.positions.astype(np.float64)
    i = f.indices
    M = f.view_proj.astype(np.float64).reshape(4, 4)
    c = p @ M[:, :3].T + M[:, 3]
    vis = f.visible.astype(bool)
    # no visible triangle lies entirely outside one clip plane
    for d in (c[:, 3] + c[:, 0], c[:, 3] - c[:, 0], c[:, 3] + c[:, 1], c[:, 3] - c[:, 1],
              c[:, 3] + c[:, 2], c[:, 3] - c[:, 2]):
        assert not (d[i[vis]] < 0).all(1).any()


def test_meshes_are_welded_and_closed():
    for pos, tris in (scenes.box_mesh(5), scenes.cylinder_mesh(36, 4), scenes.icosphere(2)):
        # closed 2-manifold: every undirected edge is shared by exactly two triangles
        e = np.sort(np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]), 1)
        _, cnt = np.unique(e, axis=0, return_counts=True)
        assert (cnt == 2).all()
        # outward orientation: signed volume positive
        p = pos[tris]
        vol = np.einsum("ij,ij->i", p[:, 0], np.cross(p[:, 1], p[:, 2])).sum() / 6
        assert vol > 0


def test_scatter_frame_is_many_charts():
    f = scenes.scatter_frame(0)
    assert f.num_triangles == 24000 * 12 and f.num_vertices == 24000 * 8
    assert scenes.scatter_frame(0).digest() == f.digest()
    # every box is a closed 12-triangle object: the visible faces of one box
    # share vertices, so the visible boxes are the charts
    vis = f.visible.reshape(-1, 12).any(1)
    assert int(vis.sum()) >= 20000
