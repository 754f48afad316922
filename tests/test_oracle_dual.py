"""Pins of the low-resolution companion atlas (App. "Depth-of-Field" and
"Foveated Rendering": one packing, its coordinates scaled by 2^-k per axis
into an atlas of side omega / 2^k).

The low map is checked texel by texel against an exact float64
point-in-triangle test of the UVs scaled by 2^-k (away from edges, where the
1/256 snapping may decide either way), and every owned texel against the
scaled box membership in exact integers.
"""
import numpy as np
import pytest

import oracle
from synth import scenes


def _edge_dist(X, Y, ax, ay, bx, by):
    dx, dy = bx - ax, by - ay
    n = np.hypot(dx, dy)
    if n == 0:
        return np.full_like(X, np.inf)
    return np.abs(dx * (Y - ay) - dy * (X - ax)) / n


@pytest.mark.parametrize("seed,omega,k,g", [(2, 1024, 1, 2), (7, 2048, 3, 8), (13, 1024, 2, 1)])
def test_low_map_vs_exact(seed, omega, k, g):
    f = scenes.grid_frame(seed, atlas_size=omega)
    r = oracle.build_frame(f, gutter=g, low_shift=k)
    ol = omega >> k
    occ = r["occupancy_low"]
    assert occ.shape == (ol, ol)
    uv = r["uv"].astype(np.float64) / (1 << k)
    L = r["L"]
    want = np.full((ol, ol), -1, np.int64)
    ambiguous = np.zeros((ol, ol), bool)
    tx = np.arange(ol)
    for t in np.nonzero(r["nonempty"])[0]:
        c = r["chart_of_tri"][t]
        P = uv[f.indices[t]]
        x0, x1 = int(np.floor(P[:, 0].min() - 1)), int(np.ceil(P[:, 0].max() + 1))
        y0, y1 = int(np.floor(P[:, 1].min() - 1)), int(np.ceil(P[:, 1].max() + 1))
        xs = tx[max(0, x0):max(0, min(ol, x1))]
        ys = tx[max(0, y0):max(0, min(ol, y1))]
        if xs.size == 0 or ys.size == 0:
            continue
        X, Y = np.meshgrid(xs + 0.5, ys + 0.5)
        e = [(P[(q + 1) % 3, 0] - P[q, 0]) * (Y - P[q, 1]) - (P[(q + 1) % 3, 1] - P[q, 1]) * (X - P[q, 0])
             for q in range(3)]
        inside = ((e[0] >= 0) & (e[1] >= 0) & (e[2] >= 0)) | ((e[0] <= 0) & (e[1] <= 0) & (e[2] <= 0))
        d = np.minimum.reduce([_edge_dist(X, Y, P[q, 0], P[q, 1], P[(q + 1) % 3, 0], P[(q + 1) % 3, 1])
                               for q in range(3)])
        bx, by, ba, bb = r["x"][c], r["y"][c], r["a"][c], r["b"][c]
        inbox = ((2 * bx * ol <= (2 * X) * L) & ((2 * X) * L < 2 * (bx + ba) * ol) &
                 (2 * by * ol <= (2 * Y) * L) & ((2 * Y) * L < 2 * (by + bb) * ol))
        sub_w = want[ys[0]:ys[-1] + 1, xs[0]:xs[-1] + 1]
        sub_a = ambiguous[ys[0]:ys[-1] + 1, xs[0]:xs[-1] + 1]
        sub_w[inside & inbox] = c
        sub_a |= d < 4.0 / 256
    agree = (occ == want) | ambiguous
    assert agree.all(), int((~agree).sum())
    assert (occ >= 0).sum() > 100
    assert r["occupied_low"] == int((occ >= 0).sum())


def test_low_map_owner_inside_scaled_box():
    f = scenes.orbit_frame(33, atlas_size=2048)
    k = 2
    r = oracle.build_frame(f, gutter=4, low_shift=k)
    occ = r["occupancy_low"]
    ol, L = 2048 >> k, r["L"]
    ty, tx = np.nonzero(occ >= 0)
    c = occ[ty, tx]
    x, y = r["x"][c].astype(np.int64), r["y"][c].astype(np.int64)
    a, b = r["a"][c].astype(np.int64), r["b"][c].astype(np.int64)
    assert (2 * x * ol <= (2 * tx + 1) * L).all() and ((2 * tx + 1) * L < 2 * (x + a) * ol).all()
    assert (2 * y * ol <= (2 * ty + 1) * L).all() and ((2 * ty + 1) * L < 2 * (y + b) * ol).all()
    # the high-resolution outputs do not depend on the low map
    r0 = oracle.build_frame(f, gutter=4)
    assert np.array_equal(r0["occupancy"], r["occupancy"])
