"""Pins for the oracle's UV map and occupancy (CPU only).

* UV (Appendix "Shading and Rasterization": uniform scale S then a rigid map
  per chart): for every visible triangle the screen-pixel -> atlas-texel map is
  a similarity with factor rate * S_eff and positive orientation, so texture
  stretch L2 = Linf = 1 / (rate * S_eff); at S_eff = 1 this reproduces the
  paper's Table of stretch at fixed scale factors (tests/golden).
* occupancy: every claimed texel lies in its chart's placed box, each texel
  has at most one owner, and away from triangle edges the claim agrees with an
  exact float64 point-in-triangle test of the texel centre against the
  unsnapped UV triangles.
"""
import json
import os

import numpy as np
import pytest

import oracle
from synth import scenes

STRETCH = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "stretch_fixed_rate.json")))


def _pixel_coords(clip, W, H):
    c = clip.astype(np.float64)
    nx, ny = c[:, 0] / c[:, 3], c[:, 1] / c[:, 3]
    return np.stack([(nx + 1) * 0.5 * W, (1 - ny) * 0.5 * H], 1)


def _jacobians(frame_, r):
    clip = r["clip"]
    P = _pixel_coords(clip, frame_.width, frame_.height)
    uv = r["uv"].astype(np.float64)
    idx = frame_.indices
    vis = frame_.visible.astype(bool) & (clip[idx, 3] > 0).all(1)
    t = np.nonzero(vis)[0]
    p0, p1, p2 = P[idx[t, 0]], P[idx[t, 1]], P[idx[t, 2]]
    u0, u1, u2 = uv[idx[t, 0]], uv[idx[t, 1]], uv[idx[t, 2]]
    A = np.stack([p1 - p0, p2 - p0], 2)  # columns
    B = np.stack([u1 - u0, u2 - u0], 2)
    area = np.abs(np.linalg.det(A)) / 2
    keep = area > 30.0  # well-conditioned triangles only
    Jm = B[keep] @ np.linalg.inv(A[keep])
    return Jm, area[keep]


@pytest.mark.parametrize("maker", [lambda: scenes.grid_frame(2, 1024), lambda: scenes.orbit_frame(17)])
def test_uv_similarity(maker):
    f = maker()
    r = oracle.build_frame(f, want_occupancy=False)
    Jm, _ = _jacobians(f, r)
    assert Jm.shape[0] > 20
    sv = np.linalg.svd(Jm, compute_uv=False)
    scale = f.rate * r["s_eff"]
    assert np.allclose(sv, scale, rtol=1e-3)
    assert (np.linalg.det(Jm) > 0).all()


def test_stretch_matches_paper_table():
    for row in STRETCH["rows"]:
        sf = row["scale_factor"]
        f = scenes.grid_frame(4, atlas_size=2048, rate=sf)
        r = oracle.build_frame(f, want_occupancy=False)
        assert r["s_eff"] == 1.0 and r["jstar"] == 64
        Jm, area = _jacobians(f, r)
        sv = np.linalg.svd(Jm, compute_uv=False)  # texels per pixel
        stretch = 1.0 / sv  # pixels per texel along each axis
        L2 = np.sqrt((area * (stretch ** 2).mean(1)).sum() / area.sum())
        Linf = stretch.max()
        assert abs(L2 - row["L2"]) < 1e-3 and abs(Linf - row["Linf"]) < 1e-3


def test_uv_inside_placed_box():
    f = scenes.orbit_frame(33)
    r = oracle.build_frame(f, want_occupancy=False)
    clip = r["clip"]
    cov = r["chart_of_vert"]
    inside = (np.abs(clip[:, 0]) <= clip[:, 3]) & (np.abs(clip[:, 1]) <= clip[:, 3]) & (clip[:, 3] > 0)
    v = np.nonzero((cov >= 0) & inside)[0]
    c = cov[v]
    q = f.atlas_size / r["L"]
    uv = r["uv"][v].astype(np.float64)
    lo_u, hi_u = (r["x"][c] + 1) * q, (r["x"][c] + r["a"][c] - 1) * q
    lo_v, hi_v = (r["y"][c] + 1) * q, (r["y"][c] + r["b"][c] - 1) * q
    eps = 1e-3
    assert ((uv[:, 0] >= lo_u - eps) & (uv[:, 0] <= hi_u + eps)).all()
    assert ((uv[:, 1] >= lo_v - eps) & (uv[:, 1] <= hi_v + eps)).all()
    assert np.isnan(r["uv"][cov < 0]).all()


def _edge_dist(px, py, ax, ay, bx, by):
    ex, ey = bx - ax, by - ay
    ln = np.hypot(ex, ey)
    return np.abs(ex * (py - ay) - ey * (px - ax)) / np.maximum(ln, 1e-300)


@pytest.mark.parametrize("seed,omega,rate", [(5, 256, 0.25), (9, 512, 0.5)])
def test_occupancy_vs_exact_point_in_triangle(seed, omega, rate):
    f = scenes.grid_frame(seed, atlas_size=omega, rate=rate)
    r = oracle.build_frame(f)
    occ = r["occupancy"]
    clip, uv = r["clip"], r["uv"].astype(np.float64)
    assert not ((clip[:, 3] + clip[:, 2]) < 0).any()  # no near crossing in this case
    want = np.full((omega, omega), -1, np.int64)
    ambiguous = np.zeros((omega, omega), bool)
    L = r["L"]
    tx = np.arange(omega)
    for t in np.nonzero(r["nonempty"])[0]:
        c = r["chart_of_tri"][t]
        P = uv[f.indices[t]]
        x0, x1 = int(np.floor(P[:, 0].min() - 1)), int(np.ceil(P[:, 0].max() + 1))
        y0, y1 = int(np.floor(P[:, 1].min() - 1)), int(np.ceil(P[:, 1].max() + 1))
        xs = tx[max(0, x0):max(0, min(omega, x1))]
        ys = tx[max(0, y0):max(0, min(omega, y1))]
        if xs.size == 0 or ys.size == 0:
            continue
        X, Y = np.meshgrid(xs + 0.5, ys + 0.5)
        e = [(P[(k + 1) % 3, 0] - P[k, 0]) * (Y - P[k, 1]) - (P[(k + 1) % 3, 1] - P[k, 1]) * (X - P[k, 0])
             for k in range(3)]
        inside = ((e[0] >= 0) & (e[1] >= 0) & (e[2] >= 0)) | ((e[0] <= 0) & (e[1] <= 0) & (e[2] <= 0))
        d = np.minimum.reduce([_edge_dist(X, Y, P[k, 0], P[k, 1], P[(k + 1) % 3, 0], P[(k + 1) % 3, 1])
                               for k in range(3)])
        bx, by, ba, bb = r["x"][c], r["y"][c], r["a"][c], r["b"][c]
        inbox = ((2 * bx * omega <= (2 * X - 0) * L) & ((2 * X) * L < 2 * (bx + ba) * omega) &
                 (2 * by * omega <= (2 * Y) * L) & ((2 * Y) * L < 2 * (by + bb) * omega))
        sub_w = want[ys[0]:ys[-1] + 1, xs[0]:xs[-1] + 1]
        sub_a = ambiguous[ys[0]:ys[-1] + 1, xs[0]:xs[-1] + 1]
        sub_w[inside & inbox] = c
        sub_a |= d < 4.0 / 256
    agree = (occ == want) | ambiguous
    assert agree.all(), int((~agree).sum())
    assert (occ >= 0).sum() > 1000


def test_occupancy_owner_inside_box_and_count():
    f = scenes.orbit_frame(40, atlas_size=1024)
    r = oracle.build_frame(f)
    occ = r["occupancy"]
    omega, L = f.atlas_size, r["L"]
    ty, tx = np.nonzero(occ >= 0)
    c = occ[ty, tx]
    assert (2 * r["x"][c].astype(np.int64) * omega <= (2 * tx + 1) * L).all()
    assert ((2 * tx + 1) * L < 2 * (r["x"][c] + r["a"][c]).astype(np.int64) * omega).all()
    assert (2 * r["y"][c].astype(np.int64) * omega <= (2 * ty + 1) * L).all()
    assert ((2 * ty + 1) * L < 2 * (r["y"][c] + r["b"][c]).astype(np.int64) * omega).all()
    assert r["occupied"] == int((occ >= 0).sum())


# ---------------------------------------------------------------------------
# the near-plane case of the occupancy (O10): a triangle that crosses the
# near plane claims the texels of its near-clipped polygon (a triangle or a
# quad), fanned from its first vertex
# ---------------------------------------------------------------------------
def _exact_poly(T):
    """Float64 polygon of a triangle's visible part in front of the near
    plane, clipped in exact rationals (None when nothing is in front)."""
    from fractions import Fraction
    dn = T[:, 3].astype(np.float64) + T[:, 2]
    if not (dn < 0).any():
        return T.astype(np.float64), False
    P = [[Fraction(float(v)) for v in T[k]] for k in range(3)]
    out = []
    for i in range(3):
        S, E = P[i], P[(i + 1) % 3]
        dS, dE = S[3] + S[2], E[3] + E[2]
        if (dS >= 0) != (dE >= 0):
            t = dS / (dS - dE)
            out.append([S[k] + t * (E[k] - S[k]) for k in range(4)])
        if dE >= 0:
            out.append(E)
    return np.array([[float(v) for v in p] for p in out]), True


def _map64(P, r, c, f, s, q, g=1):
    # the chart's map (O9) evaluated in float64 on the float32 chart records
    x0, y1 = float(r["frame"][c, 0]), float(r["frame"][c, 3])
    tw = float(r["target"][c, 0])
    nx, ny = P[:, 0] / P[:, 3], P[:, 1] / P[:, 3]
    px = (nx - x0) * (0.5 * f.width) * f.rate
    py = (y1 - ny) * (0.5 * f.height) * f.rate
    lx, ly = (py, tw - px) if r["rotated"][c] else (px, py)
    return np.stack([(r["x"][c] + g + lx * s) * q, (r["y"][c] + g + ly * s) * q], 1)


@pytest.mark.parametrize("maker", [lambda: scenes.grid_near_frame(1, atlas_size=512),
                                   lambda: scenes.grid_near_frame(4, atlas_size=512, rate=0.5),
                                   lambda: scenes.floor_near_frame(2, atlas_size=512)])
def test_occupancy_near_exact(maker):
    f = maker()
    r = oracle.build_frame(f)
    assert r["status"] == 0
    occ, omega, L = r["occupancy"], f.atlas_size, r["L"]
    s = float(np.float32(r["jstar"]) / np.float32(64))
    q = float(np.float32(omega) / np.float32(L))
    clip = r["clip"]
    want = np.full((omega, omega), -1, np.int64)
    ambiguous = np.zeros((omega, omega), bool)
    near_claims = {3: 0, 4: 0}
    tx = np.arange(omega)
    for t in np.nonzero(r["nonempty"])[0]:
        c = int(r["chart_of_tri"][t])
        P, crossed = _exact_poly(clip[f.indices[t]])
        if P.shape[0] < 3 or (P[:, 3] <= 0).any():
            continue
        Q = _map64(P, r, c, f, s, q)
        n = Q.shape[0]
        x0, x1 = int(np.floor(Q[:, 0].min() - 1)), int(np.ceil(Q[:, 0].max() + 1))
        y0, y1 = int(np.floor(Q[:, 1].min() - 1)), int(np.ceil(Q[:, 1].max() + 1))
        xs = tx[max(0, x0):max(0, min(omega, x1))]
        ys = tx[max(0, y0):max(0, min(omega, y1))]
        if xs.size == 0 or ys.size == 0:
            continue
        X, Y = np.meshgrid(xs + 0.5, ys + 0.5)
        e = [(Q[(k + 1) % n, 0] - Q[k, 0]) * (Y - Q[k, 1]) - (Q[(k + 1) % n, 1] - Q[k, 1]) * (X - Q[k, 0])
             for k in range(n)]
        inside = np.logical_and.reduce([ek >= 0 for ek in e]) | np.logical_and.reduce([ek <= 0 for ek in e])
        d = np.minimum.reduce([_edge_dist(X, Y, Q[k, 0], Q[k, 1], Q[(k + 1) % n, 0], Q[(k + 1) % n, 1])
                               for k in range(n)])
        bx, by, ba, bb = r["x"][c], r["y"][c], r["a"][c], r["b"][c]
        inbox = ((2 * bx * omega <= (2 * X) * L) & ((2 * X) * L < 2 * (bx + ba) * omega) &
                 (2 * by * omega <= (2 * Y) * L) & ((2 * Y) * L < 2 * (by + bb) * omega))
        sl = (slice(ys[0], ys[-1] + 1), slice(xs[0], xs[-1] + 1))
        claim = inside & inbox & (d >= 4.0 / 256)
        want[sl][inside & inbox] = c
        ambiguous[sl] |= d < 4.0 / 256
        if crossed:
            near_claims[n] += int(claim.sum())
    agree = (occ == want) | ambiguous
    assert agree.all(), int((~agree).sum())
    # the near branch was taken: clipped triangles and clipped quads claim texels
    assert near_claims[3] > 0 and near_claims[4] > 0, near_claims


def test_uv_nan_behind_eye():
    # a vertex of a visible triangle with w <= 0 has no image: its UV is NaN,
    # while the triangle's near-clipped part still claims texels
    f = scenes.floor_near_frame(2, atlas_size=512)
    r = oracle.build_frame(f)
    clip = r["clip"]
    behind = (r["chart_of_vert"] >= 0) & (clip[:, 3] <= 0)
    assert behind.sum() >= 1
    assert np.isnan(r["uv"][behind]).all()
    front = (r["chart_of_vert"] >= 0) & (clip[:, 3] > 0)
    assert not np.isnan(r["uv"][front]).any()
    tris_behind = np.nonzero(f.visible.astype(bool) & (clip[f.indices, 3] <= 0).any(1))[0]
    claimed = set(np.unique(r["occupancy"][r["occupancy"] >= 0]).tolist())
    assert any(int(r["chart_of_tri"][t]) in claimed for t in tris_behind)


# ---------------------------------------------------------------------------
# per-corner UVs of edge-connected charts (O9')
# ---------------------------------------------------------------------------
def _checker_frame(seed=0, omega=1024):
    # quads of the grid visible in a checkerboard (the others hidden): many
    # vertices are shared by edge-connected charts that meet only there
    f = scenes.grid_frame(seed, atlas_size=omega)
    q = np.arange(f.num_triangles) // 2
    i, j = q // 64, q % 64
    f.visible = (f.visible.astype(bool) & (((i // 2 + j // 2) % 2) == 0)).astype(np.uint8)
    return f


def test_uv_corners_similarity_and_seams():
    f = _checker_frame()
    r = oracle.build_frame(f, edge_only=True, want_occupancy=False)
    uvc = r["uv"].astype(np.float64)          # [T][3][2]
    assert uvc.shape == (f.num_triangles, 3, 2)
    clip = r["clip"]
    vis = f.visible.astype(bool)
    assert np.isnan(uvc[~vis]).all()
    P = _pixel_coords(clip, f.width, f.height)
    t = np.nonzero(vis & (clip[f.indices, 3] > 0).all(1))[0]
    p = P[f.indices[t]]
    A = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]], 2)
    B = np.stack([uvc[t, 1] - uvc[t, 0], uvc[t, 2] - uvc[t, 0]], 2)
    keep = np.abs(np.linalg.det(A)) / 2 > 30.0
    Jm = B[keep] @ np.linalg.inv(A[keep])
    assert keep.sum() > 20
    assert np.allclose(np.linalg.svd(Jm, compute_uv=False), f.rate * r["s_eff"], rtol=1e-3)
    assert (np.linalg.det(Jm) > 0).all()
    # corners of one vertex agree inside a chart and differ across charts
    cot = r["chart_of_tri"]
    seen, same, diff = {}, 0, 0
    for tt in t:
        for k in range(3):
            key = int(f.indices[tt, k])
            if key in seen:
                c0, uv0 = seen[key]
                if c0 == cot[tt]:
                    assert np.array_equal(uv0, uvc[tt, k])
                    same += 1
                else:
                    diff += int(not np.array_equal(uv0, uvc[tt, k]))
            else:
                seen[key] = (cot[tt], uvc[tt, k])
    assert same > 100 and diff > 10


def test_occupancy_edge_only_exact():
    # the occupancy of edge-connected charts: each triangle claims the texels
    # of its own chart's map (the per-corner UVs), exactly away from edges
    f = _checker_frame(5, omega=512)
    f.rate = 0.5
    r = oracle.build_frame(f, edge_only=True)
    occ, omega, L = r["occupancy"], f.atlas_size, r["L"]
    uvc = r["uv"].astype(np.float64)
    want = np.full((omega, omega), -1, np.int64)
    ambiguous = np.zeros((omega, omega), bool)
    tx = np.arange(omega)
    for t in np.nonzero(r["nonempty"])[0]:
        c = r["chart_of_tri"][t]
        P = uvc[t]
        if np.isnan(P).any():
            continue
        x0, x1 = int(np.floor(P[:, 0].min() - 1)), int(np.ceil(P[:, 0].max() + 1))
        y0, y1 = int(np.floor(P[:, 1].min() - 1)), int(np.ceil(P[:, 1].max() + 1))
        xs = tx[max(0, x0):max(0, min(omega, x1))]
        ys = tx[max(0, y0):max(0, min(omega, y1))]
        if xs.size == 0 or ys.size == 0:
            continue
        X, Y = np.meshgrid(xs + 0.5, ys + 0.5)
        e = [(P[(k + 1) % 3, 0] - P[k, 0]) * (Y - P[k, 1]) - (P[(k + 1) % 3, 1] - P[k, 1]) * (X - P[k, 0])
             for k in range(3)]
        inside = ((e[0] >= 0) & (e[1] >= 0) & (e[2] >= 0)) | ((e[0] <= 0) & (e[1] <= 0) & (e[2] <= 0))
        d = np.minimum.reduce([_edge_dist(X, Y, P[k, 0], P[k, 1], P[(k + 1) % 3, 0], P[(k + 1) % 3, 1])
                               for k in range(3)])
        bx, by, ba, bb = r["x"][c], r["y"][c], r["a"][c], r["b"][c]
        inbox = ((2 * bx * omega <= (2 * X) * L) & ((2 * X) * L < 2 * (bx + ba) * omega) &
                 (2 * by * omega <= (2 * Y) * L) & ((2 * Y) * L < 2 * (by + bb) * omega))
        sl = (slice(ys[0], ys[-1] + 1), slice(xs[0], xs[-1] + 1))
        want[sl][inside & inbox] = c
        ambiguous[sl] |= d < 4.0 / 256
    agree = (occ == want) | ambiguous
    assert agree.all(), int((~agree).sum())
    assert (occ >= 0).sum() > 1000 and r["occupancy_conflicts"] == 0
