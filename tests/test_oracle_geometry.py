"""Pins for the oracle's clip transform, per-triangle boxes, chart frames and
ordering (CPU only).

* clip: exact small-integer products (an operand transposed or a term dropped
  changes the result).
* per-triangle boxes: exact float64 clipping against all six planes gives the
  true visible extent E; the method's box must contain E (it is conservative,
  Sec. bounding boxes) and must equal E bit for bit when nothing is clipped.
* chart frames: a numpy group-by min/max; sizes against the viewport formula
  evaluated in float64 within rounding.
* order: the lexicographic (height desc, root asc) order written as a sort key.
"""
import math

import numpy as np
import pytest

import oracle
from synth import scenes


def test_clip_exact_integers():
    rng = np.random.default_rng(0)
    M = rng.integers(-8, 9, size=(4, 4)).astype(np.float32)
    pos = rng.integers(-50, 51, size=(200, 3)).astype(np.float32)
    got = oracle.clip(pos, M.ravel())
    want = np.concatenate([pos.astype(np.int64), np.ones((200, 1), np.int64)], 1) @ M.astype(np.int64).T
    assert np.array_equal(got, want.astype(np.float32))


def test_clip_matches_float64():
    f = scenes.orbit_frame(5)
    got = oracle.clip(f.positions, f.view_proj).astype(np.float64)
    M = f.view_proj.astype(np.float64).reshape(4, 4)
    want = f.positions.astype(np.float64) @ M[:, :3].T + M[:, 3]
    scale = np.abs(f.positions.astype(np.float64)) @ np.abs(M[:, :3]).T + np.abs(M[:, 3])
    assert (np.abs(got - want) <= 4 * np.finfo(np.float32).eps * scale).all()


# ---------------------------------------------------------------------------
# exact visible extent in float64
# ---------------------------------------------------------------------------
_PLANES = [lambda p: p[3] + p[0], lambda p: p[3] - p[0], lambda p: p[3] + p[1],
           lambda p: p[3] - p[1], lambda p: p[3] + p[2], lambda p: p[3] - p[2]]


def _clip_all(poly):
    for d in _PLANES:
        out = []
        n = len(poly)
        for i in range(n):
            S, E = poly[i], poly[(i + 1) % n]
            dS, dE = d(S), d(E)
            if (dS >= 0) != (dE >= 0):
                t = dS / (dS - dE)
                out.append(S + t * (E - S))
            if dE >= 0:
                out.append(E)
        poly = out
        if not poly:
            return []
    return poly


def _exact_box(tri64, with_minw=False):
    poly = _clip_all([tri64[k] for k in range(3)])
    if not poly:
        return (None, None) if with_minw else None
    P = np.array(poly)
    nx, ny = P[:, 0] / P[:, 3], P[:, 1] / P[:, 3]
    box = np.array([nx.min(), ny.min(), nx.max(), ny.max()])
    return (box, P[:, 3].min()) if with_minw else box


def _random_clip_triangles(rng, n, spread):
    # world-like triangles seen by a GL camera: w = distance, z from a GL
    # depth mapping, x and y up to `spread` times outside the frustum
    near, far = 0.1, 100.0
    out = []
    for _ in range(n):
        zc = rng.uniform(-3.0, 30.0, 3) if rng.uniform() < 0.5 else rng.uniform(0.2, 30.0, 3)
        w = zc.copy()
        z = (far + near) / (far - near) * w - 2 * far * near / (far - near)
        x = rng.uniform(-spread, spread, 3) * np.abs(w) + rng.normal(0, 0.3, 3)
        y = rng.uniform(-spread, spread, 3) * np.abs(w) + rng.normal(0, 0.3, 3)
        out.append(np.stack([x, y, z, w], 1))
    return np.array(out, np.float32)


def _boxes(tris, side_clip=True):
    n = tris.shape[0]
    clip = np.ascontiguousarray(tris.reshape(-1, 4))
    idx = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    return oracle.triangle_boxes(clip, idx, np.ones(n, np.uint8), side_clip)


def test_box_exact_when_inside():
    rng = np.random.default_rng(1)
    tris = _random_clip_triangles(rng, 3000, 0.8)
    box, ne = _boxes(tris)
    checked = 0
    for t in range(tris.shape[0]):
        T64 = tris[t].astype(np.float64)
        inside = all(d(T64[k]) >= 0 for d in _PLANES for k in range(3))
        if not inside:
            continue
        E = _exact_box(T64).astype(np.float32)
        assert ne[t] == 1
        assert np.array_equal(box[t], E), (t, box[t], E)
        checked += 1
    assert checked > 100


def test_box_conservative():
    rng = np.random.default_rng(2)
    tris = _random_clip_triangles(rng, 4000, 2.5)
    box, ne = _boxes(tris)
    nonempty_exact = 0
    for t in range(tris.shape[0]):
        E, minw = _exact_box(tris[t].astype(np.float64), with_minw=True)
        if ne[t] == 0:
            # empty only if the triangle is entirely outside one plane
            T64 = tris[t].astype(np.float64)
            assert any(all(d(T64[k]) < 0 for k in range(3)) for d in _PLANES)
            assert E is None
            continue
        if E is None:
            continue  # outside the volume without being outside a single plane
        nonempty_exact += 1
        # float32 rounding of the clip intersection, magnified by 1/w
        mag = float(np.abs(tris[t]).max())
        tol = 1e-6 + 64 * float(np.finfo(np.float32).eps) * mag / minw
        assert box[t, 0] <= E[0] + tol and box[t, 1] <= E[1] + tol
        assert box[t, 2] >= E[2] - tol and box[t, 3] >= E[3] - tol
        assert -1.0 <= box[t, 0] <= box[t, 2] <= 1.0 and -1.0 <= box[t, 1] <= box[t, 3] <= 1.0
    assert nonempty_exact > 1000


def test_box_single_side_plane_is_tight():
    # a triangle crossing exactly one side plane (and not near) is clipped by
    # that plane, which makes the box the exact visible extent up to rounding
    rng = np.random.default_rng(3)
    tris = _random_clip_triangles(rng, 6000, 1.4)
    box, ne = _boxes(tris)
    checked = 0
    for t in range(tris.shape[0]):
        T64 = tris[t].astype(np.float64)
        crossing = [i for i, d in enumerate(_PLANES) if min(d(T64[k]) for k in range(3)) < 0]
        if len(crossing) != 1 or crossing[0] == 4:
            continue
        E, minw = _exact_box(T64, with_minw=True)
        if E is None:
            continue
        tol = 1e-6 + 64 * float(np.finfo(np.float32).eps) * float(np.abs(tris[t]).max()) / minw
        assert np.allclose(box[t], E, atol=tol, rtol=0), (box[t], E)
        checked += 1
    assert checked > 200


def test_box_near_clip_tighter_than_blinn_alone():
    # Appendix "Bounding Box Computation Alternatives": clipping at the near
    # plane gives a box no larger than Blinn's estimate of the whole triangle
    rng = np.random.default_rng(4)
    tris = _random_clip_triangles(rng, 3000, 1.0)
    box, ne = _boxes(tris)
    for t in range(tris.shape[0]):
        T = tris[t].astype(np.float64)
        dn = T[:, 3] + T[:, 2]
        if not (dn.min() < 0 <= dn.max()) or ne[t] == 0:
            continue
        if (T[:, 3] <= 0).any():
            blinn = np.array([-1, -1, 1, 1.0])
        else:
            cx = np.clip(T[:, 0], -T[:, 3], T[:, 3]) / T[:, 3]
            cy = np.clip(T[:, 1], -T[:, 3], T[:, 3]) / T[:, 3]
            blinn = np.array([cx.min(), cy.min(), cx.max(), cy.max()])
        assert box[t, 0] >= blinn[0] - 1e-6 and box[t, 2] <= blinn[2] + 1e-6


def test_box_side_clip_flag():
    rng = np.random.default_rng(5)
    tris = _random_clip_triangles(rng, 2000, 2.0)
    b1, n1 = _boxes(tris, True)
    b0, n0 = _boxes(tris, False)
    assert np.array_equal(n0, n1)
    a1 = (b1[:, 2] - b1[:, 0]) * (b1[:, 3] - b1[:, 1])
    a0 = (b0[:, 2] - b0[:, 0]) * (b0[:, 3] - b0[:, 1])
    assert (a1[n1 == 1] <= a0[n1 == 1]).all()
    assert (a1 < a0).sum() > 10


# ---------------------------------------------------------------------------
# chart frames and order
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("rate", [0.5, 1.0, 2.0])
def test_chart_frames_groupby(rate):
    f = scenes.orbit_frame(11)
    clip = oracle.clip(f.positions, f.view_proj)
    cot, cov, roots = oracle.charts(f.indices, f.num_vertices, f.visible)
    box, ne = oracle.triangle_boxes(clip, f.indices, f.visible)
    C = roots.shape[0]
    frame, target, oriented, rot, key = oracle.chart_frames(box, ne, cot, C, f.width, f.height, rate)
    want = np.zeros((C, 4), np.float64)
    want[:, :2], want[:, 2:] = np.inf, -np.inf
    sel = ne == 1
    np.minimum.at(want[:, 0], cot[sel], box[sel, 0])
    np.minimum.at(want[:, 1], cot[sel], box[sel, 1])
    np.maximum.at(want[:, 2], cot[sel], box[sel, 2])
    np.maximum.at(want[:, 3], cot[sel], box[sel, 3])
    want[~np.isfinite(want)] = 0.0
    assert np.array_equal(frame, want.astype(np.float32))
    assert not np.signbit(frame[frame == 0]).any()
    tw = (want[:, 2] - want[:, 0]) * f.width / 2 * rate
    th = (want[:, 3] - want[:, 1]) * f.height / 2 * rate
    assert np.allclose(target[:, 0], tw, rtol=1e-6, atol=1e-5)
    assert np.allclose(target[:, 1], th, rtol=1e-6, atol=1e-5)
    assert (oriented[:, 0] <= oriented[:, 1]).all()
    assert np.array_equal(rot == 1, target[:, 0] > target[:, 1])
    assert key.tolist() == [min(math.ceil(float(h)), 8191) for h in oriented[:, 1]]


def test_order_lexicographic():
    rng = np.random.default_rng(7)
    for C in (0, 1, 5, 300, 5000):
        key = rng.integers(0, 40 if C > 10 else 3, size=C).astype(np.int32)
        got = oracle.order(key)
        want = sorted(range(C), key=lambda c: (-int(key[c]), c))
        assert got.tolist() == want


# ---------------------------------------------------------------------------
# the near-plane special case (O4 ii; App. "Bounding Box Computation
# Alternatives": a triangle that crosses the near plane is clipped there
# before Blinn's divide)
# ---------------------------------------------------------------------------
def _exact_near_clip(T):
    """Sutherland-Hodgman against w + z >= 0 in exact rationals on the float32
    inputs (edges c0->c1, c1->c2, c2->c0; the intersection before the end
    vertex)."""
    from fractions import Fraction
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
    return out


def _near_crossers(rng, n):
    tris = _random_clip_triangles(rng, n, 1.2)
    dn = tris[:, :, 3] + tris[:, :, 2]
    return tris[(dn.min(1) < 0) & (dn.max(1) >= 0)]


def _frame_near_crossers(f):
    clip = oracle.clip(f.positions, f.view_proj)
    T = clip[f.indices]
    dn = T[:, :, 3] + T[:, :, 2]
    sel = f.visible.astype(bool) & (dn.min(1) < 0) & (dn.max(1) >= 0)
    return T[sel]


def test_near_polygon_exact():
    # the near-clipped polygon equals exact clipping of the same float32
    # vertices within the rounding of t and of one lerp per component, with
    # the vertices in the same order; both shapes (quad: one vertex behind
    # near, triangle: two behind) occur
    rng = np.random.default_rng(11)
    tris = np.concatenate([_near_crossers(rng, 3000)] +
                          [_frame_near_crossers(f) for f in
                           (scenes.grid_near_frame(1), scenes.floor_near_frame(2))])
    eps = float(np.finfo(np.float32).eps)
    counts = {3: 0, 4: 0}
    for T in tris:
        got = oracle.near_polygon(T)
        want = _exact_near_clip(T)
        assert got.shape[0] == len(want) and len(want) in (3, 4)
        counts[len(want)] += 1
        mag = float(np.abs(T).max())
        for k in range(len(want)):
            w = np.array([float(v) for v in want[k]])
            assert np.abs(got[k].astype(np.float64) - w).max() <= 8 * eps * mag, (T, got, want)
        # the clipped polygon lies on or in front of the near plane, up to rounding
        assert ((got[:, 3].astype(np.float64) + got[:, 2]) >= -8 * eps * mag).all()
    assert counts[3] > 40 and counts[4] > 100, counts


def test_box_near_only_is_tight():
    # a triangle that crosses the near plane and no other plane is clipped at
    # near, so its box is the exact visible extent up to rounding (a wrong
    # plane, a dropped intersection or a swapped end point would show here)
    rng = np.random.default_rng(12)
    tris = np.concatenate([_near_crossers(rng, 6000)] +
                          [_frame_near_crossers(f) for f in
                           (scenes.grid_near_frame(s) for s in range(4))])
    box, ne = _boxes(tris)
    checked = 0
    for t in range(tris.shape[0]):
        T64 = tris[t].astype(np.float64)
        crossing = [i for i, d in enumerate(_PLANES) if min(d(T64[k]) for k in range(3)) < 0]
        if crossing != [4]:
            continue
        E, minw = _exact_box(T64, with_minw=True)
        assert ne[t] == 1 and E is not None
        tol = 1e-6 + 64 * float(np.finfo(np.float32).eps) * float(np.abs(tris[t]).max()) / minw
        assert np.allclose(box[t], E, atol=tol, rtol=0), (box[t], E)
        checked += 1
    assert checked > 100, checked


def test_near_frames_have_near_crossers():
    # the seeded near-plane frames hold visible triangles of both clipped
    # shapes, and the coarse floor and the low city camera also hold visible
    # triangles with a vertex behind the eye (w <= 0)
    for f in (scenes.grid_near_frame(0), scenes.floor_near_frame(0)):
        clip = oracle.clip(f.positions, f.view_proj)
        dn = (clip[:, 3] + clip[:, 2])[f.indices]
        vis = f.visible.astype(bool)
        assert (vis & ((dn < 0).sum(1) == 1)).sum() >= 3
        assert (vis & ((dn < 0).sum(1) == 2)).sum() >= 2
    f = scenes.floor_near_frame(2)
    clip = oracle.clip(f.positions, f.view_proj)
    assert (f.visible.astype(bool) & (clip[f.indices, 3] <= 0).any(1)).sum() >= 1
