"""Pins of the footprint-aware push oracle (per-column footprint profiles in
place of full boxes in the push of Sec. "Box Packing").

Each step is checked against something other than itself:
  * the push with full-height profiles equals the box push (O7, pinned in
    test_oracle_pack);
  * the push against a literal simulation on an explicit cell grid (a box
    rises from below until its next step would overlap an occupied cell);
  * the full-scale profile against exact rational clipping of each snapped
    polygon to each column strip (fractions.Fraction, Sutherland-Hodgman);
  * the pooled profile against a brute force over the cells each fine cell
    touches at scale j/J, dilated by the gutter;
  * whole frames: the footprint packing never lets two charts claim one texel,
    every occupied texel lies in its chart's placed profile, and the chosen
    scale is never below the box packing's.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
from synth import scenes

INT_MAX = np.iinfo(np.int32).max


# ---------------------------------------------------------------------------
# the push
# ---------------------------------------------------------------------------
def _random_sizes(rng, C, lo=1.0, hi=40.0):
    w = rng.uniform(lo, hi, C).astype(np.float32)
    h = rng.uniform(lo, hi, C).astype(np.float32)
    rot = w > h
    bw, bh = np.where(rot, h, w), np.where(rot, w, h)
    key = np.minimum(np.ceil(bh).astype(np.int32), 8191)
    o = np.argsort(-key, kind="stable")
    return np.ascontiguousarray(bw[o]), np.ascontiguousarray(bh[o])


@pytest.mark.parametrize("seed", range(6))
def test_full_profiles_equal_box_push(seed):
    rng = np.random.default_rng(seed)
    sbw, sbh = _random_sizes(rng, 200)
    for j in (8, 33, 64):
        cd = oracle.candidate(sbw, sbh, j, 64, 256)
        a, b = cd["a"], cd["b"]
        poff = np.concatenate([[0], np.cumsum(a[:-1].astype(np.int64))])
        top = np.zeros(int(a.sum()), np.int32)
        bot = np.repeat(b - 1, a).astype(np.int32)
        fp = oracle.candidate_fp(a, b, top, bot, poff, 256)
        for k in ("fit", "m", "L", "rows"):
            assert fp[k] == cd[k], (j, k)
        if cd["m"] <= 256:
            assert fp["H"] == cd["H"]
            assert np.array_equal(fp["x"], cd["x"]) and np.array_equal(fp["y"], cd["y"])


def _grid_push(a, b, top, bot, poff, x, rows_of, omega, L):
    """Literal simulation: rows of boxes in order; a box starts below every
    occupied cell and rises one row at a time while the next position is free
    (y >= 0). Returns (y, H, grid)."""
    C = a.shape[0]
    depth = 2 * int(b.sum()) + 4
    grid = np.zeros((depth, L), bool)
    y = np.zeros(C, np.int64)
    i = 0
    while i < C:
        e = i
        while e < C and rows_of[e] == rows_of[i]:
            e += 1
        for k in range(i, e):
            cols = [(q, top[poff[k] + q], bot[poff[k] + q]) for q in range(a[k])
                    if bot[poff[k] + q] >= 0]

            def free(yy):
                return all(not grid[yy + t:yy + bt + 1, x[k] + q].any() for q, t, bt in cols)

            yy = depth - int(b.max()) - 1
            assert free(yy)
            while yy > 0 and free(yy - 1):
                yy -= 1
            y[k] = yy
        for k in range(i, e):   # the row's writes after all its reads
            for q in range(a[k]):
                t, bt = top[poff[k] + q], bot[poff[k] + q]
                if bt >= 0:
                    assert not grid[y[k] + t:y[k] + bt + 1, x[k] + q].any(), "overlap"
                    grid[y[k] + t:y[k] + bt + 1, x[k] + q] = True
        i = e
    occ_rows = np.nonzero(grid.any(1))[0]
    H = int(occ_rows.max()) + 1 if occ_rows.size else 0
    return y, H


@pytest.mark.parametrize("seed", range(8))
def test_push_matches_grid_simulation(seed):
    rng = np.random.default_rng(100 + seed)
    omega = 64
    sbw, sbh = _random_sizes(rng, 40, 1.0, 14.0)
    cd = oracle.candidate(sbw, sbh, 64, 64, omega)
    a, b = cd["a"], cd["b"]
    poff = np.concatenate([[0], np.cumsum(a[:-1].astype(np.int64))])
    n = int(a.sum())
    top = np.full(n, INT_MAX, np.int32)
    bot = np.full(n, -1, np.int32)
    for i in range(a.shape[0]):
        for q in range(a[i]):
            if rng.random() < 0.2:
                continue  # empty column
            t0 = int(rng.integers(0, b[i]))
            t1 = int(rng.integers(t0, b[i]))
            top[poff[i] + q], bot[poff[i] + q] = t0, t1
    fp = oracle.candidate_fp(a, b, top, bot, poff, omega)
    assert fp["m"] == cd["m"] and fp["L"] == cd["L"]
    if cd["m"] > omega:
        pytest.skip("candidate rejected by its overflow")
    assert np.array_equal(fp["x"], cd["x"])
    rows_of = np.array([p >> 6 for p in poff])
    y, H = _grid_push(a, b, top, bot, poff, fp["x"], rows_of, omega, fp["L"])
    assert np.array_equal(fp["y"], y)
    assert fp["H"] == H and fp["fit"] == (H <= fp["L"])


def test_tall_box_rejected():
    a = np.array([4, 4], np.int32)
    b = np.array([10, 2 * 64 + 1], np.int32)
    top = np.zeros(8, np.int32)
    bot = np.zeros(8, np.int32)
    fp = oracle.candidate_fp(a, b, top, bot, np.array([0, 4], np.int64), 64)
    assert not fp["fit"] and fp["H"] == -1


# ---------------------------------------------------------------------------
# the full-scale profile
# ---------------------------------------------------------------------------
def _clip_half(poly, x0, keep_right):
    out = []
    n = len(poly)
    for i in range(n):
        S, E = poly[i], poly[(i + 1) % n]
        iS = S[0] >= x0 if keep_right else S[0] <= x0
        iE = E[0] >= x0 if keep_right else E[0] <= x0
        if iS != iE:
            t = (x0 - S[0]) / (E[0] - S[0])
            out.append((x0, S[1] + t * (E[1] - S[1])))
        if iE:
            out.append(E)
    return out


def _snapped_local(f, r, t, near=False):
    """Snapped chart-local polygon of triangle t (1/256 units), float32 chain
    of the UV map before scale and gutter; None if it claims nothing. A
    triangle crossing the near plane gives "near", or with near=True its
    near-clipped polygon (the oracle's clip, pinned against exact clipping in
    test_oracle_geometry)."""
    c = int(r["chart_of_tri"][t])
    if c < 0 or not r["nonempty"][t]:
        return None, c
    clip = r["clip"]
    P = [clip[int(v)] for v in f.indices[t]]
    if any(np.float32(p[3] + p[2]) < 0 for p in P):
        if not near:
            return "near", c
        P = list(oracle.near_polygon(np.array(P)))
        if not all(p[3] > 0 for p in P):
            return None, c
    x0 = np.float32(r["frame"][c, 0])
    y1 = np.float32(r["frame"][c, 3])
    tw = np.float32(r["target"][c, 0])
    hw, hh = np.float32(0.5) * np.float32(f.width), np.float32(0.5) * np.float32(f.height)
    rate = np.float32(f.rate)
    out = []
    for p in P:
        nx, ny = np.float32(p[0]) / np.float32(p[3]), np.float32(p[1]) / np.float32(p[3])
        px = np.float32(np.float32(np.float32(nx - x0) * hw) * rate)
        py = np.float32(np.float32(np.float32(y1 - ny) * hh) * rate)
        lx, ly = (py, np.float32(tw - px)) if r["rotated"][c] else (px, py)
        out.append((int(np.rint(np.float32(lx * np.float32(256)))),
                    int(np.rint(np.float32(ly * np.float32(256))))))
    return out, c


def _near_case(k):
    return [scenes.grid_near_frame(1), scenes.grid_near_frame(4, rate=0.5),
            scenes.floor_near_frame(2)][k]


@pytest.mark.parametrize("case", ["grid2", "grid7", "near0", "near1", "near2"])
def test_fine_profile_exact(case):
    near = case.startswith("near")
    f = _near_case(int(case[4:])) if near else scenes.grid_frame(int(case[4:]))
    r = oracle.build_frame(f, want_occupancy=False)
    foff, ft, fb = oracle.fine_profiles(r["clip"], f.indices, r["nonempty"], r["chart_of_tri"],
                                        r["frame"], r["target"], r["oriented"], r["rotated"],
                                        f.width, f.height, f.rate)
    C = r["num_charts"]
    uc = np.floor(r["oriented"][:, 0]).astype(np.int64) + 1
    rc = np.floor(r["oriented"][:, 1]).astype(np.int64) + 1
    assert np.array_equal(np.diff(foff), uc)
    ref_t = np.full(ft.shape, INT_MAX, np.int64)
    ref_b = np.full(fb.shape, -1, np.int64)
    shapes = {3: 0, 4: 0}
    for t in np.nonzero(f.visible)[0]:
        poly, c = _snapped_local(f, r, t, near=near)
        assert poly != "near"      # the small scene never crosses the near plane
        if poly is None:
            continue
        if near and any(r["clip"][int(v), 3] + r["clip"][int(v), 2] < 0 for v in f.indices[t]):
            shapes[len(poly)] += 1
        poly = [(Fraction(x), Fraction(y)) for x, y in poly]
        xs = [p[0] for p in poly]
        u0 = min(uc[c] - 1, max(0, math.floor(min(xs) / 256)))
        u1 = min(uc[c] - 1, max(0, math.floor(max(xs) / 256)))
        for u in range(u0, u1 + 1):
            q = poly
            if u > 0:
                q = _clip_half(q, Fraction(256 * u), True)
            if u < uc[c] - 1 and q:
                q = _clip_half(q, Fraction(256 * (u + 1)), False)
            if not q:
                continue
            lo = math.floor(min(p[1] for p in q) / 256)
            hi = math.floor(max(p[1] for p in q) / 256)
            lo, hi = min(rc[c] - 1, max(0, lo)), min(rc[c] - 1, max(0, hi))
            k = foff[c] + u
            ref_t[k] = min(ref_t[k], lo)
            ref_b[k] = max(ref_b[k], hi)
    assert np.array_equal(ft.astype(np.int64), ref_t)
    assert np.array_equal(fb.astype(np.int64), ref_b)
    if near:   # near-clipped triangles and quads both took part
        assert shapes[3] > 0 and shapes[4] > 0, shapes
    # every chart has some footprint
    for c in range(C):
        assert (fb[foff[c]:foff[c + 1]] >= 0).any()


# ---------------------------------------------------------------------------
# pooling to a candidate scale
# ---------------------------------------------------------------------------
def _pool_brute(ft, fb, Rc, a, b, j, J, g):
    Uc = ft.shape[0]
    s = Fraction(j, J)
    cells = set()
    for u in range(Uc):
        if fb[u] < 0:
            continue
        k0 = math.floor(u * s)
        k1 = a - g - 1 if u == Uc - 1 else math.floor((u + 1) * s)
        for rr in range(int(ft[u]), int(fb[u]) + 1):
            q0 = math.floor(rr * s)
            q1 = b if rr == Rc - 1 else math.floor((rr + 1) * s)
            for k in range(k0, k1 + 1):
                if k + g >= a:
                    continue
                for d in range(k, k + 2 * g + 1):      # box column k + g, dilated by g
                    if d >= a:
                        continue
                    for row in range(q0, min(q1 + 2 * g, b - 1) + 1):
                        cells.add((d, row))
    top = np.full(a, INT_MAX, np.int64)
    bot = np.full(a, -1, np.int64)
    for d, row in cells:
        top[d] = min(top[d], row)
        bot[d] = max(bot[d], row)
    return top, bot


@pytest.mark.parametrize("seed", range(10))
def test_pool_matches_brute_force(seed):
    rng = np.random.default_rng(500 + seed)
    J = 16 if seed % 2 else 64
    g = 1 + seed % 2
    Uc = int(rng.integers(1, 30))
    Rc = int(rng.integers(1, 20))
    ft = np.full(Uc, INT_MAX, np.int32)
    fb = np.full(Uc, -1, np.int32)
    for u in range(Uc):
        if rng.random() < 0.25:
            continue
        t0 = int(rng.integers(0, Rc))
        ft[u], fb[u] = t0, int(rng.integers(t0, Rc))
    bw = Uc - 1 + rng.random() * 0.999
    bh = Rc - 1 + rng.random() * 0.999
    for j in range(1, J + 1):
        s = np.float32(j) / np.float32(J)
        a = max(2, int(math.ceil(np.float32(bw) * s))) + 2 * g
        b = max(2, int(math.ceil(np.float32(bh) * s))) + 2 * g
        top, bot = oracle.pool_profile(ft, fb, Rc, a, b, j, J, g)
        bt, bb = _pool_brute(ft, fb, Rc, a, b, j, J, g)
        assert np.array_equal(top.astype(np.int64), bt), j
        assert np.array_equal(bot.astype(np.int64), bb), j


# ---------------------------------------------------------------------------
# whole frames
# ---------------------------------------------------------------------------
def _profile_of(r, c):
    w = r["fp_winner"]
    i = int(r["rank"][c])
    o, a = int(w["prof_off"][i]), int(w["a"][i])
    return w["top"][o:o + a], w["bot"][o:o + a]


def _frames():
    return [scenes.grid_frame(3, atlas_size=256), scenes.grid_frame(11, atlas_size=512, rate=2.0),
            scenes.orbit_frame(20, atlas_size=512)]


@pytest.mark.parametrize("k", range(3))
def test_frames_footprint_packing(k):
    f = _frames()[k]
    rb = oracle.build_frame(f)
    rf = oracle.build_frame(f, footprint=True)
    assert rb["status"] == 0 and rf["status"] == 0
    cb, cf = rb["cand"], rf["cand"]
    # same sizes, fold and overflow; a footprint frontline never rises above the box one
    assert np.array_equal(cb[:, 1], cf[:, 1]) and np.array_equal(cb[:, 2], cf[:, 2])
    both = (cb[:, 0] == 1)
    assert (cf[both, 0] == 1).all() and (cf[both, 3] <= cb[both, 3]).all()
    # the chosen effective scale is at least the box packing's
    jb, jf = rb["jstar"], rf["jstar"]
    assert jf * rb["L"] >= jb * rf["L"]
    # footprints never share a texel
    assert rf["occupancy_conflicts"] == 0 and rb["occupancy_conflicts"] == 0
    # every occupied texel lies in its chart's placed profile (closed cells)
    occ = rf["occupancy"]
    omega, L = f.atlas_size, rf["L"]
    ys, xs = np.nonzero(occ >= 0)
    assert ys.size > 0
    rf["fp_winner"] = rf["fp_cands"][jf - 1]
    for ty, tx in zip(ys, xs):
        c = int(occ[ty, tx])
        top, bot = _profile_of(rf, c)
        px = Fraction((2 * int(tx) + 1) * L, 2 * omega) - int(rf["x"][c])
        py = Fraction((2 * int(ty) + 1) * L, 2 * omega) - int(rf["y"][c])
        cols = {math.floor(px)} | ({int(px) - 1} if px.denominator == 1 else set())
        rows = {math.floor(py)} | ({int(py) - 1} if py.denominator == 1 else set())
        assert any(0 <= d < top.shape[0] and bot[d] >= 0 and top[d] <= q <= bot[d]
                   for d in cols for q in rows), (c, tx, ty)


def test_gutter_zero_rejected():
    f = scenes.grid_frame(3, atlas_size=256)
    with pytest.raises(ValueError):
        oracle.build_frame(f, footprint=True, gutter=0)
