"""CPU oracle of the FastAtlas per-frame atlasing path (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package. The GPU library never uses it. The arithmetic
lives in ``fa_oracle.cpp`` (single-threaded, float32 in a fixed order, built
with ``-ffp-contract=off``); this module only marshals numpy arrays and calls
the steps in the paper's order:

  clip -> charts -> per-triangle boxes -> chart frames/sizes -> order ->
  J candidate packings -> selection -> UVs -> occupancy.

No step here is parity-unpinned: every step has an independent pin in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fa_oracle.cpp")
_LIB = os.path.join(_HERE, "libfa_oracle.so")

STATUS_OK = 0
STATUS_NOFIT = 4


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (-O2, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i64, i32, f32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_float
        L.oracle_clip.argtypes = [P, i64, P, P]
        L.oracle_adjacency.argtypes = [P, i64, P]
        L.oracle_charts.argtypes = [P, i64, i64, P, P, P, P]
        L.oracle_charts.restype = i64
        L.oracle_triangle_boxes.argtypes = [P, P, P, i64, ctypes.c_int, P, P]
        L.oracle_chart_frames.argtypes = [P, P, P, i64, i64, i32, i32, f32, P, P, P, P, P]
        L.oracle_order.argtypes = [P, i64, P]
        L.oracle_candidate.argtypes = [P, P, i64, i32, i32, i32, i32, i32, P, P, P, P, P]
        L.oracle_select.argtypes = [P, i32]
        L.oracle_select.restype = i32
        L.oracle_uv.argtypes = [P, i64, P, P, P, P, P, P, i32, i32, f32, i32, i32, i32, i64, i32, P]
        L.oracle_occupancy.argtypes = [P, P, P, P, i64, P, P, P, P, P, P, P, i32, i32, f32, i32,
                                       i32, i32, i64, i32, P, P]
        L.oracle_occupancy.restype = i64
        L.oracle_visibility.argtypes = [P, i64, P, i64, P, P, ctypes.c_double, i32, i32, i32, P]
        L.oracle_reuse_flags.argtypes = [P, i64, P, i64, P, P, P, P]
        L.oracle_fine_profiles.argtypes = [P, P, P, P, i64, P, P, P, P, i32, i32, f32, P, P, P]
        L.oracle_pool_profile.argtypes = [P, P, i32, i32, i32, i32, i32, i32, i32, P, P]
        L.oracle_candidate_fp.argtypes = [P, P, P, P, P, i64, i32, P, P, P]
        L.oracle_reuse_flags.restype = i64
        L.oracle_charts_edge.argtypes = [P, i64, i64, P, P, P, P]
        L.oracle_charts_edge.restype = i64
        L.oracle_uv_corners.argtypes = [P, P, i64, P, P, P, P, P, P, i32, i32, f32, i32, i32,
                                        i32, i64, i32, P]
        L.oracle_near_polygon.argtypes = [P, P]
        L.oracle_near_polygon.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------------------
# individual steps
# ---------------------------------------------------------------------------
def clip(positions, view_proj):
    pos = _c(positions, np.float32)
    M = _c(view_proj, np.float32).ravel()
    out = np.empty((pos.shape[0], 4), np.float32)
    lib().oracle_clip(_p(pos), pos.shape[0], _p(M), _p(out))
    return out


def visibility(positions, indices, view_proj, eye, near, width, height, coarse=0):
    """Visible triangles of a view (App. "Detecting Visible Triangles"): uint8 [T]."""
    pos = _c(positions, np.float32)
    idx = _c(indices, np.int32)
    M = _c(view_proj, np.float32).ravel()
    e = _c(np.asarray(eye, np.float64), np.float64)
    out = np.empty(idx.shape[0], np.uint8)
    lib().oracle_visibility(_p(pos), pos.shape[0], _p(idx), idx.shape[0], _p(M), _p(e),
                            float(near), int(width), int(height), int(coarse), _p(out))
    return out


def reuse_flags(positions, indices, key_view_proj, key_visible, visible):
    """Temporal reuse classification (Sec. "Temporal Reuse"): (flags uint8 [T]
    with 0 not visible / 1 reuse / 2 shade, number reused)."""
    pos = _c(positions, np.float32)
    idx = _c(indices, np.int32)
    M = _c(key_view_proj, np.float32).ravel()
    kv = _c(key_visible, np.uint8)
    v = _c(visible, np.uint8)
    out = np.empty(idx.shape[0], np.uint8)
    n = lib().oracle_reuse_flags(_p(pos), pos.shape[0], _p(idx), idx.shape[0], _p(M), _p(kv),
                                 _p(v), _p(out))
    return out, int(n)


def adjacency(indices):
    idx = _c(indices, np.int32)
    out = np.empty((idx.shape[0], 3), np.int32)
    lib().oracle_adjacency(_p(idx), idx.shape[0], _p(out))
    return out


def charts(indices, num_vertices, visible, edge_only=False):
    """O3 charts (shared vertices), or with edge_only the O3' variant (shared
    edges only). Returns (chart_of_tri, chart_of_vert, roots)."""
    idx = _c(indices, np.int32)
    vis = _c(visible, np.uint8)
    T = idx.shape[0]
    cot = np.empty(T, np.int32)
    cov = np.empty(num_vertices, np.int32)
    roots = np.empty(max(T, 1), np.int32)
    fn = lib().oracle_charts_edge if edge_only else lib().oracle_charts
    C = fn(_p(idx), T, num_vertices, _p(vis), _p(cot), _p(cov), _p(roots))
    return cot, cov, roots[:C].copy()


def triangle_boxes(clip_xyzw, indices, visible, side_clip=True):
    c = _c(clip_xyzw, np.float32)
    idx = _c(indices, np.int32)
    vis = _c(visible, np.uint8)
    T = idx.shape[0]
    box = np.empty((T, 4), np.float32)
    ne = np.empty(T, np.uint8)
    lib().oracle_triangle_boxes(_p(c), _p(idx), _p(vis), T, int(side_clip), _p(box), _p(ne))
    return box, ne


def near_polygon(tri_clip):
    """The triangle (3 x xyzw clip coordinates) clipped against the near plane
    w + z >= 0 as O4 (ii), O10 and FP1 clip it: float32 [n, 4], n in 0, 3, 4."""
    t = _c(tri_clip, np.float32).reshape(3, 4)
    out = np.zeros((4, 4), np.float32)
    n = lib().oracle_near_polygon(_p(t), _p(out))
    return out[:n].copy()


def chart_frames(box, nonempty, chart_of_tri, C, W, H, rate):
    box, ne, cot = _c(box, np.float32), _c(nonempty, np.uint8), _c(chart_of_tri, np.int32)
    frame = np.zeros((C, 4), np.float32)
    target = np.zeros((C, 2), np.float32)
    oriented = np.zeros((C, 2), np.float32)
    rot = np.zeros(C, np.int32)
    key = np.zeros(C, np.int32)
    lib().oracle_chart_frames(_p(box), _p(ne), _p(cot), cot.shape[0], C, W, H, float(rate),
                              _p(frame), _p(target), _p(oriented), _p(rot), _p(key))
    return frame, target, oriented, rot, key


def order(key):
    k = _c(key, np.int32)
    out = np.empty(k.shape[0], np.int32)
    lib().oracle_order(_p(k), k.shape[0], _p(out))
    return out


def candidate(sbw, sbh, j, J, omega, gutter=1, min_box=2):
    """One candidate packing. Returns dict(fit, m, L, H, rows, x, y, a, b)
    with per-box arrays in sorted order."""
    w, h = _c(sbw, np.float32), _c(sbh, np.float32)
    C = w.shape[0]
    x, y, a, b = (np.empty(C, np.int32) for _ in range(4))
    out = np.zeros(5, np.int64)
    lib().oracle_candidate(_p(w), _p(h), C, j, J, omega, gutter, min_box, _p(x), _p(y), _p(a),
                           _p(b), _p(out))
    return dict(fit=bool(out[0]), m=int(out[1]), L=int(out[2]), H=int(out[3]), rows=int(out[4]),
                x=x, y=y, a=a, b=b)


def fine_profiles(clip_c, indices, nonempty, chart_of_tri, frame, target, oriented, rotated,
                  W, H, rate):
    """Full-scale footprint profile of every chart (FP1). Returns (foff, ft, fb):
    chart c owns columns foff[c] .. foff[c + 1] - 1 (Uc = floor(bw) + 1 of
    them); empty columns hold ft = INT32_MAX, fb = -1."""
    C = oriented.shape[0]
    uc = np.floor(np.asarray(oriented, np.float32)[:, 0]).astype(np.int64) + 1
    foff = np.zeros(C + 1, np.int64)
    foff[1:] = np.cumsum(uc)
    n = int(foff[-1])
    ft = np.full(n, np.iinfo(np.int32).max, np.int32)
    fb = np.full(n, -1, np.int32)
    idx = _c(indices, np.int32)
    lib().oracle_fine_profiles(_p(_c(clip_c, np.float32)), _p(idx), _p(_c(nonempty, np.uint8)),
                               _p(_c(chart_of_tri, np.int32)), idx.shape[0],
                               _p(_c(frame, np.float32)), _p(_c(target, np.float32)),
                               _p(_c(oriented, np.float32)), _p(_c(rotated, np.int32)), int(W),
                               int(H), float(rate), _p(foff), _p(ft), _p(fb))
    return foff, ft, fb


def pool_profile(ft_c, fb_c, Rc, a, b, j, J, gutter):
    """Profile (top, bottom per column) of one chart's a x b box at candidate j
    (FP2) from its full-scale columns ft_c, fb_c and row count Rc."""
    ft_c, fb_c = _c(ft_c, np.int32), _c(fb_c, np.int32)
    top = np.empty(int(a), np.int32)
    bot = np.empty(int(a), np.int32)
    lib().oracle_pool_profile(_p(ft_c), _p(fb_c), ft_c.shape[0], int(Rc), int(a), int(b), int(j),
                              int(J), int(gutter), _p(top), _p(bot))
    return top, bot


def candidate_fp(a_o, b_o, top, bot, poff_o, omega):
    """Footprint-aware push of one candidate (FP3; inputs in packing order)."""
    C = a_o.shape[0]
    x = np.empty(C, np.int32)
    y = np.empty(C, np.int32)
    out = np.zeros(5, np.int64)
    lib().oracle_candidate_fp(_p(_c(a_o, np.int32)), _p(_c(b_o, np.int32)), _p(_c(top, np.int32)),
                              _p(_c(bot, np.int32)), _p(_c(poff_o, np.int64)),
                              C, int(omega), _p(x), _p(y), _p(out))
    return dict(fit=bool(out[0]), m=int(out[1]), L=int(out[2]), H=int(out[3]), rows=int(out[4]),
                x=x, y=y)


def footprint_candidate(fine, oriented, j, J, omega, gutter, order_, box_cd):
    """Candidate j with the footprint-aware push; sizes (a, b) and fold from
    the box candidate, profiles pooled from the full-scale ones (FP2).
    Boxes are in packing order; prof_off[i] = fold position X_i."""
    foff, ft, fb = fine
    a_o, b_o = box_cd["a"], box_cd["b"]
    C = a_o.shape[0]
    poff_o = np.zeros(C, np.int64)
    if C:
        poff_o[1:] = np.cumsum(a_o[:-1].astype(np.int64))
    n = int(poff_o[-1] + a_o[-1]) if C else 0
    top = np.empty(n, np.int32)
    bot = np.empty(n, np.int32)
    rc = np.floor(np.asarray(oriented, np.float32)[:, 1]).astype(np.int64) + 1
    for i in range(C):
        c = int(order_[i])
        t, b_ = pool_profile(ft[foff[c]:foff[c + 1]], fb[foff[c]:foff[c + 1]], rc[c], a_o[i],
                             b_o[i], j, J, gutter)
        top[poff_o[i]:poff_o[i] + a_o[i]] = t
        bot[poff_o[i]:poff_o[i] + a_o[i]] = b_
    fp = candidate_fp(a_o, b_o, top, bot, poff_o, omega)
    fp.update(a=a_o, b=b_o, top=top, bot=bot, prof_off=poff_o, H_box=box_cd["H"])
    return fp


def select(cand_table):
    ct = _c(cand_table, np.int64)
    return int(lib().oracle_select(_p(ct), ct.shape[0]))


# ---------------------------------------------------------------------------
# the whole path
# ---------------------------------------------------------------------------
def build_atlas(positions, indices, visible, view_proj, width, height, atlas_size, rate,
                J=64, gutter=1, min_box=2, side_clip=True, want_occupancy=True,
                want_adjacency=False, low_shift=0, footprint=False, edge_only=False):
    """Run every step on one frame. Returns a dict of all intermediate and
    final results (per-chart arrays are indexed by chart index). low_shift = k
    > 0 adds the occupancy of the same packing scaled into an atlas of side
    omega / 2^k (App. "Depth-of-Field" and "Foveated Rendering": the low
    resolution atlas reuses the packing, coordinates scaled per axis).
    footprint=True packs with the footprint-aware push (per-column profiles
    of each chart's footprint instead of its full box). edge_only=True takes
    the edge-connected charts (O3') and returns per-corner UVs [T][3][2]."""
    pos = _c(positions, np.float32)
    idx = _c(indices, np.int32)
    vis = _c(visible, np.uint8)
    T, V = idx.shape[0], pos.shape[0]
    omega, W, H = int(atlas_size), int(width), int(height)
    r = dict()
    r["clip"] = clip(pos, view_proj)
    if want_adjacency:
        r["nbr"] = adjacency(idx)
    cot, cov, roots = charts(idx, V, vis, edge_only=edge_only)
    C = roots.shape[0]
    r.update(chart_of_tri=cot, chart_of_vert=cov, roots=roots, num_charts=C)
    box, ne = triangle_boxes(r["clip"], idx, vis, side_clip)
    r.update(tri_box=box, nonempty=ne)
    frame, target, oriented, rot, key = chart_frames(box, ne, cot, C, W, H, rate)
    r.update(frame=frame, target=target, oriented=oriented, rotated=rot, key=key)
    o = order(key)
    rank = np.empty(C, np.int32)
    rank[o] = np.arange(C, dtype=np.int32)
    r.update(order=o, rank=rank)
    sbw = np.ascontiguousarray(oriented[o, 0])
    sbh = np.ascontiguousarray(oriented[o, 1])
    table = np.zeros((J, 5), np.int64)
    cands = []
    if footprint:
        if gutter < 1:
            raise ValueError("the footprint-aware push needs a gutter of at least 1")
        fine = fine_profiles(r["clip"], idx, ne, cot, frame, target, oriented, rot, W, H, rate)
        r["fine_profiles"] = fine
    for j in range(1, J + 1):
        cd = candidate(sbw, sbh, j, J, omega, gutter, min_box)
        if footprint:
            cd = footprint_candidate(fine, oriented, j, J, omega, gutter, o, cd)
        cands.append(cd)
        table[j - 1] = [cd["fit"], cd["m"], cd["L"], cd["H"], cd["rows"]]
    r["cand"] = table
    if footprint:
        r["fp_cands"] = cands
    js = select(table)
    r["jstar"] = js
    px = np.zeros(C, np.int32)
    py = np.zeros(C, np.int32)
    pa = np.zeros(C, np.int32)
    pb = np.zeros(C, np.int32)
    if js == 0:
        r.update(status=STATUS_NOFIT, L=0, H=0, s_eff=0.0, x=px, y=py, a=pa, b=pb)
        return r
    w = cands[js - 1]
    px[o], py[o], pa[o], pb[o] = w["x"], w["y"], w["a"], w["b"]
    L = w["L"]
    s = np.float32(js) / np.float32(J)
    q = np.float32(omega) / np.float32(L)
    r.update(status=STATUS_OK, L=L, H=w["H"], s_eff=float(np.float32(s * q)), x=px, y=py, a=pa,
             b=pb)
    clip_c = r["clip"]
    if edge_only:
        uv = np.empty((T, 3, 2), np.float32)
        lib().oracle_uv_corners(_p(clip_c), _p(idx), T, _p(cot), _p(frame), _p(target), _p(rot),
                                _p(px), _p(py), W, H, float(rate), js, J, omega, L, gutter,
                                _p(uv))
    else:
        uv = np.empty((V, 2), np.float32)
        lib().oracle_uv(_p(clip_c), V, _p(cov), _p(frame), _p(target), _p(rot), _p(px), _p(py),
                        W, H, float(rate), js, J, omega, L, gutter, _p(uv))
    r["uv"] = uv
    conflicts = np.zeros(1, np.int64)
    if want_occupancy:
        occ = np.empty((omega, omega), np.int32)
        n = lib().oracle_occupancy(_p(clip_c), _p(idx), _p(ne), _p(cot), T, _p(frame), _p(target),
                                   _p(rot), _p(px), _p(py), _p(pa), _p(pb), W, H, float(rate), js,
                                   J, omega, L, gutter, _p(occ), _p(conflicts))
        r.update(occupancy=occ, occupied=int(n), occupancy_conflicts=int(conflicts[0]))
    if low_shift:
        ol = omega >> int(low_shift)
        occ_l = np.empty((ol, ol), np.int32)
        n = lib().oracle_occupancy(_p(clip_c), _p(idx), _p(ne), _p(cot), T, _p(frame), _p(target),
                                   _p(rot), _p(px), _p(py), _p(pa), _p(pb), W, H, float(rate), js,
                                   J, ol, L, gutter, _p(occ_l), _p(conflicts))
        r.update(occupancy_low=occ_l, occupied_low=int(n),
                 occupancy_low_conflicts=int(conflicts[0]))
    return r


def build_frame(frame, **kw):
    """build_atlas on a synth.scenes.Frame."""
    return build_atlas(frame.positions, frame.indices, frame.visible, frame.view_proj,
                       frame.width, frame.height, frame.atlas_size, frame.rate, **kw)
