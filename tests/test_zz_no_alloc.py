"""The allocation-free entry point (fa_build_atlas_static) against
fa_build_atlas on the same frames: two calls in a row, the second on a
smaller mesh, then out-of-range indices (reported on the device) and a good
frame again. Results must be identical (integers and float bits; UVs within
1e-4 texels)."""
import ctypes

import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu


def _fa():
    import paper_2502_17712_amd as fa
    return fa


def _orbit_part(k):
    # the first 60000 triangles of an orbit frame (all its vertices): a mesh
    # inside the static limits, larger than the grid
    f = scenes.orbit_frame(k, atlas_size=2048)
    f.indices = np.ascontiguousarray(f.indices[:60000])
    f.visible = np.ascontiguousarray(f.visible[:60000])
    f.scene_key = 88001 + k
    f.name += "/first60000"
    return f


def _poison(o):
    for t in (o.chart_of_tri, o.chart_of_vert, o.occupancy, o.candidates, o.charts, o.meta):
        t.fill_(-7)
    o.uv.fill_(-7.0)


def _static(fa, f, mesh, out):
    _poison(out)
    vis = torch.as_tensor(f.visible).cuda()
    fa.build_atlas_static(mesh, vis, f.view_proj, f.width, f.height, f.atlas_size, f.rate,
                          out=out)
    torch.cuda.synchronize()
    return out.to_numpy()


def _same(a, b):
    assert a["meta"] == b["meta"], (a["meta"], b["meta"])
    for k in ("chart_of_tri", "chart_of_vert", "occupancy", "candidates"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["charts"], b["charts"])
    ua, ub = a["uv"], b["uv"]
    assert np.array_equal(np.isnan(ua), np.isnan(ub))
    fin = ~np.isnan(ua)
    assert np.abs(ua[fin] - ub[fin]).max(initial=0.0) <= 1e-4


def test_static_matches_context_path():
    fa = _fa()
    frames = [_orbit_part(12), scenes.grid_frame(3)]   # the second call is smaller
    assert frames[1].num_triangles < frames[0].num_triangles
    # library default knobs on both sides (the static entry point has no
    # tuning table; the raster's tile count in meta depends on the knobs)
    ctx = fa.Context(max(f.num_triangles for f in frames), max(f.num_vertices for f in frames),
                     max_charts=fa.STATIC_MAX_CHARTS, max_atlas=4096, tuning_table=None)
    for f in frames:
        print(f"[gpu] static vs context: {f.name} T={f.num_triangles}", flush=True)
        mesh = fa.Mesh(f.positions, f.indices, f.scene_key)
        want = ctx.build_atlas(mesh, torch.as_tensor(f.visible).cuda(), f.view_proj, f.width,
                               f.height, f.atlas_size, f.rate)
        torch.cuda.synchronize()
        want = want.to_numpy()
        assert want["meta"]["status"] == 0 and want["meta"]["num_charts"] > 0
        out = fa.AtlasOutputs(f.num_triangles, f.num_vertices, fa.STATIC_MAX_CHARTS,
                              f.atlas_size, 64)
        _same(_static(fa, f, mesh, out), want)
    ctx.close()


def test_static_many_charts():
    # 3000 charts: the order runs over several workgroups in both entry points
    fa = _fa()
    f = scenes.scatter_frame(0, count=3000, atlas_size=2048)
    ctx = fa.Context(f.num_triangles, f.num_vertices, max_charts=fa.STATIC_MAX_CHARTS,
                     max_atlas=2048, tuning_table=None)
    print(f"[gpu] static vs context: {f.name} T={f.num_triangles}", flush=True)
    mesh = fa.Mesh(f.positions, f.indices, f.scene_key)
    want = ctx.build_atlas(mesh, torch.as_tensor(f.visible).cuda(), f.view_proj, f.width,
                           f.height, f.atlas_size, f.rate)
    torch.cuda.synchronize()
    want = want.to_numpy()
    assert want["meta"]["status"] == 0 and want["meta"]["num_charts"] > 1024
    out = fa.AtlasOutputs(f.num_triangles, f.num_vertices, fa.STATIC_MAX_CHARTS, f.atlas_size, 64)
    _same(_static(fa, f, mesh, out), want)
    ctx.close()


def test_static_errors_and_recovery():
    fa = _fa()
    f = scenes.grid_frame(5)
    out = fa.AtlasOutputs(f.num_triangles, f.num_vertices, fa.STATIC_MAX_CHARTS, f.atlas_size, 64)
    # out-of-range indices: found on the device, reported in meta->status
    bad = fa.Mesh(f.positions, np.where(f.indices == 11, f.num_vertices + 5, f.indices), 88100)
    print("[gpu] static: out-of-range indices", flush=True)
    g = _static(fa, f, bad, out)
    assert g["meta"]["status"] == fa.FA_ERR_INVALID_ARG
    # a good frame right after is correct again
    ctx = fa.Context(f.num_triangles, f.num_vertices, max_charts=fa.STATIC_MAX_CHARTS,
                     max_atlas=1024, tuning_table=None)
    mesh = fa.Mesh(f.positions, f.indices, f.scene_key)
    want = ctx.build_atlas(mesh, torch.as_tensor(f.visible).cuda(), f.view_proj, f.width,
                           f.height, f.atlas_size, f.rate)
    torch.cuda.synchronize()
    print("[gpu] static: good frame after the error", flush=True)
    _same(_static(fa, f, mesh, out), want.to_numpy())
    ctx.close()
    # above the static limits: a synchronous error, nothing enqueued
    big = fa.Mesh(np.zeros((10, 3), np.float32),
                  np.zeros((fa.STATIC_MAX_TRIANGLES + 1, 3), np.int32), 88200)
    vis = torch.zeros(fa.STATIC_MAX_TRIANGLES + 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(fa.FastAtlasError) as e:
        fa.build_atlas_static(big, vis, f.view_proj, f.width, f.height, 1024, 1.0, out=out)
    assert e.value.code == fa.FA_ERR_CAPACITY
