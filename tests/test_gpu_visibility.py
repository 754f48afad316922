"""Parity of the GPU visible-triangle pass (fa_visibility) with the oracle.

Bar: the visible sets are bytes, so they must be identical. Cases: the three
scene families (the large one with its 480x270 coarse depth buffer, also at
factors 1, 4 and 64), hand-built occlusion scenes, argument errors, and the
device visible set feeding the atlas path.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import scenes

pytestmark = pytest.mark.gpu

_CTX = {}


def _fa():
    import paper_2502_17712_amd as fa
    return fa


def _ctx(T=2_300_000, V=1_200_000):
    if (T, V) not in _CTX:
        _CTX[(T, V)] = _fa().Context(T, V, max_charts=65536, max_atlas=4096)
    return _CTX[(T, V)]


_MESH = {}


def _mesh(f):
    key = (f.scene_key, f.num_triangles)
    if key not in _MESH:
        _MESH[key] = _fa().Mesh(f.positions, f.indices, f.scene_key)
    return _MESH[key]


def _gpu(f, coarse=None, ctx=None):
    c = f.coarse if coarse is None else coarse
    print(f"[gpu] visibility {f.name} T={f.num_triangles} coarse={c}", flush=True)
    ctx = ctx or _ctx()
    v = ctx.visibility(_mesh(f), f.view_proj, f.width, f.height, f.eye, f.near, c)
    torch.cuda.synchronize()
    return v.cpu().numpy()


def _ora(f, coarse=None):
    c = f.coarse if coarse is None else coarse
    return oracle.visibility(f.positions, f.indices, f.view_proj, f.eye, f.near, f.width,
                             f.height, c)


@pytest.mark.parametrize("seed", [0, 9, 17, 33])
def test_grid(seed):
    f = scenes.grid_frame(seed)
    assert np.array_equal(_gpu(f), _ora(f))


@pytest.mark.parametrize("frame", [0, 31, 77])
def test_orbit(frame):
    f = scenes.orbit_frame(frame)
    assert np.array_equal(_gpu(f), _ora(f))
    assert np.array_equal(_gpu(f, coarse=2), _ora(f, coarse=2))


@pytest.mark.parametrize("frame", [0, 13])
def test_city_coarse(frame):
    f = scenes.city_frame(frame)
    g = _gpu(f)
    assert np.array_equal(g, _ora(f))
    assert np.array_equal(g, f.visible)


@pytest.mark.parametrize("coarse", [1, 4, 64])
def test_city_other_grids(coarse):
    f = scenes.city_frame(21)
    assert np.array_equal(_gpu(f, coarse=coarse), _ora(f, coarse=coarse))


def _camera(W=64, H=64, near=0.1):
    return scenes.make_camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), W, H, near, 100.0, up=(0, 1, 0))


def _quad(z, half, cx=0.0, cy=0.0):
    p = np.array([[cx - half, cy - half, z], [cx + half, cy - half, z],
                  [cx + half, cy + half, z], [cx - half, cy + half, z]], np.float32)
    return p, np.array([[0, 1, 2], [0, 2, 3]], np.int32)


def test_hand_built_occlusion():
    fa = _fa()
    parts = [_quad(-2.0, 1.0), _quad(-5.0, 1.0), _quad(-3.0, 0.2, cx=2.5), _quad(-4.0, 4.0)]
    pos, tri, off = [], [], 0
    for p, t in parts:
        pos.append(p)
        tri.append(t + off)
        off += p.shape[0]
    pos, tri = np.concatenate(pos), np.concatenate(tri)
    cam = _camera()
    mesh = fa.Mesh(pos, tri, 77001)
    ctx = _ctx()
    for coarse in (0, 1, 2, 8):
        g = ctx.visibility(mesh, cam.view_proj, 64, 64, cam.eye, cam.near, coarse).cpu().numpy()
        o = oracle.visibility(pos, tri, cam.view_proj, cam.eye, cam.near, 64, 64, coarse)
        assert np.array_equal(g, o), coarse
    assert o.tolist()[:4] == [1, 1, 0, 0]


def test_nothing_visible_and_errors():
    fa = _fa()
    ctx = _ctx()
    # camera looking away from every triangle: no candidate, no occluder
    away = scenes.make_camera((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 64, 64, 0.1, 100.0, up=(0, 1, 0))
    pos, tri = _quad(-2.0, 1.0)
    m0 = fa.Mesh(pos, tri, 77002)
    v = ctx.visibility(m0, away.view_proj, 64, 64, away.eye, away.near, 8)
    torch.cuda.synchronize()
    assert v.cpu().numpy().tolist() == [0, 0]
    f = scenes.grid_frame(1)
    m = _mesh(f)
    for kw in (dict(coarse=65), dict(coarse=-1), dict(near=0.0), dict(near=float("nan"))):
        args = dict(coarse=0, near=f.near)
        args.update(kw)
        with pytest.raises(fa.FastAtlasError):
            ctx.visibility(m, f.view_proj, f.width, f.height, f.eye, args["near"], args["coarse"])
    with pytest.raises(fa.FastAtlasError):
        ctx.visibility(m, f.view_proj, 0, f.height, f.eye, f.near, 0)
    bad = fa.Mesh(f.positions, np.full((4, 3), f.num_vertices, np.int32), 77003)
    with pytest.raises(fa.FastAtlasError):
        ctx.visibility(bad, f.view_proj, f.width, f.height, f.eye, f.near, 0)


def test_device_visibility_feeds_atlas():
    # visible set made on the device, then the atlas of the same frame: equal to
    # the oracle's atlas of the generator's frame
    fa = _fa()
    f = scenes.orbit_frame(12)
    ctx = _ctx()
    m = _mesh(f)
    vis = ctx.visibility(m, f.view_proj, f.width, f.height, f.eye, f.near, f.coarse)
    out = ctx.build_atlas(m, vis, f.view_proj, f.width, f.height, f.atlas_size, f.rate)
    torch.cuda.synchronize()
    g = out.to_numpy()
    r = oracle.build_frame(f)
    assert np.array_equal(g["chart_of_tri"], r["chart_of_tri"])
    assert fa.parse_meta(out.meta)["chosen_j"] == r["jstar"]
    assert np.array_equal(g["occupancy"], r["occupancy"])


def test_serve_device_visibility_equals_precomputed():
    """Requests that leave visibility to the device give the same atlases as
    the same requests carrying the generator's visible sets."""
    fa = _fa()
    from paper_2502_17712_amd import serve
    from synth import requests as rq
    meshes_np = {k: v for k, v in rq.scene_meshes().items() if k != "city"}
    meshes = {k: fa.Mesh(p, t, key) for k, (p, t, key) in meshes_np.items()}
    pools = {"grid": rq.pose_pool("grid", 3, seed=4), "orbit": rq.pose_pool("orbit", 3, seed=5)}
    stream = rq.poisson_stream(4000.0, 16, pools, clients=4, seed=6)
    reqs_dev, reqs_pre = [], []
    for rid, (a, c, s, i, om, r) in enumerate(stream):
        pz = pools[s][i]
        common = dict(arrival=a * 0.05, client=c, eye=tuple(pz.eye), near=pz.near,
                      coarse=pz.coarse)
        reqs_dev.append(serve.Request(rid, s, None, pz.view_proj, pz.width, pz.height, om, r,
                                      **common))
        reqs_pre.append(serve.Request(rid, s, torch.as_tensor(pz.visible).cuda(), pz.view_proj,
                                      pz.width, pz.height, om, r, **common))
    print("[gpu] serve 16 requests with device visibility on 4 slots", flush=True)
    srv = serve.Server(meshes, slots=4, hbm_budget=2 << 30, max_charts=8192, max_atlas=4096)
    dev = {q.rid: q for q in srv.run(reqs_dev, keep_outputs=True)}
    pre = {q.rid: q for q in srv.run(reqs_pre, keep_outputs=True)}
    srv.close()
    for rid in dev:
        a, b = dev[rid].out.to_numpy(), pre[rid].out.to_numpy()
        for k in ("chart_of_tri", "chart_of_vert", "occupancy", "candidates"):
            assert np.array_equal(a[k], b[k]), (rid, k)
        assert a["meta"] == b["meta"]


@pytest.mark.parametrize("key,frames", [(10, (11, 14, 19)), (0, (0, 3))])
def test_reuse_flags(key, frames):
    kf = scenes.orbit_frame(key)
    ctx = _ctx()
    m = _mesh(kf)
    kvis = torch.as_tensor(kf.visible).cuda()
    for k in frames:
        f = scenes.orbit_frame(k)
        print(f"[gpu] reuse flags key {key} frame {k}", flush=True)
        flags, reused = ctx.reuse_flags(m, kf.view_proj, kvis, torch.as_tensor(f.visible).cuda())
        torch.cuda.synchronize()
        ref, n = oracle.reuse_flags(f.positions, f.indices, kf.view_proj, kf.visible, f.visible)
        assert np.array_equal(flags.cpu().numpy(), ref)
        assert int(reused.item()) == n
