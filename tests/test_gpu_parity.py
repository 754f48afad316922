"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, element by element.

Bar: bit-exact chart ids, chart boxes (float bits), sizes, order, candidate
table, placements, layout meta and occupancy; UVs within 1e-4 texels (they
are computed with the same float32 operations, so they are expected to be
bit-identical too).
"""
import collections
import sys

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


def ctx_for(J=64, gutter=1, flags=0, max_charts=65536, T=2_300_000, V=1_200_000):
    # no tuning table: the knob tests set the knobs they check, and a table
    # entry for the frame's shape would take precedence
    key = (J, gutter, flags, max_charts, T, V)
    if key not in _CTX:
        _CTX[key] = _fa().Context(T, V, max_charts=max_charts, max_atlas=8192, num_scales=J,
                                  gutter=gutter, flags=flags, tuning_table=None)
    return _CTX[key]


_MESH = {}


def mesh_for(frame):
    fa = _fa()
    k = (frame.scene_key, frame.num_triangles)
    if k not in _MESH:
        _MESH[k] = fa.Mesh(frame.positions, frame.indices, frame.scene_key)
    return _MESH[k]


def run_gpu(frame, ctx, occupancy=True):
    print(f"[gpu] {frame.name} T={frame.num_triangles} omega={frame.atlas_size} r={frame.rate}",
          flush=True)
    mesh = mesh_for(frame)
    vis = torch.as_tensor(frame.visible).cuda()
    out = ctx.outputs(mesh, frame.atlas_size, occupancy=occupancy)
    ctx.build_atlas(mesh, vis, frame.view_proj, frame.width, frame.height, frame.atlas_size,
                    frame.rate, out=out)
    torch.cuda.synchronize()
    return out.to_numpy()


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def compare(g, r, occupancy=True):
    m = g["meta"]
    assert m["status"] == r["status"], (m, r["status"])
    assert m["num_charts"] == r["num_charts"]
    assert m["visible_triangles"] == int(np.count_nonzero(r["chart_of_tri"] >= 0))
    assert np.array_equal(g["chart_of_tri"], r["chart_of_tri"])
    assert np.array_equal(g["chart_of_vert"], r["chart_of_vert"])
    ch = g["charts"]
    C = r["num_charts"]
    assert ch.shape[0] == C
    assert np.array_equal(ch["root_tri"], r["roots"])
    assert np.array_equal(bits(ch["ndc_box"]), bits(r["frame"]))
    assert np.array_equal(bits(ch["target_w"]), bits(r["target"][:, 0]))
    assert np.array_equal(bits(ch["target_h"]), bits(r["target"][:, 1]))
    assert np.array_equal(bits(ch["oriented_w"]), bits(r["oriented"][:, 0]))
    assert np.array_equal(bits(ch["oriented_h"]), bits(r["oriented"][:, 1]))
    assert np.array_equal(ch["rotated"], r["rotated"])
    assert np.array_equal(ch["key"], r["key"])
    assert np.array_equal(ch["order_rank"], r["rank"])
    cand = g["candidates"]
    rc = r["cand"]
    assert np.array_equal(cand[:, 0], rc[:, 0])
    assert np.array_equal(cand[:, 1], rc[:, 1]) and np.array_equal(cand[:, 2], rc[:, 2])
    fit = rc[:, 0] == 1
    assert np.array_equal(cand[fit, 3], rc[fit, 3])
    assert m["chosen_j"] == r["jstar"]
    if r["status"] != 0:
        return
    assert (m["layout_width"], m["layout_height"]) == (r["L"], r["H"])
    assert m["rows"] == r["cand"][r["jstar"] - 1, 4]
    assert np.float32(m["s_eff"]) == np.float32(r["s_eff"])
    for k in ("x", "y"):
        assert np.array_equal(ch[k], r[k]), k
    assert np.array_equal(ch["w"], r["a"]) and np.array_equal(ch["h"], r["b"])
    gu, ru = g["uv"], r["uv"]
    assert np.array_equal(np.isnan(gu), np.isnan(ru))
    fin = ~np.isnan(ru)
    if fin.any():
        assert np.abs(gu[fin] - ru[fin]).max() <= 1e-4
        print(f"  uv bit-identical: {np.mean(bits(gu[fin]) == bits(ru[fin])):.6f}")
    if occupancy:
        assert m["occupied_texels"] == r["occupied"]
        assert np.array_equal(g["occupancy"], r["occupancy"])


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", list(range(64)))
def test_grid_frames(seed):
    f = scenes.grid_frame(seed)
    g = run_gpu(f, ctx_for())
    compare(g, oracle.build_frame(f))


@pytest.mark.parametrize("J,gutter,omega,rate", [(16, 0, 256, 1.0), (32, 1, 128, 1.0),
                                                 (64, 0, 512, 2.0), (64, 1, 64, 0.5)])
def test_grid_variants(J, gutter, omega, rate):
    f = scenes.grid_frame(5, atlas_size=omega, rate=rate)
    g = run_gpu(f, ctx_for(J=J, gutter=gutter))
    compare(g, oracle.build_frame(f, J=J, gutter=gutter))


@pytest.mark.parametrize("first", list(range(0, 120, 8)))
def test_orbit_frames(first):
    # all 120 frames of the orbit, eight per test
    for frame in range(first, first + 8):
        f = scenes.orbit_frame(frame)
        g = run_gpu(f, ctx_for())
        compare(g, oracle.build_frame(f))


def test_orbit_no_side_clip():
    f = scenes.orbit_frame(33)
    g = run_gpu(f, ctx_for(flags=_fa().FA_FLAG_NO_SIDE_CLIP))
    compare(g, oracle.build_frame(f, side_clip=False))


@pytest.mark.parametrize("frame", [0, 8, 16, 24])
@pytest.mark.parametrize("rate", [1.0, 0.5, 2.0])
def test_city_frame_full(frame, rate):
    f = scenes.city_frame(frame, rate=rate)
    g = run_gpu(f, ctx_for())
    compare(g, oracle.build_frame(f))


@pytest.mark.parametrize("frame", [0, 5, 10])
@pytest.mark.parametrize("rate", [1.0, 2.0])
def test_scatter_many_charts(frame, rate):
    # ~20k charts per frame: ordering and packing at the chart counts where
    # the paper's packing cost grows, past the packer's in-LDS capacity
    f = scenes.scatter_frame(frame, rate=rate)
    r = oracle.build_frame(f)
    assert r["num_charts"] >= 10000
    compare(run_gpu(f, ctx_for()), r)


@pytest.mark.parametrize("count,frame", [(1000, 2), (1500, 0), (1500, 3), (1800, 5),
                                         (2200, 1)])
def test_scatter_order_around_lds_capacity(count, frame):
    """Frames of about 900 to 2100 charts: the chart order keeps up to 2048
    charts in one workgroup's LDS and splits larger frames over 32 workgroups;
    both sides of that limit match the oracle."""
    f = scenes.scatter_frame(frame, count=count)
    r = oracle.build_frame(f)
    assert 800 <= r["num_charts"] <= 2200, r["num_charts"]
    compare(run_gpu(f, ctx_for()), r)


def test_city_frames_more():
    for fr in (9, 23):
        f = scenes.city_frame(fr)
        g = run_gpu(f, ctx_for())
        compare(g, oracle.build_frame(f, want_occupancy=False), occupancy=False)


@pytest.mark.parametrize("knob,value", [(1, 256), (1, 512), (2, 0), (2, 16), (2, 1024),
                                        (2, 4096), (3, 0), (5, 0), (5, 1), (5, 2), (5, 3),
                                        (5, 4), (6, 0), (6, 1), (6, 4096), (7, 2048),
                                        (7, 8192)])
def test_tuning_knobs_do_not_change_results(knob, value):
    fa = _fa()
    ctx = ctx_for()
    old = ctx.get_tuning(knob)
    ctx.set_tuning(knob, value)
    try:
        for f in (scenes.orbit_frame(21), scenes.city_frame(5)):
            g = run_gpu(f, ctx)
            compare(g, oracle.build_frame(f))
    finally:
        ctx.set_tuning(knob, old)
    with pytest.raises(fa.FastAtlasError):
        ctx.set_tuning(knob, {1: 3, 2: -1, 3: 3, 5: 6, 6: 4097, 7: 1024}[knob])


# ---------------------------------------------------------------------------
def _random_mesh(rng, T, V):
    idx = rng.integers(0, V, size=(T, 3)).astype(np.int32)
    for t in range(1, T, 3):
        idx[t, 0], idx[t, 1] = idx[t - 1, 1], idx[t - 1, 0]
    idx[5] = [3, 3, 4]  # degenerate edges
    return idx


@pytest.mark.parametrize("which", ["grid", "orbit", "city", "random"])
def test_adjacency(which):
    fa = _fa()
    if which == "grid":
        f = scenes.grid_frame(0)
        pos, idx, key = f.positions, f.indices, 77001
    elif which == "orbit":
        f = scenes.orbit_frame(0)
        pos, idx, key = f.positions, f.indices, 77002
    elif which == "city":
        pos, idx = scenes.city_scene()
        key = 77003
    else:
        rng = np.random.default_rng(3)
        idx = _random_mesh(rng, 3000, 400)
        pos = rng.normal(size=(400, 3)).astype(np.float32)
        key = 77004
    print(f"[gpu] adjacency {which} T={idx.shape[0]}", flush=True)
    mesh = fa.Mesh(pos, idx, key)
    nbr = ctx_for().adjacency(mesh)
    torch.cuda.synchronize()
    assert np.array_equal(nbr.cpu().numpy(), oracle.adjacency(idx))


# ---------------------------------------------------------------------------
def _oracle_pack(sizes, omega, J=64, g=1, mmin=2):
    w, h = sizes[:, 0], sizes[:, 1]
    rot = (w > h).astype(np.int32)
    bw, bh = np.where(rot == 1, h, w), np.where(rot == 1, w, h)
    key = np.minimum(np.ceil(bh).astype(np.int64), 8191).astype(np.int32)
    o = oracle.order(key)
    sbw, sbh = np.ascontiguousarray(bw[o]), np.ascontiguousarray(bh[o])
    table = np.zeros((J, 5), np.int64)
    cands = []
    for j in range(1, J + 1):
        cd = oracle.candidate(sbw, sbh, j, J, omega, g, mmin)
        cands.append(cd)
        table[j - 1] = [cd["fit"], cd["m"], cd["L"], cd["H"], cd["rows"]]
    js = oracle.select(table)
    pl = np.zeros((sizes.shape[0], 5), np.int64)
    if js:
        w_ = cands[js - 1]
        pl[o, 0], pl[o, 1], pl[o, 2], pl[o, 3] = w_["x"], w_["y"], w_["a"], w_["b"]
    pl[:, 4] = rot
    return js, table, pl


# 1024 and 1025 boxes sit on either side of the one-workgroup order; above
# it the order runs in 32 chunks (1025: a short last chunk)
@pytest.mark.parametrize("n,omega,seed", [(0, 1024, 0), (1, 64, 1), (7, 64, 2), (1000, 1024, 3),
                                          (1024, 1024, 6), (1025, 2048, 7), (20000, 4096, 4),
                                          (33000, 4096, 8), (60000, 8192, 5)])
def test_pack_boxes(n, omega, seed):
    rng = np.random.default_rng(seed)
    # heavy-tailed sizes: many tiny boxes, some large ones
    sizes = (rng.pareto(1.6, size=(n, 2)) * 6.0).astype(np.float32)
    sizes = np.minimum(sizes, omega * 0.9).astype(np.float32)
    print(f"[gpu] pack n={n} omega={omega}", flush=True)
    ctx = ctx_for()
    pl, meta, cand = ctx.pack_boxes(torch.as_tensor(sizes).cuda(), omega)
    torch.cuda.synchronize()
    m = _fa().parse_meta(meta)
    js, table, want = _oracle_pack(sizes, omega)
    assert m["chosen_j"] == js and m["num_charts"] == n
    c = cand.cpu().numpy()
    assert np.array_equal(c[:, 0], table[:, 0]) and np.array_equal(c[:, 2], table[:, 2])
    if js:
        assert m["layout_width"] == table[js - 1, 2] and m["layout_height"] == table[js - 1, 3]
        assert np.array_equal(pl.cpu().numpy(), want)


# ---------------------------------------------------------------------------
def test_empty_and_single_visible():
    fa = _fa()
    f = scenes.grid_frame(1)
    for vis in (np.zeros_like(f.visible), np.eye(1, f.num_triangles, 4000, dtype=np.uint8)[0]):
        f.visible = vis
        g = run_gpu(f, ctx_for())
        compare(g, oracle.build_frame(f))


def test_nofit_reported_on_device():
    f = scenes.grid_frame(2, atlas_size=16, rate=2.0)
    g = run_gpu(f, ctx_for())
    r = oracle.build_frame(f)
    assert r["status"] == oracle.STATUS_NOFIT
    compare(g, r)


def test_capacity_reported_on_device():
    f = scenes.orbit_frame(2)
    ctx = ctx_for(max_charts=8)
    g = run_gpu(f, ctx, occupancy=False)
    assert g["meta"]["status"] == _fa().FA_ERR_CAPACITY
    assert g["meta"]["num_charts"] > 8


def test_invalid_arguments_raise():
    fa = _fa()
    f = scenes.grid_frame(0)
    ctx = ctx_for()
    mesh = mesh_for(f)
    vis = torch.as_tensor(f.visible).cuda()
    for om, r in ((1000, 1.0), (16384, 1.0), (1024, 0.0), (1024, float("nan"))):
        with pytest.raises(fa.FastAtlasError) as e:
            ctx.build_atlas(mesh, vis, f.view_proj, f.width, f.height, om, r)
        assert e.value.code == fa.FA_ERR_INVALID_ARG
    bad = fa.Mesh(f.positions, np.where(f.indices == 7, 10**6, f.indices), 99123)
    with pytest.raises(fa.FastAtlasError):
        ctx.build_atlas(bad, vis, f.view_proj, f.width, f.height, 1024, 1.0)


def test_deterministic_repeats():
    f = scenes.orbit_frame(45)
    ctx = ctx_for()
    outs = [run_gpu(f, ctx) for _ in range(3)]
    for o in outs[1:]:
        for k in ("chart_of_tri", "chart_of_vert", "occupancy", "candidates"):
            assert np.array_equal(o[k], outs[0][k])
        assert np.array_equal(o["charts"], outs[0]["charts"])
        assert np.array_equal(bits(o["uv"]), bits(outs[0]["uv"]))


def test_stage_timing_one_event_per_kernel():
    fa = _fa()
    f = scenes.orbit_frame(7)
    ctx = ctx_for()
    ctx.set_stage_timing(True)
    try:
        g = run_gpu(f, ctx)
        st = ctx.stage_times()
    finally:
        ctx.set_stage_timing(False)
    assert list(st) == fa.STAGES and len(st) == 21
    assert all(v >= 0.0 for v in st.values())
    # timing changes nothing
    compare(g, oracle.build_frame(f))


def test_batch_equals_single():
    fa = _fa()
    ctx = ctx_for()
    frames = [scenes.orbit_frame(k, atlas_size=om, rate=r)
              for k, om, r in ((3, 1024, 1.0), (40, 2048, 0.5), (80, 512, 2.0))]
    mesh = mesh_for(frames[0])
    outs = [ctx.outputs(mesh, f.atlas_size) for f in frames]
    vis = [torch.as_tensor(f.visible).cuda() for f in frames]
    ctx.build_atlas_batch(mesh, [(vis[i], f.view_proj, f.width, f.height, f.atlas_size, f.rate)
                                 for i, f in enumerate(frames)], outs)
    torch.cuda.synchronize()
    for f, o in zip(frames, outs):
        compare(o.to_numpy(), oracle.build_frame(f))


def _orbit_batch_frames():
    return [scenes.orbit_frame(k, atlas_size=om, rate=r)
            for k, om, r in ((5, 1024, 1.0), (33, 2048, 0.5), (61, 512, 2.0), (90, 1024, 1.0),
                             (100, 256, 0.5), (118, 4096, 2.0))]


_MULTI = {}


def _multi_ctx():
    if "c" not in _MULTI:
        f = scenes.orbit_frame(0)
        _MULTI["c"] = _fa().Context(f.num_triangles, f.num_vertices, max_charts=8192,
                                    max_atlas=4096, max_views=4)
    return _MULTI["c"]


def test_batch_concurrent_slots():
    ctx = _multi_ctx()
    frames = _orbit_batch_frames()
    mesh = mesh_for(frames[0])
    outs = [ctx.outputs(mesh, f.atlas_size) for f in frames]
    vis = [torch.as_tensor(f.visible).cuda() for f in frames]
    print("[gpu] batch of 6 views on 4 slots", flush=True)
    ctx.build_atlas_batch(mesh, [(vis[i], f.view_proj, f.width, f.height, f.atlas_size, f.rate)
                                 for i, f in enumerate(frames)], outs)
    torch.cuda.synchronize()
    for f, o in zip(frames, outs):
        compare(o.to_numpy(), oracle.build_frame(f))


def test_batch_graph_replays():
    fa = _fa()
    ctx = _multi_ctx()
    ctx.set_tuning(fa.FA_TUNE_BATCH_GRAPH, 1)
    try:
        frames = _orbit_batch_frames()[:5]
        mesh = mesh_for(frames[0])
        outs = [ctx.outputs(mesh, f.atlas_size) for f in frames]
        vis = [torch.as_tensor(f.visible).cuda() for f in frames]
        desc = [(vis[i], f.view_proj, f.width, f.height, f.atlas_size, f.rate)
                for i, f in enumerate(frames)]
        want = [oracle.build_frame(f) for f in frames]
        other = scenes.orbit_frame(7)
        for rep in range(3):
            print(f"[gpu] batch graph replay {rep}", flush=True)
            for o in outs:  # poison every output so a stale replay cannot pass
                for t in (o.chart_of_tri, o.chart_of_vert, o.occupancy, o.candidates):
                    t.fill_(-7)
                o.uv.fill_(-7.0)
                o.charts.fill_(-7)
                o.meta.fill_(-7)
            ctx.build_atlas_batch(mesh, desc, outs)
            # eager work between replays
            g = run_gpu(other, ctx)
            junk = torch.randn(1 << 20, device="cuda").sum()
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
            for o, r in zip(outs, want):
                compare(o.to_numpy(), r)
        compare(g, oracle.build_frame(other))
    finally:
        ctx.set_tuning(fa.FA_TUNE_BATCH_GRAPH, 0)


def test_serve_mix_equals_alone():
    """Continuous batching: each request's results are identical alone and in
    the mix (many requests in flight on 4 slots, uneven sizes)."""
    import paper_2502_17712_amd as fa
    from paper_2502_17712_amd import serve
    from synth import requests as rq
    meshes_np = rq.scene_meshes()
    meshes = {k: fa.Mesh(p, t, key) for k, (p, t, key) in meshes_np.items()}
    pools = {"grid": rq.pose_pool("grid", 4, seed=1), "orbit": rq.pose_pool("orbit", 4, seed=2),
             "city": rq.pose_pool("city", 3, seed=3)}
    stream = rq.poisson_stream(5000.0, 30, pools, clients=8, seed=3)
    assert {s for (_, _, s, _, _, _) in stream} == {"grid", "orbit", "city"}
    vis = {(s, i): torch.as_tensor(pools[s][i].visible).cuda() for s in pools
           for i in range(len(pools[s]))}
    reqs = []
    for rid, (a, c, s, i, om, r) in enumerate(stream):
        pz = pools[s][i]
        reqs.append(serve.Request(rid, s, vis[(s, i)], pz.view_proj, pz.width, pz.height, om, r,
                                  arrival=a * 0.05, client=c))
    print("[gpu] serve mix of 30 requests on 4 slots", flush=True)
    srv = serve.Server(meshes, slots=4, hbm_budget=8 << 30, max_charts=8192, max_atlas=4096)
    res = {r.rid: r for r in srv.run(reqs, keep_outputs=True)}
    srv.close()
    # the mix really overlapped: some request started before another finished
    ivs = sorted((r.start, r.finish) for r in res.values())
    overlaps = sum(1 for (s0, f0), (s1, _) in zip(ivs, ivs[1:]) if s1 < f0)
    assert overlaps >= 2, ivs
    alone = fa.Context(max(m.num_triangles for m in meshes.values()),
                       max(m.num_vertices for m in meshes.values()), max_charts=8192,
                       max_atlas=4096)
    for q in reqs:
        mesh = meshes[q.scene]
        o = alone.build_atlas(mesh, q.visible, q.view_proj, q.width, q.height, q.atlas_size,
                              q.rate)
        torch.cuda.synchronize()
        a, b = o.to_numpy(), res[q.rid].out.to_numpy()
        for k in ("chart_of_tri", "chart_of_vert", "occupancy", "candidates"):
            assert np.array_equal(a[k], b[k]), (q.rid, k)
        assert np.array_equal(a["charts"], b["charts"])
        assert np.array_equal(bits(a["uv"]), bits(b["uv"]))
        assert a["meta"] == b["meta"]
    # back-pressure: a budget that holds one request at a time still serves all,
    # one after another
    small = {k: meshes[k] for k in ("grid", "orbit")}
    few = [q for q in reqs if q.scene in small][:8]
    srv = serve.Server(small, slots=4, max_charts=8192, max_atlas=4096, hbm_budget=1)
    srv.budget = max(srv.request_bytes(q) for q in few)
    out = srv.run(few)
    srv.close()
    assert sorted(r.rid for r in out) == sorted(q.rid for q in few)
    for r in out:
        assert r.meta["status"] == 0
    ivs = sorted((r.start, r.finish) for r in out)
    assert all(s1 >= f0 - 1e-3 for (_, f0), (s1, _) in zip(ivs, ivs[1:]))


def test_serve_batched_mix_equals_alone():
    """Micro-batched serving: requests that arrive together are atlased in
    batched calls of up to 6 views of one scene; each request's results,
    written into recycled output buffers full of stale values, are identical
    to the same request run alone, with precomputed and device-computed
    visible sets."""
    import paper_2502_17712_amd as fa
    from paper_2502_17712_amd import serve
    from synth import requests as rq
    meshes_np = rq.scene_meshes()
    meshes = {k: fa.Mesh(p, t, key) for k, (p, t, key) in meshes_np.items()}
    pools = {"grid": rq.pose_pool("grid", 4, seed=1), "orbit": rq.pose_pool("orbit", 4, seed=2),
             "city": rq.pose_pool("city", 3, seed=3)}
    stream = rq.poisson_stream(5000.0, 36, pools, clients=8, seed=5)
    vis = {(s, i): torch.as_tensor(pools[s][i].visible).cuda() for s in pools
           for i in range(len(pools[s]))}
    reqs = []
    for rid, (a, c, s, i, om, r) in enumerate(stream):
        pz = pools[s][i]
        # every third request leaves its visible set to the device
        reqs.append(serve.Request(rid, s, None if rid % 3 == 2 else vis[(s, i)], pz.view_proj,
                                  pz.width, pz.height, om, r, arrival=a * 0.01, client=c,
                                  eye=tuple(pz.eye), near=pz.near, coarse=pz.coarse))
    print("[gpu] micro-batched serve of 36 requests, 2 slots of 6 views", flush=True)
    srv = serve.Server(meshes, slots=2, hbm_budget=8 << 30, max_charts=8192, max_atlas=4096,
                       batch=6)
    ctx0 = srv.slots[0][0]
    for q in reqs:  # stale buffers in the pool: every output element must be rewritten
        key = (q.scene, q.atlas_size)
        if len(srv.pool[key]) < 2:
            o = ctx0.outputs(meshes[q.scene], q.atlas_size)
            for t in (o.chart_of_tri, o.chart_of_vert, o.charts, o.occupancy, o.meta,
                      o.candidates):
                t.fill_(0x5A5A5A5A)
            o.uv.fill_(1234.5)
            srv.pool[key].append(o)
    torch.cuda.synchronize()
    res = {r.rid: r for r in srv.run(reqs, keep_outputs=True)}
    srv.close()
    assert sorted(res) == [q.rid for q in reqs]
    # batches formed: several requests share a slot and a start
    groups = collections.Counter((r.slot, r.start) for r in res.values())
    assert max(groups.values()) >= 2, groups
    alone = fa.Context(max(m.num_triangles for m in meshes.values()),
                       max(m.num_vertices for m in meshes.values()), max_charts=8192,
                       max_atlas=4096)
    for q in reqs:
        mesh = meshes[q.scene]
        v = q.visible
        if v is None:
            v = alone.visibility(mesh, q.view_proj, q.width, q.height, q.eye, q.near, q.coarse)
        o = alone.build_atlas(mesh, v, q.view_proj, q.width, q.height, q.atlas_size, q.rate)
        torch.cuda.synchronize()
        a, b = o.to_numpy(), res[q.rid].out.to_numpy()
        for k in ("chart_of_tri", "chart_of_vert", "occupancy", "candidates"):
            assert np.array_equal(a[k], b[k]), (q.rid, k)
        assert np.array_equal(a["charts"], b["charts"]), q.rid
        assert np.array_equal(bits(a["uv"]), bits(b["uv"])), q.rid
        # the meta read from pinned host memory is the output's own record
        assert a["meta"] == b["meta"] == res[q.rid].meta, q.rid
    alone.close()


@pytest.mark.parametrize("link,hooks", [(0, 0), (0, 1), (0, 2), (0, 3), (0, 4), (0, 5), (1, 0),
                                        (1, 1), (1, 2), (1, 3), (1, 4), (1, 5)])
def test_union_find_modes_all_combinations(link, hooks):
    """Every (start link, edge-hook mode) pair gives the oracle's charts, frame
    after frame (the charts do not depend on how the union-find gets there)."""
    ctx = ctx_for()
    old = (ctx.get_tuning(3), ctx.get_tuning(5))
    ctx.set_tuning(3, link)
    ctx.set_tuning(5, hooks)
    try:
        for fr in (0, 16):
            f = scenes.city_frame(fr)
            r = oracle.build_frame(f, want_occupancy=False)
            for rep in range(3):
                g = run_gpu(f, ctx, occupancy=False)
                assert np.array_equal(g["chart_of_tri"], r["chart_of_tri"]), (fr, rep)
                assert np.array_equal(g["chart_of_vert"], r["chart_of_vert"]), (fr, rep)
    finally:
        ctx.set_tuning(3, old[0])
        ctx.set_tuning(5, old[1])


def _bowtie_frame():
    """The 8k grid with every corner a vertex of its own, except that the two
    triangles of each grid quad keep one common vertex: charts are bowtie
    pairs joined only through a vertex, and a tile of 2048 visible triangles
    names about 5120 distinct vertices, more than the 4096 slots of the
    vertex-hashed tile pass, so some references overflow its table."""
    f = scenes.grid_frame(4, atlas_size=2048)
    tris = f.indices
    T = tris.shape[0]
    ind = np.arange(3 * T, dtype=np.int32).reshape(T, 3)
    for k in range(0, T - 1, 2):
        common = [c for c in tris[k] if c in tris[k + 1]]
        if common:
            ca = int(np.flatnonzero(tris[k] == common[0])[0])
            cb = int(np.flatnonzero(tris[k + 1] == common[0])[0])
            ind[k + 1, cb] = ind[k, ca]
    f.positions = np.ascontiguousarray(f.positions[tris.reshape(-1)])
    f.indices = ind
    f.scene_key = 4242
    f.name = "grid8k-bowties"
    return f


@pytest.mark.parametrize("hooks", [0, 1, 2, 3, 4, 5])
def test_union_find_vertex_only_charts(hooks):
    """Charts joined only through a vertex, with more distinct vertices per
    tile than the vertex-hashed tile table holds, in every hook mode."""
    f = _bowtie_frame()
    r = oracle.build_frame(f)
    assert r["num_charts"] < int(np.count_nonzero(f.visible))  # pairs did merge
    ctx = ctx_for()
    old = ctx.get_tuning(5)
    ctx.set_tuning(5, hooks)
    try:
        g = run_gpu(f, ctx)
        compare(g, r)
    finally:
        ctx.set_tuning(5, old)


# ---------------------------------------------------------------------------
# footprint-aware push
# ---------------------------------------------------------------------------
FP = 4  # FA_FLAG_FOOTPRINT_PUSH


def _fp_frame(kind, k, omega, rate):
    if kind == "grid":
        return scenes.grid_frame(k, atlas_size=omega, rate=rate)
    if kind == "orbit":
        return scenes.orbit_frame(k, atlas_size=omega, rate=rate)
    if kind == "scatter":  # 6000 boxes: several thousand charts, the many-chart order
        return scenes.scatter_frame(k, rate=rate, atlas_size=omega, count=6000)
    return scenes.city_frame(k, rate=rate, atlas_size=omega)


@pytest.mark.parametrize("kind,k,omega,rate", [("grid", 3, 256, 1.0), ("grid", 11, 512, 2.0),
                                               ("grid", 20, 1024, 1.0), ("orbit", 20, 512, 1.0),
                                               ("orbit", 77, 2048, 1.0), ("city", 5, 4096, 1.0),
                                               ("city", 9, 2048, 2.0), ("scatter", 2, 4096, 1.0)])
def test_footprint_push(kind, k, omega, rate):
    f = _fp_frame(kind, k, omega, rate)
    g = run_gpu(f, ctx_for(flags=FP))
    r = oracle.build_frame(f, footprint=True)
    compare(g, r)
    assert r["occupancy_conflicts"] == 0


@pytest.mark.parametrize("J,gutter,omega,rate", [(16, 2, 256, 1.0), (32, 1, 1024, 2.0),
                                                 (64, 3, 128, 0.5)])
def test_footprint_variants(J, gutter, omega, rate):
    f = scenes.grid_frame(9, atlas_size=omega, rate=rate)
    g = run_gpu(f, ctx_for(J=J, gutter=gutter, flags=FP))
    compare(g, oracle.build_frame(f, J=J, gutter=gutter, footprint=True))


def test_footprint_empty_frame_and_batch():
    fa = _fa()
    ctx = ctx_for(flags=FP)
    f = scenes.grid_frame(2, atlas_size=512)
    mesh = mesh_for(f)
    # nothing visible: no charts, the largest scale
    none = torch.zeros(f.num_triangles, dtype=torch.uint8, device="cuda")
    out = ctx.outputs(mesh, 512)
    ctx.build_atlas(mesh, none, f.view_proj, f.width, f.height, 512, 1.0, out=out)
    torch.cuda.synchronize()
    m = fa.parse_meta(out.meta)
    assert m["status"] == 0 and m["num_charts"] == 0 and m["chosen_j"] == 64
    # views of a batch (one mesh) equal the single-frame results
    frames = [scenes.orbit_frame(k, atlas_size=512) for k in (5, 40, 90)]
    mesh = mesh_for(frames[0])
    vis = [torch.as_tensor(x.visible).cuda() for x in frames]
    outs = [ctx.outputs(mesh, 512) for _ in frames]
    ctx.build_atlas_batch(mesh, [(v, x.view_proj, x.width, x.height, 512, 1.0)
                                 for v, x in zip(vis, frames)], outs)
    torch.cuda.synchronize()
    for x, o in zip(frames, outs):
        compare(o.to_numpy(), oracle.build_frame(x, footprint=True))


def test_footprint_capacity_many_charts():
    # the profile-column total above the capacity, found by the many-chart
    # order (its last workgroup sums every chunk)
    fa = _fa()
    f = _fp_frame("scatter", 4, 4096, 1.0)
    assert oracle.build_frame(f)["num_charts"] > 1024
    ctx = fa.Context(f.num_triangles, f.num_vertices, max_charts=65536, max_atlas=4096, flags=FP,
                     max_profile_columns=2000, tuning_table=None)
    g = run_gpu(f, ctx)
    assert g["meta"]["status"] == fa.FA_ERR_CAPACITY
    ctx.close()


def test_footprint_capacity_and_dual_rejected():
    fa = _fa()
    f = scenes.grid_frame(6, atlas_size=512)
    small = fa.Context(10_000, 5_000, max_charts=4096, max_atlas=1024, flags=FP,
                       max_profile_columns=8)
    g = run_gpu(f, small)
    assert g["meta"]["status"] == fa.FA_ERR_CAPACITY
    mesh = mesh_for(f)
    vis = torch.as_tensor(f.visible).cuda()
    with pytest.raises(fa.FastAtlasError):
        small.build_dual_atlas(mesh, vis, f.view_proj, f.width, f.height, 512, 1.0, 1)
