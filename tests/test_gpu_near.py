"""GPU parity on frames whose visible triangles cross the near plane.

The near plane is the special case of the box step (Sec. "Computing Bounding
Boxes of Projected Visible Sub-Charts"; App. "Bounding Box Computation
Alternatives"): a triangle that crosses it is clipped there before Blinn's
divide, its occupancy is the near-clipped polygon (a triangle or a quad)
fanned from its first vertex, its footprint profile is that polygon's, and a
vertex behind the eye (w <= 0) has no UV (NaN). Each case first counts the
near-crossing visible triangles, so a pass proves the branch ran. Same bar as
test_gpu_parity: integers and float bits exact, UVs within 1e-4 texels with
the NaN pattern equal.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import scenes
from tests.test_gpu_parity import FP, compare, ctx_for, mesh_for, run_gpu

pytestmark = pytest.mark.gpu


def _near_counts(f):
    M = f.view_proj.astype(np.float32).reshape(4, 4)
    p = f.positions
    c = np.stack([((M[i, 0] * p[:, 0] + M[i, 1] * p[:, 1]) + M[i, 2] * p[:, 2]) + M[i, 3]
                  for i in range(4)], 1)
    dn = (c[:, 3] + c[:, 2])[f.indices]
    vis = f.visible.astype(bool)
    behind = (dn < 0).sum(1)
    return (int((vis & (behind == 1)).sum()), int((vis & (behind == 2)).sum()),
            int((vis & (c[f.indices, 3] <= 0).any(1)).sum()))


def _frame(kind, k, omega, rate):
    if kind == "grid":
        return scenes.grid_near_frame(k, atlas_size=omega, rate=rate)
    if kind == "floor":
        return scenes.floor_near_frame(k, atlas_size=omega, rate=rate)
    return scenes.city_near_frame(k, rate=rate, atlas_size=omega)


CASES = ([("grid", s, 1024, 1.0) for s in range(8)] +
         [("grid", 2, 512, 0.5), ("grid", 5, 2048, 2.0)] +
         [("floor", s, 512, 1.0) for s in range(8)] +
         [("city", k, 4096, 1.0) for k in (0, 8, 16, 24)] + [("city", 8, 4096, 2.0)])


@pytest.mark.parametrize("kind,k,omega,rate", CASES)
def test_near_frames(kind, k, omega, rate):
    f = _frame(kind, k, omega, rate)
    quads, tris, behind = _near_counts(f)
    print(f"  near crossers: {quads} quads, {tris} triangles, {behind} with w <= 0", flush=True)
    assert quads + tris > 0
    if kind in ("floor", "city"):
        assert behind > 0 or kind == "floor"
    g = run_gpu(f, ctx_for())
    r = oracle.build_frame(f)
    compare(g, r)
    # the vertices behind the eye of visible triangles: NaN on both sides
    clip = r["clip"]
    nan_rule = (r["chart_of_vert"] >= 0) & (clip[:, 3] <= 0)
    assert np.isnan(g["uv"][nan_rule]).all()


@pytest.mark.parametrize("kind,k,omega,rate", [("grid", 1, 1024, 1.0), ("grid", 4, 512, 0.5),
                                               ("floor", 2, 512, 1.0), ("floor", 7, 256, 2.0),
                                               ("city", 0, 4096, 1.0), ("city", 16, 2048, 2.0)])
def test_near_frames_footprint_push(kind, k, omega, rate):
    f = _frame(kind, k, omega, rate)
    assert sum(_near_counts(f)[:2]) > 0
    g = run_gpu(f, ctx_for(flags=FP))
    r = oracle.build_frame(f, footprint=True)
    compare(g, r)
    assert r["occupancy_conflicts"] == 0


@pytest.mark.parametrize("kind,k", [("grid", 3), ("floor", 1), ("city", 24)])
def test_near_frames_no_side_clip(kind, k):
    f = _frame(kind, k, 1024 if kind != "city" else 4096, 1.0)
    g = run_gpu(f, ctx_for(flags=1))
    compare(g, oracle.build_frame(f, side_clip=False))


def test_near_frame_dual_atlas():
    import paper_2502_17712_amd as fa
    f = scenes.grid_near_frame(6, atlas_size=1024)
    ctx = ctx_for(gutter=4)
    mesh = mesh_for(f)
    vis = torch.as_tensor(f.visible).cuda()
    out, low = ctx.build_dual_atlas(mesh, vis, f.view_proj, f.width, f.height, 1024, 1.0, 2)
    torch.cuda.synchronize()
    r = oracle.build_frame(f, gutter=4, low_shift=2)
    compare(out.to_numpy(), r)
    assert np.array_equal(low.cpu().numpy(), r["occupancy_low"])
    assert fa.parse_meta(out.meta)["status"] == 0
