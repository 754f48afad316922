"""Benchmark of the per-frame atlasing hot path on one MI355X.

Workload (one step = one frame atlased end to end: clip, charts, boxes,
order, 64-candidate packing, selection, UVs, occupancy): the seeded
~2.2M-triangle scene (terrain + 400 displaced spheres, boxes, cylinders),
3840x2160 view on a 32-frame yaw orbit, frustum + backface + coarse
depth-buffer occlusion, 4096^2 atlas, 1.0 texel/pixel. Inputs (mesh,
visible sets) are resident in HBM before timing; the per-scene adjacency is
built once and timed separately.

Prints one JSON line (rank 0). See the design doc for the roofline accounting.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atlas ms/frame (2M tris, 4K view); batched views/s vs plain; p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(T, V, Tv, Vv, C, J, omega):
    """Bytes the method must move per frame (inputs read once, outputs written once)."""
    return (T * 1 + Tv * (12 + 12) + Vv * 12 + T * 4 + V * 4 + V * 8 + C * 64 + J * C * 16
            + omega * omega * 4)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--frames", type=int, default=32, help="distinct orbit frames")
    ap.add_argument("--rate", type=float, default=1.0)
    ap.add_argument("--atlas", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2502_17712_amd as fa
    from synth import scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t0 = time.time()
    pos, tris = scenes.city_scene()
    frames = [scenes.city_frame(f, rate=args.rate, atlas_size=args.atlas)
              for f in range(0, 32, max(1, 32 // args.frames))][: args.frames]
    log(f"generated {len(frames)} frames in {time.time() - t0:.1f}s; T={tris.shape[0]} "
        f"V={pos.shape[0]}")
    T, V = tris.shape[0], pos.shape[0]
    ctx = fa.Context(T, V, max_charts=65536, max_atlas=args.atlas)
    mesh = fa.Mesh(pos, tris, frames[0].scene_key)
    vis = [torch.as_tensor(f.visible).to(dev) for f in frames]
    out = ctx.outputs(mesh, args.atlas)
    stream = torch.cuda.current_stream()

    # per-scene adjacency (resident afterwards), timed on its own
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.adjacency(mesh)
    e1.record(stream)
    torch.cuda.synchronize()
    adjacency_ms = e0.elapsed_time(e1)

    def step(k):
        f = frames[k % len(frames)]
        ctx.build_atlas(mesh, vis[k % len(frames)], f.view_proj, f.width, f.height,
                        f.atlas_size, f.rate, out=out, stream=stream)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        step(k)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    per = np.array([a.elapsed_time(b) for a, b in evs])
    meta = fa.parse_meta(out.meta)
    assert meta["status"] == fa.FA_OK, meta

    # per-stage breakdown (separate pass with stage events)
    ctx.set_stage_timing(True)
    stage_acc = {}
    for k in range(min(64, args.steps)):
        step(k)
        torch.cuda.synchronize()
        for name, ms in ctx.stage_times().items():
            stage_acc.setdefault(name, []).append(ms)
    ctx.set_stage_timing(False)
    stages = {k: float(np.mean(v)) for k, v in stage_acc.items()}

    # frame statistics for the roofline accounting
    stats = []
    for k, f in enumerate(frames):
        step(k)
        torch.cuda.synchronize()
        m = fa.parse_meta(out.meta)
        used = np.zeros(V, bool)
        used[tris[f.visible.astype(bool)].ravel()] = True
        stats.append((int(f.visible.sum()), int(used.sum()), m["num_charts"]))
    Tv, Vv, C = (float(np.mean([s[i] for s in stats])) for i in range(3))
    B = algorithmic_bytes(T, V, Tv, Vv, C, 64, args.atlas)

    # batched views vs the plain per-view path
    batch = None
    if not args.no_batch:
        views = scenes.batch_views(16)
        bouts = [ctx.outputs(mesh, v.atlas_size) for v in views]
        bvis = [torch.as_tensor(v.visible).to(dev) for v in views]
        desc = [(bvis[i], v.view_proj, v.width, v.height, v.atlas_size, v.rate)
                for i, v in enumerate(views)]
        for _ in range(2):
            ctx.build_atlas_batch(mesh, desc, bouts, stream=stream)
        torch.cuda.synchronize()
        reps = 10
        w1 = time.perf_counter()
        for _ in range(reps):
            ctx.build_atlas_batch(mesh, desc, bouts, stream=stream)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - w1) / reps
        w2 = time.perf_counter()
        for _ in range(reps):
            for i, v in enumerate(views):
                ctx.build_atlas(mesh, bvis[i], v.view_proj, v.width, v.height, v.atlas_size,
                                v.rate, out=bouts[i], stream=stream)
        torch.cuda.synchronize()
        tp = (time.perf_counter() - w2) / reps
        batch = dict(views=16, batched_views_per_s=16 / tb, plain_views_per_s=16 / tp,
                     speedup=tp / tb)

    # CPU oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        n = max(1, args.cpu_frames)
        c0 = time.perf_counter()
        for f in frames[:n]:
            oracle.build_frame(f)
        cms = (time.perf_counter() - c0) / n * 1e3
        cpu = dict(value=cms, unit="ms/frame", cores=1, kind="oracle",
                   sample=f"{n} frames of the same workload, single-threaded C++ oracle",
                   host_cpu=platform.processor() or platform.machine(), nproc=os.cpu_count())

    ms = float(per.mean())
    res = {
        "metric": METRIC,
        "value": ms,
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+i32",
        "data": "synthetic (seeded scene generator)",
        "config": {"workload": "city2m_3840x2160_atlas4096_rate1", "triangles": T,
                   "vertices": V, "frames": len(frames), "atlas": args.atlas, "rate": args.rate,
                   "num_scales": 64, "visible_tris_mean": Tv, "charts_mean": C},
        "p50_ms": float(np.percentile(per, 50)),
        "p99_ms": float(np.percentile(per, 99)),
        "frames_per_s": 1e3 / ms,
        "triangles_per_s": T / (ms * 1e-3),
        "adjacency_ms": adjacency_ms,
        "stages_ms": stages,
        "algorithmic_bytes_per_frame": B,
        "frame_hbm_roofline_frac": B / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "batch": batch,
        "cpu_baseline": cpu,
        "roofline": None,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
