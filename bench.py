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
import gc
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
HERE = os.path.dirname(os.path.abspath(__file__))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(T, V, Tv, Vv, C, J, omega):
    """Bytes the method must move per frame (inputs read once, outputs written once)."""
    return (T * 1 + Tv * (12 + 12) + Vv * 12 + T * 4 + V * 4 + V * 8 + C * 64 + J * C * 16
            + omega * omega * 4)


def kernel_bytes(name, T, V, Tv, Vv, C, J, omega, occupied):
    """Algorithmic bytes of one launch of a kernel (what it must read and write
    at minimum); the per-unit figures are listed in the design doc."""
    per = {
        "prologue": V * (4 + 4) + T * (1 + 4),
        "vis_compact": T * 1 + Tv * 4,
        "uf_hook": Tv * (4 + 12 + 3 + 4),
        "uf_vertex_min": Tv * (4 + 4 + 12 + 12),
        "uf_vertex_hook": Tv * (4 + 12 + 12 + 4),
        "uf_flatten": Tv * (4 + 4 + 4),
        "assign_roots": Tv * (4 + 4) + C * (4 + 4 + 16),
        "gather_boxes": Tv * (4 + 4 + 4 + 12 + 36 + 12) + C * 16,
        "sizes_order": C * (16 + 64 + 8 + 16),
        "pack": J * C * (8 + 16),
        "select_place": C * (16 + 16),
        "uv": V * (4 + 8) + Vv * 12 + C * 64,
        "occ_fill": omega * omega * 4,
        "occ_small": Tv * (4 + 4 + 12 + 36) + occupied * 4,
        # the two occupancy raster kernels are one job split by footprint size:
        # geometry of every visible triangle read once, every covered texel
        # written once; the small-footprint launch also computes the UVs
        # (chart of every vertex read, UV of every vertex written, position
        # of every vertex with a chart read, chart records read)
        "occ_small+occ_big": Tv * (4 + 4 + 12 + 36) + occupied * 4
                             + V * (4 + 8) + Vv * 12 + C * 64,
        "occ_raster_only": Tv * (4 + 4 + 12 + 36) + occupied * 4,
        "occ_count": omega * omega * 4,
    }
    return per.get(name)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current sources of that kernel; else None."""
    import hashlib
    path = os.path.join(HERE, "profiles", "traffic_occ_raster_city4k.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel") != kernel:
        return None
    for name in ("k_raster.hip", "fa_internal.h"):
        src = os.path.join(HERE, "paper_2502_17712_amd", "csrc", name)
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != fields.get(f"sha256 {name}"):
            return None
    return float(fields["hbm_bytes_per_launch"])


def rocprof_kernel_ms(kernel):
    """Average duration (ms) of `kernel` from the committed rocprofv3 kernel
    trace of the bench workload, if it was taken on the current sources; the
    two occupancy raster kernels are summed. None otherwise."""
    import hashlib
    path = os.path.join(HERE, "profiles", "kernels_city2m_4k_atlas4096.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    for line in txt.splitlines():
        if line.startswith("- sha256 "):
            name, digest = line[len("- sha256 "):].split(":", 1)
            src = os.path.join(HERE, "paper_2502_17712_amd", "csrc", name.strip())
            if (not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest()
                    != digest.strip().strip("`")):
                return None
    names = {"occ_small+occ_big": ("k_occ_small", "k_occ_big")}.get(kernel, ("k_" + kernel,))
    total = 0.0
    for n in names:
        hit = None
        for line in txt.splitlines():
            cells = [c.strip().strip("`") for c in line.split("|")]
            if len(cells) > 3 and cells[1].startswith(n) and (cells[1] == n or
                                                             cells[1].startswith(n + "<")):
                try:
                    hit = float(cells[3]) * 1e-3  # average, microseconds
                except ValueError:
                    pass
                break
        if hit is None:
            return None
        total += hit
    return total


def dependent_phases(ctx, fa):
    """Kernel launches of one frame (box push, with occupancy): the 21 timing
    stages minus the ones this configuration leaves empty."""
    hooks = ctx.get_tuning(fa.FA_TUNE_UF_EDGE_HOOKS)
    n = 21 - 4  # visible-count and root-count scans folded in; no footprint stages
    n -= 3  # UVs, occupancy fill and frame record run inside other launches
    n -= 1 if hooks >= 4 else 0  # vertex minima lowered by the tile kernel
    n += 1 if hooks == 2 else 0  # tile kernel and cross-tile hooks share a stage
    n -= 1 if hooks == 0 else 0  # no edge-hook kernel
    return n


def extras(args, ctx, mesh, frames, vis, out, stream, dev, T):
    """No-occupancy frame time, device copy bandwidth, the device visibility
    pass and temporal reuse on the benchmark frames."""
    import torch

    # the same frames without the occupancy output (UVs and placements only)
    out_nocc = ctx.outputs(mesh, args.atlas, occupancy=False)
    for k in range(8):
        f = frames[k % len(frames)]
        ctx.build_atlas(mesh, vis[k % len(frames)], f.view_proj, f.width, f.height,
                        f.atlas_size, f.rate, out=out_nocc, stream=stream)
    evn = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(len(frames) * 2)]
    for k, (a_, b_) in enumerate(evn):
        f = frames[k % len(frames)]
        a_.record(stream)
        ctx.build_atlas(mesh, vis[k % len(frames)], f.view_proj, f.width, f.height,
                        f.atlas_size, f.rate, out=out_nocc, stream=stream)
        b_.record(stream)
    torch.cuda.synchronize()
    ms_nocc = float(np.mean([a_.elapsed_time(b_) for a_, b_ in evn]))
    del out_nocc

    # plain device copy bandwidth on this GPU (context for the roofline)
    cpa = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    cpb = torch.empty_like(cpa)
    cpa.fill_(1)
    cpb.copy_(cpa)
    c0_, c1_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0_.record(stream)
    for _ in range(5):
        cpb.copy_(cpa)
    c1_.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * cpa.numel() / (c0_.elapsed_time(c1_) * 1e-3) / 1e9
    del cpa, cpb

    # the visible-triangle pass on the device (coarse depth buffer), alone and
    # followed by the atlas of the same frame
    vbuf = torch.empty(T, dtype=torch.uint8, device=dev)
    for f in frames[:4]:
        ctx.visibility(mesh, f.view_proj, f.width, f.height, f.eye, f.near, f.coarse, out=vbuf,
                       stream=stream)
    torch.cuda.synchronize()
    evv = []
    for k in range(len(frames) * 2):
        f = frames[k % len(frames)]
        a_, m_, b_ = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        a_.record(stream)
        ctx.visibility(mesh, f.view_proj, f.width, f.height, f.eye, f.near, f.coarse, out=vbuf,
                       stream=stream)
        m_.record(stream)
        ctx.build_atlas(mesh, vbuf, f.view_proj, f.width, f.height, f.atlas_size, f.rate,
                        out=out, stream=stream)
        b_.record(stream)
        evv.append((a_, m_, b_))
    torch.cuda.synchronize()
    visibility = dict(coarse=frames[0].coarse,
                      visibility_ms=float(np.mean([a_.elapsed_time(m_) for a_, m_, _ in evv])),
                      visibility_plus_atlas_ms=float(np.mean([a_.elapsed_time(b_)
                                                              for a_, _, b_ in evv])))
    assert torch.equal(vbuf.cpu(), torch.as_tensor(frames[(len(evv) - 1) % len(frames)].visible))
    del vbuf

    # temporal reuse over the frame sequence, a key frame every 10 frames
    fr_re, ms_re = [], []
    for k in range(len(frames)):
        if k % 10 == 0:
            key_f, key_v = frames[k], vis[k]
            continue
        a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a_.record(stream)
        _, reused_ = ctx.reuse_flags(mesh, key_f.view_proj, key_v, vis[k], stream=stream)
        b_.record(stream)
        torch.cuda.synchronize()
        ms_re.append(a_.elapsed_time(b_))
        fr_re.append(int(reused_.item()) / max(1, int(frames[k].visible.sum())))
    reuse = dict(key_interval=10, mean_reused_fraction=float(np.mean(fr_re)) if fr_re else None,
                 min_reused_fraction=float(np.min(fr_re)) if fr_re else None,
                 flags_ms=float(np.mean(ms_re)) if ms_re else None)
    return ms_nocc, copy_gbs, visibility, reuse


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(args, frames):
    """Time the oracle (test infrastructure, single-threaded C++) on this
    host, pinned to one core: the 64 grid seeds, the 120 orbit frames and
    four city frames at rates 0.5, 1 and 2 (frames 0, 8, 16, 24 of the
    orbit; the city frames of the timed workload, re-rated)."""
    import dataclasses

    import oracle
    from synth import scenes
    oracle.lib()  # built and loaded before the clock starts
    allowed = os.sched_getaffinity(0)
    core = min(allowed)
    os.sched_setaffinity(0, {core})  # this thread only: the oracle runs in it

    def run(frs):
        ts = []
        for f in frs:
            c0 = time.perf_counter()
            oracle.build_frame(f)
            ts.append((time.perf_counter() - c0) * 1e3)
        return dict(mean_ms=float(np.mean(ts)), p50_ms=float(np.median(ts)), frames=len(ts))
    try:
        per = {}
        per["grid8k_1280x720_atlas1024"] = run([scenes.grid_frame(k) for k in range(64)])
        per["orbit86k_1920x1080_atlas2048"] = run([scenes.orbit_frame(k) for k in range(120)])
        base = {f.name: f for f in frames}
        city = [base.get(f"city2m/s2f{k}") or scenes.city_frame(k, atlas_size=args.atlas)
                for k in (0, 8, 16, 24)]
        for r_ in (0.5, 1.0, 2.0):
            per[f"city2m_3840x2160_atlas{args.atlas}_rate{r_:g}"] = run(
                [dataclasses.replace(f, rate=r_) for f in city])
    finally:
        os.sched_setaffinity(0, allowed)
    main_key = f"city2m_3840x2160_atlas{args.atlas}_rate{args.rate:g}"
    value = per[main_key]["mean_ms"] if main_key in per else None
    return dict(value=value, unit="ms/frame", cores=1, kind="oracle",
                sample=("oracle pinned to one core: 64 grid seeds, 120 orbit frames, city frames "
                        "0/8/16/24 at rates 0.5/1/2; value = the city frames at the bench rate"),
                per_workload=per, pinned_core=core, host_cpu=host_cpu_model(),
                nproc=os.cpu_count())


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
    ap.add_argument("--autotune", action="store_true",
                    help="tune the knobs per workload first and write a tuning table "
                         "(default: the committed table)")
    ap.add_argument("--tune-out", default="tuning_table.txt",
                    help="where --autotune writes the table it found")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-dual", action="store_true")
    ap.add_argument("--no-footprint", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the no-occupancy, copy, visibility and reuse measurements")
    ap.add_argument("--serve-rate", type=float, nargs="+",
                    default=[60.0, 250.0, 1000.0, 2000.0, 5000.0, 10000.0, 20000.0, 50000.0])
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run 4 plain device copies of 256 MiB (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel(), "copies": 4}))
        return
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2502_17712_amd as fa
    TUNED = (fa.FA_TUNE_OCC_SMALL_TEXELS, fa.FA_TUNE_OCC_LANE_TEXELS, fa.FA_TUNE_UF_LINK_INIT,
             fa.FA_TUNE_UF_EDGE_HOOKS, fa.FA_TUNE_PACK_BLOCK, fa.FA_TUNE_UF_TILE)
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

    tuning = None
    if args.autotune:
        # greedy search per frame shape (the small, medium and large workloads)
        # with the loaded table cleared; writes a tuning table
        from paper_2502_17712_amd import autotune
        ctx.load_tuning_table("")
        lines, tuning = [], {}

        defaults = {k: ctx.get_tuning(k) for k in autotune.KNOBS}

        def tune_on(name, ctx_, mesh_, frs, out_):
            for k, v in defaults.items():  # every search starts from the library defaults
                ctx_.set_tuning(k, v)
            vs = [torch.as_tensor(f.visible).to(dev) for f in frs]
            cyc = [0]

            def one(k):
                f = frs[k % len(frs)]
                ctx_.build_atlas(mesh_, vs[k % len(frs)], f.view_proj, f.width, f.height,
                                 f.atlas_size, f.rate, out=out_, stream=stream)

            def tune_step():  # every trial sees the same spread of frames
                one(cyc[0])
                cyc[0] += 1
            rep = autotune.tune(ctx_, tune_step, out_, reps=max(len(frs), 16),
                                ref_run=lambda: one(0))
            tuning[name] = rep
            log("autotune:", name, json.dumps(rep["choice"]))
            return rep["choice"]
        g0, o0 = scenes.grid_frame(0), scenes.orbit_frame(0)
        gctx = fa.Context(o0.num_triangles, o0.num_vertices, max_charts=65536, max_atlas=4096,
                          tuning_table=None)
        gmesh = fa.Mesh(g0.positions, g0.indices, g0.scene_key)
        ch = tune_on("grid8k", gctx, gmesh, [g0], gctx.outputs(gmesh, 1024))
        lines.append(autotune.table_line(0, 20000, 0, 64, ch, "8k-triangle grid, 1024^2"))
        omesh = fa.Mesh(o0.positions, o0.indices, o0.scene_key)
        ofr = [scenes.orbit_frame(k) for k in range(0, 120, 15)]
        ch = tune_on("orbit86k", gctx, omesh, ofr, gctx.outputs(omesh, 2048))
        lines.append(autotune.table_line(20001, 150000, 0, 64, ch, "86k-triangle orbit, 2048^2"))
        gctx.close()
        # the many-chart workload (24,000 boxes, ~23k charts per frame)
        s0 = scenes.scatter_frame(0)
        smesh = fa.Mesh(s0.positions, s0.indices, s0.scene_key)
        sfr = [scenes.scatter_frame(k) for k in range(0, 16, 2)]
        ch = tune_on("scatter288k", ctx, smesh, sfr, ctx.outputs(smesh, 4096))
        lines.append(autotune.table_line(150001, 500000, 0, 64, ch,
                                         "288k-triangle scatter, ~23k charts, 4096^2"))
        ch = tune_on("city2m", ctx, mesh, frames, out)
        lines.append(autotune.table_line(500001, 1 << 30, 0, 64, ch,
                                         "2.2M-triangle city, 4096^2"))
        text = autotune.table_text(lines, "written by bench.py --autotune on one MI355X")
        out_dir = os.path.dirname(os.path.abspath(args.tune_out))
        os.makedirs(out_dir, exist_ok=True)
        with open(args.tune_out, "w") as fh:
            fh.write(text)
        ctx.load_tuning_table(text)
        log("tuning table:\n" + text)
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

    ms_nocc = copy_gbs = visibility = reuse = None
    if not args.no_extras:
        ms_nocc, copy_gbs, visibility, reuse = extras(args, ctx, mesh, frames, vis, out, stream,
                                                      dev, T)

    # per-kernel live times (separate pass with an event after every kernel)
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
    occupied = float(meta["occupied_texels"])
    # the dominant kernel; the two occupancy raster kernels count as one
    timed = {k: v for k, v in stages.items() if k not in ("occ_small", "occ_big")}
    if "occ_small" in stages:
        timed["occ_small+occ_big"] = stages["occ_small"] + stages.get("occ_big", 0.0)
    dom = max(timed, key=timed.get) if timed else None
    roofline = None
    if dom is not None:
        kb = kernel_bytes(dom, T, V, Tv, Vv, C, 64, args.atlas, occupied)
        ach = kb / (timed[dom] * 1e-3) / 1e9 if kb else None
        rp = rocprof_kernel_ms(dom)
        roofline = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": (ach / HBM_PEAK_GBS) if ach else None,
                    "traffic": measured_traffic(dom), "kernel_ms": timed[dom],
                    "time_basis": ("HIP events on the launch stream before and after each "
                                   "kernel, stage-timing pass over the timed frames"),
                    "algorithmic_bytes": kb,
                    "rocprof_kernel_ms": rp,
                    "frac_rocprof": (kb / (rp * 1e-3) / 1e9 / HBM_PEAK_GBS) if (kb and rp)
                    else None}
        if dom == "occ_small+occ_big":
            # the same launches priced on the raster's own bytes (without the
            # UVs that run in the small-footprint launch's spare workgroups)
            kr = kernel_bytes("occ_raster_only", T, V, Tv, Vv, C, 64, args.atlas, occupied)
            roofline["raster_only_algorithmic_bytes"] = kr
            roofline["raster_only_frac"] = kr / (timed[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS

    # secondary workloads: the small and medium scenes, other rates on the large one
    def time_frames(ctx_, mesh_, frs, reps=3):
        """mesh_: one mesh for every frame, or one per frame. A warm-up pass
        over all frames (adjacency built, caches warm), then `reps` timed
        passes."""
        ms_ = mesh_ if isinstance(mesh_, list) else [mesh_] * len(frs)
        vs = [torch.as_tensor(f.visible).to(dev) for f in frs]
        outs_ = {om: ctx_.outputs(ms_[0], om) for om in {f.atlas_size for f in frs}}
        for m_, f, v in zip(ms_, frs, vs):
            ctx_.build_atlas(m_, v, f.view_proj, f.width, f.height, f.atlas_size, f.rate,
                             out=outs_[f.atlas_size], stream=stream)
        torch.cuda.synchronize()
        # events made beforehand and the garbage collector held off: a
        # collection pass inside the timed loop stalls the host between an
        # event and the frame's launches, and the GPU waits idle
        ts = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps * len(frs))]
        gc.collect()
        gc.disable()
        try:
            for rep in range(reps):
                for k, (m_, f, v) in enumerate(zip(ms_, frs, vs)):
                    a, b = ts[rep * len(frs) + k]
                    a.record(stream)
                    ctx_.build_atlas(m_, v, f.view_proj, f.width, f.height, f.atlas_size,
                                     f.rate, out=outs_[f.atlas_size], stream=stream)
                    b.record(stream)
            torch.cuda.synchronize()
        finally:
            gc.enable()
        per_ = np.array([a.elapsed_time(b) for a, b in ts])
        return dict(mean_ms=float(per_.mean()), p50_ms=float(np.percentile(per_, 50)),
                    p99_ms=float(np.percentile(per_, 99)), max_ms=float(per_.max()),
                    frames=len(frs))
    secondary = {}
    if not args.no_secondary:
        sctx = fa.Context(T, V, max_charts=65536, max_atlas=4096)
        for knob_ in TUNED:
            sctx.set_tuning(knob_, ctx.get_tuning(knob_))
        gfr = [scenes.grid_frame(s) for s in range(64)]  # every seed is its own mesh
        secondary["grid8k_1280x720_atlas1024"] = time_frames(
            sctx, [fa.Mesh(g.positions, g.indices, g.scene_key) for g in gfr], gfr)
        o0 = scenes.orbit_frame(0)
        secondary["orbit86k_1920x1080_atlas2048"] = time_frames(
            sctx, fa.Mesh(o0.positions, o0.indices, o0.scene_key),
            [scenes.orbit_frame(k) for k in range(120)])
        for r_ in (0.5, 2.0):
            secondary[f"city2m_3840x2160_atlas4096_rate{r_}"] = time_frames(
                ctx, mesh, [scenes.city_frame(k, rate=r_) for k in range(0, 32, 8)])
        # many charts: ordering and packing at ~20k charts per frame
        sfr = [scenes.scatter_frame(k) for k in range(8)]
        smesh = fa.Mesh(sfr[0].positions, sfr[0].indices, sfr[0].scene_key)
        res_sc = time_frames(sctx, smesh, sfr)
        sv = [torch.as_tensor(f.visible).to(dev) for f in sfr]
        sout = sctx.outputs(smesh, 4096)
        sctx.set_stage_timing(True)
        st_acc, charts_ = {}, []
        for f, v in zip(sfr, sv):
            sctx.build_atlas(smesh, v, f.view_proj, f.width, f.height, f.atlas_size, f.rate,
                             out=sout, stream=stream)
            torch.cuda.synchronize()
            charts_.append(fa.parse_meta(sout.meta)["num_charts"])
            for sn, ms_ in sctx.stage_times().items():
                st_acc.setdefault(sn, []).append(ms_)
        sctx.set_stage_timing(False)
        res_sc["charts_mean"] = float(np.mean(charts_))
        res_sc["stages_ms"] = {k_: float(np.mean(v_)) for k_, v_ in st_acc.items()
                               if k_ in ("sizes_order", "pack", "select_place")}
        secondary["scatter24k_3840x2160_atlas4096"] = res_sc
        sctx.close()
        log("secondary:", json.dumps(secondary))

    # dual atlas: an 8K full-rate atlas and its 1K companion (same packing)
    dual = None
    if not args.no_dual:
        dctx = fa.Context(T, V, max_charts=65536, max_atlas=8192, gutter=8)
        for knob_ in TUNED:
            dctx.set_tuning(knob_, ctx.get_tuning(knob_))
        dfr = [scenes.city_frame(k, rate=args.rate, atlas_size=8192) for k in range(0, 32, 8)]
        dvis = [torch.as_tensor(f.visible).to(dev) for f in dfr]
        dout = dctx.outputs(mesh, 8192)
        dlow = torch.empty((1024, 1024), dtype=torch.int32, device=dev)

        def dual_step(k, both):
            f = dfr[k % len(dfr)]
            if both:
                dctx.build_dual_atlas(mesh, dvis[k % len(dfr)], f.view_proj, f.width, f.height,
                                      8192, f.rate, 3, out=dout, occupancy_low=dlow,
                                      stream=stream)
            else:
                dctx.build_atlas(mesh, dvis[k % len(dfr)], f.view_proj, f.width, f.height, 8192,
                                 f.rate, out=dout, stream=stream)
        res_d = {}
        for both in (False, True):
            for k in range(4):
                dual_step(k, both)
            evd = []
            for k in range(16):
                a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a_.record(stream)
                dual_step(k, both)
                b_.record(stream)
                evd.append((a_, b_))
            torch.cuda.synchronize()
            res_d["dual_ms" if both else "single_8k_ms"] = float(
                np.mean([a_.elapsed_time(b_) for a_, b_ in evd]))
        dual = dict(atlas=8192, low_atlas=1024, gutter=8, frames=len(dfr), **res_d)
        del dout, dlow
        dctx.close()

    # footprint-aware push against the box push on the same frames
    footprint = None
    if not args.no_footprint:
        fctx = fa.Context(T, V, max_charts=65536, max_atlas=args.atlas,
                          flags=fa.FA_FLAG_FOOTPRINT_PUSH)
        for knob_ in TUNED:
            fctx.set_tuning(knob_, ctx.get_tuning(knob_))
        footprint = {}
        o0 = scenes.orbit_frame(0)
        omesh = fa.Mesh(o0.positions, o0.indices, o0.scene_key)
        cases = [(f"city2m_3840x2160_atlas{args.atlas}_rate{r_:g}", mesh, args.atlas, r_,
                  [scenes.city_frame(k, rate=r_, atlas_size=args.atlas) for k in range(0, 32, 8)])
                 for r_ in (1.0, 2.0)]
        cases.append(("orbit86k_1920x1080_atlas512_rate1", omesh, 512, 1.0,
                      [scenes.orbit_frame(k, atlas_size=512) for k in range(0, 120, 15)]))
        for case_name, mesh_, atlas_, r_, ffr in cases:
            fvis = [torch.as_tensor(f.visible).to(dev) for f in ffr]
            res_f = {}
            for name_, c_ in (("box", ctx), ("footprint", fctx)):
                o_ = c_.outputs(mesh_, atlas_)

                def fstep(k):
                    f = ffr[k % len(ffr)]
                    c_.build_atlas(mesh_, fvis[k % len(ffr)], f.view_proj, f.width, f.height,
                                   atlas_, r_, out=o_, stream=stream)
                metas = []
                for k in range(len(ffr)):
                    fstep(k)
                    torch.cuda.synchronize()
                    metas.append(fa.parse_meta(o_.meta))
                assert all(m_["status"] == fa.FA_OK for m_ in metas), metas
                evf = []
                for k in range(32):
                    a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a_.record(stream)
                    fstep(k)
                    b_.record(stream)
                    evf.append((a_, b_))
                torch.cuda.synchronize()
                res_f[name_] = dict(
                    ms_per_frame=float(np.mean([a_.elapsed_time(b_) for a_, b_ in evf])),
                    chosen_j=[m_["chosen_j"] for m_ in metas],
                    s_eff_mean=float(np.mean([m_["s_eff"] for m_ in metas])),
                    fill_fraction_mean=float(np.mean([m_["occupied_texels"] for m_ in metas]))
                    / float(atlas_) ** 2,
                    layout_height_over_width=float(np.mean(
                        [m_["layout_height"] / m_["layout_width"] for m_ in metas])))
                if name_ == "footprint":
                    c_.set_stage_timing(True)
                    acc_ = {}
                    for k in range(8):
                        fstep(k)
                        torch.cuda.synchronize()
                        for sn, ms_ in c_.stage_times().items():
                            acc_.setdefault(sn, []).append(ms_)
                    c_.set_stage_timing(False)
                    res_f[name_]["stages_ms"] = {
                        sn: float(np.mean(acc_[sn])) for sn in ("fp_count", "fp_raster", "pack")}
                del o_
            footprint[case_name] = dict(frames=len(ffr), **res_f)
        fctx.close()
        log("footprint:", json.dumps(footprint))

    # batched views vs the plain per-view path
    batch = None
    if not args.no_batch:
        views = scenes.batch_views(16)
        bctx = fa.Context(T, V, max_charts=65536, max_atlas=4096, max_views=16)
        for knob_ in TUNED:
            bctx.set_tuning(knob_, ctx.get_tuning(knob_))
        bouts = [bctx.outputs(mesh, v.atlas_size) for v in views]
        bvis = [torch.as_tensor(v.visible).to(dev) for v in views]
        desc = [(bvis[i], v.view_proj, v.width, v.height, v.atlas_size, v.rate)
                for i, v in enumerate(views)]
        reps = 10

        def timed(fn):
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            w_ = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - w_) / reps

        def plain():
            for i, v in enumerate(views):
                bctx.build_atlas(mesh, bvis[i], v.view_proj, v.width, v.height, v.atlas_size,
                                 v.rate, out=bouts[i], stream=stream)
        def snapshot():
            torch.cuda.synchronize()
            out_ = []
            for o in bouts:
                d = o.to_numpy()
                out_.append((d["meta"], d["chart_of_tri"], d["chart_of_vert"], d["charts"],
                             d["occupancy"], d["candidates"], d["uv"].view(np.uint32)))
                for t_ in (o.chart_of_tri, o.occupancy, o.charts, o.meta):
                    t_.fill_(-7)  # the next mode must write everything again
            return out_

        def same(a_, b_):
            return all(x == y if isinstance(x, dict) else np.array_equal(x, y)
                       for va, vb in zip(a_, b_) for x, y in zip(va, vb))
        tp = timed(plain)
        want_b = snapshot()
        bctx.set_tuning(fa.FA_TUNE_BATCH_GRAPH, 0)
        tb = timed(lambda: bctx.build_atlas_batch(mesh, desc, bouts, stream=stream))
        ok_streams = same(snapshot(), want_b)
        bctx.set_tuning(fa.FA_TUNE_BATCH_GRAPH, 1)
        tg = timed(lambda: bctx.build_atlas_batch(mesh, desc, bouts, stream=stream))
        ok_graph = same(snapshot(), want_b)
        # one launch per stage for all 16 views, eager and captured
        bctx.set_tuning(fa.FA_TUNE_BATCH_LAUNCH, 1)
        bctx.set_tuning(fa.FA_TUNE_BATCH_GRAPH, 0)
        tl = timed(lambda: bctx.build_atlas_batch(mesh, desc, bouts, stream=stream))
        ok_launch = same(snapshot(), want_b)
        bctx.set_tuning(fa.FA_TUNE_BATCH_GRAPH, 1)
        tlg = timed(lambda: bctx.build_atlas_batch(mesh, desc, bouts, stream=stream))
        ok_launch_graph = same(snapshot(), want_b)
        bctx.close()
        ok_all = ok_streams and ok_graph and ok_launch and ok_launch_graph
        assert ok_all, "batched outputs differ from the per-view path"
        best = min(tb, tg, tl, tlg)
        batch = dict(views=16, slots=16, outputs_equal_plain=bool(ok_all),
                     plain_views_per_s=16 / tp,
                     batched_views_per_s=16 / best,
                     batched_streams_views_per_s=16 / tb, batched_graph_views_per_s=16 / tg,
                     batched_launch_views_per_s=16 / tl,
                     batched_launch_graph_views_per_s=16 / tlg,
                     speedup=tp / best)

    # served: continuous batching over the three scenes vs one-at-a-time FIFO
    served = None
    if not args.no_serve:
        from paper_2502_17712_amd import serve
        from synth import requests as rq
        mnp = rq.scene_meshes()
        smeshes = {k: fa.Mesh(p_, t_, key) for k, (p_, t_, key) in mnp.items()}
        pools = {"grid": rq.pose_pool("grid", 16, 1), "orbit": rq.pose_pool("orbit", 16, 2),
                 "city": rq.pose_pool("city", 4, 3)}
        svis = {(s, i): torch.as_tensor(pools[s][i].visible).to(dev) for s in pools
                for i in range(len(pools[s]))}

        def make_reqs(lam, n, device_vis=False):
            out_ = []
            for rid, (a, c, s, i, om, r) in enumerate(rq.poisson_stream(lam, n, pools, seed=7)):
                pz = pools[s][i]
                out_.append(serve.Request(rid, s, None if device_vis else svis[(s, i)],
                                          pz.view_proj, pz.width, pz.height, om, r, arrival=a,
                                          client=c, eye=tuple(pz.eye), near=pz.near,
                                          coarse=pz.coarse))
            return out_
        served = {}
        # continuous: 8 slots of one request; fifo: one slot; micro_batched:
        # 4 slots of up to 8 same-scene requests in one batched call
        for kind, slots, nb in (("continuous", 8, 1), ("fifo", 1, 1), ("micro_batched", 4, 8)):
            srv = serve.Server(smeshes, slots=slots, hbm_budget=16 << 30, max_atlas=4096,
                               tuning={k_: ctx.get_tuning(k_) for k_ in TUNED}, batch=nb)
            srv.run(make_reqs(max(args.serve_rate), 256))  # warm-up (fills the output pool)
            served[kind] = {}
            for lam in args.serve_rate:
                reqs = make_reqs(lam, min(args.serve_requests, int(lam * 5) + 64))
                w3 = time.perf_counter()
                res_ = srv.run(reqs)
                wall3 = time.perf_counter() - w3
                assert all(r.meta["status"] == 0 for r in res_)
                served[kind][f"{lam:g}"] = dict(slots=slots, batch=nb, offered_req_per_s=lam,
                                                 **serve.summarize(res_, wall3))
            if slots > 1:
                # the same stream with the visible sets computed on the device
                lam = max(args.serve_rate)
                reqs = make_reqs(lam, args.serve_requests, device_vis=True)
                w3 = time.perf_counter()
                res_ = srv.run(reqs)
                wall3 = time.perf_counter() - w3
                assert all(r.meta["status"] == 0 for r in res_)
                served[kind + "_device_visibility"] = {f"{lam:g}": dict(
                    slots=slots, batch=nb, offered_req_per_s=lam,
                    **serve.summarize(res_, wall3))}
            srv.close()
        log("served:", json.dumps(served))

    # CPU oracle beside the GPU: the single-threaded oracle pinned to one core
    # of this host, on every frame of the two smaller workloads and on four
    # frames of the large one at each rate (the value: the large one at the
    # bench rate, the workload of the line)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, frames)

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
        "config": {"workload": f"city2m_3840x2160_atlas{args.atlas}_rate{args.rate:g}",
                   "triangles": T, "vertices": V, "frames": min(len(frames), args.steps),
                   "orbit_frames": len(frames), "atlas": args.atlas, "rate": args.rate,
                   "num_scales": 64, "visible_tris_mean": Tv, "charts_mean": C},
        "p50_ms": float(np.percentile(per, 50)),
        "p99_ms": float(np.percentile(per, 99)),
        "frames_per_s": 1e3 / ms,
        "triangles_per_s": T / (ms * 1e-3),
        "adjacency_ms": adjacency_ms,
        "stages_ms": stages,
        "tuning": tuning,
        "tuning_table": (os.path.relpath(fa.TUNING_TABLE, HERE)
                         if os.path.exists(fa.TUNING_TABLE) else None),
        "large_tiles": meta["large_tiles"],
        "algorithmic_bytes_per_frame": B,
        "frame_hbm_roofline_frac": B / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "no_occupancy": None if ms_nocc is None else {
            "ms_per_frame": ms_nocc, "algorithmic_bytes": B - 4.0 * args.atlas * args.atlas,
            "hbm_roofline_frac": (B - 4.0 * args.atlas * args.atlas) / (ms_nocc * 1e-3)
            / (HBM_PEAK_GBS * 1e9)},
        "dependent_phases": dependent_phases(ctx, fa),
        "pack_rows_at_chosen_scale": meta["rows"],
        "copy_gbs": copy_gbs,
        "device_visibility": visibility,
        "temporal_reuse": reuse,
        "dual_atlas": dual,
        "footprint_push": footprint,
        "batch": batch,
        "served": served,
        "secondary": secondary,
        "cpu_baseline": cpu,
        "roofline": roofline,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
