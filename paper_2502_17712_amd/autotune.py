"""Autotuner for the library's performance knobs (fa_set_tuning).

Greedy coordinate descent over the knobs on a representative workload: for
each knob in turn, every allowed value is timed with HIP events (mean of
`reps` runs, so that a setting with a slow tail is not preferred) and the
fastest is kept. Every knob value must give identical
results; the tuner checks that by comparing all outputs of each trial with
the reference run, and refuses (raises) on any difference.
"""
from __future__ import annotations

import json

import torch

from . import (FA_TUNE_OCC_LANE_TEXELS, FA_TUNE_OCC_SMALL_TEXELS, FA_TUNE_PACK_BLOCK,
               FA_TUNE_UF_EDGE_HOOKS, FA_TUNE_UF_LINK_INIT, FA_TUNE_UF_TILE, AtlasOutputs,
               Context)

KNOBS = {
    FA_TUNE_OCC_SMALL_TEXELS: [64, 16, 32, 128, 256],
    FA_TUNE_OCC_LANE_TEXELS: [64, 0, 16, 256],
    FA_TUNE_UF_LINK_INIT: [1, 0],
    FA_TUNE_UF_EDGE_HOOKS: [5, 4, 2, 3, 1, 0],
    FA_TUNE_UF_TILE: [4096, 2048, 8192],
    FA_TUNE_PACK_BLOCK: [256, 512, 1024],
}
NAMES = {FA_TUNE_PACK_BLOCK: "pack_block", FA_TUNE_OCC_SMALL_TEXELS: "occ_small_texels",
         FA_TUNE_UF_LINK_INIT: "uf_link_init", FA_TUNE_UF_EDGE_HOOKS: "uf_edge_hooks",
         FA_TUNE_OCC_LANE_TEXELS: "occ_lane_texels", FA_TUNE_UF_TILE: "uf_tile"}


def _snapshot(out: AtlasOutputs):
    # chart records past the frame's chart count are not outputs of the frame
    n = int(out.meta[1].item())
    ts = [out.chart_of_tri, out.chart_of_vert, out.charts[:n], out.meta[:12]]
    for t in (out.uv, out.occupancy, out.candidates):
        if t is not None:
            ts.append(t)
    return [t.clone() for t in ts]


def _same(a, b):
    return all(torch.equal(x.view(torch.int32) if x.dtype == torch.float32 else x,
                           y.view(torch.int32) if y.dtype == torch.float32 else y)
               for x, y in zip(a, b))


def _time(run, reps, stream):
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    run()
    for a, b in evs:
        a.record(stream)
        run()
        b.record(stream)
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in evs) / len(evs)


def tune(ctx: Context, run, out: AtlasOutputs, reps: int = 30, knobs=None, stream=None,
         ref_run=None):
    """run(): enqueue one representative call writing into `out` (it may cycle
    through several inputs); ref_run() (default: run) enqueues the one call
    whose outputs every knob value must reproduce.
    Returns {"choice": {name: value}, "trials": {name: {value: ms}}}."""
    knobs = knobs or KNOBS
    stream = stream or torch.cuda.current_stream()
    ref_run = ref_run or run
    ref_run()
    torch.cuda.synchronize()
    ref = _snapshot(out)
    report = {"choice": {}, "trials": {}}
    for knob, values in knobs.items():
        trials = {}
        for v in values:
            ctx.set_tuning(knob, v)
            ms = _time(run, reps, stream)
            ref_run()
            torch.cuda.synchronize()
            if not _same(_snapshot(out), ref):
                raise RuntimeError(f"knob {NAMES[knob]}={v} changed the results")
            trials[v] = ms
        best = min(trials, key=trials.get)
        ctx.set_tuning(knob, best)
        report["choice"][NAMES[knob]] = best
        report["trials"][NAMES[knob]] = trials
    return report


def save(report, path):
    with open(path, "w") as f:
        json.dump(report, f, indent=1)


TABLE_ORDER = ("pack_block", "occ_small_texels", "occ_lane_texels", "uf_link_init",
               "uf_edge_hooks", "uf_tile")


def table_line(t_lo, t_hi, omega, J, choice, note=""):
    """One tuning-table entry (fa_load_tuning_table) from a tune() choice."""
    vals = " ".join(str(int(choice[k])) for k in TABLE_ORDER)
    return f"{t_lo} {t_hi} {omega} {J} {vals}" + (f"  # {note}" if note else "")


def table_text(lines, header=""):
    head = ["# t_lo t_hi omega J pack_block small_texels lane_texels uf_link_init "
            "uf_edge_hooks uf_tile"]
    if header:
        head.insert(0, "# " + header)
    return "\n".join(head + list(lines)) + "\n"
