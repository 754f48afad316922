"""Continuous-batching request server over the atlasing library.

Requests (scene, camera, visible set, atlas size, rate) arrive over time from
many clients. A request either brings its visible set or leaves it to the
device: then the slot runs the visible-triangle pass (fa_visibility) on the
request's camera first, so the whole request stays on the GPU. The server owns `slots` execution slots; each slot is a library
context (its own scratch and resident scene adjacency) bound to its own HIP
stream. A request is admitted as soon as it has arrived, a slot is free and
its output memory fits in the HBM budget; admitted requests run concurrently
on the device, and a request that arrives while others run is admitted the
moment a slot and memory free up. A request reserves its outputs plus its
frame's working set (reservation_bytes) until it completes. Completion is detected by polling an event
per request; latency = completion - arrival on the host clock.

Every request's results are exactly those of the same request run alone: the
library's outputs depend only on the request's inputs, and slots share no
scratch.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from . import AtlasOutputs, Context, Mesh, parse_meta


@dataclasses.dataclass
class Request:
    rid: int
    scene: str
    visible: torch.Tensor | None  # uint8 [T] on the device, or None: computed on the device
    view_proj: np.ndarray      # float32 [16]
    width: int
    height: int
    atlas_size: int
    rate: float
    arrival: float = 0.0       # seconds after the start of the run
    client: int = 0
    eye: tuple = (0.0, 0.0, 0.0)  # camera position (device visibility)
    near: float = 0.1             # w at the near plane (device visibility)
    coarse: int = 8               # coarse depth-buffer factor (device visibility)


@dataclasses.dataclass
class Result:
    rid: int
    latency: float
    arrival: float
    start: float
    finish: float
    slot: int
    meta: dict
    out: AtlasOutputs | None


def output_bytes(T, V, max_charts, atlas_size, J):
    """Device bytes one request's outputs occupy."""
    return T * 4 + V * 4 + V * 8 + max_charts * 64 + atlas_size * atlas_size * 4 + 64 + J * 16


def reservation_bytes(T, V, max_charts, atlas_size, J):
    """What admission reserves for one request: its outputs plus the frame's
    working set in the slot's scratch, T (9 B: chart, parent, visibility) +
    V (32 B: UV, vertex chart and vertex minimum take 16 B; the rest is
    headroom) + max_charts (64 B record + 16 B per candidate) + 4 omega^2
    (occupancy) + 1 MiB."""
    return (9 * T + 32 * V + max_charts * (64 + 16 * J) + 4 * atlas_size * atlas_size
            + (1 << 20))


class Server:
    def __init__(self, meshes: dict, slots: int = 8, hbm_budget: int = 16 << 30,
                 max_charts: int = 65536, max_atlas: int = 4096, num_scales: int = 64,
                 tuning: dict | None = None):
        self.meshes = meshes
        self.max_charts, self.J = max_charts, num_scales
        T = max(m.num_triangles for m in meshes.values())
        V = max(m.num_vertices for m in meshes.values())
        self.slots = []
        for _ in range(slots):
            ctx = Context(T, V, max_charts=max_charts, max_atlas=max_atlas,
                          num_scales=num_scales)
            for knob, val in (tuning or {}).items():
                ctx.set_tuning(knob, val)
            stream = torch.cuda.Stream()
            for m in meshes.values():  # scene adjacency stays resident per slot
                ctx.adjacency(m, stream=stream)
            with torch.cuda.stream(stream):
                vis_buf = torch.empty(T, dtype=torch.uint8, device="cuda")
            self.slots.append((ctx, stream, vis_buf))
        torch.cuda.synchronize()
        self.budget = int(hbm_budget)

    def request_bytes(self, r: Request) -> int:
        m = self.meshes[r.scene]
        return reservation_bytes(m.num_triangles, m.num_vertices, self.max_charts, r.atlas_size,
                                 self.J)

    def run(self, requests, keep_outputs=False, clock=time.perf_counter, spin_sleep=0.0):
        """Serve `requests` (arrival times relative to the start). Returns the
        results in completion order."""
        for r in requests:
            if self.request_bytes(r) > self.budget:
                raise ValueError(f"request {r.rid} needs more than the whole HBM budget")
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        free = list(range(len(self.slots)))[::-1]
        inflight = []  # (request, slot, event, out, start, bytes)
        reserved = 0
        results = []
        t0 = clock()
        while pending or inflight:
            now = clock() - t0
            # admission: arrived, slot free, memory available (FIFO, no overtaking)
            while pending and free and pending[0].arrival <= now:
                r = pending[0]
                need = self.request_bytes(r)
                if reserved + need > self.budget:
                    break
                pending.popleft()
                k = free.pop()
                ctx, stream, vis_buf = self.slots[k]
                mesh = self.meshes[r.scene]
                with torch.cuda.stream(stream):
                    out = ctx.outputs(mesh, r.atlas_size)
                    vis = r.visible
                    if vis is None:
                        vis = ctx.visibility(mesh, r.view_proj, r.width, r.height, r.eye,
                                             r.near, r.coarse, out=vis_buf[:mesh.num_triangles],
                                             stream=stream)
                    ctx.build_atlas(mesh, vis, r.view_proj, r.width, r.height,
                                    r.atlas_size, r.rate, out=out, stream=stream)
                    ev = torch.cuda.Event()
                    ev.record(stream)
                reserved += need
                inflight.append((r, k, ev, out, clock() - t0, need))
            # completions
            still = []
            for item in inflight:
                r, k, ev, out, start, need = item
                if ev.query():
                    fin = clock() - t0
                    results.append(Result(r.rid, fin - r.arrival, r.arrival, start, fin, k,
                                          parse_meta(out.meta), out if keep_outputs else None))
                    reserved -= need
                    free.append(k)
                else:
                    still.append(item)
            inflight = still
            if not inflight and pending and pending[0].arrival > clock() - t0:
                # idle until the next arrival
                wait = pending[0].arrival - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
            elif spin_sleep:
                time.sleep(spin_sleep)
        return results

    def close(self):
        for ctx, _, _ in self.slots:
            ctx.close()
        self.slots = []


def summarize(results, wall=None):
    lat = np.array([r.latency for r in results]) * 1e3
    fin = max(r.finish for r in results) if results else 0.0
    first = min(r.arrival for r in results) if results else 0.0
    span = wall if wall is not None else max(fin - first, 1e-9)
    return dict(requests=len(results), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
                req_per_s=len(results) / span)
