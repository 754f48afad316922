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

With batch > 1 a slot takes up to `batch` arrived requests of one scene at
once (the oldest arrived request and the next arrived requests of its scene,
which may overtake requests of other scenes) and atlases them in one batched
call (fa_build_atlas_batch with one launch per stage for all its views); a
slot that finds a single request runs the plain per-view call. Under light
load batches stay at one request; as arrivals outpace the device they grow,
and the per-request host work (marshalling, submission, completion events)
is shared by the batch.

Output buffers come from a pool per scene and atlas size (filled by the
requests whose outputs the caller does not keep), and each request's meta record is copied to
pinned host memory on its stream, so completion is read without a blocking
device copy.

Python's cyclic garbage collector is paused while run() serves (pause_gc):
a full collection in a process holding torch walks every live object and can
stall the loop for tens of milliseconds, a latency spike for every request in
flight. The loop itself makes no reference cycles.

Every request's results are exactly those of the same request run alone: the
library's outputs depend only on the request's inputs (every output element is
written by each call, so a recycled buffer carries nothing over), and slots
share no scratch.
"""
from __future__ import annotations

import collections
import dataclasses
import gc
import time

import numpy as np
import torch

from . import (FA_TUNE_BATCH_GRAPH, FA_TUNE_BATCH_LAUNCH, META_DTYPE, AtlasOutputs,
               Context, Mesh)


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
                 tuning: dict | None = None, batch: int = 1):
        if batch < 1:
            raise ValueError("batch must be >= 1")
        self.meshes = meshes
        self.batch = int(batch)
        self.max_charts, self.J = max_charts, num_scales
        T = max(m.num_triangles for m in meshes.values())
        V = max(m.num_vertices for m in meshes.values())
        self.slots = []
        for _ in range(slots):
            ctx = Context(T, V, max_charts=max_charts, max_atlas=max_atlas,
                          num_scales=num_scales, max_views=self.batch)
            for knob, val in (tuning or {}).items():
                ctx.set_tuning(knob, val)
            if self.batch > 1:
                # one launch per stage for the whole batch; no cached graph
                # (every batch brings other buffers)
                ctx.set_tuning(FA_TUNE_BATCH_LAUNCH, 1)
                ctx.set_tuning(FA_TUNE_BATCH_GRAPH, 0)
            stream = torch.cuda.Stream()
            for m in meshes.values():  # scene adjacency stays resident per slot
                ctx.adjacency(m, stream=stream)
            with torch.cuda.stream(stream):
                vis_buf = torch.empty((self.batch, T), dtype=torch.uint8, device="cuda")
            self.slots.append((ctx, stream, vis_buf))
        # one pinned meta row per request a slot can hold
        self.host_meta = torch.zeros((slots * self.batch, 16), dtype=torch.int32,
                                     pin_memory=True)
        self.host_meta_np = self.host_meta.numpy()
        self.pool = collections.defaultdict(list)  # (scene, atlas) -> free outputs
        torch.cuda.synchronize()
        self.budget = int(hbm_budget)

    def request_bytes(self, r: Request) -> int:
        m = self.meshes[r.scene]
        return reservation_bytes(m.num_triangles, m.num_vertices, self.max_charts, r.atlas_size,
                                 self.J)

    def _outputs(self, ctx, r):
        free = self.pool[(r.scene, r.atlas_size)]
        if free:
            return free.pop()
        return ctx.outputs(self.meshes[r.scene], r.atlas_size)

    def _take_group(self, now, reserved):
        """The next batch to admit: the oldest pending request (if it has
        arrived and fits) and, for batch > 1, the following arrived requests
        of its scene that fit. Removes them from self._pending."""
        pending = self._pending
        if not pending or pending[0].arrival > now:
            return [], reserved
        head = pending[0]
        need = self.request_bytes(head)
        if reserved + need > self.budget:
            return [], reserved
        pending.popleft()
        group, reserved = [(head, need)], reserved + need
        i = 0
        while len(group) < self.batch and i < len(pending):
            q = pending[i]
            if q.arrival > now:
                break
            if q.scene == head.scene:
                nq = self.request_bytes(q)
                if reserved + nq > self.budget:
                    break
                del pending[i]
                group.append((q, nq))
                reserved += nq
            else:
                i += 1
        return group, reserved

    def run(self, requests, keep_outputs=False, clock=time.perf_counter, spin_sleep=0.0,
            pause_gc=True):
        """Serve `requests` (arrival times relative to the start). Returns the
        results in completion order."""
        for r in requests:
            if self.request_bytes(r) > self.budget:
                raise ValueError(f"request {r.rid} needs more than the whole HBM budget")
        was_enabled = gc.isenabled()
        if pause_gc:
            gc.disable()
        try:
            return self._serve(requests, keep_outputs, clock, spin_sleep)
        finally:
            if was_enabled:
                gc.enable()

    def _serve(self, requests, keep_outputs, clock, spin_sleep):
        self._pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        pending = self._pending
        free = list(range(len(self.slots)))[::-1]
        inflight = []  # (group [(request, out, bytes)], slot, event, start)
        reserved = 0
        results = []
        t0 = clock()
        while pending or inflight:
            now = clock() - t0
            # admission: arrived, slot free, memory available (FIFO heads)
            while free:
                group, reserved = self._take_group(now, reserved)
                if not group:
                    break
                k = free.pop()
                ctx, stream, vis_buf = self.slots[k]
                mesh = self.meshes[group[0][0].scene]
                T = mesh.num_triangles
                with torch.cuda.stream(stream):
                    outs, vis = [], []
                    for i, (r, _) in enumerate(group):
                        outs.append(self._outputs(ctx, r))
                        v = r.visible
                        if v is None:
                            v = ctx.visibility(mesh, r.view_proj, r.width, r.height, r.eye,
                                               r.near, r.coarse, out=vis_buf[i, :T],
                                               stream=stream)
                        vis.append(v)
                    if len(group) == 1:
                        r = group[0][0]
                        ctx.build_atlas(mesh, vis[0], r.view_proj, r.width, r.height,
                                        r.atlas_size, r.rate, out=outs[0], stream=stream)
                    else:
                        ctx.build_atlas_batch(
                            mesh, [(vis[i], r.view_proj, r.width, r.height, r.atlas_size,
                                    r.rate) for i, (r, _) in enumerate(group)],
                            outs, stream=stream)
                    base = k * self.batch
                    for i, o in enumerate(outs):
                        self.host_meta[base + i].copy_(o.meta, non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(stream)
                start = clock() - t0
                inflight.append(([(r, outs[i], need) for i, (r, need) in enumerate(group)],
                                 k, ev, start))
            # completions
            still = []
            for item in inflight:
                group, k, ev, start = item
                if ev.query():
                    fin = clock() - t0
                    base = k * self.batch
                    for i, (r, out, need) in enumerate(group):
                        row = self.host_meta_np[base + i].view(META_DTYPE)[0]
                        meta = {f: row[f].item() for f in META_DTYPE.names}
                        results.append(Result(r.rid, fin - r.arrival, r.arrival, start, fin, k,
                                              meta, out if keep_outputs else None))
                        reserved -= need
                        if not keep_outputs:
                            self.pool[(r.scene, r.atlas_size)].append(out)
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
        self.pool.clear()


def summarize(results, wall=None):
    lat = np.array([r.latency for r in results]) * 1e3
    fin = max(r.finish for r in results) if results else 0.0
    first = min(r.arrival for r in results) if results else 0.0
    span = wall if wall is not None else max(fin - first, 1e-9)
    return dict(requests=len(results), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
                req_per_s=len(results) / span)
