"""Seeded request streams for the served workload: per-scene pools of poses
(camera, resolution, visible set) and Poisson arrivals from many clients.

A request = (scene, pose from the pool, atlas size, rate); resolutions are
drawn from {1280x720, 1920x1080, 2560x1440, 3840x2160}, atlas sizes from
{1024, 2048, 4096}, rates from {0.5, 1, 2}.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import scenes

RES = [(1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)]
ATLAS = [1024, 2048, 4096]
RATES = [0.5, 1.0, 2.0]


@dataclasses.dataclass
class Pose:
    scene: str
    view_proj: np.ndarray
    width: int
    height: int
    visible: np.ndarray
    eye: np.ndarray = None   # camera position
    near: float = 0.0        # w at the near plane
    coarse: int = 0          # coarse depth-buffer factor of `visible`


def scene_meshes():
    """name -> (positions, indices, scene_key) of the three served scenes."""
    g = scenes.grid_frame(0)
    o = scenes.orbit_frame(0)
    cp, ct = scenes.city_scene()
    return {"grid": (g.positions, g.indices, 5001), "orbit": (o.positions, o.indices, 5002),
            "city": (cp, ct, 5003)}


def pose_pool(name, n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        W, H = RES[int(rng.integers(0, 4))]
        if name == "grid":
            # the served grid scene (scene_meshes), seen from a seeded yaw
            f = scenes.grid_frame(0)
            pos, tris = f.positions, f.indices
            el = np.radians(45.0)
            yaw = rng.uniform(0, 2 * np.pi)
            eye = 2.5 * np.array([np.cos(el) * np.cos(yaw), np.cos(el) * np.sin(yaw), np.sin(el)])
            cam = scenes.make_camera(eye, (0, 0, 0), W, H, 0.05, 100.0)
            vis = scenes.visible_set(pos, tris, cam)
            coarse = 0
        elif name == "orbit":
            pos, tris, th0 = scenes._cached("orbit", lambda: scenes.scene_orbit(1))
            th = th0 + 2 * np.pi * int(rng.integers(0, 120)) / 120.0
            eye = np.array([6 * np.cos(th), 6 * np.sin(th), 2.0])
            cam = scenes.make_camera(eye, (0, 0, 0), W, H, 0.05, 100.0)
            vis = scenes.visible_set(pos, tris, cam)
            coarse = 0
        else:
            pos, tris = scenes.city_scene()
            cam = scenes.city_camera(4000 + seed * 1000 + k, int(rng.integers(0, 32)), W, H)
            vis = scenes.visible_set(pos, tris, cam, coarse_occlusion=True)
            coarse = 8
        out.append(Pose(name, cam.view_proj, W, H, vis, cam.eye, cam.near, coarse))
    return out


def poisson_stream(rate_per_s, n_requests, pools, clients=64, seed=0, mix=(1, 1, 1)):
    """Arrivals of `clients` independent Poisson clients (each rate/clients),
    merged; returns [(arrival_s, client, scene, pose_index, atlas, rate)]."""
    rng = np.random.default_rng(seed)
    names = list(pools)
    p = np.asarray(mix, float)[: len(names)]
    p = p / p.sum()
    per = rate_per_s / clients
    events = []
    k_per_client = int(np.ceil(n_requests / clients)) + 2
    for c in range(clients):
        t = np.cumsum(rng.exponential(1.0 / per, size=k_per_client))
        for a in t:
            events.append((float(a), c))
    events.sort()
    events = events[:n_requests]
    out = []
    for a, c in events:
        s = names[int(rng.choice(len(names), p=p))]
        out.append((a, c, s, int(rng.integers(0, len(pools[s]))),
                    ATLAS[int(rng.integers(0, 3))], RATES[int(rng.integers(0, 3))]))
    return out
