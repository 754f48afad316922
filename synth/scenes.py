"""Seeded synthetic scenes, cameras and visible-triangle sets.

This module produces the *inputs* of the per-frame atlasing path (mesh,
visible set, camera, atlas size, texel-to-pixel rate). It holds none of the
atlasing method's arithmetic: both the GPU library and the CPU oracle consume
exactly the arrays built here.

The paper measures on archive scenes that are not available here; these
seeded stand-ins reproduce their scale (about 2M triangles for the large
scene, 1080p/2160p views, 1K-8K atlases). The visible set follows the paper's
definition of a visibility-buffer input (Appendix, "Detecting Visible
Triangles"): front-facing, inside the view volume and, for the large scene, not
hidden behind a coarse depth buffer.

Conventions
-----------
* RNG: ``numpy.random.default_rng(seed)``.
* Meshes are welded per object and counter-clockwise seen from outside.
* Value-noise fBm: lattice values from a splitmix64 hash of the integer cell,
  smoothstep interpolation, lacunarity 2, gain 0.5; float64, cast to float32.
* Camera: OpenGL perspective (fovy 60 deg, aspect W/H), ``view_proj = P @ V``
  computed in float64 and stored float32 row-major; clip = M @ [x, y, z, 1].
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

# --------------------------------------------------------------------------
# hashing / noise
# --------------------------------------------------------------------------
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        return z ^ (z >> np.uint64(31))


def _lattice(cells, seed: int) -> np.ndarray:
    """Hash of integer lattice coordinates -> value in [-1, 1)."""
    h = np.full(cells[0].shape, np.uint64(seed * 0x632BE59BD9B4E019 & 0xFFFFFFFFFFFFFFFF))
    with np.errstate(over="ignore"):
        for c in cells:
            h = _splitmix64(h ^ (c.astype(np.int64).view(np.uint64)))
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 / float(1 << 53)) - 1.0


def _smooth(t):
    return t * t * (3.0 - 2.0 * t)


def value_noise(p: np.ndarray, seed: int) -> np.ndarray:
    """Value noise in d = p.shape[1] dimensions (2 or 3), range about [-1, 1]."""
    d = p.shape[1]
    base = np.floor(p)
    frac = p - base
    base = base.astype(np.int64)
    s = _smooth(frac)
    out = np.zeros(p.shape[0])
    for corner in range(1 << d):
        offs = [(corner >> k) & 1 for k in range(d)]
        w = np.ones(p.shape[0])
        cells = []
        for k in range(d):
            w = w * (s[:, k] if offs[k] else (1.0 - s[:, k]))
            cells.append(base[:, k] + offs[k])
        out += w * _lattice(cells, seed)
    return out


def fbm(p: np.ndarray, octaves: int, seed: int) -> np.ndarray:
    total = np.zeros(p.shape[0])
    amp, freq = 0.5, 1.0
    for o in range(octaves):
        total += amp * value_noise(p * freq, seed * 131 + o)
        amp *= 0.5
        freq *= 2.0
    return total


# --------------------------------------------------------------------------
# primitive meshes (float64 positions, int64 indices, CCW outward)
# --------------------------------------------------------------------------
def grid_mesh(n: int, lo: float, hi: float):
    """(n+1)x(n+1) vertex grid over [lo,hi]^2 in the xy plane, diagonal
    (i,j)->(i+1,j+1); vertex (i, j) has x from column j and y from row i."""
    ax = np.linspace(lo, hi, n + 1)
    X, Y = np.meshgrid(ax, ax)  # rows = i (y), cols = j (x)
    pos = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    v00 = (i * (n + 1) + j).ravel()
    v01 = v00 + 1
    v10 = v00 + (n + 1)
    v11 = v10 + 1
    tris = np.empty((2 * n * n, 3), np.int64)
    tris[0::2] = np.stack([v00, v01, v11], 1)
    tris[1::2] = np.stack([v00, v11, v10], 1)
    return pos, tris


def icosphere(level: int):
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    for _ in range(level):
        nv = v.shape[0]
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        key = np.minimum(e[:, 0], e[:, 1]) * nv + np.maximum(e[:, 0], e[:, 1])
        uk, inv = np.unique(key, return_inverse=True)
        a, b = uk // nv, uk % nv
        mid = v[a] + v[b]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        v = np.concatenate([v, mid])
        nf = f.shape[0]
        ab, bc, ca = inv[:nf] + nv, inv[nf:2 * nf] + nv, inv[2 * nf:] + nv
        f = np.concatenate([
            np.stack([f[:, 0], ab, ca], 1), np.stack([f[:, 1], bc, ab], 1),
            np.stack([f[:, 2], ca, bc], 1), np.stack([ab, bc, ca], 1)])
    # orient outward
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    flip = (n * v[f].mean(1)).sum(1) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return v, f


def _weld(pos, tris, quantum):
    q = np.round(pos / quantum).astype(np.int64)
    _, first, inv = np.unique(q, axis=0, return_index=True, return_inverse=True)
    order = np.argsort(first)
    remap = np.empty_like(order)
    remap[order] = np.arange(order.size)
    return pos[first[order]], remap[inv.ravel()][tris]


def box_mesh(n: int):
    """Unit cube [-0.5,0.5]^3 with n x n quads per face, welded."""
    faces = [((0.5, -0.5, -0.5), (0, 1, 0), (0, 0, 1)),
             ((-0.5, -0.5, -0.5), (0, 0, 1), (0, 1, 0)),
             ((-0.5, 0.5, -0.5), (0, 0, 1), (1, 0, 0)),
             ((-0.5, -0.5, -0.5), (1, 0, 0), (0, 0, 1)),
             ((-0.5, -0.5, 0.5), (1, 0, 0), (0, 1, 0)),
             ((-0.5, -0.5, -0.5), (0, 1, 0), (1, 0, 0))]
    P, Tl = [], []
    base = 0
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    qi, qj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    qi, qj = qi.ravel(), qj.ravel()
    for o, e1, e2 in faces:
        o, e1, e2 = np.array(o, float), np.array(e1, float), np.array(e2, float)
        P.append(o + np.outer(ii / n, e1) + np.outer(jj / n, e2))
        v00 = base + qi * (n + 1) + qj
        v10 = v00 + (n + 1)
        v01 = v00 + 1
        v11 = v10 + 1
        Tl.append(np.stack([v00, v10, v11], 1))
        Tl.append(np.stack([v00, v11, v01], 1))
        base += (n + 1) ** 2
    return _weld(np.concatenate(P), np.concatenate(Tl), 0.25 / n)


def cylinder_mesh(seg: int, bands: int):
    """Radius 1, z in [0,1], seg x bands side quads plus triangle-fan caps."""
    th = 2 * np.pi * np.arange(seg) / seg
    ring = np.stack([np.cos(th), np.sin(th)], 1)
    side = np.concatenate([np.concatenate([ring, np.full((seg, 1), k / bands)], 1)
                           for k in range(bands + 1)])
    pos = np.concatenate([side, [[0, 0, 0]], [[0, 0, 1]]])
    cb, ct = side.shape[0], side.shape[0] + 1
    k, s = np.meshgrid(np.arange(bands), np.arange(seg), indexing="ij")
    k, s = k.ravel(), s.ravel()
    a = k * seg + s
    b = k * seg + (s + 1) % seg
    c = (k + 1) * seg + (s + 1) % seg
    d = (k + 1) * seg + s
    tris = [np.stack([a, b, c], 1), np.stack([a, c, d], 1)]
    s = np.arange(seg)
    tris.append(np.stack([np.full(seg, cb), (s + 1) % seg, s], 1))
    top = bands * seg
    tris.append(np.stack([np.full(seg, ct), top + s, top + (s + 1) % seg], 1))
    return pos, np.concatenate(tris)


def _rot_uniform(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


class _Builder:
    def __init__(self):
        self.P, self.T, self.nv = [], [], 0

    def add(self, pos, tris):
        self.P.append(pos)
        self.T.append(tris + self.nv)
        self.nv += pos.shape[0]

    def done(self):
        return (np.concatenate(self.P).astype(np.float32),
                np.concatenate(self.T).astype(np.int32))


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------
def scene_grid(seed: int):
    """64x64-quad heightfield grid, 8192 triangles, 4225 vertices."""
    rng = np.random.default_rng(seed)
    pos, tris = grid_mesh(64, -1.0, 1.0)
    pos[:, 2] = 0.2 * np.sin(3 * pos[:, 0]) * np.cos(2 * pos[:, 1]) + rng.normal(0, 0.02, pos.shape[0])
    yaw = rng.uniform(0, 2 * np.pi)
    return pos.astype(np.float32), tris.astype(np.int32), yaw


def scene_orbit(seed: int = 1):
    """~86.5k triangles: displaced icosphere plus 100 boxes and 100 cylinders."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    v, f = icosphere(5)
    r = 1.0 + 0.1 * fbm(v * 2.0, 4, seed)
    b.add(v * r[:, None], f)
    bp, bt = box_mesh(5)
    cp, ct = cylinder_mesh(36, 4)
    cp = cp * np.array([0.5, 0.5, 1.0]) - np.array([0, 0, 0.5])

    def centre():
        while True:
            c = rng.uniform(-4, 4, 3)
            if np.linalg.norm(c) >= 1.5:
                return c
    for kind in (0, 1):
        for _ in range(100):
            c = centre()
            R = _rot_uniform(rng)
            S = rng.uniform(0.1, 0.4, 3)
            p, t = (bp, bt) if kind == 0 else (cp, ct)
            b.add((p * S) @ R.T + c, t)
    theta0 = float(np.random.default_rng(seed).uniform(0, 2 * np.pi))
    pos, tris = b.done()
    return pos, tris, theta0


def terrain_height(x, y, seed: int):
    p = np.stack([np.asarray(x, float).ravel() / 25.0, np.asarray(y, float).ravel() / 25.0], 1)
    return 3.0 * fbm(p, 6, seed)


def scene_city(seed: int = 2):
    """~2.24M triangles: 512x512-vertex terrain plus 400 instances."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    pos, tris = grid_mesh(511, -100.0, 100.0)
    pos[:, 2] = terrain_height(pos[:, 0], pos[:, 1], seed)
    b.add(pos, tris)
    sv, sf = icosphere(4)
    bp, bt = box_mesh(16)
    cp, ct = cylinder_mesh(64, 12)
    for k in range(400):
        u = rng.uniform()
        xy = rng.uniform(-90, 90, 2)
        h = float(terrain_height(xy[0:1], xy[1:2], seed)[0])
        R = _rot_z(rng.uniform(0, 2 * np.pi))
        if u < 0.7:
            rad = rng.uniform(0.5, 2.0)
            disp = 1.0 + 0.1 * fbm(sv * 2.0, 4, seed * 1000 + k)
            p = sv * (rad * disp)[:, None] + np.array([xy[0], xy[1], h + 0.8 * rad])
            b.add(p, sf)
        elif u < 0.85:
            S = np.array([rng.uniform(0.5, 3.0), rng.uniform(0.5, 3.0), rng.uniform(0.5, 3.0)])
            p = (bp * S + np.array([0, 0, 0.5 * S[2] - 0.2])) @ R.T + np.array([xy[0], xy[1], h])
            b.add(p, bt)
        else:
            rad, hh = rng.uniform(0.3, 1.5), rng.uniform(0.5, 4.0)
            p = (cp * np.array([rad, rad, hh]) - np.array([0, 0, 0.2])) @ R.T + np.array([xy[0], xy[1], h])
            b.add(p, ct)
    return b.done()


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
def perspective(fovy_deg, aspect, near, far):
    f = 1.0 / math.tan(math.radians(fovy_deg) / 2)
    return np.array([[f / aspect, 0, 0, 0], [0, f, 0, 0],
                     [0, 0, (far + near) / (near - far), 2 * far * near / (near - far)],
                     [0, 0, -1, 0]], np.float64)


def look_at(eye, target, up=(0, 0, 1)):
    eye, target, up = (np.asarray(a, np.float64) for a in (eye, target, up))
    f = target - eye
    f /= np.linalg.norm(f)
    s = np.cross(f, up)
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    V = np.eye(4)
    V[0, :3], V[1, :3], V[2, :3] = s, u, -f
    V[0, 3], V[1, 3], V[2, 3] = -s @ eye, -u @ eye, f @ eye
    return V


@dataclasses.dataclass
class Camera:
    view_proj: np.ndarray  # float32 [16], row-major
    width: int
    height: int
    eye: np.ndarray  # float64 [3]
    near: float


def make_camera(eye, target, width, height, near, far, up=(0, 0, 1)):
    M = perspective(60.0, width / height, near, far) @ look_at(eye, target, up)
    return Camera(M.astype(np.float32).ravel(), int(width), int(height),
                  np.asarray(eye, np.float64), float(near))


# --------------------------------------------------------------------------
# visibility (input generation; float64)
# --------------------------------------------------------------------------
def _clip64(pos, cam):
    # elementwise, in a fixed order ((m0 x + m1 y) + m2 z) + m3 per row, so the
    # result does not depend on a BLAS kernel's summation order or FMA use
    M = cam.view_proj.astype(np.float64).reshape(4, 4)
    p = pos.astype(np.float64)
    x, y, z = p[:, 0:1], p[:, 1:2], p[:, 2:3]
    return ((x * M[:, 0] + y * M[:, 1]) + z * M[:, 2]) + M[:, 3]


def visible_set(pos, tris, cam, coarse_occlusion=False):
    """uint8 [T]: front-facing, not entirely outside one clip plane and
    (optionally) not hidden behind a (W/8)x(H/8) coarse depth buffer."""
    p = pos.astype(np.float64)
    p0, p1, p2 = p[tris[:, 0]], p[tris[:, 1]], p[tris[:, 2]]
    a, b, d = p1 - p0, p2 - p0, cam.eye - p0
    n0 = a[:, 1] * b[:, 2] - a[:, 2] * b[:, 1]
    n1 = a[:, 2] * b[:, 0] - a[:, 0] * b[:, 2]
    n2 = a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]
    front = ((n0 * d[:, 0] + n1 * d[:, 1]) + n2 * d[:, 2]) > 0
    c = _clip64(pos, cam)
    cx, cy, cz, cw = c[:, 0], c[:, 1], c[:, 2], c[:, 3]
    outside_all = np.zeros(tris.shape[0], bool)
    for d in (cw + cx, cw - cx, cw + cy, cw - cy, cw + cz, cw - cz):
        dt = d[tris]
        outside_all |= (dt < 0).all(1)
    vis = front & ~outside_all
    if coarse_occlusion:
        vis &= _coarse_occlusion(c, tris, vis, cam)
    return vis.astype(np.uint8)


def _coarse_occlusion(c, tris, cand, cam):
    Wc, Hc = cam.width // 8, cam.height // 8
    w = c[:, 3]
    tw = w[tris]
    all_front = (tw > cam.near).all(1)
    occ_ids = np.nonzero(cand & all_front)[0]
    t3 = tris[occ_ids]
    sx = (c[:, 0] / w * 0.5 + 0.5) * Wc
    sy = (0.5 - c[:, 1] / w * 0.5) * Hc
    sz = c[:, 2] / w
    X, Y, Z = sx[t3], sy[t3], sz[t3]
    ix0 = np.clip(np.ceil(X.min(1) - 0.5), 0, Wc - 1).astype(np.int64)
    ix1 = np.clip(np.floor(X.max(1) - 0.5), -1, Wc - 1).astype(np.int64)
    iy0 = np.clip(np.ceil(Y.min(1) - 0.5), 0, Hc - 1).astype(np.int64)
    iy1 = np.clip(np.floor(Y.max(1) - 0.5), -1, Hc - 1).astype(np.int64)
    nx = np.maximum(ix1 - ix0 + 1, 0)
    ny = np.maximum(iy1 - iy0 + 1, 0)
    cnt = nx * ny
    tot = int(cnt.sum())
    rep = np.repeat(np.arange(occ_ids.size), cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    loc = np.arange(tot) - start
    nxr = nx[rep]
    px = ix0[rep] + loc % nxr
    py = iy0[rep] + loc // nxr
    cxp, cyp = px + 0.5, py + 0.5
    x0, x1, x2 = X[rep, 0], X[rep, 1], X[rep, 2]
    y0, y1, y2 = Y[rep, 0], Y[rep, 1], Y[rep, 2]
    e0 = (x2 - x1) * (cyp - y1) - (y2 - y1) * (cxp - x1)
    e1 = (x0 - x2) * (cyp - y2) - (y0 - y2) * (cxp - x2)
    e2 = (x1 - x0) * (cyp - y0) - (y1 - y0) * (cxp - x0)
    area = e0 + e1 + e2
    inside = (area != 0) & (((e0 >= 0) & (e1 >= 0) & (e2 >= 0)) | ((e0 <= 0) & (e1 <= 0) & (e2 <= 0)))
    sel = np.nonzero(inside)[0]
    area_s = area[sel]
    zs = (e0[sel] * Z[rep[sel], 0] + e1[sel] * Z[rep[sel], 1] + e2[sel] * Z[rep[sel], 2]) / area_s
    pix = py[sel] * Wc + px[sel]
    D = np.full(Wc * Hc, np.inf)
    np.minimum.at(D, pix, zs)
    covered = np.zeros(occ_ids.size, bool)
    covered[rep[sel]] = True
    passes = np.zeros(occ_ids.size, bool)
    ok = zs <= D[pix] + 1e-6
    passes[rep[sel][ok]] = True
    keep_local = ~covered | passes
    keep = np.ones(tris.shape[0], bool)
    keep[occ_ids] = keep_local  # triangles straddling the near plane are never culled here
    return keep


# --------------------------------------------------------------------------
# frames (what one call of the atlasing path consumes)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Frame:
    name: str
    positions: np.ndarray   # float32 [V,3]
    indices: np.ndarray     # int32 [T,3]
    visible: np.ndarray     # uint8 [T]
    view_proj: np.ndarray   # float32 [16] row-major
    width: int
    height: int
    atlas_size: int
    rate: float
    scene_key: int
    eye: np.ndarray = None  # float64 [3], camera position (visibility input)
    near: float = 0.0       # near-plane distance (w at the near plane)
    coarse: int = 0         # coarse depth-buffer factor of the visible set (0: none)

    @property
    def num_triangles(self):
        return int(self.indices.shape[0])

    @property
    def num_vertices(self):
        return int(self.positions.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.positions, self.indices, self.visible, self.view_proj):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(np.array([self.width, self.height, self.atlas_size], np.int64).tobytes())
        h.update(np.array([self.rate], np.float32).tobytes())
        return h.hexdigest()


_CACHE: dict = {}


def _cached(key, fn):
    if key not in _CACHE:
        _CACHE[key] = fn()
    return _CACHE[key]


def grid_frame(seed: int, atlas_size: int = 1024, rate: float = 1.0) -> Frame:
    """Small case: 8192-triangle heightfield, 1280x720 view, 1024^2 atlas."""
    pos, tris, yaw = scene_grid(seed)
    el = math.radians(45.0)
    eye = 2.5 * np.array([math.cos(el) * math.cos(yaw), math.cos(el) * math.sin(yaw), math.sin(el)])
    cam = make_camera(eye, (0, 0, 0), 1280, 720, 0.05, 100.0)
    vis = visible_set(pos, tris, cam)
    return Frame(f"grid8k/seed{seed}", pos, tris, vis, cam.view_proj, 1280, 720,
                 atlas_size, rate, 1000 + seed, cam.eye, cam.near, 0)


def orbit_frame(frame: int, atlas_size: int = 2048, rate: float = 1.0) -> Frame:
    """~86.5k-triangle scene, 1920x1080 view on a 120-frame orbit, 2048^2 atlas."""
    pos, tris, theta0 = _cached("orbit", lambda: scene_orbit(1))
    th = theta0 + 2 * np.pi * frame / 120.0
    eye = np.array([6 * math.cos(th), 6 * math.sin(th), 2.0])
    cam = make_camera(eye, (0, 0, 0), 1920, 1080, 0.05, 100.0)
    vis = visible_set(pos, tris, cam)
    return Frame(f"orbit86k/f{frame}", pos, tris, vis, cam.view_proj, 1920, 1080,
                 atlas_size, rate, 2001, cam.eye, cam.near, 0)


def city_scene():
    return _cached("city", lambda: scene_city(2))


def city_camera(seed: int, frame: int, width: int, height: int, nframes: int = 32):
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-60, 60, 2)
    yaw0 = rng.uniform(0, 2 * np.pi)
    h = float(terrain_height(xy[0:1], xy[1:2], 2)[0])
    eye = np.array([xy[0], xy[1], h + 4.0])
    yaw = yaw0 + 2 * np.pi * frame / nframes
    pitch = math.radians(-10.0)
    d = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    return make_camera(eye, eye + d, width, height, 0.1, 1000.0)


def city_frame(frame: int = 0, rate: float = 1.0, atlas_size: int = 4096,
               width: int = 3840, height: int = 2160, seed: int = 2) -> Frame:
    """~2.24M-triangle scene, 3840x2160 view, 4096^2 atlas, coarse occlusion."""
    pos, tris = city_scene()
    cam = city_camera(seed, frame, width, height)
    vis = visible_set(pos, tris, cam, coarse_occlusion=True)
    return Frame(f"city2m/s{seed}f{frame}", pos, tris, vis, cam.view_proj, width, height,
                 atlas_size, rate, 3002, cam.eye, cam.near, 8)


# --------------------------------------------------------------------------
# near-plane frames: cameras close enough to the geometry that visible
# triangles cross the near plane (the special case of the box step), some of
# them with vertices behind the eye (w <= 0)
# --------------------------------------------------------------------------
def _grazing_dir(yaw, pitch):
    return np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw),
                     math.sin(pitch)])


def grid_near_frame(seed: int, atlas_size: int = 1024, rate: float = 1.0) -> Frame:
    """The 8192-triangle heightfield of grid_frame(seed) seen from a grazing
    camera 0.05-0.15 above the surface with near = 0.4, so that tens of
    visible triangles cross the near plane (with one or two vertices in front
    of it)."""
    pos, tris, yaw = scene_grid(seed)
    rng = np.random.default_rng(10_000 + seed)
    xy = rng.uniform(-0.6, 0.6, 2)
    k = int(np.argmin(((pos[:, :2].astype(np.float64) - xy) ** 2).sum(1)))
    eye = np.array([xy[0], xy[1], float(pos[k, 2]) + rng.uniform(0.05, 0.15)])
    d = _grazing_dir(yaw, math.radians(rng.uniform(-25.0, 0.0)))
    cam = make_camera(eye, eye + d, 1280, 720, 0.4, 100.0)
    vis = visible_set(pos, tris, cam)
    return Frame(f"gridnear/seed{seed}", pos, tris, vis, cam.view_proj, 1280, 720,
                 atlas_size, rate, 1000 + seed, cam.eye, cam.near, 0)


def scene_floor(seed: int):
    """16x16-quad floor over [-4, 4]^2 (512 triangles of side 0.5) with
    N(0, 0.05) height noise."""
    rng = np.random.default_rng(seed)
    pos, tris = grid_mesh(16, -4.0, 4.0)
    pos[:, 2] = rng.normal(0, 0.05, pos.shape[0])
    return pos.astype(np.float32), tris.astype(np.int32)


def floor_near_frame(seed: int, atlas_size: int = 512, rate: float = 1.0) -> Frame:
    """A coarse floor seen from 0.15 above it with near = 0.3: the large
    triangles under the camera reach behind the eye (w <= 0) and cross the
    near plane."""
    pos, tris = scene_floor(6000)
    rng = np.random.default_rng(6000 + seed)
    eye = np.array([*rng.uniform(-1.0, 1.0, 2), 0.15])
    d = _grazing_dir(rng.uniform(0, 2 * np.pi), math.radians(rng.uniform(-30.0, -5.0)))
    cam = make_camera(eye, eye + d, 1280, 720, 0.3, 100.0)
    vis = visible_set(pos, tris, cam)
    return Frame(f"floornear/seed{seed}", pos, tris, vis, cam.view_proj, 1280, 720,
                 atlas_size, rate, 6000, cam.eye, cam.near, 0)


def city_near_frame(frame: int = 0, rate: float = 1.0, atlas_size: int = 4096,
                    width: int = 3840, height: int = 2160, seed: int = 2) -> Frame:
    """The ~2.24M-triangle scene from the orbit of city_frame, with the eye
    lowered to 0.05 above the terrain: the terrain triangles around the eye
    cross the near plane (0.1) and some reach behind it."""
    pos, tris = city_scene()
    c0 = city_camera(seed, frame, width, height)
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-60, 60, 2)
    yaw0 = rng.uniform(0, 2 * np.pi)
    eye = np.array([xy[0], xy[1], float(terrain_height(xy[0:1], xy[1:2], 2)[0]) + 0.05])
    assert np.allclose(eye[:2], c0.eye[:2])
    d = _grazing_dir(yaw0 + 2 * np.pi * frame / 32, math.radians(-10.0))
    cam = make_camera(eye, eye + d, width, height, 0.1, 1000.0)
    vis = visible_set(pos, tris, cam, coarse_occlusion=True)
    return Frame(f"citynear/s{seed}f{frame}", pos, tris, vis, cam.view_proj, width, height,
                 atlas_size, rate, 3002, cam.eye, cam.near, 8)


_RES = [(1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)]


def batch_views(n: int = 16, base_seed: int = 3000):
    """Views of the ~2.24M-triangle scene with seeded uneven resolution, atlas
    size and rate: view i uses seed base_seed + i."""
    pos, tris = city_scene()
    views = []
    for i in range(n):
        rng = np.random.default_rng(base_seed + i)
        W, H = _RES[int(rng.integers(0, 4))]
        om = [1024, 2048, 4096][int(rng.integers(0, 3))]
        r = [0.5, 1.0, 2.0][int(rng.integers(0, 3))]
        cam = city_camera(base_seed + i, 0, W, H)
        vis = visible_set(pos, tris, cam, coarse_occlusion=True)
        views.append(Frame(f"city2m/view{i}", pos, tris, vis, cam.view_proj, W, H, om, r, 3002,
                           cam.eye, cam.near, 8))
    return views


# --------------------------------------------------------------------------
# many-chart frames: thousands of small separate objects in view, so that the
# ordering and packing stages see the chart counts of the paper's archive
# scenes (thousands to tens of thousands of charts per frame)
# --------------------------------------------------------------------------
def scene_scatter(seed: int = 4, count: int = 24000):
    """``count`` small boxes (12 triangles each, side 0.05-0.2, random
    orientation) scattered through the view volume of a camera at the
    origin looking along +x: distance 4-40, lateral positions inside 95% of
    a 60-degree vertical, 16:9 field of view."""
    rng = np.random.default_rng(seed)
    bp, bt = box_mesh(1)
    b = _Builder()
    ty = math.tan(math.radians(30.0)) * 0.95
    tx = ty * 16.0 / 9.0
    for _ in range(count):
        d = rng.uniform(4.0, 40.0)
        c = np.array([d, rng.uniform(-tx, tx) * d, rng.uniform(-ty, ty) * d])
        R = _rot_uniform(rng)
        s = rng.uniform(0.05, 0.2)
        b.add((bp * s) @ R.T + c, bt)
    return b.done()


def scatter_frame(frame: int = 0, rate: float = 1.0, atlas_size: int = 4096,
                  width: int = 3840, height: int = 2160, seed: int = 4,
                  count: int = 24000) -> Frame:
    """~24k small boxes (288k triangles), 3840x2160 view, 4096^2 atlas: about
    20k charts per frame (every visible box is its own chart). Frame f turns
    the camera by f degrees of yaw about the origin. `count` boxes instead of
    24,000 give a scene of 12 x count triangles (its own scene key)."""
    pos, tris = _cached(("scatter", seed, count), lambda: scene_scatter(seed, count))
    yaw = math.radians(float(frame))
    eye = np.zeros(3)
    d = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    cam = make_camera(eye, eye + d, width, height, 0.1, 1000.0)
    vis = visible_set(pos, tris, cam)
    key = 4000 + seed if count == 24000 else 7_000_000 + 16 * count + seed
    name = "scatter24k" if count == 24000 else f"scatter{count}"
    return Frame(f"{name}/s{seed}f{frame}", pos, tris, vis, cam.view_proj, width, height,
                 atlas_size, rate, key, cam.eye, cam.near, 0)
