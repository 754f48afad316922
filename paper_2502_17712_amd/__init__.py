"""Python binding of the gfx950 per-frame atlasing library (libfastatlas.so).

Argument marshalling only: every step of the path runs in the library's HIP
kernels. PyTorch provides device memory and streams. The library must be
built (``python -m paper_2502_17712_amd.build`` or ``__graft_entry__.build()``)
and is loaded after ``torch`` so that both share one HIP runtime. There is no
fallback: importing without the built library raises.

C-ABI names are mirrored one to one (``fa_create``, ``fa_build_atlas``, ...);
``Context`` is a convenience wrapper that allocates the output tensors.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, c_double, c_float, c_int, c_int32, c_int64, c_uint32, c_uint64,
                    c_void_p)

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastatlas.so")

FA_OK, FA_ERR_INVALID_ARG, FA_ERR_OUT_OF_MEMORY, FA_ERR_CAPACITY = 0, 1, 2, 3
FA_ERR_NOFIT, FA_ERR_DEVICE, FA_ERR_UNSUPPORTED = 4, 5, 6
FA_FLAG_NO_SIDE_CLIP = 1
FA_FLAG_EDGE_ONLY_CHARTS = 2
FA_FLAG_FOOTPRINT_PUSH = 4
FA_TUNE_PACK_BLOCK, FA_TUNE_OCC_SMALL_TEXELS, FA_TUNE_UF_LINK_INIT, FA_TUNE_BATCH_GRAPH = 1, 2, 3, 4
FA_TUNE_UF_EDGE_HOOKS, FA_TUNE_OCC_LANE_TEXELS, FA_TUNE_UF_TILE = 5, 6, 7
FA_TUNE_BATCH_LAUNCH = 8


class fa_config(ctypes.Structure):
    _fields_ = [("device", c_int32), ("num_scales", c_int32), ("max_triangles", c_int64),
                ("max_vertices", c_int64), ("max_charts", c_int32), ("max_atlas", c_int32),
                ("gutter", c_int32), ("min_box", c_int32), ("flags", c_uint32),
                ("max_views", c_int32), ("max_profile_columns", c_int64),
                ("hbm_budget_bytes", c_int64)]


class fa_mesh(ctypes.Structure):
    _fields_ = [("positions", c_void_p), ("indices", c_void_p), ("num_vertices", c_int64),
                ("num_triangles", c_int64), ("scene_key", c_uint64)]


class fa_camera(ctypes.Structure):
    _fields_ = [("view_proj", c_float * 16), ("width", c_int32), ("height", c_int32)]


class fa_atlas_out(ctypes.Structure):
    _fields_ = [("chart_of_tri", c_void_p), ("chart_of_vert", c_void_p), ("uv", c_void_p),
                ("charts", c_void_p), ("occupancy", c_void_p), ("meta", c_void_p),
                ("candidates", c_void_p)]


class fa_view(ctypes.Structure):
    _fields_ = [("visible", c_void_p), ("cam", fa_camera), ("atlas_size", c_int32),
                ("texel_per_pixel", c_float), ("out", fa_atlas_out)]


CHART_DTYPE = np.dtype([("root_tri", "<i4"), ("x", "<i4"), ("y", "<i4"), ("w", "<i4"),
                        ("h", "<i4"), ("rotated", "<i4"), ("order_rank", "<i4"), ("key", "<i4"),
                        ("ndc_box", "<f4", (4,)), ("target_w", "<f4"), ("target_h", "<f4"),
                        ("oriented_w", "<f4"), ("oriented_h", "<f4")])
META_DTYPE = np.dtype([("status", "<i4"), ("num_charts", "<i4"), ("chosen_j", "<i4"),
                       ("num_scales", "<i4"), ("atlas_size", "<i4"), ("layout_width", "<i4"),
                       ("layout_height", "<i4"), ("rows", "<i4"), ("s_eff", "<f4"),
                       ("rate", "<f4"), ("occupied_texels", "<i8"), ("visible_triangles", "<i8"),
                       ("large_tiles", "<i8")])
assert CHART_DTYPE.itemsize == 64 and META_DTYPE.itemsize == 64

EXPORTS = ["fa_create", "fa_destroy", "fa_status_string", "fa_scene_adjacency", "fa_scene_evict",
           "fa_build_atlas", "fa_build_atlas_batch", "fa_pack_boxes", "fa_set_tuning",
           "fa_get_tuning", "fa_load_tuning_table", "fa_set_stage_timing", "fa_stage_times",
           "fa_visibility",
           "fa_reuse_flags", "fa_build_dual_atlas", "fa_build_atlas_static", "fa_device_bytes"]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2502_17712_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    lib.fa_create.argtypes = [POINTER(fa_config), POINTER(c_void_p)]
    lib.fa_create.restype = c_int
    lib.fa_destroy.argtypes = [c_void_p]
    lib.fa_destroy.restype = None
    lib.fa_status_string.argtypes = [c_int]
    lib.fa_status_string.restype = ctypes.c_char_p
    lib.fa_scene_adjacency.argtypes = [c_void_p, POINTER(fa_mesh), c_void_p, c_void_p]
    lib.fa_scene_evict.argtypes = [c_void_p, c_uint64]
    lib.fa_build_atlas.argtypes = [c_void_p, POINTER(fa_mesh), c_void_p, POINTER(fa_camera),
                                   c_int32, c_float, POINTER(fa_atlas_out), c_void_p]
    lib.fa_build_atlas_batch.argtypes = [c_void_p, POINTER(fa_mesh), c_int32, POINTER(fa_view),
                                         c_void_p]
    lib.fa_pack_boxes.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p,
                                  c_void_p, c_void_p]
    lib.fa_set_tuning.argtypes = [c_void_p, c_int, c_int]
    lib.fa_get_tuning.argtypes = [c_void_p, c_int]
    lib.fa_load_tuning_table.argtypes = [c_void_p, ctypes.c_char_p]
    lib.fa_set_stage_timing.argtypes = [c_void_p, c_int]
    lib.fa_stage_times.argtypes = [c_void_p, POINTER(c_float), c_int]
    lib.fa_visibility.argtypes = [c_void_p, POINTER(fa_mesh), POINTER(fa_camera),
                                  POINTER(c_double), c_double, c_int32, c_void_p, c_void_p]
    lib.fa_reuse_flags.argtypes = [c_void_p, POINTER(fa_mesh), POINTER(fa_camera), c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_void_p]
    lib.fa_build_dual_atlas.argtypes = [c_void_p, POINTER(fa_mesh), c_void_p, POINTER(fa_camera),
                                        c_int32, c_float, c_int32, POINTER(fa_atlas_out),
                                        c_void_p, c_void_p]
    lib.fa_device_bytes.argtypes = [c_void_p]
    lib.fa_device_bytes.restype = c_int64
    lib.fa_build_atlas_static.argtypes = [POINTER(fa_mesh), c_void_p, POINTER(fa_camera), c_int32,
                                          c_float, POINTER(fa_atlas_out), c_void_p]
    for n in ("fa_scene_adjacency", "fa_scene_evict", "fa_build_atlas", "fa_build_atlas_batch",
              "fa_pack_boxes", "fa_set_tuning", "fa_get_tuning", "fa_load_tuning_table",
              "fa_set_stage_timing",
              "fa_stage_times", "fa_visibility", "fa_reuse_flags", "fa_build_dual_atlas",
              "fa_build_atlas_static"):
        getattr(lib, n).restype = c_int
    return lib


_lib = _load()

# same names as the C ABI
fa_create = _lib.fa_create
fa_destroy = _lib.fa_destroy
fa_status_string = _lib.fa_status_string
fa_scene_adjacency = _lib.fa_scene_adjacency
fa_scene_evict = _lib.fa_scene_evict
fa_build_atlas = _lib.fa_build_atlas
fa_build_atlas_batch = _lib.fa_build_atlas_batch
fa_pack_boxes = _lib.fa_pack_boxes
fa_set_tuning = _lib.fa_set_tuning
fa_get_tuning = _lib.fa_get_tuning
fa_load_tuning_table = _lib.fa_load_tuning_table
fa_set_stage_timing = _lib.fa_set_stage_timing
fa_stage_times = _lib.fa_stage_times
fa_visibility = _lib.fa_visibility
fa_reuse_flags = _lib.fa_reuse_flags
fa_build_dual_atlas = _lib.fa_build_dual_atlas
fa_build_atlas_static = _lib.fa_build_atlas_static
fa_device_bytes = _lib.fa_device_bytes
STATIC_MAX_TRIANGLES, STATIC_MAX_VERTICES, STATIC_MAX_CHARTS = 65536, 65536, 4096

STAGES = ["prologue", "vis_scan", "vis_compact", "uf_hook", "uf_vertex_min", "uf_vertex_hook",
          "uf_flatten", "chart_scan", "assign_roots", "gather_boxes", "sizes_order", "fp_count",
          "fp_raster", "pack", "select_place", "uv", "occ_fill", "occ_small", "occ_big",
          "occ_count", "meta"]


class FastAtlasError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {fa_status_string(code).decode()} ({code})")
        self.code = code


def _check(code, what):
    if code != FA_OK:
        raise FastAtlasError(code, what)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def parse_meta(meta_tensor) -> dict:
    a = meta_tensor.detach().cpu().numpy().view(META_DTYPE)[0]
    return {k: a[k].item() for k in META_DTYPE.names}


def parse_charts(charts_tensor, n) -> np.ndarray:
    return charts_tensor.detach().cpu().numpy().view(CHART_DTYPE).reshape(-1)[:n].copy()


class Mesh:
    """Device copy of a mesh (positions float32 [V,3], indices int32 [T,3])."""

    def __init__(self, positions, indices, scene_key, device="cuda"):
        self.positions = torch.as_tensor(np.ascontiguousarray(positions, np.float32)).to(device)
        self.indices = torch.as_tensor(np.ascontiguousarray(indices, np.int32)).to(device)
        self.scene_key = int(scene_key)
        self.c = fa_mesh(self.positions.data_ptr(), self.indices.data_ptr(),
                         self.positions.shape[0], self.indices.shape[0], self.scene_key)

    @property
    def num_triangles(self):
        return int(self.indices.shape[0])

    @property
    def num_vertices(self):
        return int(self.positions.shape[0])


def make_camera(view_proj, width, height) -> fa_camera:
    cam = fa_camera()
    vp = np.asarray(view_proj, np.float32).ravel()
    for i in range(16):
        cam.view_proj[i] = float(vp[i])
    cam.width, cam.height = int(width), int(height)
    return cam


class AtlasOutputs:
    """Device output buffers of one view."""

    def __init__(self, T, V, max_charts, atlas_size, J, uv=True, occupancy=True,
                 candidates=True, device="cuda", uv_corners=False):
        self.chart_of_tri = torch.empty(T, dtype=torch.int32, device=device)
        self.chart_of_vert = torch.empty(V, dtype=torch.int32, device=device)
        # per vertex [V, 2], or per corner [T, 3, 2] for edge-connected charts
        uv_shape = (T, 3, 2) if uv_corners else (V, 2)
        self.uv = torch.empty(uv_shape, dtype=torch.float32, device=device) if uv else None
        self.charts = torch.zeros((max_charts, 16), dtype=torch.int32, device=device)
        self.occupancy = (torch.empty((atlas_size, atlas_size), dtype=torch.int32, device=device)
                          if occupancy else None)
        self.meta = torch.zeros(16, dtype=torch.int32, device=device)
        self.candidates = (torch.zeros((J, 4), dtype=torch.int32, device=device)
                           if candidates else None)
        self.atlas_size = atlas_size

    def c(self) -> fa_atlas_out:
        return fa_atlas_out(self.chart_of_tri.data_ptr(), self.chart_of_vert.data_ptr(),
                            None if self.uv is None else self.uv.data_ptr(),
                            self.charts.data_ptr(),
                            None if self.occupancy is None else self.occupancy.data_ptr(),
                            self.meta.data_ptr(),
                            None if self.candidates is None else self.candidates.data_ptr())

    def to_numpy(self) -> dict:
        m = parse_meta(self.meta)
        r = dict(meta=m, chart_of_tri=self.chart_of_tri.cpu().numpy(),
                 chart_of_vert=self.chart_of_vert.cpu().numpy(),
                 charts=parse_charts(self.charts, max(m["num_charts"], 0)
                                     if m["status"] in (FA_OK, FA_ERR_NOFIT) else 0))
        if self.uv is not None:
            r["uv"] = self.uv.cpu().numpy()
        if self.occupancy is not None:
            r["occupancy"] = self.occupancy.cpu().numpy()
        if self.candidates is not None:
            r["candidates"] = self.candidates.cpu().numpy()
        return r


def build_atlas_static(mesh: Mesh, visible, view_proj, width, height, atlas_size, rate,
                       out: AtlasOutputs = None, stream=None):
    """fa_build_atlas_static: one frame with no device allocation inside the
    library (fixed J = 64, gutter 1, min_box 2). `out` (allocated here when
    None) must have at least STATIC_MAX_CHARTS chart records."""
    if out is None:
        out = AtlasOutputs(mesh.num_triangles, mesh.num_vertices, STATIC_MAX_CHARTS, atlas_size, 64)
    cam = make_camera(view_proj, width, height)
    oc = out.c()
    _check(fa_build_atlas_static(ctypes.byref(mesh.c), _ptr(visible), ctypes.byref(cam),
                                 int(atlas_size), float(rate), ctypes.byref(oc),
                                 _stream_handle(stream)), "fa_build_atlas_static")
    return out


# Knobs by frame shape chosen by the project's autotuner on an MI355X
# (autotune.tune_table); every context loads it unless told otherwise.
TUNING_TABLE = os.path.join(_HERE, "tuning_gfx950.txt")


class Context:
    """Owns an fa_ctx (scratch + resident scene adjacency) on one device.
    tuning_table: path of a tuning table to load (default: TUNING_TABLE when
    the file exists; None: no table)."""

    def __init__(self, max_triangles, max_vertices, max_charts=65536, max_atlas=8192,
                 num_scales=64, gutter=1, min_box=2, flags=0, device=0, max_views=1,
                 max_profile_columns=0, hbm_budget_bytes=0, tuning_table="default"):
        cfg = fa_config(device, num_scales, max_triangles, max_vertices, max_charts, max_atlas,
                        gutter, min_box, flags, max_views, max_profile_columns, hbm_budget_bytes)
        h = c_void_p()
        _check(fa_create(ctypes.byref(cfg), ctypes.byref(h)), "fa_create")
        self.h = h
        self.cfg = cfg
        if tuning_table == "default":
            tuning_table = TUNING_TABLE if os.path.exists(TUNING_TABLE) else None
        if tuning_table is not None:
            with open(tuning_table) as fh:
                self.load_tuning_table(fh.read())

    def load_tuning_table(self, text: str):
        """Knobs by frame shape (fa_load_tuning_table); '' clears the table."""
        _check(fa_load_tuning_table(self.h, text.encode()), "fa_load_tuning_table")

    def close(self):
        if getattr(self, "h", None):
            fa_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_bytes(self):
        """Device bytes the context holds now (fa_device_bytes)."""
        return int(fa_device_bytes(self.h))

    def outputs(self, mesh: Mesh, atlas_size, uv=True, occupancy=True, candidates=True):
        return AtlasOutputs(mesh.num_triangles, mesh.num_vertices, self.cfg.max_charts, atlas_size,
                            self.cfg.num_scales, uv, occupancy, candidates,
                            uv_corners=bool(self.cfg.flags & FA_FLAG_EDGE_ONLY_CHARTS))

    def adjacency(self, mesh: Mesh, stream=None):
        nbr = torch.empty((mesh.num_triangles, 3), dtype=torch.int32, device="cuda")
        _check(fa_scene_adjacency(self.h, ctypes.byref(mesh.c), _ptr(nbr), _stream_handle(stream)),
               "fa_scene_adjacency")
        return nbr

    def visibility(self, mesh: Mesh, view_proj, width, height, eye, near, coarse=0, out=None,
                   stream=None):
        """Visible triangles of a view on the device: uint8 [T] (see fa_visibility)."""
        if out is None:
            out = torch.empty(mesh.num_triangles, dtype=torch.uint8, device="cuda")
        cam = make_camera(view_proj, width, height)
        e = (c_double * 3)(*[float(x) for x in eye])
        _check(fa_visibility(self.h, ctypes.byref(mesh.c), ctypes.byref(cam), e, float(near),
                             int(coarse), _ptr(out), _stream_handle(stream)), "fa_visibility")
        return out

    def reuse_flags(self, mesh: Mesh, key_view_proj, key_visible, visible, stream=None):
        """Temporal reuse flags (0 not visible, 1 reuse, 2 shade) and the reused count
        (a device int64 tensor), see fa_reuse_flags."""
        flags = torch.empty(mesh.num_triangles, dtype=torch.uint8, device="cuda")
        reused = torch.empty(1, dtype=torch.int64, device="cuda")
        cam = make_camera(key_view_proj, 1, 1)
        _check(fa_reuse_flags(self.h, ctypes.byref(mesh.c), ctypes.byref(cam), _ptr(key_visible),
                              _ptr(visible), _ptr(flags), _ptr(reused), _stream_handle(stream)),
               "fa_reuse_flags")
        return flags, reused

    def build_dual_atlas(self, mesh: Mesh, visible, view_proj, width, height, atlas_size, rate,
                         low_shift, out: AtlasOutputs = None, occupancy_low=None, stream=None):
        """fa_build_dual_atlas: returns (outputs, low-resolution occupancy map)."""
        if out is None:
            out = self.outputs(mesh, atlas_size)
        if occupancy_low is None:
            ol = int(atlas_size) >> int(low_shift)
            occupancy_low = torch.empty((ol, ol), dtype=torch.int32, device="cuda")
        cam = make_camera(view_proj, width, height)
        oc = out.c()
        _check(fa_build_dual_atlas(self.h, ctypes.byref(mesh.c), _ptr(visible), ctypes.byref(cam),
                                   int(atlas_size), float(rate), int(low_shift), ctypes.byref(oc),
                                   _ptr(occupancy_low), _stream_handle(stream)),
               "fa_build_dual_atlas")
        return out, occupancy_low

    def build_atlas(self, mesh: Mesh, visible, view_proj, width, height, atlas_size, rate,
                    out: AtlasOutputs = None, stream=None):
        if out is None:
            out = self.outputs(mesh, atlas_size)
        cam = make_camera(view_proj, width, height)
        oc = out.c()
        _check(fa_build_atlas(self.h, ctypes.byref(mesh.c), _ptr(visible), ctypes.byref(cam),
                              int(atlas_size), float(rate), ctypes.byref(oc),
                              _stream_handle(stream)), "fa_build_atlas")
        return out

    def build_atlas_batch(self, mesh: Mesh, views, outs, stream=None):
        """views: list of (visible, view_proj, width, height, atlas_size, rate)."""
        arr = (fa_view * len(views))()
        for i, (vis, vp, W, H, om, r) in enumerate(views):
            arr[i].visible = vis.data_ptr()
            arr[i].cam = make_camera(vp, W, H)
            arr[i].atlas_size = int(om)
            arr[i].texel_per_pixel = float(r)
            arr[i].out = outs[i].c()
        _check(fa_build_atlas_batch(self.h, ctypes.byref(mesh.c), len(views), arr,
                                    _stream_handle(stream)), "fa_build_atlas_batch")
        return outs

    def pack_boxes(self, sizes, atlas_size, stream=None):
        """sizes: float32 cuda tensor [n,2]. Returns (placements [n,5], meta, candidates)."""
        n = int(sizes.shape[0])
        pl = torch.empty((max(n, 1), 5), dtype=torch.int32, device="cuda")
        meta = torch.zeros(16, dtype=torch.int32, device="cuda")
        cand = torch.zeros((self.cfg.num_scales, 4), dtype=torch.int32, device="cuda")
        _check(fa_pack_boxes(self.h, _ptr(sizes), n, int(atlas_size), _ptr(pl), _ptr(meta),
                             _ptr(cand), _stream_handle(stream)), "fa_pack_boxes")
        return pl[:n], meta, cand

    def set_tuning(self, knob, value):
        _check(fa_set_tuning(self.h, int(knob), int(value)), "fa_set_tuning")

    def get_tuning(self, knob):
        return int(fa_get_tuning(self.h, int(knob)))

    def set_stage_timing(self, enable=True):
        _check(fa_set_stage_timing(self.h, int(enable)), "fa_set_stage_timing")

    def stage_times(self):
        buf = (c_float * 32)()
        n = fa_stage_times(self.h, buf, 32)
        return {STAGES[i]: buf[i] for i in range(n)}
