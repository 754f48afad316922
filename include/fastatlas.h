/*
 * fastatlas.h - C ABI of the MI355X (gfx950) per-frame atlasing library.
 *
 * The library implements the per-frame part of FastAtlas ("FastAtlas:
 * Real-Time Compact Atlases for Texture Space Shading", Vining et al.,
 * Eurographics 2025): it groups the visible triangles of a frame into charts
 * (Sec. "Chart Computation", Appendix "GPU Union Find", Alg. 1), bounds each
 * chart's visible projection (Sec. "Computing Bounding Boxes of Projected
 * Visible Sub-Charts"), orders the boxes (Sec. "Box Ordering via Cuckoo
 * Hashing"), searches J candidate scales and packs the boxes into a fixed
 * omega x omega atlas (Secs. "Parallel Atlas and Scale Factor Computation",
 * "Box Packing"), and maps every chart vertex into the atlas (Appendix
 * "Shading and Rasterization").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array pointer is a DEVICE pointer on the context's device, owned by
 *   the caller, unless a comment says "host". The context owns its scratch
 *   memory and the resident per-scene adjacency.
 * - Calls enqueue work on `stream` (a hipStream_t; NULL = the legacy default
 *   stream) and return immediately. Inputs must stay alive and unmodified and
 *   outputs must not be read until that work has completed.
 * - The synchronous return value reports argument and capacity errors found
 *   on the host (FA_ERR_INVALID_ARG, FA_ERR_CAPACITY, FA_ERR_OUT_OF_MEMORY,
 *   FA_ERR_DEVICE). Conditions discovered on the device (no candidate scale
 *   fits: FA_ERR_NOFIT; more charts than max_charts: FA_ERR_CAPACITY; a
 *   bounded wait between the workgroups of the chart order of a frame with
 *   more than 2048 charts (1024 for fa_pack_boxes) that gave up, which the
 *   ordering's design rules out
 *   short of a device fault: FA_ERR_DEVICE) are written to meta->status when
 *   the stream work completes.
 * - A context is not thread-safe: use it from one host thread at a time.
 *   Calls on one context must not overlap on different streams (they share
 *   the context's scratch); use one context per concurrent stream.
 * - Float arithmetic is IEEE float32 in a fixed order without contraction, so
 *   every integer result (chart ids, sizes, placements, occupancy) is exactly
 *   reproducible.
 */
#ifndef FASTATLAS_H
#define FASTATLAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum fa_status {
  FA_OK = 0,
  FA_ERR_INVALID_ARG = 1,   /* bad pointer, size, atlas size or rate          */
  FA_ERR_OUT_OF_MEMORY = 2, /* device allocation failed                       */
  FA_ERR_CAPACITY = 3,      /* above max_triangles / max_vertices / max_charts */
  FA_ERR_NOFIT = 4,         /* no candidate scale fits the atlas              */
  FA_ERR_DEVICE = 5,        /* a HIP call failed, or the device is not gfx950 */
  FA_ERR_UNSUPPORTED = 6
};

/* Option bits of fa_config.flags. */
enum {
  /* Clip straddling triangles against the near plane only (Blinn's estimate
     otherwise); the default also tries the side and far planes and keeps the
     smallest box (Sec. bounding boxes). */
  FA_FLAG_NO_SIDE_CLIP = 1u << 0,
  /* Edge-connected charts (Sec. "Chart Computation": charts grow across
     shared edges): visible triangles are joined across shared undirected
     edges only, without the vertex merge of Appendix "GPU Union Find", so a
     vertex can belong to several charts. Then uv is per corner: [T][3][2],
     corner k of triangle t at uv[(3t + k) * 2], mapped through the chart of
     t (NaN for invisible triangles and corners with w <= 0), and
     chart_of_vert[v] is the smallest chart index among the visible
     triangles using v. The union-find hook-mode knob chooses between a
     global edge hook (1) and LDS tiles of shared edges plus the edges
     between tiles (any other value). */
  FA_FLAG_EDGE_ONLY_CHARTS = 1u << 1,
  /* Footprint-aware push (Sec. "Box Packing" generalized to non-rectangular
     footprints): each chart's footprint is measured once per frame as a
     full-scale per-column profile (top and bottom row of every unit column of
     its chart-local layout, geometry outside the chart frame folded onto the
     border cells), pooled exactly to each candidate scale and dilated by the
     gutter; the push raises a box until its profile, not its full box, meets
     the frontline. Sizes, fold, overflow, mirrored rows and selection are the
     box packer's; boxes may overlap where their footprints do not. Needs a
     gutter >= 1 (fa_create returns FA_ERR_INVALID_ARG otherwise); not
     available with fa_build_dual_atlas (FA_ERR_UNSUPPORTED). fa_pack_boxes
     has no footprints and always uses the box push. */
  FA_FLAG_FOOTPRINT_PUSH = 1u << 2
};

typedef struct fa_config {
  int32_t device;        /* HIP device ordinal                                  */
  int32_t num_scales;    /* J candidate scales j/J, 1..64 (paper: 64)           */
  int64_t max_triangles; /* capacity, >= every mesh's triangle count            */
  int64_t max_vertices;  /* capacity, >= every mesh's vertex count              */
  int32_t max_charts;    /* capacity for charts per frame (<= 1048576)          */
  int32_t max_atlas;     /* largest atlas side, power of two 16..8192           */
  int32_t gutter;        /* texels added on each side of every box (usually 1)  */
  int32_t min_box;       /* minimum box side in texels before the gutter (2)    */
  uint32_t flags;        /* FA_FLAG_*                                           */
  int32_t max_views;     /* views per fa_build_atlas_batch call (>= 1)          */
  int64_t max_profile_columns; /* with FA_FLAG_FOOTPRINT_PUSH: capacity for the
                              full-scale profile columns of one frame, the sum
                              over charts of floor(oriented width) + 1 (0: 64 x
                              max_atlas; at most 2^28); a frame above it ends
                              with FA_ERR_CAPACITY in meta->status          */
  int64_t hbm_budget_bytes; /* cap on the device memory the context holds
                              (scratch, resident scene adjacency, visibility
                              buffers); 0: no cap. fa_create fails with
                              FA_ERR_OUT_OF_MEMORY when the scratch alone
                              exceeds it. Before a new scene's adjacency
                              (12 B per triangle, plus its sort buffers while
                              it is built) or a larger visibility buffer
                              would exceed it, the least recently used
                              resident scenes are evicted (after waiting for
                              the device); if it still does not fit, the call
                              returns FA_ERR_OUT_OF_MEMORY                   */
} fa_config;

typedef struct fa_mesh {
  const float* positions;   /* [V][3] object-space xyz                          */
  const int32_t* indices;   /* [T][3] vertex indices, 0 <= i < V                 */
  int64_t num_vertices;     /* V                                                */
  int64_t num_triangles;    /* T                                                */
  uint64_t scene_key;       /* adjacency is built once per key and kept resident */
} fa_mesh;

typedef struct fa_camera {
  float view_proj[16]; /* host: row-major 4x4, clip = M * (x, y, z, 1), GL clip
                          volume -w <= x, y, z <= w                             */
  int32_t width;       /* viewport in pixels                                   */
  int32_t height;
} fa_camera;

/* One chart of the frame (64 bytes). Layout-space boxes are integers in a
 * square of side layout_width L; atlas texel = layout * atlas_size / L. */
typedef struct fa_chart {
  int32_t root_tri;   /* lowest triangle index of the chart                     */
  int32_t x, y;       /* layout-space top-left of the box (gutter included)     */
  int32_t w, h;       /* layout-space box size (gutter included)                */
  int32_t rotated;    /* 1: turned 90 degrees so the box is at least as tall    */
  int32_t order_rank; /* position in the packing order                          */
  int32_t key;        /* ordering key: min(ceil(oriented height), 8191)         */
  float ndc_box[4];   /* conservative NDC box x0, y0, x1, y1                    */
  float target_w;     /* screen size in pixels times rate (before rotation)    */
  float target_h;
  float oriented_w;   /* target size after the optional rotation               */
  float oriented_h;
} fa_chart;

typedef struct fa_atlas_meta {
  int32_t status;        /* fa_status of the device-side work                    */
  int32_t num_charts;    /* C                                                    */
  int32_t chosen_j;      /* chosen candidate j (scale j over J), 0 if none fits  */
  int32_t num_scales;    /* J                                                    */
  int32_t atlas_size;    /* omega                                                */
  int32_t layout_width;  /* L = omega + horizontal overflow of the chosen scale  */
  int32_t layout_height; /* H, highest box top of the chosen packing            */
  int32_t rows;          /* folded rows of the chosen packing                    */
  float s_eff;           /* effective uniform scale (j / J) times omega / L      */
  float rate;            /* requested texels per pixel (per axis)                */
  int64_t occupied_texels; /* texels claimed in the occupancy map (0 if none)    */
  int64_t visible_triangles;
  int64_t large_tiles;   /* diagnostic: 16x16-texel tiles rasterized cooperatively
                            (depends on the small_texels knob)                  */
} fa_atlas_meta;

typedef struct fa_atlas_out {
  int32_t* chart_of_tri;  /* [T] chart index, -1 for invisible triangles        */
  int32_t* chart_of_vert; /* [V] chart index, -1 if unused; may be NULL         */
  float* uv;              /* [V][2] atlas texels, origin top-left, v down; NaN
                             when the vertex is unmapped or has w <= 0; may be
                             NULL. [T][3][2] per corner with
                             FA_FLAG_EDGE_ONLY_CHARTS                         */
  fa_chart* charts;       /* [max_charts]                                       */
  int32_t* occupancy;     /* [omega][omega] owning chart or -1; may be NULL      */
  fa_atlas_meta* meta;    /* [1]                                                */
  int32_t* candidates;    /* [J][4] per candidate j (row j - 1): fit (1: the
                             packing fits the atlas), m, L, H; may be NULL.
                             m and L are exact for every candidate; H is the
                             packing height when fit = 1, and when fit = 0
                             either -1 (rejected before the push: overflow
                             m > omega, or a box side above 2 omega) or a
                             height above L at which the push stopped      */
} fa_atlas_out;

typedef struct fa_view {
  const uint8_t* visible; /* [T] 0/1 visible-triangle buffer                    */
  fa_camera cam;
  int32_t atlas_size;
  float texel_per_pixel;
  fa_atlas_out out;
} fa_view;

typedef struct fa_ctx fa_ctx;

/* Create a context on cfg->device: checks the device is gfx950 and allocates
 * scratch sized from the capacities. Unset fields (0) take defaults: J=64,
 * min_box=2, max_atlas=8192, max_charts=65536, max_views=1, no memory cap
 * (gutter 0 means no gutter; the usual value is 1).
 * Returns FA_OK and *out_ctx, or an error and *out_ctx = NULL. */
int fa_create(const fa_config* cfg, fa_ctx** out_ctx);

/* Free the context, its scratch and every resident scene. No work may be in
 * flight on the context. */
void fa_destroy(fa_ctx* ctx);

/* Device bytes the context holds now (scratch, resident scenes, visibility
 * buffers; see fa_config.hbm_budget_bytes), or -1 for a NULL context. */
int64_t fa_device_bytes(const fa_ctx* ctx);

const char* fa_status_string(int status);

/* Build (or reuse) the resident triangle adjacency of mesh->scene_key: the
 * twin relation of the half-edge structure in the paper's data-structure
 * table. Half-edge h = 3t+e joins indices[t][e] -> indices[t][(e+1)%3];
 * half-edges with the same undirected edge, taken in order of h, point to
 * the triangle of the next one cyclically; lone and degenerate edges give -1.
 * nbr_out ([T][3], may be NULL) receives a copy. */
int fa_scene_adjacency(fa_ctx* ctx, const fa_mesh* mesh, int32_t* nbr_out, void* stream);

/* Drop the resident adjacency of one scene (no work may be in flight). */
int fa_scene_evict(fa_ctx* ctx, uint64_t scene_key);

/* Visible triangles of a view (App. "Detecting Visible Triangles": a depth
 * pre-pass, then every triangle's samples are tested against the depth buffer
 * with "less or equal" and the triangles that pass are marked). float64.
 * A triangle is a candidate iff it faces the eye, (b-a) x (c-a) . (eye-a) > 0
 * with positions a, b, c, and no clip plane (-w <= x, y, z <= w, clip =
 * view_proj * (x, y, z, 1)) has all three vertices outside. coarse = 0:
 * visible = candidate. coarse = k > 0: a depth buffer of (W/k) x (H/k)
 * samples at pixel centres (x right, y down) is filled by the candidates whose
 * three w exceed near_w, with the NDC z interpolated by edge-function
 * weights; such a candidate stays visible iff it covers no sample or one of
 * its samples has z <= depth + 1e-6; candidates crossing the near plane stay
 * visible. eye: world-space camera position (3 doubles, host); near_w: w at
 * the near plane (> 0). visible: device [T], written 0/1. Uses the context's
 * visibility scratch; the first call at a larger coarse grid allocates it
 * (later calls with grids up to that size allocate nothing). Errors:
 * FA_ERR_INVALID_ARG (null pointers, bad sizes, coarse outside 0..64,
 * non-finite camera, near_w <= 0, out-of-range indices), FA_ERR_CAPACITY
 * (mesh larger than the context). */
int fa_visibility(fa_ctx* ctx, const fa_mesh* mesh, const fa_camera* cam, const double* eye,
                  double near_w, int32_t coarse, uint8_t* visible, void* stream);

/* Temporal reuse classification (Sec. "Temporal Reuse"): after a key frame
 * whose atlas was shaded in full, a later frame only re-shades triangles that
 * are newly visible or were partially visible in the key frame (a vertex with
 * max(|x|, |y|) >= w in the key frame's clip space, float32, clip =
 * key_cam->view_proj * (x, y, z, 1) summed left to right); the rest reuse the
 * key frame's shading. flags: device [T], 0 = not visible now, 1 = reuse,
 * 2 = shade. key_visible, visible: device [T] 0/1. reused: device int64 [1]
 * receiving the number of 1 flags, or NULL. Errors: FA_ERR_INVALID_ARG (null
 * pointers, non-finite camera, out-of-range indices), FA_ERR_CAPACITY. */
int fa_reuse_flags(fa_ctx* ctx, const fa_mesh* mesh, const fa_camera* key_cam,
                   const uint8_t* key_visible, const uint8_t* visible, uint8_t* flags,
                   int64_t* reused, void* stream);

/* Atlas one frame: charts, boxes, order, J-candidate packing, selection,
 * per-vertex UVs and (if out->occupancy) the atlas occupancy map.
 * visible: [T] 0/1. atlas_size: power of two, 16 <= atlas_size <= max_atlas.
 * texel_per_pixel: rate r > 0, per axis (paper's shading-rate multiplier). */
int fa_build_atlas(fa_ctx* ctx, const fa_mesh* mesh, const uint8_t* visible,
                   const fa_camera* cam, int32_t atlas_size, float texel_per_pixel,
                   fa_atlas_out* out, void* stream);

/* Atlas one frame as fa_build_atlas, plus the occupancy of the same packing
 * in a low-resolution companion atlas of side atlas_size >> low_shift (App.
 * "Depth-of-Field" and "Foveated Rendering": one packing serves a full-rate
 * atlas and a reduced-rate one, its coordinates scaled by 2^-low_shift per
 * axis; the caller's UVs for it are uv * 2^-low_shift). occupancy_low: device
 * [(atlas_size >> low_shift)^2], the same definition as the occupancy map
 * with omega = atlas_size >> low_shift (meta->occupied_texels stays the
 * full-rate count). To keep charts apart in the low atlas, configure a gutter
 * of at least 2^low_shift texels (charts whose triangles leave the view can
 * still reach their box edge). low_shift: 1..6, atlas_size >> low_shift >= 16.
 * Errors as fa_build_atlas, plus FA_ERR_INVALID_ARG for a bad low_shift or a
 * null occupancy_low, and FA_ERR_UNSUPPORTED on a context created with
 * FA_FLAG_FOOTPRINT_PUSH (overlapping boxes can share texels at the lower
 * resolution). */
int fa_build_dual_atlas(fa_ctx* ctx, const fa_mesh* mesh, const uint8_t* visible,
                        const fa_camera* cam, int32_t atlas_size, float texel_per_pixel,
                        int32_t low_shift, fa_atlas_out* out, int32_t* occupancy_low,
                        void* stream);

/* Atlas n views of one mesh (views: host array of n descriptors, each with its
 * own visibility, camera, atlas size, rate and outputs). Views run
 * concurrently on the context's max_views scratch slots and streams, forked
 * from and joined back into `stream`. Every view's results equal what
 * fa_build_atlas gives for it. The outputs of different views must not
 * overlap. */
int fa_build_atlas_batch(fa_ctx* ctx, const fa_mesh* mesh, int32_t n, const fa_view* views,
                         void* stream);

/* FastAtlas packing alone (Sec. "FastAtlas Packing": its only input is the
 * box dimensions). sizes: [n][2] box width and height in texels at scale 1.
 * Boxes are oriented, ordered by (ceil(height) desc, index asc), packed at J
 * candidate scales and the best fitting one is chosen.
 * placements: [n][5] x, y, w, h, rotated (layout space, gutter included).
 * meta: as for fa_build_atlas (num_charts = n, no occupancy). */
int fa_pack_boxes(fa_ctx* ctx, const float* sizes, int32_t n, int32_t atlas_size,
                  int32_t* placements, fa_atlas_meta* meta, int32_t* candidates, void* stream);

/* Allocation-free atlasing, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). The same frame as fa_build_atlas with a fixed configuration
 * (J = 64, gutter 1, min_box 2, no flags, default knobs) and no context:
 * every scratch buffer, including the triangle adjacency (rebuilt on every
 * call, nothing stays resident), lives in one static device array of
 * FA_STATIC_SCRATCH_MIB MiB that each device holds for the life of the
 * process. The call allocates nothing and never synchronizes; it runs on the
 * current device and enqueues on `stream`. Limits: T <= FA_STATIC_MAX_TRIANGLES,
 * V <= FA_STATIC_MAX_VERTICES (FA_ERR_CAPACITY above them), at most
 * FA_STATIC_MAX_CHARTS charts (FA_ERR_CAPACITY in meta->status),
 * atlas_size a power of two 16..8192. Out-of-range indices are found on the
 * device: meta->status = FA_ERR_INVALID_ARG and no other output is valid.
 * Arguments, outputs and the other errors are as for fa_build_atlas
 * (candidates, when given, has 64 rows). Every call on a device shares that
 * device's array, which keeps the last call's contents: calls that overlap
 * on one device (different streams, or different host threads) race, so
 * order them on one stream. The first call on a device sets it up (device
 * check, address of its copy of the array) and returns FA_ERR_DEVICE if the
 * device is not gfx950. */
#define FA_STATIC_MAX_TRIANGLES 65536
#define FA_STATIC_MAX_VERTICES 65536
#define FA_STATIC_MAX_CHARTS 4096
#define FA_STATIC_SCRATCH_MIB 24
int fa_build_atlas_static(const fa_mesh* mesh, const uint8_t* visible, const fa_camera* cam,
                          int32_t atlas_size, float texel_per_pixel, fa_atlas_out* out,
                          void* stream);

/* Performance knobs of one context. Every accepted value produces identical
 * results; only the speed changes (an autotuner may pick any of them).
 *   FA_TUNE_PACK_BLOCK        threads per candidate packing: 256, 512, 1024
 *   FA_TUNE_OCC_SMALL_TEXELS  footprints (texel range of a fan triangle) of
 *                             more texels are queued and cut into 16x16
 *                             tiles shared by all waves (0..4096, default 64)
 *   FA_TUNE_OCC_LANE_TEXELS   footprints up to this many texels are
 *                             rasterized by one lane (scattered stores);
 *                             larger ones (up to FA_TUNE_OCC_SMALL_TEXELS)
 *                             by their wave, 64 texels per step with
 *                             coalesced stores (0..4096, default 64)
 *   FA_TUNE_UF_LINK_INIT      1: a triangle starts linked to its smallest
 *                             visible edge neighbour (Alg. 1); 0: to itself
 *                             (used when FA_TUNE_UF_EDGE_HOOKS is 0 or 1)
 *   FA_TUNE_UF_EDGE_HOOKS     1: join across shared edges, then across shared
 *                             vertices (Alg. 1); 2: shared edges
 *                             inside tiles of 2048 visible triangles joined in
 *                             LDS first, then the edges between tiles, then
 *                             vertices; 3: the tiles in LDS, then vertices
 *                             (edges between tiles are shared vertices);
 *                             4: as 3, with the vertex minima taken from the
 *                             tiles' local roots in the same pass;
 *                             5 (default): as 4, tiles of 2048 entries joined
 *                             in LDS through shared vertices (an LDS hash
 *                             table of vertex ids) instead of shared edges;
 *                             0: vertices only
 *                             (every shared edge is a shared vertex: the
 *                             charts are the same for all six)
 *   FA_TUNE_UF_TILE           visible-list entries per LDS union-find tile
 *                             (modes 2, 3, 4): 2048, 4096 (default), 8192
 *   FA_TUNE_BATCH_GRAPH       1: fa_build_atlas_batch captures its views into
 *                             a hipGraph once per distinct set of view
 *                             descriptors and replays it (one launch); 0: off
 *   FA_TUNE_BATCH_LAUNCH      1: fa_build_atlas_batch runs every stage of up to
 *                             max_views views as one kernel launch (one grid
 *                             row of workgroups per view), when the context
 *                             uses hook mode 5 and neither
 *                             FA_FLAG_FOOTPRINT_PUSH nor FA_FLAG_EDGE_ONLY_CHARTS,
 *                             every view has uv and occupancy outputs, the
 *                             mesh has triangles and n <= 256; otherwise (and
 *                             with 0, the default) each view is launched on
 *                             its own slot stream
 * fa_set_tuning returns FA_ERR_INVALID_ARG for unknown knobs or values;
 * fa_get_tuning returns the current value or -1. */
enum { FA_TUNE_PACK_BLOCK = 1, FA_TUNE_OCC_SMALL_TEXELS = 2, FA_TUNE_UF_LINK_INIT = 3,
       FA_TUNE_BATCH_GRAPH = 4, FA_TUNE_UF_EDGE_HOOKS = 5, FA_TUNE_OCC_LANE_TEXELS = 6,
       FA_TUNE_UF_TILE = 7, FA_TUNE_BATCH_LAUNCH = 8 };
int fa_set_tuning(fa_ctx* ctx, int knob, int value);
int fa_get_tuning(fa_ctx* ctx, int knob);

/* Knobs by frame shape, as an autotuner writes them (text in host memory,
 * copied; it replaces the context's previous table). One entry per line, '#'
 * starts a comment:
 *   t_lo t_hi omega J pack_block small_texels lane_texels uf_link_init
 *   uf_edge_hooks uf_tile
 * A frame on a mesh of T triangles (fa_mesh.num_triangles, not the visible
 * count) at atlas side omega with the context's J uses the first entry with
 * t_lo <= T <= t_hi, omega equal (0: any) and J equal (0:
 * any); frames no entry matches use the fa_set_tuning values. Applies to
 * fa_build_atlas, fa_build_dual_atlas and the per-view batch path; batched
 * launches take pack_block, small_texels and lane_texels from the entry
 * every view of the call matches (the context's values when the views match
 * different entries) and always run the vertex-hashed union-find tiles.
 * Results never depend on the knobs.
 * Errors: FA_ERR_INVALID_ARG for a null argument, a malformed line or a value
 * fa_set_tuning would refuse (the previous table is kept). An empty text
 * clears the table. */
int fa_load_tuning_table(fa_ctx* ctx, const char* text);

/* Per-kernel timing: when enabled, fa_build_atlas (with uv and occupancy
 * outputs) records an event after each of its 21 stages (a stage is one
 * kernel, or none when the configuration folds it into another); fa_stage_times
 * (after the stream completed) fills up to n floats with milliseconds for, in
 * order: prologue (state, per-vertex and per-triangle scratch, union-find
 * start), vis_scan,
 * vis_compact (list of the visible triangles), uf_hook, uf_vertex_min,
 * uf_vertex_hook, uf_flatten, chart_scan, assign_roots, gather_boxes,
 * sizes_order, fp_count, fp_raster (footprint profiles: item counts and
 * profile clear, then the item scan and the balanced raster; empty without
 * FA_FLAG_FOOTPRINT_PUSH), pack, select_place, uv, occ_fill, occ_small,
 * occ_big, occ_count, meta; it returns the number filled (0 if none recorded).
 * Enabling costs a little host time and device idle time between kernels. */
int fa_set_stage_timing(fa_ctx* ctx, int enable);
int fa_stage_times(fa_ctx* ctx, float* ms_host, int n);

#ifdef __cplusplus
}
#endif

#endif /* FASTATLAS_H */
