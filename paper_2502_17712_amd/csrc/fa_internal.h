// Internal declarations of the gfx950 atlasing library: device-side frame
// state, per-frame parameters, wave/block primitives and the host-side launch
// functions of each stage. Not part of the public ABI (include/fastatlas.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fastatlas.h"

namespace fa {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // default threads per workgroup
constexpr int kMaxScales = 64;       // J <= 64 candidate scales
constexpr int kKeyCap = 8191;        // height keys are 13-bit (max box height 8192)
constexpr int kTriTile = 1024;       // triangles per workgroup in the root scan
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortTile = 2048;      // keys per workgroup in one radix pass
constexpr int kCandStride = 8;       // int32 per candidate in the table
constexpr int kMaxAtlas = 8192;
constexpr int kCountGrid = 256;      // workgroups of the occupancy count
constexpr int kOrderGroups = 32;     // workgroups of the chart order above 1024 charts
static_assert(kOrderGroups <= kCountGrid, "the order's chunk sums use Work::partial");
constexpr int kOccBigGrid = 2048;    // blocks of the large-footprint raster
constexpr int64_t kBigCap = 1 << 20; // queue capacity (more: rasterized where found)


// Device-resident results of one frame that later stages read (kept on the
// device so that no stage needs a host round trip).
struct FrameState {
  int32_t status;
  int32_t num_charts;
  int32_t jstar;
  int32_t layout_w;
  int32_t layout_h;
  int32_t rows;
  float s_star;       // j*/J
  float q_star;       // omega/L*
  int32_t visible;    // visible triangles (length of the visible list)
  int32_t fp_columns; // full-scale footprint profile columns of the frame (footprint push)
  unsigned long long occupied;
  uint32_t ticket;    // workgroups of the occupancy count that have finished
  uint32_t order_claim[5];  // many-chart order: chunks claimed per phase
  uint32_t order_done[4];   // ... and chunks finished per phase
};

// Constants of one visibility pass, passed by value (float64).
struct VisParams {
  double M[16];   // view_proj, row-major
  double eye[3];  // camera position
  double near_w;  // w at the near plane
  int32_t Wc, Hc; // depth-buffer samples per row and column
  int32_t coarse; // 0: facing and frustum only
};

// Key-frame camera of the temporal reuse classification (float32).
struct KeyClip {
  float M[16];
};

// Per-frame constants passed by value.
struct FrameParams {
  float M[16];
  int32_t W, H;
  int32_t omega, log2omega;
  float rate;
  int32_t J, gutter, min_box;
  uint32_t flags;
  int32_t max_charts;
  int32_t edge_hooks;  // union-find edge hooks: 0 none, 1 global, 2 LDS tiles + between tiles, 3 LDS
                       // tiles, 4 LDS tiles that also lower the vertex minima, 5 LDS tiles joined
                       // through shared vertices
  int32_t uf_tile;     // visible-list entries per LDS union-find tile (2048, 4096, 8192)
  int32_t fp_cap;      // footprint push: capacity of the profile columns (0: box push)
  int64_t pool_stride; // footprint push: pooled profile entries per candidate
};

// Clip position of vertex v: clip = M (x, y, z, 1)^T, each row summed left to
// right. The one definition every kernel uses, so that every reader of a
// vertex gets the same bits; the frame stores no clip positions (reading the
// 12-byte position costs less than writing and reading back 16 bytes).
__device__ __forceinline__ float4 clip_of(const float* __restrict__ pos, int64_t v,
                                          const FrameParams& p) {
  const float x = pos[3 * v], y = pos[3 * v + 1], z = pos[3 * v + 2];
  float r[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float acc = p.M[4 * i] * x;
    acc = acc + p.M[4 * i + 1] * y;
    acc = acc + p.M[4 * i + 2] * z;
    r[i] = acc + p.M[4 * i + 3];
  }
  return make_float4(r[0], r[1], r[2], r[3]);
}

// Scratch buffers of one context (sized by the capacities).
struct Work {
  const float* pos;      // [V][3] the frame's mesh positions (set per frame; clip positions are
                         // computed where they are read, with clip_of)
  int32_t* parent;       // [T]
  int32_t* vmin;         // [V]
  int32_t* cov;          // [V] when the caller passes no chart_of_vert
  uint32_t* tile_count;  // [T/kTriTile + 1]
  uint32_t* tile_vis;    // [T/kTriTile + 1] visible triangles per tile
  uint32_t* accum;       // [max_charts][4] order-preserving encoded min/max
  uint32_t* keys_a;      // [max_charts]
  int32_t* vals_a;
  uint32_t* keys_b;
  int32_t* vals_b;
  uint32_t* hist;        // [kRadix * max(tiles(max_charts), kOrderGroups)]
  float2* sorted_wh;     // [max_charts] oriented sizes in packing order
  long long* cand_x;     // [J][max_charts] prefix sums
  uint32_t* cand_ab;     // [J][max_charts] a | b << 16
  int32_t* cand_y;       // [J][max_charts]
  int32_t* cand_tab;     // [J][kCandStride] fit, m, L, H, rows
  int32_t* vlist;        // [T] visible triangles in ascending order
  unsigned long long* partial;  // [kCountGrid] per-block occupied texel counts
  ulonglong2* big;       // [kBigCap] queued large occupancy footprints: code, tiles
  int4* big_fp;          // [kBigCap][3] their footprints (edge data, texel range, chart)
  unsigned long long* big_counter; // [1] queued footprints << 40 | queued tiles
  fa_chart* pack_charts; // [max_charts] chart records of the packer-only entry
  int32_t* cand_rs;      // [J][max_charts + 1] row starts of each candidate (frames above
                         // the LDS capacity of the packer)
  int4* chart_tex;       // [max_charts] texel range of each placed box (lo_x, hi_x, lo_y, hi_y)
  int32_t* fp_off;       // [max_charts + 1] first profile column of each chart (footprint push)
  int2* fp_prof;         // [max_profile_columns] full-scale (top, bottom) row of each column
  unsigned long long* fp_group;  // [T/64 + 2] profile-raster items of each group of 64 list entries,
                         // then their exclusive prefix and the total
  uint32_t* fp_pool;     // [J][pool_stride] pooled profile of every box at every candidate
  FrameState* state;     // [1]
};

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ unsigned long long lanes_below() {
  return (1ull << lane_id()) - 1ull;
}

// Order-preserving map float -> uint32 (after turning -0 into +0), so that
// integer atomics compute exact float min/max independent of order.
__device__ __forceinline__ uint32_t ord_of(float f) {
  f = f + 0.0f;
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float float_of(uint32_t e) {
  return __uint_as_float((e & 0x80000000u) ? (e & 0x7FFFFFFFu) : ~e);
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (T)__shfl_xor(v, o, kWave));
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (T)__shfl_xor(v, o, kWave));
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += (T)__shfl_xor(v, o, kWave);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T u = (T)__shfl_up(v, o, kWave);
    if (l >= o) v += u;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_incl_max_scan(T v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T u = (T)__shfl_up(v, o, kWave);
    if (l >= o) v = max(v, u);
  }
  return v;
}

// Block-wide inclusive sum scan; `sh` holds blockDim.x/64 elements. Ends
// with a barrier so `sh` may be reused afterwards. *total gets the block sum.
template <typename T>
__device__ __forceinline__ T block_incl_scan(T v, T* sh, T* total) {
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  T x = wave_incl_scan(v);
  if (lane_id() == kWave - 1) sh[w] = x;
  __syncthreads();
  T before = 0, all = 0;
  for (int k = 0; k < nw; ++k) {
    T s = sh[k];
    if (k < w) before += s;
    all += s;
  }
  __syncthreads();
  *total = all;
  return x + before;
}

template <typename T>
__device__ __forceinline__ T block_max(T v, T* sh) {
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  T x = wave_max(v);
  if (lane_id() == 0) sh[w] = x;
  __syncthreads();
  T m = sh[0];
  for (int k = 1; k < nw; ++k) m = max(m, sh[k]);
  __syncthreads();
  return m;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  T x = wave_sum(v);
  if (lane_id() == 0) sh[w] = x;
  __syncthreads();
  T m = 0;
  for (int k = 0; k < nw; ++k) m += sh[k];
  __syncthreads();
  return m;
}

// ---------------------------------------------------------------------------
// cross-lane primitives on the DPP (data-parallel primitives) network: the
// lane moves ride on VALU instructions instead of LDS permutes. Every lane of
// the wave must be active.
// ---------------------------------------------------------------------------
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  // lanes without a source (outside their row, or rows not in ROWS) read 0
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ int dpp_keep(int v) {
  // lanes without a source keep their own value
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}

// Maximum over each row of 16 lanes; every lane of the row receives it
// (pairs, quads, half rows, rows).
__device__ __forceinline__ int row16_max(int v) {
  v = max(v, dpp_keep<0xB1>(v));   // quad_perm [1, 0, 3, 2]
  v = max(v, dpp_keep<0x4E>(v));   // quad_perm [2, 3, 0, 1]
  v = max(v, dpp_keep<0x141>(v));  // row_half_mirror
  v = max(v, dpp_keep<0x140>(v));  // row_mirror
  return v;
}

// Maximum over the wave (uniform result).
__device__ __forceinline__ int wave_max_dpp(int v) {
  v = row16_max(v);
  const int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  const int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  return max(max(a, b), max(c, d));
}

// Inclusive prefix sum over the wave: shifts by 1, 2, 4 and 8 lanes inside
// each row of 16, then the totals of rows 0 and 2 into rows 1 and 3, then
// the total of rows 0-1 into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t v) {
  v += dpp_u32<0x111>(v);       // row_shr:1
  v += dpp_u32<0x112>(v);       // row_shr:2
  v += dpp_u32<0x114>(v);       // row_shr:4
  v += dpp_u32<0x118>(v);       // row_shr:8
  v += dpp_u32<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_u32<0x143, 0xC>(v);  // row_bcast:31
  return v;
}

// Block-wide inclusive sum of 32-bit values with one barrier: `sh` holds
// NW words and must not be the `sh` of the previous call (callers alternate
// two buffers). *total gets the block sum.
template <int NT>
__device__ __forceinline__ uint32_t block_incl_scan_dpp(uint32_t v, uint32_t* sh,
                                                        uint32_t* total) {
  constexpr int NW = NT / kWave;
  const int w = threadIdx.x / kWave;
  const uint32_t x = wave_incl_scan_dpp(v);
  if (lane_id() == kWave - 1) sh[w] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const uint32_t s = sh[k];
    before += k < w ? s : 0u;
    all += s;
  }
  *total = all;
  return x + before;
}

__host__ __device__ __forceinline__ int64_t floor_div64(int64_t a, int64_t b) {
  int64_t q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}
__host__ __device__ __forceinline__ int64_t ceil_div64(int64_t a, int64_t b) {
  return -floor_div64(-a, b);
}

// ---------------------------------------------------------------------------
// host-side stage launchers (each enqueues on `st`)
// ---------------------------------------------------------------------------
// Records an event after each kernel when per-kernel timing is on.
struct Marker {
  hipEvent_t* ev = nullptr;
  int n = 0, cap = 0;
  void operator()(hipStream_t s) {
    if (ev && n < cap) (void)hipEventRecord(ev[n++], s);
  }
};

// Device-side index check of the allocation-free entry point: clear the flag,
// then set it if any of the n indices is outside [0, V). The guard, launched
// after the visible list is built, turns a set flag into FA_ERR_INVALID_ARG
// in the frame state and an empty visible list, so no later kernel reads
// an index.
hipError_t launch_index_check(const int32_t* idx, int64_t n, int64_t V, int32_t* flag,
                              hipStream_t st);
hipError_t launch_index_guard(const int32_t* flag, const Work& w, hipStream_t st);

hipError_t launch_prologue(int64_t V, const uint8_t* vis, const int32_t* nbr,
                           int64_t T, const FrameParams& p, const Work& w, int32_t* cov,
                           int32_t* cot, int uf_init, Marker& mk, hipStream_t st);
// occ_fill: when not NULL, this [omega][omega] occupancy map is filled with -1
// by workgroups past the union-find tiles (hook mode 5) or past the box
// gather (the other modes); both kernels are bound by dependent loads and
// leave memory bandwidth free.
hipError_t launch_charts(const uint8_t* vis, const int32_t* idx, const int32_t* nbr, int64_t T,
                         const FrameParams& p, const Work& w, int32_t* cot, int32_t* cov,
                         fa_chart* charts, int32_t* occ_fill, Marker& mk, hipStream_t st);
hipError_t launch_order(const FrameParams& p, const Work& w, fa_chart* charts, int from_accum,
                        hipStream_t st);
// footprint push: the full-scale profile of every chart (clear, then raster)
hipError_t launch_footprint(const int32_t* idx, int64_t T, const FrameParams& p, const Work& w,
                            const int32_t* cot, const fa_chart* charts, Marker& mk,
                            hipStream_t st);
// footprint: pack with the chart profiles (p.fp_cap > 0 and a frame's charts)
hipError_t launch_pack(const FrameParams& p, const Work& w, int block, bool footprint,
                       hipStream_t st);
hipError_t launch_select_place(const FrameParams& p, const Work& w, fa_chart* charts,
                               int32_t* cand_out, hipStream_t st);
hipError_t launch_uv(const int64_t V, const FrameParams& p, const Work& w, const int32_t* cov,
                     const fa_chart* charts, float* uv, hipStream_t st);
// per-corner UVs [T][3][2] of edge-connected charts
hipError_t launch_uv_corners(const int32_t* idx, int64_t T, const FrameParams& p, const Work& w,
                             const int32_t* cot, const fa_chart* charts, float* uv,
                             hipStream_t st);
// What an occupancy pass does besides the raster: fill the map with -1 first
// (unless an earlier launch already did), compute the per-vertex UVs beside
// the raster (uv != NULL: V vertices, chart of each vertex in cov), and count
// the occupied texels and write the frame record (meta != NULL: the frame's
// own atlas; a scaled copy is drawn without).
struct OccExtras {
  bool fill = true;
  float* uv = nullptr;
  const int32_t* cov = nullptr;
  int64_t V = 0;
  fa_atlas_meta* meta = nullptr;
};
hipError_t launch_occupancy(const int32_t* idx, int64_t T, const FrameParams& p, const Work& w,
                            const int32_t* cot, const fa_chart* charts, int32_t* occ,
                            int small_texels, int lane_texels, const OccExtras& x, Marker& mk,
                            hipStream_t st);
// Occupancy of the frame's packing drawn into an atlas of side p.omega (a
// scaled copy of the frame's atlas): box ranges for that side, then the
// occupancy kernels.
hipError_t launch_occupancy_scaled(const int32_t* idx, int64_t T, const FrameParams& p,
                                   const Work& w, const int32_t* cot, const fa_chart* charts,
                                   int32_t* occ, int small_texels, int lane_texels,
                                   hipStream_t st);
unsigned visible_grid(int64_t T);  // blocks of the kernels that walk the visible list
hipError_t launch_reuse_flags(const float* pos, const int32_t* idx, int64_t T, const KeyClip& kc,
                              const uint8_t* key_vis, const uint8_t* vis, uint8_t* flags,
                              unsigned long long* reused, hipStream_t st);
hipError_t launch_visibility(const float* pos, const int32_t* idx, int64_t T, const VisParams& q,
                             int32_t* occl, uint32_t* count, unsigned long long* depth,
                             uint8_t* vis, hipStream_t st);
// Frame record without an occupancy map.
hipError_t launch_meta(const FrameParams& p, const Work& w, fa_atlas_meta* meta,
                       hipStream_t st);

// Tuning knobs a frame reads (every accepted value gives the same results).
struct Knobs {
  int pack_block;    // threads per candidate packing
  int small_texels;  // occupancy: queue footprints above this many texels
  int lane_texels;   // occupancy: one lane per footprint up to this many texels
  int uf_link_init;  // union-find start linked to the smallest edge neighbour
};
// Every stage of one frame (clip transform to frame record) on stream st with
// the scratch buffers of w and the scene adjacency nbr. index_flag: NULL, or
// the device flag of launch_index_check (the frame then stops with
// FA_ERR_INVALID_ARG in meta->status when it is set). Returns FA_OK or
// FA_ERR_DEVICE (a launch failed).
int run_frame_core(const Knobs& kn, const Work& w, const fa_mesh* mesh, const int32_t* nbr,
                   const uint8_t* visible, const FrameParams& p, const fa_atlas_out* out,
                   const int32_t* index_flag, Marker& mk, hipStream_t st);

// ---------------------------------------------------------------------------
// batched frames: every stage of n views of one mesh in one launch per stage
// (grid y = view), each view with its own scratch slot and outputs
// ---------------------------------------------------------------------------
struct BatchView {
  FrameParams p;
  Work w;
  const uint8_t* visible;
  int32_t* cot;        // chart_of_tri [T]
  int32_t* cov;        // chart_of_vert [V] (the slot's scratch when the caller has none)
  float* uv;           // [V][2]
  fa_chart* charts;    // [max_charts]
  int32_t* occ;        // [omega][omega]
  fa_atlas_meta* meta;
  int32_t* cand_out;   // [J][4] or NULL
};
// The views (device array dev[0..n)) use hook mode 5, the box push, and all
// have occupancy and UVs; host[0..n) is the same array on the host (for the
// launch shapes). Every view's results equal fa_build_atlas's for it.
hipError_t launch_charts_batched(const BatchView* dev, int n, const float* pos,
                                 const int32_t* idx, const int32_t* nbr, int64_t T, int64_t V,
                                 hipStream_t st);
hipError_t launch_order_batched(const BatchView* dev, int n, hipStream_t st);
hipError_t launch_pack_batched(const BatchView* dev, int n, int J, int64_t max_charts, int block,
                               hipStream_t st);
hipError_t launch_occupancy_batched(const BatchView* dev, int n, const int32_t* idx, int64_t T,
                                    int64_t V, int small_texels, int lane_texels,
                                    hipStream_t st);

// packer-only path: sizes [n][2] -> charts' oriented sizes and keys
hipError_t launch_pack_prepare(const float* sizes, int32_t n, const FrameParams& p,
                               const Work& w, fa_chart* charts, hipStream_t st);
hipError_t launch_pack_emit(int32_t n, const fa_chart* charts, int32_t* placements,
                            const Work& w, hipStream_t st);
hipError_t pack_kernel_attributes(int max_dyn_bytes);

// adjacency (per scene): sorts 3T half-edge keys; tmp buffers from the caller
struct AdjTmp {
  unsigned long long* keys_a;
  unsigned long long* keys_b;
  int32_t* vals_a;
  int32_t* vals_b;
  uint32_t* hist;
  uint32_t* part;  // per-chunk sums of the histogram scan
  uint32_t* n_dev;
};
size_t adjacency_hist_words(int64_t T);
size_t adjacency_part_words(int64_t T);
hipError_t launch_adjacency(const int32_t* idx, int64_t T, int64_t V, const AdjTmp& tmp,
                            int32_t* nbr, hipStream_t st);

}  // namespace fa
