// Host runtime of the gfx950 atlasing library: context and scratch arena,
// resident per-scene adjacency, argument validation and stage orchestration
// behind the C ABI of include/fastatlas.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "fa_internal.h"

using namespace fa;

namespace {

// One entry of the tuning table: the knobs for frames of T in [t_lo, t_hi]
// triangles at atlas side omega (0: any) with J candidates (0: any).
struct TuneEntry {
  int64_t t_lo, t_hi;
  int32_t omega, J;
  int32_t pack_block, small_texels, lane_texels, uf_link_init, uf_edge_hooks, uf_tile;
};

struct Scene {
  int32_t* nbr = nullptr;
  int64_t T = 0, V = 0;
  uint64_t last_use = 0;  // use counter of the context when last used (LRU eviction)
};

size_t scene_bytes(int64_t T) { return (size_t)std::max<int64_t>(1, 3 * T) * 4; }

enum { kStages = 21 };

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kMaxBatchViews = 256;  // views per batched call (more: per-view launches)

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int log2i(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

// Footprint push: pooled profile entries per candidate. A box of chart c is
// a = max(min_box, ceil(w s)) + 2 gutter <= floor(w) + 1 + min_box + 2 gutter
// columns wide, so one candidate's fold is at most the profile columns plus
// (min_box + 2 gutter) per chart.
size_t pool_stride(const fa_config& cfg) {
  return (size_t)cfg.max_profile_columns +
         (size_t)cfg.max_charts * (size_t)(cfg.min_box + 2 * cfg.gutter);
}

}  // namespace

struct fa_ctx {
  fa_config cfg{};
  std::vector<Work> slots;          // one scratch set per concurrent view
  std::vector<void*> arenas;
  std::vector<hipStream_t> slot_streams;
  std::vector<hipEvent_t> slot_join;
  hipEvent_t ev_fork = nullptr, ev_done = nullptr;
  hipStream_t cap_stream = nullptr;  // batch graphs are captured and launched here
  size_t arena_bytes = 0;
  size_t held_bytes = 0;             // every device allocation the context holds now
  uint64_t use_clock = 0;
  std::unordered_map<uint64_t, Scene> scenes;
  int batch_graph = 0;
  int batch_launch = 0;               // 1: one launch per stage for all views of a batch
  BatchView* bv_dev = nullptr;        // [kMaxBatchViews] descriptors of the batched views
  BatchView* bv_host = nullptr;       // their pinned host staging copy
  hipEvent_t ev_upload = nullptr;     // the last upload from bv_host has been read
  std::string graph_sig;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool timing = false;
  hipEvent_t ev[kStages + 1] = {};
  bool ev_recorded = false;
  int ev_marks = 0;
  int pack_block = 1024;
  int small_texels = 64;
  int lane_texels = 64;
  int uf_link_init = 1;
  int uf_edge_hooks = 5;
  int uf_tile = 4096;
  std::vector<TuneEntry> table;    // knobs by frame shape (fa_load_tuning_table)
  int32_t* check_flag = nullptr;  // device int for index validation
  // visibility pass scratch: occluder list [max_triangles] + its counter, and
  // a depth buffer that grows to the largest grid asked for
  int32_t* vis_list = nullptr;
  uint32_t* vis_count = nullptr;
  unsigned long long* vis_depth = nullptr;
  int64_t vis_depth_cap = 0;
};

namespace {
__global__ void k_check_indices(const int32_t* idx, int64_t n, int64_t V, int32_t* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = idx[i];
    if (v < 0 || (int64_t)v >= V) atomicExch(bad, 1);
  }
}
}  // namespace

extern "C" {

const char* fa_status_string(int status) {
  switch (status) {
    case FA_OK: return "ok";
    case FA_ERR_INVALID_ARG: return "invalid argument";
    case FA_ERR_OUT_OF_MEMORY: return "out of device memory";
    case FA_ERR_CAPACITY: return "capacity exceeded";
    case FA_ERR_NOFIT: return "no candidate scale fits the atlas";
    case FA_ERR_DEVICE: return "device error";
    case FA_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

int fa_create(const fa_config* cfg_in, fa_ctx** out_ctx) {
  if (!out_ctx) return FA_ERR_INVALID_ARG;
  *out_ctx = nullptr;
  if (!cfg_in) return FA_ERR_INVALID_ARG;
  fa_config cfg = *cfg_in;
  if (cfg.num_scales == 0) cfg.num_scales = 64;
  if (cfg.max_atlas == 0) cfg.max_atlas = kMaxAtlas;
  if (cfg.max_charts == 0) cfg.max_charts = 65536;
  if (cfg.min_box == 0) cfg.min_box = 2;
  if (cfg.max_views == 0) cfg.max_views = 1;
  if (cfg.num_scales < 1 || cfg.num_scales > kMaxScales) return FA_ERR_INVALID_ARG;
  if (!is_pow2(cfg.max_atlas) || cfg.max_atlas < 16 || cfg.max_atlas > kMaxAtlas)
    return FA_ERR_INVALID_ARG;
  if (cfg.max_charts < 1 || cfg.max_charts > (1 << 20)) return FA_ERR_INVALID_ARG;
  if (cfg.max_triangles < 0 || cfg.max_triangles > (int64_t(1) << 30)) return FA_ERR_INVALID_ARG;
  if (cfg.max_vertices < 0 || cfg.max_vertices > (int64_t(1) << 31) - 1) return FA_ERR_INVALID_ARG;
  if (cfg.gutter < 0 || cfg.gutter > 64 || cfg.min_box < 1 || cfg.min_box > 64)
    return FA_ERR_INVALID_ARG;
  if (cfg.max_views < 1) return FA_ERR_INVALID_ARG;
  if (cfg.hbm_budget_bytes < 0) return FA_ERR_INVALID_ARG;
  const bool footprint = (cfg.flags & FA_FLAG_FOOTPRINT_PUSH) != 0;
  if (footprint && cfg.max_profile_columns == 0)
    cfg.max_profile_columns = 64 * (int64_t)cfg.max_atlas;
  if (footprint && (cfg.gutter < 1 || cfg.max_profile_columns < 1 ||
                    cfg.max_profile_columns > (int64_t(1) << 28)))
    return FA_ERR_INVALID_ARG;
  if (!footprint) cfg.max_profile_columns = 0;

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || cfg.device < 0 || cfg.device >= ndev)
    return FA_ERR_DEVICE;
  if (hipSetDevice(cfg.device) != hipSuccess) return FA_ERR_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, cfg.device) != hipSuccess) return FA_ERR_DEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FA_ERR_DEVICE;

  fa_ctx* ctx = new (std::nothrow) fa_ctx();
  if (!ctx) return FA_ERR_OUT_OF_MEMORY;
  ctx->cfg = cfg;
  const size_t T = (size_t)std::max<int64_t>(cfg.max_triangles, 1);
  const size_t V = (size_t)std::max<int64_t>(cfg.max_vertices, 1);
  const size_t C = (size_t)cfg.max_charts, J = (size_t)cfg.num_scales;
  const size_t tiles = T / kTriTile + 2;
  const size_t sort_tiles = std::max<size_t>(C / kSortTile + 2, kOrderGroups);
  struct Part { void** p; size_t bytes; };
  ctx->slots.resize(cfg.max_views);
  for (int v = 0; v < cfg.max_views; ++v) {
    Work& w = ctx->slots[v];
    std::vector<Part> parts = {
        {(void**)&w.parent, 4 * T},
        {(void**)&w.vmin, 4 * V},                {(void**)&w.cov, 4 * V},
        {(void**)&w.tile_count, 4 * tiles},
        {(void**)&w.tile_vis, 4 * tiles},
        {(void**)&w.accum, 16 * C},              {(void**)&w.keys_a, 4 * C},
        {(void**)&w.vals_a, 4 * C},              {(void**)&w.keys_b, 4 * C},
        {(void**)&w.vals_b, 4 * C},              {(void**)&w.hist, 4 * kRadix * sort_tiles},
        {(void**)&w.sorted_wh, 8 * C},           {(void**)&w.cand_x, 8 * J * C},
        {(void**)&w.cand_ab, 4 * J * C},         {(void**)&w.cand_y, 4 * J * C},
        {(void**)&w.cand_tab, 4 * kCandStride * J},
        {(void**)&w.vlist, 4 * T},
        {(void**)&w.big, 16 * std::min<size_t>(2 * T, (size_t)kBigCap)},
        {(void**)&w.big_fp, 48 * std::min<size_t>(2 * T, (size_t)kBigCap)},
        {(void**)&w.big_counter, 8},             {(void**)&w.partial, 8 * kCountGrid},
        {(void**)&w.pack_charts, sizeof(fa_chart) * C}, {(void**)&w.chart_tex, 16 * C},
        {(void**)&w.cand_rs, 4 * J * (C + 1)},
        {(void**)&w.fp_off, footprint ? 4 * (C + 1) : 4},
        {(void**)&w.fp_prof, footprint ? 8 * (size_t)cfg.max_profile_columns : 8},
        {(void**)&w.fp_group, footprint ? 8 * (T / kWave + 2) : 8},
        {(void**)&w.fp_pool, footprint ? 4 * J * pool_stride(cfg) : 4},
        {(void**)&w.state, sizeof(FrameState)}};
    size_t total = 0;
    for (auto& p : parts) total += align_up(p.bytes);
    void* arena = nullptr;
    if (hipMalloc(&arena, total) != hipSuccess) {
      fa_destroy(ctx);
      return FA_ERR_OUT_OF_MEMORY;
    }
    ctx->arenas.push_back(arena);
    ctx->arena_bytes += total;
    ctx->held_bytes += total;
    char* base = static_cast<char*>(arena);
    for (auto& p : parts) {
      *p.p = base;
      base += align_up(p.bytes);
    }
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      fa_destroy(ctx);
      return FA_ERR_DEVICE;
    }
    ctx->slot_streams.push_back(s);
    ctx->slot_join.push_back(e);
  }
  ctx->held_bytes += 4 + sizeof(BatchView) * kMaxBatchViews;
  if (cfg.hbm_budget_bytes > 0 && (int64_t)ctx->held_bytes > cfg.hbm_budget_bytes) {
    fa_destroy(ctx);
    return FA_ERR_OUT_OF_MEMORY;
  }
  if (hipMalloc(&ctx->check_flag, 4) != hipSuccess ||
      hipMalloc(&ctx->bv_dev, sizeof(BatchView) * kMaxBatchViews) != hipSuccess ||
      hipHostMalloc((void**)&ctx->bv_host, sizeof(BatchView) * kMaxBatchViews,
                    hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_upload, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_done, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    fa_destroy(ctx);
    return FA_ERR_DEVICE;
  }
  if (pack_kernel_attributes(2 * cfg.max_atlas * (int)sizeof(int32_t)) != hipSuccess) {
    fa_destroy(ctx);
    return FA_ERR_DEVICE;
  }
  for (int i = 0; i <= kStages; ++i) (void)hipEventCreate(&ctx->ev[i]);
  *out_ctx = ctx;
  return FA_OK;
}

void fa_destroy(fa_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->cfg.device);
  (void)hipDeviceSynchronize();
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  for (auto& kv : ctx->scenes) (void)hipFree(kv.second.nbr);
  ctx->scenes.clear();
  for (int i = 0; i <= kStages; ++i)
    if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
  for (hipStream_t s : ctx->slot_streams) (void)hipStreamDestroy(s);
  for (hipEvent_t e : ctx->slot_join) (void)hipEventDestroy(e);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_done) (void)hipEventDestroy(ctx->ev_done);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (void* a : ctx->arenas) (void)hipFree(a);
  if (ctx->check_flag) (void)hipFree(ctx->check_flag);
  if (ctx->bv_dev) (void)hipFree(ctx->bv_dev);
  if (ctx->bv_host) (void)hipHostFree(ctx->bv_host);
  if (ctx->ev_upload) (void)hipEventDestroy(ctx->ev_upload);
  if (ctx->vis_list) (void)hipFree(ctx->vis_list);
  if (ctx->vis_count) (void)hipFree(ctx->vis_count);
  if (ctx->vis_depth) (void)hipFree(ctx->vis_depth);
  delete ctx;
}

// The cached batch graph bakes in the resident adjacency of its scene and the
// knobs of the tuning table: drop it whenever a scene's adjacency is freed or
// a table is loaded.
static void drop_graph(fa_ctx* ctx) {
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  ctx->graph_exec = nullptr;
  ctx->graph = nullptr;
  ctx->graph_sig.clear();
}

static void free_scene(fa_ctx* ctx, std::unordered_map<uint64_t, Scene>::iterator it) {
  drop_graph(ctx);
  (void)hipFree(it->second.nbr);
  ctx->held_bytes -= scene_bytes(it->second.T);
  ctx->scenes.erase(it);
}

// Make room for `need` more bytes under the context's budget by evicting the
// least recently used resident scenes (not `keep`). Work on `st` is waited
// for first. false: the budget cannot hold it even with no scene resident.
static bool make_room(fa_ctx* ctx, size_t need, uint64_t keep, hipStream_t st) {
  const int64_t budget = ctx->cfg.hbm_budget_bytes;
  if (budget <= 0) return true;
  bool synced = false;
  while ((int64_t)(ctx->held_bytes + need) > budget) {
    auto victim = ctx->scenes.end();
    for (auto it = ctx->scenes.begin(); it != ctx->scenes.end(); ++it)
      if (it->first != keep &&
          (victim == ctx->scenes.end() || it->second.last_use < victim->second.last_use))
        victim = it;
    if (victim == ctx->scenes.end()) return false;
    if (!synced) {
      (void)hipDeviceSynchronize();  // nothing may still read the victim
      synced = true;
    }
    free_scene(ctx, victim);
  }
  return true;
}

static int get_scene(fa_ctx* ctx, const fa_mesh* mesh, hipStream_t st, Scene** out) {
  auto it = ctx->scenes.find(mesh->scene_key);
  if (it != ctx->scenes.end() && it->second.T == mesh->num_triangles &&
      it->second.V == mesh->num_vertices) {
    it->second.last_use = ++ctx->use_clock;
    *out = &it->second;
    return FA_OK;
  }
  if (it != ctx->scenes.end()) {
    (void)hipStreamSynchronize(st);
    free_scene(ctx, it);
  }
  const int64_t T = mesh->num_triangles, V = mesh->num_vertices;
  // the indices are read by every later kernel: reject out-of-range ones once
  int32_t zero = 0, bad = 0;
  if (hipMemcpyAsync(ctx->check_flag, &zero, 4, hipMemcpyHostToDevice, st) != hipSuccess)
    return FA_ERR_DEVICE;
  if (T > 0)
    k_check_indices<<<1024, kBlock, 0, st>>>(mesh->indices, 3 * T, V, ctx->check_flag);
  if (hipMemcpyAsync(&bad, ctx->check_flag, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return FA_ERR_DEVICE;
  if (bad) return FA_ERR_INVALID_ARG;
  Scene sc;
  sc.T = T;
  sc.V = V;
  sc.last_use = ++ctx->use_clock;
  const int64_t n = 3 * T;
  const size_t tmp_bytes = T > 0 ? align_up(8 * n) * 2 + align_up(4 * n) * 2 +
                                       align_up(4 * adjacency_hist_words(T)) +
                                       align_up(4 * adjacency_part_words(T)) + 256
                                 : 0;
  // the adjacency and, while it is built, its sort buffers must fit the budget
  if (!make_room(ctx, scene_bytes(T) + tmp_bytes, mesh->scene_key, st))
    return FA_ERR_OUT_OF_MEMORY;
  if (hipMalloc(&sc.nbr, scene_bytes(T)) != hipSuccess) return FA_ERR_OUT_OF_MEMORY;
  if (T > 0) {
    AdjTmp tmp{};
    size_t hist_words = adjacency_hist_words(T);
    void* blk = nullptr;
    const size_t bytes = tmp_bytes;
    if (hipMalloc(&blk, bytes) != hipSuccess) {
      (void)hipFree(sc.nbr);
      return FA_ERR_OUT_OF_MEMORY;
    }
    char* b = static_cast<char*>(blk);
    tmp.keys_a = (unsigned long long*)b; b += align_up(8 * n);
    tmp.keys_b = (unsigned long long*)b; b += align_up(8 * n);
    tmp.vals_a = (int32_t*)b; b += align_up(4 * n);
    tmp.vals_b = (int32_t*)b; b += align_up(4 * n);
    tmp.hist = (uint32_t*)b; b += align_up(4 * hist_words);
    tmp.part = (uint32_t*)b;
    hipError_t e = launch_adjacency(mesh->indices, T, V, tmp, sc.nbr, st);
    hipError_t e2 = hipStreamSynchronize(st);
    (void)hipFree(blk);
    if (e != hipSuccess || e2 != hipSuccess) {
      (void)hipFree(sc.nbr);
      return FA_ERR_DEVICE;
    }
  }
  ctx->held_bytes += scene_bytes(T);
  auto res = ctx->scenes.emplace(mesh->scene_key, sc);
  *out = &res.first->second;
  return FA_OK;
}

static int check_mesh(const fa_ctx* ctx, const fa_mesh* mesh) {
  if (!mesh || !mesh->positions || !mesh->indices) return FA_ERR_INVALID_ARG;
  if (mesh->num_triangles < 0 || mesh->num_vertices < 0) return FA_ERR_INVALID_ARG;
  if (mesh->num_triangles > ctx->cfg.max_triangles || mesh->num_vertices > ctx->cfg.max_vertices)
    return FA_ERR_CAPACITY;
  return FA_OK;
}

int fa_scene_adjacency(fa_ctx* ctx, const fa_mesh* mesh, int32_t* nbr_out, void* stream) {
  if (!ctx) return FA_ERR_INVALID_ARG;
  int rc = check_mesh(ctx, mesh);
  if (rc) return rc;
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  Scene* sc = nullptr;
  rc = get_scene(ctx, mesh, st, &sc);
  if (rc) return rc;
  if (nbr_out && mesh->num_triangles > 0 &&
      hipMemcpyAsync(nbr_out, sc->nbr, 12 * mesh->num_triangles, hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
    return FA_ERR_DEVICE;
  return FA_OK;
}

int fa_visibility(fa_ctx* ctx, const fa_mesh* mesh, const fa_camera* cam, const double* eye,
                  double near_w, int32_t coarse, uint8_t* visible, void* stream) {
  if (!ctx || !cam || !eye) return FA_ERR_INVALID_ARG;
  int rc = check_mesh(ctx, mesh);
  if (rc) return rc;
  if (!visible && mesh->num_triangles > 0) return FA_ERR_INVALID_ARG;
  if (cam->width < 1 || cam->width > 16384 || cam->height < 1 || cam->height > 16384)
    return FA_ERR_INVALID_ARG;
  if (coarse < 0 || coarse > 64 || !(near_w > 0.0) || !std::isfinite(near_w))
    return FA_ERR_INVALID_ARG;
  VisParams q{};
  for (int i = 0; i < 16; ++i) {
    if (!std::isfinite(cam->view_proj[i])) return FA_ERR_INVALID_ARG;
    q.M[i] = (double)cam->view_proj[i];
  }
  for (int k = 0; k < 3; ++k) {
    if (!std::isfinite(eye[k])) return FA_ERR_INVALID_ARG;
    q.eye[k] = eye[k];
  }
  q.near_w = near_w;
  q.Wc = coarse > 0 ? cam->width / coarse : 0;
  q.Hc = coarse > 0 ? cam->height / coarse : 0;
  q.coarse = (q.Wc > 0 && q.Hc > 0) ? coarse : 0;
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  Scene* sc = nullptr;  // validates the indices once per scene
  rc = get_scene(ctx, mesh, st, &sc);
  if (rc) return rc;
  if (!ctx->vis_list) {
    const size_t T = (size_t)std::max<int64_t>(ctx->cfg.max_triangles, 1);
    if (!make_room(ctx, 4 * T + 4, mesh->scene_key, st)) return FA_ERR_OUT_OF_MEMORY;
    if (hipMalloc(&ctx->vis_list, 4 * T) != hipSuccess ||
        hipMalloc(&ctx->vis_count, 4) != hipSuccess)
      return FA_ERR_OUT_OF_MEMORY;
    ctx->held_bytes += 4 * T + 4;
  }
  const int64_t nd = (int64_t)q.Wc * q.Hc;
  if (nd > ctx->vis_depth_cap) {
    (void)hipStreamSynchronize(st);
    if (ctx->vis_depth) (void)hipFree(ctx->vis_depth);
    ctx->held_bytes -= 8 * (size_t)ctx->vis_depth_cap;
    ctx->vis_depth = nullptr;
    ctx->vis_depth_cap = 0;
    if (!make_room(ctx, 8 * (size_t)nd, mesh->scene_key, st)) return FA_ERR_OUT_OF_MEMORY;
    if (hipMalloc(&ctx->vis_depth, 8 * (size_t)nd) != hipSuccess) return FA_ERR_OUT_OF_MEMORY;
    ctx->vis_depth_cap = nd;
    ctx->held_bytes += 8 * (size_t)nd;
  }
  if (launch_visibility(mesh->positions, mesh->indices, mesh->num_triangles, q, ctx->vis_list,
                        ctx->vis_count, ctx->vis_depth, visible, st) != hipSuccess)
    return FA_ERR_DEVICE;
  return FA_OK;
}

int fa_reuse_flags(fa_ctx* ctx, const fa_mesh* mesh, const fa_camera* key_cam,
                   const uint8_t* key_visible, const uint8_t* visible, uint8_t* flags,
                   int64_t* reused, void* stream) {
  if (!ctx || !key_cam) return FA_ERR_INVALID_ARG;
  int rc = check_mesh(ctx, mesh);
  if (rc) return rc;
  if (mesh->num_triangles > 0 && (!key_visible || !visible || !flags)) return FA_ERR_INVALID_ARG;
  KeyClip kc{};
  for (int i = 0; i < 16; ++i) {
    if (!std::isfinite(key_cam->view_proj[i])) return FA_ERR_INVALID_ARG;
    kc.M[i] = key_cam->view_proj[i];
  }
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  Scene* sc = nullptr;  // validates the indices once per scene
  rc = get_scene(ctx, mesh, st, &sc);
  if (rc) return rc;
  if (launch_reuse_flags(mesh->positions, mesh->indices, mesh->num_triangles, kc, key_visible,
                         visible, flags, reinterpret_cast<unsigned long long*>(reused),
                         st) != hipSuccess)
    return FA_ERR_DEVICE;
  return FA_OK;
}

int fa_scene_evict(fa_ctx* ctx, uint64_t scene_key) {
  if (!ctx) return FA_ERR_INVALID_ARG;
  auto it = ctx->scenes.find(scene_key);
  if (it == ctx->scenes.end()) return FA_ERR_INVALID_ARG;
  (void)hipSetDevice(ctx->cfg.device);
  (void)hipDeviceSynchronize();
  free_scene(ctx, it);
  return FA_OK;
}

static int frame_params(const fa_ctx* ctx, const fa_camera* cam, int32_t atlas, float rate,
                        FrameParams* p) {
  if (!is_pow2(atlas) || atlas < 16 || atlas > ctx->cfg.max_atlas) return FA_ERR_INVALID_ARG;
  if (!(rate > 0.0f) || !(rate <= 64.0f)) return FA_ERR_INVALID_ARG;
  std::memset(p, 0, sizeof(*p));
  if (cam) {
    if (cam->width < 1 || cam->width > 16384 || cam->height < 1 || cam->height > 16384)
      return FA_ERR_INVALID_ARG;
    for (int i = 0; i < 16; ++i) {
      if (!std::isfinite(cam->view_proj[i])) return FA_ERR_INVALID_ARG;
      p->M[i] = cam->view_proj[i];
    }
    p->W = cam->width;
    p->H = cam->height;
  }
  p->omega = atlas;
  p->log2omega = log2i(atlas);
  p->rate = rate;
  p->J = ctx->cfg.num_scales;
  p->gutter = ctx->cfg.gutter;
  p->min_box = ctx->cfg.min_box;
  p->flags = ctx->cfg.flags;
  p->max_charts = ctx->cfg.max_charts;
  p->edge_hooks = ctx->uf_edge_hooks;
  p->uf_tile = ctx->uf_tile;
  p->fp_cap = (int32_t)ctx->cfg.max_profile_columns;
  p->pool_stride = (int64_t)pool_stride(ctx->cfg);
  return FA_OK;
}


}  // extern "C"

namespace fa {
// Every stage of one frame on stream st with scratch w (see fa_internal.h).
int run_frame_core(const Knobs& kn, const Work& slot, const fa_mesh* mesh, const int32_t* nbr,
                   const uint8_t* visible, const FrameParams& p, const fa_atlas_out* out,
                   const int32_t* index_flag, Marker& mk, hipStream_t st) {
  const int64_t T = mesh->num_triangles, V = mesh->num_vertices;
  Work w = slot;
  w.pos = mesh->positions;
  int32_t* cov = out->chart_of_vert ? out->chart_of_vert : w.cov;
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
  mk(st);
  // start links: the LDS tile kernels write every start themselves (edge-only
  // charts use them unless the global edge hook is chosen)
  const bool tiles_start = (p.flags & FA_FLAG_EDGE_ONLY_CHARTS) ? p.edge_hooks != 1
                                                                : p.edge_hooks >= 2;
  ok(launch_prologue(V, visible, nbr, T, p, w, cov, out->chart_of_tri,
                     tiles_start ? 0 : (kn.uf_link_init ? 2 : 1), mk, st));
  if (index_flag) ok(launch_index_guard(index_flag, w, st));
  // the occupancy map is filled with -1 by spare workgroups of the box gather
  int32_t* occ_fill = T > 0 ? out->occupancy : nullptr;
  ok(launch_charts(visible, mesh->indices, nbr, T, p, w, out->chart_of_tri, cov, out->charts,
                   occ_fill, mk, st));
  ok(launch_order(p, w, out->charts, 1, st));
  mk(st);
  ok(launch_footprint(mesh->indices, T, p, w, out->chart_of_tri, out->charts, mk, st));
  ok(launch_pack(p, w, kn.pack_block, p.fp_cap > 0, st));
  mk(st);
  ok(launch_select_place(p, w, out->charts, out->candidates, st));
  mk(st);
  // per-vertex UVs run beside the occupancy raster when there is one
  const bool edge_only = (p.flags & FA_FLAG_EDGE_ONLY_CHARTS) != 0;
  const bool uv_with_occ = out->uv && out->occupancy && !edge_only;
  if (out->uv && !uv_with_occ) {
    if (edge_only)
      ok(launch_uv_corners(mesh->indices, T, p, w, out->chart_of_tri, out->charts, out->uv, st));
    else
      ok(launch_uv(V, p, w, cov, out->charts, out->uv, st));
  }
  mk(st);
  if (out->occupancy) {
    OccExtras x;
    x.fill = occ_fill == nullptr;
    if (uv_with_occ) {
      x.uv = out->uv;
      x.cov = cov;
      x.V = V;
    }
    x.meta = out->meta;  // the count launch writes the frame record
    ok(launch_occupancy(mesh->indices, T, p, w, out->chart_of_tri, out->charts, out->occupancy,
                        kn.small_texels, kn.lane_texels, x, mk, st));
  } else {
    ok(launch_meta(p, w, out->meta, st));
  }
  mk(st);
  return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}
}  // namespace fa

extern "C" {

// The knobs of a frame: the first tuning-table entry matching its shape,
// else the context's own.
static Knobs frame_knobs(const fa_ctx* ctx, int64_t T, FrameParams* p) {
  for (const TuneEntry& e : ctx->table) {
    if (T < e.t_lo || T > e.t_hi || (e.omega && e.omega != p->omega) || (e.J && e.J != p->J))
      continue;
    p->edge_hooks = e.uf_edge_hooks;
    p->uf_tile = e.uf_tile;
    return Knobs{e.pack_block, e.small_texels, e.lane_texels, e.uf_link_init};
  }
  return Knobs{ctx->pack_block, ctx->small_texels, ctx->lane_texels, ctx->uf_link_init};
}

static int run_frame(fa_ctx* ctx, const Work& w, const fa_mesh* mesh, Scene* sc,
                     const uint8_t* visible, const FrameParams& p_in, const fa_atlas_out* out,
                     hipStream_t st) {
  // one event after every kernel (names in order: fa_stage_times)
  Marker mk;
  if (ctx->timing) { mk.ev = ctx->ev; mk.cap = kStages + 1; }
  FrameParams p = p_in;
  const Knobs kn = frame_knobs(ctx, mesh->num_triangles, &p);
  const int rc = run_frame_core(kn, w, mesh, sc->nbr, visible, p, out, nullptr, mk, st);
  ctx->ev_marks = mk.n;
  ctx->ev_recorded = ctx->timing && mk.n == kStages + 1;
  return rc;
}

int fa_build_atlas(fa_ctx* ctx, const fa_mesh* mesh, const uint8_t* visible,
                   const fa_camera* cam, int32_t atlas_size, float texel_per_pixel,
                   fa_atlas_out* out, void* stream) {
  if (!ctx || !visible || !cam || !out) return FA_ERR_INVALID_ARG;
  if (!out->chart_of_tri || !out->charts || !out->meta) return FA_ERR_INVALID_ARG;
  int rc = check_mesh(ctx, mesh);
  if (rc) return rc;
  FrameParams p;
  rc = frame_params(ctx, cam, atlas_size, texel_per_pixel, &p);
  if (rc) return rc;
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  Scene* sc = nullptr;
  rc = get_scene(ctx, mesh, st, &sc);
  if (rc) return rc;
  return run_frame(ctx, ctx->slots[0], mesh, sc, visible, p, out, st);
}

int fa_build_dual_atlas(fa_ctx* ctx, const fa_mesh* mesh, const uint8_t* visible,
                        const fa_camera* cam, int32_t atlas_size, float texel_per_pixel,
                        int32_t low_shift, fa_atlas_out* out, int32_t* occupancy_low,
                        void* stream) {
  if (!ctx || !visible || !cam || !out || !occupancy_low) return FA_ERR_INVALID_ARG;
  if (!out->chart_of_tri || !out->charts || !out->meta) return FA_ERR_INVALID_ARG;
  if (low_shift < 1 || low_shift > 6 || (atlas_size >> low_shift) < 16) return FA_ERR_INVALID_ARG;
  if (ctx->cfg.flags & FA_FLAG_FOOTPRINT_PUSH) return FA_ERR_UNSUPPORTED;
  int rc = check_mesh(ctx, mesh);
  if (rc) return rc;
  FrameParams p;
  rc = frame_params(ctx, cam, atlas_size, texel_per_pixel, &p);
  if (rc) return rc;
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  Scene* sc = nullptr;
  rc = get_scene(ctx, mesh, st, &sc);
  if (rc) return rc;
  Work w = ctx->slots[0];
  rc = run_frame(ctx, w, mesh, sc, visible, p, out, st);
  if (rc) return rc;
  w.pos = mesh->positions;
  FrameParams pl = p;
  pl.omega = atlas_size >> low_shift;
  pl.log2omega = p.log2omega - low_shift;
  if (launch_occupancy_scaled(mesh->indices, mesh->num_triangles, pl, w, out->chart_of_tri,
                              out->charts, occupancy_low, ctx->small_texels, ctx->lane_texels,
                              st) != hipSuccess)
    return FA_ERR_DEVICE;
  return FA_OK;
}

// Views run concurrently, view i on scratch slot i % max_views and that
// slot's stream, forked from and joined back into the caller's stream. With
// the batch-graph knob, the forked work is captured once into a hipGraph
// (keyed by every byte of the descriptors) and replayed as one launch.
static int enqueue_views(fa_ctx* ctx, const fa_mesh* mesh, Scene* sc, int32_t n,
                         const fa_view* views, const std::vector<FrameParams>& ps,
                         hipStream_t origin) {
  const int S = std::min<int>(n, (int)ctx->slots.size());
  if (hipEventRecord(ctx->ev_fork, origin) != hipSuccess) return FA_ERR_DEVICE;
  for (int k = 0; k < S; ++k)
    if (hipStreamWaitEvent(ctx->slot_streams[k], ctx->ev_fork, 0) != hipSuccess)
      return FA_ERR_DEVICE;
  for (int i = 0; i < n; ++i) {
    const int k = i % S;
    int rc = run_frame(ctx, ctx->slots[k], mesh, sc, views[i].visible, ps[i], &views[i].out,
                       ctx->slot_streams[k]);
    if (rc) return rc;
  }
  for (int k = 0; k < S; ++k) {
    if (hipEventRecord(ctx->slot_join[k], ctx->slot_streams[k]) != hipSuccess ||
        hipStreamWaitEvent(origin, ctx->slot_join[k], 0) != hipSuccess)
      return FA_ERR_DEVICE;
  }
  return FA_OK;
}

// Batched launches: the views' descriptors are in ctx->bv_dev; views
// [r0, r0 + S) run as one round on slots 0..S-1, one launch per stage, with
// the packing and raster-split knobs kn.
static int enqueue_batched(fa_ctx* ctx, const fa_mesh* mesh, Scene* sc, int32_t n,
                           const Knobs& kn, hipStream_t st) {
  const int S = (int)ctx->slots.size();
  const int64_t T = mesh->num_triangles, V = mesh->num_vertices;
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
  for (int r0 = 0; r0 < n; r0 += S) {
    const int m = std::min(S, n - r0);
    const BatchView* d = ctx->bv_dev + r0;
    ok(launch_charts_batched(d, m, mesh->positions, mesh->indices, sc->nbr, T, V, st));
    ok(launch_order_batched(d, m, st));
    ok(launch_pack_batched(d, m, ctx->cfg.num_scales, ctx->cfg.max_charts, kn.pack_block, st));
    ok(launch_occupancy_batched(d, m, mesh->indices, T, V, kn.small_texels, kn.lane_texels, st));
  }
  return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

// The knobs of a batched round: the tuning-table entry of the views' shape
// when every view picks the same one, else the context's own. (The batched
// union-find is always the vertex-hashed tile mode, whatever the entry's
// hook mode; the charts are the same in every mode.)
static Knobs batch_knobs(const fa_ctx* ctx, int64_t T, int32_t n,
                         const std::vector<FrameParams>& ps) {
  FrameParams q = ps[0];
  const Knobs k0 = frame_knobs(ctx, T, &q);
  for (int i = 1; i < n; ++i) {
    q = ps[i];
    const Knobs ki = frame_knobs(ctx, T, &q);
    if (ki.pack_block != k0.pack_block || ki.small_texels != k0.small_texels ||
        ki.lane_texels != k0.lane_texels)
      return Knobs{ctx->pack_block, ctx->small_texels, ctx->lane_texels, ctx->uf_link_init};
  }
  return k0;
}

// The batched launches cover the default configuration: vertex-hashed
// union-find tiles, the box push, and every view with UVs and occupancy.
static bool batchable(const fa_ctx* ctx, const fa_mesh* mesh, int32_t n, const fa_view* views) {
  if (!ctx->batch_launch || n > kMaxBatchViews || mesh->num_triangles <= 0) return false;
  if (ctx->uf_edge_hooks != 5) return false;
  if (ctx->cfg.flags & (FA_FLAG_FOOTPRINT_PUSH | FA_FLAG_EDGE_ONLY_CHARTS)) return false;
  for (int i = 0; i < n; ++i)
    if (!views[i].out.uv || !views[i].out.occupancy) return false;
  return true;
}

int fa_build_atlas_batch(fa_ctx* ctx, const fa_mesh* mesh, int32_t n, const fa_view* views,
                         void* stream) {
  if (!ctx || n < 0 || (n > 0 && !views)) return FA_ERR_INVALID_ARG;
  int rc = check_mesh(ctx, mesh);
  if (rc) return rc;
  std::vector<FrameParams> ps(n);
  for (int i = 0; i < n; ++i) {
    const fa_view& v = views[i];
    if (!v.visible || !v.out.chart_of_tri || !v.out.charts || !v.out.meta) return FA_ERR_INVALID_ARG;
    rc = frame_params(ctx, &v.cam, v.atlas_size, v.texel_per_pixel, &ps[i]);
    if (rc) return rc;
  }
  if (n == 0) return FA_OK;
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  Scene* sc = nullptr;
  rc = get_scene(ctx, mesh, st, &sc);
  if (rc) return rc;
  const bool batched = batchable(ctx, mesh, n, views);
  const Knobs bkn = batch_knobs(ctx, mesh->num_triangles, n, ps);
  if (batched) {
    // descriptors of every view (view i on slot i % S), staged in pinned
    // memory once the previous batch's upload has been read
    const int S = (int)ctx->slots.size();
    if (hipEventSynchronize(ctx->ev_upload) != hipSuccess) return FA_ERR_DEVICE;
    BatchView* hv = ctx->bv_host;
    for (int i = 0; i < n; ++i) {
      const fa_view& v = views[i];
      BatchView& b = hv[i];
      b.p = ps[i];
      b.w = ctx->slots[i % S];
      b.w.pos = mesh->positions;
      b.visible = v.visible;
      b.cot = v.out.chart_of_tri;
      b.cov = v.out.chart_of_vert ? v.out.chart_of_vert : b.w.cov;
      b.uv = v.out.uv;
      b.charts = v.out.charts;
      b.occ = v.out.occupancy;
      b.meta = v.out.meta;
      b.cand_out = v.out.candidates;
    }
    if (hipMemcpyAsync(ctx->bv_dev, hv, sizeof(BatchView) * (size_t)n, hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipEventRecord(ctx->ev_upload, st) != hipSuccess)
      return FA_ERR_DEVICE;
    if (!ctx->batch_graph) return enqueue_batched(ctx, mesh, sc, n, bkn, st);
  }
  const bool timing = ctx->timing;
  ctx->timing = false;  // no stage events inside a batch
  if (!ctx->batch_graph) {
    rc = enqueue_views(ctx, mesh, sc, n, views, ps, st);
    ctx->timing = timing;
    return rc;
  }
  // everything the captured launches bake in: the mesh and view descriptors,
  // the scene's resident adjacency and every knob that picks kernels
  std::string sig(reinterpret_cast<const char*>(mesh), sizeof(fa_mesh));
  sig.append(reinterpret_cast<const char*>(views), sizeof(fa_view) * (size_t)n);
  const int64_t knobs[9] = {(int64_t)(intptr_t)sc->nbr, ctx->pack_block, ctx->small_texels,
                            ctx->lane_texels,          ctx->uf_link_init, ctx->uf_edge_hooks,
                            ctx->uf_tile,              (int64_t)ctx->cfg.flags, batched ? 1 : 0};
  sig.append(reinterpret_cast<const char*>(knobs), sizeof(knobs));
  if (!ctx->graph_exec || sig != ctx->graph_sig) {
    drop_graph(ctx);
    if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      ctx->timing = timing;
      return FA_ERR_DEVICE;
    }
    rc = batched ? enqueue_batched(ctx, mesh, sc, n, bkn, ctx->cap_stream)
                 : enqueue_views(ctx, mesh, sc, n, views, ps, ctx->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
    ctx->timing = timing;
    if (rc || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc ? rc : FA_ERR_DEVICE;
    }
    if (hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      ctx->graph_exec = nullptr;
      return FA_ERR_DEVICE;
    }
    ctx->graph = g;
    ctx->graph_sig = sig;
  }
  ctx->timing = timing;
  if (hipEventRecord(ctx->ev_fork, st) != hipSuccess ||
      hipStreamWaitEvent(ctx->cap_stream, ctx->ev_fork, 0) != hipSuccess ||
      hipGraphLaunch(ctx->graph_exec, ctx->cap_stream) != hipSuccess ||
      hipEventRecord(ctx->ev_done, ctx->cap_stream) != hipSuccess ||
      hipStreamWaitEvent(st, ctx->ev_done, 0) != hipSuccess)
    return FA_ERR_DEVICE;
  return FA_OK;
}

int fa_pack_boxes(fa_ctx* ctx, const float* sizes, int32_t n, int32_t atlas_size,
                  int32_t* placements, fa_atlas_meta* meta, int32_t* candidates, void* stream) {
  if (!ctx || n < 0 || (n > 0 && (!sizes || !placements)) || !meta) return FA_ERR_INVALID_ARG;
  if (n > ctx->cfg.max_charts) return FA_ERR_CAPACITY;
  FrameParams p;
  int rc = frame_params(ctx, nullptr, atlas_size, 1.0f, &p);
  if (rc) return rc;
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  const Work& w = ctx->slots[0];
  fa_chart* charts = w.pack_charts;
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
  ok(launch_pack_prepare(sizes, n, p, w, charts, st));
  ok(launch_order(p, w, charts, 0, st));
  ok(launch_pack(p, w, ctx->pack_block, false, st));
  ok(launch_select_place(p, w, charts, candidates, st));
  ok(launch_pack_emit(n, charts, placements, w, st));
  ok(launch_meta(p, w, meta, st));
  return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

// Parse a tuning table (see fastatlas.h); every value must be one that
// fa_set_tuning accepts for its knob.
int fa_load_tuning_table(fa_ctx* ctx, const char* text) {
  if (!ctx || !text) return FA_ERR_INVALID_ARG;
  std::vector<TuneEntry> tab;
  const char* q = text;
  while (*q) {
    const char* e = q;
    while (*e && *e != '\n') ++e;
    std::string line(q, e);
    q = *e ? e + 1 : e;
    const size_t hash = line.find('#');
    if (hash != std::string::npos) line.resize(hash);
    if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
    long long v[10];
    int used = 0;
    if (std::sscanf(line.c_str(), "%lld %lld %lld %lld %lld %lld %lld %lld %lld %lld %n", &v[0],
                    &v[1], &v[2], &v[3], &v[4], &v[5], &v[6], &v[7], &v[8], &v[9], &used) != 10 ||
        line.find_first_not_of(" \t\r", (size_t)used) != std::string::npos)
      return FA_ERR_INVALID_ARG;
    TuneEntry t{v[0], v[1], (int32_t)v[2], (int32_t)v[3], (int32_t)v[4], (int32_t)v[5],
                (int32_t)v[6], (int32_t)v[7], (int32_t)v[8], (int32_t)v[9]};
    const bool ok = t.t_lo >= 0 && t.t_hi >= t.t_lo && (t.omega == 0 || is_pow2(t.omega)) &&
                    t.J >= 0 && t.J <= kMaxScales &&
                    (t.pack_block == 256 || t.pack_block == 512 || t.pack_block == 1024) &&
                    t.small_texels >= 0 && t.small_texels <= 4096 && t.lane_texels >= 0 &&
                    t.lane_texels <= 4096 && (t.uf_link_init == 0 || t.uf_link_init == 1) &&
                    t.uf_edge_hooks >= 0 && t.uf_edge_hooks <= 5 &&
                    (t.uf_tile == 2048 || t.uf_tile == 4096 || t.uf_tile == 8192);
    if (!ok) return FA_ERR_INVALID_ARG;
    tab.push_back(t);
  }
  ctx->table = std::move(tab);
  drop_graph(ctx);  // a captured batch baked in the previous table's knobs
  return FA_OK;
}

int fa_set_tuning(fa_ctx* ctx, int knob, int value) {
  if (!ctx) return FA_ERR_INVALID_ARG;
  switch (knob) {
    case FA_TUNE_PACK_BLOCK:
      if (value != 256 && value != 512 && value != 1024) return FA_ERR_INVALID_ARG;
      ctx->pack_block = value;
      return FA_OK;
    case FA_TUNE_OCC_SMALL_TEXELS:
      if (value < 0 || value > 4096) return FA_ERR_INVALID_ARG;
      ctx->small_texels = value;
      return FA_OK;
    case FA_TUNE_UF_LINK_INIT:
      if (value != 0 && value != 1) return FA_ERR_INVALID_ARG;
      ctx->uf_link_init = value;
      return FA_OK;
    case FA_TUNE_BATCH_GRAPH:
      if (value != 0 && value != 1) return FA_ERR_INVALID_ARG;
      ctx->batch_graph = value;
      return FA_OK;
    case FA_TUNE_UF_EDGE_HOOKS:
      if (value < 0 || value > 5) return FA_ERR_INVALID_ARG;
      ctx->uf_edge_hooks = value;
      return FA_OK;
    case FA_TUNE_UF_TILE:
      if (value != 2048 && value != 4096 && value != 8192) return FA_ERR_INVALID_ARG;
      ctx->uf_tile = value;
      return FA_OK;
    case FA_TUNE_OCC_LANE_TEXELS:
      if (value < 0 || value > 4096) return FA_ERR_INVALID_ARG;
      ctx->lane_texels = value;
      return FA_OK;
    case FA_TUNE_BATCH_LAUNCH:
      if (value != 0 && value != 1) return FA_ERR_INVALID_ARG;
      ctx->batch_launch = value;
      return FA_OK;
    default:
      return FA_ERR_INVALID_ARG;
  }
}

int fa_get_tuning(fa_ctx* ctx, int knob) {
  if (!ctx) return -1;
  switch (knob) {
    case FA_TUNE_PACK_BLOCK: return ctx->pack_block;
    case FA_TUNE_OCC_SMALL_TEXELS: return ctx->small_texels;
    case FA_TUNE_UF_LINK_INIT: return ctx->uf_link_init;
    case FA_TUNE_BATCH_GRAPH: return ctx->batch_graph;
    case FA_TUNE_UF_EDGE_HOOKS: return ctx->uf_edge_hooks;
    case FA_TUNE_UF_TILE: return ctx->uf_tile;
    case FA_TUNE_OCC_LANE_TEXELS: return ctx->lane_texels;
    case FA_TUNE_BATCH_LAUNCH: return ctx->batch_launch;
    default: return -1;
  }
}

int64_t fa_device_bytes(const fa_ctx* ctx) {
  return ctx ? (int64_t)ctx->held_bytes : -1;
}

int fa_set_stage_timing(fa_ctx* ctx, int enable) {
  if (!ctx) return FA_ERR_INVALID_ARG;
  ctx->timing = enable != 0;
  ctx->ev_recorded = false;
  return FA_OK;
}

int fa_stage_times(fa_ctx* ctx, float* ms, int n) {
  if (!ctx || !ms) return FA_ERR_INVALID_ARG;
  if (!ctx->ev_recorded) return 0;
  int k = 0;
  for (int i = 0; i < kStages && k < n; ++i, ++k) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, ctx->ev[i], ctx->ev[i + 1]) != hipSuccess) t = -1.0f;
    ms[k] = t;
  }
  return k;
}

}  // extern "C"
