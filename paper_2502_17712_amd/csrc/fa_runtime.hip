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

struct Scene {
  int32_t* nbr = nullptr;
  int64_t T = 0, V = 0;
};

enum { kStages = 6 };

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int log2i(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

}  // namespace

struct fa_ctx {
  fa_config cfg{};
  Work w{};
  void* arena = nullptr;
  size_t arena_bytes = 0;
  std::unordered_map<uint64_t, Scene> scenes;
  bool timing = false;
  hipEvent_t ev[kStages + 1] = {};
  bool ev_recorded = false;
  int pack_block = 256;
  int small_texels = 64;
  int32_t* check_flag = nullptr;  // device int for index validation
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
  const size_t sort_tiles = C / kSortTile + 2;
  struct Part { void** p; size_t bytes; };
  Work& w = ctx->w;
  std::vector<Part> parts = {
      {(void**)&w.clip, sizeof(float4) * V},   {(void**)&w.parent, 4 * T},
      {(void**)&w.vmin, 4 * V},                {(void**)&w.cov, 4 * V},
      {(void**)&w.tile_count, 4 * tiles},      {(void**)&w.tile_off, 4 * tiles},
      {(void**)&w.accum, 16 * C},              {(void**)&w.keys_a, 4 * C},
      {(void**)&w.vals_a, 4 * C},              {(void**)&w.keys_b, 4 * C},
      {(void**)&w.vals_b, 4 * C},              {(void**)&w.hist, 4 * kRadix * sort_tiles},
      {(void**)&w.sorted_wh, 8 * C},           {(void**)&w.cand_x, 8 * J * C},
      {(void**)&w.cand_ab, 4 * J * C},         {(void**)&w.cand_y, 4 * J * C},
      {(void**)&w.cand_tab, 4 * kCandStride * J}, {(void**)&w.big, 8 * T},
      {(void**)&w.pack_charts, sizeof(fa_chart) * C},
      {(void**)&w.state, sizeof(FrameState)},  {(void**)&ctx->check_flag, 4}};
  size_t total = 0;
  for (auto& p : parts) total += align_up(p.bytes);
  if (hipMalloc(&ctx->arena, total) != hipSuccess) {
    delete ctx;
    return FA_ERR_OUT_OF_MEMORY;
  }
  ctx->arena_bytes = total;
  char* base = static_cast<char*>(ctx->arena);
  for (auto& p : parts) {
    *p.p = base;
    base += align_up(p.bytes);
  }
  if (pack_kernel_attributes(2 * cfg.max_atlas * (int)sizeof(int32_t)) != hipSuccess) {
    (void)hipFree(ctx->arena);
    delete ctx;
    return FA_ERR_DEVICE;
  }
  for (int i = 0; i <= kStages; ++i) (void)hipEventCreate(&ctx->ev[i]);
  *out_ctx = ctx;
  return FA_OK;
}

void fa_destroy(fa_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->cfg.device);
  for (auto& kv : ctx->scenes) (void)hipFree(kv.second.nbr);
  ctx->scenes.clear();
  for (int i = 0; i <= kStages; ++i)
    if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
  (void)hipFree(ctx->arena);
  delete ctx;
}

static int get_scene(fa_ctx* ctx, const fa_mesh* mesh, hipStream_t st, Scene** out) {
  auto it = ctx->scenes.find(mesh->scene_key);
  if (it != ctx->scenes.end() && it->second.T == mesh->num_triangles &&
      it->second.V == mesh->num_vertices) {
    *out = &it->second;
    return FA_OK;
  }
  if (it != ctx->scenes.end()) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(it->second.nbr);
    ctx->scenes.erase(it);
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
  if (hipMalloc(&sc.nbr, std::max<int64_t>(1, 3 * T) * 4) != hipSuccess) return FA_ERR_OUT_OF_MEMORY;
  if (T > 0) {
    AdjTmp tmp{};
    const int64_t n = 3 * T;
    size_t hist_words = adjacency_hist_words(T);
    void* blk = nullptr;
    size_t bytes = align_up(8 * n) * 2 + align_up(4 * n) * 2 + align_up(4 * hist_words) + 256;
    if (hipMalloc(&blk, bytes) != hipSuccess) {
      (void)hipFree(sc.nbr);
      return FA_ERR_OUT_OF_MEMORY;
    }
    char* b = static_cast<char*>(blk);
    tmp.keys_a = (unsigned long long*)b; b += align_up(8 * n);
    tmp.keys_b = (unsigned long long*)b; b += align_up(8 * n);
    tmp.vals_a = (int32_t*)b; b += align_up(4 * n);
    tmp.vals_b = (int32_t*)b; b += align_up(4 * n);
    tmp.hist = (uint32_t*)b;
    hipError_t e = launch_adjacency(mesh->indices, T, V, tmp, sc.nbr, st);
    hipError_t e2 = hipStreamSynchronize(st);
    (void)hipFree(blk);
    if (e != hipSuccess || e2 != hipSuccess) {
      (void)hipFree(sc.nbr);
      return FA_ERR_DEVICE;
    }
  }
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

int fa_scene_evict(fa_ctx* ctx, uint64_t scene_key) {
  if (!ctx) return FA_ERR_INVALID_ARG;
  auto it = ctx->scenes.find(scene_key);
  if (it == ctx->scenes.end()) return FA_ERR_INVALID_ARG;
  (void)hipSetDevice(ctx->cfg.device);
  (void)hipDeviceSynchronize();
  (void)hipFree(it->second.nbr);
  ctx->scenes.erase(it);
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
  return FA_OK;
}

static inline void mark(fa_ctx* ctx, int i, hipStream_t st) {
  if (ctx->timing) (void)hipEventRecord(ctx->ev[i], st);
}

static int run_frame(fa_ctx* ctx, const fa_mesh* mesh, Scene* sc, const uint8_t* visible,
                     const FrameParams& p, fa_atlas_out* out, hipStream_t st) {
  const Work& w = ctx->w;
  const int64_t T = mesh->num_triangles, V = mesh->num_vertices;
  int32_t* cov = out->chart_of_vert ? out->chart_of_vert : w.cov;
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
  mark(ctx, 0, st);
  ok(launch_frame_init(w, st));
  ok(launch_clip(mesh->positions, V, p, w, cov, st));
  ok(launch_charts(visible, mesh->indices, sc->nbr, T, p, w, out->chart_of_tri, cov, out->charts,
                   st));
  mark(ctx, 1, st);
  ok(launch_chart_sizes(p, w, out->charts, st));
  mark(ctx, 2, st);
  ok(launch_order(p, w, out->charts, st));
  mark(ctx, 3, st);
  ok(launch_pack(p, w, ctx->pack_block, st));
  ok(launch_select_place(p, w, out->charts, out->candidates, st));
  mark(ctx, 4, st);
  if (out->uv) ok(launch_uv(V, p, w, cov, out->charts, out->uv, st));
  mark(ctx, 5, st);
  if (out->occupancy)
    ok(launch_occupancy(mesh->indices, T, p, w, out->chart_of_tri, out->charts, out->occupancy,
                        ctx->small_texels, st));
  ok(launch_meta(p, w, out->meta, st));
  mark(ctx, 6, st);
  ctx->ev_recorded = ctx->timing;
  return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
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
  return run_frame(ctx, mesh, sc, visible, p, out, st);
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
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FA_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  Scene* sc = nullptr;
  rc = get_scene(ctx, mesh, st, &sc);
  if (rc) return rc;
  for (int i = 0; i < n; ++i) {
    fa_atlas_out o = views[i].out;
    rc = run_frame(ctx, mesh, sc, views[i].visible, ps[i], &o, st);
    if (rc) return rc;
  }
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
  const Work& w = ctx->w;
  fa_chart* charts = w.pack_charts;
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
  ok(launch_frame_init(w, st));
  ok(launch_pack_prepare(sizes, n, p, w, charts, st));
  ok(launch_order(p, w, charts, st));
  ok(launch_pack(p, w, ctx->pack_block, st));
  ok(launch_select_place(p, w, charts, candidates, st));
  ok(launch_pack_emit(n, charts, placements, w, st));
  ok(launch_meta(p, w, meta, st));
  return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
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
