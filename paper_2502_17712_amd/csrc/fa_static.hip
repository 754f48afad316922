// Allocation-free entry point: fa_build_atlas_static atlases one frame with
// every scratch buffer (the frame's working set and the triangle adjacency,
// rebuilt per call) carved from one file-scope device array, so the call
// makes no device allocation. For callers that cannot allocate: code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "fa_internal.h"

using namespace fa;

namespace {

// Fixed configuration and limits of the static path.
constexpr int64_t kStaticT = FA_STATIC_MAX_TRIANGLES;
constexpr int64_t kStaticV = FA_STATIC_MAX_VERTICES;
constexpr int64_t kStaticC = FA_STATIC_MAX_CHARTS;
constexpr int64_t kStaticJ = 64;
constexpr size_t kScratchBytes = size_t(FA_STATIC_SCRATCH_MIB) << 20;
constexpr int kMaxDevices = 64;

// The scratch of every call on a device (each device holds its own copy, at
// its own address, for the life of the process). Host code never passes this
// name to a kernel or a copy: it is a host-side stand-in; the device address
// comes from hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
  char* ptr = nullptr;  // device address of `scratch` on this device
  int rc = -1;          // FA_OK once set up; an error code if the set-up failed
};
DeviceScratch g_dev[kMaxDevices];
std::mutex g_mu;

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Carve the scratch at `base` (nullptr: only measure). Returns the bytes used.
size_t carve(char* base, Work* w, AdjTmp* adj, int32_t** nbr, int32_t** flag) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += a256(bytes);
    return p;
  };
  const size_t T = kStaticT, V = kStaticV, C = kStaticC, J = kStaticJ;
  const size_t tiles = T / kTriTile + 2,
               sort_tiles = std::max<size_t>(C / kSortTile + 2, kOrderGroups);
  const size_t big = std::min<size_t>(2 * T, (size_t)kBigCap);
  Work& x = *w;
  x = Work{};
  x.pos = nullptr;  // the frame's mesh positions, set per frame
  x.parent = (int32_t*)take(4 * T);
  x.vmin = (int32_t*)take(4 * V);
  x.cov = (int32_t*)take(4 * V);
  x.tile_count = (uint32_t*)take(4 * tiles);
  x.tile_vis = (uint32_t*)take(4 * tiles);
  x.accum = (uint32_t*)take(16 * C);
  x.keys_a = (uint32_t*)take(4 * C);
  x.vals_a = (int32_t*)take(4 * C);
  x.keys_b = (uint32_t*)take(4 * C);
  x.vals_b = (int32_t*)take(4 * C);
  x.hist = (uint32_t*)take(4 * kRadix * sort_tiles);
  x.sorted_wh = (float2*)take(8 * C);
  x.cand_x = (long long*)take(8 * J * C);
  x.cand_ab = (uint32_t*)take(4 * J * C);
  x.cand_y = (int32_t*)take(4 * J * C);
  x.cand_tab = (int32_t*)take(4 * kCandStride * J);
  x.vlist = (int32_t*)take(4 * T);
  x.partial = (unsigned long long*)take(8 * kCountGrid);
  x.big = (ulonglong2*)take(16 * big);
  x.big_fp = (int4*)take(48 * big);
  x.big_counter = (unsigned long long*)take(8);
  x.pack_charts = nullptr;  // packer-only entry: not used here
  x.cand_rs = (int32_t*)take(4 * J * (C + 1));
  x.chart_tex = (int4*)take(16 * C);
  x.fp_off = (int32_t*)take(4);        // no footprint push on this path
  x.fp_prof = (int2*)take(8);
  x.fp_group = (unsigned long long*)take(8);
  x.fp_pool = (uint32_t*)take(4);
  x.state = (FrameState*)take(sizeof(FrameState));
  *nbr = (int32_t*)take(12 * T);
  const size_t n = 3 * T;
  adj->keys_a = (unsigned long long*)take(8 * n);
  adj->keys_b = (unsigned long long*)take(8 * n);
  adj->vals_a = (int32_t*)take(4 * n);
  adj->vals_b = (int32_t*)take(4 * n);
  adj->hist = (uint32_t*)take(4 * adjacency_hist_words(kStaticT));
  adj->part = (uint32_t*)take(4 * adjacency_part_words(kStaticT));
  adj->n_dev = nullptr;
  *flag = (int32_t*)take(4);
  return off;
}

// Once per device, with that device current: the device address of its copy
// of `scratch`, the device check and the packer's LDS attribute.
int setup_device(int dev) {
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceScratch& d = g_dev[dev];
  if (d.rc >= 0) return d.rc;
  d.rc = FA_ERR_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return d.rc;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return d.rc;
  Work w;
  AdjTmp a;
  int32_t *nbr = nullptr, *flag = nullptr;
  if (carve(nullptr, &w, &a, &nbr, &flag) > kScratchBytes) return d.rc;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return d.rc;
  if (pack_kernel_attributes(2 * kMaxAtlas * (int)sizeof(int32_t)) != hipSuccess) return d.rc;
  d.ptr = static_cast<char*>(p);
  d.rc = FA_OK;
  return d.rc;
}

}  // namespace

extern "C" int fa_build_atlas_static(const fa_mesh* mesh, const uint8_t* visible,
                                     const fa_camera* cam, int32_t atlas_size,
                                     float texel_per_pixel, fa_atlas_out* out, void* stream) {
  if (!mesh || !visible || !cam || !out) return FA_ERR_INVALID_ARG;
  if (!out->chart_of_tri || !out->charts || !out->meta) return FA_ERR_INVALID_ARG;
  if (!mesh->positions || !mesh->indices || mesh->num_triangles < 0 || mesh->num_vertices < 0)
    return FA_ERR_INVALID_ARG;
  if (mesh->num_triangles > kStaticT || mesh->num_vertices > kStaticV) return FA_ERR_CAPACITY;
  if (!(atlas_size >= 16 && atlas_size <= kMaxAtlas && (atlas_size & (atlas_size - 1)) == 0))
    return FA_ERR_INVALID_ARG;
  if (!(texel_per_pixel > 0.0f) || !(texel_per_pixel <= 64.0f)) return FA_ERR_INVALID_ARG;
  if (cam->width < 1 || cam->width > 16384 || cam->height < 1 || cam->height > 16384)
    return FA_ERR_INVALID_ARG;
  FrameParams p{};
  for (int i = 0; i < 16; ++i) {
    if (!std::isfinite(cam->view_proj[i])) return FA_ERR_INVALID_ARG;
    p.M[i] = cam->view_proj[i];
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FA_ERR_DEVICE;
  const int rc = setup_device(dev);
  if (rc != FA_OK) return rc;
  Work w;
  AdjTmp adj;
  int32_t *nbr = nullptr, *flag = nullptr;
  carve(g_dev[dev].ptr, &w, &adj, &nbr, &flag);
  p.W = cam->width;
  p.H = cam->height;
  p.omega = atlas_size;
  int l = 0;
  while ((1 << l) < atlas_size) ++l;
  p.log2omega = l;
  p.rate = texel_per_pixel;
  p.J = (int32_t)kStaticJ;
  p.gutter = 1;
  p.min_box = 2;
  p.flags = 0;
  p.max_charts = (int32_t)kStaticC;
  p.edge_hooks = 5;
  p.uf_tile = 4096;
  p.fp_cap = 0;
  p.pool_stride = 0;
  hipStream_t st = (hipStream_t)stream;
  const int64_t T = mesh->num_triangles, V = mesh->num_vertices;
  if (launch_index_check(mesh->indices, 3 * T, V, flag, st) != hipSuccess ||
      launch_adjacency(mesh->indices, T, V, adj, nbr, st) != hipSuccess)
    return FA_ERR_DEVICE;
  const Knobs kn{1024, 64, 64, 1};
  Marker none;
  return run_frame_core(kn, w, mesh, nbr, visible, p, out, flag, none, st);
}
