// Chart stages of the per-frame path on gfx950:
//   clip transform, union-find charts (Appendix "GPU Union Find", Alg. 1),
//   root compaction, per-triangle conservative boxes (Sec. "Computing Bounding
//   Boxes of Projected Visible Sub-Charts") reduced per chart, chart sizes.
#include <algorithm>
#include <climits>

#include "fa_internal.h"

namespace fa {
namespace {

// ---------------------------------------------------------------------------
// union-find over visible triangles. parent[x] <= x always holds; a root has
// parent[x] == x. Path halving stores are agent-scope atomics so they stay
// coherent with the hooking compare-and-swaps across the chip's L2 caches.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int uf_root(int32_t* parent, int x) {
  int cur = parent[x];
  if (cur == x) return x;
  int prev = x;
  for (;;) {
    int nxt = parent[cur];
    if (nxt >= cur) return cur;  // parent[cur] == cur
    __hip_atomic_store(&parent[prev], nxt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    prev = cur;
    cur = nxt;
  }
}

// Join the trees of u and v: the larger root is hooked below the smaller one
// with a compare-and-swap; on failure continue from the value that won.
__device__ __forceinline__ void uf_join(int32_t* parent, int u, int v) {
  int ru = uf_root(parent, u), rv = uf_root(parent, v);
  while (ru != rv) {
    if (ru < rv) {
      int old = atomicCAS(&parent[rv], rv, ru);
      if (old == rv) return;
      rv = old;
    } else {
      int old = atomicCAS(&parent[ru], ru, rv);
      if (old == ru) return;
      ru = old;
    }
  }
}

// Prologue of a frame: frame state, clip transform of every vertex
// (clip = M (x, y, z, 1)^T, rows summed left to right), per-vertex scratch, and
// the union-find start of every triangle. Blocks [0, vblocks) handle
// vertices, the rest triangles. With link_neighbours a visible triangle starts
// linked to the smallest of itself and its visible edge neighbours (Alg. 1,
// first loop); otherwise it starts as its own root (same final labels).
__global__ void k_prologue(const float* __restrict__ pos, int64_t V, FrameParams p,
                           float4* __restrict__ clip, int32_t* __restrict__ vmin,
                           int32_t* __restrict__ cov, const uint8_t* __restrict__ vis,
                           const int32_t* __restrict__ nbr, int64_t T,
                           int32_t* __restrict__ parent, int link_neighbours, unsigned vblocks,
                           FrameState* st, unsigned long long* big_counter) {
  if (blockIdx.x < vblocks) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      FrameState s = {};
      s.status = FA_OK;
      *st = s;
      *big_counter = 0ull;
    }
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const float x = pos[3 * v], y = pos[3 * v + 1], z = pos[3 * v + 2];
    float r[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float acc = p.M[4 * i] * x;
      acc = acc + p.M[4 * i + 1] * y;
      acc = acc + p.M[4 * i + 2] * z;
      r[i] = acc + p.M[4 * i + 3];
    }
    clip[v] = make_float4(r[0], r[1], r[2], r[3]);
    vmin[v] = INT_MAX;
    cov[v] = -1;
    return;
  }
  const int64_t t = (int64_t)(blockIdx.x - vblocks) * blockDim.x + threadIdx.x;
  if (t >= T) return;
  if (!vis[t]) { parent[t] = -1; return; }
  int q = (int)t;
  if (link_neighbours) {
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int n = nbr[3 * t + e];
      if (n >= 0 && vis[n]) q = min(q, n);
    }
  }
  parent[t] = q;
}

// Hook across every shared edge once (u < v) (Alg. 1, second loop) and record
// for every vertex the smallest visible triangle using it. The record only has
// to name some triangle of the charts meeting at the vertex; the smallest
// triangle serves as well as its root does in Alg. 1's third loop.
__global__ void k_uf_hook(const uint8_t* __restrict__ vis, const int32_t* __restrict__ nbr,
                          const int32_t* __restrict__ idx, int64_t T, int32_t* parent,
                          int32_t* __restrict__ vmin) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T || !vis[t]) return;
#pragma unroll
  for (int e = 0; e < 3; ++e) atomicMin(&vmin[idx[3 * t + e]], (int)t);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    int n = nbr[3 * t + e];
    if (n > t && vis[n]) uf_join(parent, (int)t, n);
  }
}

// Vertex hook: join every visible triangle with the recorded triangle of each
// of its vertices, merging charts that share only a vertex.
__global__ void k_uf_vertex_hook(const uint8_t* __restrict__ vis, const int32_t* __restrict__ idx,
                                 int64_t T, int32_t* parent, const int32_t* __restrict__ vmin) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T || !vis[t]) return;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    int m = vmin[idx[3 * t + e]];
    if (m != (int)t) uf_join(parent, (int)t, m);
  }
}

// Flatten every visible triangle to its root and count roots per tile of
// kTriTile consecutive triangles.
__global__ void k_uf_flatten_count(const uint8_t* __restrict__ vis, int64_t T, int32_t* parent,
                                   uint32_t* __restrict__ tile_count,
                                   uint32_t* __restrict__ tile_vis) {
  __shared__ uint32_t sh[kBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kTriTile + (int64_t)threadIdx.x * 4;
  uint32_t roots = 0, visible = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int64_t t = base + k;
    if (t < T && vis[t]) {
      int r = uf_root(parent, (int)t);
      parent[t] = r;
      roots += (r == (int)t);
      visible += 1;
    }
  }
  uint32_t rs = block_sum<uint32_t>(roots, sh);
  uint32_t vs = block_sum<uint32_t>(visible, sh);
  if (threadIdx.x == 0) {
    tile_count[blockIdx.x] = rs;
    tile_vis[blockIdx.x] = vs;
  }
}

// Exclusive scan of the per-tile root counts (one workgroup); C = total.
__global__ void k_scan_tiles(const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ vis_cnt,
                             uint32_t* __restrict__ off, int64_t ntiles, int32_t max_charts,
                             FrameState* st) {
  __shared__ uint32_t sh[1024 / kWave];
  __shared__ unsigned long long shv[1024 / kWave];
  uint32_t run = 0;
  unsigned long long nvis = 0;
  for (int64_t b0 = 0; b0 < ntiles; b0 += blockDim.x) {
    int64_t b = b0 + threadIdx.x;
    uint32_t v = b < ntiles ? cnt[b] : 0;
    nvis += b < ntiles ? vis_cnt[b] : 0;
    uint32_t tot;
    uint32_t inc = block_incl_scan<uint32_t>(v, sh, &tot);
    if (b < ntiles) off[b] = run + inc - v;
    run += tot;
  }
  nvis = block_sum<unsigned long long>(nvis, shv);
  if (threadIdx.x == 0) {
    st->visible = nvis;
    st->num_charts = (int32_t)run;
    if ((int64_t)run > (int64_t)max_charts) st->status = FA_ERR_CAPACITY;
  }
}

// Chart index of each root = its rank among roots (roots ascend with the
// triangle index, so chart indices ascend with the chart's lowest triangle).
__global__ void k_assign_roots(const uint8_t* __restrict__ vis, int64_t T,
                               const int32_t* __restrict__ parent,
                               const uint32_t* __restrict__ off, int32_t* __restrict__ cot,
                               fa_chart* __restrict__ charts, uint32_t* __restrict__ accum,
                               const FrameState* __restrict__ st) {
  __shared__ uint32_t sh[kBlock / kWave];
  if (st->status != FA_OK) return;
  const int64_t base = (int64_t)blockIdx.x * kTriTile + (int64_t)threadIdx.x * 4;
  bool root[4];
  uint32_t mine = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int64_t t = base + k;
    root[k] = t < T && vis[t] && parent[t] == (int)t;
    mine += root[k];
  }
  uint32_t tot;
  uint32_t c = off[blockIdx.x] + block_incl_scan<uint32_t>(mine, sh, &tot) - mine;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!root[k]) continue;
    int64_t t = base + k;
    cot[t] = (int32_t)c;
    charts[c].root_tri = (int32_t)t;
    uint4 init = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u);
    reinterpret_cast<uint4*>(accum)[c] = init;
    ++c;
  }
}

// ---------------------------------------------------------------------------
// per-triangle conservative box (NDC)
// ---------------------------------------------------------------------------
// plane distances: 0 left w+x, 1 right w-x, 2 bottom w+y, 3 top w-y,
//                  4 near w+z, 5 far w-z
template <int P>
__device__ __forceinline__ float pdist(const float4& q) {
  if (P == 0) return q.w + q.x;
  if (P == 1) return q.w - q.x;
  if (P == 2) return q.w + q.y;
  if (P == 3) return q.w - q.y;
  if (P == 4) return q.w + q.z;
  return q.w - q.z;
}

struct Quad {
  float4 v0, v1, v2, v3;
  int n;
};

__device__ __forceinline__ void quad_put(Quad& q, const float4& p) {
  if (q.n == 0) q.v0 = p;
  else if (q.n == 1) q.v1 = p;
  else if (q.n == 2) q.v2 = p;
  else q.v3 = p;
  q.n++;
}

// One edge S->E of a Sutherland-Hodgman pass against plane P.
template <int P>
__device__ __forceinline__ void sh_edge(Quad& q, const float4& S, const float4& E) {
  const float dS = pdist<P>(S), dE = pdist<P>(E);
  const bool inS = dS >= 0.0f, inE = dE >= 0.0f;
  if (inS != inE) {
    const float4 A = inS ? S : E;
    const float4 B = inS ? E : S;
    const float dA = inS ? dS : dE;
    const float dB = inS ? dE : dS;
    const float t = dA / (dA - dB);
    float4 I;
    I.x = A.x + t * (B.x - A.x);
    I.y = A.y + t * (B.y - A.y);
    I.z = A.z + t * (B.z - A.z);
    I.w = A.w + t * (B.w - A.w);
    quad_put(q, I);
  }
  if (inE) quad_put(q, E);
}

template <int P>
__device__ __forceinline__ Quad clip_tri(const float4& a, const float4& b, const float4& c) {
  Quad q;
  q.n = 0;
  q.v0 = q.v1 = q.v2 = q.v3 = a;
  sh_edge<P>(q, a, b);
  sh_edge<P>(q, b, c);
  sh_edge<P>(q, c, a);
  return q;
}

__device__ __forceinline__ void blinn_vertex(const float4& p, float& nx, float& ny) {
  nx = fminf(fmaxf(p.x, -p.w), p.w) / p.w;
  ny = fminf(fmaxf(p.y, -p.w), p.w) / p.w;
}

// Blinn's coverage estimate of a polygon of 3 or 4 vertices.
__device__ __forceinline__ float4 blinn_box(const Quad& q) {
  bool bad = !(q.v0.w > 0.0f) || !(q.v1.w > 0.0f) || !(q.v2.w > 0.0f) ||
             (q.n == 4 && !(q.v3.w > 0.0f));
  if (bad) return make_float4(-1.0f, -1.0f, 1.0f, 1.0f);
  float x0, y0, x, y;
  blinn_vertex(q.v0, x0, y0);
  float4 b = make_float4(x0, y0, x0, y0);
  blinn_vertex(q.v1, x, y);
  b.x = fminf(b.x, x); b.y = fminf(b.y, y); b.z = fmaxf(b.z, x); b.w = fmaxf(b.w, y);
  blinn_vertex(q.v2, x, y);
  b.x = fminf(b.x, x); b.y = fminf(b.y, y); b.z = fmaxf(b.z, x); b.w = fmaxf(b.w, y);
  if (q.n == 4) {
    blinn_vertex(q.v3, x, y);
    b.x = fminf(b.x, x); b.y = fminf(b.y, y); b.z = fmaxf(b.z, x); b.w = fmaxf(b.w, y);
  }
  return b;
}

__device__ __forceinline__ float box_area(const float4& b) { return (b.z - b.x) * (b.w - b.y); }

template <int P>
__device__ __forceinline__ void try_plane(const float4& a, const float4& b, const float4& c,
                                          float4& best, float& best_area) {
  if (pdist<P>(a) < 0.0f || pdist<P>(b) < 0.0f || pdist<P>(c) < 0.0f) {
    float4 bp = blinn_box(clip_tri<P>(a, b, c));
    float ar = box_area(bp);
    if (ar < best_area) { best = bp; best_area = ar; }
  }
}

template <int P>
__device__ __forceinline__ bool all_out(const float4& a, const float4& b, const float4& c) {
  return pdist<P>(a) < 0.0f && pdist<P>(b) < 0.0f && pdist<P>(c) < 0.0f;
}

// Returns false when the triangle is entirely outside one plane of the view
// volume; otherwise the near-clipped or best-single-plane-clipped Blinn box.
__device__ __forceinline__ bool triangle_ndc_box(const float4& a, const float4& b,
                                                 const float4& c, bool side_clip, float4& box) {
  if (all_out<0>(a, b, c) || all_out<1>(a, b, c) || all_out<2>(a, b, c) ||
      all_out<3>(a, b, c) || all_out<4>(a, b, c) || all_out<5>(a, b, c))
    return false;
  if (pdist<4>(a) < 0.0f || pdist<4>(b) < 0.0f || pdist<4>(c) < 0.0f) {
    box = blinn_box(clip_tri<4>(a, b, c));
    return true;
  }
  Quad t;
  t.v0 = a; t.v1 = b; t.v2 = c; t.v3 = a; t.n = 3;
  float4 best = blinn_box(t);
  if (side_clip) {
    float ar = box_area(best);
    try_plane<0>(a, b, c, best, ar);
    try_plane<1>(a, b, c, best, ar);
    try_plane<2>(a, b, c, best, ar);
    try_plane<3>(a, b, c, best, ar);
    try_plane<5>(a, b, c, best, ar);
  }
  box = best;
  return true;
}

// Gather: chart of every visible triangle and its vertices, and the chart's
// box as the union of its triangles' boxes. Each thread handles kGatherItems
// triangles; lanes of a wave with the same chart are reduced in registers,
// then merged into a small per-workgroup table in LDS, and only the table is
// flushed with global atomics (large charts would otherwise serialize on
// their four accumulator words).
constexpr int kGatherItems = 8;
constexpr int kSlots = 64;

__global__ __launch_bounds__(kBlock) void k_gather_boxes(
    const uint8_t* __restrict__ vis, const int32_t* __restrict__ idx, int64_t T,
    const int32_t* __restrict__ parent, const float4* __restrict__ clip, int32_t* cot,
    int32_t* __restrict__ cov, uint32_t* __restrict__ accum, uint32_t flags,
    const FrameState* __restrict__ st) {
  __shared__ int32_t skey[kSlots];
  __shared__ uint32_t sbox[kSlots][4];
  if (st->status != FA_OK) return;
  for (int i = threadIdx.x; i < kSlots; i += blockDim.x) {
    skey[i] = -1;
    sbox[i][0] = sbox[i][1] = 0xFFFFFFFFu;
    sbox[i][2] = sbox[i][3] = 0u;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * (kBlock * kGatherItems);
  for (int k = 0; k < kGatherItems; ++k) {
    const int64_t t = base + (int64_t)k * kBlock + threadIdx.x;
    const bool valid = t < T;
    const bool visible = valid && vis[t];
    int c = -1;
    bool has = false;
    float4 box = make_float4(0.f, 0.f, 0.f, 0.f);
    if (visible) {
      c = cot[parent[t]];
      const int i0 = idx[3 * t], i1 = idx[3 * t + 1], i2 = idx[3 * t + 2];
      cov[i0] = c;
      cov[i1] = c;
      cov[i2] = c;
      has = triangle_ndc_box(clip[i0], clip[i1], clip[i2], !(flags & FA_FLAG_NO_SIDE_CLIP), box);
    }
    if (valid) cot[t] = c;
    const uint32_t e0 = ord_of(box.x), e1 = ord_of(box.y), e2 = ord_of(box.z), e3 = ord_of(box.w);
    unsigned long long todo = __ballot(has);
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int cl = __shfl(c, leader, kWave);
      const bool mine = has && c == cl;
      const unsigned long long grp = __ballot(mine);
      const uint32_t a0 = wave_min<uint32_t>(mine ? e0 : 0xFFFFFFFFu);
      const uint32_t a1 = wave_min<uint32_t>(mine ? e1 : 0xFFFFFFFFu);
      const uint32_t a2 = wave_max<uint32_t>(mine ? e2 : 0u);
      const uint32_t a3 = wave_max<uint32_t>(mine ? e3 : 0u);
      if (lane_id() == leader) {
        int h = cl & (kSlots - 1), slot = -1;
        for (int probe = 0; probe < kSlots; ++probe) {
          const int prev = atomicCAS(&skey[h], -1, cl);
          if (prev == -1 || prev == cl) { slot = h; break; }
          h = (h + 1) & (kSlots - 1);
        }
        if (slot >= 0) {
          atomicMin(&sbox[slot][0], a0);
          atomicMin(&sbox[slot][1], a1);
          atomicMax(&sbox[slot][2], a2);
          atomicMax(&sbox[slot][3], a3);
        } else {
          atomicMin(&accum[4 * cl + 0], a0);
          atomicMin(&accum[4 * cl + 1], a1);
          atomicMax(&accum[4 * cl + 2], a2);
          atomicMax(&accum[4 * cl + 3], a3);
        }
      }
      todo &= ~grp;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSlots; i += blockDim.x) {
    const int cl = skey[i];
    if (cl < 0) continue;
    atomicMin(&accum[4 * cl + 0], sbox[i][0]);
    atomicMin(&accum[4 * cl + 1], sbox[i][1]);
    atomicMax(&accum[4 * cl + 2], sbox[i][2]);
    atomicMax(&accum[4 * cl + 3], sbox[i][3]);
  }
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t launch_prologue(const float* pos, int64_t V, const uint8_t* vis, const int32_t* nbr,
                           int64_t T, const FrameParams& p, const Work& w, int32_t* cov,
                           int uf_link_init, hipStream_t st) {
  const unsigned vb = std::max(1u, grid_for(V, kBlock));
  k_prologue<<<vb + grid_for(T, kBlock), kBlock, 0, st>>>(pos, V, p, w.clip, w.vmin, cov, vis, nbr,
                                                          T, w.parent, uf_link_init, vb, w.state,
                                                          w.big_counter);
  return hipGetLastError();
}

hipError_t launch_charts(const uint8_t* vis, const int32_t* idx, const int32_t* nbr, int64_t T,
                         const FrameParams& p, const Work& w, int32_t* cot, int32_t* cov,
                         fa_chart* charts, Marker& mk, hipStream_t st) {
  const int64_t ntiles = (T + kTriTile - 1) / kTriTile;
  if (T > 0) {
    const unsigned g = grid_for(T, kBlock);
    k_uf_hook<<<g, kBlock, 0, st>>>(vis, nbr, idx, T, w.parent, w.vmin);
    mk(st);
    k_uf_vertex_hook<<<g, kBlock, 0, st>>>(vis, idx, T, w.parent, w.vmin);
    mk(st);
    k_uf_flatten_count<<<(unsigned)ntiles, kBlock, 0, st>>>(vis, T, w.parent, w.tile_count,
                                                            w.tile_vis);
  }
  mk(st);
  k_scan_tiles<<<1, 1024, 0, st>>>(w.tile_count, w.tile_vis, w.tile_off, ntiles, p.max_charts,
                                   w.state);
  mk(st);
  if (T > 0) {
    k_assign_roots<<<(unsigned)ntiles, kBlock, 0, st>>>(vis, T, w.parent, w.tile_off, cot, charts,
                                                        w.accum, w.state);
    mk(st);
    k_gather_boxes<<<grid_for(T, kBlock * kGatherItems), kBlock, 0, st>>>(
        vis, idx, T, w.parent, w.clip, cot, cov, w.accum, p.flags, w.state);
  }
  mk(st);
  return hipGetLastError();
}

}  // namespace fa
