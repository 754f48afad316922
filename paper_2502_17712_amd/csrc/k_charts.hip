// Chart stages of the per-frame path on gfx950:
//   clip transform, union-find charts (Appendix "GPU Union Find", Alg. 1),
//   root compaction, per-triangle conservative boxes (Sec. "Computing Bounding
//   Boxes of Projected Visible Sub-Charts") reduced per chart.
//
// Visible triangles are a small fraction of a scene (about 13% of the 2.2M
// triangles of a 4K frame), so the prologue compacts them once, in ascending
// index order, into a dense list; every later per-triangle kernel walks that
// list with full waves instead of masking out invisible lanes.
#include <algorithm>
#include <climits>

#include "fa_internal.h"

namespace fa {
namespace {

// ---------------------------------------------------------------------------
// union-find over visible triangles. parent[x] <= x always holds; a root has
// parent[x] == x. Walks inside a join use plain loads: a stale value (the
// eight XCDs have separate L2 caches) is an older ancestor, and the hooking
// compare-and-swap always sees the current value. Reads whose value is the
// result (vertex minima, the flattened root, the root test) are agent-scope
// atomic loads; every write of parent[] is an agent-scope atomic store.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int aload(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void astore(int32_t* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int uf_root(int32_t* parent, int x) {
  int cur = parent[x];
  if (cur == x) return x;
  int prev = x;
  for (;;) {
    int nxt = parent[cur];
    if (nxt >= cur) return cur;  // parent[cur] == cur
    astore(&parent[prev], nxt);
    prev = cur;
    cur = nxt;
  }
}

// The roots of u and of v by uf_root's walk, the two walks advancing
// together so that their dependent loads overlap.
__device__ __forceinline__ void uf_root2(int32_t* parent, int u, int v, int& ru, int& rv) {
  int cu = parent[u], cv = parent[v], pu = u, pv = v;
  bool du = cu == u, dv = cv == v;
  while (!(du && dv)) {
    const int nu = du ? cu : parent[cu];
    const int nv = dv ? cv : parent[cv];
    if (!du) {
      if (nu >= cu) {
        du = true;
      } else {
        astore(&parent[pu], nu);
        pu = cu;
        cu = nu;
      }
    }
    if (!dv) {
      if (nv >= cv) {
        dv = true;
      } else {
        astore(&parent[pv], nv);
        pv = cv;
        cv = nv;
      }
    }
  }
  ru = cu;
  rv = cv;
}

// Join the trees of u and v: the larger root is hooked below the smaller one
// with a compare-and-swap; on failure continue from the value that won.
__device__ __forceinline__ void uf_join(int32_t* parent, int u, int v) {
  int ru, rv;
  uf_root2(parent, u, v, ru, rv);
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

constexpr int kProVerts = 4;  // vertices per prologue thread
static_assert(kTriTile % kBlock == 0, "prologue threads take whole strides of a tile");

// Prologue of a frame: frame state, per-vertex scratch (vertex minima and
// chart_of_vert = -1; clip positions are computed where they are read),
// chart_of_tri = -1, the union-find start of every visible triangle and the
// visible count of every tile of kTriTile triangles. Blocks [0, vblocks)
// handle vertices, the rest triangle tiles. uf_init 2: a visible triangle
// starts linked to the smallest of itself and its visible edge neighbours
// (Alg. 1, first loop); 1: as its own root (same labels); 0: not written (a
// later pass writes it).
__device__ __forceinline__ void k_prologue_body(int64_t V, int32_t* __restrict__ vmin,
                           int32_t* __restrict__ cov, const uint8_t* __restrict__ vis,
                           const int32_t* __restrict__ nbr, int64_t T,
                           int32_t* __restrict__ parent, int32_t* __restrict__ cot,
                           uint32_t* __restrict__ tile_vis, int uf_init,
                           unsigned vblocks, FrameState* st,
                           unsigned long long* __restrict__ big_counter) {
  __shared__ uint32_t sh[kBlock / kWave];
  if (blockIdx.x < vblocks) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      FrameState s = {};
      s.status = FA_OK;
      *st = s;
      *big_counter = 0ull;
    }
    // kProVerts vertices per thread, a workgroup apart (contiguous stores)
    const int64_t v0 = (int64_t)blockIdx.x * (blockDim.x * kProVerts) + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kProVerts; ++k) {
      const int64_t v = v0 + (int64_t)k * blockDim.x;
      if (v < V) {
        astore(&vmin[v], INT_MAX);
        cov[v] = -1;
      }
    }
    return;
  }
  // four triangles of the tile per thread, a workgroup apart
  const unsigned tile = blockIdx.x - vblocks;
  const int64_t base = (int64_t)tile * kTriTile + (int64_t)threadIdx.x;
  uint32_t nv = 0;
#pragma unroll
  for (int k = 0; k < kTriTile / kBlock; ++k) {
    const int64_t t = base + (int64_t)k * kBlock;
    if (t >= T) break;
    cot[t] = -1;
    if (!vis[t]) continue;
    ++nv;
    int q = (int)t;
    if (uf_init == 2) {
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const int n = nbr[3 * t + e];
        if (n >= 0 && vis[n]) q = min(q, n);
      }
    }
    if (uf_init) astore(&parent[t], q);
  }
  nv = block_sum<uint32_t>(nv, sh);
  if (threadIdx.x == 0) tile_vis[tile] = nv;
}
__global__ void k_prologue(int64_t V, int32_t* __restrict__ vmin,
                           int32_t* __restrict__ cov, const uint8_t* __restrict__ vis,
                           const int32_t* __restrict__ nbr, int64_t T,
                           int32_t* __restrict__ parent, int32_t* __restrict__ cot,
                           uint32_t* __restrict__ tile_vis, int uf_init,
                           unsigned vblocks, FrameState* st,
                           unsigned long long* __restrict__ big_counter) {
  k_prologue_body(V, vmin, cov, vis, nbr, T, parent, cot, tile_vis, uf_init, vblocks, st, big_counter);
}

// Sum of cnt[0 .. n) by one workgroup (the exclusive prefix of tile n);
// each thread issues eight loads before it adds any.
__device__ __forceinline__ uint32_t tiles_before(const uint32_t* __restrict__ cnt, int64_t n,
                                                 uint32_t* sh) {
  uint32_t v = 0;
  for (int64_t u0 = threadIdx.x; u0 < n; u0 += 8 * (int64_t)blockDim.x) {
    uint32_t x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t u = u0 + (int64_t)j * blockDim.x;
      x[j] = u < n ? cnt[u] : 0u;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) v += x[j];
  }
  return block_sum<uint32_t>(v, sh);
}

// Exclusive prefix of the tiles' visible counts, in place, by one
// workgroup: each thread takes kScanPer consecutive tiles, one block scan
// (the compaction of a batched launch then reads its tile's offset instead of
// summing every earlier tile, which with many views in one launch costs more
// than this extra launch; one frame keeps the sums).
constexpr int kScanPer = 4;
__device__ __forceinline__ void k_tile_scan_body(uint32_t* tile_vis, unsigned tiles) {
  __shared__ uint32_t sh[1024 / kWave];
  uint32_t run = 0;
  for (unsigned b0 = 0; b0 < tiles; b0 += blockDim.x * kScanPer) {
    const unsigned i0 = b0 + threadIdx.x * kScanPer;
    uint32_t v[kScanPer], mine = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      v[k] = i0 + k < tiles ? tile_vis[i0 + k] : 0u;
      mine += v[k];
    }
    uint32_t tot;
    uint32_t at = run + block_incl_scan<uint32_t>(mine, sh, &tot) - mine;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      if (i0 + k < tiles) tile_vis[i0 + k] = at;
      at += v[k];
    }
    run += tot;
  }
}

// Stable compaction of the visible triangles into vlist (ascending index).
// For one frame each workgroup sums the visible counts of the tiles before
// its own (a few thousand words at most) instead of waiting for a separate
// scan; batched launches scan first (scanned). The last workgroup records
// the total.
__device__ __forceinline__ void k_vis_compact_body(const uint8_t* __restrict__ vis, int64_t T,
                              const uint32_t* __restrict__ tile_vis, int32_t* __restrict__ vlist,
                              FrameState* __restrict__ st, bool scanned = false) {
  __shared__ uint32_t sh[kBlock / kWave];
  // scanned: tile_vis holds each tile's exclusive prefix (k_tile_scan_body)
  const uint32_t off = scanned ? tile_vis[blockIdx.x] : tiles_before(tile_vis, blockIdx.x, sh);
  const int64_t base = (int64_t)blockIdx.x * kTriTile + (int64_t)threadIdx.x * 4;
  bool f[4];
  uint32_t mine = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    f[k] = base + k < T && vis[base + k];
    mine += f[k];
  }
  uint32_t tot;
  uint32_t at = off + block_incl_scan<uint32_t>(mine, sh, &tot) - mine;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (f[k]) vlist[at++] = (int32_t)(base + k);
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) st->visible = (int32_t)(off + tot);
}
__global__ void k_vis_compact(const uint8_t* __restrict__ vis, int64_t T,
                              const uint32_t* __restrict__ tile_vis, int32_t* __restrict__ vlist,
                              FrameState* __restrict__ st) {
  k_vis_compact_body(vis, T, tile_vis, vlist, st);
}

// Hook across every shared edge once (u < v) (Alg. 1, second loop).
// With tile > 0 only edges leaving the entry's tile of `tile` consecutive
// list entries are hooked (the others were joined inside the tile).
__global__ void k_uf_hook(const uint8_t* __restrict__ vis, const int32_t* __restrict__ nbr,
                          const int32_t* __restrict__ vlist, int32_t* parent, int tile,
                          const FrameState* __restrict__ st) {
  const int nv = st->visible;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) {
    const int t = vlist[i];
    const int last = tile > 0 ? vlist[min(nv, (i / tile + 1) * tile) - 1] : -1;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int n = nbr[3 * (int64_t)t + e];
      if (n > t && n > last && vis[n]) uf_join(parent, t, n);
    }
  }
}

// Edges between tiles, after the LDS pass: an edge (t, n) joins the sets of
// parent[t] and parent[n] (ancestors of t and n). Lanes of a wave whose edges
// name the same pair of parents keep only the lowest lane, so a pair that many
// edges along a tile border share is hooked once per wave instead of every
// lane contending for the same root.
__global__ void k_uf_cross(const uint8_t* __restrict__ vis, const int32_t* __restrict__ nbr,
                           const int32_t* __restrict__ vlist, int32_t* parent, int tile,
                           const FrameState* __restrict__ st) {
  const int nv = st->visible;
  const int lane = lane_id();
  for (int i0 = blockIdx.x * blockDim.x; i0 < nv; i0 += gridDim.x * blockDim.x) {
    const int i = i0 + threadIdx.x;
    const bool valid = i < nv;
    const int t = valid ? vlist[i] : 0;
    const int last = valid ? vlist[min(nv, (i / tile + 1) * tile) - 1] : 0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int n = valid ? nbr[3 * (int64_t)t + e] : -1;
      bool want = valid && n > last && vis[n];
      int a = 0, b = 0;
      if (want) {
        a = parent[t];
        b = parent[n];
        if (a > b) { const int s = a; a = b; b = s; }
        want = a != b;
      }
      // keep the lowest lane of every distinct (a, b)
      unsigned long long todo = __ballot(want);
      bool keep = false;
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int la = __shfl(a, leader, kWave), lb = __shfl(b, leader, kWave);
        const bool same = want && a == la && b == lb;
        if (lane == leader) keep = true;
        todo &= ~__ballot(same);
      }
      if (keep) uf_join(parent, a, b);
    }
  }
}

// Edge hooks inside one tile of TILE consecutive entries of the visible
// list, in LDS: entries are local indices (ascending with the triangle index),
// a shared edge whose other triangle lies in the tile joins the two local sets
// (larger local root hooked below the smaller by compare-and-swap). Then every
// entry's parent becomes the smallest triangle of its local set, which is a
// valid union-find start for the vertex passes; edges leaving the tile are
// shared vertices too, so those passes complete the charts.

__device__ __forceinline__ int lds_get(int* a, int i) {
  return __hip_atomic_load(&a[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_put(int* a, int i, int v) {
  __hip_atomic_store(&a[i], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int lds_root(int* lp, int x) {
  int p = lds_get(lp, x);
  while (p != x) {  // path splitting
    const int gp = lds_get(lp, p);
    if (gp != p) lds_put(lp, x, gp);
    x = p;
    p = gp;
  }
  return x;
}
__device__ __forceinline__ void lds_join(int* lp, int a, int b) {
  int ra = lds_root(lp, a), rb = lds_root(lp, b);
  while (ra != rb) {
    if (ra > rb) { const int s = ra; ra = rb; rb = s; }
    const int old = atomicCAS(&lp[rb], rb, ra);
    if (old == rb) return;
    rb = lds_root(lp, old);
  }
}

// With idx (hook mode 4), every entry also lowers the minimum of its three
// vertices to its local root: a vertex minimum only has to name some
// triangle of a set that touches the vertex, so the local root serves, and
// the vertex hook then joins every set that touches a common vertex (which
// covers the edges between tiles too).
template <int TILE, int NT>
__global__ __launch_bounds__(NT) void k_uf_local(const uint8_t* __restrict__ vis,
                                                 const int32_t* __restrict__ nbr,
                                                 const int32_t* __restrict__ vlist,
                                                 int32_t* __restrict__ parent,
                                                 const int32_t* __restrict__ idx,
                                                 int32_t* __restrict__ vmin,
                                                 const FrameState* __restrict__ st) {
  __shared__ int lv[TILE];
  __shared__ int lp[TILE];
  const int nv = st->visible;
  const int64_t s0 = (int64_t)blockIdx.x * TILE;
  if (s0 >= nv) return;
  const int cnt = (int)min<int64_t>(TILE, nv - s0);
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    lv[i] = vlist[s0 + i];
    lp[i] = i;
  }
  __syncthreads();
  const int last = lv[cnt - 1];
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int t = lv[i];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int n = nbr[3 * (int64_t)t + e];
      if (n > t && n <= last && vis[n]) {
        int lo = i + 1, hi = cnt - 1;  // n is in lv[lo..hi]
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (lv[mid] < n) lo = mid + 1; else hi = mid;
        }
        lds_join(lp, i, lo);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int t = lv[i], r = lv[lds_root(lp, i)];
    astore(&parent[t], r);
    if (idx) {
#pragma unroll
      for (int e = 0; e < 3; ++e) atomicMin(&vmin[idx[3 * (int64_t)t + e]], r);
    }
  }
}

// Hook mode 5: the tile of TILE list entries is joined in LDS through shared
// vertices instead of shared edges (a shared edge is a shared vertex): every
// vertex reference is entered into an LDS hash table of (vertex << 32 |
// entry) words, where the first entry to claim a vertex owns it; every entry
// is joined with the owners of its vertices, and so all entries naming one
// vertex end in one set. This also merges the pieces of a chart that touch
// only at a vertex inside the tile. A vertex that finds no free slot is
// skipped (the global vertex pass merges through every vertex anyway). Then,
// as in mode 4, each entry's parent becomes its local root and its vertices'
// minima are lowered to it.
// Workgroups past the tiles fill the occupancy map with -1 (occ_fill, n4
// 16-byte words) while the tiles' dependent loads leave memory bandwidth free.
template <int TILE, int NT, int HS>
__device__ __forceinline__ void k_uf_local_vertex_body(const int32_t* __restrict__ idx,
                                                        const int32_t* __restrict__ vlist,
                                                        int32_t* __restrict__ parent,
                                                        int32_t* __restrict__ vmin,
                                                        const FrameState* __restrict__ st,
                                                        int4* __restrict__ occ_fill, int64_t n4) {
  static_assert((HS & (HS - 1)) == 0, "hash slots: a power of two");
  static_assert(TILE % NT == 0, "whole entries per thread");
  constexpr int kPer = TILE / NT;  // entries per thread: i = threadIdx.x + k NT
  constexpr unsigned long long kFree = ~0ull;
  __shared__ int lv[TILE];
  __shared__ int lp[TILE];
  __shared__ unsigned long long tab[HS];
  const int nv = st->visible;
  const int64_t s0 = (int64_t)blockIdx.x * TILE;
  if (s0 >= nv) {
    if (occ_fill) {
      const int64_t active = ((int64_t)nv + TILE - 1) / TILE;
      const int64_t nb = (int64_t)gridDim.x - active;
      const int4 neg = make_int4(-1, -1, -1, -1);
      for (int64_t i = ((int64_t)blockIdx.x - active) * NT + threadIdx.x; i < n4; i += nb * NT)
        occ_fill[i] = neg;
    }
    return;
  }
  const int cnt = (int)min<int64_t>(TILE, nv - s0);
  // every entry's triangle and vertices are loaded up front (the loads of
  // a thread's entries overlap) and kept in registers until the end
  int tk[kPer], vk[kPer][3];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * NT;
    tk[k] = i < cnt ? vlist[s0 + i] : 0;
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * NT;
#pragma unroll
    for (int e = 0; e < 3; ++e) vk[k][e] = i < cnt ? idx[3 * (int64_t)tk[k] + e] : 0;
    if (i < cnt) {
      lv[i] = tk[k];
      lp[i] = i;
    }
  }
  for (int h = threadIdx.x; h < HS; h += NT) tab[h] = kFree;
  __syncthreads();
  // 1. every vertex reference enters the hash table; the first entry to
  //    claim a vertex's slot owns it
  int hs[kPer][3];  // slot of each reference, -1 when the table had no room
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * NT;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      hs[k][e] = -1;
      if (i >= cnt) continue;
      const int v = vk[k][e];
      const unsigned long long mine = ((unsigned long long)(uint32_t)v << 32) | (uint32_t)i;
      uint32_t h = ((uint32_t)v * 2654435761u) & (HS - 1);
      for (int probe = 0; probe < 32; ++probe) {
        const unsigned long long old = atomicCAS(&tab[h], kFree, mine);
        if (old == kFree) {  // first entry with this vertex
          hs[k][e] = (int)h;
          break;
        }
        if ((uint32_t)(old >> 32) == (uint32_t)v) {  // another entry owns it
          hs[k][e] = (int)h;
          break;
        }
        h = (h + 1) & (HS - 1);
      }
    }
  }
  __syncthreads();
  // 2. each entry starts linked to the smallest of itself and the owners of
  //    its vertices (never above itself, so no cycles), then one step
  //    towards that node's own start
  int mo[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * NT;
    mo[k] = i;
#pragma unroll
    for (int e = 0; e < 3; ++e)
      if (hs[k][e] >= 0) mo[k] = min(mo[k], (int)(uint32_t)tab[hs[k][e]]);
    if (i < cnt) lp[i] = mo[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * NT;
    if (i >= cnt) continue;
    const int q = lds_get(lp, mo[k]);
    if (q != mo[k]) lds_put(lp, i, q);
  }
  __syncthreads();
  // 3. each entry joins the owners of its other vertices (none when both
  //    already hang from the same node)
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * NT;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      if (hs[k][e] < 0) continue;
      const int o = (int)(uint32_t)tab[hs[k][e]];
      if (o == mo[k] || lds_get(lp, o) == lds_get(lp, i)) continue;
      lds_join(lp, i, o);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * NT;
    if (i >= cnt) continue;
    const int r = lv[lds_root(lp, i)];
    astore(&parent[tk[k]], r);
    // every reference to a vertex in the tile is in this set, so the owner's
    // reference alone lowers the vertex minimum (and each reference that
    // found no slot lowers its own)
#pragma unroll
    for (int e = 0; e < 3; ++e)
      if (hs[k][e] < 0 || (int)(uint32_t)tab[hs[k][e]] == i) atomicMin(&vmin[vk[k][e]], r);
  }
}
template <int TILE, int NT, int HS>
__global__ __launch_bounds__(NT) void k_uf_local_vertex(const int32_t* __restrict__ idx,
                                                        const int32_t* __restrict__ vlist,
                                                        int32_t* __restrict__ parent,
                                                        int32_t* __restrict__ vmin,
                                                        const FrameState* __restrict__ st,
                                                        int4* __restrict__ occ_fill, int64_t n4) {
  k_uf_local_vertex_body<TILE, NT, HS>(idx, vlist, parent, vmin, st, occ_fill, n4);
}

// Vertex minimum (Alg. 1, third loop): every visible triangle is compressed
// to its current root and every vertex records the smallest root among its
// visible triangles. The compression keeps the vertex hook's walks short.
__global__ void k_uf_vertex_min(const int32_t* __restrict__ idx,
                                const int32_t* __restrict__ vlist, int32_t* parent,
                                int32_t* __restrict__ vmin, const FrameState* __restrict__ st) {
  const int nv = st->visible;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) {
    const int t = vlist[i];
    const int r = uf_root(parent, t);
    if (r != t) astore(&parent[t], r);
#pragma unroll
    for (int e = 0; e < 3; ++e) atomicMin(&vmin[idx[3 * (int64_t)t + e]], r);
  }
}

// Threads per vertex-hook workgroup: one workgroup's pair set then covers
// 1024 list entries (four times the repeats of 256-thread workgroups; one
// frame's hook 21.6 -> 19.7 us).
constexpr unsigned kHookThreads = 1024;

// Vertex hook: join every visible triangle with the recorded root of each of
// its vertices, merging charts that share only a vertex. parent[t] is an
// ancestor of t: a vertex whose minimum equals it needs no join, which skips
// most of them; along a tile border many lanes of a wave name the same
// (parent, minimum) pair, and only the lowest lane of each pair joins, once
// per workgroup (an LDS set of the pairs taken).
__device__ __forceinline__ void k_uf_vertex_hook_body(const int32_t* __restrict__ idx,
                                 const int32_t* __restrict__ vlist, int32_t* parent,
                                 const int32_t* __restrict__ vmin,
                                 const FrameState* __restrict__ st) {
  // ordered (parent, minimum) pairs this workgroup has joined or is
  // joining: a repeated pair needs no second join
  constexpr int kPairSlots = 512;
  __shared__ unsigned long long pairs[kPairSlots];
  for (int h = threadIdx.x; h < kPairSlots; h += blockDim.x) pairs[h] = ~0ull;
  __syncthreads();
  const int nv = st->visible;
  const int lane = lane_id();
  for (int i0 = blockIdx.x * blockDim.x; i0 < nv; i0 += gridDim.x * blockDim.x) {
    const int i = i0 + threadIdx.x;
    const bool valid = i < nv;
    int pt = 0, m[3] = {0, 0, 0};
    if (valid) {
      const int t = vlist[i];
#pragma unroll
      for (int e = 0; e < 3; ++e) m[e] = aload(&vmin[idx[3 * (int64_t)t + e]]);
      pt = aload(&parent[t]);
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      bool want = valid && m[e] != pt && (e < 1 || m[e] != m[0]) && (e < 2 || m[e] != m[1]);
      const int a = min(pt, m[e]), b = max(pt, m[e]);
      unsigned long long todo = __ballot(want);
      bool keep = false;
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int la = __shfl(a, leader, kWave), lb = __shfl(b, leader, kWave);
        if (lane == leader) keep = true;
        todo &= ~__ballot(want && a == la && b == lb);
      }
      if (keep) {
        const unsigned long long key = ((unsigned long long)(uint32_t)a << 32) | (uint32_t)b;
        uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 40) & (kPairSlots - 1);
        bool fresh = true;
        for (int probe = 0; probe < 16; ++probe) {
          const unsigned long long old = atomicCAS(&pairs[h], ~0ull, key);
          if (old == ~0ull) break;
          if (old == key) {
            fresh = false;
            break;
          }
          h = (h + 1) & (kPairSlots - 1);
        }
        if (fresh) uf_join(parent, a, b);  // a full table only costs extra joins
      }
    }
  }
}
__global__ __launch_bounds__(kHookThreads) void k_uf_vertex_hook(const int32_t* __restrict__ idx,
                                 const int32_t* __restrict__ vlist, int32_t* parent,
                                 const int32_t* __restrict__ vmin,
                                 const FrameState* __restrict__ st) {
  k_uf_vertex_hook_body(idx, vlist, parent, vmin, st);
}

// Flatten every visible triangle to its root and count roots per tile of
// kTriTile consecutive entries of the visible list. The walk here only reads:
// a path-halving store by one thread (parent[x] = a grandparent it read
// earlier) could land after another thread has set parent[x] to the root and
// leave x pointing at a non-root, which the later stages would read as the
// chart's root.
__device__ __forceinline__ void k_uf_flatten_count_body(const int32_t* __restrict__ vlist, int32_t* parent,
                                   uint32_t* __restrict__ tile_count,
                                   const FrameState* __restrict__ st) {
  __shared__ uint32_t sh[kBlock / kWave];
  const int nv = st->visible;
  const int64_t base = (int64_t)blockIdx.x * kTriTile + (int64_t)threadIdx.x * 4;
  if ((int64_t)blockIdx.x * kTriTile >= nv) return;
  // the four walks of a thread advance together, so that their dependent
  // loads are in flight at the same time (constant indices keep the arrays
  // in registers)
  int t[4], r[4], up[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) t[k] = base + k < nv ? vlist[base + k] : -1;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r[k] = t[k];
    up[k] = t[k] >= 0 ? aload(&parent[t[k]]) : t[k];
  }
  bool more = true;
  while (more) {
    more = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (up[k] != r[k]) {
        r[k] = up[k];
        up[k] = aload(&parent[r[k]]);
        more = true;
      }
    }
  }
  uint32_t roots = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (t[k] < 0) continue;
    if (r[k] != t[k]) astore(&parent[t[k]], r[k]);
    roots += (r[k] == t[k]);
  }
  roots = block_sum<uint32_t>(roots, sh);
  if (threadIdx.x == 0) tile_count[blockIdx.x] = roots;
}
__global__ void k_uf_flatten_count(const int32_t* __restrict__ vlist, int32_t* parent,
                                   uint32_t* __restrict__ tile_count,
                                   const FrameState* __restrict__ st) {
  k_uf_flatten_count_body(vlist, parent, tile_count, st);
}

// Chart index of each root = its rank among roots; the visible list ascends
// with the triangle index, so chart indices ascend with the chart's lowest
// triangle. Each workgroup sums the root counts of the tiles before its own;
// the last one records the chart count (above max_charts: FA_ERR_CAPACITY;
// no chart index at or past max_charts is written, and every later stage
// stops on the status).
__device__ __forceinline__ void k_assign_roots_body(const int32_t* __restrict__ vlist,
                               const int32_t* __restrict__ parent,
                               const uint32_t* __restrict__ tile_count, int32_t* __restrict__ cot,
                               fa_chart* __restrict__ charts, uint32_t* __restrict__ accum,
                               int32_t max_charts, FrameState* __restrict__ st) {
  __shared__ uint32_t sh[kBlock / kWave];
  if (st->status != FA_OK) return;
  const int nv = st->visible;
  if ((int64_t)blockIdx.x * kTriTile >= nv) return;
  const uint32_t off = tiles_before(tile_count, blockIdx.x, sh);
  const int64_t base = (int64_t)blockIdx.x * kTriTile + (int64_t)threadIdx.x * 4;
  bool root[4];
  int tv[4];
  uint32_t mine = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + k;
    tv[k] = i < nv ? vlist[i] : -1;
    root[k] = tv[k] >= 0 && aload(&parent[tv[k]]) == tv[k];
    mine += root[k];
  }
  uint32_t tot;
  uint32_t c = off + block_incl_scan<uint32_t>(mine, sh, &tot) - mine;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!root[k]) continue;
    if (c < (uint32_t)max_charts) {
      cot[tv[k]] = (int32_t)c;
      charts[c].root_tri = tv[k];
      reinterpret_cast<uint4*>(accum)[c] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u);
    }
    ++c;
  }
  if ((int64_t)(blockIdx.x + 1) * kTriTile >= nv && threadIdx.x == 0) {
    const uint32_t total = off + tot;
    st->num_charts = (int32_t)total;  // reported even when above the capacity
    if (total > (uint32_t)max_charts) st->status = FA_ERR_CAPACITY;
  }
}
__global__ void k_assign_roots(const int32_t* __restrict__ vlist,
                               const int32_t* __restrict__ parent,
                               const uint32_t* __restrict__ tile_count, int32_t* __restrict__ cot,
                               fa_chart* __restrict__ charts, uint32_t* __restrict__ accum,
                               int32_t max_charts, FrameState* __restrict__ st) {
  k_assign_roots_body(vlist, parent, tile_count, cot, charts, accum, max_charts, st);
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

// Append a vertex. Value selects on every slot (not a branch per slot, which
// the optimizer turns into a runtime-indexed store that moves the polygon to
// scratch memory).
__device__ __forceinline__ float4 pick(bool c, const float4& a, const float4& b) {
  return make_float4(c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z, c ? a.w : b.w);
}
__device__ __forceinline__ void quad_put(Quad& q, const float4& p) {
  const int n = q.n;
  q.v0 = pick(n == 0, p, q.v0);
  q.v1 = pick(n == 1, p, q.v1);
  q.v2 = pick(n == 2, p, q.v2);
  q.v3 = pick(n >= 3, p, q.v3);
  q.n = n + 1;
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
// entries of the visible list, issuing the dependent loads of all its entries
// level by level (list, root, chart and indices, clip vertices) so that their
// latencies overlap; lanes of a wave with the same chart are reduced in
// registers, then merged into a small per-workgroup table in LDS, and only the
// table is flushed with global atomics (large charts would otherwise
// serialize on their four accumulator words).
constexpr int kGatherItems = 2;
// threads per gather workgroup: one LDS chart table per 1024 entries
// (256: 16.4 us, 512: 13.9 us, 1024: 16.4 us for one city frame)
constexpr int kGatherBlock = 512;
constexpr int kSlots = 64;
constexpr unsigned kFillBlocks = 1024;  // least workgroups that fill the occupancy map
constexpr unsigned kFillGroups = 256;   // the same for the 1024-thread union-find tiles

__device__ __forceinline__ void k_gather_boxes_body(
    const int32_t* __restrict__ vlist, const int32_t* __restrict__ idx,
    const int32_t* __restrict__ parent, const float* __restrict__ pos, int32_t* cot,
    int32_t* __restrict__ cov, uint32_t* __restrict__ accum, const FrameParams& p,
    const FrameState* __restrict__ st, int4* __restrict__ occ_fill, int64_t n4) {
  __shared__ int32_t skey[kSlots];
  __shared__ uint32_t sbox[kSlots][4];
  const int nv = st->visible;
  const int64_t per = kGatherBlock * kGatherItems;
  const int64_t active = (nv + per - 1) / per;
  if ((int64_t)blockIdx.x >= active) {
    // workgroups past the gather's own fill the occupancy map with -1
    if (occ_fill) {
      const int64_t nb = (int64_t)gridDim.x - active;
      const int4 neg = make_int4(-1, -1, -1, -1);
      for (int64_t i = ((int64_t)blockIdx.x - active) * kGatherBlock + threadIdx.x; i < n4;
           i += nb * kGatherBlock)
        occ_fill[i] = neg;
    }
    return;
  }
  if (st->status != FA_OK) return;
  const int64_t base = (int64_t)blockIdx.x * per;
  for (int i = threadIdx.x; i < kSlots; i += blockDim.x) {
    skey[i] = -1;
    sbox[i][0] = sbox[i][1] = 0xFFFFFFFFu;
    sbox[i][2] = sbox[i][3] = 0u;
  }
  __syncthreads();
  int tv[kGatherItems], cv[kGatherItems], vi[kGatherItems][3];
  float4 q[kGatherItems][3];
#pragma unroll
  for (int k = 0; k < kGatherItems; ++k) {
    const int64_t i = base + (int64_t)k * kGatherBlock + threadIdx.x;
    tv[k] = i < nv ? vlist[i] : -1;
  }
#pragma unroll
  for (int k = 0; k < kGatherItems; ++k) cv[k] = tv[k] >= 0 ? aload(&parent[tv[k]]) : 0;
#pragma unroll
  for (int k = 0; k < kGatherItems; ++k) {
    const int t = max(tv[k], 0);
    cv[k] = tv[k] >= 0 ? cot[cv[k]] : -1;
#pragma unroll
    for (int e = 0; e < 3; ++e) vi[k][e] = tv[k] >= 0 ? idx[3 * (int64_t)t + e] : 0;
  }
#pragma unroll
  for (int k = 0; k < kGatherItems; ++k)
#pragma unroll
    for (int e = 0; e < 3; ++e) q[k][e] = clip_of(pos, vi[k][e], p);
  // items are taken from slot 0 and shifted down after each one: constant
  // indices keep the arrays in registers (the clipping body is too large to
  // unroll, and a runtime index would move them to scratch memory)
  for (int k = 0; k < kGatherItems; ++k) {
    const bool valid = tv[0] >= 0;
    const int c = cv[0];
    bool has = false;
    float4 box = make_float4(0.f, 0.f, 0.f, 0.f);
    if (valid) {
      cot[tv[0]] = c;
      if (p.flags & FA_FLAG_EDGE_ONLY_CHARTS) {
        // a vertex may touch several edge-connected charts: keep the smallest
        // (chart_of_vert starts at -1, the largest unsigned value)
#pragma unroll
        for (int e = 0; e < 3; ++e)
          atomicMin(reinterpret_cast<uint32_t*>(&cov[vi[0][e]]), (uint32_t)c);
      } else {
        cov[vi[0][0]] = c;
        cov[vi[0][1]] = c;
        cov[vi[0][2]] = c;
      }
      has = triangle_ndc_box(q[0][0], q[0][1], q[0][2], !(p.flags & FA_FLAG_NO_SIDE_CLIP), box);
    }
#pragma unroll
    for (int m = 0; m + 1 < kGatherItems; ++m) {
      tv[m] = tv[m + 1];
      cv[m] = cv[m + 1];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        vi[m][e] = vi[m + 1][e];
        q[m][e] = q[m + 1][e];
      }
    }
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
__global__ __launch_bounds__(kGatherBlock) void k_gather_boxes(
    const int32_t* __restrict__ vlist, const int32_t* __restrict__ idx,
    const int32_t* __restrict__ parent, const float* __restrict__ pos, int32_t* cot,
    int32_t* __restrict__ cov, uint32_t* __restrict__ accum, FrameParams p,
    const FrameState* __restrict__ st, int4* __restrict__ occ_fill, int64_t n4) {
  k_gather_boxes_body(vlist, idx, parent, pos, cot, cov, accum, p, st, occ_fill, n4);
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

__global__ void k_flag_clear(int32_t* flag) { *flag = 0; }

__global__ void k_index_check(const int32_t* __restrict__ idx, int64_t n, int64_t V,
                              int32_t* flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = idx[i];
    bad = bad || v < 0 || (int64_t)v >= V;
  }
  if (__ballot(bad) && lane_id() == 0) atomicExch(flag, 1);
}

__global__ void k_index_guard(const int32_t* __restrict__ flag, FrameState* st) {
  if (*flag) {
    st->status = FA_ERR_INVALID_ARG;
    st->visible = 0;
  }
}

// ---- batched wrappers (view = blockIdx.y) --------------------------------
__global__ void k_prologue_b(const BatchView* __restrict__ bv, int64_t V, const int32_t* __restrict__ nbr, int64_t T,
                             unsigned vblocks) {
  const BatchView& v = bv[blockIdx.y];
  k_prologue_body(V, v.w.vmin, v.cov, v.visible, nbr, T, v.w.parent, v.cot,
                  v.w.tile_vis, 0, vblocks, v.w.state, v.w.big_counter);
}
__global__ __launch_bounds__(1024) void k_tile_scan_b(const BatchView* __restrict__ bv,
                                                      unsigned tiles) {
  k_tile_scan_body(bv[blockIdx.y].w.tile_vis, tiles);
}
__global__ void k_vis_compact_b(const BatchView* __restrict__ bv, int64_t T) {
  const BatchView& v = bv[blockIdx.y];
  k_vis_compact_body(v.visible, T, v.w.tile_vis, v.w.vlist, v.w.state, true);
}
__global__ __launch_bounds__(1024) void k_uf_local_vertex_b(const BatchView* __restrict__ bv,
                                                            const int32_t* __restrict__ idx) {
  const BatchView& v = bv[blockIdx.y];
  k_uf_local_vertex_body<2048, 1024, 4096>(idx, v.w.vlist, v.w.parent, v.w.vmin, v.w.state,
                                           reinterpret_cast<int4*>(v.occ),
                                           (int64_t)v.p.omega * v.p.omega / 4);
}
__global__ __launch_bounds__(kHookThreads) void k_uf_vertex_hook_b(const BatchView* __restrict__ bv,
                                   const int32_t* __restrict__ idx) {
  const BatchView& v = bv[blockIdx.y];
  k_uf_vertex_hook_body(idx, v.w.vlist, v.w.parent, v.w.vmin, v.w.state);
}
__global__ void k_uf_flatten_count_b(const BatchView* __restrict__ bv) {
  const BatchView& v = bv[blockIdx.y];
  k_uf_flatten_count_body(v.w.vlist, v.w.parent, v.w.tile_count, v.w.state);
}
__global__ void k_assign_roots_b(const BatchView* __restrict__ bv) {
  const BatchView& v = bv[blockIdx.y];
  k_assign_roots_body(v.w.vlist, v.w.parent, v.w.tile_count, v.cot, v.charts, v.w.accum,
                      v.p.max_charts, v.w.state);
}
__global__ __launch_bounds__(kGatherBlock) void k_gather_boxes_b(const BatchView* __restrict__ bv,
                                                           const int32_t* __restrict__ idx) {
  const BatchView& v = bv[blockIdx.y];
  k_gather_boxes_body(v.w.vlist, idx, v.w.parent, v.w.pos, v.cot, v.cov, v.w.accum, v.p,
                      v.w.state, nullptr, 0);
}

}  // namespace

hipError_t launch_index_check(const int32_t* idx, int64_t n, int64_t V, int32_t* flag,
                              hipStream_t st) {
  k_flag_clear<<<1, 1, 0, st>>>(flag);
  if (n > 0)
    k_index_check<<<(unsigned)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        idx, n, V, flag);
  return hipGetLastError();
}

hipError_t launch_index_guard(const int32_t* flag, const Work& w, hipStream_t st) {
  k_index_guard<<<1, 1, 0, st>>>(flag, w.state);
  return hipGetLastError();
}

unsigned visible_grid(int64_t T) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((T + kBlock - 1) / kBlock, 2048));
}

hipError_t launch_prologue(int64_t V, const uint8_t* vis, const int32_t* nbr,
                           int64_t T, const FrameParams& p, const Work& w, int32_t* cov,
                           int32_t* cot, int uf_init, Marker& mk, hipStream_t st) {
  const unsigned vb = std::max(1u, grid_for(V, kBlock * kProVerts));
  const unsigned tt = grid_for(T, kTriTile);
  k_prologue<<<vb + tt, kBlock, 0, st>>>(V, w.vmin, cov, vis, nbr, T, w.parent,
                                         cot, w.tile_vis, uf_init, vb, w.state,
                                         w.big_counter);
  mk(st);
  mk(st);  // (the visible-count scan is part of the compaction)
  if (T > 0) k_vis_compact<<<tt, kBlock, 0, st>>>(vis, T, w.tile_vis, w.vlist, w.state);
  mk(st);
  return hipGetLastError();
}

hipError_t launch_charts(const uint8_t* vis, const int32_t* idx, const int32_t* nbr, int64_t T,
                         const FrameParams& p, const Work& w, int32_t* cot, int32_t* cov,
                         fa_chart* charts, int32_t* occ_fill, Marker& mk, hipStream_t st) {
  const unsigned g = visible_grid(T);
  const unsigned vt = std::max(1u, grid_for(T, kTriTile));
  const int64_t n4 = (int64_t)p.omega * p.omega / 4;
  bool fill_done = false;
  if (T > 0 && (p.flags & FA_FLAG_EDGE_ONLY_CHARTS)) {
    // edge-connected charts: shared edges only, no vertex passes
    if (p.edge_hooks == 1) {
      k_uf_hook<<<g, kBlock, 0, st>>>(vis, nbr, w.vlist, w.parent, 0, w.state);
    } else {
      const int tile = p.uf_tile;
      if (tile == 8192)
        k_uf_local<8192, 1024><<<std::max(1u, grid_for(T, 8192)), 1024, 0, st>>>(
            vis, nbr, w.vlist, w.parent, nullptr, w.vmin, w.state);
      else if (tile == 4096)
        k_uf_local<4096, 1024><<<std::max(1u, grid_for(T, 4096)), 1024, 0, st>>>(
            vis, nbr, w.vlist, w.parent, nullptr, w.vmin, w.state);
      else
        k_uf_local<2048, 512><<<std::max(1u, grid_for(T, 2048)), 512, 0, st>>>(
            vis, nbr, w.vlist, w.parent, nullptr, w.vmin, w.state);
      k_uf_cross<<<g, kBlock, 0, st>>>(vis, nbr, w.vlist, w.parent, tile, w.state);
    }
    mk(st);
    mk(st);
    mk(st);
    k_uf_flatten_count<<<vt, kBlock, 0, st>>>(w.vlist, w.parent, w.tile_count, w.state);
  } else if (T > 0) {
    if (p.edge_hooks == 1) {
      k_uf_hook<<<g, kBlock, 0, st>>>(vis, nbr, w.vlist, w.parent, 0, w.state);
    } else if (p.edge_hooks == 5) {
      // tiles of 2048 entries and a 4096-slot table (at most ~3/4 full); at
      // least kFillGroups workgroups past the largest visible list fill the
      // occupancy map
      k_uf_local_vertex<2048, 1024, 4096>
          <<<std::max(1u, grid_for(T, 2048)) + (occ_fill ? kFillGroups : 0u), 1024, 0, st>>>(
              idx, w.vlist, w.parent, w.vmin, w.state, reinterpret_cast<int4*>(occ_fill), n4);
      fill_done = true;
    } else if (p.edge_hooks >= 2) {
      const int tile = p.uf_tile;
      const int32_t* vidx = p.edge_hooks == 4 ? idx : nullptr;
      if (tile == 8192)
        k_uf_local<8192, 1024><<<std::max(1u, grid_for(T, 8192)), 1024, 0, st>>>(
            vis, nbr, w.vlist, w.parent, vidx, w.vmin, w.state);
      else if (tile == 4096)
        k_uf_local<4096, 1024><<<std::max(1u, grid_for(T, 4096)), 1024, 0, st>>>(
            vis, nbr, w.vlist, w.parent, vidx, w.vmin, w.state);
      else
        k_uf_local<2048, 512><<<std::max(1u, grid_for(T, 2048)), 512, 0, st>>>(
            vis, nbr, w.vlist, w.parent, vidx, w.vmin, w.state);
      if (p.edge_hooks == 2)
        k_uf_cross<<<g, kBlock, 0, st>>>(vis, nbr, w.vlist, w.parent, tile, w.state);
    }
    mk(st);
    if (p.edge_hooks < 4)  // modes 4, 5: the tile kernel lowered the vertex minima
      k_uf_vertex_min<<<g, kBlock, 0, st>>>(idx, w.vlist, w.parent, w.vmin, w.state);
    mk(st);
    k_uf_vertex_hook<<<std::max(1u, g * kBlock / kHookThreads), kHookThreads, 0, st>>>(
        idx, w.vlist, w.parent, w.vmin, w.state);
    mk(st);
    k_uf_flatten_count<<<vt, kBlock, 0, st>>>(w.vlist, w.parent, w.tile_count, w.state);
  } else {
    mk(st);
    mk(st);
    mk(st);
  }
  mk(st);
  mk(st);  // (the root-count scan is part of the root assignment)
  if (T > 0) {
    k_assign_roots<<<vt, kBlock, 0, st>>>(w.vlist, w.parent, w.tile_count, cot, charts, w.accum,
                                          p.max_charts, w.state);
    mk(st);
    // the fill, unless the union-find tile kernel did it: at least kFillBlocks
    // workgroups beyond the largest visible list
    int32_t* gfill = fill_done ? nullptr : occ_fill;
    const unsigned fill_blocks = gfill ? kFillBlocks : 0u;
    k_gather_boxes<<<grid_for(T, kGatherBlock * kGatherItems) + fill_blocks, kGatherBlock, 0,
                     st>>>(
        w.vlist, idx, w.parent, w.pos, cot, cov, w.accum, p, w.state,
        reinterpret_cast<int4*>(gfill), n4);
  } else {
    mk(st);
  }
  mk(st);
  return hipGetLastError();
}

hipError_t launch_charts_batched(const BatchView* dev, int n, const float* pos,
                                 const int32_t* idx, const int32_t* nbr, int64_t T, int64_t V,
                                 hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned vb = std::max(1u, grid_for(V, kBlock * kProVerts));
  const unsigned tt = grid_for(T, kTriTile);
  const unsigned vt = std::max(1u, tt);
  k_prologue_b<<<dim3(vb + tt, n), kBlock, 0, st>>>(dev, V, nbr, T, vb);
  if (T > 0) {
    k_tile_scan_b<<<dim3(1, n), 1024, 0, st>>>(dev, tt);
    k_vis_compact_b<<<dim3(tt, n), kBlock, 0, st>>>(dev, T);
    k_uf_local_vertex_b<<<dim3(std::max(1u, grid_for(T, 2048)) + kFillGroups, n), 1024, 0, st>>>(
        dev, idx);
    k_uf_vertex_hook_b<<<dim3(std::max(1u, visible_grid(T) * kBlock / kHookThreads), n),
                         kHookThreads, 0, st>>>(dev, idx);
    k_uf_flatten_count_b<<<dim3(vt, n), kBlock, 0, st>>>(dev);
    k_assign_roots_b<<<dim3(vt, n), kBlock, 0, st>>>(dev);
    k_gather_boxes_b<<<dim3(grid_for(T, kGatherBlock * kGatherItems), n), kGatherBlock, 0, st>>>(
        dev, idx);
  }
  return hipGetLastError();
}

}  // namespace fa
