// Atlas-space stages on gfx950:
//   UV emission (Appendix "Shading and Rasterization": every chart is scaled
//   by the chosen uniform scale, then moved rigidly from its NDC box to its
//   atlas box) and the atlas occupancy map (which chart owns each texel).
//
// Occupancy of texel (tx, ty) is chart c iff its centre lies in c's placed
// box (exact integer test in layout space, gutter included) and inside one of
// c's visible triangles mapped to the atlas (near-clipped when the triangle
// crosses the near plane), snapped to 1/256 texel with round-to-nearest-even,
// fan-triangulated from the first vertex, edges inclusive. Small footprints
// are rasterized by one lane, medium ones by their wave, large ones are queued
// and cut into 16x16 tiles shared by all waves.
#include <algorithm>
#include <climits>

#include "fa_internal.h"

namespace fa {
namespace {

struct ChartXform {
  float x0, y1, tw, halfW, halfH, rate, s, q, ox, oy;
  int rot;
};

__device__ __forceinline__ ChartXform chart_xform(const fa_chart& ch, const FrameParams& p,
                                                  const FrameState& st) {
  ChartXform m;
  m.x0 = ch.ndc_box[0];
  m.y1 = ch.ndc_box[3];
  m.tw = ch.target_w;
  m.halfW = 0.5f * (float)p.W;
  m.halfH = 0.5f * (float)p.H;
  m.rate = p.rate;
  m.s = st.s_star;
  m.q = (float)p.omega / (float)st.layout_w;  // omega/L (the atlas side being drawn)
  m.ox = (float)(ch.x + p.gutter);
  m.oy = (float)(ch.y + p.gutter);
  m.rot = ch.rotated;
  return m;
}

// clip-space point (w > 0) -> atlas texel coordinates
__device__ __forceinline__ float2 to_atlas(const ChartXform& m, float X, float Y, float w) {
  const float nx = X / w, ny = Y / w;
  const float px = ((nx - m.x0) * m.halfW) * m.rate;
  const float py = ((m.y1 - ny) * m.halfH) * m.rate;
  const float lx = m.rot ? py : px;
  const float ly = m.rot ? (m.tw - px) : py;
  return make_float2((m.ox + lx * m.s) * m.q, (m.oy + ly * m.s) * m.q);
}

// Per-vertex UVs of workgroup ub of a UV grid (k_uv, or the workgroups past
// the small-footprint raster's own, which need the same placement and run
// beside the raster instead of after it): each thread takes PER vertices a
// workgroup apart, so every load and store of a wave is one contiguous run,
// and issues their chart loads before any dependent load.
template <int PER>
__device__ __forceinline__ void uv_block(unsigned ub, const FrameParams& p,
                                         const float* __restrict__ pos,
                                         const int32_t* __restrict__ cov,
                                         const fa_chart* __restrict__ charts,
                                         float2* __restrict__ uv, int64_t V,
                                         const FrameState* __restrict__ stp) {
  const FrameState st = *stp;
  const int64_t v0 = (int64_t)ub * (blockDim.x * PER) + threadIdx.x;
  int c[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int64_t v = v0 + (int64_t)k * blockDim.x;
    c[k] = (v < V && st.status == FA_OK) ? cov[v] : -1;
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int64_t v = v0 + (int64_t)k * blockDim.x;
    float2 r = make_float2(__builtin_nanf(""), __builtin_nanf(""));
    if (c[k] >= 0) {  // a vertex without a chart needs no position
      const float4 q = clip_of(pos, v, p);
      if (q.w > 0.0f) r = to_atlas(chart_xform(charts[c[k]], p, st), q.x, q.y, q.w);
    }
    if (v < V) uv[v] = r;
  }
}

// Vertices per UV thread: 4 for one frame; 8 in batched launches, whose
// grids hold every view's UV workgroups (fewer, longer waves launch faster
// there, and cost one frame about 0.2 us).
constexpr int kUvPerFrame = 4, kUvPerBatch = 8;

__global__ void k_uv(int64_t V, FrameParams p, const float* __restrict__ pos,
                     const int32_t* __restrict__ cov, const fa_chart* __restrict__ charts,
                     float2* __restrict__ uv, const FrameState* __restrict__ stp) {
  uv_block<kUvPerFrame>(blockIdx.x, p, pos, cov, charts, uv, V, stp);
}

// Per-corner UVs of edge-connected charts: corner k of triangle t is its
// vertex mapped through the chart of t (a vertex on a seam between charts
// gets one UV per chart). One thread per triangle writes its 24 bytes.
__global__ void k_uv_corners(int64_t T, FrameParams p, const int32_t* __restrict__ idx,
                             const float* __restrict__ pos, const int32_t* __restrict__ cot,
                             const fa_chart* __restrict__ charts, float2* __restrict__ uv,
                             const FrameState* __restrict__ stp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const FrameState st = *stp;
  const int c = st.status == FA_OK ? cot[t] : -1;
  const float nan = __builtin_nanf("");
  if (c < 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) uv[3 * t + k] = make_float2(nan, nan);
    return;
  }
  const ChartXform m = chart_xform(charts[c], p, st);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float4 q = clip_of(pos, idx[3 * t + k], p);
    uv[3 * t + k] = q.w > 0.0f ? to_atlas(m, q.x, q.y, q.w) : make_float2(nan, nan);
  }
}

// ---------------------------------------------------------------------------
// occupancy
// ---------------------------------------------------------------------------
struct Footprint {
  int32_t ax, ay;          // vertex a (1/256 texel)
  int32_t bx, by, cx, cy;  // vertices b and c relative to a
  int tx0, tx1, ty0, ty1;  // inclusive texel range to test (non-empty)
  int chart;
  int neg;                 // signed area < 0
};

template <int P>
__device__ __forceinline__ float pd(const float4& q) {
  if (P == 0) return q.w + q.x;
  if (P == 1) return q.w - q.x;
  if (P == 2) return q.w + q.y;
  if (P == 3) return q.w - q.y;
  if (P == 4) return q.w + q.z;
  return q.w - q.z;
}
template <int P>
__device__ __forceinline__ bool outside(const float4& a, const float4& b, const float4& c) {
  return pd<P>(a) < 0.0f && pd<P>(b) < 0.0f && pd<P>(c) < 0.0f;
}

__device__ __forceinline__ float4 pick4(bool c, const float4& a, const float4& b) {
  return make_float4(c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z, c ? a.w : b.w);
}

// near-plane Sutherland-Hodgman of one triangle into up to 4 vertices; each
// output slot is written with value selects (a runtime index into `o` would
// move the polygon to scratch memory)
__device__ __forceinline__ int near_clip(const float4& a, const float4& b, const float4& c,
                                         float4* o) {
  int n = 0;
  float4 o0 = a, o1 = a, o2 = a, o3 = a;
  auto put = [&](const float4& v) {
    o0 = pick4(n == 0, v, o0);
    o1 = pick4(n == 1, v, o1);
    o2 = pick4(n == 2, v, o2);
    o3 = pick4(n >= 3, v, o3);
    ++n;
  };
  const float4 in[3] = {a, b, c};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float4 S = in[i], E = in[i == 2 ? 0 : i + 1];
    const float dS = pd<4>(S), dE = pd<4>(E);
    const bool iS = dS >= 0.0f, iE = dE >= 0.0f;
    if (iS != iE) {
      const float4 A = iS ? S : E, B = iS ? E : S;
      const float dA = iS ? dS : dE, dB = iS ? dE : dS;
      const float t = dA / (dA - dB);
      float4 I;
      I.x = A.x + t * (B.x - A.x);
      I.y = A.y + t * (B.y - A.y);
      I.z = A.z + t * (B.z - A.z);
      I.w = A.w + t * (B.w - A.w);
      put(I);
    }
    if (iE) put(E);
  }
  o[0] = o0;
  o[1] = o1;
  o[2] = o2;
  o[3] = o3;
  return n;
}

__device__ __forceinline__ int32_t snap(float u) {
  const float lim = 268435456.0f;  // 2^28 (1/256-texel units)
  return (int32_t)__builtin_rintf(fminf(fmaxf(u * 256.0f, -lim), lim));
}

// The near-clipped polygon of visible triangle t mapped to snapped atlas
// coordinates (1/256 texel, |value| <= 2^28); n = 0 when it claims nothing.
struct SnapPoly {
  int32_t u[4], v[4];
  int n;
  int chart;
};

__device__ __forceinline__ void snap_polygon(int64_t t, const int32_t* __restrict__ idx,
                                             const float* __restrict__ pos,
                                             const int32_t* __restrict__ cot,
                                             const fa_chart* __restrict__ charts,
                                             const FrameParams& p, const FrameState& st,
                                             SnapPoly& sp) {
  sp.n = 0;
  const int c = cot[t];
  sp.chart = c;
  if (c < 0) return;
  const float4 a = clip_of(pos, idx[3 * t], p), b = clip_of(pos, idx[3 * t + 1], p),
               cc = clip_of(pos, idx[3 * t + 2], p);
  if (outside<0>(a, b, cc) || outside<1>(a, b, cc) || outside<2>(a, b, cc) ||
      outside<3>(a, b, cc) || outside<4>(a, b, cc) || outside<5>(a, b, cc))
    return;
  float4 poly[4];
  int n;
  if (pd<4>(a) < 0.0f || pd<4>(b) < 0.0f || pd<4>(cc) < 0.0f) {
    n = near_clip(a, b, cc, poly);
  } else {
    poly[0] = a; poly[1] = b; poly[2] = cc; poly[3] = cc; n = 3;
  }
  // constant indices only (a runtime index would place the polygon in memory)
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k < n && !(poly[k].w > 0.0f)) return;
  const ChartXform m = chart_xform(charts[c], p, st);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k < n) {
      const float2 q = to_atlas(m, poly[k].x, poly[k].y, poly[k].w);
      sp.u[k] = snap(q.x);
      sp.v[k] = snap(q.y);
    }
  }
  sp.n = n;
}

// Fan triangle f (0 or 1) of a snapped polygon: vertices 0, f+1, f+2, with
// its texel range: texel centres (256 t + 128) inside the bounding box of the
// snapped triangle and inside the chart's placed box (`box` = lo_x, hi_x,
// lo_y, hi_y, the exact integer membership range of the box).
__device__ __forceinline__ bool fan_footprint(const SnapPoly& sp, int f, const int4 box, int omega,
                                              Footprint& fp) {
  if (f + 2 >= sp.n) return false;
  const int32_t ax = sp.u[0], ay = sp.v[0];
  // constant indices only (a runtime index would put the polygon in scratch)
  const bool f1 = f != 0;
  const int32_t ub = f1 ? sp.u[2] : sp.u[1], vb = f1 ? sp.v[2] : sp.v[1];
  const int32_t uc = f1 ? sp.u[3] : sp.u[2], vc = f1 ? sp.v[3] : sp.v[2];
  fp.ax = ax; fp.ay = ay;
  fp.bx = ub - ax; fp.by = vb - ay;
  fp.cx = uc - ax; fp.cy = vc - ay;
  const int64_t area = (int64_t)fp.bx * fp.cy - (int64_t)fp.by * fp.cx;
  if (area == 0) return false;
  fp.neg = area < 0;
  const int32_t umin = min(ax, min(ub, uc)), umax = max(ax, max(ub, uc));
  const int32_t vmin = min(ay, min(vb, vc)), vmax = max(ay, max(vb, vc));
  // ceil((x - 128) / 256) and floor((x - 128) / 256) as arithmetic shifts
  const int lo_x = max(box.x, max(0, (umin + 127) >> 8));
  const int hi_x = min(box.y, min(omega - 1, (umax - 128) >> 8));
  const int lo_y = max(box.z, max(0, (vmin + 127) >> 8));
  const int hi_y = min(box.w, min(omega - 1, (vmax - 128) >> 8));
  if (lo_x > hi_x || lo_y > hi_y) return false;
  fp.tx0 = lo_x; fp.tx1 = hi_x; fp.ty0 = lo_y; fp.ty1 = hi_y;
  fp.chart = sp.chart;
  return true;
}

// A queued footprint travels whole (three 16-byte words), so the tile kernel
// needs no dependent loads to rebuild it.
__device__ __forceinline__ void put_footprint(int4* d, const Footprint& f) {
  d[0] = make_int4(f.ax, f.ay, f.bx, f.by);
  d[1] = make_int4(f.cx, f.cy, f.tx0, f.tx1);
  d[2] = make_int4(f.ty0, f.ty1, f.chart, f.neg);
}
__device__ __forceinline__ Footprint get_footprint(const int4* d) {
  const int4 a = d[0], b = d[1], c = d[2];
  Footprint f;
  f.ax = a.x; f.ay = a.y; f.bx = a.z; f.by = a.w;
  f.cx = b.x; f.cy = b.y; f.tx0 = b.z; f.tx1 = b.w;
  f.ty0 = c.x; f.ty1 = c.y; f.chart = c.z; f.neg = c.w;
  return f;
}

// The three edge functions at the centre of texel (tx, ty), exact in 64-bit
// integers (inputs within 2^31, products within 2^61), negated when the
// triangle is clockwise so that "covered" is always "all three >= 0":
//   e0 = (b-a) x (p-a), e1 = (c-b) x (p-b), e2 = (a-c) x (p-c).
struct Edges {
  int64_t e0, e1, e2;
};
__device__ __forceinline__ Edges edges_at(const Footprint& fp, int tx, int ty) {
  const int32_t px = 256 * tx + 128 - fp.ax, py = 256 * ty + 128 - fp.ay;
  Edges e;
  e.e0 = (int64_t)fp.bx * py - (int64_t)fp.by * px;
  e.e1 = (int64_t)(fp.cx - fp.bx) * (py - fp.by) - (int64_t)(fp.cy - fp.by) * (px - fp.bx);
  e.e2 = (int64_t)fp.cy * px - (int64_t)fp.cx * py;
  if (fp.neg) { e.e0 = -e.e0; e.e1 = -e.e1; e.e2 = -e.e2; }
  return e;
}
// change of the edge functions per texel step in x and in y
__device__ __forceinline__ Edges step_x(const Footprint& fp) {
  const int64_t s = fp.neg ? -256 : 256;
  return Edges{-s * fp.by, -s * (fp.cy - fp.by), s * fp.cy};
}
__device__ __forceinline__ Edges step_y(const Footprint& fp) {
  const int64_t s = fp.neg ? -256 : 256;
  return Edges{s * fp.bx, s * (fp.cx - fp.bx), -s * fp.cx};
}
__device__ __forceinline__ bool inside(const Edges& e) { return (e.e0 | e.e1 | e.e2) >= 0; }
__device__ __forceinline__ void add(Edges& e, const Edges& d) {
  e.e0 += d.e0; e.e1 += d.e1; e.e2 += d.e2;
}
__device__ __forceinline__ Edges madd(const Edges& a, int64_t k, const Edges& b) {
  return Edges{a.e0 + k * b.e0, a.e1 + k * b.e1, a.e2 + k * b.e2};
}

__global__ void k_occ_fill(int4* __restrict__ occ, int64_t n4, const FrameState* __restrict__ st) {
  const int4 neg = make_int4(-1, -1, -1, -1);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x)
    occ[i] = neg;
}

// All texels of a footprint by one lane, row by row, edge functions stepped.
__device__ __forceinline__ void raster_lane(const Footprint& fp, int32_t* __restrict__ occ,
                                            int omega) {
  Edges r = edges_at(fp, fp.tx0, fp.ty0);
  const Edges dx = step_x(fp), dy = step_y(fp);
  for (int ty = fp.ty0; ty <= fp.ty1; ++ty) {
    int32_t* row = occ + (int64_t)ty * omega;
    Edges e = r;
    for (int tx = fp.tx0; tx <= fp.tx1; ++tx) {
      if (inside(e)) row[tx] = fp.chart;
      add(e, dx);
    }
    add(r, dy);
  }
}

__device__ __forceinline__ int rl(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// The texels of every lane's footprint (n texels; 0 for none), concatenated in
// lane order and row-major inside a footprint, by the whole wave 64 at a time:
// the lane taking texel g finds the footprint holding it by a binary search
// over the wave's inclusive prefix of n and fetches that footprint from its
// lane. Neighbouring lanes then write neighbouring texels of one row, so the
// stores coalesce (one lane per footprint scatters 4-byte stores over the
// map, several times slower).
__device__ __forceinline__ void raster_expand(const Footprint& f, int n, int32_t* __restrict__ occ,
                                              int omega) {
  const int lane = lane_id();
  const int incl = wave_incl_scan<int>(n);
  const int total = __shfl(incl, kWave - 1, kWave);
  const int start = incl - n;
  for (int c = 0; c < total; c += kWave) {
    const int g = c + lane;
    int pos = 0;  // first lane whose inclusive prefix exceeds g
#pragma unroll
    for (int s = kWave / 2; s > 0; s >>= 1) {
      const int v = __shfl(incl, pos + s - 1, kWave);
      if (v <= g) pos += s;
    }
    Footprint o;
    o.ax = __shfl(f.ax, pos, kWave);
    o.ay = __shfl(f.ay, pos, kWave);
    o.bx = __shfl(f.bx, pos, kWave);
    o.by = __shfl(f.by, pos, kWave);
    o.cx = __shfl(f.cx, pos, kWave);
    o.cy = __shfl(f.cy, pos, kWave);
    o.tx0 = __shfl(f.tx0, pos, kWave);
    o.tx1 = __shfl(f.tx1, pos, kWave);
    o.ty0 = __shfl(f.ty0, pos, kWave);
    o.chart = __shfl(f.chart, pos, kWave);
    o.neg = __shfl(f.neg, pos, kWave);
    const int li = g - __shfl(start, pos, kWave);
    const int nx = max(o.tx1 - o.tx0 + 1, 1);  // lanes past the total read an unused lane
    int row = (int)((float)li / (float)nx);
    if (row * nx > li) --row;
    else if ((row + 1) * nx <= li) ++row;
    const int tx = o.tx0 + (li - row * nx), ty = o.ty0 + row;
    if (g < total && inside(edges_at(o, tx, ty))) occ[(int64_t)ty * omega + tx] = o.chart;
  }
}

constexpr int kOccTile = 16;                   // queued footprints are cut into 16x16 tiles
constexpr unsigned long long kSlotShift = 40;  // queue counter: footprints << 40 | tiles

// Occupancy of the visible triangles. Per fan footprint (texel range of n
// texels): n <= lane_texels by its own lane; lane_texels < n <= small_texels
// by the wave's coalesced expansion; larger ones are queued for k_occ_big. Both fans of every
// triangle are set up first and the queue is reserved with one atomic per
// workgroup and step (a single counter serializes at about 12 ns per atomic);
// the rasterization after it runs without barriers.
constexpr int kOccSmallBlock = 256;

__device__ __forceinline__ uint32_t tiles_of(const Footprint& fp, uint32_t* tiles_x) {
  *tiles_x = (uint32_t)((fp.tx1 - fp.tx0 + kOccTile) / kOccTile);
  return *tiles_x * (uint32_t)((fp.ty1 - fp.ty0 + kOccTile) / kOccTile);
}

template <int UV_PER>
__device__ __forceinline__ void k_occ_small_body(
    const int32_t* __restrict__ idx, const int32_t* __restrict__ vlist, FrameParams p,
    const float* __restrict__ pos, const int32_t* __restrict__ cot,
    const fa_chart* __restrict__ charts, const int4* __restrict__ chart_tex,
    int32_t* __restrict__ occ, ulonglong2* __restrict__ big, int4* __restrict__ big_fp,
    uint32_t big_cap, int small_texels,
    int lane_texels, unsigned long long* __restrict__ big_counter,
    const FrameState* __restrict__ stp, unsigned occ_blocks, int64_t V,
    const int32_t* __restrict__ cov, float2* __restrict__ uv) {
  __shared__ uint32_t wcnt[kOccSmallBlock / kWave], wtil[kOccSmallBlock / kWave];
  __shared__ unsigned long long bbase;
  if (blockIdx.x >= occ_blocks) {
    uv_block<UV_PER>(blockIdx.x - occ_blocks, p, pos, cov, charts, uv, V, stp);
    return;
  }
  const FrameState st = *stp;
  if (st.status != FA_OK) return;
  const int nv = st.visible;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  // the launch's block size, as a constant: a loop over a runtime wave count
  // is unrolled eight times with live temporaries (100 instead of 89 VGPRs:
  // four instead of five resident waves per SIMD)
  constexpr int nw = kOccSmallBlock / kWave;
  constexpr unsigned long long kLow = (1ull << kSlotShift) - 1;
  for (int i0 = blockIdx.x * blockDim.x; i0 < nv; i0 += occ_blocks * blockDim.x) {
    const int i = i0 + threadIdx.x;
    const bool valid = i < nv;
    SnapPoly sp;
    sp.n = 0;
    sp.chart = -1;
    const int t = valid ? vlist[i] : 0;
    if (valid) snap_polygon(t, idx, pos, cot, charts, p, st, sp);
    Footprint fa, fb;
    const int4 box = sp.n > 0 ? chart_tex[sp.chart] : make_int4(0, -1, 0, -1);
    const bool oka = sp.n > 0 && fan_footprint(sp, 0, box, p.omega, fa);
    const bool okb = sp.n > 3 && fan_footprint(sp, 1, box, p.omega, fb);
    const int na = oka ? (fa.tx1 - fa.tx0 + 1) * (fa.ty1 - fa.ty0 + 1) : 0;
    const int nb = okb ? (fb.tx1 - fb.tx0 + 1) * (fb.ty1 - fb.ty0 + 1) : 0;
    const bool wa = oka && na > small_texels, wb = okb && nb > small_texels;
    uint32_t txa = 0, txb = 0;
    const uint32_t nta = wa ? tiles_of(fa, &txa) : 0u, ntb = wb ? tiles_of(fb, &txb) : 0u;
    // queue order: wave-major, then lane, fan a before fan b
    const uint32_t mine = (uint32_t)wa + (uint32_t)wb, mine_t = nta + ntb;
    const uint32_t c_in = wave_incl_scan<uint32_t>(mine) - mine;
    const uint32_t t_in = wave_incl_scan<uint32_t>(mine_t) - mine_t;
    if (lane == kWave - 1) {
      wcnt[w] = c_in + mine;
      wtil[w] = t_in + mine_t;
    }
    __syncthreads();
    uint32_t c_before = 0, t_before = 0, c_all = 0, t_all = 0;
    for (int k = 0; k < nw; ++k) {
      const uint32_t c = wcnt[k], tl = wtil[k];
      if (k < w) {
        c_before += c;
        t_before += tl;
      }
      c_all += c;
      t_all += tl;
    }
    if (threadIdx.x == 0 && c_all)
      bbase = atomicAdd(big_counter, ((unsigned long long)c_all << kSlotShift) | t_all);
    __syncthreads();
    bool qa = false, qb = false;
    if (c_all) {
      const unsigned long long old = bbase;
      unsigned long long slot = (old >> kSlotShift) + c_before + c_in;
      unsigned long long tile = (old & kLow) + t_before + t_in;
      // x: footprint code | tiles across << 32; y: first tile | tiles << 40
      if (wa && slot < big_cap) {
        big[slot] = make_ulonglong2((unsigned long long)(2 * (int64_t)t) |
                                        ((unsigned long long)txa << 32),
                                    tile | ((unsigned long long)nta << kSlotShift));
        put_footprint(big_fp + 3 * slot, fa);
        qa = true;
      }
      slot += wa;
      tile += nta;
      if (wb && slot < big_cap) {
        big[slot] = make_ulonglong2((unsigned long long)(2 * (int64_t)t + 1) |
                                        ((unsigned long long)txb << 32),
                                    tile | ((unsigned long long)ntb << kSlotShift));
        put_footprint(big_fp + 3 * slot, fb);
        qb = true;
      }
    }
    const bool ca = oka && !qa && na > lane_texels, cb = okb && !qb && nb > lane_texels;
    if (oka && !qa && !ca) raster_lane(fa, occ, p.omega);
    if (okb && !qb && !cb) raster_lane(fb, occ, p.omega);
    raster_expand(fa, ca ? na : 0, occ, p.omega);
    if (__ballot(cb)) raster_expand(fb, cb ? nb : 0, occ, p.omega);
  }
}
__global__ __launch_bounds__(kOccSmallBlock) void k_occ_small(
    const int32_t* __restrict__ idx, const int32_t* __restrict__ vlist, FrameParams p,
    const float* __restrict__ pos, const int32_t* __restrict__ cot,
    const fa_chart* __restrict__ charts, const int4* __restrict__ chart_tex,
    int32_t* __restrict__ occ, ulonglong2* __restrict__ big, int4* __restrict__ big_fp,
    uint32_t big_cap, int small_texels,
    int lane_texels, unsigned long long* __restrict__ big_counter,
    const FrameState* __restrict__ stp, unsigned occ_blocks, int64_t V,
    const int32_t* __restrict__ cov, float2* __restrict__ uv) {
  k_occ_small_body<kUvPerFrame>(idx, vlist, p, pos, cot, charts, chart_tex, occ, big, big_fp,
                                big_cap, small_texels, lane_texels, big_counter, stp, occ_blocks,
                                V, cov, uv);
}

// Queued footprints: their texel ranges cut into 16x16 tiles, concatenated,
// are split evenly over all waves of the grid; a wave finds its first
// footprint by a 64-way search over the (increasing) first-tile indices and
// walks forward, 4 texels per lane.
__device__ __forceinline__ void k_occ_big_body(
    const int32_t* __restrict__ idx, FrameParams p, const float* __restrict__ pos,
    const int32_t* __restrict__ cot, const fa_chart* __restrict__ charts,
    const int4* __restrict__ chart_tex, int32_t* __restrict__ occ,
    const ulonglong2* __restrict__ big, const int4* __restrict__ big_fp, uint32_t big_cap,
    const unsigned long long* __restrict__ big_counter, const FrameState* __restrict__ stp) {
  const FrameState st = *stp;
  if (st.status != FA_OK) return;
  const unsigned long long ctr =
      __hip_atomic_load(big_counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t nent = (uint32_t)min<unsigned long long>(ctr >> kSlotShift, big_cap);
  if (nent == 0) return;
  constexpr unsigned long long kLow = (1ull << kSlotShift) - 1;
  const ulonglong2 lastv = big[nent - 1];
  const uint64_t total = (lastv.y & kLow) + (lastv.y >> kSlotShift);
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  // the wave index through readfirstlane: the compiler then knows it (and all
  // loop bounds below) to be uniform and keeps the tile loop's control scalar
  const uint64_t wid = (uint64_t)blockIdx.x * (kBlock / kWave) +
                       (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const uint64_t per = (total + nwaves - 1) / nwaves;
  const uint64_t k0 = wid * per, k1 = min<uint64_t>(total, k0 + per);
  if (k0 >= k1) return;
  const int lane = lane_id();
  // last entry whose first tile <= k0; entry 0 starts at tile 0
  uint32_t lo = 0, hi = nent;
  while (hi - lo > 1) {
    const uint32_t step = (hi - lo + kWave - 1) / kWave;
    const uint32_t probe = lo + (uint32_t)lane * step;
    const bool le = probe < hi && (big[probe].y & kLow) <= k0;
    const int cnt = __popcll(__ballot(le));
    lo += (uint32_t)(cnt - 1) * step;
    hi = min(hi, lo + step);
  }
  // The wave's footprints are set up 64 at a time, one per lane (their
  // dependent loads overlap), then rasterized one after another with the
  // footprint broadcast from its lane.
  const int lx = lane % kOccTile, ly = lane / kOccTile;
  constexpr int kRows = kWave / kOccTile;
  for (uint32_t e0 = lo; e0 < nent;) {
    const uint32_t my = e0 + (uint32_t)lane;
    uint64_t base = 0, nt = 0;
    uint32_t tiles_x = 1;
    bool mine = false, ok = false;
    Footprint f;
    f.ax = f.ay = f.bx = f.by = f.cx = f.cy = 0;
    f.tx0 = f.tx1 = f.ty0 = f.ty1 = f.chart = f.neg = 0;
    if (my < nent) {
      const ulonglong2 ent = big[my];
      base = ent.y & kLow;
      nt = ent.y >> kSlotShift;
      tiles_x = (uint32_t)(ent.x >> 32);
      mine = base < k1;
      if (mine) {
        f = get_footprint(big_fp + 3 * (int64_t)my);
        ok = true;
      }
    }
    const int cnt = __popcll(__ballot(mine));  // entries start in order: a prefix of lanes
    for (int j = 0; j < cnt; ++j) {
      if (!rl((int)ok, j)) continue;
      Footprint fp;
      fp.ax = rl(f.ax, j); fp.ay = rl(f.ay, j);
      fp.bx = rl(f.bx, j); fp.by = rl(f.by, j);
      fp.cx = rl(f.cx, j); fp.cy = rl(f.cy, j);
      fp.tx0 = rl(f.tx0, j); fp.tx1 = rl(f.tx1, j);
      fp.ty0 = rl(f.ty0, j); fp.ty1 = rl(f.ty1, j);
      fp.chart = rl(f.chart, j); fp.neg = rl(f.neg, j);
      const uint64_t bj = ((uint64_t)(uint32_t)rl((int)(uint32_t)(base >> 32), j) << 32) |
                          (uint32_t)rl((int)(uint32_t)base, j);
      const uint64_t nj = (uint64_t)(uint32_t)rl((int)(uint32_t)nt, j);
      const uint32_t txj = (uint32_t)rl((int)tiles_x, j);
      // a footprint has fewer than 2^32 tiles (at most (omega / 16)^2)
      const uint32_t t0 = (uint32_t)((k0 > bj ? k0 : bj) - bj);
      const uint32_t t1 = (uint32_t)((k1 < bj + nj ? k1 : bj + nj) - bj);
      // The edge functions are linear in the texel: at the lane's texel they
      // are their value at the tile's first texel (uniform, scalar unit) plus
      // the lane's offset, fixed per footprint.
      const Edges dx = step_x(fp), dy = step_y(fp);
      const Edges off = madd(madd(Edges{0, 0, 0}, lx, dx), ly, dy);
      const Edges dq = madd(Edges{0, 0, 0}, kRows, dy);
      const int64_t row_step = (int64_t)kRows * p.omega;
      uint32_t ti = t0 % txj, tj = t0 / txj;  // tile column and row, stepped below
      for (uint32_t tt = t0; tt < t1; ++tt) {
        const int ox = fp.tx0 + kOccTile * (int)ti, oy = fp.ty0 + kOccTile * (int)tj;
        const Edges eo = edges_at(fp, ox, oy);
        Edges ev{eo.e0 + off.e0, eo.e1 + off.e1, eo.e2 + off.e2};
        const int tx = ox + lx, ty0 = oy + ly;
        const bool col = tx <= fp.tx1;
        int32_t* dst = occ + (int64_t)ty0 * p.omega + tx;
#pragma unroll
        for (int q = 0; q < kOccTile / kRows; ++q) {
          if (col && ty0 + q * kRows <= fp.ty1 && inside(ev)) *dst = fp.chart;
          add(ev, dq);
          dst += row_step;
        }
        if (++ti == txj) {
          ti = 0;
          ++tj;
        }
      }
    }
    if (cnt < kWave) break;
    e0 += kWave;
  }
}
__global__ __launch_bounds__(kBlock) void k_occ_big(
    const int32_t* __restrict__ idx, FrameParams p, const float* __restrict__ pos,
    const int32_t* __restrict__ cot, const fa_chart* __restrict__ charts,
    const int4* __restrict__ chart_tex, int32_t* __restrict__ occ,
    const ulonglong2* __restrict__ big, const int4* __restrict__ big_fp, uint32_t big_cap,
    const unsigned long long* __restrict__ big_counter, const FrameState* __restrict__ stp) {
  k_occ_big_body(idx, p, pos, cot, charts, chart_tex, occ, big, big_fp, big_cap, big_counter, stp);
}

// Frame record for the caller (one thread); `occ` is the occupied texel count
// when the occupancy map was built.
__device__ __forceinline__ void write_meta(const FrameParams& p, FrameState* stp,
                                           const unsigned long long* __restrict__ big_counter,
                                           bool with_occ, unsigned long long occ,
                                           fa_atlas_meta* __restrict__ meta) {
  if (with_occ && stp->status == FA_OK) stp->occupied = occ;
  const FrameState st = *stp;
  fa_atlas_meta m;
  m.status = st.status;
  m.num_charts = st.num_charts;
  m.chosen_j = st.jstar;
  m.num_scales = p.J;
  m.atlas_size = p.omega;
  m.layout_width = st.layout_w;
  m.layout_height = st.layout_h;
  m.rows = st.rows;
  m.s_eff = st.status == FA_OK ? st.s_star * st.q_star : 0.0f;
  m.rate = p.rate;
  m.occupied_texels = (int64_t)st.occupied;
  m.visible_triangles = (int64_t)st.visible;
  m.large_tiles = (int64_t)(__hip_atomic_load(big_counter, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT) &
                            ((1ull << 40) - 1));
  *meta = m;
}

__global__ void k_meta(FrameParams p, FrameState* stp,
                       const unsigned long long* __restrict__ big_counter,
                       fa_atlas_meta* __restrict__ meta) {
  if (threadIdx.x == 0) write_meta(p, stp, big_counter, false, 0ull, meta);
}

// Occupied texels and the frame record in one launch: every workgroup counts
// its share of the map and publishes the sum; the last one to finish (the
// one that draws the last ticket) adds them up and writes the record.
constexpr int kCountBlock = 1024;
__device__ __forceinline__ void k_occ_count_meta_body(
    FrameParams p, const int4* __restrict__ occ, int64_t n4,
    unsigned long long* __restrict__ partial, FrameState* stp,
    const unsigned long long* __restrict__ big_counter, fa_atlas_meta* __restrict__ meta) {
  __shared__ unsigned long long sh[kCountBlock / kWave];
  __shared__ uint32_t last;
  // eight 16-byte loads in flight per thread
  constexpr int U = 8;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t c32 = 0;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n4; i0 += U * stride) {
    int4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = i0 + u * stride < n4 ? occ[i0 + u * stride] : make_int4(-1, -1, -1, -1);
#pragma unroll
    for (int u = 0; u < U; ++u)
      c32 += (v[u].x >= 0) + (v[u].y >= 0) + (v[u].z >= 0) + (v[u].w >= 0);
  }
  // one thread counts at most 4 texels per 16-byte word it reads: far below 2^32
  const unsigned long long cnt = block_sum<unsigned long long>((unsigned long long)c32, sh);
  if (threadIdx.x == 0) {
    // the sum is stored at device scope and has completed (s_waitcnt on every
    // counter) before the ticket is taken, so whoever draws the last ticket
    // reads it with its device-scope load; no cache-wide release is needed
    __hip_atomic_store(&partial[blockIdx.x], cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);
    const uint32_t before = __hip_atomic_fetch_add(&stp->ticket, 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
    last = before == gridDim.x - 1 ? 1u : 0u;
  }
  __syncthreads();
  if (!last) return;
  unsigned long long all = 0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x)
    all += __hip_atomic_load(&partial[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  all = block_sum<unsigned long long>(all, sh);
  if (threadIdx.x == 0) write_meta(p, stp, big_counter, true, all, meta);
}
__global__ __launch_bounds__(kCountBlock) void k_occ_count_meta(
    FrameParams p, const int4* __restrict__ occ, int64_t n4,
    unsigned long long* __restrict__ partial, FrameState* stp,
    const unsigned long long* __restrict__ big_counter, fa_atlas_meta* __restrict__ meta) {
  k_occ_count_meta_body(p, occ, n4, partial, stp, big_counter, meta);
}

// ---- batched wrappers (view = blockIdx.y) --------------------------------
__global__ __launch_bounds__(kOccSmallBlock) void k_occ_small_b(
    const BatchView* __restrict__ bv, const int32_t* __restrict__ idx, uint32_t big_cap,
    int small_texels, int lane_texels, unsigned occ_blocks, int64_t V) {
  const BatchView& v = bv[blockIdx.y];
  k_occ_small_body<kUvPerBatch>(idx, v.w.vlist, v.p, v.w.pos, v.cot, v.charts, v.w.chart_tex, v.occ, v.w.big,
                   v.w.big_fp, big_cap, small_texels, lane_texels, v.w.big_counter, v.w.state,
                   occ_blocks, V, v.cov, reinterpret_cast<float2*>(v.uv));
}
__global__ __launch_bounds__(kBlock) void k_occ_big_b(const BatchView* __restrict__ bv,
                                                      const int32_t* __restrict__ idx,
                                                      uint32_t big_cap) {
  const BatchView& v = bv[blockIdx.y];
  k_occ_big_body(idx, v.p, v.w.pos, v.cot, v.charts, v.w.chart_tex, v.occ, v.w.big, v.w.big_fp,
                 big_cap, v.w.big_counter, v.w.state);
}
__global__ __launch_bounds__(kCountBlock) void k_occ_count_meta_b(
    const BatchView* __restrict__ bv) {
  const BatchView& v = bv[blockIdx.y];
  k_occ_count_meta_body(v.p, reinterpret_cast<const int4*>(v.occ),
                        (int64_t)v.p.omega * v.p.omega / 4, v.w.partial, v.w.state,
                        v.w.big_counter, v.meta);
}

}  // namespace

hipError_t launch_uv(const int64_t V, const FrameParams& p, const Work& w, const int32_t* cov,
                     const fa_chart* charts, float* uv, hipStream_t st) {
  if (V > 0)
    k_uv<<<(unsigned)((V + kBlock * kUvPerFrame - 1) / (kBlock * kUvPerFrame)), kBlock, 0, st>>>(
        V, p, w.pos, cov, charts, reinterpret_cast<float2*>(uv), w.state);
  return hipGetLastError();
}

hipError_t launch_uv_corners(const int32_t* idx, int64_t T, const FrameParams& p, const Work& w,
                             const int32_t* cot, const fa_chart* charts, float* uv,
                             hipStream_t st) {
  if (T > 0)
    k_uv_corners<<<(unsigned)((T + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        T, p, idx, w.pos, cot, charts, reinterpret_cast<float2*>(uv), w.state);
  return hipGetLastError();
}

hipError_t launch_occupancy(const int32_t* idx, int64_t T, const FrameParams& p, const Work& w,
                            const int32_t* cot, const fa_chart* charts, int32_t* occ,
                            int small_texels, int lane_texels, const OccExtras& x, Marker& mk,
                            hipStream_t st) {
  const int64_t n4 = (int64_t)p.omega * p.omega / 4;
  if (x.fill) {
    const unsigned fill_grid = (unsigned)std::min<int64_t>((n4 + kBlock - 1) / kBlock, 4096);
    k_occ_fill<<<fill_grid, kBlock, 0, st>>>(reinterpret_cast<int4*>(occ), n4, w.state);
  }
  mk(st);
  const uint32_t cap = (uint32_t)std::min<int64_t>(2 * std::max<int64_t>(T, 1), kBigCap);
  const int64_t V = x.uv ? x.V : 0;
  const unsigned occ_blocks = T > 0 ? visible_grid(T) : 0;
  const unsigned uv_blocks = (unsigned)((V + kOccSmallBlock * kUvPerFrame - 1) /
                                         (kOccSmallBlock * kUvPerFrame));
  if (occ_blocks + uv_blocks > 0)
    k_occ_small<<<occ_blocks + uv_blocks, kOccSmallBlock, 0, st>>>(
        idx, w.vlist, p, w.pos, cot, charts, w.chart_tex, occ, w.big, w.big_fp, cap, small_texels,
        lane_texels, w.big_counter, w.state, occ_blocks, V, x.cov,
        reinterpret_cast<float2*>(x.uv));
  mk(st);
  if (T > 0)
    k_occ_big<<<kOccBigGrid, kBlock, 0, st>>>(idx, p, w.pos, cot, charts, w.chart_tex, occ,
                                              w.big, w.big_fp, cap, w.big_counter, w.state);
  mk(st);
  if (x.meta)  // a scaled copy (no frame record) needs no count
    k_occ_count_meta<<<kCountGrid, kCountBlock, 0, st>>>(p, reinterpret_cast<const int4*>(occ), n4,
                                                         w.partial, w.state, w.big_counter, x.meta);
  mk(st);
  return hipGetLastError();
}

namespace {
// Texel range of every placed box for an atlas of side p.omega (the same exact
// integer membership test as at placement), and an empty large-footprint
// queue: the start of an occupancy pass at another atlas side.
__global__ void k_chart_tex(FrameParams p, const fa_chart* __restrict__ charts,
                            int4* __restrict__ chart_tex, unsigned long long* __restrict__ big_counter,
                            const FrameState* __restrict__ stp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) *big_counter = 0ull;
  const FrameState st = *stp;
  if (st.status != FA_OK || c >= st.num_charts) return;
  const fa_chart& ch = charts[c];
  const int64_t om = p.omega, L = st.layout_w, L2 = 2 * L;
  chart_tex[c] = make_int4((int)ceil_div64(2 * (int64_t)ch.x * om - L, L2),
                           (int)ceil_div64(2 * ((int64_t)ch.x + ch.w) * om - L, L2) - 1,
                           (int)ceil_div64(2 * (int64_t)ch.y * om - L, L2),
                           (int)ceil_div64(2 * ((int64_t)ch.y + ch.h) * om - L, L2) - 1);
}
}  // namespace

hipError_t launch_occupancy_scaled(const int32_t* idx, int64_t T, const FrameParams& p,
                                   const Work& w, const int32_t* cot, const fa_chart* charts,
                                   int32_t* occ, int small_texels, int lane_texels,
                                   hipStream_t st) {
  k_chart_tex<<<(unsigned)((p.max_charts + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      p, charts, w.chart_tex, w.big_counter, w.state);
  Marker none;
  OccExtras x;
  return launch_occupancy(idx, T, p, w, cot, charts, occ, small_texels, lane_texels, x, none, st);
}

namespace {
// ---------------------------------------------------------------------------
// footprint push: full-scale profile of every chart
// ---------------------------------------------------------------------------
// Column u of chart c (prof[fp_off[c] + u], u < floor(oriented width) + 1)
// holds the first and last row, on the unit grid of the chart-local layout
// before scale and gutter, that the chart's snapped polygons reach inside the
// closed strip [u, u + 1] (first and last strips open outwards, rows clamped
// to the chart's floor(oriented height) + 1 rows). Exact integer arithmetic
// on the 1/256 snapped vertices: a side crossing's row is the floor of an
// exact rational. Empty column: (INT_MAX, -1).

// floor((py + (x0 - px) (qy - py) / (qx - px)) / 256), px != qx. Below 2^52
// the numerator and divisor are exact doubles: the rounded quotient is within
// one of the floor, and the exact integer remainder settles it.
__device__ __forceinline__ int32_t crossing_row(int64_t px, int64_t py, int64_t qx, int64_t qy,
                                                int64_t x0) {
  int64_t num = py * (qx - px) + (x0 - px) * (qy - py);
  int64_t den = qx - px;
  if (den < 0) {
    num = -num;
    den = -den;
  }
  const int64_t d = 256 * den;
  const int64_t lim = int64_t(1) << 52;
  if (num > -lim && num < lim) {
    int64_t q = (int64_t)floor((double)num / (double)d);
    const int64_t r = num - q * d;
    if (r < 0) --q;
    else if (r >= d) ++q;
    return (int32_t)q;
  }
  return (int32_t)floor_div64(num, d);
}

// Setup of one visible-list entry for the profile raster: its near-clipped
// polygon snapped to the chart-local unit grid (1/256), the chart's column
// and row counts and first profile entry, and the columns [u0, u0 + cnt) it
// reaches (cnt = 0: nothing).
struct FpSetup {
  int32_t X[4], Y[4];
  int n, Uc, Rc, off, u0, cnt;
};
__device__ __forceinline__ void fp_setup(int i, int nv, const int32_t* __restrict__ vlist,
                                         const int32_t* __restrict__ idx,
                                         const float* __restrict__ pos,
                                         const int32_t* __restrict__ cot,
                                         const fa_chart* __restrict__ charts,
                                         const int32_t* __restrict__ fp_off, const FrameParams& p,
                                         FpSetup& s) {
#pragma unroll
  for (int k = 0; k < 4; ++k) s.X[k] = s.Y[k] = 0;
  s.n = 0; s.Uc = 1; s.Rc = 1; s.off = 0; s.u0 = 0; s.cnt = 0;
  if (i >= nv) return;
  const float halfW = 0.5f * (float)p.W, halfH = 0.5f * (float)p.H;
  const int t = vlist[i];
  const int c = cot[t];
  const float4 a = clip_of(pos, idx[3 * (int64_t)t], p),
               b = clip_of(pos, idx[3 * (int64_t)t + 1], p),
               cc = clip_of(pos, idx[3 * (int64_t)t + 2], p);
  const bool out = c < 0 || outside<0>(a, b, cc) || outside<1>(a, b, cc) ||
                   outside<2>(a, b, cc) || outside<3>(a, b, cc) || outside<4>(a, b, cc) ||
                   outside<5>(a, b, cc);
  if (out) return;
  float4 poly[4];
  int n;
  if (pd<4>(a) < 0.0f || pd<4>(b) < 0.0f || pd<4>(cc) < 0.0f) {
    n = near_clip(a, b, cc, poly);
  } else {
    poly[0] = a; poly[1] = b; poly[2] = cc; poly[3] = cc; n = 3;
  }
  bool ok = n > 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) ok = ok && (k >= n || poly[k].w > 0.0f);
  if (!ok) return;
  const fa_chart& ch = charts[c];
  const float x0 = ch.ndc_box[0], y1 = ch.ndc_box[3], tw = ch.target_w;
  const int rot = ch.rotated;
  int32_t xmin = INT_MAX, xmax = INT_MIN;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k < n) {
      const float nx = poly[k].x / poly[k].w, ny = poly[k].y / poly[k].w;
      const float px = ((nx - x0) * halfW) * p.rate;
      const float py = ((y1 - ny) * halfH) * p.rate;
      s.X[k] = snap(rot ? py : px);
      s.Y[k] = snap(rot ? (tw - px) : py);
      xmin = min(xmin, s.X[k]);
      xmax = max(xmax, s.X[k]);
    }
  }
  s.n = n;
  s.Uc = (int)floorf(ch.oriented_w) + 1;
  s.Rc = (int)floorf(ch.oriented_h) + 1;
  s.off = fp_off[c];
  s.u0 = min(s.Uc - 1, max(0, xmin >> 8));
  s.cnt = min(s.Uc - 1, max(0, xmax >> 8)) - s.u0 + 1;
}

// Count: the (triangle, column) items of every group of 64 consecutive
// visible-list entries (group g = entries 64 g .. 64 g + 63), one wave per
// group; the blocks past the groups clear the profile.
__global__ __launch_bounds__(kBlock) void k_fp_count(
    const int32_t* __restrict__ vlist, const int32_t* __restrict__ idx,
    const float* __restrict__ pos, const int32_t* __restrict__ cot,
    const fa_chart* __restrict__ charts, const int32_t* __restrict__ fp_off,
    unsigned long long* __restrict__ group_items, int2* __restrict__ prof, unsigned count_blocks,
    FrameParams p, const FrameState* __restrict__ stp) {
  if (stp->status != FA_OK) return;
  if (blockIdx.x >= count_blocks) {
    const int ncol = stp->fp_columns;
    const int64_t stride = (int64_t)(gridDim.x - count_blocks) * blockDim.x;
    for (int64_t e = (int64_t)(blockIdx.x - count_blocks) * blockDim.x + threadIdx.x; e < ncol;
         e += stride)
      prof[e] = make_int2(INT_MAX, -1);
    return;
  }
  const int nv = stp->visible;
  const int groups = (nv + kWave - 1) / kWave;
  const int nw = (int)(count_blocks * (blockDim.x / kWave));
  for (int g = (int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave); g < groups;
       g += nw) {
    FpSetup s;
    fp_setup(g * kWave + lane_id(), nv, vlist, idx, pos, cot, charts, fp_off, p, s);
    const int tot = wave_sum<int>(s.cnt);
    if (lane_id() == 0) group_items[g] = (unsigned long long)tot;
  }
}

// Scan: exclusive prefix of the groups' item counts in place, the total after
// the last group (one workgroup).
__global__ __launch_bounds__(1024) void k_fp_scan(unsigned long long* __restrict__ group_items,
                                                 const FrameState* __restrict__ stp) {
  __shared__ unsigned long long sh[1024 / kWave];
  if (stp->status != FA_OK) return;
  const int groups = (stp->visible + kWave - 1) / kWave;
  const int per = (groups + 1023) / 1024;
  const int b = min(groups, (int)threadIdx.x * per), e = min(groups, b + per);
  unsigned long long sum = 0;
  for (int g = b; g < e; ++g) sum += group_items[g];
  unsigned long long total = 0;
  unsigned long long run = block_incl_scan<unsigned long long>(sum, sh, &total) - sum;
  for (int g = b; g < e; ++g) {
    const unsigned long long v = group_items[g];
    group_items[g] = run;
    run += v;
  }
  if (threadIdx.x == 0) group_items[groups] = total;
}

// Raster: the frame's (triangle, column) items are split evenly over all
// waves (a wave's share is a contiguous range of the groups' items), so the
// columns of a few large triangles no longer load one wave. A wave finds the
// group holding its first item by a 64-way search over the group prefix and
// walks forward; for each group it touches, its lanes set up the group's 64
// entries again and the wave takes that group's items in its range 64 at a
// time (owner found by a binary search over the inclusive column counts).
// Neighbouring triangles share columns: when the columns of a wave's items
// of a group span fewer than kFpWin profile entries they are reduced in a
// per-wave LDS window and flushed with one pair of global atomics per
// touched entry.
constexpr int kFpWin = 1024;

__global__ __launch_bounds__(kBlock) void k_fp_raster(
    const int32_t* __restrict__ vlist, const int32_t* __restrict__ idx,
    const float* __restrict__ pos, const int32_t* __restrict__ cot,
    const fa_chart* __restrict__ charts, const int32_t* __restrict__ fp_off,
    const unsigned long long* __restrict__ group_first, int2* __restrict__ prof, FrameParams p,
    const FrameState* __restrict__ stp) {
  __shared__ int2 win_all[kBlock / kWave][kFpWin];
  if (stp->status != FA_OK) return;
  const int nv = stp->visible;
  const int groups = (nv + kWave - 1) / kWave;
  if (groups == 0) return;
  const unsigned long long total = group_first[groups];
  const int lane = lane_id();
  const unsigned long long nwaves = gridDim.x * (blockDim.x / kWave);
  const unsigned long long wave = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const unsigned long long per = (total + nwaves - 1) / nwaves;
  const unsigned long long k0 = min(total, wave * per), k1 = min(total, k0 + per);
  if (k0 >= k1) return;
  int2* win = win_all[threadIdx.x / kWave];
  for (int e = lane; e < kFpWin; e += kWave) win[e] = make_int2(INT_MAX, -1);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  // last group whose first item <= k0 (group 0 starts at item 0)
  int lo = 0, hi = groups;
  while (hi - lo > 1) {
    const int step = (hi - lo + kWave - 1) / kWave;
    const int probe = lo + lane * step;
    const bool le = probe < hi && group_first[probe] <= k0;
    const int c = __popcll(__ballot(le));
    lo += (c - 1) * step;
    hi = min(hi, lo + step);
  }
  for (int g = lo; g < groups; ++g) {
    const unsigned long long gfirst = group_first[g];
    if (gfirst >= k1) break;
    FpSetup s;
    fp_setup(g * kWave + lane, nv, vlist, idx, pos, cot, charts, fp_off, p, s);
    const int incl = wave_incl_scan<int>(s.cnt);
    const int gtot = __shfl(incl, kWave - 1, kWave);
    // this wave's items of the group: [ia, ib) in group-local numbering
    const int ia = (int)(k0 > gfirst ? k0 - gfirst : 0ull);
    const int ib = (int)min<unsigned long long>((unsigned long long)gtot, k1 - gfirst);
    if (ia >= ib) continue;
    // profile entries this wave's items of the group touch: [elo, ehi] (a
    // lane's items are [incl - cnt, incl), its columns from u0 on)
    const int st0 = incl - s.cnt;
    const int ja = max(st0, ia), jb = min(incl, ib) - 1;
    const bool mine = s.cnt > 0 && ja <= jb;
    const int elo = wave_min<int>(mine ? s.off + s.u0 + (ja - st0) : INT_MAX);
    const int ehi = wave_max<int>(mine ? s.off + s.u0 + (jb - st0) : INT_MIN);
    const bool use_win = ehi - elo < kFpWin;
    for (int w0 = ia; w0 < ib; w0 += kWave) {
      const int item = w0 + lane;
      int o = 0;  // owner: the first lane whose inclusive count exceeds item
#pragma unroll
      for (int step = 32; step > 0; step >>= 1)
        if (__shfl(incl, o + step - 1, kWave) <= item) o += step;
      o = min(o, kWave - 1);
      const int on = __shfl(s.n, o, kWave);
      int32_t PX[4], PY[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        PX[k] = __shfl(s.X[k], o, kWave);
        PY[k] = __shfl(s.Y[k], o, kWave);
      }
      const int oUc = __shfl(s.Uc, o, kWave), oRc = __shfl(s.Rc, o, kWave);
      const int ooff = __shfl(s.off, o, kWave);
      const int u =
          __shfl(s.u0, o, kWave) + item - (__shfl(incl, o, kWave) - __shfl(s.cnt, o, kWave));
      if (item >= ib) continue;
      const bool open_l = u == 0, open_r = u == oUc - 1;
      const int64_t sl = 256 * (int64_t)u, sr = sl + 256;
      int32_t rlo = INT_MAX, rhi = INT_MIN;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k < on && (open_l || PX[k] >= sl) && (open_r || PX[k] <= sr)) {
          rlo = min(rlo, PY[k] >> 8);
          rhi = max(rhi, PY[k] >> 8);
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k >= on) continue;
        // next vertex with constant indices: k + 1, or vertex 0 after the last
        const bool wrap = k + 1 >= on;
        const int64_t Px = PX[k], Py = PY[k];
        const int64_t Qx = wrap ? PX[0] : PX[k < 3 ? k + 1 : 0];
        const int64_t Qy = wrap ? PY[0] : PY[k < 3 ? k + 1 : 0];
        if (Px == Qx) continue;
        const int64_t lo2 = min(Px, Qx), hi2 = max(Px, Qx);
        if (!open_l && lo2 < sl && sl < hi2) {
          const int32_t r = crossing_row(Px, Py, Qx, Qy, sl);
          rlo = min(rlo, r);
          rhi = max(rhi, r);
        }
        if (!open_r && lo2 < sr && sr < hi2) {
          const int32_t r = crossing_row(Px, Py, Qx, Qy, sr);
          rlo = min(rlo, r);
          rhi = max(rhi, r);
        }
      }
      if (rlo > rhi) continue;
      rlo = min(oRc - 1, max(0, rlo));
      rhi = min(oRc - 1, max(0, rhi));
      if (use_win) {
        atomicMin(&win[ooff + u - elo].x, rlo);
        atomicMax(&win[ooff + u - elo].y, rhi);
      } else {
        atomicMin(&prof[ooff + u].x, rlo);
        atomicMax(&prof[ooff + u].y, rhi);
      }
    }
    if (use_win) {
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      for (int e = lane; e <= ehi - elo; e += kWave) {
        const int2 v = win[e];
        if (v.y >= 0) {
          atomicMin(&prof[elo + e].x, v.x);
          atomicMax(&prof[elo + e].y, v.y);
          win[e] = make_int2(INT_MAX, -1);
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
  }
}
}  // namespace

hipError_t launch_footprint(const int32_t* idx, int64_t T, const FrameParams& p, const Work& w,
                            const int32_t* cot, const fa_chart* charts, Marker& mk,
                            hipStream_t st) {
  if (p.fp_cap > 0) {
    // one wave per group of 64 entries, then the blocks that clear the profile
    const unsigned cb = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((T + kBlock - 1) / kBlock, 2048));
    const unsigned clear = (unsigned)std::min<int64_t>(1024, (p.fp_cap + kBlock - 1) / kBlock);
    k_fp_count<<<cb + clear, kBlock, 0, st>>>(w.vlist, idx, w.pos, cot, charts, w.fp_off,
                                              w.fp_group, w.fp_prof, cb, p, w.state);
  }
  mk(st);
  if (p.fp_cap > 0 && T > 0) {
    k_fp_scan<<<1, 1024, 0, st>>>(w.fp_group, w.state);
    k_fp_raster<<<visible_grid(T), kBlock, 0, st>>>(w.vlist, idx, w.pos, cot, charts, w.fp_off,
                                                    w.fp_group, w.fp_prof, p, w.state);
  }
  mk(st);
  return hipGetLastError();
}

hipError_t launch_meta(const FrameParams& p, const Work& w, fa_atlas_meta* meta,
                       hipStream_t st) {
  k_meta<<<1, kWave, 0, st>>>(p, w.state, w.big_counter, meta);
  return hipGetLastError();
}

hipError_t launch_occupancy_batched(const BatchView* dev, int n, const int32_t* idx, int64_t T,
                                    int64_t V, int small_texels, int lane_texels,
                                    hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const uint32_t cap = (uint32_t)std::min<int64_t>(2 * std::max<int64_t>(T, 1), kBigCap);
  const unsigned occ_blocks = T > 0 ? visible_grid(T) : 0;
  const unsigned uv_blocks = (unsigned)((V + kOccSmallBlock * kUvPerBatch - 1) /
                                         (kOccSmallBlock * kUvPerBatch));
  if (occ_blocks + uv_blocks > 0)
    k_occ_small_b<<<dim3(occ_blocks + uv_blocks, n), kOccSmallBlock, 0, st>>>(
        dev, idx, cap, small_texels, lane_texels, occ_blocks, V);
  if (T > 0) k_occ_big_b<<<dim3(kOccBigGrid, n), kBlock, 0, st>>>(dev, idx, cap);
  k_occ_count_meta_b<<<dim3(kCountGrid, n), kCountBlock, 0, st>>>(dev);
  return hipGetLastError();
}

}  // namespace fa
