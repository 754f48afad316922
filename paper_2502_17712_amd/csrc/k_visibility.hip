// Visible-triangle pass on gfx950 (App. "Detecting Visible Triangles": a depth
// pre-pass fills a depth buffer, a second pass tests each triangle's samples
// against it with "less or equal" and marks the triangles that pass).
//
// float64 throughout, fixed operation order, no contraction:
//   candidate  faces the eye ((b-a) x (c-a) . (eye-a) > 0) and no clip plane
//              has all three vertices outside;
//   occluder   candidate with every w > near (only these write and test depth);
//   depth      samples at the centres of a (W/k) x (H/k) grid; a covered
//              sample (edge functions all >= 0 or all <= 0, area != 0) gets the
//              NDC z interpolated with the edge-function weights; the buffer
//              keeps the minimum (64-bit order-preserving keys, atomicMin);
//   marking    an occluder stays visible iff it covers no sample (it cannot be
//              proven hidden) or some covered sample has z <= D + 1e-6;
//              candidates crossing the near plane stay visible.
// Small footprints are walked by their own lane, larger ones by their wave.
#include <cmath>

#include "fa_internal.h"

namespace fa {
namespace {

__device__ __forceinline__ double4 clip64(const VisParams& q, const float* __restrict__ pos,
                                          int64_t v) {
  const double x = pos[3 * v], y = pos[3 * v + 1], z = pos[3 * v + 2];
  double r[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    r[i] = ((q.M[4 * i] * x + q.M[4 * i + 1] * y) + q.M[4 * i + 2] * z) + q.M[4 * i + 3];
  return make_double4(r[0], r[1], r[2], r[3]);
}

// order-preserving key of a finite double (smaller value -> smaller key)
__device__ __forceinline__ unsigned long long dkey(double d) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(d);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double dval(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  return __longlong_as_double((long long)b);
}

// the depth buffer and the occluder count are produced by atomics (possibly
// on other XCDs): read them with agent-scope loads
__device__ __forceinline__ unsigned long long dload(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_vis_clear(unsigned long long* __restrict__ depth, int64_t n,
                            uint32_t* __restrict__ count) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = 0u;
  const unsigned long long inf = 0xFFF0000000000000ull;  // dkey(+infinity)
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    depth[i] = inf;
}

// Candidates and occluders. Occluders are gathered per workgroup in LDS and
// appended to the global list with one atomic per full buffer (a single
// counter serializes at about 12 ns per atomic).
constexpr int kCullBlock = 1024;
constexpr int kCullBuf = 8192;

__global__ __launch_bounds__(kCullBlock) void k_vis_cull(const float* __restrict__ pos,
                                                         const int32_t* __restrict__ idx,
                                                         int64_t T, VisParams q,
                                                         uint8_t* __restrict__ vis,
                                                         int32_t* __restrict__ occl,
                                                         uint32_t* __restrict__ count) {
  __shared__ int32_t buf[kCullBuf];
  __shared__ uint32_t sh[kCullBlock / kWave];
  __shared__ uint32_t gbase;
  uint32_t fill = 0;  // entries in buf (block-uniform)
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < T;
       b0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = b0 + threadIdx.x;
    bool occluder = false;
    if (t < T) {
      const int64_t i0 = idx[3 * t], i1 = idx[3 * t + 1], i2 = idx[3 * t + 2];
      double a[3], b[3], d[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double q0 = pos[3 * i0 + k], q1 = pos[3 * i1 + k], q2 = pos[3 * i2 + k];
        a[k] = q1 - q0;
        b[k] = q2 - q0;
        d[k] = q.eye[k] - q0;
      }
      const double n0 = a[1] * b[2] - a[2] * b[1];
      const double n1 = a[2] * b[0] - a[0] * b[2];
      const double n2 = a[0] * b[1] - a[1] * b[0];
      const bool front = ((n0 * d[0] + n1 * d[1]) + n2 * d[2]) > 0.0;
      const double4 c0 = clip64(q, pos, i0), c1 = clip64(q, pos, i1), c2 = clip64(q, pos, i2);
      const bool outside =
          (c0.w + c0.x < 0.0 && c1.w + c1.x < 0.0 && c2.w + c2.x < 0.0) ||
          (c0.w - c0.x < 0.0 && c1.w - c1.x < 0.0 && c2.w - c2.x < 0.0) ||
          (c0.w + c0.y < 0.0 && c1.w + c1.y < 0.0 && c2.w + c2.y < 0.0) ||
          (c0.w - c0.y < 0.0 && c1.w - c1.y < 0.0 && c2.w - c2.y < 0.0) ||
          (c0.w + c0.z < 0.0 && c1.w + c1.z < 0.0 && c2.w + c2.z < 0.0) ||
          (c0.w - c0.z < 0.0 && c1.w - c1.z < 0.0 && c2.w - c2.z < 0.0);
      const bool cand = front && !outside;
      vis[t] = cand ? 1 : 0;
      occluder = q.coarse > 0 && cand && c0.w > q.near_w && c1.w > q.near_w && c2.w > q.near_w;
    }
    uint32_t tot;
    const uint32_t one = occluder ? 1u : 0u;
    const uint32_t at = block_incl_scan<uint32_t>(one, sh, &tot) - one;
    if (fill + tot > (uint32_t)kCullBuf) {  // flush the full buffer first
      if (threadIdx.x == 0) gbase = atomicAdd(count, fill);
      __syncthreads();
      for (uint32_t k = threadIdx.x; k < fill; k += blockDim.x) occl[gbase + k] = buf[k];
      __syncthreads();
      fill = 0;
    }
    if (occluder) buf[fill + at] = (int32_t)t;
    fill += tot;
  }
  __syncthreads();
  if (fill) {
    if (threadIdx.x == 0) gbase = atomicAdd(count, fill);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < fill; k += blockDim.x) occl[gbase + k] = buf[k];
  }
}

// Screen footprint of an occluder: vertices in coarse pixels (x right, y down)
// with their NDC z, and the range of sample centres inside its bounding box.
struct Shot {
  double X[3], Y[3], Z[3];
  int ix0, ix1, iy0, iy1;
};

__device__ __forceinline__ void shot_of(const VisParams& q, const float* __restrict__ pos,
                                        const int32_t* __restrict__ idx, int64_t t, Shot& s) {
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const double4 c = clip64(q, pos, idx[3 * t + e]);
    s.X[e] = ((c.x / c.w) * 0.5 + 0.5) * (double)q.Wc;
    s.Y[e] = (0.5 - (c.y / c.w) * 0.5) * (double)q.Hc;
    s.Z[e] = c.z / c.w;
  }
  const double xmin = fmin(fmin(s.X[0], s.X[1]), s.X[2]), xmax = fmax(fmax(s.X[0], s.X[1]), s.X[2]);
  const double ymin = fmin(fmin(s.Y[0], s.Y[1]), s.Y[2]), ymax = fmax(fmax(s.Y[0], s.Y[1]), s.Y[2]);
  s.ix0 = (int)fmin(fmax(ceil(xmin - 0.5), 0.0), (double)(q.Wc - 1));
  s.ix1 = (int)fmin(fmax(floor(xmax - 0.5), -1.0), (double)(q.Wc - 1));
  s.iy0 = (int)fmin(fmax(ceil(ymin - 0.5), 0.0), (double)(q.Hc - 1));
  s.iy1 = (int)fmin(fmax(floor(ymax - 0.5), -1.0), (double)(q.Hc - 1));
}

// depth of sample (px, py) if the footprint covers it
__device__ __forceinline__ bool sample(const Shot& s, int px, int py, double& z) {
  const double cx = (double)px + 0.5, cy = (double)py + 0.5;
  const double e0 = (s.X[2] - s.X[1]) * (cy - s.Y[1]) - (s.Y[2] - s.Y[1]) * (cx - s.X[1]);
  const double e1 = (s.X[0] - s.X[2]) * (cy - s.Y[2]) - (s.Y[0] - s.Y[2]) * (cx - s.X[2]);
  const double e2 = (s.X[1] - s.X[0]) * (cy - s.Y[0]) - (s.Y[1] - s.Y[0]) * (cx - s.X[0]);
  const double area = (e0 + e1) + e2;
  const bool in = area != 0.0 &&
                  ((e0 >= 0.0 && e1 >= 0.0 && e2 >= 0.0) || (e0 <= 0.0 && e1 <= 0.0 && e2 <= 0.0));
  if (!in) return false;
  z = ((e0 * s.Z[0] + e1 * s.Z[1]) + e2 * s.Z[2]) / area;
  return true;
}

__device__ __forceinline__ double rl_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ Shot rl_shot(const Shot& s, int lane) {
  Shot r;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    r.X[e] = rl_d(s.X[e], lane);
    r.Y[e] = rl_d(s.Y[e], lane);
    r.Z[e] = rl_d(s.Z[e], lane);
  }
  r.ix0 = __builtin_amdgcn_readlane(s.ix0, lane);
  r.ix1 = __builtin_amdgcn_readlane(s.ix1, lane);
  r.iy0 = __builtin_amdgcn_readlane(s.iy0, lane);
  r.iy1 = __builtin_amdgcn_readlane(s.iy1, lane);
  return r;
}

constexpr int kVisLaneSamples = 32;  // larger footprints are walked by the wave

template <bool MARK>
__global__ __launch_bounds__(kBlock) void k_vis_depth(const float* __restrict__ pos,
                                                      const int32_t* __restrict__ idx,
                                                      VisParams q,
                                                      const int32_t* __restrict__ occl,
                                                      const uint32_t* __restrict__ count,
                                                      unsigned long long* __restrict__ depth,
                                                      uint8_t* __restrict__ vis) {
  const int n_occ = (int)__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int lane = lane_id();
  for (int b0 = blockIdx.x * blockDim.x; b0 < n_occ; b0 += gridDim.x * blockDim.x) {
    const int i = b0 + threadIdx.x;
    Shot s;
    int n = 0, nx = 1;
    int t = -1;
    if (i < n_occ) {
      t = occl[i];
      shot_of(q, pos, idx, t, s);
      nx = max(s.ix1 - s.ix0 + 1, 0);
      n = nx * max(s.iy1 - s.iy0 + 1, 0);
    }
    const bool big = n > kVisLaneSamples;
    bool any = false, pass = false;
    if (!big) {
      for (int k = 0; k < n && !pass; ++k) {
        const int px = s.ix0 + k % nx, py = s.iy0 + k / nx;
        double z;
        if (!sample(s, px, py, z)) continue;
        const int64_t pix = (int64_t)py * q.Wc + px;
        if (MARK) {
          any = true;
          if (z <= dval(dload(&depth[pix])) + 1e-6) pass = true;
        } else {
          atomicMin(&depth[pix], dkey(z));
        }
      }
    }
    for (unsigned long long bm = __ballot(big); bm; bm &= bm - 1) {
      const int src = __ffsll((long long)bm) - 1;
      const Shot w = rl_shot(s, src);
      const int wnx = w.ix1 - w.ix0 + 1, wn = wnx * (w.iy1 - w.iy0 + 1);
      bool wany = false, wpass = false;
      for (int k0 = 0; k0 < wn; k0 += kWave) {
        const int k = k0 + lane;
        double z;
        if (k < wn && sample(w, w.ix0 + k % wnx, w.iy0 + k / wnx, z)) {
          const int64_t pix = (int64_t)(w.iy0 + k / wnx) * q.Wc + (w.ix0 + k % wnx);
          if (MARK) {
            wany = true;
            if (z <= dval(dload(&depth[pix])) + 1e-6) wpass = true;
          } else {
            atomicMin(&depth[pix], dkey(z));
          }
        }
        if (MARK && __ballot(wpass)) break;
      }
      if (MARK) {
        const bool ga = __ballot(wany) != 0, gp = __ballot(wpass) != 0;
        if (lane == src) { any = ga; pass = gp; }
      }
    }
    if (MARK && t >= 0) vis[t] = (!any || pass) ? 1 : 0;
  }
}

// Temporal reuse classification (Sec. "Temporal Reuse"): 0 not visible now,
// 1 reuse the key frame's shading, 2 shade (newly visible, or some vertex had
// max(|x|, |y|) >= w in the key frame's clip space, float32 as the atlas path
// computes it). One atomic per wave counts the reused triangles.
__global__ void k_zero64(unsigned long long* p) { *p = 0ull; }

__global__ __launch_bounds__(kBlock) void k_reuse_flags(
    const float* __restrict__ pos, const int32_t* __restrict__ idx, int64_t T, KeyClip kc,
    const uint8_t* __restrict__ key_vis, const uint8_t* __restrict__ vis,
    uint8_t* __restrict__ flags, unsigned long long* __restrict__ reused) {
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < T;
       b0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = b0 + threadIdx.x;
    bool reuse = false;
    if (t < T) {
      uint8_t f = 0;
      if (vis[t]) {
        bool partial = false;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const int64_t v = idx[3 * t + e];
          const float x = pos[3 * v], y = pos[3 * v + 1], z = pos[3 * v + 2];
          float r[4];
#pragma unroll
          for (int i = 0; i < 4; i += 1) {
            if (i == 2) { r[i] = 0.0f; continue; }  // z is not needed
            float acc = kc.M[4 * i] * x;
            acc = acc + kc.M[4 * i + 1] * y;
            acc = acc + kc.M[4 * i + 2] * z;
            r[i] = acc + kc.M[4 * i + 3];
          }
          if (fmaxf(fabsf(r[0]), fabsf(r[1])) >= r[3]) partial = true;
        }
        reuse = key_vis[t] != 0 && !partial;
        f = reuse ? 1 : 2;
      }
      flags[t] = f;
    }
    if (reused) {
      const unsigned long long m = __ballot(reuse);
      if (m && lane_id() == __ffsll((long long)m) - 1)
        atomicAdd(reused, (unsigned long long)__popcll(m));
    }
  }
}

}  // namespace

hipError_t launch_reuse_flags(const float* pos, const int32_t* idx, int64_t T, const KeyClip& kc,
                              const uint8_t* key_vis, const uint8_t* vis, uint8_t* flags,
                              unsigned long long* reused, hipStream_t st) {
  if (reused) k_zero64<<<1, 1, 0, st>>>(reused);
  if (T > 0) {
    const unsigned g = (unsigned)std::min<int64_t>((T + kBlock - 1) / kBlock, 8192);
    k_reuse_flags<<<g, kBlock, 0, st>>>(pos, idx, T, kc, key_vis, vis, flags, reused);
  }
  return hipGetLastError();
}

hipError_t launch_visibility(const float* pos, const int32_t* idx, int64_t T, const VisParams& q,
                             int32_t* occl, uint32_t* count, unsigned long long* depth,
                             uint8_t* vis, hipStream_t st) {
  const int64_t nd = q.coarse > 0 ? (int64_t)q.Wc * q.Hc : 0;
  const unsigned cg = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nd + kBlock - 1) / kBlock, 1024));
  k_vis_clear<<<cg, kBlock, 0, st>>>(depth, nd, count);
  if (T == 0) return hipGetLastError();
  const unsigned g = (unsigned)std::min<int64_t>((T + kCullBlock - 1) / kCullBlock, 256);
  k_vis_cull<<<g, kCullBlock, 0, st>>>(pos, idx, T, q, vis, occl, count);
  if (q.coarse > 0) {
    const unsigned og = visible_grid(T);
    k_vis_depth<false><<<og, kBlock, 0, st>>>(pos, idx, q, occl, count, depth, vis);
    k_vis_depth<true><<<og, kBlock, 0, st>>>(pos, idx, q, occl, count, depth, vis);
  }
  return hipGetLastError();
}

}  // namespace fa
