// Stable LSD radix sort of (key, value) pairs on gfx950 and its two users:
//   * per-scene triangle adjacency: half-edges sorted by undirected edge key
//     (the twin relation of the half-edge structure in the paper's
//     data-structure table);
//   * per-frame box order (Sec. "Box Ordering via Cuckoo Hashing"): height
//     descending, ties by the chart's lowest triangle index. The paper buckets
//     by height with a cuckoo hash whose in-bucket order is only required to
//     repeat across frames; a stable 13-bit sort gives the lexicographic order
//     the paper names as its ordering criterion.
//
// One pass = tile histograms -> one exclusive scan over (digit, tile) ->
// stable scatter. Within a tile, items are ranked round by round; inside a
// wave, lanes with equal digits are found with eight ballots.
#include "fa_internal.h"

namespace fa {
namespace {

template <typename K>
__global__ void k_radix_hist(const K* __restrict__ keys, const int32_t* __restrict__ n_dev,
                             int64_t n_host, int shift, uint32_t* __restrict__ hist) {
  const int64_t n = n_dev ? min((int64_t)*n_dev, n_host) : n_host;
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  const int64_t b = blockIdx.x;
  if (b >= ntiles) return;
  __shared__ uint32_t h[kRadix];
  for (int d = threadIdx.x; d < kRadix; d += blockDim.x) h[d] = 0;
  __syncthreads();
  for (int k = 0; k < kSortTile; k += blockDim.x) {
    int64_t i = b * kSortTile + k + threadIdx.x;
    if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += blockDim.x) hist[(int64_t)d * ntiles + b] = h[d];
}

// Exclusive scan of the digit-major histogram in three launches: every
// workgroup of 1024 threads sums its chunk of kScanChunk words (4 per
// thread), one workgroup scans those sums, and every workgroup scans its
// chunk again from its offset.
constexpr int kScanThreads = 1024;
constexpr int kScanChunk = 4 * kScanThreads;

__device__ __forceinline__ int64_t hist_words(const int32_t* n_dev, int64_t n_host) {
  const int64_t n = n_dev ? min((int64_t)*n_dev, n_host) : n_host;
  return (n + kSortTile - 1) / kSortTile * kRadix;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ hist,
                                                              const int32_t* __restrict__ n_dev,
                                                              int64_t n_host,
                                                              uint32_t* __restrict__ part) {
  __shared__ uint32_t sh[kScanThreads / kWave];
  const int64_t total = hist_words(n_dev, n_host);
  const int64_t i0 = (int64_t)blockIdx.x * kScanChunk + 4 * (int64_t)threadIdx.x;
  if ((int64_t)blockIdx.x * kScanChunk >= total) return;
  uint32_t v = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) v += i0 + k < total ? hist[i0 + k] : 0u;
  v = block_sum<uint32_t>(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_parts(uint32_t* __restrict__ part,
                                                             const int32_t* __restrict__ n_dev,
                                                             int64_t n_host) {
  __shared__ uint32_t sh[kScanThreads / kWave];
  const int64_t nb = (hist_words(n_dev, n_host) + kScanChunk - 1) / kScanChunk;
  uint32_t run = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kScanThreads) {
    const int64_t i = c0 + threadIdx.x;
    const uint32_t v = i < nb ? part[i] : 0u;
    uint32_t tot;
    const uint32_t ex = run + block_incl_scan<uint32_t>(v, sh, &tot) - v;
    if (i < nb) part[i] = ex;
    run += tot;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(uint32_t* __restrict__ hist,
                                                             const int32_t* __restrict__ n_dev,
                                                             int64_t n_host,
                                                             const uint32_t* __restrict__ part) {
  __shared__ uint32_t sh[kScanThreads / kWave];
  const int64_t total = hist_words(n_dev, n_host);
  if ((int64_t)blockIdx.x * kScanChunk >= total) return;
  const int64_t i0 = (int64_t)blockIdx.x * kScanChunk + 4 * (int64_t)threadIdx.x;
  uint32_t v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = i0 + k < total ? hist[i0 + k] : 0u;
  const uint32_t mine = v[0] + v[1] + v[2] + v[3];
  uint32_t tot;
  uint32_t pre = part[blockIdx.x] + block_incl_scan<uint32_t>(mine, sh, &tot) - mine;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (i0 + k < total) hist[i0 + k] = pre;
    pre += v[k];
  }
}

// Stable scatter; blockDim.x == kRadix == 256 (4 waves).
template <typename K>
__global__ __launch_bounds__(kRadix) void k_radix_scatter(
    const K* __restrict__ kin, const int32_t* __restrict__ vin, K* __restrict__ kout,
    int32_t* __restrict__ vout, const int32_t* __restrict__ n_dev, int64_t n_host, int shift,
    const uint32_t* __restrict__ hist) {
  const int64_t n = n_dev ? min((int64_t)*n_dev, n_host) : n_host;
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  const int64_t b = blockIdx.x;
  if (b >= ntiles) return;
  constexpr int NW = kRadix / kWave;
  __shared__ uint32_t base[kRadix];
  __shared__ uint32_t wcnt[NW][kRadix];
  const int tid = threadIdx.x, w = tid / kWave;
  base[tid] = hist[(int64_t)tid * ntiles + b];
  for (int round = 0; round < kSortTile / kRadix; ++round) {
#pragma unroll
    for (int k = 0; k < NW; ++k) wcnt[k][tid] = 0;
    __syncthreads();
    const int64_t i = b * kSortTile + (int64_t)round * kRadix + tid;
    const bool valid = i < n;
    K key = valid ? kin[i] : (K)0;
    const uint32_t d = (uint32_t)(key >> shift) & (kRadix - 1);
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const bool on = (d >> bit) & 1u;
      const unsigned long long bb = __ballot(on);
      m &= on ? bb : ~bb;
    }
    const unsigned long long below = m & lanes_below();
    const uint32_t rank = (uint32_t)__popcll(below);
    if (valid && below == 0) wcnt[w][d] = (uint32_t)__popcll(m);
    __syncthreads();
    {
      uint32_t run = base[tid];
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        uint32_t c = wcnt[k][tid];
        wcnt[k][tid] = run;
        run += c;
      }
      base[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = wcnt[w][d] + rank;
      kout[pos] = key;
      vout[pos] = vin[i];
    }
    __syncthreads();
  }
}

template <typename K>
hipError_t radix_sort(K* keys_a, int32_t* vals_a, K* keys_b, int32_t* vals_b, uint32_t* hist,
                      uint32_t* part, const int32_t* n_dev, int64_t n_cap, int bits,
                      hipStream_t st, bool* in_b) {
  const unsigned tiles = (unsigned)((n_cap + kSortTile - 1) / kSortTile);
  const unsigned chunks =
      std::max(1u, (unsigned)(((int64_t)tiles * kRadix + kScanChunk - 1) / kScanChunk));
  bool flip = false;
  for (int shift = 0; shift < bits; shift += kRadixBits) {
    const K* ki = flip ? keys_b : keys_a;
    const int32_t* vi = flip ? vals_b : vals_a;
    K* ko = flip ? keys_a : keys_b;
    int32_t* vo = flip ? vals_a : vals_b;
    if (tiles) k_radix_hist<K><<<tiles, kRadix, 0, st>>>(ki, n_dev, n_cap, shift, hist);
    k_scan_reduce<<<chunks, kScanThreads, 0, st>>>(hist, n_dev, n_cap, part);
    k_scan_parts<<<1, kScanThreads, 0, st>>>(part, n_dev, n_cap);
    k_scan_apply<<<chunks, kScanThreads, 0, st>>>(hist, n_dev, n_cap, part);
    if (tiles)
      k_radix_scatter<K><<<tiles, kRadix, 0, st>>>(ki, vi, ko, vo, n_dev, n_cap, shift, hist);
    flip = !flip;
  }
  *in_b = flip;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// adjacency
// ---------------------------------------------------------------------------
__global__ void k_edge_keys(const int32_t* __restrict__ idx, int64_t T, unsigned long long V,
                            unsigned long long* __restrict__ keys, int32_t* __restrict__ vals) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= 3 * T) return;
  const int64_t t = h / 3;
  const int e = (int)(h - 3 * t);
  const unsigned long long a = (uint32_t)idx[3 * t + e];
  const unsigned long long b = (uint32_t)idx[3 * t + (e == 2 ? 0 : e + 1)];
  keys[h] = (a == b) ? V * V : (a < b ? a * V + b : b * V + a);
  vals[h] = (int32_t)h;
}

// In each run of equal keys, every half-edge points at the triangle of the
// next half-edge of the run (cyclically); lone and degenerate edges get -1.
__global__ void k_edge_runs(const unsigned long long* __restrict__ keys,
                            const int32_t* __restrict__ vals, int64_t n, unsigned long long deg,
                            int32_t* __restrict__ nbr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long k = keys[i];
  int32_t out = -1;
  if (k != deg) {
    const bool nxt = i + 1 < n && keys[i + 1] == k;
    const bool prv = i > 0 && keys[i - 1] == k;
    if (nxt) {
      out = vals[i + 1] / 3;
    } else if (prv) {
      int64_t s = i - 1;
      while (s > 0 && keys[s - 1] == k) --s;
      out = vals[s] / 3;
    }
  }
  nbr[vals[i]] = out;
}

// ---------------------------------------------------------------------------
// per-frame chart sizes and order, one workgroup of 1024 threads
// ---------------------------------------------------------------------------
// Chart frame and target size (Sec. bounding boxes, last paragraph; Sec.
// fixed shading rate): the union of the triangles' NDC boxes (all empty ->
// zero box, -0 -> +0), viewport transform times the rate, rotation so the box
// is at least as tall as wide (Sec. "Box Ordering…"), 13-bit height key.
__device__ __forceinline__ void chart_size(const FrameParams& p, const uint4 e, fa_chart& ch,
                                           uint32_t& key_out, float2& oriented) {
  float x0 = 0.0f, y0 = 0.0f, x1 = 0.0f, y1 = 0.0f;
  if (e.z != 0u) {
    x0 = float_of(e.x);
    y0 = float_of(e.y);
    x1 = float_of(e.z);
    y1 = float_of(e.w);
  }
  x0 = x0 + 0.0f; y0 = y0 + 0.0f; x1 = x1 + 0.0f; y1 = y1 + 0.0f;
  const float halfW = 0.5f * (float)p.W, halfH = 0.5f * (float)p.H;
  const float tw = ((x1 - x0) * halfW) * p.rate;
  const float th = ((y1 - y0) * halfH) * p.rate;
  const int rot = tw > th ? 1 : 0;
  const float bw = rot ? th : tw, bh = rot ? tw : th;
  const int key = min((int)ceilf(bh), kKeyCap);
  ch.ndc_box[0] = x0; ch.ndc_box[1] = y0; ch.ndc_box[2] = x1; ch.ndc_box[3] = y1;
  ch.target_w = tw; ch.target_h = th;
  ch.oriented_w = bw; ch.oriented_h = bh;
  ch.rotated = rot;
  ch.key = key;
  key_out = (uint32_t)(kKeyCap - key);
  oriented = make_float2(bw, bh);
}

// Sizes (when from_accum) and the stable order by (height desc, chart asc):
// two 8-bit LSD radix passes over the 13-bit keys in one workgroup, items
// ranked 1024 at a time (ballot matching inside a wave, per-wave digit counts
// across the 16 waves), then the sorted oriented sizes for the packer. Frames
// of up to kOrderLds charts keep keys, values and sizes in LDS throughout
// (only the final order goes to global memory). With
// fp_off (footprint push): each chart's full-scale profile columns,
// floor(oriented width) + 1, are laid out in chart order (exclusive scan);
// a total above the capacity ends the frame with FA_ERR_CAPACITY.
constexpr int kOrderThreads = 1024;
constexpr int kOrderLds = 2048;     // most charts whose keys, values and sizes fit in LDS
constexpr int kOrderSingle = 1024;  // most charts one workgroup orders in global memory

// The body for one placement of the keys and values (LDS or global memory),
// so that every access of the sort has a known address space.
template <bool LDS>
__device__ __forceinline__ void order_body(const FrameParams& p, const uint32_t* __restrict__ accum,
                                           fa_chart* __restrict__ charts, uint32_t* KA,
                                           int32_t* VA, uint32_t* KB, int32_t* VB, float2* lwh,
                                           int32_t* __restrict__ vals_out,
                                           float2* __restrict__ sorted_wh, int from_accum,
                                           int32_t* __restrict__ fp_off, FrameState* st, int C,
                                           uint32_t* base, uint32_t (*wcnt)[kRadix],
                                           uint32_t* sh, long long* sh64) {
  constexpr int NW = kOrderThreads / kWave;
  const int tid = threadIdx.x, w = tid / kWave;
  if (from_accum) {
    for (int c = tid; c < C; c += kOrderThreads) {
      uint32_t key;
      // the box words were reduced with atomics (possibly on other XCDs):
      // read them with agent-scope loads, not through a maybe-stale L2 line
      uint4 box;
      box.x = __hip_atomic_load(&accum[4 * c + 0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      box.y = __hip_atomic_load(&accum[4 * c + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      box.z = __hip_atomic_load(&accum[4 * c + 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      box.w = __hip_atomic_load(&accum[4 * c + 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      float2 wh;
      chart_size(p, box, charts[c], key, wh);
      KA[c] = key;
      VA[c] = c;
      if (LDS) lwh[c] = wh;
    }
    __syncthreads();
  }
  for (int pass = 0; pass < 2; ++pass) {
    const int shift = kRadixBits * pass;
    const uint32_t* kin = pass ? KB : KA;
    const int32_t* vin = pass ? VB : VA;
    uint32_t* kout = pass ? KA : KB;
    int32_t* vout = pass ? VA : VB;
    if (tid < kRadix) base[tid] = 0;
    __syncthreads();
    for (int c = tid; c < C; c += kOrderThreads) atomicAdd(&base[(kin[c] >> shift) & (kRadix - 1)], 1u);
    __syncthreads();
    {
      const uint32_t v = tid < kRadix ? base[tid] : 0u;
      uint32_t tot;
      const uint32_t ex = block_incl_scan_dpp<kOrderThreads>(v, sh, &tot) - v;
      __syncthreads();  // (sh is reused by the next scan)
      if (tid < kRadix) base[tid] = ex;
    }
    for (int c0 = 0; c0 < C; c0 += kOrderThreads) {
      uint32_t* flat = &wcnt[0][0];
#pragma unroll
      for (int k = 0; k < NW * kRadix / kOrderThreads; ++k) flat[tid + k * kOrderThreads] = 0u;
      __syncthreads();
      const int i = c0 + tid;
      const bool valid = i < C;
      const uint32_t key = valid ? kin[i] : 0u;
      const int32_t val = valid ? vin[i] : 0;
      const uint32_t d = (key >> shift) & (kRadix - 1);
      unsigned long long m = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < kRadixBits; ++bit) {
        const bool on = (d >> bit) & 1u;
        const unsigned long long bb = __ballot(on);
        m &= on ? bb : ~bb;
      }
      const unsigned long long below = m & lanes_below();
      const uint32_t rank = (uint32_t)__popcll(below);
      if (valid && below == 0) wcnt[w][d] = (uint32_t)__popcll(m);
      __syncthreads();
      if (tid < kRadix) {
        uint32_t run = base[tid];
#pragma unroll
        for (int k = 0; k < NW; ++k) {
          const uint32_t c = wcnt[k][tid];
          wcnt[k][tid] = run;
          run += c;
        }
        base[tid] = run;
      }
      __syncthreads();
      if (valid) {
        const uint32_t pos = wcnt[w][d] + rank;
        kout[pos] = key;
        vout[pos] = val;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < C; i += kOrderThreads) {
    const int c = VA[i];
    fa_chart& ch = charts[c];
    if (LDS) {
      sorted_wh[i] = lwh[c];
      vals_out[i] = c;
    } else {
      sorted_wh[i] = make_float2(ch.oriented_w, ch.oriented_h);
    }
    ch.order_rank = i;
  }
  if (fp_off) {
    long long run = 0;
    for (int base0 = 0; base0 < C; base0 += kOrderThreads) {
      const int c = base0 + tid;
      const long long n =
          c < C ? (long long)floorf(LDS ? lwh[c].x : charts[c].oriented_w) + 1 : 0;
      long long tot;
      const long long incl = block_incl_scan<long long>(n, sh64, &tot);
      if (c < C) fp_off[c] = (int32_t)min(run + incl - n, (long long)p.fp_cap);
      run += tot;
    }
    if (tid == 0) {
      fp_off[C] = (int32_t)min(run, (long long)p.fp_cap);
      st->fp_columns = (int32_t)min(run, (long long)p.fp_cap);
      if (run > p.fp_cap) st->status = FA_ERR_CAPACITY;
    }
  }
}

// ---- many charts: the same two passes over kOrderGroups chunks ------------
// Above kOrderLds charts one workgroup spends most of its time waiting on
// global memory round by round, so frames with many charts split the items
// into kOrderGroups contiguous chunks, processed by the launch's workgroups
// in five phases: sizes and digit-0 histograms, digit-0 scatter, digit-1
// histograms, digit-1 scatter, copy into packing order. In every phase each
// workgroup claims chunks from a counter until none are left; the next phase
// starts once every chunk of this one is finished. A chunk's digit offsets
// come from all the histograms (digit-major, so the sort stays stable) and
// the in-workgroup ranking above. Any one resident workgroup can finish a
// phase by itself, so the order makes progress however few of the launch's
// workgroups the device runs at once (other streams may hold the rest).
// Everything another workgroup reads goes through agent-scope loads and
// stores (the workgroups sit on different XCDs, each with its own L2).

// Claim the next chunk of a phase (uniform over the workgroup).
__device__ __forceinline__ int claim_chunk(uint32_t* ctr, int* slot) {
  __syncthreads();  // every thread has read the previous claim
  if (threadIdx.x == 0)
    *slot = (int)__hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return *slot;
}

// A chunk is finished once every thread's stores have completed.
__device__ __forceinline__ void chunk_done(uint32_t* ctr) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until all kOrderGroups chunks of a phase are finished. Only chunks
// that some running workgroup has claimed are outstanding, so the wait ends;
// it is bounded anyway, and a workgroup that gives up reports FA_ERR_DEVICE.
constexpr uint32_t kSyncSpins = 1u << 22;
__device__ __forceinline__ bool phase_wait(uint32_t* ctr, FrameState* st, int* flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               (uint32_t)kOrderGroups &&
           spins < kSyncSpins) {
      __builtin_amdgcn_s_sleep(2);
      ++spins;
    }
    *flag = spins < kSyncSpins;
    if (!*flag) st->status = FA_ERR_DEVICE;
  }
  __syncthreads();
  return *flag != 0;
}

__device__ __forceinline__ uint32_t aload_u(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void astore_u(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t aload_i(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void astore_i(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Digit histogram of keys [lo, hi) into row `b` of the block-major table.
__device__ __forceinline__ void chunk_hist(const uint32_t* kin, int lo, int hi, int shift, int b,
                                           uint32_t* hist, uint32_t* cnt) {
  const int tid = threadIdx.x;
  if (tid < kRadix) cnt[tid] = 0;
  __syncthreads();
  for (int i = lo + tid; i < hi; i += kOrderThreads)
    atomicAdd(&cnt[(aload_u(&kin[i]) >> shift) & (kRadix - 1)], 1u);
  __syncthreads();
  if (tid < kRadix) astore_u(&hist[b * kRadix + tid], cnt[tid]);
}

// This workgroup's first output position per digit: all items of smaller
// digits, then the items of the same digit in earlier chunks.
__device__ __forceinline__ void chunk_base(const uint32_t* hist, int b, uint32_t* base,
                                           uint32_t* sh) {
  const int tid = threadIdx.x;
  uint32_t tot = 0, before = 0;
  if (tid < kRadix) {
    uint32_t x[kOrderGroups];
#pragma unroll
    for (int g = 0; g < kOrderGroups; ++g) x[g] = aload_u(&hist[g * kRadix + tid]);
#pragma unroll
    for (int g = 0; g < kOrderGroups; ++g) {
      tot += x[g];
      before += g < b ? x[g] : 0u;
    }
  }
  uint32_t all;
  const uint32_t incl = block_incl_scan_dpp<kOrderThreads>(tot, sh, &all);
  if (tid < kRadix) base[tid] = incl - tot + before;
  __syncthreads();
}

// Stable scatter of items [lo, hi) by the digit at `shift`, from this
// workgroup's offsets `base`.
__device__ __forceinline__ void chunk_scatter(const uint32_t* kin, const int32_t* vin,
                                              uint32_t* kout, int32_t* vout, int lo, int hi,
                                              int shift, uint32_t* base,
                                              uint32_t (*wcnt)[kRadix]) {
  constexpr int NW = kOrderThreads / kWave;
  const int tid = threadIdx.x, w = tid / kWave;
  for (int c0 = lo; c0 < hi; c0 += kOrderThreads) {
    uint32_t* flat = &wcnt[0][0];
#pragma unroll
    for (int k = 0; k < NW * kRadix / kOrderThreads; ++k) flat[tid + k * kOrderThreads] = 0u;
    __syncthreads();
    const int i = c0 + tid;
    const bool valid = i < hi;
    const uint32_t key = valid ? aload_u(&kin[i]) : 0u;
    const int32_t val = valid ? aload_i(&vin[i]) : 0;
    const uint32_t d = (key >> shift) & (kRadix - 1);
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const bool on = (d >> bit) & 1u;
      const unsigned long long bb = __ballot(on);
      m &= on ? bb : ~bb;
    }
    const unsigned long long below = m & lanes_below();
    const uint32_t rank = (uint32_t)__popcll(below);
    if (valid && below == 0) wcnt[w][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (tid < kRadix) {
      uint32_t run = base[tid];
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const uint32_t c = wcnt[k][tid];
        wcnt[k][tid] = run;
        run += c;
      }
      base[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = wcnt[w][d] + rank;
      astore_u(&kout[pos], key);
      astore_i(&vout[pos], val);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void order_multi(const FrameParams& p, const uint32_t* __restrict__ accum,
                                            fa_chart* __restrict__ charts, uint32_t* KA,
                                            int32_t* VA, uint32_t* KB, int32_t* VB,
                                            float2* __restrict__ sorted_wh, int from_accum,
                                            int32_t* __restrict__ fp_off, FrameState* st, int C,
                                            uint32_t* hist, unsigned long long* part,
                                            uint32_t* base, uint32_t (*wcnt)[kRadix],
                                            uint32_t* sh, long long* sh64, int* flag,
                                            int* slot) {
  const int tid = threadIdx.x;
  constexpr int G = kOrderGroups;
  const int chunk = (C + G - 1) / G;
  // phase 0: sizes of a chunk's charts (the oriented size also as agent-scope
  // words: another workgroup copies it into the packing order), the chunk's
  // footprint columns and its digit-0 histogram
  for (int ch; (ch = claim_chunk(&st->order_claim[0], slot)) < G;) {
    const int lo = min(C, ch * chunk), hi = min(C, lo + chunk);
    long long cols = 0;
    for (int c = lo + tid; c < hi; c += kOrderThreads) {
      float2 wh;
      if (from_accum) {
        uint4 box;
        box.x = aload_u(&accum[4 * c + 0]);
        box.y = aload_u(&accum[4 * c + 1]);
        box.z = aload_u(&accum[4 * c + 2]);
        box.w = aload_u(&accum[4 * c + 3]);
        uint32_t key;
        chart_size(p, box, charts[c], key, wh);
        astore_u(&KA[c], key);
        astore_i(&VA[c], c);
        astore_i(reinterpret_cast<int32_t*>(&charts[c].oriented_w), __float_as_int(wh.x));
        astore_i(reinterpret_cast<int32_t*>(&charts[c].oriented_h), __float_as_int(wh.y));
      } else {
        wh = make_float2(charts[c].oriented_w, charts[c].oriented_h);
      }
      if (fp_off) cols += (long long)floorf(wh.x) + 1;
    }
    if (fp_off) {
      const long long sum = block_sum<long long>(cols, sh64);
      if (tid == 0)
        __hip_atomic_store(&part[ch], (unsigned long long)sum, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    chunk_hist(KA, lo, hi, 0, ch, hist, base);
    chunk_done(&st->order_done[0]);
  }
  if (!phase_wait(&st->order_done[0], st, flag)) return;
  // phase 1: footprint columns in chart order, digit-0 scatter
  for (int ch; (ch = claim_chunk(&st->order_claim[1], slot)) < G;) {
    const int lo = min(C, ch * chunk), hi = min(C, lo + chunk);
    if (fp_off) {
      long long run = 0, total = 0;  // earlier chunks' columns, all chunks'
      // (four loads at a time: all 32 at once spill registers to scratch)
#pragma unroll 4
      for (int g = 0; g < G; ++g) {
        const long long v = (long long)__hip_atomic_load(&part[g], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
        run += g < ch ? v : 0;
        total += v;
      }
      for (int c0 = lo; c0 < hi; c0 += kOrderThreads) {
        const int c = c0 + tid;
        const long long n =
            c < hi ? (long long)floorf(__int_as_float(aload_i(
                         reinterpret_cast<const int32_t*>(&charts[c].oriented_w)))) + 1
                   : 0;
        long long tot;
        const long long incl = block_incl_scan<long long>(n, sh64, &tot);
        if (c < hi) fp_off[c] = (int32_t)min(run + incl - n, (long long)p.fp_cap);
        run += tot;
      }
      if (ch == G - 1 && tid == 0) {
        fp_off[C] = (int32_t)min(total, (long long)p.fp_cap);
        st->fp_columns = (int32_t)min(total, (long long)p.fp_cap);
        if (total > p.fp_cap) st->status = FA_ERR_CAPACITY;
      }
    }
    chunk_base(hist, ch, base, sh);
    chunk_scatter(KA, VA, KB, VB, lo, hi, 0, base, wcnt);
    chunk_done(&st->order_done[1]);
  }
  if (!phase_wait(&st->order_done[1], st, flag)) return;
  // phase 2: digit-1 histograms of the digit-0 order
  for (int ch; (ch = claim_chunk(&st->order_claim[2], slot)) < G;) {
    const int lo = min(C, ch * chunk), hi = min(C, lo + chunk);
    chunk_hist(KB, lo, hi, kRadixBits, ch, hist, base);
    chunk_done(&st->order_done[2]);
  }
  if (!phase_wait(&st->order_done[2], st, flag)) return;
  // phase 3: digit-1 scatter
  for (int ch; (ch = claim_chunk(&st->order_claim[3], slot)) < G;) {
    const int lo = min(C, ch * chunk), hi = min(C, lo + chunk);
    chunk_base(hist, ch, base, sh + kOrderThreads / kWave);
    chunk_scatter(KB, VB, KA, VA, lo, hi, kRadixBits, base, wcnt);
    chunk_done(&st->order_done[3]);
  }
  if (!phase_wait(&st->order_done[3], st, flag)) return;
  // phase 4: sizes in packing order and each chart's rank
  for (int ch; (ch = claim_chunk(&st->order_claim[4], slot)) < G;) {
    const int lo = min(C, ch * chunk), hi = min(C, lo + chunk);
    for (int i = lo + tid; i < hi; i += kOrderThreads) {
      const int c = aload_i(&VA[i]);
      const float w =
          __int_as_float(aload_i(reinterpret_cast<const int32_t*>(&charts[c].oriented_w)));
      const float h =
          __int_as_float(aload_i(reinterpret_cast<const int32_t*>(&charts[c].oriented_h)));
      sorted_wh[i] = make_float2(w, h);
      charts[c].order_rank = i;
    }
  }
}

__device__ __forceinline__ void k_sizes_order_body(
    FrameParams p, const uint32_t* __restrict__ accum, fa_chart* __restrict__ charts,
    uint32_t* __restrict__ keys_a, int32_t* __restrict__ vals_a, uint32_t* __restrict__ keys_b,
    int32_t* __restrict__ vals_b, float2* __restrict__ sorted_wh, int from_accum,
    int32_t* __restrict__ fp_off, FrameState* __restrict__ st, uint32_t* __restrict__ hist,
    unsigned long long* __restrict__ part) {
  constexpr int NW = kOrderThreads / kWave;
  __shared__ uint32_t base[kRadix];
  __shared__ uint32_t wcnt[NW][kRadix];
  __shared__ uint32_t sh[2 * NW];
  __shared__ long long sh64[NW];
  __shared__ uint32_t lk[2][kOrderLds];
  __shared__ int32_t lv[2][kOrderLds];
  __shared__ float2 lwh[kOrderLds];
  __shared__ int flag, slot;
  if (st->status != FA_OK) return;
  const int C = min(st->num_charts, p.max_charts);
  const bool in_lds = from_accum && C <= kOrderLds;
  if (gridDim.x > 1 && !in_lds && C > kOrderSingle) {
    order_multi(p, accum, charts, keys_a, vals_a, keys_b, vals_b, sorted_wh, from_accum, fp_off,
                st, C, hist, part, base, wcnt, sh, sh64, &flag, &slot);
    return;
  }
  if (blockIdx.x != 0) return;
  if (in_lds)
    order_body<true>(p, accum, charts, lk[0], lv[0], lk[1], lv[1], lwh, vals_a, sorted_wh,
                     from_accum, fp_off, st, C, base, wcnt, sh, sh64);
  else
    order_body<false>(p, accum, charts, keys_a, vals_a, keys_b, vals_b, nullptr, vals_a,
                      sorted_wh, from_accum, fp_off, st, C, base, wcnt, sh, sh64);
}
__global__ __launch_bounds__(kOrderThreads) void k_sizes_order(
    FrameParams p, const uint32_t* __restrict__ accum, fa_chart* __restrict__ charts,
    uint32_t* __restrict__ keys_a, int32_t* __restrict__ vals_a, uint32_t* __restrict__ keys_b,
    int32_t* __restrict__ vals_b, float2* __restrict__ sorted_wh, int from_accum,
    int32_t* __restrict__ fp_off, FrameState* __restrict__ st, uint32_t* __restrict__ hist,
    unsigned long long* __restrict__ part) {
  k_sizes_order_body(p, accum, charts, keys_a, vals_a, keys_b, vals_b, sorted_wh, from_accum,
                     fp_off, st, hist, part);
}

__global__ __launch_bounds__(kOrderThreads) void k_sizes_order_b(const BatchView* __restrict__ bv) {
  const BatchView& v = bv[blockIdx.y];
  k_sizes_order_body(v.p, v.w.accum, v.charts, v.w.keys_a, v.w.vals_a, v.w.keys_b, v.w.vals_b,
                     v.w.sorted_wh, 1, nullptr, v.w.state, v.w.hist, v.w.partial);
}

}  // namespace

size_t adjacency_hist_words(int64_t T) {
  return (size_t)((3 * T + kSortTile - 1) / kSortTile + 1) * kRadix;
}

size_t adjacency_part_words(int64_t T) {
  return adjacency_hist_words(T) / kScanChunk + 2;
}

hipError_t launch_adjacency(const int32_t* idx, int64_t T, int64_t V, const AdjTmp& tmp,
                            int32_t* nbr, hipStream_t st) {
  const int64_t n = 3 * T;
  if (n == 0) return hipSuccess;
  const unsigned long long deg = (unsigned long long)V * (unsigned long long)V;
  int bits = 1;
  while (bits < 64 && (deg >> bits) != 0) ++bits;
  k_edge_keys<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(idx, T, (unsigned long long)V,
                                                                       tmp.keys_a, tmp.vals_a);
  bool in_b = false;
  hipError_t e = radix_sort<unsigned long long>(tmp.keys_a, tmp.vals_a, tmp.keys_b, tmp.vals_b,
                                                tmp.hist, tmp.part, nullptr, n, bits, st, &in_b);
  if (e != hipSuccess) return e;
  k_edge_runs<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      in_b ? tmp.keys_b : tmp.keys_a, in_b ? tmp.vals_b : tmp.vals_a, n, deg, nbr);
  return hipGetLastError();
}

hipError_t launch_order(const FrameParams& p, const Work& w, fa_chart* charts, int from_accum,
                        hipStream_t st) {
  int32_t* fp_off = (from_accum && p.fp_cap > 0) ? w.fp_off : nullptr;
  k_sizes_order<<<kOrderGroups, kOrderThreads, 0, st>>>(p, w.accum, charts, w.keys_a, w.vals_a,
                                                        w.keys_b, w.vals_b, w.sorted_wh,
                                                        from_accum, fp_off, w.state, w.hist,
                                                        w.partial);
  return hipGetLastError();
}

hipError_t launch_order_batched(const BatchView* dev, int n, hipStream_t st) {
  if (n > 0) k_sizes_order_b<<<dim3(kOrderGroups, n), kOrderThreads, 0, st>>>(dev);
  return hipGetLastError();
}

}  // namespace fa
