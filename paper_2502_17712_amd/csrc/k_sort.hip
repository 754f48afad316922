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

// Exclusive scan of the digit-major histogram (one workgroup). Each thread
// owns a contiguous segment: sum, block scan of the sums, then write.
__global__ void k_radix_scan(uint32_t* __restrict__ hist, const int32_t* __restrict__ n_dev,
                             int64_t n_host) {
  __shared__ uint32_t sh[1024 / kWave];
  const int64_t n = n_dev ? min((int64_t)*n_dev, n_host) : n_host;
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  const int64_t total = ntiles * kRadix;
  const int64_t seg = (total + blockDim.x - 1) / blockDim.x;
  const int64_t s0 = min(total, (int64_t)threadIdx.x * seg), s1 = min(total, s0 + seg);
  uint32_t sum = 0;
  for (int64_t i = s0; i < s1; ++i) sum += hist[i];
  uint32_t tot;
  uint32_t run = block_incl_scan<uint32_t>(sum, sh, &tot) - sum;
  for (int64_t i = s0; i < s1; ++i) {
    uint32_t v = hist[i];
    hist[i] = run;
    run += v;
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
                      const int32_t* n_dev, int64_t n_cap, int bits, hipStream_t st, bool* in_b) {
  const unsigned tiles = (unsigned)((n_cap + kSortTile - 1) / kSortTile);
  bool flip = false;
  for (int shift = 0; shift < bits; shift += kRadixBits) {
    const K* ki = flip ? keys_b : keys_a;
    const int32_t* vi = flip ? vals_b : vals_a;
    K* ko = flip ? keys_a : keys_b;
    int32_t* vo = flip ? vals_a : vals_b;
    if (tiles) k_radix_hist<K><<<tiles, kRadix, 0, st>>>(ki, n_dev, n_cap, shift, hist);
    k_radix_scan<<<1, 1024, 0, st>>>(hist, n_dev, n_cap);
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
// per-frame order
// ---------------------------------------------------------------------------
__global__ void k_sorted_sizes(const int32_t* __restrict__ order, fa_chart* __restrict__ charts,
                               float2* __restrict__ wh, const FrameState* __restrict__ st) {
  if (st->status != FA_OK) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= st->num_charts) return;
  const int c = order[i];
  fa_chart& ch = charts[c];
  wh[i] = make_float2(ch.oriented_w, ch.oriented_h);
  ch.order_rank = i;
}

}  // namespace

size_t adjacency_hist_words(int64_t T) {
  return (size_t)((3 * T + kSortTile - 1) / kSortTile + 1) * kRadix;
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
                                                tmp.hist, nullptr, n, bits, st, &in_b);
  if (e != hipSuccess) return e;
  k_edge_runs<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      in_b ? tmp.keys_b : tmp.keys_a, in_b ? tmp.vals_b : tmp.vals_a, n, deg, nbr);
  return hipGetLastError();
}

hipError_t launch_order(const FrameParams& p, const Work& w, fa_chart* charts, hipStream_t st) {
  bool in_b = false;
  hipError_t e = radix_sort<uint32_t>(w.keys_a, w.vals_a, w.keys_b, w.vals_b, w.hist,
                                      &w.state->num_charts, p.max_charts, 13, st, &in_b);
  if (e != hipSuccess) return e;
  // 13 bits take two passes, so the sorted order is back in keys_a / vals_a
  k_sorted_sizes<<<(unsigned)((p.max_charts + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      in_b ? w.vals_b : w.vals_a, charts, w.sorted_wh, w.state);
  return hipGetLastError();
}

}  // namespace fa
