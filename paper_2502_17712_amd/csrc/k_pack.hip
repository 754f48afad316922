// FastAtlas packing on gfx950 (Secs. "Parallel Atlas and Scale Factor
// Computation" and "Box Packing").
//
// One workgroup evaluates one candidate scale j/J:
//   sizes   a = max(m_min, ceil(w * j/J)) + 2g, b likewise for the height;
//   fold    exclusive prefix sum X of the widths (64-bit), row = X >> log2(omega),
//           offset = X & (omega - 1), overflow m = max(offset + a - omega);
//           layout width L = omega + m (the rows are later rescaled by omega/L);
//   mirror  rows with row % 3 != 0 run right to left;
//   push    row by row, a box rises to the top of the frontline under its span
//           and raises that span by its height. The frontline (L <= 2 omega
//           columns) lives in LDS; the boxes of a row have disjoint spans, so
//           each wave takes whole boxes and one barrier per row orders rows.
// A candidate fits iff m <= omega and the layout height H <= L. Selection takes
// the largest effective scale (j/J) * omega / L, compared exactly.
//
// Footprint push (a generalization of the push to non-rectangular charts):
// a box meets the frontline with its footprint profile instead of its full
// height. The profile of content column k (box column k + g) at scale j/J is
// pooled from the chart's full-scale profile: the fine columns whose scaled
// cells touch k give top row T = floor(min top * j / J) and bottom row B =
// floor((max bottom + 1) * j / J) (inclusive), or the box bottom when they
// reach the chart's last row; the gutter then widens it by g columns and
// rows. With top[d] / bottom[d] = min(b - 1, 2g + B) the widened profile of
// box column d:
//   y = max(0, max_d F[x+d] - top[d]),  F[x+d] = y + bottom[d] + 1,
// computed per content column k (its widened window is d in [k, k + 2g]):
// y = max over k of (max F over the window) - T_k, and, since the new
// frontline value only grows, F[x+d] = max over the k covering d of
// min(y + b, y + 2g + B_k + 1), applied with LDS atomic max.
#include <climits>

#include "fa_internal.h"

namespace fa {
namespace {

// Footprint push: candidates of frames with at most kPackLds charts keep
// their prefix sums and sizes in LDS next to the frontline.
constexpr int kPackLds = 4096;

// Footprint push in three launches: MODE 1 sizes, fold, overflow and row
// starts (to global memory; tab[3] = -1 marks a rejected candidate, tab[5]
// the number of rows with boxes), then k_fp_pool, then MODE 2 the push. (The
// box push is k_pack_box.)
template <int NT, int MODE>
__global__ __launch_bounds__(NT) void k_pack(const float2* __restrict__ wh,
                                             const FrameState* __restrict__ st, FrameParams p,
                                             long long* __restrict__ cand_x,
                                             uint32_t* __restrict__ cand_ab,
                                             int32_t* __restrict__ cand_y,
                                             int32_t* __restrict__ cand_rs,
                                             int32_t* __restrict__ cand_tab, int64_t stride,
                                             const uint32_t* __restrict__ fp_pool,
                                             int64_t pool_stride) {
  // [2 * omega] frontline, then the LDS copies of X, AB and the row starts
  extern __shared__ int32_t F[];
  __shared__ long long sh64[NT / kWave];
  __shared__ int32_t sh32[NT / kWave];
  __shared__ int32_t Hsh[2];
  constexpr int NW = NT / kWave;

  if (st->status != FA_OK) return;
  const int j = blockIdx.x + 1;
  const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
  const int C = st->num_charts;
  const int omega = p.omega, lg = p.log2omega;
  long long* Xg = cand_x + (int64_t)(j - 1) * stride;
  uint32_t* ABg = cand_ab + (int64_t)(j - 1) * stride;
  int32_t* RSg = cand_rs + (int64_t)(j - 1) * (stride + 1);
  const bool in_lds = C <= kPackLds;
  long long* X = in_lds ? reinterpret_cast<long long*>(F + 2 * omega) : Xg;
  uint32_t* AB = in_lds ? reinterpret_cast<uint32_t*>(F + 2 * omega + 2 * kPackLds) : ABg;
  int32_t* RS = (in_lds && MODE != 1) ? F + 2 * omega + 3 * kPackLds : RSg;
  int32_t* Y = cand_y + (int64_t)(j - 1) * stride;
  int32_t* tab = cand_tab + (j - 1) * kCandStride;
  long long m, rows;
  int nr;

  if constexpr (MODE != 2) {
    const float s = (float)j / (float)p.J;
    const int pad = 2 * p.gutter;
    // ---- sizes, fold and overflow -----------------------------------------
    long long run = 0, mloc = 0;
    int bad = 0;
    for (int base = 0; base < C; base += NT) {
      const int i = base + tid;
      int a = 0, b = 0;
      if (i < C) {
        const float2 v = wh[i];
        const int wi = (int)ceilf(v.x * s);
        const int hi = (int)ceilf(v.y * s);
        a = max(p.min_box, wi) + pad;
        b = max(p.min_box, hi) + pad;
      }
      long long tot;
      const long long incl = block_incl_scan<long long>((long long)a, sh64, &tot);
      const long long Xi = run + incl - a;
      run += tot;
      if (i < C) {
        Xg[i] = Xi;
        if (a > 2 * omega || b > 2 * omega) bad = 1;  // cannot fit: m > omega or H > L
        const uint32_t ca = (uint32_t)min(a, 2 * omega + 1), cb = (uint32_t)min(b, 2 * omega + 1);
        ABg[i] = ca | (cb << 16);
        if (in_lds) {
          X[i] = Xi;
          AB[i] = ca | (cb << 16);
        }
        mloc = max(mloc, (Xi & (long long)(omega - 1)) + a - omega);
      }
    }
    m = block_max<long long>(mloc, sh64);
    bad = block_max<int>(bad, sh32);
    rows = C > 0 ? (X[C - 1] >> lg) + 1 : 0;
    if (m > omega || bad) {
      if (tid == 0) {
        tab[0] = 0;
        tab[1] = (int32_t)min(m, (long long)INT_MAX);
        tab[2] = (int32_t)min(m + omega, (long long)INT_MAX);
        tab[3] = -1;
        tab[4] = (int32_t)min(rows, (long long)INT_MAX);
      }
      return;
    }
    // ---- row starts: first box of every non-empty row, in order ------------
    nr = 0;
    for (int base = 0; base < C; base += NT) {
      const int i = base + tid;
      const int first = (i < C && (i == 0 || (X[i] >> lg) != (X[i - 1] >> lg))) ? 1 : 0;
      int tot;
      const int incl = block_incl_scan<int>(first, sh32, &tot);
      if (first) RS[nr + incl - 1] = i;
      nr += tot;
    }
    if (tid == 0) RS[nr] = C;
    if constexpr (MODE == 1) {
      if (tid == 0) {
        tab[0] = 0;
        tab[1] = (int32_t)m;
        tab[2] = omega + (int)m;
        tab[3] = 0;
        tab[4] = (int32_t)min(rows, (long long)INT_MAX);
        tab[5] = nr;
      }
      return;
    }
  } else {
    if (tab[3] < 0) return;  // rejected by its fold
    m = tab[1];
    rows = tab[4];
    nr = tab[5];
    if (in_lds) {
      for (int i = tid; i < C; i += NT) {
        X[i] = Xg[i];
        AB[i] = ABg[i];
      }
      for (int i = tid; i <= nr; i += NT) RS[i] = RSg[i];
    }
  }
  const int L = omega + (int)m;
  for (int c = tid; c < L; c += NT) F[c] = 0;
  if (tid < 2) Hsh[tid] = 0;
  const uint32_t* pool = fp_pool + (int64_t)(j - 1) * pool_stride;
  __syncthreads();

  // ---- push: row by row; the boxes of a row have disjoint spans, so each
  // wave takes whole boxes (a strided read-max, then a strided write) and
  // one barrier per row orders the rows. The height test reads a slot that
  // no wave can touch again before every wave has read it.
  int Hw = 0;
  // footprint push: the pooled values do not depend on the frontline, so each
  // wave loads its next box's first R x 64 columns while it pushes the current
  constexpr int R = 4;
  constexpr uint32_t kEmpty = 0xFFFFFFFFu;
  uint32_t nxt[R];
  int prr = 0, pk = 0;
  auto advance = [&](bool first) {
    if (!first) pk += NW;
    else pk = nr > 0 ? RS[0] + w : 0;
    while (prr < nr && pk >= RS[prr + 1]) {
      ++prr;
      if (prr < nr) pk = RS[prr] + w;
    }
  };
  auto prefetch = [&]() {
    if (prr >= nr) return;
    const uint32_t* src = pool + X[pk];
    const int ncol = (int)(AB[pk] & 0xFFFFu) - p.gutter;
#pragma unroll
    for (int rk = 0; rk < R; ++rk) {
      const int kk = lane + rk * kWave;
      nxt[rk] = kk < ncol ? src[kk] : kEmpty;
    }
  };
  if constexpr (MODE == 2) {
    advance(true);
    prefetch();
  }
  for (int rr = 0; rr < nr; ++rr) {
    const int s0 = RS[rr], s1 = RS[rr + 1];
    const long long r = X[s0] >> lg;
    const bool right = (r % 3) != 0;
    {
      for (int k = s0 + w; k < s1; k += NW) {
        const long long Xk = X[k];
        const uint32_t ab = AB[k];
        const int a = (int)(ab & 0xFFFFu), b = (int)(ab >> 16);
        const int o = (int)(Xk - (r << lg));
        const int x = right ? L - o - a : o;
        {
          // one lane per content column; the pooled values come from k_fp_pool
          const int g = p.gutter, ncol = a - g;
          const uint32_t* src = pool + Xk;
          uint32_t keep[R];
  #pragma unroll
          for (int rk = 0; rk < R; ++rk) keep[rk] = nxt[rk];
          advance(false);
          prefetch();
          int mx = 0;
          auto rise = [&](int kk, uint32_t q) {
            if (q == kEmpty) return;
            const int dend = min(kk + 2 * g, a - 1);
            int fm = 0;
            for (int d = kk; d <= dend; ++d) fm = max(fm, F[x + d]);
            mx = max(mx, fm - (int)(q & 0xFFFFu));
          };
  #pragma unroll
          for (int rk = 0; rk < R; ++rk) rise(lane + rk * kWave, keep[rk]);
          for (int kk = lane + R * kWave; kk < ncol; kk += kWave) rise(kk, src[kk]);
          const int y = wave_max<int>(mx);
          int hv = 0;
          auto raise = [&](int kk, uint32_t q) {
            if (q == kEmpty) return;
            const int Bk = (int)(q >> 16);
            const int v = Bk == 0x7FFF ? y + b : min(y + b, y + 2 * g + Bk + 1);
            const int dend = min(kk + 2 * g, a - 1);
            for (int d = kk; d <= dend; ++d) atomicMax(&F[x + d], v);
            hv = max(hv, v);
          };
  #pragma unroll
          for (int rk = 0; rk < R; ++rk) raise(lane + rk * kWave, keep[rk]);
          for (int kk = lane + R * kWave; kk < ncol; kk += kWave) raise(kk, src[kk]);
          Hw = max(Hw, wave_max<int>(hv));
          if (lane == 0) Y[k] = y;
        }
      }
    }
    Hw = wave_max<int>(Hw);  // lane 0 publishes the wave's height
    if (lane == 0) atomicMax(&Hsh[rr & 1], Hw);
    __syncthreads();
    if (Hsh[rr & 1] > L) break;
  }
  if (tid == 0) {
    const int H = nr > 0 ? max(Hsh[0], Hsh[1]) : 0;
    tab[0] = H <= L ? 1 : 0;
    tab[1] = (int32_t)m;
    tab[2] = L;
    tab[3] = H;
    tab[4] = (int32_t)min(rows, (long long)INT_MAX);
  }
}

// Box push of one candidate per workgroup (the default packing). Everything
// the row loop reads is in LDS, so its only global accesses are the stores of
// the box positions, which no later instruction of the workgroup waits for:
//   [2 omega]  frontline F (int32)
//   [kcap]     fold position of each box of the current chunk, relative to
//              the chunk's first box (uint32: a chunk spans less than 2^32)
//   [kcap]     a | b << 16 of each box of the chunk
//   [kcap + 1] chunk-local starts of the chunk's row segments
// Frames with more than kcap charts are pushed in chunks of kcap boxes in
// order, reloaded from the fold written to global memory; a row that
// straddles two chunks is pushed as two segments (its boxes have disjoint
// spans, so the split changes nothing). Two barriers per segment (its narrow
// boxes, then its wider ones); cross-lane maxima and scans use DPP lane
// moves.
constexpr int kFoldItems = 4;  // consecutive boxes per thread in the fold
constexpr int kNarrow = 8;     // boxes up to this wide are pushed by one lane

// Dynamic LDS of the box push: frontline plus kcap boxes of 12 bytes.
constexpr int kBoxPushLds = 131072;
__host__ __device__ inline int box_kcap(int omega) {
  return ((kBoxPushLds - 8 * omega - 4) / 12) & ~63;
}

template <int NT>
__device__ __forceinline__ void k_pack_box_body(const float2* __restrict__ wh,
                                                 const FrameState* __restrict__ st, FrameParams p,
                                                 long long* __restrict__ cand_x,
                                                 uint32_t* __restrict__ cand_ab,
                                                 int32_t* __restrict__ cand_y,
                                                 int32_t* __restrict__ cand_tab, int64_t stride,
                                                 int kcap) {
  extern __shared__ int32_t F[];
  constexpr int NW = NT / kWave;
  __shared__ uint32_t shs[2][NW];
  __shared__ int32_t shm[NW], shb[NW];
  __shared__ int32_t Hsh[3];
  __shared__ long long last_x;
  __shared__ long long sh64[NW];
  __shared__ int32_t WM[2048], WW[256], LC[2][2];  // mid and wide box lists, their counts

  if (st->status != FA_OK) return;
  const int j = blockIdx.x + 1;
  const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
  const int C = st->num_charts;
  const int omega = p.omega, lg = p.log2omega;
  long long* Xg = cand_x + (int64_t)(j - 1) * stride;
  uint32_t* ABg = cand_ab + (int64_t)(j - 1) * stride;
  int32_t* Y = cand_y + (int64_t)(j - 1) * stride;
  int32_t* tab = cand_tab + (j - 1) * kCandStride;
  uint32_t* Xr = reinterpret_cast<uint32_t*>(F + 2 * omega);
  uint32_t* AB = Xr + kcap;
  int32_t* RS = reinterpret_cast<int32_t*>(AB + kcap);

  // ---- sizes, fold and overflow: kFoldItems consecutive boxes per thread, a
  // thread-local prefix, then one block scan of the thread sums; the first
  // chunk goes straight to LDS
  const float s = (float)j / (float)p.J;
  const int pad = 2 * p.gutter;
  long long run = 0;
  int mloc = INT_MIN, bad = 0;
  if (tid == 0) last_x = 0;
  // the frontline is cleared up front (its widest extent, 2 omega): the
  // fold's barriers order it before the push
  for (int c = tid; c < 2 * omega; c += NT) F[c] = 0;
  if (tid < 3) Hsh[tid] = 0;
  if (tid < 4) LC[tid >> 1][tid & 1] = 0;
  int pass = 0;
  for (int base = 0; base < C; base += kFoldItems * NT, ++pass) {
    const int i0 = base + kFoldItems * tid;
    int a[kFoldItems], b[kFoldItems];
    uint32_t own = 0;
#pragma unroll
    for (int u = 0; u < kFoldItems; ++u) {
      a[u] = b[u] = 0;
      if (i0 + u < C) {
        const float2 v = wh[i0 + u];
        a[u] = max(p.min_box, (int)ceilf(v.x * s)) + pad;
        b[u] = max(p.min_box, (int)ceilf(v.y * s)) + pad;
        if (a[u] > 2 * omega || b[u] > 2 * omega) bad = 1;  // cannot fit: m > omega or H > L
        a[u] = min(a[u], 2 * omega + 1);  // (the clamp only touches rejected candidates)
        b[u] = min(b[u], 2 * omega + 1);
      }
      own += (uint32_t)a[u];
    }
    uint32_t tot;
    const uint32_t incl = block_incl_scan_dpp<NT>(own, shs[pass & 1], &tot);
    long long Xi = run + (long long)(incl - own);
    run += tot;
    uint32_t xs[kFoldItems], abs_[kFoldItems];
#pragma unroll
    for (int u = 0; u < kFoldItems; ++u) {
      const int i = i0 + u;
      xs[u] = (uint32_t)Xi;
      abs_[u] = (uint32_t)a[u] | ((uint32_t)b[u] << 16);
      if (i < C) {
        Xg[i] = Xi;
        ABg[i] = abs_[u];
        if (i == C - 1) last_x = Xi;
        mloc = max(mloc, (int)(Xi & (long long)(omega - 1)) + a[u] - omega);
        Xi += a[u];
      }
    }
    // the first chunk to LDS, one 16-byte store per array (i0 is a multiple
    // of 4 and kcap of 64; entries past C are never read)
    if (i0 < kcap) {
      *reinterpret_cast<uint4*>(Xr + i0) = make_uint4(xs[0], xs[1], xs[2], xs[3]);
      *reinterpret_cast<uint4*>(AB + i0) = make_uint4(abs_[0], abs_[1], abs_[2], abs_[3]);
    }
  }
  {
    const int wm = wave_max_dpp(mloc), wb = wave_max_dpp(bad);
    if (lane == 0) {
      shm[w] = wm;
      shb[w] = wb;
    }
  }
  __syncthreads();
  int m = 0;
  bad = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    m = max(m, shm[k]);
    bad = max(bad, shb[k]);
  }
  if (bad) {
    // a box side above 2 omega rejects the candidate; its overflow m and row
    // count are still reported exactly, from the unclamped widths in 64 bits
    long long run2 = 0, ml = 0, lx = 0;
    for (int base = 0; base < C; base += NT) {
      const int i = base + tid;
      long long a = 0;
      if (i < C) a = max(p.min_box, (int)ceilf(wh[i].x * s)) + pad;
      long long tot;
      const long long incl = block_incl_scan<long long>(a, sh64, &tot);
      const long long Xi = run2 + incl - a;
      run2 += tot;
      if (i < C) {
        ml = max(ml, (Xi & (long long)(omega - 1)) + a - omega);
        if (i == C - 1) lx = Xi;
      }
    }
    ml = block_max<long long>(ml, sh64);
    lx = block_max<long long>(lx, sh64);
    if (tid == 0) {
      tab[0] = 0;
      tab[1] = (int32_t)min(ml, (long long)INT_MAX);
      tab[2] = (int32_t)min(ml + omega, (long long)INT_MAX);
      tab[3] = -1;
      tab[4] = (int32_t)min((lx >> lg) + 1, (long long)INT_MAX);
    }
    return;
  }
  const long long rows = C > 0 ? (last_x >> lg) + 1 : 0;
  if (m > omega) {
    if (tid == 0) {
      tab[0] = 0;
      tab[1] = m;
      tab[2] = m + omega;
      tab[3] = -1;
      tab[4] = (int32_t)min(rows, (long long)INT_MAX);
    }
    return;
  }
  const int L = omega + m;

  int Hw = 0, seg = 0;
  bool over = false;
  const int sub = lane >> 4, sl = lane & 15;
  for (int c0 = 0; c0 < C && !over; c0 += kcap) {
    const int cn = min(kcap, C - c0);
    long long xbase = 0;
    if (c0 > 0) {
      // the previous chunk's segments are done (the barrier ending the last
      // one); reload the next chunk from the fold in global memory
      xbase = Xg[c0];
      constexpr int U = 4;  // loads in flight per thread
      for (int i0 = tid; i0 < cn; i0 += U * NT) {
        long long xv[U];
        uint32_t abv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * NT;
          xv[u] = i < cn ? Xg[c0 + i] : 0;
          abv[u] = i < cn ? ABg[c0 + i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * NT;
          if (i < cn) {
            Xr[i] = (uint32_t)(xv[u] - xbase);
            AB[i] = abv[u];
          }
        }
      }
      __syncthreads();
    }
    // ---- chunk-local segment starts (first box of each row in the chunk)
    int nr = 0;
    for (int base = 0; base < cn; base += kFoldItems * NT, ++pass) {
      const int i0 = base + kFoldItems * tid;
      uint32_t fl = 0, own = 0;
      if (i0 < cn) {
        const uint4 q = *reinterpret_cast<const uint4*>(Xr + i0);
        const uint32_t xv[kFoldItems + 1] = {i0 > 0 ? Xr[i0 - 1] : 0u, q.x, q.y, q.z, q.w};
#pragma unroll
        for (int u = 0; u < kFoldItems; ++u) {
          const int i = i0 + u;
          const bool f =
              i < cn && (i == 0 || ((xbase + xv[u + 1]) >> lg) != ((xbase + xv[u]) >> lg));
          fl |= (uint32_t)f << u;
          own += f;
        }
      }
      uint32_t tot;
      int at = nr + (int)(block_incl_scan_dpp<NT>(own, shs[pass & 1], &tot) - own);
#pragma unroll
      for (int u = 0; u < kFoldItems; ++u)
        if (fl >> u & 1u) RS[at++] = i0 + u;
      nr += (int)tot;
    }
    if (tid == 0) RS[nr] = cn;
    __syncthreads();

    // ---- push, segment by segment, in two phases. A: the threads take the
    // segment's boxes in order; a box at most kNarrow columns wide is pushed
    // by its own lane, the others go to a list of mid boxes (up to 64
    // columns) or of wide ones. B (after a barrier): the mid boxes four per
    // wave step, 16 lanes each; the wide boxes one per wave. Boxes of a row
    // have disjoint spans, so the order inside a segment changes nothing.
    // Bounds of the lists: a row's boxes lie in L <= 2 omega <= 16384
    // columns, so at most 1820 are wider than 8 and 252 wider than 64.
    int s0 = 0, s1 = nr > 0 ? RS[1] : 0;
    long long r = nr > 0 ? (xbase + Xr[0]) >> lg : 0;
    for (int rr = 0; rr < nr; ++rr, ++seg) {
      // next segment: its end and its row
      const int s1n = rr + 2 <= nr ? RS[rr + 2] : cn;
      const uint32_t xfirst = rr + 1 < nr ? Xr[s1] : 0u;
      const int hprev = Hsh[(seg + 2) % 3];  // the height after segment seg - 1
      const long long rbase = (r << lg) - xbase;
      const bool right = (r % 3) != 0;
      int* cnt = LC[seg & 1];
      for (int k = s0 + tid; k < s1; k += NT) {
        const uint32_t ab = AB[k];
        const int a = (int)(ab & 0xFFFFu), b = (int)(ab >> 16);
        const int o = (int)((long long)Xr[k] - rbase);
        const int x = right ? L - o - a : o;
        const bool narrow = a <= kNarrow;
        if (narrow) {
          int v[kNarrow];
#pragma unroll
          for (int c = 0; c < kNarrow; ++c) v[c] = c < a ? F[x + c] : 0;
          int mx = 0;
#pragma unroll
          for (int c = 0; c < kNarrow; ++c) mx = max(mx, v[c]);
#pragma unroll
          for (int c = 0; c < kNarrow; ++c)
            if (c < a) F[x + c] = mx + b;
          Y[c0 + k] = mx;
          Hw = max(Hw, mx + b);
        }
        const bool wide = a > kWave;
        const unsigned long long mm = __ballot(!narrow && !wide), mw = __ballot(wide);
        const unsigned long long below = lanes_below();
        int bm = 0, bw = 0;
        if (lane == __ffsll((long long)__ballot(true)) - 1) {
          if (mm) bm = atomicAdd(&cnt[0], __popcll(mm));
          if (mw) bw = atomicAdd(&cnt[1], __popcll(mw));
        }
        bm = __builtin_amdgcn_readfirstlane(bm);
        bw = __builtin_amdgcn_readfirstlane(bw);
        if (!narrow && !wide) WM[bm + __popcll(mm & below)] = k;
        if (wide) WW[bw + __popcll(mw & below)] = k;
      }
      __syncthreads();
      const int nm = cnt[0], nwd = cnt[1];
      if (tid == 0) {
        LC[(seg + 1) & 1][0] = 0;
        LC[(seg + 1) & 1][1] = 0;
      }
      for (int e0 = 4 * w; e0 < nm; e0 += 4 * NW) {
        const int e = e0 + sub;
        int a = 0, b = 0, x = 0, k = 0;
        if (e < nm) {
          k = WM[e];
          const uint32_t ab = AB[k];
          a = (int)(ab & 0xFFFFu);
          b = (int)(ab >> 16);
          const int o = (int)((long long)Xr[k] - rbase);
          x = right ? L - o - a : o;
        }
        int mx = 0;
        for (int c = x + sl; c < x + a; c += 16) mx = max(mx, F[c]);
        mx = row16_max(mx);
        for (int c = x + sl; c < x + a; c += 16) F[c] = mx + b;
        if (e < nm && sl == 0) Y[c0 + k] = mx;
        if (e < nm) Hw = max(Hw, mx + b);
      }
      for (int e = w; e < nwd; e += NW) {
        const int k = WW[e];
        const uint32_t ab = AB[k];
        const int a = (int)(ab & 0xFFFFu), b = (int)(ab >> 16);
        const int o = (int)((long long)Xr[k] - rbase);
        const int x = right ? L - o - a : o;
        int mx = 0;
        for (int c = x + lane; c < x + a; c += kWave) mx = max(mx, F[c]);
        const int y = wave_max_dpp(mx);
        for (int c = x + lane; c < x + a; c += kWave) F[c] = y + b;
        if (lane == 0) Y[c0 + k] = y;
        Hw = max(Hw, y + b);
      }
      const int hw = wave_max_dpp(Hw);
      if (lane == 0) atomicMax(&Hsh[seg % 3], hw);
      __syncthreads();
      // every wave read the same settled value: all leave at the same segment
      if (hprev > L) {
        over = true;
        break;
      }
      s0 = s1;
      s1 = s1n;
      r = (xbase + xfirst) >> lg;
    }
  }
  if (tid == 0) {
    const int H = C > 0 ? max(Hsh[0], max(Hsh[1], Hsh[2])) : 0;
    tab[0] = H <= L ? 1 : 0;
    tab[1] = m;
    tab[2] = L;
    tab[3] = H;
    tab[4] = (int32_t)min(rows, (long long)INT_MAX);
  }
}
template <int NT>
__global__ __launch_bounds__(NT) void k_pack_box(const float2* __restrict__ wh,
                                                 const FrameState* __restrict__ st, FrameParams p,
                                                 long long* __restrict__ cand_x,
                                                 uint32_t* __restrict__ cand_ab,
                                                 int32_t* __restrict__ cand_y,
                                                 int32_t* __restrict__ cand_tab, int64_t stride,
                                                 int kcap) {
  k_pack_box_body<NT>(wh, st, p, cand_x, cand_ab, cand_y, cand_tab, stride, kcap);
}

// Footprint push: pooled profile of every box of every candidate that its
// fold did not reject, content column k of box i at pool[X_i + k] as
// T | B << 16 (B = 0x7FFF: the box bottom; 0xFFFFFFFF: empty). One lane per
// fold position of candidate blockIdx.y + 1: the box is the last one starting
// at or before it (binary search over the fold), positions in the box's
// right gutter are skipped.
__global__ __launch_bounds__(kBlock) void k_fp_pool(
    const float2* __restrict__ wh, const FrameState* __restrict__ st, FrameParams p,
    const long long* __restrict__ cand_x, const uint32_t* __restrict__ cand_ab,
    const int32_t* __restrict__ cand_tab, int64_t stride, const int32_t* __restrict__ order,
    const int32_t* __restrict__ fp_off, const int2* __restrict__ fp_prof,
    uint32_t* __restrict__ fp_pool, int64_t pool_stride) {
  if (st->status != FA_OK) return;
  const int j = blockIdx.y + 1;
  if (cand_tab[(j - 1) * kCandStride + 3] < 0) return;
  const int C = st->num_charts;
  if (C == 0) return;
  const int J = p.J;
  const long long* X = cand_x + (int64_t)(j - 1) * stride;
  const uint32_t* AB = cand_ab + (int64_t)(j - 1) * stride;
  uint32_t* pool = fp_pool + (int64_t)(j - 1) * pool_stride;
  const long long end = X[C - 1] + (long long)(AB[C - 1] & 0xFFFFu);
  for (long long pos = (long long)blockIdx.x * kBlock + threadIdx.x; pos < end;
       pos += (long long)gridDim.x * kBlock) {
    int lo = 0, hi = C - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (X[mid] <= pos) lo = mid;
      else hi = mid - 1;
    }
    const int i = lo;
    const int kk = (int)(pos - X[i]);
    if (kk >= (int)(AB[i] & 0xFFFFu) - p.gutter) continue;
    const float2 sz = wh[i];
    const int Uc = (int)floorf(sz.x) + 1, Rc = (int)floorf(sz.y) + 1;
    const int2* pr = fp_prof + fp_off[order[i]];
    const int u0 = min(Uc - 1, max(0, (kk * J + j - 1) / j - 1));
    const int u1 = min(Uc - 1, ((kk + 1) * J + j - 1) / j - 1);
    int tmin = INT_MAX, bmax = -1;
#pragma unroll 4
    for (int u = u0; u <= u1; ++u) {
      const int2 v = pr[u];
      if (v.y >= 0) {
        tmin = min(tmin, v.x);
        bmax = max(bmax, v.y);
      }
    }
    uint32_t q = 0xFFFFFFFFu;
    if (bmax >= 0) {
      const int T = tmin * j / J;
      const int B = bmax == Rc - 1 ? 0x7FFF : min((bmax + 1) * j / J, 0x7FFF);
      q = (uint32_t)T | ((uint32_t)B << 16);
    }
    pool[pos] = q;
  }
}

// Selection and placement in one kernel: every workgroup reduces the J
// candidate records (one lane per candidate) to the largest effective scale
// j/L_j among fitting candidates (ties -> larger j), workgroup 0 publishes it,
// then every thread places one chart from the chosen candidate.
__device__ __forceinline__ bool sel_better(int j1, int L1, int j2, int L2) {
  if (j1 == 0) return false;
  if (j2 == 0) return true;
  const long long a = (long long)j1 * L2, b = (long long)j2 * L1;
  return a > b || (a == b && j1 > j2);
}

__device__ __forceinline__ void k_select_place_body(
    FrameParams p, const int32_t* __restrict__ cand_tab, FrameState* st,
    int32_t* __restrict__ cand_out, const int32_t* __restrict__ order,
    const long long* __restrict__ cand_x, const uint32_t* __restrict__ cand_ab,
    const int32_t* __restrict__ cand_y, int64_t stride, fa_chart* __restrict__ charts,
    int4* __restrict__ chart_tex) {
  __shared__ int sj, sL;
  const bool ok = st->status == FA_OK;
  const int C = st->num_charts;
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid < p.J && cand_out) {
    const int32_t* t = cand_tab + tid * kCandStride;
    int32_t* o = cand_out + 4 * tid;
    o[0] = ok ? t[0] : 0; o[1] = ok ? t[1] : 0; o[2] = ok ? t[2] : 0; o[3] = ok ? t[3] : 0;
  }
  if (!ok) return;
  if (blockIdx.x > 0 && (int64_t)blockIdx.x * kBlock >= C) return;
  if (tid < kWave) {
    int j = 0, L = 1, H = 0, rows = 0;
    if (tid < p.J) {
      const int32_t* t = cand_tab + tid * kCandStride;
      if (t[0]) { j = tid + 1; L = t[2]; H = t[3]; rows = t[4]; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const int oj = __shfl_xor(j, o, kWave), oL = __shfl_xor(L, o, kWave);
      const int oH = __shfl_xor(H, o, kWave), orows = __shfl_xor(rows, o, kWave);
      if (sel_better(oj, oL, j, L)) { j = oj; L = oL; H = oH; rows = orows; }
    }
    if (tid == 0) {
      sj = j;
      sL = L;
      if (blockIdx.x == 0) {
        st->jstar = j;
        if (!j) {
          st->status = FA_ERR_NOFIT;
        } else {
          st->layout_w = L;
          st->layout_h = H;
          st->rows = rows;
          st->s_star = (float)j / (float)p.J;
          st->q_star = (float)p.omega / (float)L;
        }
      }
    }
  }
  __syncthreads();
  const int jm = sj - 1, L = sL;
  const int i = blockIdx.x * kBlock + tid;
  if (jm < 0 || i >= C) return;
  const long long Xi = cand_x[(int64_t)jm * stride + i];
  const uint32_t ab = cand_ab[(int64_t)jm * stride + i];
  const int a = (int)(ab & 0xFFFFu), b = (int)(ab >> 16);
  const long long r = Xi >> p.log2omega;
  const int o = (int)(Xi - (r << p.log2omega));
  fa_chart& ch = charts[order[i]];
  const int x = (r % 3 == 0) ? o : L - o - a, y = cand_y[(int64_t)jm * stride + i];
  ch.x = x;
  ch.y = y;
  ch.w = a;
  ch.h = b;
  if (chart_tex) {
    // texels t whose centre lies in the box: 2 x omega <= (2t+1) L < 2 (x+w) omega
    const int64_t om = p.omega, L2 = 2 * (int64_t)L;
    chart_tex[order[i]] = make_int4(
        (int)ceil_div64(2 * (int64_t)x * om - L, L2),
        (int)ceil_div64(2 * ((int64_t)x + a) * om - L, L2) - 1,
        (int)ceil_div64(2 * (int64_t)y * om - L, L2),
        (int)ceil_div64(2 * ((int64_t)y + b) * om - L, L2) - 1);
  }
}
__global__ __launch_bounds__(kBlock) void k_select_place(
    FrameParams p, const int32_t* __restrict__ cand_tab, FrameState* st,
    int32_t* __restrict__ cand_out, const int32_t* __restrict__ order,
    const long long* __restrict__ cand_x, const uint32_t* __restrict__ cand_ab,
    const int32_t* __restrict__ cand_y, int64_t stride, fa_chart* __restrict__ charts,
    int4* __restrict__ chart_tex) {
  k_select_place_body(p, cand_tab, st, cand_out, order, cand_x, cand_ab, cand_y, stride, charts, chart_tex);
}

// ---- batched wrappers (view = blockIdx.y) --------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void k_pack_box_b(const BatchView* __restrict__ bv,
                                                   int64_t stride) {
  const BatchView& v = bv[blockIdx.y];
  k_pack_box_body<NT>(v.w.sorted_wh, v.w.state, v.p, v.w.cand_x, v.w.cand_ab, v.w.cand_y,
                      v.w.cand_tab, stride, box_kcap(v.p.omega));
}
__global__ __launch_bounds__(kBlock) void k_select_place_b(const BatchView* __restrict__ bv,
                                                           int64_t stride) {
  const BatchView& v = bv[blockIdx.y];
  k_select_place_body(v.p, v.w.cand_tab, v.w.state, v.cand_out, v.w.vals_a, v.w.cand_x,
                      v.w.cand_ab, v.w.cand_y, stride, v.charts, v.w.chart_tex);
}

// ---- packer-only entry: box sizes in, placements out ---------------------
__global__ void k_pack_state(FrameState* st, int32_t n) {
  if (threadIdx.x == 0) {
    FrameState s = {};
    s.status = FA_OK;
    s.num_charts = n;
    *st = s;
  }
}

__global__ void k_pack_prepare(const float* __restrict__ sizes, int32_t n,
                               fa_chart* __restrict__ charts, uint32_t* __restrict__ keys,
                               int32_t* __restrict__ vals, FrameState* st) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const float tw = sizes[2 * c], th = sizes[2 * c + 1];
  const float lim = 16777216.0f;  // 2^24 texels
  if (!(tw >= 0.0f && tw <= lim && th >= 0.0f && th <= lim)) {
    st->status = FA_ERR_INVALID_ARG;  // every writer stores the same value
    return;
  }
  const int rot = tw > th ? 1 : 0;
  const float bw = rot ? th : tw, bh = rot ? tw : th;
  const int key = min((int)ceilf(bh), kKeyCap);
  fa_chart& ch = charts[c];
  ch.root_tri = c;
  ch.ndc_box[0] = ch.ndc_box[1] = ch.ndc_box[2] = ch.ndc_box[3] = 0.0f;
  ch.target_w = tw;
  ch.target_h = th;
  ch.oriented_w = bw;
  ch.oriented_h = bh;
  ch.rotated = rot;
  ch.key = key;
  keys[c] = (uint32_t)(kKeyCap - key);
  vals[c] = c;
}

__global__ void k_pack_emit(int32_t n, const fa_chart* __restrict__ charts,
                            int32_t* __restrict__ out, const FrameState* __restrict__ st) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || st->status != FA_OK) return;
  const fa_chart& ch = charts[c];
  out[5 * c + 0] = ch.x;
  out[5 * c + 1] = ch.y;
  out[5 * c + 2] = ch.w;
  out[5 * c + 3] = ch.h;
  out[5 * c + 4] = ch.rotated;
}

}  // namespace

namespace {

hipError_t box_attributes() {
  const void* ks[6] = {(const void*)k_pack_box<256>,    (const void*)k_pack_box<512>,
                       (const void*)k_pack_box<1024>,   (const void*)k_pack_box_b<256>,
                       (const void*)k_pack_box_b<512>, (const void*)k_pack_box_b<1024>};
  for (const void* k : ks) {
    const hipError_t e =
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kBoxPushLds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void box_launch(const FrameParams& p, const Work& w, int block, hipStream_t st) {
  const int64_t stride = p.max_charts;
  const int kcap = box_kcap(p.omega);
  const size_t dyn = (size_t)8 * p.omega + (size_t)12 * kcap + 4;
  if (block == 1024)
    k_pack_box<1024><<<p.J, 1024, dyn, st>>>(w.sorted_wh, w.state, p, w.cand_x, w.cand_ab,
                                             w.cand_y, w.cand_tab, stride, kcap);
  else if (block == 512)
    k_pack_box<512><<<p.J, 512, dyn, st>>>(w.sorted_wh, w.state, p, w.cand_x, w.cand_ab,
                                           w.cand_y, w.cand_tab, stride, kcap);
  else
    k_pack_box<256><<<p.J, 256, dyn, st>>>(w.sorted_wh, w.state, p, w.cand_x, w.cand_ab,
                                           w.cand_y, w.cand_tab, stride, kcap);
}

template <int MODE>
hipError_t pack_attributes(int max_dyn_bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_pack<256, MODE>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, max_dyn_bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_pack<512, MODE>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, max_dyn_bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_pack<1024, MODE>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, max_dyn_bytes);
}

template <int MODE>
void pack_launch(const FrameParams& p, const Work& w, int block, size_t dyn, hipStream_t st) {
  const int64_t stride = p.max_charts;
  if (block == 1024)
    k_pack<1024, MODE><<<p.J, 1024, dyn, st>>>(w.sorted_wh, w.state, p, w.cand_x, w.cand_ab,
                                               w.cand_y, w.cand_rs, w.cand_tab, stride,
                                               w.fp_pool, p.pool_stride);
  else if (block == 512)
    k_pack<512, MODE><<<p.J, 512, dyn, st>>>(w.sorted_wh, w.state, p, w.cand_x, w.cand_ab,
                                             w.cand_y, w.cand_rs, w.cand_tab, stride, w.fp_pool,
                                             p.pool_stride);
  else
    k_pack<256, MODE><<<p.J, 256, dyn, st>>>(w.sorted_wh, w.state, p, w.cand_x, w.cand_ab,
                                             w.cand_y, w.cand_rs, w.cand_tab, stride, w.fp_pool,
                                             p.pool_stride);
}
}  // namespace

hipError_t pack_kernel_attributes(int max_frontline_bytes) {
  const int max_dyn_bytes = max_frontline_bytes + kPackLds * 16 + 4;
  hipError_t e = box_attributes();
  if (e == hipSuccess) e = pack_attributes<1>(max_dyn_bytes);
  if (e == hipSuccess) e = pack_attributes<2>(max_dyn_bytes);
  return e;
}

hipError_t launch_pack(const FrameParams& p, const Work& w, int block, bool footprint,
                       hipStream_t st) {
  const size_t dyn = (size_t)2 * p.omega * sizeof(int32_t) + (size_t)kPackLds * 16 + 4;
  if (!footprint) {
    box_launch(p, w, block, st);
    return hipGetLastError();
  }
  pack_launch<1>(p, w, block, dyn, st);
  k_fp_pool<<<dim3(32, p.J), kBlock, 0, st>>>(w.sorted_wh, w.state, p, w.cand_x, w.cand_ab,
                                              w.cand_tab, p.max_charts, w.vals_a, w.fp_off,
                                              w.fp_prof, w.fp_pool, p.pool_stride);
  pack_launch<2>(p, w, block, dyn, st);
  return hipGetLastError();
}

hipError_t launch_select_place(const FrameParams& p, const Work& w, fa_chart* charts,
                               int32_t* cand_out, hipStream_t st) {
  k_select_place<<<(unsigned)((p.max_charts + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      p, w.cand_tab, w.state, cand_out, w.vals_a, w.cand_x, w.cand_ab, w.cand_y, p.max_charts,
      charts, w.chart_tex);
  return hipGetLastError();
}

hipError_t launch_pack_prepare(const float* sizes, int32_t n, const FrameParams& p, const Work& w,
                               fa_chart* charts, hipStream_t st) {
  (void)p;
  k_pack_state<<<1, 64, 0, st>>>(w.state, n);
  if (n > 0)
    k_pack_prepare<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        sizes, n, charts, w.keys_a, w.vals_a, w.state);
  return hipGetLastError();
}

hipError_t launch_pack_emit(int32_t n, const fa_chart* charts, int32_t* placements,
                            const Work& w, hipStream_t st) {
  if (n > 0)
    k_pack_emit<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, charts, placements,
                                                                         w.state);
  return hipGetLastError();
}

hipError_t launch_pack_batched(const BatchView* dev, int n, int J, int64_t max_charts, int block,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const size_t dyn = (size_t)kBoxPushLds;  // each view sizes its chunks from its own omega
  if (block == 1024)
    k_pack_box_b<1024><<<dim3(J, n), 1024, dyn, st>>>(dev, max_charts);
  else if (block == 512)
    k_pack_box_b<512><<<dim3(J, n), 512, dyn, st>>>(dev, max_charts);
  else
    k_pack_box_b<256><<<dim3(J, n), 256, dyn, st>>>(dev, max_charts);
  k_select_place_b<<<dim3((unsigned)((max_charts + kBlock - 1) / kBlock), n), kBlock, 0, st>>>(
      dev, max_charts);
  return hipGetLastError();
}

}  // namespace fa
