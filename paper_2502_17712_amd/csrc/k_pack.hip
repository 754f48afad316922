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

// Candidates of frames with at most kPackLds charts keep their prefix sums
// and sizes in LDS next to the frontline, so the sequential row loop never
// waits on global memory.
constexpr int kPackLds = 4096;
constexpr int kRowInf = 1 << 29;  // pooled bottom that reaches the box bottom

// Pooled full-scale profile of content column k at scale j/J (false: empty).
__device__ __forceinline__ bool pool_column(const int2* __restrict__ pr, int Uc, int Rc, int k,
                                            int j, int J, int& T, int& B) {
  const int lo = min(Uc - 1, max(0, (k * J + j - 1) / j - 1));
  const int hi = min(Uc - 1, ((k + 1) * J + j - 1) / j - 1);
  int tmin = INT_MAX, bmax = -1;
  for (int u = lo; u <= hi; ++u) {
    const int2 v = pr[u];
    if (v.y >= 0) {
      tmin = min(tmin, v.x);
      bmax = max(bmax, v.y);
    }
  }
  if (bmax < 0) return false;
  T = tmin * j / J;
  B = bmax == Rc - 1 ? kRowInf : (bmax + 1) * j / J;
  return true;
}

template <int NT, bool FP>
__global__ __launch_bounds__(NT) void k_pack(const float2* __restrict__ wh,
                                             const FrameState* __restrict__ st, FrameParams p,
                                             long long* __restrict__ cand_x,
                                             uint32_t* __restrict__ cand_ab,
                                             int32_t* __restrict__ cand_y,
                                             int32_t* __restrict__ cand_rs,
                                             int32_t* __restrict__ cand_tab, int64_t stride,
                                             const int32_t* __restrict__ order,
                                             const int32_t* __restrict__ fp_off,
                                             const int2* __restrict__ fp_prof) {
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
  const bool in_lds = C <= kPackLds;
  long long* X = in_lds ? reinterpret_cast<long long*>(F + 2 * omega) : Xg;
  uint32_t* AB = in_lds ? reinterpret_cast<uint32_t*>(F + 2 * omega + 2 * kPackLds) : ABg;
  int32_t* RS = in_lds ? F + 2 * omega + 3 * kPackLds : cand_rs + (int64_t)(j - 1) * (stride + 1);
  int32_t* Y = cand_y + (int64_t)(j - 1) * stride;
  int32_t* tab = cand_tab + (j - 1) * kCandStride;
  const float s = (float)j / (float)p.J;
  const int pad = 2 * p.gutter;

  // ---- sizes, fold and overflow -------------------------------------------
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
  const long long m = block_max<long long>(mloc, sh64);
  bad = block_max<int>(bad, sh32);
  const long long rows = C > 0 ? (X[C - 1] >> lg) + 1 : 0;
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
  const int L = omega + (int)m;

  // ---- row starts: first box of every non-empty row, in order --------------
  int nr = 0;
  for (int base = 0; base < C; base += NT) {
    const int i = base + tid;
    const int first = (i < C && (i == 0 || (X[i] >> lg) != (X[i - 1] >> lg))) ? 1 : 0;
    int tot;
    const int incl = block_incl_scan<int>(first, sh32, &tot);
    if (first) RS[nr + incl - 1] = i;
    nr += tot;
  }
  if (tid == 0) RS[nr] = C;
  for (int c = tid; c < L; c += NT) F[c] = 0;
  if (tid < 2) Hsh[tid] = 0;
  __syncthreads();

  // ---- push: row by row; the boxes of a row have disjoint spans, so each
  // wave takes whole boxes (a strided read-max, then a strided write) and
  // one barrier per row orders the rows. The height test reads a slot that
  // no wave can touch again before every wave has read it.
  int Hw = 0;
  for (int rr = 0; rr < nr; ++rr) {
    const int s0 = RS[rr], s1 = RS[rr + 1];
    const long long r = X[s0] >> lg;
    const bool right = (r % 3) != 0;
    for (int k = s0 + w; k < s1; k += NW) {
      const long long Xk = X[k];
      const uint32_t ab = AB[k];
      const int a = (int)(ab & 0xFFFFu), b = (int)(ab >> 16);
      const int o = (int)(Xk - (r << lg));
      const int x = right ? L - o - a : o;
      if constexpr (!FP) {
        int mx = 0;
        for (int c = x + lane; c < x + a; c += kWave) mx = max(mx, F[c]);
        const int y = wave_max<int>(mx);
        for (int c = x + lane; c < x + a; c += kWave) F[c] = y + b;
        if (lane == 0) Y[k] = y;
        Hw = max(Hw, y + b);
      } else {
        const int g = p.gutter, ncol = a - g;
        const float2 sz = wh[k];
        const int Uc = (int)floorf(sz.x) + 1, Rc = (int)floorf(sz.y) + 1;
        const int2* pr = fp_prof + fp_off[order[k]];
        int mx = 0;
        for (int kk = lane; kk < ncol; kk += kWave) {
          int Tk, Bk;
          if (pool_column(pr, Uc, Rc, kk, j, p.J, Tk, Bk)) {
            const int dend = min(kk + 2 * g, a - 1);
            int fm = 0;
            for (int d = kk; d <= dend; ++d) fm = max(fm, F[x + d]);
            mx = max(mx, fm - Tk);
          }
        }
        const int y = wave_max<int>(mx);
        int hv = 0;
        for (int kk = lane; kk < ncol; kk += kWave) {
          int Tk, Bk;
          if (pool_column(pr, Uc, Rc, kk, j, p.J, Tk, Bk)) {
            const int v = Bk >= kRowInf ? y + b : min(y + b, y + 2 * g + Bk + 1);
            const int dend = min(kk + 2 * g, a - 1);
            for (int d = kk; d <= dend; ++d) atomicMax(&F[x + d], v);
            hv = max(hv, v);
          }
        }
        Hw = max(Hw, wave_max<int>(hv));  // lane 0 publishes the wave's height
        if (lane == 0) Y[k] = y;
      }
    }
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

__global__ __launch_bounds__(kBlock) void k_select_place(
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
template <bool FP>
hipError_t pack_attributes(int max_dyn_bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_pack<256, FP>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, max_dyn_bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_pack<512, FP>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, max_dyn_bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_pack<1024, FP>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, max_dyn_bytes);
}

template <bool FP>
void pack_launch(const FrameParams& p, const Work& w, int block, size_t dyn, hipStream_t st) {
  const int64_t stride = p.max_charts;
  if (block == 1024)
    k_pack<1024, FP><<<p.J, 1024, dyn, st>>>(w.sorted_wh, w.state, p, w.cand_x, w.cand_ab,
                                             w.cand_y, w.cand_rs, w.cand_tab, stride, w.vals_a,
                                             w.fp_off, w.fp_prof);
  else if (block == 512)
    k_pack<512, FP><<<p.J, 512, dyn, st>>>(w.sorted_wh, w.state, p, w.cand_x, w.cand_ab,
                                           w.cand_y, w.cand_rs, w.cand_tab, stride, w.vals_a,
                                           w.fp_off, w.fp_prof);
  else
    k_pack<256, FP><<<p.J, 256, dyn, st>>>(w.sorted_wh, w.state, p, w.cand_x, w.cand_ab,
                                           w.cand_y, w.cand_rs, w.cand_tab, stride, w.vals_a,
                                           w.fp_off, w.fp_prof);
}
}  // namespace

hipError_t pack_kernel_attributes(int max_frontline_bytes) {
  const int max_dyn_bytes = max_frontline_bytes + kPackLds * 16 + 4;
  const hipError_t e = pack_attributes<false>(max_dyn_bytes);
  if (e != hipSuccess) return e;
  return pack_attributes<true>(max_dyn_bytes);
}

hipError_t launch_pack(const FrameParams& p, const Work& w, int block, bool footprint,
                       hipStream_t st) {
  const size_t dyn = (size_t)2 * p.omega * sizeof(int32_t) + (size_t)kPackLds * 16 + 4;
  if (footprint) pack_launch<true>(p, w, block, dyn, st);
  else pack_launch<false>(p, w, block, dyn, st);
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

}  // namespace fa
