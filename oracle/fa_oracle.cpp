// FastAtlas per-frame atlasing: plain, slow, single-threaded CPU oracle.
//
// TEST INFRASTRUCTURE ONLY. This file is the checker the GPU library is
// compared against; the library never calls, links or loads it. It shares no
// code, header, table or constant generator with the GPU path.
//
// Arithmetic is IEEE float32 in a fixed operation order (built with
// -ffp-contract=off, no fast-math), integers are exact. float32 follows the
// paper's own implementation language (GLSL compute shaders, whose `float` is
// IEEE single precision) and is what decides every integer size below.
//
// Paper: "FastAtlas: Real-Time Compact Atlases for Texture Space Shading"
// (Vining et al., Eurographics 2025). Each function names the passage it
// follows. Where the paper is silent or ambiguous the reading taken is stated
// in the comment and listed in the design notes.
//
// Parity status per step:
//   adjacency, clip, charts, per-triangle boxes, chart frames, order, fold,
//   push, select, UV, occupancy, visibility, reuse flags, footprint profiles,
//   pooled profiles and the footprint push: pinned by independent tests
//   (brute force, closed forms, exact double clipping, invariants, an
//   independent vectorized implementation); see tests/test_oracle_*.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <queue>
#include <utility>
#include <vector>

namespace {

struct V4 { float x, y, z, w; };
struct Box { float x0, y0, x1, y1; };

enum Plane { PL = 0, PR = 1, PB = 2, PT = 3, PN = 4, PF = 5 };

// Signed distance of a clip-space point to one face of the GL clip volume
// -w <= x,y,z <= w (Sec. "Computing Bounding Boxes of Projected Visible
// Sub-Charts": points are transformed by the 4x4 perspective matrix).
float plane_dist(const V4& p, int plane) {
  switch (plane) {
    case PL: return p.w + p.x;
    case PR: return p.w - p.x;
    case PB: return p.w + p.y;
    case PT: return p.w - p.y;
    case PN: return p.w + p.z;
    default: return p.w - p.z;
  }
}

// Sutherland-Hodgman against a single plane. Clipping a triangle against one
// plane yields a triangle or a quad (Sec. bounding boxes: "clipping against
// one plane produces either triangles or quads"). Edges are walked
// c0->c1, c1->c2, c2->c0; an intersection is computed from the inside end A
// towards the outside end B.
int clip_one_plane(const V4* in, int n, int plane, V4* out) {
  int k = 0;
  for (int i = 0; i < n; ++i) {
    const V4& S = in[i];
    const V4& E = in[(i + 1) % n];
    float dS = plane_dist(S, plane);
    float dE = plane_dist(E, plane);
    bool inS = dS >= 0.0f, inE = dE >= 0.0f;
    if (inS != inE) {
      const V4& A = inS ? S : E;
      const V4& B = inS ? E : S;
      float dA = inS ? dS : dE;
      float dB = inS ? dE : dS;
      float t = dA / (dA - dB);
      V4 P;
      P.x = A.x + t * (B.x - A.x);
      P.y = A.y + t * (B.y - A.y);
      P.z = A.z + t * (B.z - A.z);
      P.w = A.w + t * (B.w - A.w);
      out[k++] = P;
    }
    if (inE) out[k++] = E;
  }
  return k;
}

// Blinn's conservative screen coverage: clamp x and y of every vertex to
// [-w, w], divide by w, take the bounding box. A vertex with w <= 0 makes the
// estimate the whole screen [-1,1]^2.
Box blinn(const V4* p, int n) {
  for (int i = 0; i < n; ++i)
    if (!(p[i].w > 0.0f)) return Box{-1.0f, -1.0f, 1.0f, 1.0f};
  Box b{0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    float nx = std::fmin(std::fmax(p[i].x, -p[i].w), p[i].w) / p[i].w;
    float ny = std::fmin(std::fmax(p[i].y, -p[i].w), p[i].w) / p[i].w;
    if (i == 0) { b.x0 = b.x1 = nx; b.y0 = b.y1 = ny; continue; }
    b.x0 = std::fmin(b.x0, nx); b.x1 = std::fmax(b.x1, nx);
    b.y0 = std::fmin(b.y0, ny); b.y1 = std::fmax(b.y1, ny);
  }
  return b;
}

float box_area(const Box& b) { return (b.x1 - b.x0) * (b.y1 - b.y0); }

// Per-triangle conservative NDC box of the visible part of one triangle.
// Clip against the near plane when the triangle crosses it, otherwise against
// the frustum plane whose clip shrinks the box most (strict <, planes tried in
// the order left, right, bottom, top, far), then apply Blinn.
// Returns false when the triangle lies entirely outside one plane.
bool triangle_box(const V4 c[3], bool side_clip, Box* out) {
  float d[6][3];
  for (int p = 0; p < 6; ++p)
    for (int k = 0; k < 3; ++k) d[p][k] = plane_dist(c[k], p);
  bool straddle[6];
  for (int p = 0; p < 6; ++p) {
    if (d[p][0] < 0.0f && d[p][1] < 0.0f && d[p][2] < 0.0f) return false;
    straddle[p] = d[p][0] < 0.0f || d[p][1] < 0.0f || d[p][2] < 0.0f;
  }
  V4 poly[4];
  if (straddle[PN]) {
    int n = clip_one_plane(c, 3, PN, poly);
    *out = blinn(poly, n);
    return true;
  }
  Box best = blinn(c, 3);
  if (side_clip) {
    const int order[5] = {PL, PR, PB, PT, PF};
    for (int q = 0; q < 5; ++q) {
      int p = order[q];
      if (!straddle[p]) continue;
      int n = clip_one_plane(c, 3, p, poly);
      Box bp = blinn(poly, n);
      if (box_area(bp) < box_area(best)) best = bp;
    }
  }
  *out = best;
  return true;
}

int64_t floor_div(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

V4 load_clip(const float* clip, int64_t v) {
  return V4{clip[4 * v + 0], clip[4 * v + 1], clip[4 * v + 2], clip[4 * v + 3]};
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// O1  clip transform: clip_v = M * (x, y, z, 1) with M row-major, each row
// summed left to right (Sec. bounding boxes, the p^p = P p^h product).
// ---------------------------------------------------------------------------
void oracle_clip(const float* pos, int64_t V, const float* M, float* clip) {
  for (int64_t v = 0; v < V; ++v) {
    float x = pos[3 * v], y = pos[3 * v + 1], z = pos[3 * v + 2];
    for (int i = 0; i < 4; ++i)
      clip[4 * v + i] = ((M[4 * i] * x + M[4 * i + 1] * y) + M[4 * i + 2] * z) + M[4 * i + 3];
  }
}

// ---------------------------------------------------------------------------
// O2  triangle adjacency (the twin relation of the half-edge structure in the
// data-structure table). Half-edge h = 3t+e joins idx[t][e] -> idx[t][(e+1)%3].
// Non-degenerate half-edges are sorted by (undirected edge key, h); within a
// run of equal keys each half-edge points at the triangle of the next
// half-edge of the run, cyclically. Runs of length 1 and degenerate edges -> -1.
// ---------------------------------------------------------------------------
void oracle_adjacency(const int32_t* idx, int64_t T, int32_t* nbr) {
  std::vector<std::pair<uint64_t, int64_t>> he;
  he.reserve(3 * T);
  for (int64_t t = 0; t < T; ++t)
    for (int e = 0; e < 3; ++e) {
      uint32_t a = (uint32_t)idx[3 * t + e], b = (uint32_t)idx[3 * t + (e + 1) % 3];
      nbr[3 * t + e] = -1;
      if (a == b) continue;
      uint64_t key = ((uint64_t)std::min(a, b) << 32) | (uint64_t)std::max(a, b);
      he.push_back({key, 3 * t + e});
    }
  std::sort(he.begin(), he.end());
  size_t i = 0;
  while (i < he.size()) {
    size_t j = i;
    while (j < he.size() && he[j].first == he[i].first) ++j;
    if (j - i >= 2)
      for (size_t k = i; k < j; ++k) {
        size_t nx = (k + 1 < j) ? k + 1 : i;
        nbr[he[k].second] = (int32_t)(he[nx].second / 3);
      }
    i = j;
  }
}

// ---------------------------------------------------------------------------
// O3  charts (Sec. "Chart Computation"; Appendix "GPU Union Find", Alg. 1).
// A chart is a connected component of the visible triangles. Alg. 1 first
// joins triangles across shared edges, then merges charts that share a vertex
// so that every vertex belongs to exactly one chart; its final result is the
// component structure of "shares at least one vertex index". This function
// computes that by breadth-first search. Labels are component minima, chart
// indices ascend with the label. Invisible triangles and unused vertices: -1.
// `roots` receives the label (root triangle) of each chart.
// ---------------------------------------------------------------------------
int64_t oracle_charts(const int32_t* idx, int64_t T, int64_t V, const uint8_t* vis,
                      int32_t* chart_of_tri, int32_t* chart_of_vert, int32_t* roots) {
  std::vector<int64_t> start(V + 1, 0);
  for (int64_t t = 0; t < T; ++t)
    if (vis[t])
      for (int e = 0; e < 3; ++e) start[idx[3 * t + e] + 1]++;
  for (int64_t v = 0; v < V; ++v) start[v + 1] += start[v];
  std::vector<int64_t> fill(start.begin(), start.end() - 1);
  std::vector<int32_t> inc(start[V]);
  for (int64_t t = 0; t < T; ++t)
    if (vis[t])
      for (int e = 0; e < 3; ++e) inc[fill[idx[3 * t + e]]++] = (int32_t)t;
  for (int64_t t = 0; t < T; ++t) chart_of_tri[t] = -1;
  for (int64_t v = 0; v < V; ++v) chart_of_vert[v] = -1;
  int64_t C = 0;
  std::queue<int64_t> q;
  for (int64_t s = 0; s < T; ++s) {
    if (!vis[s] || chart_of_tri[s] >= 0) continue;
    roots[C] = (int32_t)s;  // first unvisited visible triangle = component minimum
    chart_of_tri[s] = (int32_t)C;
    q.push(s);
    while (!q.empty()) {
      int64_t t = q.front();
      q.pop();
      for (int e = 0; e < 3; ++e) {
        int32_t v = idx[3 * t + e];
        chart_of_vert[v] = (int32_t)C;
        for (int64_t k = start[v]; k < start[v + 1]; ++k) {
          int32_t u = inc[k];
          if (chart_of_tri[u] < 0) { chart_of_tri[u] = (int32_t)C; q.push(u); }
        }
      }
    }
    ++C;
  }
  return C;
}

// ---------------------------------------------------------------------------
// O3' edge-connected charts (the variant that stops after the first joining
// step of Sec. "Chart Computation": visible triangles are joined across shared
// edges only, without the vertex merge of the appendix). Two triangles share
// an undirected edge iff they share two distinct vertex indices. Components
// are found by breadth-first search over an edge -> triangles table; labels
// are component minima and chart indices ascend with the label, as in O3. A
// vertex may now lie in several charts, so its UV is per corner (O9');
// chart_of_vert[v] is the smallest chart index among the visible triangles
// using v (-1 if none).
// ---------------------------------------------------------------------------
int64_t oracle_charts_edge(const int32_t* idx, int64_t T, int64_t V, const uint8_t* vis,
                           int32_t* chart_of_tri, int32_t* chart_of_vert, int32_t* roots) {
  std::vector<std::pair<uint64_t, int32_t>> edges;  // (undirected edge key, triangle)
  for (int64_t t = 0; t < T; ++t) {
    if (!vis[t]) continue;
    for (int e = 0; e < 3; ++e) {
      uint32_t a = (uint32_t)idx[3 * t + e], b = (uint32_t)idx[3 * t + (e + 1) % 3];
      if (a == b) continue;
      uint64_t key = ((uint64_t)std::min(a, b) << 32) | (uint64_t)std::max(a, b);
      edges.push_back({key, (int32_t)t});
    }
  }
  std::sort(edges.begin(), edges.end());
  // triangles of one edge are a contiguous run; each triangle lists the runs
  // of its edges
  std::vector<std::vector<std::pair<size_t, size_t>>> runs_of(T);
  for (size_t i = 0; i < edges.size();) {
    size_t j = i;
    while (j < edges.size() && edges[j].first == edges[i].first) ++j;
    for (size_t k = i; k < j; ++k) runs_of[edges[k].second].push_back({i, j});
    i = j;
  }
  for (int64_t t = 0; t < T; ++t) chart_of_tri[t] = -1;
  for (int64_t v = 0; v < V; ++v) chart_of_vert[v] = -1;
  int64_t C = 0;
  std::queue<int64_t> q;
  for (int64_t s = 0; s < T; ++s) {
    if (!vis[s] || chart_of_tri[s] >= 0) continue;
    roots[C] = (int32_t)s;
    chart_of_tri[s] = (int32_t)C;
    q.push(s);
    while (!q.empty()) {
      int64_t t = q.front();
      q.pop();
      for (const auto& r : runs_of[t])
        for (size_t k = r.first; k < r.second; ++k) {
          int32_t u = edges[k].second;
          if (chart_of_tri[u] < 0) { chart_of_tri[u] = (int32_t)C; q.push(u); }
        }
    }
    ++C;
  }
  for (int64_t t = 0; t < T; ++t) {
    if (chart_of_tri[t] < 0) continue;
    for (int e = 0; e < 3; ++e) {
      int32_t& cv = chart_of_vert[idx[3 * t + e]];
      if (cv < 0 || chart_of_tri[t] < cv) cv = chart_of_tri[t];
    }
  }
  return C;
}

// ---------------------------------------------------------------------------
// O4  per-triangle boxes (Sec. bounding boxes; Appendix "Bounding Box
// Computation Alternatives"). box[t] = (x0, y0, x1, y1) in NDC; nonempty[t]=0
// for invisible triangles and triangles entirely outside one clip plane.
// ---------------------------------------------------------------------------
void oracle_triangle_boxes(const float* clip, const int32_t* idx, const uint8_t* vis, int64_t T,
                           int side_clip, float* box, uint8_t* nonempty) {
  for (int64_t t = 0; t < T; ++t) {
    nonempty[t] = 0;
    box[4 * t] = box[4 * t + 1] = box[4 * t + 2] = box[4 * t + 3] = 0.0f;
    if (!vis[t]) continue;
    V4 c[3] = {load_clip(clip, idx[3 * t]), load_clip(clip, idx[3 * t + 1]),
               load_clip(clip, idx[3 * t + 2])};
    Box b;
    if (!triangle_box(c, side_clip != 0, &b)) continue;
    nonempty[t] = 1;
    box[4 * t] = b.x0; box[4 * t + 1] = b.y0; box[4 * t + 2] = b.x1; box[4 * t + 3] = b.y1;
  }
}

// The polygon O4 (ii), O10 and FP1 use for a triangle that crosses the near
// plane: the triangle (clip coordinates, 3 x xyzw) clipped against w + z >= 0
// by clip_one_plane. Returns the vertex count (0, 3 or 4) and writes the
// vertices to poly (4 x xyzw).
int32_t oracle_near_polygon(const float* tri, float* poly) {
  V4 c[3] = {load_clip(tri, 0), load_clip(tri, 1), load_clip(tri, 2)};
  V4 p[4];
  int n = clip_one_plane(c, 3, PN, p);
  for (int k = 0; k < n; ++k) {
    poly[4 * k] = p[k].x; poly[4 * k + 1] = p[k].y; poly[4 * k + 2] = p[k].z; poly[4 * k + 3] = p[k].w;
  }
  return n;
}

// ---------------------------------------------------------------------------
// O5  chart frame and target size. The chart box is the union of its
// triangles' boxes (all empty -> zero box); the viewport transform maps NDC
// width 2 to the screen size (Sec. bounding boxes, last paragraph), the rate
// multiplies the pixel size (Sec. fixed shading rate), boxes are oriented to
// be at least as tall as wide (Sec. "Box Ordering"), and the ordering key is
// the integer height, capped at max_H - 1 = 8191.
// ---------------------------------------------------------------------------
void oracle_chart_frames(const float* box, const uint8_t* nonempty, const int32_t* chart_of_tri,
                         int64_t T, int64_t C, int32_t W, int32_t H, float rate,
                         float* frame /*[C][4]*/, float* target /*[C][2] tw, th*/,
                         float* oriented /*[C][2] bw, bh*/, int32_t* rotated, int32_t* key) {
  std::vector<uint8_t> has(C, 0);
  for (int64_t t = 0; t < T; ++t) {
    if (!nonempty[t]) continue;
    int64_t c = chart_of_tri[t];
    const float* b = box + 4 * t;
    float* f = frame + 4 * c;
    if (!has[c]) { f[0] = b[0]; f[1] = b[1]; f[2] = b[2]; f[3] = b[3]; has[c] = 1; continue; }
    f[0] = std::fmin(f[0], b[0]); f[1] = std::fmin(f[1], b[1]);
    f[2] = std::fmax(f[2], b[2]); f[3] = std::fmax(f[3], b[3]);
  }
  float halfW = 0.5f * (float)W, halfH = 0.5f * (float)H;
  for (int64_t c = 0; c < C; ++c) {
    float* f = frame + 4 * c;
    if (!has[c]) f[0] = f[1] = f[2] = f[3] = 0.0f;
    for (int k = 0; k < 4; ++k) f[k] = f[k] + 0.0f;  // -0 -> +0
    float tw = ((f[2] - f[0]) * halfW) * rate;
    float th = ((f[3] - f[1]) * halfH) * rate;
    target[2 * c] = tw;
    target[2 * c + 1] = th;
    int rot = tw > th ? 1 : 0;
    rotated[c] = rot;
    float bw = rot ? th : tw, bh = rot ? tw : th;
    oriented[2 * c] = bw;
    oriented[2 * c + 1] = bh;
    int k = (int)std::ceil(bh);
    key[c] = k < 8191 ? k : 8191;
  }
}

// ---------------------------------------------------------------------------
// O6  deterministic order (Sec. "Box Ordering via Cuckoo Hashing"): height
// descending, ties by the chart's lowest triangle index ascending (= chart
// index, since chart indices ascend with the root triangle).
// ---------------------------------------------------------------------------
void oracle_order(const int32_t* key, int64_t C, int32_t* order) {
  std::vector<int32_t> o(C);
  std::iota(o.begin(), o.end(), 0);
  std::stable_sort(o.begin(), o.end(), [&](int32_t a, int32_t b) { return key[a] > key[b]; });
  for (int64_t i = 0; i < C; ++i) order[i] = o[i];
}

// ---------------------------------------------------------------------------
// O7  one candidate scale j/J (Sec. "Parallel Atlas and Scale Factor
// Computation", Sec. "Box Packing"). Inputs are the oriented sizes in sorted
// order. Sizes: ceil at the candidate scale, minimum m_min, plus a gutter g on
// each side. Fold: exclusive prefix sum of widths; high bits = row, low bits =
// offset (omega is a power of two). Overflow m = largest excess over omega;
// layout width L = omega + m (rows are later rescaled by omega/L). Rows r with
// r mod 3 == 0 run left to right, the other two of every three run right to
// left. Push: advancing frontline, row by row: a box rises to the highest
// frontline value under its span, then raises that span by its height.
// out = {fit, m, L, H, rows}. fit iff m <= omega and H <= L.
// ---------------------------------------------------------------------------
void oracle_candidate(const float* sbw, const float* sbh, int64_t C, int32_t j, int32_t J,
                      int32_t omega, int32_t gutter, int32_t min_box,
                      int32_t* x, int32_t* y, int32_t* a, int32_t* b, int64_t* out) {
  float s = (float)j / (float)J;
  int log2w = 0;
  while ((1 << log2w) < omega) ++log2w;
  std::vector<int64_t> X(C), row(C), off(C);
  int64_t run = 0, m = 0;
  for (int64_t i = 0; i < C; ++i) {
    int wi = (int)std::ceil(sbw[i] * s);
    int hi = (int)std::ceil(sbh[i] * s);
    a[i] = std::max(min_box, wi) + 2 * gutter;
    b[i] = std::max(min_box, hi) + 2 * gutter;
    X[i] = run;
    run += a[i];
    row[i] = X[i] >> log2w;
    off[i] = X[i] & (int64_t)(omega - 1);
    m = std::max(m, off[i] + a[i] - omega);
  }
  int64_t L = omega + m;
  int64_t rows = C ? row[C - 1] + 1 : 0;
  out[1] = m;
  out[2] = L;
  out[4] = rows;
  if (m > omega) {  // wider than the frontline can hold: reject
    out[0] = 0;
    out[3] = -1;
    for (int64_t i = 0; i < C; ++i) x[i] = y[i] = 0;
    return;
  }
  for (int64_t i = 0; i < C; ++i)
    x[i] = (int32_t)((row[i] % 3 == 0) ? off[i] : L - off[i] - a[i]);
  std::vector<int64_t> F(L, 0);
  int64_t Hmax = 0;
  int64_t i = 0;
  while (i < C) {
    int64_t e = i;
    while (e < C && row[e] == row[i]) ++e;
    for (int64_t k = i; k < e; ++k) {  // all reads of the row first
      int64_t top = 0;
      for (int64_t col = x[k]; col < x[k] + a[k]; ++col) top = std::max(top, F[col]);
      y[k] = (int32_t)top;
    }
    for (int64_t k = i; k < e; ++k) {  // then the row's writes
      for (int64_t col = x[k]; col < x[k] + a[k]; ++col) F[col] = y[k] + b[k];
      Hmax = std::max(Hmax, (int64_t)y[k] + b[k]);
    }
    i = e;
  }
  out[3] = Hmax;
  out[0] = Hmax <= L ? 1 : 0;
}

// ---------------------------------------------------------------------------
// O8  scale selection: among fitting candidates the largest effective scale
// (j/J) * omega/L_j, compared exactly as j*L_k vs k*L_j; ties -> larger j.
// cand[j-1] = {fit, m, L, H, rows}. Returns j* or 0 when nothing fits.
// ---------------------------------------------------------------------------
int32_t oracle_select(const int64_t* cand, int32_t J) {
  int32_t best = 0;
  int64_t bestL = 1;
  for (int32_t j = 1; j <= J; ++j) {
    const int64_t* c = cand + 5 * (j - 1);
    if (!c[0]) continue;
    if (best == 0 || (int64_t)j * bestL >= (int64_t)best * c[2]) { best = j; bestL = c[2]; }
  }
  return best;
}

// ---------------------------------------------------------------------------
// O9  chart -> atlas map (Appendix "Shading and Rasterization": scale by S,
// then a per-chart rigid map from the chart's NDC box to its atlas box).
// Atlas texels, origin top-left, v down (image rows follow -NDC y); a rotated
// chart turns by +90 degrees: (lx, ly) = (py, tw - px).
// ---------------------------------------------------------------------------
struct ChartMap {
  float x0, y1, tw, halfW, halfH, rate, s, q, ox, oy;
  int rot;
};

static inline void map_point(const ChartMap& cm, float X, float Y, float w, float* u, float* v) {
  float nx = X / w, ny = Y / w;
  float px = ((nx - cm.x0) * cm.halfW) * cm.rate;
  float py = ((cm.y1 - ny) * cm.halfH) * cm.rate;
  float lx = cm.rot ? py : px;
  float ly = cm.rot ? (cm.tw - px) : py;
  *u = (cm.ox + lx * cm.s) * cm.q;
  *v = (cm.oy + ly * cm.s) * cm.q;
}

static ChartMap chart_map(const float* frame, const float* target, const int32_t* rotated,
                          const int32_t* px, const int32_t* py, int64_t c, int32_t W, int32_t H,
                          float rate, float s, float q, int32_t gutter) {
  ChartMap cm;
  cm.x0 = frame[4 * c];
  cm.y1 = frame[4 * c + 3];
  cm.tw = target[2 * c];
  cm.halfW = 0.5f * (float)W;
  cm.halfH = 0.5f * (float)H;
  cm.rate = rate;
  cm.s = s;
  cm.q = q;
  cm.ox = (float)(px[c] + gutter);
  cm.oy = (float)(py[c] + gutter);
  cm.rot = rotated[c];
  return cm;
}

// place_x/place_y: per-chart layout position (indexed by chart, not by rank).
void oracle_uv(const float* clip, int64_t V, const int32_t* chart_of_vert, const float* frame,
               const float* target, const int32_t* rotated, const int32_t* place_x,
               const int32_t* place_y, int32_t W, int32_t H, float rate, int32_t jstar, int32_t J,
               int32_t omega, int64_t L, int32_t gutter, float* uv) {
  float s = (float)jstar / (float)J;
  float q = (float)omega / (float)L;
  for (int64_t v = 0; v < V; ++v) {
    int32_t c = chart_of_vert[v];
    V4 p = load_clip(clip, v);
    if (c < 0 || !(p.w > 0.0f)) { uv[2 * v] = uv[2 * v + 1] = NAN; continue; }
    ChartMap cm = chart_map(frame, target, rotated, place_x, place_y, c, W, H, rate, s, q, gutter);
    map_point(cm, p.x, p.y, p.w, &uv[2 * v], &uv[2 * v + 1]);
  }
}

// O9' per-corner UVs (edge-connected charts): corner k of triangle t is vertex
// idx[3t+k] mapped through the chart of t, the same map as O9; NaN for
// invisible triangles and corners with w <= 0. uv is [T][3][2].
void oracle_uv_corners(const float* clip, const int32_t* idx, int64_t T,
                       const int32_t* chart_of_tri, const float* frame, const float* target,
                       const int32_t* rotated, const int32_t* place_x, const int32_t* place_y,
                       int32_t W, int32_t H, float rate, int32_t jstar, int32_t J, int32_t omega,
                       int64_t L, int32_t gutter, float* uv) {
  float s = (float)jstar / (float)J;
  float q = (float)omega / (float)L;
  for (int64_t t = 0; t < T; ++t) {
    int32_t c = chart_of_tri[t];
    for (int k = 0; k < 3; ++k) {
      float* o = uv + 2 * (3 * t + k);
      V4 p = load_clip(clip, idx[3 * t + k]);
      if (c < 0 || !(p.w > 0.0f)) { o[0] = o[1] = NAN; continue; }
      ChartMap cm = chart_map(frame, target, rotated, place_x, place_y, c, W, H, rate, s, q, gutter);
      map_point(cm, p.x, p.y, p.w, &o[0], &o[1]);
    }
  }
}

// ---------------------------------------------------------------------------
// O10 atlas occupancy (not defined by the paper; the footprint each chart
// claims in the atlas). occ[ty][tx] = c iff the texel centre lies in chart
// c's placed box (exact integer test in layout space, box includes the gutter)
// and in one of c's visible triangles mapped through O9, near-clipped when the
// triangle crosses the near plane, snapped to 1/256 texel (round to nearest
// even, clamped to +-2^28), fan-triangulated from its first vertex, edges
// inclusive. Triangles with an empty box in O4 claim nothing.
// Returns the number of occupied texels; `conflicts` (optional) counts texel
// claims by a second chart (none when the packing keeps footprints apart).
// ---------------------------------------------------------------------------
int64_t oracle_occupancy(const float* clip, const int32_t* idx, const uint8_t* nonempty,
                         const int32_t* chart_of_tri, int64_t T, const float* frame,
                         const float* target, const int32_t* rotated, const int32_t* place_x,
                         const int32_t* place_y, const int32_t* box_a, const int32_t* box_b,
                         int32_t W, int32_t H, float rate, int32_t jstar, int32_t J, int32_t omega,
                         int64_t L, int32_t gutter, int32_t* occ, int64_t* conflicts) {
  const int64_t N = (int64_t)omega * omega;
  if (conflicts) *conflicts = 0;
  for (int64_t i = 0; i < N; ++i) occ[i] = -1;
  float s = (float)jstar / (float)J;
  float q = (float)omega / (float)L;
  const float lim = 268435456.0f;  // 2^28
  for (int64_t t = 0; t < T; ++t) {
    if (!nonempty[t]) continue;
    int32_t c = chart_of_tri[t];
    V4 tri[3] = {load_clip(clip, idx[3 * t]), load_clip(clip, idx[3 * t + 1]),
                 load_clip(clip, idx[3 * t + 2])};
    V4 poly[4];
    int n = 3;
    bool cross_near = plane_dist(tri[0], PN) < 0.0f || plane_dist(tri[1], PN) < 0.0f ||
                      plane_dist(tri[2], PN) < 0.0f;
    if (cross_near) n = clip_one_plane(tri, 3, PN, poly);
    else for (int k = 0; k < 3; ++k) poly[k] = tri[k];
    bool ok = true;
    for (int k = 0; k < n; ++k) ok = ok && poly[k].w > 0.0f;
    if (!ok) continue;
    ChartMap cm = chart_map(frame, target, rotated, place_x, place_y, c, W, H, rate, s, q, gutter);
    int64_t U[4], Vv[4];
    for (int k = 0; k < n; ++k) {
      float u, v;
      map_point(cm, poly[k].x, poly[k].y, poly[k].w, &u, &v);
      float su = std::fmin(std::fmax(u * 256.0f, -lim), lim);
      float sv = std::fmin(std::fmax(v * 256.0f, -lim), lim);
      U[k] = (int64_t)std::rint(su);
      Vv[k] = (int64_t)std::rint(sv);
    }
    // texel range of the chart box: 2*x*omega <= (2tx+1)*L < 2*(x+a)*omega
    int64_t bx = place_x[c], by = place_y[c], ba = box_a[c], bb = box_b[c];
    for (int f = 1; f + 1 < n; ++f) {
      int64_t ax = U[0], ay = Vv[0], bxv = U[f], byv = Vv[f], cx = U[f + 1], cy = Vv[f + 1];
      int64_t area = (bxv - ax) * (cy - ay) - (byv - ay) * (cx - ax);
      if (area == 0) continue;
      int64_t umin = std::min({ax, bxv, cx}), umax = std::max({ax, bxv, cx});
      int64_t vmin = std::min({ay, byv, cy}), vmax = std::max({ay, byv, cy});
      // only texel centres inside the triangle's bounding box can be covered
      int64_t ty_lo = std::max<int64_t>(0, floor_div(vmin - 128 + 255, 256));
      int64_t ty_hi = std::min<int64_t>(omega - 1, floor_div(vmax - 128, 256));
      int64_t tx_lo = std::max<int64_t>(0, floor_div(umin - 128 + 255, 256));
      int64_t tx_hi = std::min<int64_t>(omega - 1, floor_div(umax - 128, 256));
      for (int64_t ty = ty_lo; ty <= ty_hi; ++ty) {
        int64_t pyc = 256 * ty + 128;
        if (!(2 * by * omega <= (2 * ty + 1) * L && (2 * ty + 1) * L < 2 * (by + bb) * omega)) continue;
        for (int64_t tx = tx_lo; tx <= tx_hi; ++tx) {
          int64_t pxc = 256 * tx + 128;
          if (!(2 * bx * omega <= (2 * tx + 1) * L && (2 * tx + 1) * L < 2 * (bx + ba) * omega)) continue;
          int64_t e0 = (bxv - ax) * (pyc - ay) - (byv - ay) * (pxc - ax);
          int64_t e1 = (cx - bxv) * (pyc - byv) - (cy - byv) * (pxc - bxv);
          int64_t e2 = (ax - cx) * (pyc - cy) - (ay - cy) * (pxc - cx);
          bool in = area > 0 ? (e0 >= 0 && e1 >= 0 && e2 >= 0) : (e0 <= 0 && e1 <= 0 && e2 <= 0);
          if (in) {
            int32_t& o = occ[ty * omega + tx];
            if (conflicts && o >= 0 && o != c) ++*conflicts;
            o = c;
          }
        }
      }
    }
  }
  int64_t cnt = 0;
  for (int64_t i = 0; i < N; ++i) cnt += occ[i] >= 0;
  return cnt;
}

// ---------------------------------------------------------------------------
// V   visible triangles of a view (App. "Detecting Visible Triangles": a depth
// pre-pass fills a depth buffer, a second pass tests every triangle's samples
// against it with "less or equal" and marks the triangles that pass).
// Readings: float64 throughout; a triangle is a candidate iff it faces the eye
// ((b-a) x (c-a) . (eye-a) > 0) and no clip plane has all three vertices
// outside; with coarse = k > 0 the depth buffer has (W/k) x (H/k) samples at
// pixel centres, only candidates with every w > near_w write it (their
// depth is the NDC z interpolated with edge-function weights), and such a
// triangle stays visible iff it covers no sample (it cannot be proven hidden:
// the conservative side) or one covered sample has z <= D + 1e-6; candidates
// crossing the near plane stay visible. coarse = 0: candidates only.
// ---------------------------------------------------------------------------
void oracle_visibility(const float* pos, int64_t V, const int32_t* idx, int64_t T,
                       const float* Mf, const double* eye, double near_w, int32_t W, int32_t H,
                       int32_t coarse, uint8_t* vis) {
  double M[16];
  for (int i = 0; i < 16; ++i) M[i] = (double)Mf[i];
  std::vector<double> c(4 * (size_t)V);
  for (int64_t v = 0; v < V; ++v) {
    const double x = pos[3 * v], y = pos[3 * v + 1], z = pos[3 * v + 2];
    for (int i = 0; i < 4; ++i)
      c[4 * v + i] = ((M[4 * i] * x + M[4 * i + 1] * y) + M[4 * i + 2] * z) + M[4 * i + 3];
  }
  std::vector<uint8_t> occluder(T, 0);
  for (int64_t t = 0; t < T; ++t) {
    const int64_t i0 = idx[3 * t], i1 = idx[3 * t + 1], i2 = idx[3 * t + 2];
    double a[3], b[3], d[3];
    for (int k = 0; k < 3; ++k) {
      const double q0 = pos[3 * i0 + k], q1 = pos[3 * i1 + k], q2 = pos[3 * i2 + k];
      a[k] = q1 - q0;
      b[k] = q2 - q0;
      d[k] = eye[k] - q0;
    }
    const double n0 = a[1] * b[2] - a[2] * b[1];
    const double n1 = a[2] * b[0] - a[0] * b[2];
    const double n2 = a[0] * b[1] - a[1] * b[0];
    const bool front = ((n0 * d[0] + n1 * d[1]) + n2 * d[2]) > 0.0;
    bool outside = false;
    for (int pl = 0; pl < 6 && !outside; ++pl) {
      const int k = pl / 2;  // x, y, z
      const double sgn = (pl % 2 == 0) ? 1.0 : -1.0;
      int out = 0;
      for (int e = 0; e < 3; ++e) {
        const int64_t v = idx[3 * t + e];
        const double w = c[4 * v + 3], u = c[4 * v + k];
        const double dist = sgn > 0 ? w + u : w - u;
        out += dist < 0.0;
      }
      outside = out == 3;
    }
    vis[t] = (front && !outside) ? 1 : 0;
    occluder[t] = vis[t] && c[4 * i0 + 3] > near_w && c[4 * i1 + 3] > near_w &&
                  c[4 * i2 + 3] > near_w;
  }
  if (coarse <= 0) return;
  const int64_t Wc = W / coarse, Hc = H / coarse;
  if (Wc <= 0 || Hc <= 0) return;
  std::vector<double> D((size_t)(Wc * Hc), INFINITY);
  // screen position of a vertex in coarse pixels (x right, y down) and NDC z
  auto screen = [&](int64_t v, double* X, double* Y, double* Z) {
    const double w = c[4 * v + 3];
    *X = ((c[4 * v + 0] / w) * 0.5 + 0.5) * (double)Wc;
    *Y = (0.5 - (c[4 * v + 1] / w) * 0.5) * (double)Hc;
    *Z = c[4 * v + 2] / w;
  };
  // visit every sample centre covered by triangle t: fn(pixel, depth)
  auto covered = [&](int64_t t, auto&& fn) {
    double X[3], Y[3], Z[3];
    for (int e = 0; e < 3; ++e) screen(idx[3 * t + e], &X[e], &Y[e], &Z[e]);
    const double xmin = std::min({X[0], X[1], X[2]}), xmax = std::max({X[0], X[1], X[2]});
    const double ymin = std::min({Y[0], Y[1], Y[2]}), ymax = std::max({Y[0], Y[1], Y[2]});
    const int64_t ix0 = (int64_t)std::min(std::max(std::ceil(xmin - 0.5), 0.0), (double)(Wc - 1));
    const int64_t ix1 = (int64_t)std::min(std::max(std::floor(xmax - 0.5), -1.0), (double)(Wc - 1));
    const int64_t iy0 = (int64_t)std::min(std::max(std::ceil(ymin - 0.5), 0.0), (double)(Hc - 1));
    const int64_t iy1 = (int64_t)std::min(std::max(std::floor(ymax - 0.5), -1.0), (double)(Hc - 1));
    for (int64_t py = iy0; py <= iy1; ++py) {
      for (int64_t px = ix0; px <= ix1; ++px) {
        const double cx = (double)px + 0.5, cy = (double)py + 0.5;
        const double e0 = (X[2] - X[1]) * (cy - Y[1]) - (Y[2] - Y[1]) * (cx - X[1]);
        const double e1 = (X[0] - X[2]) * (cy - Y[2]) - (Y[0] - Y[2]) * (cx - X[2]);
        const double e2 = (X[1] - X[0]) * (cy - Y[0]) - (Y[1] - Y[0]) * (cx - X[0]);
        const double area = (e0 + e1) + e2;
        const bool in = area != 0.0 && ((e0 >= 0 && e1 >= 0 && e2 >= 0) ||
                                        (e0 <= 0 && e1 <= 0 && e2 <= 0));
        if (!in) continue;
        const double z = ((e0 * Z[0] + e1 * Z[1]) + e2 * Z[2]) / area;
        fn(py * Wc + px, z);
      }
    }
  };
  for (int64_t t = 0; t < T; ++t)
    if (occluder[t]) covered(t, [&](int64_t pix, double z) { D[pix] = std::min(D[pix], z); });
  for (int64_t t = 0; t < T; ++t) {
    if (!occluder[t]) continue;
    bool any = false, pass = false;
    covered(t, [&](int64_t pix, double z) {
      any = true;
      if (z <= D[pix] + 1e-6) pass = true;
    });
    vis[t] = (!any || pass) ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// R   temporal reuse classification (Sec. "Temporal Reuse"): a key frame's
// atlas is shaded in full; a later frame re-shades only triangles that are
// newly visible (visible now, not in the key frame) or were partially visible
// in the key frame (some vertex with max(|x|, |y|) >= w in the key frame's
// clip space, i.e. part of it was off screen and never shaded). Every other
// visible triangle reuses the key frame's shading.
// flags[t] = 0 not visible now, 1 reuse, 2 shade. Clip coordinates follow O1
// (float32, fixed order). Returns the number of reused triangles.
// ---------------------------------------------------------------------------
int64_t oracle_reuse_flags(const float* pos, int64_t V, const int32_t* idx, int64_t T,
                           const float* key_M, const uint8_t* key_vis, const uint8_t* vis,
                           uint8_t* flags) {
  std::vector<float> kc(4 * (size_t)V);
  oracle_clip(pos, V, key_M, kc.data());
  int64_t reused = 0;
  for (int64_t t = 0; t < T; ++t) {
    if (!vis[t]) { flags[t] = 0; continue; }
    bool partial = false;
    for (int e = 0; e < 3; ++e) {
      const float* q = &kc[4 * (size_t)idx[3 * t + e]];
      if (std::max(std::fabs(q[0]), std::fabs(q[1])) >= q[3]) partial = true;
    }
    const bool reuse = key_vis[t] && !partial;
    flags[t] = reuse ? 1 : 2;
    reused += reuse;
  }
  return reused;
}

// ---------------------------------------------------------------------------
// FP  footprint-aware push: an extension of the box push (Sec. "Box Packing")
// for non-rectangular charts. Each chart contributes per-column profiles
// (top, bottom row) of its footprint instead of its full box, so a chart can
// rise into the empty corners under its neighbours in the frontline.
//
// FP1 full-scale profile. Chart c's footprint is measured once per frame on
// the unit grid of its chart-local layout coordinates (lx, ly) of O9 before
// the scale s and the gutter: columns u in [0, Uc), Uc = floor(bw) + 1, rows
// r in [0, Rc), Rc = floor(bh) + 1 ((bw, bh): the oriented size of O5). Every
// triangle that claims texels in O10 (non-empty box, near-clipped polygon
// with all w > 0) is mapped to (lx, ly), snapped to 1/256 (round to nearest
// even, clamped to +-2^28) and, in every column u its x-range touches, covers
// the rows floor(ymin) .. floor(ymax) of its exact extent inside the closed
// strip [u, u + 1]; the first strip extends to -inf, the last to +inf, and
// rows are clamped to [0, Rc - 1], so geometry outside the chart frame folds
// onto the frame's border cells. Exact: the extent is taken over the vertices
// inside the strip and the edges' crossings of its sides, each crossing's row
// a floor of an exact rational.
// ---------------------------------------------------------------------------
namespace {

// floor((Py + (X0 - Px) (Qy - Py) / (Qx - Px)) / 256) for Px != Qx
int64_t crossing_row(int64_t Px, int64_t Py, int64_t Qx, int64_t Qy, int64_t X0) {
  int64_t num = Py * (Qx - Px) + (X0 - Px) * (Qy - Py);
  int64_t den = Qx - Px;
  if (den < 0) { num = -num; den = -den; }
  return floor_div(num, 256 * den);
}

}  // namespace

void oracle_fine_profiles(const float* clip, const int32_t* idx, const uint8_t* nonempty,
                          const int32_t* chart_of_tri, int64_t T, const float* frame,
                          const float* target, const float* oriented, const int32_t* rotated,
                          int32_t W, int32_t H, float rate, const int64_t* foff,
                          int32_t* ft, int32_t* fb) {
  const float lim = 268435456.0f;  // 2^28
  for (int64_t t = 0; t < T; ++t) {
    if (!nonempty[t]) continue;
    const int32_t c = chart_of_tri[t];
    V4 tri[3] = {load_clip(clip, idx[3 * t]), load_clip(clip, idx[3 * t + 1]),
                 load_clip(clip, idx[3 * t + 2])};
    V4 poly[4];
    int n = 3;
    const bool cross_near = plane_dist(tri[0], PN) < 0.0f || plane_dist(tri[1], PN) < 0.0f ||
                            plane_dist(tri[2], PN) < 0.0f;
    if (cross_near) n = clip_one_plane(tri, 3, PN, poly);
    else for (int k = 0; k < 3; ++k) poly[k] = tri[k];
    bool ok = true;
    for (int k = 0; k < n; ++k) ok = ok && poly[k].w > 0.0f;
    if (!ok || n < 1) continue;
    const float x0 = frame[4 * c], y1 = frame[4 * c + 3], tw = target[2 * c];
    const float halfW = 0.5f * (float)W, halfH = 0.5f * (float)H;
    int64_t X[4], Y[4];
    for (int k = 0; k < n; ++k) {
      const float nx = poly[k].x / poly[k].w, ny = poly[k].y / poly[k].w;
      const float px = ((nx - x0) * halfW) * rate;
      const float py = ((y1 - ny) * halfH) * rate;
      const float lx = rotated[c] ? py : px;
      const float ly = rotated[c] ? (tw - px) : py;
      X[k] = (int64_t)std::rint(std::fmin(std::fmax(lx * 256.0f, -lim), lim));
      Y[k] = (int64_t)std::rint(std::fmin(std::fmax(ly * 256.0f, -lim), lim));
    }
    const int64_t Uc = (int64_t)std::floor(oriented[2 * c]) + 1;
    const int64_t Rc = (int64_t)std::floor(oriented[2 * c + 1]) + 1;
    int64_t xmin = X[0], xmax = X[0];
    for (int k = 1; k < n; ++k) { xmin = std::min(xmin, X[k]); xmax = std::max(xmax, X[k]); }
    const int64_t u0 = std::min(Uc - 1, std::max<int64_t>(0, floor_div(xmin, 256)));
    const int64_t u1 = std::min(Uc - 1, std::max<int64_t>(0, floor_div(xmax, 256)));
    for (int64_t u = u0; u <= u1; ++u) {
      const bool open_l = u == 0, open_r = u == Uc - 1;
      const int64_t sl = 256 * u, sr = 256 * (u + 1);
      int64_t rlo = INT64_MAX, rhi = INT64_MIN;
      for (int k = 0; k < n; ++k) {
        if ((open_l || X[k] >= sl) && (open_r || X[k] <= sr)) {
          const int64_t r = floor_div(Y[k], 256);
          rlo = std::min(rlo, r);
          rhi = std::max(rhi, r);
        }
      }
      for (int k = 0; k < n; ++k) {
        const int64_t Px = X[k], Py = Y[k], Qx = X[(k + 1) % n], Qy = Y[(k + 1) % n];
        if (Px == Qx) continue;
        const int64_t lo = std::min(Px, Qx), hi = std::max(Px, Qx);
        if (!open_l && lo < sl && sl < hi) {
          const int64_t r = crossing_row(Px, Py, Qx, Qy, sl);
          rlo = std::min(rlo, r);
          rhi = std::max(rhi, r);
        }
        if (!open_r && lo < sr && sr < hi) {
          const int64_t r = crossing_row(Px, Py, Qx, Qy, sr);
          rlo = std::min(rlo, r);
          rhi = std::max(rhi, r);
        }
      }
      if (rlo > rhi) continue;  // the polygon misses this strip
      rlo = std::min(Rc - 1, std::max<int64_t>(0, rlo));
      rhi = std::min(Rc - 1, std::max<int64_t>(0, rhi));
      int32_t& top = ft[foff[c] + u];
      int32_t& bot = fb[foff[c] + u];
      top = std::min<int32_t>(top, (int32_t)rlo);
      bot = std::max<int32_t>(bot, (int32_t)rhi);
    }
  }
}

// FP2 profile of one chart's box (a x b texels, gutter g >= 1) at candidate j
// of J (s = j/J), pooled from its full-scale profile (ft, fb over Uc columns,
// Rc rows; empty column: ft = INT32_MAX, fb = -1). The scaled cell of fine
// column u touches content columns floor(u s) .. floor((u + 1) s), so content
// column k pools fine columns ceil(k/s) - 1 .. ceil((k + 1)/s) - 1, clamped to
// the chart (columns past the last fine one pool the last one, which holds
// everything folded onto the frame's right border). Pooled rows: top T =
// floor(min ft * s); bottom B = floor((max fb + 1) * s), or the box bottom
// when the pooled cells reach the frame's last row (geometry folded onto the
// bottom border). Box column d = content column d - g; the gutter dilates the
// profile by g columns and rows: top[d] = min T, bot[d] = min(b - 1, 2g + max
// B) over content columns k in [d - 2g, d] with k + g < a; no non-empty k ->
// empty column (top = INT32_MAX, bottom = -1).
void oracle_pool_profile(const int32_t* ft, const int32_t* fb, int32_t Uc, int32_t Rc,
                         int32_t a, int32_t b, int32_t j, int32_t J, int32_t g, int32_t* top,
                         int32_t* bot) {
  const int64_t inf = INT64_MAX / 4;
  std::vector<int64_t> T(a), B(a);
  std::vector<char> has(a, 0);
  for (int64_t k = 0; k + g < a; ++k) {
    // ceil(k J / j) - 1 and ceil((k + 1) J / j) - 1, clamped to [0, Uc - 1]
    int64_t lo = (k * J + j - 1) / j - 1, hi = ((k + 1) * J + j - 1) / j - 1;
    lo = std::min<int64_t>(Uc - 1, std::max<int64_t>(0, lo));
    hi = std::min<int64_t>(Uc - 1, hi);
    int64_t tmin = INT64_MAX, bmax = -1;
    for (int64_t u = lo; u <= hi; ++u) {
      if (fb[u] < 0) continue;
      tmin = std::min<int64_t>(tmin, ft[u]);
      bmax = std::max<int64_t>(bmax, fb[u]);
    }
    if (bmax < 0) continue;
    has[k] = 1;
    T[k] = tmin * j / J;
    B[k] = bmax == Rc - 1 ? inf : (bmax + 1) * j / J;
  }
  for (int64_t d = 0; d < a; ++d) {
    int64_t tmin = INT64_MAX, bmax = -1;
    for (int64_t k = std::max<int64_t>(0, d - 2 * g); k <= d && k + g < a; ++k) {
      if (!has[k]) continue;
      tmin = std::min(tmin, T[k]);
      bmax = std::max(bmax, B[k]);
    }
    if (bmax < 0) {
      top[d] = INT32_MAX;
      bot[d] = -1;
    } else {
      top[d] = (int32_t)tmin;
      bot[d] = (int32_t)std::min<int64_t>(b - 1, 2 * g + bmax);
    }
  }
}

// FP3 candidate j with footprint profiles (inputs in packing order): sizes,
// fold, overflow and mirrored rows exactly as O7; a candidate with m > omega
// or a box taller than 2 omega (no layout of side L <= 2 omega holds it) is
// rejected. The push reads, per box, y = max(0, max over its non-empty
// columns of F[x+k] - top[k]), then sets F[x+k] = y + bottom[k] + 1 on those
// columns (all reads of a row before its writes). H = max F; fit iff H <= L.
void oracle_candidate_fp(const int32_t* a, const int32_t* b, const int32_t* top,
                         const int32_t* bot, const int64_t* poff, int64_t C, int32_t omega,
                         int32_t* x, int32_t* y, int64_t* out) {
  int log2w = 0;
  while ((1 << log2w) < omega) ++log2w;
  std::vector<int64_t> X(C), row(C), off(C);
  int64_t run = 0, m = 0;
  for (int64_t i = 0; i < C; ++i) {
    X[i] = run;
    run += a[i];
    row[i] = X[i] >> log2w;
    off[i] = X[i] & (int64_t)(omega - 1);
    m = std::max(m, off[i] + a[i] - omega);
  }
  const int64_t L = omega + m;
  out[1] = m;
  out[2] = L;
  out[4] = C ? row[C - 1] + 1 : 0;
  bool too_tall = false;
  for (int64_t i = 0; i < C; ++i) too_tall = too_tall || b[i] > 2 * omega;
  if (m > omega || too_tall) {
    out[0] = 0;
    out[3] = -1;
    for (int64_t i = 0; i < C; ++i) x[i] = y[i] = 0;
    return;
  }
  for (int64_t i = 0; i < C; ++i)
    x[i] = (int32_t)((row[i] % 3 == 0) ? off[i] : L - off[i] - a[i]);
  std::vector<int64_t> F(L, 0);
  int64_t i = 0;
  while (i < C) {
    int64_t e = i;
    while (e < C && row[e] == row[i]) ++e;
    for (int64_t k = i; k < e; ++k) {
      int64_t yy = 0;
      for (int q = 0; q < a[k]; ++q)
        if (bot[poff[k] + q] >= 0) yy = std::max(yy, F[x[k] + q] - top[poff[k] + q]);
      y[k] = (int32_t)yy;
    }
    for (int64_t k = i; k < e; ++k)
      for (int q = 0; q < a[k]; ++q)
        if (bot[poff[k] + q] >= 0) F[x[k] + q] = y[k] + bot[poff[k] + q] + 1;
    i = e;
  }
  int64_t Hm = 0;
  for (int64_t c = 0; c < L; ++c) Hm = std::max(Hm, F[c]);
  out[3] = Hm;
  out[0] = Hm <= L ? 1 : 0;
}

}  // extern "C"
