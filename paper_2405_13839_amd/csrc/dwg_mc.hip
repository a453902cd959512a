// The paper's own normal update (Sec. 4.3, Algorithm 1): the GWN at the nodes of a grid
// around the points, the iso-value w_bar (Eq. 6), the w_bar level set, one gradient per
// face from the cross product, and every face's gradient added to its k nearest input
// points, then normalised (Eq. 7).
//
// Grid. The octree frame (lo = bounding-box minimum, side = largest extent) cut into 2^depth
// cells per axis; a point's cell is its level-21 octree cell shifted down to `depth`. The
// evaluated cells are the cells holding points grown by `dilate` rings (inside the cube),
// sorted by Morton code; their corners are deduplicated (radix sort + scan) and placed at
// lo + c * side / 2^depth (FP64, rounded once to FP32).
// Level set: Marching Cubes (the paper's "standard Marching Cubes"). Corner index
// x + 2y + 4z; a corner is above when w > w_bar; the case of a cube is the 8-bit mask of its
// above corners. Its triangles come from a 256-case table that this file derives at compile
// time from one face rule: every face, walked counter-clockwise as seen from outside,
// contributes a segment per run of above corners, from the cut edge where the walk enters the
// run to the cut edge where it leaves (so a face with its two above corners on a diagonal
// separates them, and two cubes sharing a face draw the same segments: the surface is
// closed); the segments chain into loops, each written from its lowest edge number (edges
// numbered by their corner pair (u, v), u < v, in lexicographic order), loops in that order,
// and cut into the fan (v0, vi, vi+1). That winding makes (q1 - q0) x (q2 - q0) point away
// from the above corners. A vertex on edge (u, v): p_u + (w_bar - w_u) / (w_v - w_u)
// (p_v - p_u), FP64. At most 5 triangles per cube.
// Option (not the paper's): marching tetrahedra, each cube cut into 6 tetrahedra around
// the diagonal from corner 0 to corner 7, one per order (a, b, c) of the axes: 0, e_a,
// e_a + e_b, 7, in the order (x,y,z), (x,z,y), (y,x,z), (y,z,x), (z,x,y), (z,y,x). One lone
// inside (or outside) vertex L: the triangle of the crossings on the edges from L to the
// other three in tetrahedron order; two inside A < B, outside C < D: the quad e(A,C), e(A,D),
// e(B,D), e(B,C) split into (e(A,C), e(A,D), e(B,D)) and (e(A,C), e(B,D), e(B,C)); each turned
// away from the tetrahedron's inside vertices (q1 and q2 swapped when turned).
// Scatter. The k nearest points of each face centroid (the uniform-grid kNN) receive the
// face vector through 64-bit fixed-point atomic adds (scale 2^40 / (3 h^2), h = the cell
// size; |components| <= 3 h^2): integer sums do not depend on the order of the atomics, so
// the result is deterministic.
#include <cmath>

#include "dwg_internal.h"
#include "dwg_morton.h"

#define DWG_PROPAGATE_INT(expr) \
  do {                          \
    dwg_status s_ = (expr);     \
    if (s_ != DWG_OK) return s_; \
  } while (0)

namespace dwg {
namespace {

using morton::compact21;

__device__ __forceinline__ uint64_t morton3(int x, int y, int z) { return morton::code3(x, y, z); }

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 16384)); }

// Cell code of every point at `depth` (from the level-21 octree cell).
__global__ void k_mc_point_keys(const float* __restrict__ P, int64_t n, const double* __restrict__ frame, int depth,
                                uint64_t* __restrict__ key, int32_t* __restrict__ val) {
  const int sh = morton::kDepth - depth;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int c[3];
    morton::cell21(P, n, i, frame, c);
    key[i] = morton3(c[0] >> sh, c[1] >> sh, c[2] >> sh);
    val[i] = 0;
  }
}

// head[i] = 1 where sorted key i starts a run of equal keys below `limit`.
__global__ void k_mc_heads(const uint64_t* __restrict__ key, int64_t n, uint64_t limit, int32_t* __restrict__ head) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    head[i] = (key[i] < limit && (i == 0 || key[i] != key[i - 1])) ? 1 : 0;
}

// Compacts the run heads (off = exclusive scan of the heads).
__global__ void k_mc_compact(const uint64_t* __restrict__ key, int64_t n, uint64_t limit,
                             const int32_t* __restrict__ off, uint64_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (key[i] < limit && (i == 0 || key[i] != key[i - 1])) out[off[i]] = key[i];
}

// The (2 dil + 1)^3 neighbours of every occupied cell; outside the cube (or past the count)
// a sentinel 2^(3 depth) that sorts after every cell.
__global__ void k_mc_dilate(const uint64_t* __restrict__ occ, const int32_t* __restrict__ count, int64_t cap,
                            int depth, int dil, uint64_t* __restrict__ key, int32_t* __restrict__ val) {
  const int64_t o = *count;
  const int w = 2 * dil + 1, w3 = w * w * w;
  const int G = 1 << depth;
  const uint64_t sentinel = 1ull << (3 * depth);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < cap * w3; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t / w3;
    const int r = (int)(t % w3);
    uint64_t k = sentinel;
    if (c < o) {
      const uint64_t code = occ[c];
      const int x = compact21(code >> 2) + r % w - dil;
      const int y = compact21(code >> 1) + (r / w) % w - dil;
      const int z = compact21(code) + r / (w * w) - dil;
      if (x >= 0 && y >= 0 && z >= 0 && x < G && y < G && z < G) k = morton3(x, y, z);
    }
    key[t] = k;
    val[t] = 0;
  }
}

// Corner lattice keys of every cell: key = Morton code of the corner, val = 8 cell + k.
__global__ void k_mc_corner_keys(const uint64_t* __restrict__ cells, int64_t C, uint64_t* __restrict__ key,
                                 int32_t* __restrict__ val) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 8 * C; t += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t code = cells[t >> 3];
    const int k = (int)(t & 7);
    key[t] = morton3(compact21(code >> 2) + (k & 1), compact21(code >> 1) + ((k >> 1) & 1),
                     compact21(code) + ((k >> 2) & 1));
    val[t] = (int32_t)t;
  }
}

// Corner ids (rank of the distinct key), the cell-corner table and the corner positions.
__global__ void k_mc_corner_ids(const uint64_t* __restrict__ key, const int32_t* __restrict__ val, int64_t n8,
                                const int32_t* __restrict__ off, const double* __restrict__ frame,
                                const float* __restrict__ box, int depth, int32_t* __restrict__ cidx,
                                float* __restrict__ pos, int64_t ld) {
  // cell size = side / 2^depth, side = the largest extent of the bounding box (FP64)
  double side = (double)box[3] - (double)box[0];
  const double sy = (double)box[4] - (double)box[1], sz = (double)box[5] - (double)box[2];
  if (sy > side) side = sy;
  if (sz > side) side = sz;
  const double h = side / (double)(1 << depth);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n8; i += (int64_t)gridDim.x * blockDim.x) {
    const bool head = i == 0 || key[i] != key[i - 1];
    const int32_t id = head ? off[i] : off[i] - 1;
    cidx[val[i]] = id;
    if (head) {
      const uint64_t k = key[i];
      const int c[3] = {compact21(k >> 2), compact21(k >> 1), compact21(k)};
      for (int d = 0; d < 3; ++d) pos[d * ld + id] = (float)__dadd_rn(frame[d], __dmul_rn((double)c[d], h));
    }
  }
}

// The 6 tetrahedra of a cube (corner indices, x + 2y + 4z).
__constant__ int kTet[6][4] = {{0, 1, 3, 7}, {0, 1, 5, 7}, {0, 2, 3, 7}, {0, 2, 6, 7}, {0, 4, 5, 7}, {0, 4, 6, 7}};

struct Vec3 {
  double x, y, z;
};
__device__ __forceinline__ Vec3 lerp_cross(const Vec3& a, const Vec3& b, double wa, double wb, double iso) {
  const double t = (iso - wa) / (wb - wa);
  return Vec3{a.x + t * (b.x - a.x), a.y + t * (b.y - a.y), a.z + t * (b.z - a.z)};
}

// Triangles of one tetrahedron: returns the count (0..2) and writes them when out != null.
__device__ int tet_faces(const Vec3* p, const double* w, double iso, Vec3 (*out)[3], Vec3* vec) {
  bool in[4];
  int k = 0;
  for (int t = 0; t < 4; ++t) {
    in[t] = w[t] > iso;
    k += in[t] ? 1 : 0;
  }
  if (k == 0 || k == 4) return 0;
  if (!out) return (k == 2) ? 2 : 1;
  int nf;
  if (k == 1 || k == 3) {
    int lone = 0;
    for (int t = 0; t < 4; ++t)
      if (in[t] == (k == 1)) lone = t;
    int j = 0;
    for (int t = 0; t < 4; ++t)
      if (t != lone) out[0][j++] = lerp_cross(p[lone], p[t], w[lone], w[t], iso);
    nf = 1;
  } else {
    int ins[2], outs[2], a = 0, b = 0;
    for (int t = 0; t < 4; ++t) {
      if (in[t])
        ins[a++] = t;
      else
        outs[b++] = t;
    }
    const int A = ins[0], B = ins[1], C = outs[0], D = outs[1];
    const Vec3 eAC = lerp_cross(p[A], p[C], w[A], w[C], iso), eAD = lerp_cross(p[A], p[D], w[A], w[D], iso);
    const Vec3 eBD = lerp_cross(p[B], p[D], w[B], w[D], iso), eBC = lerp_cross(p[B], p[C], w[B], w[C], iso);
    out[0][0] = eAC, out[0][1] = eAD, out[0][2] = eBD;
    out[1][0] = eAC, out[1][1] = eBD, out[1][2] = eBC;
    nf = 2;
  }
  Vec3 cin{0, 0, 0};
  for (int t = 0; t < 4; ++t)
    if (in[t]) cin.x += p[t].x, cin.y += p[t].y, cin.z += p[t].z;
  cin.x /= k, cin.y /= k, cin.z /= k;
  for (int f = 0; f < nf; ++f) {
    const Vec3 &q0 = out[f][0], &q1 = out[f][1], &q2 = out[f][2];
    const double ux = q1.x - q0.x, uy = q1.y - q0.y, uz = q1.z - q0.z;
    const double vx = q2.x - q0.x, vy = q2.y - q0.y, vz = q2.z - q0.z;
    Vec3 c{uy * vz - uz * vy, uz * vx - ux * vz, ux * vy - uy * vx};
    const double cx = (q0.x + q1.x + q2.x) / 3.0, cy = (q0.y + q1.y + q2.y) / 3.0, cz = (q0.z + q1.z + q2.z) / 3.0;
    if (c.x * (cin.x - cx) + c.y * (cin.y - cy) + c.z * (cin.z - cz) > 0.0) {
      c = Vec3{-c.x, -c.y, -c.z};
      const Vec3 tmp = out[f][1];  // wind the triangle the way its vector points
      out[f][1] = out[f][2];
      out[f][2] = tmp;
    }
    vec[f] = c;
  }
  return nf;
}

// ---- Marching Cubes case table (built at compile time from the face rule above) ----
constexpr int kMcMaxTri = 5;
struct McTable {
  uint8_t ntri[256];
  uint8_t tri[256][3 * kMcMaxTri];  // edge numbers, three per triangle
};
// edge e joins corners kEdgeLo[e] < kEdgeHi[e]
constexpr int kEdgeLo[12] = {0, 0, 0, 1, 1, 2, 2, 3, 4, 4, 5, 6};
constexpr int kEdgeHi[12] = {1, 2, 4, 3, 5, 3, 6, 7, 5, 6, 7, 7};
// the corners of each face, counter-clockwise as seen from outside the cube
constexpr int kFaceCyc[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};

constexpr int mc_edge(int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  for (int e = 0; e < 12; ++e)
    if (kEdgeLo[e] == lo && kEdgeHi[e] == hi) return e;
  return -1;
}

constexpr McTable make_mc_table() {
  McTable t{};
  for (int c = 0; c < 256; ++c) {
    int next[12] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
    for (int f = 0; f < 6; ++f)
      for (int i = 0; i < 4; ++i) {
        const int a = kFaceCyc[f][i], b = kFaceCyc[f][(i + 1) & 3];
        if (((c >> a) & 1) || !((c >> b) & 1)) continue;  // the walk enters a run at (a, b)
        int j = (i + 1) & 3;
        while ((c >> kFaceCyc[f][(j + 1) & 3]) & 1) j = (j + 1) & 3;
        next[mc_edge(a, b)] = mc_edge(kFaceCyc[f][j], kFaceCyc[f][(j + 1) & 3]);
      }
    bool used[12] = {};
    int nt = 0;
    for (int e = 0; e < 12; ++e) {
      if (next[e] < 0 || used[e]) continue;
      int loop[12] = {}, len = 0;
      for (int x = e; !used[x]; x = next[x]) {
        used[x] = true;
        loop[len++] = x;
      }
      for (int v = 1; v + 1 < len; ++v, ++nt) {
        t.tri[c][3 * nt + 0] = (uint8_t)loop[0];
        t.tri[c][3 * nt + 1] = (uint8_t)loop[v];
        t.tri[c][3 * nt + 2] = (uint8_t)loop[v + 1];
      }
    }
    t.ntri[c] = (uint8_t)nt;
  }
  return t;
}
constexpr McTable kMcHost = make_mc_table();
static_assert(kMcHost.ntri[0] == 0 && kMcHost.ntri[255] == 0 && kMcHost.ntri[1] == 1, "table");
constexpr int mc_max_tri() {
  int m = 0;
  for (int c = 0; c < 256; ++c) m = kMcHost.ntri[c] > m ? kMcHost.ntri[c] : m;
  return m;
}
static_assert(mc_max_tri() == kMcMaxTri, "at most five triangles per cube");
__constant__ McTable kMc = kMcHost;

__device__ void load_cell(int64_t ci, const int32_t* __restrict__ cidx, const float* __restrict__ pos, int64_t ld,
                          const float* __restrict__ w, Vec3* p, double* wv) {
  for (int k = 0; k < 8; ++k) {
    const int64_t id = cidx[8 * ci + k];
    p[k] = Vec3{pos[id], pos[ld + id], pos[2 * ld + id]};
    wv[k] = w[id];
  }
}

__global__ void k_mt_count(int64_t C, const int32_t* __restrict__ cidx, const float* __restrict__ pos, int64_t ld,
                           const float* __restrict__ w, const double* __restrict__ iso_p, int32_t* __restrict__ cnt) {
  const double iso = *iso_p;
  for (int64_t ci = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ci < C; ci += (int64_t)gridDim.x * blockDim.x) {
    Vec3 p[8];
    double wv[8];
    load_cell(ci, cidx, pos, ld, w, p, wv);
    int c = 0;
    for (int t = 0; t < 6; ++t) {
      Vec3 tp[4];
      double tw[4];
      for (int j = 0; j < 4; ++j) {
        tp[j] = p[kTet[t][j]];
        tw[j] = wv[kTet[t][j]];
      }
      c += tet_faces(tp, tw, iso, nullptr, nullptr);
    }
    cnt[ci] = c;
  }
}

// Faces of every cell at off[ci]: centroids (planar [3][ldf]), vectors, and optionally the
// triangles ([F][9]: q0, q1, q2).
__global__ void k_mt_emit(int64_t C, const int32_t* __restrict__ cidx, const float* __restrict__ pos, int64_t ld,
                          const float* __restrict__ w, const double* __restrict__ iso_p,
                          const int32_t* __restrict__ off, int64_t fcap, float* __restrict__ cen, int64_t ldf,
                          float4* __restrict__ vec, float* __restrict__ tri, int64_t tcap) {
  const double iso = *iso_p;
  for (int64_t ci = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ci < C; ci += (int64_t)gridDim.x * blockDim.x) {
    Vec3 p[8];
    double wv[8];
    load_cell(ci, cidx, pos, ld, w, p, wv);
    int64_t f = off[ci];
    for (int t = 0; t < 6; ++t) {
      Vec3 tp[4];
      double tw[4];
      for (int j = 0; j < 4; ++j) {
        tp[j] = p[kTet[t][j]];
        tw[j] = wv[kTet[t][j]];
      }
      Vec3 out[2][3], v[2];
      const int nf = tet_faces(tp, tw, iso, out, v);
      for (int s = 0; s < nf; ++s, ++f) {
        if (f >= fcap) continue;
        if (cen) {
          cen[f] = (float)((out[s][0].x + out[s][1].x + out[s][2].x) / 3.0);
          cen[ldf + f] = (float)((out[s][0].y + out[s][1].y + out[s][2].y) / 3.0);
          cen[2 * ldf + f] = (float)((out[s][0].z + out[s][1].z + out[s][2].z) / 3.0);
        }
        if (vec) vec[f] = make_float4((float)v[s].x, (float)v[s].y, (float)v[s].z, 0.0f);
        if (tri && f < tcap)
          for (int q = 0; q < 3; ++q) {
            tri[9 * f + 3 * q + 0] = (float)out[s][q].x;
            tri[9 * f + 3 * q + 1] = (float)out[s][q].y;
            tri[9 * f + 3 * q + 2] = (float)out[s][q].z;
          }
      }
    }
  }
}

__device__ __forceinline__ int mc_case(const double* wv, double iso) {
  int c = 0;
  for (int k = 0; k < 8; ++k) c |= (wv[k] > iso ? 1 : 0) << k;
  return c;
}

__device__ __forceinline__ Vec3 mc_vertex(int e, const Vec3* p, const double* wv, double iso) {
  const int u = kEdgeLo[e], v = kEdgeHi[e];
  return lerp_cross(p[u], p[v], wv[u], wv[v], iso);
}

__global__ void k_mc_count(int64_t C, const int32_t* __restrict__ cidx, const float* __restrict__ w,
                           const double* __restrict__ iso_p, int32_t* __restrict__ cnt) {
  const double iso = *iso_p;
  for (int64_t ci = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ci < C; ci += (int64_t)gridDim.x * blockDim.x) {
    double wv[8];
    for (int k = 0; k < 8; ++k) wv[k] = w[cidx[8 * ci + k]];
    cnt[ci] = kMc.ntri[mc_case(wv, iso)];
  }
}

// Triangles of every cell at off[ci], in table order: centroids (planar [3][ldf]), face
// vectors (q1 - q0) x (q2 - q0), and optionally the triangles ([F][9]: q0, q1, q2).
__global__ void k_mc_emit(int64_t C, const int32_t* __restrict__ cidx, const float* __restrict__ pos, int64_t ld,
                          const float* __restrict__ w, const double* __restrict__ iso_p,
                          const int32_t* __restrict__ off, int64_t fcap, float* __restrict__ cen, int64_t ldf,
                          float4* __restrict__ vec, float* __restrict__ tri, int64_t tcap) {
  const double iso = *iso_p;
  for (int64_t ci = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ci < C; ci += (int64_t)gridDim.x * blockDim.x) {
    Vec3 p[8];
    double wv[8];
    load_cell(ci, cidx, pos, ld, w, p, wv);
    const int c = mc_case(wv, iso);
    const int nt = kMc.ntri[c];
    int64_t f = off[ci];
    for (int s = 0; s < nt; ++s, ++f) {
      if (f >= fcap) continue;
      const Vec3 q0 = mc_vertex(kMc.tri[c][3 * s], p, wv, iso), q1 = mc_vertex(kMc.tri[c][3 * s + 1], p, wv, iso),
                 q2 = mc_vertex(kMc.tri[c][3 * s + 2], p, wv, iso);
      const double ux = q1.x - q0.x, uy = q1.y - q0.y, uz = q1.z - q0.z;
      const double vx = q2.x - q0.x, vy = q2.y - q0.y, vz = q2.z - q0.z;
      if (cen) {
        cen[f] = (float)((q0.x + q1.x + q2.x) / 3.0);
        cen[ldf + f] = (float)((q0.y + q1.y + q2.y) / 3.0);
        cen[2 * ldf + f] = (float)((q0.z + q1.z + q2.z) / 3.0);
      }
      if (vec)
        vec[f] = make_float4((float)(uy * vz - uz * vy), (float)(uz * vx - ux * vz), (float)(ux * vy - uy * vx), 0.0f);
      if (tri && f < tcap) {
        const Vec3 q[3] = {q0, q1, q2};
        for (int k = 0; k < 3; ++k) {
          tri[9 * f + 3 * k + 0] = (float)q[k].x;
          tri[9 * f + 3 * k + 1] = (float)q[k].y;
          tri[9 * f + 3 * k + 2] = (float)q[k].z;
        }
      }
    }
  }
}

__device__ __forceinline__ double fixed_scale(const double* frame, int depth) {
  const double sc = frame[3];
  const double h = sc > 0.0 ? (2097152.0 / sc) / (double)(1 << depth) : 0.0;
  return h > 0.0 ? 1099511627776.0 / (3.0 * h * h) : 1.0;  // 2^40 / (3 h^2)
}

// Every face of the chunk adds its vector to its k nearest points (fixed point).
__global__ void k_mc_scatter(const int32_t* __restrict__ idx, int64_t m, int k, const float4* __restrict__ vec,
                             const double* __restrict__ frame, int depth, int64_t n,
                             unsigned long long* __restrict__ acc) {
  const double S = fixed_scale(frame, depth);
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < m; f += (int64_t)gridDim.x * blockDim.x) {
    const float4 v = vec[f];
    const long long a0 = llrint((double)v.x * S), a1 = llrint((double)v.y * S), a2 = llrint((double)v.z * S);
    for (int t = 0; t < k; ++t) {
      const int64_t j = idx[f * k + t];
      if (j < 0 || j >= n) continue;
      atomicAdd(&acc[3 * j + 0], (unsigned long long)a0);
      atomicAdd(&acc[3 * j + 1], (unsigned long long)a1);
      atomicAdd(&acc[3 * j + 2], (unsigned long long)a2);
    }
  }
}

__device__ double mc_block_sum(double v, double* lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += lds[k];
  return r;
}

// Eq. 7 with the face sums: n = normalize(sum) (kept when the sum is 0), in place at the
// point's original index; theta and the chord partials; restaged moments; cleared sums.
__global__ __launch_bounds__(256) void k_mc_update(const int32_t* __restrict__ perm, int64_t n,
                                                   unsigned long long* __restrict__ acc,
                                                   const double* __restrict__ frame, int depth,
                                                   const float* __restrict__ kk, float* __restrict__ N,
                                                   float4* __restrict__ src, double* __restrict__ theta,
                                                   double* __restrict__ blk, int nblk) {
  __shared__ double lds[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double cv = 0.0;
  if (i < n) {
    const int64_t o = perm[i];
    const double S = fixed_scale(frame, depth);
    const double ax = (double)(long long)acc[3 * o] / S, ay = (double)(long long)acc[3 * o + 1] / S,
                 az = (double)(long long)acc[3 * o + 2] / S;
    acc[3 * o] = acc[3 * o + 1] = acc[3 * o + 2] = 0ull;
    const float o0 = N[o], o1 = N[n + o], o2 = N[2 * n + o];
    const double l = sqrt(ax * ax + ay * ay + az * az);
    float n0 = o0, n1 = o1, n2 = o2;
    if (l > 0.0 && l <= 1.7976931348623157e308) {
      n0 = (float)(ax / l);
      n1 = (float)(ay / l);
      n2 = (float)(az / l);
    }
    const double e0 = (double)n0 - o0, e1 = (double)n1 - o1, e2 = (double)n2 - o2;
    const double ch = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    const double h = 0.5 * ch;
    theta[i] = 2.0 * asin(h < 1.0 ? h : 1.0) * 57.295779513082320876798;
    N[o] = n0;
    N[n + o] = n1;
    N[2 * n + o] = n2;
    const float k = kk[i];
    src[2 * i + 1] = make_float4(k * n0, k * n1, k * n2, 0.0f);
    cv = ch;
  }
  const double bc = mc_block_sum(cv, lds);
  if (threadIdx.x == 0) {
    blk[blockIdx.x] = 0.0;
    blk[nblk + blockIdx.x] = bc;
  }
}

// Copies the points behind the corners in the query array (columns m .. m + n).
__global__ void k_mc_append_points(const float* __restrict__ P, int64_t n, float* __restrict__ pos, int64_t ld,
                                   int64_t m) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    for (int d = 0; d < 3; ++d) pos[d * ld + m + i] = P[d * n + i];
}

// FP64 mean of w[0..n): per-block partials (fixed shuffle tree), then one block in order.
__global__ __launch_bounds__(256) void k_mc_mean_part(const float* __restrict__ w, int64_t n,
                                                      double* __restrict__ part) {
  __shared__ double lds[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += (double)w[i];
  const double b = mc_block_sum(s, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

__global__ __launch_bounds__(256) void k_mc_mean_final(const double* __restrict__ part, int nb, int64_t n,
                                                       double* __restrict__ out) {
  __shared__ double lds[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
  const double b = mc_block_sum(s, lds);
  if (threadIdx.x == 0) *out = b / (double)n;
}

__global__ void k_zero_u64(unsigned long long* __restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0ull;
}

}  // namespace

int64_t mc_key_cap(int64_t n, const McParams& mp) {
  const int64_t w = 2 * mp.dilate + 1;
  return n * w * w * w;
}

size_t carve_mc_grid(Carver& c, int64_t n, const McParams& mp, McWork* out) {
  const size_t s0 = c.used;
  McWork w{};
  w.n = n;
  w.kcap = std::max<int64_t>(mc_key_cap(n, mp), n);
  w.bpart = c.take<float>(kBboxParts);
  w.box = c.take<float>(8);
  w.frame = c.take<double>(4);
  w.key[0] = c.take<uint64_t>((size_t)w.kcap);
  w.key[1] = c.take<uint64_t>((size_t)w.kcap);
  w.val[0] = c.take<int32_t>((size_t)w.kcap);
  w.val[1] = c.take<int32_t>((size_t)w.kcap);
  w.hist = c.take<int32_t>(radix_hist_len(w.kcap));
  w.hsums = c.take<int32_t>(scan_sums_len((int64_t)radix_hist_len(w.kcap)));
  w.head = c.take<int32_t>((size_t)w.kcap + 1);
  w.hdsums = c.take<int32_t>(scan_sums_len(w.kcap));
  w.occ = c.take<uint64_t>((size_t)n);
  w.cells = c.take<uint64_t>((size_t)w.kcap);
  if (out) *out = w;
  return c.used - s0;
}

int mc_faces_per_cell(const McParams& mp) { return mp.tets ? 12 : kMcMaxTri; }

size_t carve_mc_faces(Carver& c, int64_t n, int64_t C, const McParams& mp, McWork* w) {
  const size_t s0 = c.used;
  const int k = mp.k;
  McWork t{};
  McWork* o = w ? w : &t;
  o->C = C;
  o->tets = mp.tets;
  o->mcap = 8 * C;
  o->fcap = mc_faces_per_cell(mp) * C;
  o->chunk = std::min<int64_t>(std::max<int64_t>(o->fcap, 1), int64_t(1) << 20);
  o->ckey[0] = c.take<uint64_t>((size_t)(8 * C));
  o->ckey[1] = c.take<uint64_t>((size_t)(8 * C));
  o->cval[0] = c.take<int32_t>((size_t)(8 * C));
  o->cval[1] = c.take<int32_t>((size_t)(8 * C));
  o->chist = c.take<int32_t>(radix_hist_len(8 * C));
  o->chsums = c.take<int32_t>(scan_sums_len((int64_t)radix_hist_len(8 * C)));
  o->chead = c.take<int32_t>((size_t)(8 * C) + 1);
  o->chdsums = c.take<int32_t>(scan_sums_len(8 * C));
  o->cidx = c.take<int32_t>((size_t)(8 * C));
  o->pos = c.take<float>((size_t)(3 * (o->mcap + n)));
  o->wc = c.take<float>((size_t)(o->mcap + n));
  o->iso = c.take<double>(1);
  o->ipart = c.take<double>(256);
  o->fcnt = c.take<int32_t>((size_t)C + 1);
  o->fsums = c.take<int32_t>(scan_sums_len(C));
  o->cen = c.take<float>((size_t)(3 * o->fcap));
  o->vec = c.take<float4>((size_t)o->fcap);
  o->idx = c.take<int32_t>((size_t)(o->chunk * k));
  o->dist = c.take<float>((size_t)(o->chunk * k));
  o->acc = c.take<unsigned long long>((size_t)(3 * n));
  carve_knn(c, n, o->chunk, &o->knn);
  return c.used - s0;
}

dwg_status mc_cells(const float* P, int64_t n, const McParams& mp, const McWork& w, int64_t* C_host,
                    hipStream_t st) {
  DWG_PROPAGATE_INT(morton_frame(P, n, w.bpart, w.box, w.frame, st));
  hipLaunchKernelGGL(k_mc_point_keys, dim3(grid_of(n)), dim3(256), 0, st, P, n, w.frame, mp.depth, w.key[0],
                     w.val[0]);
  DWG_TRY_LAUNCH();
  int res = 0;
  DWG_PROPAGATE_INT(radix_sort_pairs(w.key, w.val, n, 3 * mp.depth, w.hist, w.hsums, &res, st));
  const uint64_t limit = 1ull << (3 * mp.depth);
  hipLaunchKernelGGL(k_mc_heads, dim3(grid_of(n)), dim3(256), 0, st, w.key[res], n, limit, w.head);
  DWG_TRY_LAUNCH();
  DWG_PROPAGATE_INT(exclusive_scan(w.head, n, w.hdsums, st));
  hipLaunchKernelGGL(k_mc_compact, dim3(grid_of(n)), dim3(256), 0, st, w.key[res], n, limit, w.head, w.occ);
  DWG_TRY_LAUNCH();
  // grow by `dilate` rings: (2 dilate + 1)^3 candidates per occupied cell, sentinel-padded
  const int64_t nk = mc_key_cap(n, mp);
  hipLaunchKernelGGL(k_mc_dilate, dim3(grid_of(nk)), dim3(256), 0, st, w.occ, w.head + n, n, mp.depth, mp.dilate,
                     w.key[0], w.val[0]);
  DWG_TRY_LAUNCH();
  DWG_PROPAGATE_INT(radix_sort_pairs(w.key, w.val, nk, 3 * mp.depth + 1, w.hist, w.hsums, &res, st));
  hipLaunchKernelGGL(k_mc_heads, dim3(grid_of(nk)), dim3(256), 0, st, w.key[res], nk, limit, w.head);
  DWG_TRY_LAUNCH();
  DWG_PROPAGATE_INT(exclusive_scan(w.head, nk, w.hdsums, st));
  hipLaunchKernelGGL(k_mc_compact, dim3(grid_of(nk)), dim3(256), 0, st, w.key[res], nk, limit, w.head, w.cells);
  DWG_TRY_LAUNCH();
  int32_t C = 0;
  DWG_TRY_HIP(hipMemcpyAsync(&C, w.head + nk, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  DWG_TRY_HIP(hipStreamSynchronize(st));
  *C_host = C;
  return DWG_OK;
}

dwg_status mc_corners(const McParams& mp, McWork& w, int64_t* m_host, hipStream_t st) {
  const int64_t n8 = 8 * w.C;
  hipLaunchKernelGGL(k_mc_corner_keys, dim3(grid_of(n8)), dim3(256), 0, st, w.cells, w.C, w.ckey[0], w.cval[0]);
  DWG_TRY_LAUNCH();
  int res = 0;
  DWG_PROPAGATE_INT(radix_sort_pairs(w.ckey, w.cval, n8, 3 * (mp.depth + 1), w.chist, w.chsums, &res, st));
  hipLaunchKernelGGL(k_mc_heads, dim3(grid_of(n8)), dim3(256), 0, st, w.ckey[res], n8, ~0ull, w.chead);
  DWG_TRY_LAUNCH();
  DWG_PROPAGATE_INT(exclusive_scan(w.chead, n8, w.chdsums, st));
  int32_t m = 0;
  DWG_TRY_HIP(hipMemcpyAsync(&m, w.chead + n8, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  DWG_TRY_HIP(hipStreamSynchronize(st));
  w.m = m;
  w.ld = m + (mp.iso_points ? w.n : 0);
  hipLaunchKernelGGL(k_mc_corner_ids, dim3(grid_of(n8)), dim3(256), 0, st, w.ckey[res], w.cval[res], n8, w.chead,
                     w.frame, w.box, mp.depth, w.cidx, w.pos, w.ld);
  DWG_TRY_LAUNCH();
  *m_host = m;
  return DWG_OK;
}

dwg_status mc_faces(const McWork& w, float* tri, int64_t tcap, int64_t* F_host, hipStream_t st) {
  if (w.tets)
    hipLaunchKernelGGL(k_mt_count, dim3(grid_of(w.C)), dim3(256), 0, st, w.C, w.cidx, w.pos, w.ld, w.wc, w.iso,
                       w.fcnt);
  else
    hipLaunchKernelGGL(k_mc_count, dim3(grid_of(w.C)), dim3(256), 0, st, w.C, w.cidx, w.wc, w.iso, w.fcnt);
  DWG_TRY_LAUNCH();
  DWG_PROPAGATE_INT(exclusive_scan(w.fcnt, w.C, w.fsums, st));
  if (w.tets)
    hipLaunchKernelGGL(k_mt_emit, dim3(grid_of(w.C)), dim3(256), 0, st, w.C, w.cidx, w.pos, w.ld, w.wc, w.iso,
                       w.fcnt, w.fcap, w.cen, w.fcap, w.vec, tri, tcap);
  else
    hipLaunchKernelGGL(k_mc_emit, dim3(grid_of(w.C)), dim3(256), 0, st, w.C, w.cidx, w.pos, w.ld, w.wc, w.iso,
                       w.fcnt, w.fcap, w.cen, w.fcap, w.vec, tri, tcap);
  DWG_TRY_LAUNCH();
  int32_t F = 0;
  DWG_TRY_HIP(hipMemcpyAsync(&F, w.fcnt + w.C, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  DWG_TRY_HIP(hipStreamSynchronize(st));
  *F_host = F;
  return DWG_OK;
}

dwg_status mc_scatter(const McParams& mp, const McWork& w, int64_t F, hipStream_t st) {
  for (int64_t q0 = 0; q0 < F; q0 += w.chunk) {
    const int64_t m = std::min<int64_t>(w.chunk, F - q0);
    DWG_PROPAGATE_INT(knn_search(w.cen, w.fcap, q0, m, w.knn, mp.k, w.idx, w.dist, st));
    hipLaunchKernelGGL(k_mc_scatter, dim3(grid_of(m)), dim3(256), 0, st, w.idx, m, mp.k, w.vec + q0, w.frame,
                       mp.depth, w.n, w.acc);
    DWG_TRY_LAUNCH();
  }
  return DWG_OK;
}

dwg_status mc_append_points(const float* P, int64_t n, const McWork& w, hipStream_t st) {
  hipLaunchKernelGGL(k_mc_append_points, dim3(grid_of(n)), dim3(256), 0, st, P, n, w.pos, w.ld, w.m);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status mc_point_iso(const McWork& w, const float* w_points, int64_t n, hipStream_t st) {
  constexpr int kParts = 256;
  hipLaunchKernelGGL(k_mc_mean_part, dim3(kParts), dim3(256), 0, st, w_points, n, w.ipart);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_mc_mean_final, dim3(1), dim3(256), 0, st, w.ipart, kParts, n, w.iso);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status mc_clear(const McWork& w, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_of(3 * w.n)), dim3(256), 0, st, w.acc, 3 * w.n);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status mc_update(const McParams& mp, const McWork& w, const GwnWork& g, float* N, hipStream_t st) {
  const int nb = (int)cdiv(w.n, 256);
  hipLaunchKernelGGL(k_mc_update, dim3(nb), dim3(256), 0, st, g.perm_s, w.n, w.acc, w.frame, mp.depth, g.kk, N,
                     g.src, g.theta, g.blk, nb);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

}  // namespace dwg
