// Internal declarations shared by the libdwg translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "dwg.h"

namespace dwg {

// Records a printf-style detail string for dwg_last_error() on the calling thread.
void set_error(const char* fmt, ...);

#define DWG_TRY_HIP(call)                                                            \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ::dwg::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                    \
      return DWG_E_DEVICE;                                                           \
    }                                                                                \
  } while (0)

#define DWG_TRY_LAUNCH() DWG_TRY_HIP(hipGetLastError())

// ----------------------------------------------------------------------------- sizes
constexpr int kBlock = 256;    // threads per block for the all-pairs kernels (4 waves)
constexpr int kTile = 256;     // sources per LDS tile
constexpr int kQpt = 2;        // queries held in registers per thread
constexpr int kQBlock = kBlock * kQpt;  // queries per block
constexpr int kNAcc = 7;       // per-query accumulators with the gradient: w, A[3], B[3]
constexpr int kMaxSplit = 64;   // largest source split a caller may request
constexpr int64_t kAutoSplitBytes = int64_t(512) << 20;  // partial sums of an automatic split
constexpr int kRedBlock = 256;  // threads per block for O(n) epilogue / reductions
constexpr int kMaxK = 16;       // largest k for the kNN kernels

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bump allocator over the caller's workspace. With base == nullptr it only measures.
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    size_t off = used;
    used = align256(used + count * sizeof(T));
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

// Scale of the staged positions: s log2(e) for the screened kernel (s = sqrt(lambda)), 1 for
// the plain one (see dwg_pair.h).
float position_scale(const dwg_kernel_params& kp);

// Split count for the all-pairs kernels.
int choose_split(int64_t n_src, int64_t n_qry, int requested);

// Uniform grid over a reference point set (dwg_knn.hip).
struct GridParams {
  float ox, oy, oz;  // origin (minimum corner of the trimmed box)
  float h, ih;       // cell size and its inverse
  int nx, ny, nz;
  int64_t ncells;
};
struct KnnWork {
  float* bbox_part;  // [256 * 6] per-block bbox partials
  double* range;     // [6] trimmed box per axis (lo, hi)
  int64_t* below;    // [3] reference points under each axis' lo
  int32_t* hist;     // [3 * 1024] axis histograms of the trimming passes
  GridParams* gp;
  int32_t* key;      // [nr] cell of each reference point
  int32_t* start;    // [max_cells + 1] first sorted slot of each cell
  int32_t* cursor;   // [max_cells] scatter cursors
  int32_t* sums;     // scan tile totals
  float4* sorted;    // [nr] (x, y, z, index bits) in cell order
  int32_t* defer;    // [1 + mq] count and list of the queries left to the second search pass
  int64_t mq;        // most queries of one search call
};
size_t carve_knn(Carver& c, int64_t nr, int64_t mq, KnnWork* out);

// Anchor features of the learned initial normals: anchors, their grid, chunk buffers.
constexpr int64_t DWG_FEAT_ANCHORS = 4096;
struct AnchorCtx {
  float* A;            // [3][na] anchor coordinates
  int32_t* idx;        // [chunk][16]
  float* dist;         // [chunk][16]
  float* feat;         // [chunk][48]
  int64_t na, stride, chunk;
  KnnWork w;
};
size_t carve_anchor(Carver& c, int64_t n, int64_t chunk, int64_t n_anchor, AnchorCtx* out);
size_t anchor_ws_bytes(int64_t n, int64_t chunk, int64_t n_anchor);
dwg_status anchor_build(const float* P, int64_t n, const AnchorCtx& x, hipStream_t stream);
dwg_status anchor_features(const float* P, int64_t n, int64_t q0, int64_t m, const AnchorCtx& x, float* feat,
                           hipStream_t stream);
dwg_status anchor_delta(const float* P, int64_t n, const AnchorCtx& x, int k, float scale, float* delta,
                        hipStream_t stream);

// Bounding box of a planar [3][n] array: part [256 * 6] scratch, out6 = min xyz, max xyz.
constexpr int kBboxParts = 256 * 6;
dwg_status launch_bbox(const float* R, int64_t n, float* part, float* out6, hipStream_t st);
// In-place exclusive scan of a[0..n), total written to a[n]; sums has scan_sums_len(n) slots.
size_t scan_sums_len(int64_t n);
dwg_status exclusive_scan(int32_t* a, int64_t n, int32_t* sums, hipStream_t st);

// Spatial order of a point set for the all-pairs kernel (dwg_sort.hip).
struct SortWork {
  float* part;      // [kBboxParts]
  float* box;       // [8]: bbox and the mean kernel radius
  double* rpart;    // [256] radius partial sums
  uint64_t* key[2]; // [n] radix-sort keys, ping-pong
  int32_t* val;     // [n] indices (the second value buffer is the output permutation)
  int32_t* hist;    // radix_hist_len(n)
  int32_t* hsums;   // scan_sums_len(radix_hist_len(n))
};
constexpr int kSortKeyBits = 22;  // radius class (1 bit) + Morton code of a 128^3 grid (21 bits)
size_t carve_sort(Carver& c, int64_t n, SortWork* out);
// perm[i] = original index of the i-th point in spatial order (deterministic).
dwg_status spatial_sort(const float* P, int64_t n, const float* delta, float eps, const SortWork& w,
                        int32_t* perm, hipStream_t st);

// Device-side state of one GWN / iteration launch sequence, carved from the workspace.
// Sources and queries are processed in spatial order (perm_s / perm_q: sorted position ->
// original index); outputs are written back at the original indices.
struct GwnWork {
  float4* src;        // [2 * npad]: (px,py,pz,1/rho_min), (mx,my,mz,0) per sorted source
  float* part;        // [split][kNAcc][mpad] per-split partial sums (sorted queries)
  float* kk;          // [npad] a_j / (4 pi), for restaging after the update
  double* theta;      // [m] angle change in degrees (iterate)
  double* blk;        // [2 * nblk] per-block FP64 partial sums
  double* stats;      // [4] device statistics
  uint32_t* hist;     // [256] radix histogram
  uint64_t* sel;      // [2]: radix prefix, remaining count
  float4* tbox;       // [2 * ntiles] source tile boxes and radii
  float4* qbox;       // [2 * mpad / kQBlock] query block boxes
  int32_t* perm_s;    // [npad]
  int32_t* perm_q;    // [mpad] (== perm_s when the queries are the sources)
  SortWork sort;
  int64_t n_src, npad, mpad, ntiles;
  int split;
  int nblk;           // blocks of the O(n) epilogue kernels
};

size_t carve_gwn(Carver& c, int64_t n_src, int64_t n_qry, int split, bool same, GwnWork* out);

// Octree of the sources for the Sec. 5.2 traversal (dwg_tree.hip): Morton-sorted sources,
// nodes in depth-first pre-order, node summaries; carved from the workspace.
struct TreeWork {
  float* bpart;              // [kBboxParts] bbox partials
  float* box;                // [8] bbox
  double* frame;             // [4] lo xyz, 2^21 / extent
  uint64_t* key[2];          // [n] Morton codes (radix-sort ping-pong)
  int32_t* val[2];           // [n] source indices (ping-pong)
  int32_t* hist;             // [256 * nsb + 1] radix digit counts
  int32_t* hsums;            // scan tile totals
  int32_t* lev;              // [n] level range of the nodes starting at each sorted source
  int32_t* off;              // [n + 1] node offsets; off[n] = node count
  int32_t* osums;
  int4* node;                // [cap] start, end, skip, level | leaf << 8
  double4* geo;              // [cap] centre xyz, squared opening radius
  float4* mom;               // [cap] moment sum a n / 4 pi
  unsigned long long* rbits; // [cap] node radius (FP64 bits)
  uint32_t* dbits;           // [cap] largest kernel radius (FP32 bits)
  int32_t* coff;             // [cap + 1] chunk offsets (chunks of 256 sorted sources per node)
  int32_t* csums;
  double4* csum;             // [ccap] per-chunk FP64 sums of a, a px, a py, a pz
  double* scan;              // [3][n + 1] FP64 prefix sums of the staged moments
  double* sblk;              // [3][nscan] block totals
  int64_t n, cap, ccap, nsb, nscan;
  int leaf;
  double beta;
};
int64_t tree_cap(int64_t n);
size_t carve_tree(Carver& c, int64_t n, int leaf, double beta, TreeWork* out);
// Sorts the sources (perm[i] = index of the i-th sorted source) and builds the nodes; with
// area != NULL also the node centres, radii and opening radii.
dwg_status tree_build(const float* P, const float* area, const float* delta, int64_t n, float eps,
                      const TreeWork& t, int32_t* perm, hipStream_t st);
// Node moments from the staged sources of w (call after every restaging).
// Octree mode: rewrites the staged source positions as kappa (p - c_leaf), relative to the
// centre of the leaf that holds each source (after tree_build with areas and launch_stage;
// the all-pairs kernels never read sources staged this way).
dwg_status tree_stage_leaves(const GwnWork& w, const TreeWork& t, float kappa, hipStream_t st);
dwg_status tree_moments(const GwnWork& w, const TreeWork& t, hipStream_t st);
// Octree-approximated w (and grad) at the sorted queries of w into w.part (split 1).
dwg_status tree_eval(const float* Q, int64_t m, const dwg_kernel_params& kp, bool grad, const GwnWork& w,
                     const TreeWork& t, hipStream_t st);
// Work of the traversal over the m sorted queries: far dipoles (out[0]), leaf pairs (out[1]),
// wavefront steps with at least one far lane (out[2]) and wavefront leaf-loop iterations
// (out[3]); out is kTreeWorkCounts device counters.
constexpr int kTreeWorkCounts = 4;
dwg_status tree_work(const float* Q, int64_t m, const int32_t* qperm, const TreeWork& t, unsigned long long* out,
                     hipStream_t st);
dwg_status tree_export(const TreeWork& t, int32_t* nodes_out, int64_t cap_out, int64_t* count_host,
                       hipStream_t st);
// Stable LSD radix sort of (key, value) pairs on the low `bits` bits, 8 bits per pass,
// ping-ponging between key[0]/val[0] and key[1]/val[1]; *result = the buffer holding the
// sorted pairs. hist needs radix_hist_len(n) ints, hsums scan_sums_len(radix_hist_len(n)).
size_t radix_hist_len(int64_t n);
dwg_status radix_sort_pairs(uint64_t* const key[2], int32_t* const val[2], int64_t n, int bits, int32_t* hist,
                            int32_t* hsums, int* result, hipStream_t st);
// Bounding box of P and the octree frame (lo xyz, 2^21 / largest extent) in FP64.
dwg_status morton_frame(const float* P, int64_t n, float* bpart, float* box, double* frame, hipStream_t st);
// Uniform-grid kNN over reference points: build once, then query [q0, q0 + m) of a planar
// query array with leading dimension qld (no skipping; m <= the capacity carved for the grid).
// One thread searches each query to the end, in the given order: meant for query sets that
// are already in spatial order.
dwg_status knn_grid(const float* R, int64_t nr, const KnnWork& w, hipStream_t st);
dwg_status knn_search(const float* Q, int64_t qld, int64_t q0, int64_t m, const KnnWork& w, int k, int32_t* idx,
                      float* dist, hipStream_t st);

// The paper's level-set update (dwg_mc.hip): grid cells and corners, faces, scatter.
struct McParams {
  int depth;       // grid cells per axis = 2^depth
  int dilate;      // rings of neighbour cells added around the cells holding points
  int k;           // nearest points per face
  int iso_points;  // 1: w_bar = mean of w over the input points; 0: over the grid corners
  int tets;        // 1: marching tetrahedra (option); 0: Marching Cubes (the paper's)
};
struct McWork {
  // grid phase (sized by n)
  float* bpart;
  float* box;
  double* frame;           // octree frame: lo xyz, 2^21 / side
  uint64_t* key[2];        // [kcap] radix-sort ping-pong
  int32_t* val[2];
  int32_t* hist;
  int32_t* hsums;
  int32_t* head;           // [kcap + 1] run heads, then their exclusive scan
  int32_t* hdsums;
  uint64_t* occ;           // [n] occupied cell codes
  uint64_t* cells;         // [kcap] evaluated cell codes (Morton order)
  // faces phase (sized by the cell count C)
  uint64_t* ckey[2];       // [8C] corner keys
  int32_t* cval[2];
  int32_t* chist;
  int32_t* chsums;
  int32_t* chead;          // [8C + 1]
  int32_t* chdsums;
  int32_t* cidx;           // [C][8] corner id of each cell corner
  float* pos;              // [3][ld] corner positions, then the points when w_bar is taken over them
  float* wc;               // [ld] w at those queries
  double* iso;             // [1] w_bar
  double* ipart;           // [256] partial sums of w_bar
  int32_t* fcnt;           // [C + 1] faces per cell, then their exclusive scan
  int32_t* fsums;
  float* cen;              // [3][fcap] face centroids
  float4* vec;             // [fcap] face vectors
  int32_t* idx;            // [chunk][k] nearest points of a chunk of faces
  float* dist;
  unsigned long long* acc; // [n][3] fixed-point face sums
  KnnWork knn;             // uniform grid over the points
  int64_t n = 0, kcap = 0, C = 0, m = 0, ld = 0, mcap = 0, fcap = 0, chunk = 0;
  int tets = 0;            // extraction: 0 Marching Cubes, 1 marching tetrahedra
};
int64_t mc_key_cap(int64_t n, const McParams& mp);
size_t carve_mc_grid(Carver& c, int64_t n, const McParams& mp, McWork* out);
// Faces a cell can produce: 5 by Marching Cubes, 12 by marching tetrahedra.
int mc_faces_per_cell(const McParams& mp);
size_t carve_mc_faces(Carver& c, int64_t n, int64_t C, const McParams& mp, McWork* w);
dwg_status mc_cells(const float* P, int64_t n, const McParams& mp, const McWork& w, int64_t* C_host,
                    hipStream_t st);
dwg_status mc_corners(const McParams& mp, McWork& w, int64_t* m_host, hipStream_t st);
dwg_status mc_faces(const McWork& w, float* tri, int64_t tcap, int64_t* F_host, hipStream_t st);
dwg_status mc_scatter(const McParams& mp, const McWork& w, int64_t F, hipStream_t st);
dwg_status mc_clear(const McWork& w, hipStream_t st);
dwg_status mc_append_points(const float* P, int64_t n, const McWork& w, hipStream_t st);
dwg_status mc_point_iso(const McWork& w, const float* w_points, int64_t n, hipStream_t st);
dwg_status mc_update(const McParams& mp, const McWork& w, const GwnWork& g, float* N, hipStream_t st);

// Workspace bytes of the kNN / features / MLP stages for n points.
size_t knn_ws_bytes(int64_t n_ref, int64_t n_qry);
size_t mlp_ws_bytes(int64_t B);
dwg_status mlp_forward(const float* params, const float* X, int64_t B, float* Y, int64_t sr, int64_t sc,
                       hipStream_t stream);

// Launchers (all enqueue on `stream`; return DWG_OK or DWG_E_DEVICE).
dwg_status launch_order(const float* P, int64_t n, const float* delta, float eps, float kappa, const float* Q,
                        int64_t m, bool same, const GwnWork& w, hipStream_t stream);
dwg_status launch_stage(const float* P, const float* N, const float* area, const float* delta,
                        int64_t n, float eps, float kappa, const GwnWork& w, hipStream_t stream);
dwg_status launch_gwn(const float* Q, int64_t m, const dwg_kernel_params& kp, bool grad,
                      const GwnWork& w, hipStream_t stream);
dwg_status launch_combine(int64_t m, const dwg_kernel_params& kp, bool grad, float* wout,
                          float* gout, double* wmean, const GwnWork& w, hipStream_t stream);
dwg_status launch_update(int64_t n, const dwg_kernel_params& kp, float* N, const GwnWork& w,
                         hipStream_t stream);
dwg_status launch_stats(int64_t n, double top_frac, const GwnWork& w, hipStream_t stream);
dwg_status launch_random_normals(uint64_t seed, int64_t n, float* N, hipStream_t stream);

dwg_status knn_run(const float* R, int64_t nr, const float* Q, int64_t m, int self_skip,
                   const int64_t* skip_stride, int k, int32_t* idx, float* dist, void* ws,
                   size_t ws_bytes, hipStream_t stream);
dwg_status delta_from_knn(const float* dist, int64_t n, int k, float scale, float* delta,
                          hipStream_t stream);
dwg_status pca_normals(const float* P, int64_t n, int k, float* N, void* ws, hipStream_t stream);
dwg_status gauss_normals(const float* P, int64_t n, float* N, hipStream_t stream);
dwg_status voronoi_area(const float* P, int64_t n, int m, float* area, void* ws, hipStream_t stream);
dwg_status delta_window(const float* P, int64_t n, int k, float vmin, float vmax, float* delta, void* ws,
                        hipStream_t stream);
dwg_status features_run(const float* P, int64_t n, int64_t n_anchor, float* feat, void* ws,
                        size_t ws_bytes, hipStream_t stream);
dwg_status mlp_infer_run(const float* params, const float* X, int64_t B, float* Y, void* ws,
                         size_t ws_bytes, hipStream_t stream);
dwg_status mlp_train_run(float* params, float* m1, float* m2, int64_t step, float lr,
                         const float* X, const float* T, const uint8_t* mask, int64_t B,
                         float* grad_out, float* loss_out, void* ws, size_t ws_bytes,
                         hipStream_t stream);

}  // namespace dwg
