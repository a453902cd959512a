// Exact k-nearest-neighbour search on a uniform grid, the kernel radius delta (Sec. 5.2
// "Poisson Kernels": mean distance to the k nearest neighbours) and the k = 16 anchor
// features of the learned initial normals.
//
// Grid build: bounding box (deterministic two-stage min/max), trimmed per axis to the
// quantiles 1/1024 and 1 - 1/1024 of the reference points (three passes of a 1024-bin
// histogram, each refining the range the last one found), cell size from the trimmed box's
// volume with at most ~8 cells per reference point, counting sort of the reference points
// by cell (atomic cursors; the order inside a cell is arbitrary, which is harmless because
// candidates are ranked by the pair (squared distance, index)). Points outside the trimmed
// box sit in its border cells: a few points far from the rest then no longer stretch the
// cells until the whole cloud shares one, and the search stays exact because projecting
// onto a box shortens no distance (see k_knn). Query: Chebyshev rings of
// cells around the query's own cell, a row of cells (one contiguous range of the sorted
// points) at a time, keeping the k best candidates in registers, until the k-th best
// distance is below the distance to the next ring. One thread per query takes rings 0..3;
// the few queries still unfinished (isolated points) are then searched by a wavefront each
// (k_knn, k_knn_wave).
#include <cfloat>
#include <climits>
#include <cmath>

#include "dwg_internal.h"

namespace dwg {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;  // elements per thread in the block scan
constexpr int kScanTile = kScanBlock * kScanItems;


__global__ __launch_bounds__(256) void k_bbox_partial(const float* __restrict__ R, int64_t n,
                                                      float* __restrict__ part) {
  __shared__ float lds[6][256];
  float mn[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, mx[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int d = 0; d < 3; ++d) {
      const float v = R[d * n + i];
      mn[d] = fminf(mn[d], v);
      mx[d] = fmaxf(mx[d], v);
    }
  }
  for (int d = 0; d < 3; ++d) {
    lds[d][threadIdx.x] = mn[d];
    lds[3 + d][threadIdx.x] = mx[d];
  }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int d = 0; d < 3; ++d) {
        lds[d][threadIdx.x] = fminf(lds[d][threadIdx.x], lds[d][threadIdx.x + s]);
        lds[3 + d][threadIdx.x] = fmaxf(lds[3 + d][threadIdx.x], lds[3 + d][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = lds[threadIdx.x][0];
}

// Minimum and maximum per axis of the nblocks per-block partials, by one block of 256
// threads (min and max are exact in any order): v6 = (min x, min y, min z, max x, ...).
__device__ void reduce_bbox_parts(const float* __restrict__ part, int nblocks, float (*lds)[256], float* v6) {
  float v[6] = {FLT_MAX, FLT_MAX, FLT_MAX, -FLT_MAX, -FLT_MAX, -FLT_MAX};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
    for (int d = 0; d < 3; ++d) {
      v[d] = fminf(v[d], part[b * 6 + d]);
      v[3 + d] = fmaxf(v[3 + d], part[b * 6 + 3 + d]);
    }
  for (int d = 0; d < 6; ++d) lds[d][threadIdx.x] = v[d];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int d = 0; d < 3; ++d) {
        lds[d][threadIdx.x] = fminf(lds[d][threadIdx.x], lds[d][threadIdx.x + st]);
        lds[3 + d][threadIdx.x] = fmaxf(lds[3 + d][threadIdx.x], lds[3 + d][threadIdx.x + st]);
      }
    __syncthreads();
  }
  for (int d = 0; d < 6; ++d) v6[d] = lds[d][0];
}

// Final bounding box: out6 = (min x, min y, min z, max x, max y, max z). One block of 256.
__global__ __launch_bounds__(256) void k_bbox_final(const float* __restrict__ part, int nblocks,
                                                    float* __restrict__ out6) {
  __shared__ float lds[6][256];
  float v6[6];
  reduce_bbox_parts(part, nblocks, lds, v6);
  if (threadIdx.x < 6) out6[threadIdx.x] = v6[threadIdx.x];
}

// Grid box trimming. range[2d], range[2d + 1] = the current [lo, hi] of axis d (FP64) and
// below[d] = the number of reference points under lo; kTrimLevels passes of k_axis_hist /
// k_trim_refine narrow each axis to the bins that hold the ranks floor(n / 1024) and
// n - 1 - floor(n / 1024) of its coordinates.
constexpr int kTrimBins = 1024;
constexpr int kTrimLevels = 3;

// range = the bounding box (from the per-block partials, reduced by one block of 256
// threads), below = 0, histograms cleared.
__global__ __launch_bounds__(256) void k_trim_init(const float* __restrict__ part, int nblocks,
                                                   double* __restrict__ range, int64_t* __restrict__ below,
                                                   int32_t* __restrict__ hist) {
  __shared__ float lds[6][256];
  for (int i = threadIdx.x; i < 3 * kTrimBins; i += blockDim.x) hist[i] = 0;
  float v6[6];
  reduce_bbox_parts(part, nblocks, lds, v6);
  if (threadIdx.x < 3) {
    range[2 * threadIdx.x] = v6[threadIdx.x];
    range[2 * threadIdx.x + 1] = v6[3 + threadIdx.x];
    below[threadIdx.x] = 0;
  }
}

// Per axis, the histogram of the coordinates inside [lo, hi] over kTrimBins equal bins
// (LDS counts per block, then added to `hist`); NaN coordinates fall in no bin.
__global__ __launch_bounds__(256) void k_axis_hist(const float* __restrict__ R, int64_t n,
                                                   const double* __restrict__ range, int32_t* __restrict__ hist) {
  __shared__ int32_t h[3 * kTrimBins];
  for (int i = threadIdx.x; i < 3 * kTrimBins; i += blockDim.x) h[i] = 0;
  double lo[3], hi[3], sc[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = range[2 * d];
    hi[d] = range[2 * d + 1];
    sc[d] = hi[d] > lo[d] ? kTrimBins / (hi[d] - lo[d]) : 0.0;
  }
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    for (int d = 0; d < 3; ++d) {
      const double x = R[d * n + i];
      if (x >= lo[d] && x <= hi[d]) {
        int b = (int)((x - lo[d]) * sc[d]);
        b = b < kTrimBins - 1 ? b : kTrimBins - 1;
        atomicAdd(&h[d * kTrimBins + b], 1);
      }
    }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * kTrimBins; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// One block of 256 threads per axis (blockIdx.x): the bins holding ranks rlo and rhi
// (counting the points below lo) become the new range, found from an exclusive scan of the
// histogram in LDS; the histogram is cleared for the next pass. A range whose ranks are not
// found (NaN coordinates among the points) is kept.
__global__ __launch_bounds__(256) void k_trim_refine(int32_t* __restrict__ hist, double* __restrict__ range,
                                                     int64_t* __restrict__ below, int64_t rlo, int64_t rhi) {
  constexpr int kPer = kTrimBins / 256;
  __shared__ int64_t scan[256];
  __shared__ int found[2];
  __shared__ int64_t below_lo;
  const int d = blockIdx.x, t = threadIdx.x;
  int32_t* hd = hist + d * kTrimBins;
  int64_t c[kPer], sum = 0;
  for (int k = 0; k < kPer; ++k) {
    c[k] = hd[t * kPer + k];
    hd[t * kPer + k] = 0;
    sum += c[k];
  }
  scan[t] = sum;
  if (t < 2) found[t] = -1;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive scan of the per-thread sums
    const int64_t x = t >= off ? scan[t - off] : 0;
    __syncthreads();
    scan[t] += x;
    __syncthreads();
  }
  int64_t cum = below[d] + scan[t] - sum;  // points below this thread's first bin
  for (int k = 0; k < kPer; ++k) {
    if (cum <= rlo && cum + c[k] > rlo) {
      found[0] = t * kPer + k;
      below_lo = cum;
    }
    if (cum <= rhi && cum + c[k] > rhi) found[1] = t * kPer + k;
    cum += c[k];
  }
  __syncthreads();
  if (t != 0) return;
  const double lo = range[2 * d], hi = range[2 * d + 1];
  const int blo = found[0], bhi = found[1];
  if (blo < 0 || bhi < 0 || !(hi > lo)) return;
  const double w = (hi - lo) / kTrimBins;
  range[2 * d] = lo + blo * w;
  range[2 * d + 1] = bhi == kTrimBins - 1 ? hi : lo + (bhi + 1) * w;
  below[d] = below_lo;
}

// Grid parameters over the trimmed box (single thread).
__global__ void k_grid_params(const double* __restrict__ range, int64_t max_cells, GridParams* __restrict__ gp) {
  if (threadIdx.x != 0) return;
  float mn[3], mx[3];
  for (int d = 0; d < 3; ++d) {  // the FP64 range rounded outwards to FP32
    mn[d] = (float)range[2 * d];
    if ((double)mn[d] > range[2 * d]) mn[d] = nextafterf(mn[d], -INFINITY);
    mx[d] = (float)range[2 * d + 1];
    if ((double)mx[d] < range[2 * d + 1]) mx[d] = nextafterf(mx[d], INFINITY);
  }
  double ext[3];
  double emax = 0.0;
  for (int d = 0; d < 3; ++d) {
    ext[d] = (double)mx[d] - (double)mn[d];
    if (!(ext[d] >= 0.0 && ext[d] <= 1e30)) ext[d] = 1e30;  // infinite or NaN coordinates
    emax = fmax(emax, ext[d]);
  }
  if (!(emax > 0.0)) emax = 1.0;
  // slabs thinner than 1e-3 of the largest extent count as that thickness for the volume
  double vol = 1.0;
  for (int d = 0; d < 3; ++d) vol *= fmax(ext[d], 1e-3 * emax);
  double h = cbrt(vol / (double)max_cells);
  // every point of the box must fall inside the grid: grow h until the uncapped cell counts
  // multiply to at most max_cells (at most a few steps; the cap only bounds the loop)
  double dd[3] = {1.0, 1.0, 1.0};
  for (int it = 0; it < 4096; ++it) {
    double cells = 1.0;
    for (int d = 0; d < 3; ++d) {
      dd[d] = floor(ext[d] / h) + 1.0;
      cells *= dd[d];
    }
    if (cells <= (double)max_cells) break;
    h *= 1.05;
  }
  if (dd[0] * dd[1] * dd[2] > (double)max_cells) {  // not reached for finite extents; one cell
    dd[0] = dd[1] = dd[2] = 1.0;
    h = emax;
  }
  int dims[3] = {(int)dd[0], (int)dd[1], (int)dd[2]};
  GridParams g;
  g.ox = mn[0];
  g.oy = mn[1];
  g.oz = mn[2];
  g.h = (float)h;
  g.ih = (float)(1.0 / h);
  g.nx = dims[0];
  g.ny = dims[1];
  g.nz = dims[2];
  g.ncells = (int64_t)dims[0] * dims[1] * dims[2];
  *gp = g;
}

__device__ __forceinline__ void cell_of(const GridParams& g, float x, float y, float z, int& cx,
                                        int& cy, int& cz) {
  // clamped as floats before the conversion, so that points far outside the box (and NaN,
  // which fmaxf maps to 0) land in its border cells
  cx = (int)fminf(fmaxf(floorf((x - g.ox) * g.ih), 0.0f), (float)(g.nx - 1));
  cy = (int)fminf(fmaxf(floorf((y - g.oy) * g.ih), 0.0f), (float)(g.ny - 1));
  cz = (int)fminf(fmaxf(floorf((z - g.oz) * g.ih), 0.0f), (float)(g.nz - 1));
}

__global__ void k_zero_i32(int32_t* __restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

__global__ void k_cell_count(const float* __restrict__ R, int64_t n, const GridParams* __restrict__ gp,
                             int32_t* __restrict__ key, int32_t* __restrict__ count) {
  const GridParams g = *gp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int cx, cy, cz;
    cell_of(g, R[i], R[n + i], R[2 * n + i], cx, cy, cz);
    const int32_t c = (int32_t)(((int64_t)cz * g.ny + cy) * g.nx + cx);
    key[i] = c;
    atomicAdd(&count[c], 1);
  }
}

// Exclusive scan, stage 1: each block scans kScanTile elements of `a` in place and writes
// its total to `sums[block]`. Elements past `n` read as 0.
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(int32_t* __restrict__ a, int64_t n,
                                                           int32_t* __restrict__ sums) {
  __shared__ int32_t lds[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t tot = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? a[base + k] : 0;
    tot += v[k];
  }
  lds[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const int32_t x = ((int)threadIdx.x >= off) ? lds[threadIdx.x - off] : 0;
    __syncthreads();
    lds[threadIdx.x] += x;
    __syncthreads();
  }
  int32_t run = lds[threadIdx.x] - tot;  // exclusive prefix of this thread
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) a[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = lds[kScanBlock - 1];
}

// Stage 2: one block scans the tile totals serially in chunks (exclusive) and writes the
// grand total to a[n] (the end marker of the last cell).
__global__ __launch_bounds__(kScanBlock) void k_scan_sums(int32_t* __restrict__ sums, int64_t nt,
                                                          int32_t* __restrict__ a, int64_t n) {
  __shared__ int32_t lds[kScanBlock];
  const int64_t per = (nt + kScanBlock - 1) / kScanBlock;
  const int64_t b0 = (int64_t)threadIdx.x * per, b1 = min(b0 + per, nt);
  int32_t tot = 0;
  for (int64_t i = b0; i < b1; ++i) tot += sums[i];
  lds[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const int32_t x = ((int)threadIdx.x >= off) ? lds[threadIdx.x - off] : 0;
    __syncthreads();
    lds[threadIdx.x] += x;
    __syncthreads();
  }
  int32_t run = lds[threadIdx.x] - tot;
  for (int64_t i = b0; i < b1; ++i) {
    const int32_t x = sums[i];
    sums[i] = run;
    run += x;
  }
  if (threadIdx.x == kScanBlock - 1) a[n] = lds[kScanBlock - 1];
}

__global__ void k_scan_add(int32_t* __restrict__ a, int64_t n, const int32_t* __restrict__ sums) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] += sums[i / kScanTile];
}

// Scatter reference points into cell order: sorted[pos] = (x, y, z, index bits).
__global__ void k_scatter(const float* __restrict__ R, int64_t n, const int32_t* __restrict__ key,
                          const int32_t* __restrict__ start, int32_t* __restrict__ cursor,
                          float4* __restrict__ sorted) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = key[i];
    const int32_t pos = start[c] + atomicAdd(&cursor[c], 1);
    sorted[pos] = make_float4(R[i], R[n + i], R[2 * n + i], __int_as_float((int)i));
  }
}

// (d2, idx) < (e2, jdx) lexicographically
__device__ __forceinline__ bool less_pair(float d2, int i, float e2, int j) {
  return d2 < e2 || (d2 == e2 && i < j);
}

// Insert (d2, j) into the ascending list bd/bi of K entries, dropping the last (fully
// unrolled, register resident). The caller has checked that it beats the last entry.
template <int K>
__device__ __forceinline__ void insert_sorted(float d2, int j, float* bd, int* bi) {
#pragma unroll
  for (int u = K - 1; u >= 1; --u) {
    const bool up = less_pair(d2, j, bd[u - 1], bi[u - 1]);
    const bool here = !up && less_pair(d2, j, bd[u], bi[u]);
    const float nd = up ? bd[u - 1] : (here ? d2 : bd[u]);
    const int ni = up ? bi[u - 1] : (here ? j : bi[u]);
    bd[u] = nd;
    bi[u] = ni;
  }
  if (less_pair(d2, j, bd[0], bi[0])) {
    bd[0] = d2;
    bi[0] = j;
  }
}

// A query of the search: output row q, position, and the reference index it skips (-1: none).
struct KnnQuery {
  int64_t q;
  float x, y, z;
  int skip;
};

// Work item p (see k_knn): the p-th reference in cell order (SELF) or query q0 + p of Q.
template <bool SELF>
__device__ __forceinline__ KnnQuery knn_query_of(int64_t p, const float* __restrict__ Q, int64_t qld, int64_t q0,
                                                 const float4* __restrict__ sorted, int skip_mode, int64_t stride) {
  KnnQuery k;
  int64_t gq;
  if (SELF) {
    const float4 sp = sorted[p];
    k.q = gq = __float_as_int(sp.w);
    k.x = sp.x;
    k.y = sp.y;
    k.z = sp.z;
  } else {
    k.q = p;
    gq = q0 + p;
    k.x = Q[gq];
    k.y = Q[qld + gq];
    k.z = Q[2 * qld + gq];
  }
  k.skip = -1;
  if (skip_mode == 1) k.skip = (int)gq;
  if (skip_mode == 2 && (gq % stride) == 0) k.skip = (int)(gq / stride);
  return k;
}

// The cells of ring r (the cube of half-width r around cell (cx, cy, cz) minus the cube of
// half-width r - 1) in the grid row (z, y), as at most two ranges [b0, e0), [b1, e1) of
// `sorted`: the whole row [xl, xh] (clipped to the grid) when |z - cz| or |y - cy| is r, else
// its end cells cx - r and cx + r where they are inside the grid. The cells of a row are
// consecutive, so a range costs two loads of `start` however many cells it spans.
__device__ __forceinline__ void ring_row(const GridParams& g, const int32_t* __restrict__ start, int cx, int cy,
                                         int cz, int r, int z, int y, int xl, int xh, int32_t& b0, int32_t& e0,
                                         int32_t& b1, int32_t& e1) {
  const int64_t row = ((int64_t)z * g.ny + y) * g.nx;
  b0 = e0 = b1 = e1 = 0;
  if (z == cz - r || z == cz + r || y == cy - r || y == cy + r) {
    b0 = start[row + xl];
    e0 = start[row + xh + 1];
    return;
  }
  if (cx - r >= 0) {
    b0 = start[row + cx - r];
    e0 = start[row + cx - r + 1];
  }
  if (r > 0 && cx + r <= g.nx - 1) {
    b1 = start[row + cx + r];
    e1 = start[row + cx + r + 1];
  }
}

// skip_mode: 0 none; 1 reference i == query i; 2 reference i / stride when i % stride == 0.
// Queries q = 0..m-1 are points q0 + q of the planar array Q with leading dimension qld;
// results go to idx[q][K], dist[q][K].
// SELF: the queries are the references themselves (m = their count, skip_mode 1): work item p
// takes the p-th reference in cell order from `sorted` and writes the row of its original
// index, so the lanes of a wavefront search neighbouring cells (same results, in another
// order of work).
// Two passes, so that a few isolated queries (outliers, whose search spans thousands of
// cells) do not hold up the wavefronts of everyone else: k_knn (one thread per work item p)
// searches rings 0..rcap and appends the items it has not finished to defer[1..] (defer[0]
// counts them); k_knn_wave then searches each deferred item with a whole wavefront. A query's
// result, the k smallest (distance^2, index) pairs, does not depend on the order in which
// candidates are met, so it is the same whichever pass finishes it.
template <int K, bool SELF>
__global__ __launch_bounds__(256) void k_knn(const float* __restrict__ Q, int64_t qld, int64_t q0,
                                             int64_t m, const GridParams* __restrict__ gp,
                                             const int32_t* __restrict__ start,
                                             const float4* __restrict__ sorted, int skip_mode,
                                             int64_t stride, int rcap, int32_t* __restrict__ defer,
                                             int32_t* __restrict__ idx, float* __restrict__ dist) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  const GridParams g = *gp;
  const KnnQuery kq = knn_query_of<SELF>(p, Q, qld, q0, sorted, skip_mode, stride);
  const int64_t q = kq.q;
  const float qx = kq.x, qy = kq.y, qz = kq.z;
  const int skip = kq.skip;
  float bd[K];
  int bi[K];
#pragma unroll
  for (int s = 0; s < K; ++s) {
    bd[s] = INFINITY;
    bi[s] = 0x7fffffff;
  }
  int cx, cy, cz;
  cell_of(g, qx, qy, qz, cx, cy, cz);
  const int rmax = max(g.nx, max(g.ny, g.nz));
  // Rings 0..rcap, a row of cells at a time (ring_row). Every point outside the cube of
  // half-width r lies more than r h from the query, which ends the search once the k-th best
  // distance is within r h; the cube of half-width rmax holds the whole grid. (A point, or
  // the query, outside the grid's box sits in the border cell that holds its projection onto
  // the box; projecting both onto the box shortens no distance, so the bound still holds.)
  bool done = false;
  const int rlim = min(rcap, rmax);
  for (int r = 0; r <= rlim; ++r) {
    const int zl = max(cz - r, 0), zh = min(cz + r, g.nz - 1);
    const int yl = max(cy - r, 0), yh = min(cy + r, g.ny - 1);
    const int xl = max(cx - r, 0), xh = min(cx + r, g.nx - 1);
    for (int z = zl; z <= zh; ++z) {
      for (int y = yl; y <= yh; ++y) {
        int32_t b0, e0, b1, e1;
        ring_row(g, start, cx, cy, cz, r, z, y, xl, xh, b0, e0, b1, e1);
        for (int seg = 0; seg < 2; ++seg) {
          const int32_t e = seg == 0 ? e0 : e1;
          for (int32_t pp = seg == 0 ? b0 : b1; pp < e; ++pp) {
            const float4 sp = sorted[pp];
            const int j = __float_as_int(sp.w);
            if (j == skip) continue;
            const float ex = sp.x - qx, ey = sp.y - qy, ez = sp.z - qz;
            const float d2 = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
            if (!less_pair(d2, j, bd[K - 1], bi[K - 1])) continue;
            insert_sorted<K>(d2, j, bd, bi);
          }
        }
      }
    }
    const float lb = (float)r * g.h;
    if ((bd[K - 1] < INFINITY && bd[K - 1] <= lb * lb) || r >= rmax) {
      done = true;
      break;
    }
  }
  if (!done) {  // left to k_knn_wave
    defer[1 + atomicAdd(&defer[0], 1)] = (int32_t)p;
    return;
  }
#pragma unroll
  for (int s = 0; s < K; ++s) {
    idx[q * K + s] = bi[s];
    if (dist) dist[q * K + s] = sqrtf(bd[s]);
  }
}

// The items k_knn left unfinished, one wavefront per item (a grid-stride loop over the
// wavefronts of the launch). Ring by ring, the lanes share out the ring's rows of cells
// inside the grid (the rows of k_knn: whole rows where |dz| or |dy| is r, the two end cells
// elsewhere), each walking its row's one or two ranges of `sorted` a point at a time; the
// list of the k best is the same in every lane, and the candidates that beat its last entry
// are inserted one by one in lane order (ballot, then a broadcast of each). The ring test is
// then the exact one of k_knn. The work per ring is bounded by the grid's rows.
template <int K, bool SELF>
__global__ __launch_bounds__(256) void k_knn_wave(const float* __restrict__ Q, int64_t qld, int64_t q0,
                                                  int64_t m, const GridParams* __restrict__ gp,
                                                  const int32_t* __restrict__ start,
                                                  const float4* __restrict__ sorted, int skip_mode,
                                                  int64_t stride, const int32_t* __restrict__ defer,
                                                  int32_t* __restrict__ idx, float* __restrict__ dist) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t nd = defer[0];
  const GridParams g = *gp;
  const int rmax = max(g.nx, max(g.ny, g.nz));
  for (int64_t item = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; item < nd; item += nwaves) {
    const KnnQuery kq = knn_query_of<SELF>(defer[1 + item], Q, qld, q0, sorted, skip_mode, stride);
    const int64_t q = kq.q;
    const float qx = kq.x, qy = kq.y, qz = kq.z;
    const int skip = kq.skip;
    float bd[K];
    int bi[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      bd[u] = INFINITY;
      bi[u] = 0x7fffffff;
    }
    int cx, cy, cz;
    cell_of(g, qx, qy, qz, cx, cy, cz);
    for (int r = 0; r <= rmax; ++r) {
      const int zl = max(cz - r, 0), zh = min(cz + r, g.nz - 1);
      const int yl = max(cy - r, 0), yh = min(cy + r, g.ny - 1);
      const int xl = max(cx - r, 0), xh = min(cx + r, g.nx - 1);
      const int nyr = yh - yl + 1;
      const int64_t rows = (int64_t)(zh - zl + 1) * nyr;
      for (int64_t l0 = 0; l0 < rows; l0 += 64) {
        const int64_t l = l0 + lane;
        int32_t b0 = 0, e0 = 0, b1 = 0, e1 = 0;  // this lane's row: up to two ranges of sorted
        if (l < rows)
          ring_row(g, start, cx, cy, cz, r, zl + (int)(l / nyr), yl + (int)(l % nyr), xl, xh, b0, e0, b1, e1);
        for (;;) {
          const bool has = b0 < e0 || b1 < e1;
          if (__ballot(has) == 0ull) break;
          float d2 = INFINITY;
          int j = 0x7fffffff;
          bool beat = false;
          if (has) {
            const int32_t pp = b0 < e0 ? b0++ : b1++;
            const float4 sp = sorted[pp];
            j = __float_as_int(sp.w);
            const float ex = sp.x - qx, ey = sp.y - qy, ez = sp.z - qz;
            d2 = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
            beat = j != skip && less_pair(d2, j, bd[K - 1], bi[K - 1]);
          }
          unsigned long long mask = __ballot(beat);
          while (mask) {
            const int src = __ffsll((long long)mask) - 1;
            mask &= mask - 1ull;
            const float cd = __shfl(d2, src, 64);
            const int cj = __shfl(j, src, 64);
            if (less_pair(cd, cj, bd[K - 1], bi[K - 1])) insert_sorted<K>(cd, cj, bd, bi);
          }
        }
      }
      const float lb = (float)r * g.h;
      if (bd[K - 1] < INFINITY && bd[K - 1] <= lb * lb) break;
    }
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < K; ++u) {
        idx[q * K + u] = bi[u];
        if (dist) dist[q * K + u] = sqrtf(bd[u]);
      }
    }
  }
}

__global__ void k_delta(const float* __restrict__ dist, int64_t n, int k, float scale,
                        float* __restrict__ delta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int t = 0; t < k; ++t) s += dist[i * k + t];
  delta[i] = scale * (s / (float)k);
}

__global__ void k_gather_anchors(const float* __restrict__ P, int64_t n, int64_t stride, int64_t na,
                                 float* __restrict__ A) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= na) return;
  const int64_t i = a * stride;
  A[a] = P[i];
  A[na + a] = P[n + i];
  A[2 * na + a] = P[2 * n + i];
}

// feat[i][3k + d] = (anchor_k - p_i)_d / s_i, s_i = mean of the 16 anchor distances, for
// the points q0 + i, i = 0..m-1 (idx, dist, feat are chunk-local).
__global__ void k_features(const float* __restrict__ P, int64_t n, int64_t q0, int64_t m,
                           const float* __restrict__ A, int64_t na, const int32_t* __restrict__ idx,
                           const float* __restrict__ dist, float* __restrict__ feat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  float s = 0.0f;
  for (int t = 0; t < DWG_FEAT_K; ++t) s += dist[i * DWG_FEAT_K + t];
  s *= (1.0f / DWG_FEAT_K);
  const float is = s > 0.0f ? 1.0f / s : 0.0f;
  const int64_t gi = q0 + i;
  const float px = P[gi], py = P[n + gi], pz = P[2 * n + gi];
  for (int t = 0; t < DWG_FEAT_K; ++t) {
    const int64_t a = idx[i * DWG_FEAT_K + t];
    feat[i * DWG_MLP_IN + 3 * t + 0] = (A[a] - px) * is;
    feat[i * DWG_MLP_IN + 3 * t + 1] = (A[na + a] - py) * is;
    feat[i * DWG_MLP_IN + 3 * t + 2] = (A[2 * na + a] - pz) * is;
  }
}

constexpr int kBboxBlocks = 256;

int64_t max_cells_for(int64_t nr) { return std::max<int64_t>(8 * nr, 64); }

// Unit eigenvector of the smallest eigenvalue of a symmetric 3x3 matrix (FP64): eigenvalues
// by the trigonometric solution of the characteristic cubic (Smith, CACM 1961), the vector
// as the largest cross product of two rows of (A - lambda I), sign left as it falls. An
// isotropic matrix gives (0, 0, 1).
__device__ void smallest_eigvec(const double a[6], double v[3]) {
  const double a00 = a[0], a01 = a[1], a02 = a[2], a11 = a[3], a12 = a[4], a22 = a[5];
  const double p1 = a01 * a01 + a02 * a02 + a12 * a12;
  const double q = (a00 + a11 + a22) / 3.0;
  const double p2 = (a00 - q) * (a00 - q) + (a11 - q) * (a11 - q) + (a22 - q) * (a22 - q) + 2.0 * p1;
  const double p = sqrt(p2 / 6.0);
  v[0] = 0.0;
  v[1] = 0.0;
  v[2] = 1.0;
  if (!(p > 0.0)) return;
  const double b00 = (a00 - q) / p, b11 = (a11 - q) / p, b22 = (a22 - q) / p;
  const double b01 = a01 / p, b02 = a02 / p, b12 = a12 / p;
  double r = 0.5 * (b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) + b02 * (b01 * b12 - b11 * b02));
  r = fmin(1.0, fmax(-1.0, r));
  const double phi = acos(r) / 3.0;
  const double lam = q + 2.0 * p * cos(phi + 2.0943951023931954923);  // smallest
  const double r0[3] = {a00 - lam, a01, a02}, r1[3] = {a01, a11 - lam, a12}, r2[3] = {a02, a12, a22 - lam};
  double c[3][3];
  const double* rows[3][2] = {{r0, r1}, {r0, r2}, {r1, r2}};
  int best = 0;
  double bn = -1.0;
  for (int t = 0; t < 3; ++t) {
    const double* x = rows[t][0];
    const double* y = rows[t][1];
    c[t][0] = x[1] * y[2] - x[2] * y[1];
    c[t][1] = x[2] * y[0] - x[0] * y[2];
    c[t][2] = x[0] * y[1] - x[1] * y[0];
    const double nn = c[t][0] * c[t][0] + c[t][1] * c[t][1] + c[t][2] * c[t][2];
    if (nn > bn) {
      bn = nn;
      best = t;
    }
  }
  if (!(bn > 0.0)) return;
  const double inv = 1.0 / sqrt(bn);
  v[0] = c[best][0] * inv;
  v[1] = c[best][1] * inv;
  v[2] = c[best][2] * inv;
}

// PCA normals (Sec. 5.1 "Normal Initialization"): covariance of p_i and its k nearest other
// points about their mean (FP64), eigenvector of the smallest eigenvalue, turned to point away
// from the origin (n . p_i > 0; at n . p_i == 0 the largest-magnitude component positive).
__global__ void k_pca_normals(const float* __restrict__ P, int64_t n, const int32_t* __restrict__ idx, int k,
                              float* __restrict__ N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double mx = P[i], my = P[n + i], mz = P[2 * n + i];
  for (int t = 0; t < k; ++t) {
    const int64_t j = idx[i * k + t];
    mx += P[j];
    my += P[n + j];
    mz += P[2 * n + j];
  }
  const double inv = 1.0 / (double)(k + 1);
  mx *= inv;
  my *= inv;
  mz *= inv;
  double a[6] = {0, 0, 0, 0, 0, 0};
  for (int t = -1; t < k; ++t) {
    const int64_t j = t < 0 ? i : (int64_t)idx[i * k + t];
    const double x = P[j] - mx, y = P[n + j] - my, z = P[2 * n + j] - mz;
    a[0] += x * x;
    a[1] += x * y;
    a[2] += x * z;
    a[3] += y * y;
    a[4] += y * z;
    a[5] += z * z;
  }
  double v[3];
  smallest_eigvec(a, v);
  double s = v[0] * P[i] + v[1] * P[n + i] + v[2] * P[2 * n + i];
  if (s == 0.0) {
    const double m0 = fabs(v[0]), m1 = fabs(v[1]), m2 = fabs(v[2]);
    s = (m0 >= m1 && m0 >= m2) ? v[0] : (m1 >= m2 ? v[1] : v[2]);
  }
  if (s < 0.0) {
    v[0] = -v[0];
    v[1] = -v[1];
    v[2] = -v[2];
  }
  N[i] = (float)v[0];
  N[n + i] = (float)v[1];
  N[2 * n + i] = (float)v[2];
}

// Area weight of p_i (Sec. 5.1 "Computing Area Weights"): the plane through p_i normal to the
// smallest-eigenvalue eigenvector of the covariance of p_i and its m nearest other points
// (FP64), those points projected onto it, and the area of p_i's cell in the 2D Voronoi
// diagram of the projections: the square [-R, R]^2 (R = the largest projected distance, which
// bounds the cell of a point whose neighbours lie on one side) cut by the half-planes
// x . q_j <= |q_j|^2 / 2; the square's axes are u = n x e_k / |n x e_k| (e_k the axis with the
// smallest |n_k|, the first on ties) and n x u. Coincident neighbours (q_j = 0) bound nothing
// and are skipped; all-coincident neighbourhoods give 0.
__global__ __launch_bounds__(128) void k_voronoi_area(const float* __restrict__ P, int64_t n,
                                                     const int32_t* __restrict__ idx, int m,
                                                     float* __restrict__ area) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double px = P[i], py = P[n + i], pz = P[2 * n + i];
  double mx = px, my = py, mz = pz;
  for (int t = 0; t < m; ++t) {
    const int64_t j = idx[i * m + t];
    mx += P[j];
    my += P[n + j];
    mz += P[2 * n + j];
  }
  const double inv = 1.0 / (double)(m + 1);
  mx *= inv;
  my *= inv;
  mz *= inv;
  double a[6] = {0, 0, 0, 0, 0, 0};
  for (int t = -1; t < m; ++t) {
    const int64_t j = t < 0 ? i : (int64_t)idx[i * m + t];
    const double x = P[j] - mx, y = P[n + j] - my, z = P[2 * n + j] - mz;
    a[0] += x * x;
    a[1] += x * y;
    a[2] += x * z;
    a[3] += y * y;
    a[4] += y * z;
    a[5] += z * z;
  }
  double nv[3];
  smallest_eigvec(a, nv);
  // orthonormal basis (u, w) of the plane: u = nv x (the axis least aligned with nv)
  const double ax = fabs(nv[0]), ay = fabs(nv[1]), az = fabs(nv[2]);
  const double e0 = (ax <= ay && ax <= az) ? 1.0 : 0.0;
  const double e1 = (e0 == 0.0 && ay <= az) ? 1.0 : 0.0;
  const double e2 = (e0 == 0.0 && e1 == 0.0) ? 1.0 : 0.0;
  double u0 = nv[1] * e2 - nv[2] * e1, u1 = nv[2] * e0 - nv[0] * e2, u2 = nv[0] * e1 - nv[1] * e0;
  const double ul = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
  u0 /= ul;
  u1 /= ul;
  u2 /= ul;
  const double w0 = nv[1] * u2 - nv[2] * u1, w1 = nv[2] * u0 - nv[0] * u2, w2 = nv[0] * u1 - nv[1] * u0;
  double qx[kMaxK], qy[kMaxK];  // unrolled to the compile-time maximum: register resident
  double R = 0.0;
#pragma unroll
  for (int t = 0; t < kMaxK; ++t) {
    qx[t] = qy[t] = 0.0;
    if (t < m) {
      const int64_t j = idx[i * m + t];
      const double dx = P[j] - px, dy = P[n + j] - py, dz = P[2 * n + j] - pz;
      qx[t] = dx * u0 + dy * u1 + dz * u2;
      qy[t] = dx * w0 + dy * w1 + dz * w2;
      const double r = sqrt(qx[t] * qx[t] + qy[t] * qy[t]);
      R = r > R ? r : R;
    }
  }
  if (!(R > 0.0)) {
    area[i] = 0.0f;
    return;
  }
  // Cell = the square [-R, R]^2 cut by the half-planes x . q_t <= |q_t|^2 / 2 (the bisectors
  // with the projected neighbours). The origin lies strictly inside every constraint, so the
  // cell is star-shaped about it and its area is the sum over its edges of
  // (1/2) x (distance of the edge's line from the origin) x (edge length). Each line's edge is
  // the interval of the line that the other constraints leave: with x = f + s tau (f the foot
  // of the perpendicular from the origin, tau = (-n_y, n_x)), a constraint n_u . x <= b_u bounds
  // s from one side, and the edge contributes b_t (s_max - s_min) / 2. A line repeated exactly
  // (a repeated neighbour) counts once; a coincident neighbour (q = 0) bounds nothing. The
  // loops run to the compile-time maximum, so the lines stay in registers.
  constexpr int kLines = kMaxK + 4;  // neighbour bisectors, then the square's 4 edges
  auto line_of = [&](int t, double& nx, double& ny, double& b) {
    if (t < kMaxK) {
      nx = t < m ? qx[t] : 0.0;
      ny = t < m ? qy[t] : 0.0;
      b = 0.5 * (nx * nx + ny * ny);  // 0: no constraint
    } else {
      const int e = t - kMaxK;
      nx = e == 0 ? 1.0 : (e == 1 ? -1.0 : 0.0);
      ny = e == 2 ? 1.0 : (e == 3 ? -1.0 : 0.0);
      b = R;
    }
  };
  double s2 = 0.0;  // twice the area
  for (int t = 0; t < kLines; ++t) {  // (the inner loop is the unrolled one)
    double ax, ay, bt;
    line_of(t, ax, ay, bt);
    if (bt == 0.0) continue;
    const double l2 = ax * ax + ay * ay;
    const double fx = ax * bt / l2, fy = ay * bt / l2;
    const double tx = -ay, ty = ax;
    double smin = -INFINITY, smax = INFINITY;
    bool empty = false;
#pragma unroll
    for (int u = 0; u < kLines; ++u) {
      if (u == t) continue;
      double nx, ny, bu;
      line_of(u, nx, ny, bu);
      if (bu == 0.0 || empty) continue;
      if (nx == ax && ny == ay && bu == bt) {
        if (u < t) empty = true;  // the same line: only its first copy has an edge
        continue;
      }
      const double den = tx * nx + ty * ny;
      const double num = bu - (fx * nx + fy * ny);
      if (den > 0.0) {
        smax = fmin(smax, num / den);
      } else if (den < 0.0) {
        smin = fmax(smin, num / den);
      } else if (num < 0.0) {
        empty = true;  // parallel and outside
      }
    }
    if (!empty && smax > smin) s2 += bt * (smax - smin);
  }
  area[i] = (float)(0.5 * s2);
}

// Kernel radius of Sec. 5.2 "Poisson Kernels": the mean of the k nearest-neighbour distances
// that lie in [vmin, vmax]; when none does, the mean of all k clamped to [vmin, vmax].
__global__ void k_delta_window(const float* __restrict__ dist, int64_t n, int k, float vmin, float vmax,
                               float* __restrict__ delta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0, all = 0.0;
  int c = 0;
  for (int t = 0; t < k; ++t) {
    const double d = dist[i * k + t];
    all += d;
    if (d >= vmin && d <= vmax) {
      s += d;
      ++c;
    }
  }
  double r = c > 0 ? s / c : all / k;
  if (c == 0) r = r < vmin ? vmin : (r > vmax ? vmax : r);
  delta[i] = (float)r;
}

// Gauss map (Sec. 5.1 "Normal Initialization"): n_i = p_i / |p_i| (about the origin);
// a point at the origin gets (0, 0, 1).
__global__ void k_gauss_normals(const float* __restrict__ P, int64_t n, float* __restrict__ N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = P[i], y = P[n + i], z = P[2 * n + i];
  const double r = sqrt(x * x + y * y + z * z);
  if (r > 0.0) {
    N[i] = (float)(x / r);
    N[n + i] = (float)(y / r);
    N[2 * n + i] = (float)(z / r);
  } else {
    N[i] = 0.0f;
    N[n + i] = 0.0f;
    N[2 * n + i] = 1.0f;
  }
}

unsigned grid_for(int64_t n, int block = 256, int64_t cap = 65535) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, block), cap));
}

// Rings searched by the thread-per-query pass: with about 8 cells per reference point, a query
// on a sampled surface meets its neighbours within 2-3 rings (1M torus scene: the self 10-NN
// finish by ring 2 for 95% of the points, the 16 nearest of 4,096 anchors by ring 3 for 97%);
// its outliers need 4 to 11.
constexpr int kFirstPassRings = 3;

// Blocks of the wavefront-per-item pass (4 wavefronts each): 8 wavefronts per SIMD, so that
// the dependent loads of one item's ring walk overlap with those of others.
constexpr int kWaveBlocks = 2048;

// two_pass = false: the thread-per-query kernel searches every query to the end (no ring
// limit, nothing deferred), for query sets whose order already groups the isolated queries
// together (the level-set faces, emitted cell by cell in Morton order), where a wavefront per
// deferred query would only spread them out.
template <int K, bool SELF>
void launch_knn_t(int64_t m, hipStream_t st, const float* Q, int64_t qld, int64_t q0, const KnnWork& w,
                  int skip_mode, int64_t stride, bool two_pass, int32_t* idx, float* dist) {
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, w.defer, (int64_t)1);
  const int rcap = two_pass ? kFirstPassRings : INT_MAX;
  hipLaunchKernelGGL((k_knn<K, SELF>), dim3((unsigned)cdiv(m, 256)), dim3(256), 0, st, Q, qld, q0, m, w.gp,
                     w.start, w.sorted, skip_mode, stride, rcap, w.defer, idx, dist);
  if (two_pass)
    hipLaunchKernelGGL((k_knn_wave<K, SELF>), dim3(kWaveBlocks), dim3(256), 0, st, Q, qld, q0, m, w.gp, w.start,
                       w.sorted, skip_mode, stride, w.defer, idx, dist);
}

template <int K>
void launch_knn_k(int64_t m, hipStream_t st, const float* Q, int64_t qld, int64_t q0, const KnnWork& w,
                  int skip_mode, int64_t stride, bool self, bool two_pass, int32_t* idx, float* dist) {
  if (self)
    launch_knn_t<K, true>(m, st, Q, qld, q0, w, skip_mode, stride, two_pass, idx, dist);
  else
    launch_knn_t<K, false>(m, st, Q, qld, q0, w, skip_mode, stride, two_pass, idx, dist);
}

dwg_status build_grid(const float* R, int64_t nr, const KnnWork& w, hipStream_t st) {
  const int64_t mc = max_cells_for(nr);
  hipLaunchKernelGGL(k_bbox_partial, dim3(kBboxBlocks), dim3(256), 0, st, R, nr, w.bbox_part);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_trim_init, dim3(1), dim3(256), 0, st, w.bbox_part, kBboxBlocks, w.range, w.below, w.hist);
  DWG_TRY_LAUNCH();
  const int64_t rlo = nr / 1024, rhi = nr - 1 - nr / 1024;
  for (int level = 0; level < kTrimLevels; ++level) {
    hipLaunchKernelGGL(k_axis_hist, dim3(grid_for(nr, 256, 1024)), dim3(256), 0, st, R, nr, w.range, w.hist);
    DWG_TRY_LAUNCH();
    hipLaunchKernelGGL(k_trim_refine, dim3(3), dim3(256), 0, st, w.hist, w.range, w.below, rlo, rhi);
    DWG_TRY_LAUNCH();
  }
  hipLaunchKernelGGL(k_grid_params, dim3(1), dim3(64), 0, st, w.range, mc, w.gp);
  DWG_TRY_LAUNCH();
  // counts and cursors over the largest possible grid (the actual grid has <= mc cells)
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(mc + 1)), dim3(256), 0, st, w.start, mc + 1);
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(mc)), dim3(256), 0, st, w.cursor, mc);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_cell_count, dim3(grid_for(nr)), dim3(256), 0, st, R, nr, w.gp, w.key, w.start);
  DWG_TRY_LAUNCH();
  const int64_t nt = cdiv(mc, kScanTile);
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(kScanBlock), 0, st, w.start, mc, w.sums);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, w.sums, nt, w.start, mc);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)cdiv(mc, 256)), dim3(256), 0, st, w.start, mc, w.sums);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(nr)), dim3(256), 0, st, R, nr, w.key, w.start, w.cursor,
                     w.sorted);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

// self: the queries are exactly the m references of the grid, q0 = 0, skip_mode 1.
dwg_status knn_query(const float* Q, int64_t qld, int64_t q0, int64_t m, const KnnWork& w, int skip_mode,
                     int64_t stride, int k, int32_t* idx, float* dist, hipStream_t st, bool self = false,
                     bool two_pass = true) {
  if (m > w.mq) {  // the deferred list holds at most w.mq items
    set_error("internal: %lld kNN queries exceed the carved capacity %lld", (long long)m, (long long)w.mq);
    return DWG_E_INVALID;
  }
  if (m <= 0) return DWG_OK;
  switch (k) {
#define DWG_K(KK) \
  case KK: launch_knn_k<KK>(m, st, Q, qld, q0, w, skip_mode, stride, self, two_pass, idx, dist); break;
    DWG_K(1) DWG_K(2) DWG_K(3) DWG_K(4) DWG_K(5) DWG_K(6) DWG_K(7) DWG_K(8)
    DWG_K(9) DWG_K(10) DWG_K(11) DWG_K(12) DWG_K(13) DWG_K(14) DWG_K(15) DWG_K(16)
#undef DWG_K
    default: set_error("k out of range"); return DWG_E_INVALID;
  }
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

}  // namespace

dwg_status knn_grid(const float* R, int64_t nr, const KnnWork& w, hipStream_t st) { return build_grid(R, nr, w, st); }

dwg_status knn_search(const float* Q, int64_t qld, int64_t q0, int64_t m, const KnnWork& w, int k, int32_t* idx,
                      float* dist, hipStream_t st) {
  return knn_query(Q, qld, q0, m, w, 0, 1, k, idx, dist, st, false, false);
}

size_t carve_knn(Carver& c, int64_t nr, int64_t mq, KnnWork* out) {
  const int64_t mc = max_cells_for(nr);
  const size_t s0 = c.used;
  KnnWork w;
  w.mq = mq;
  w.defer = c.take<int32_t>((size_t)mq + 1);
  w.bbox_part = c.take<float>(kBboxBlocks * 6);
  w.range = c.take<double>(6);
  w.below = c.take<int64_t>(3);
  w.hist = c.take<int32_t>(3 * kTrimBins);
  w.gp = c.take<GridParams>(1);
  w.key = c.take<int32_t>((size_t)nr);
  w.start = c.take<int32_t>((size_t)mc + 1);
  w.cursor = c.take<int32_t>((size_t)mc);
  w.sums = c.take<int32_t>((size_t)cdiv(mc, kScanTile) + 1);
  w.sorted = c.take<float4>((size_t)nr);
  if (out) *out = w;
  return c.used - s0;
}

dwg_status launch_bbox(const float* R, int64_t n, float* part, float* out6, hipStream_t st) {
  hipLaunchKernelGGL(k_bbox_partial, dim3(kBboxBlocks), dim3(256), 0, st, R, n, part);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, st, part, kBboxBlocks, out6);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

size_t scan_sums_len(int64_t n) { return (size_t)cdiv(n, kScanTile) + 1; }

dwg_status exclusive_scan(int32_t* a, int64_t n, int32_t* sums, hipStream_t st) {
  const int64_t nt = cdiv(n, kScanTile);
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(kScanBlock), 0, st, a, n, sums);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, sums, nt, a, n);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, a, n, sums);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

size_t knn_ws_bytes(int64_t n_ref, int64_t n_qry) {
  (void)n_qry;
  Carver c(nullptr);
  carve_knn(c, n_ref, n_qry, nullptr);
  return c.used;
}

dwg_status knn_run(const float* R, int64_t nr, const float* Q, int64_t m, int self_skip,
                   const int64_t* skip_stride, int k, int32_t* idx, float* dist, void* ws,
                   size_t ws_bytes, hipStream_t stream) {
  (void)ws_bytes;
  (void)skip_stride;
  Carver c(ws);
  KnnWork w;
  carve_knn(c, nr, m, &w);
  dwg_status s = build_grid(R, nr, w, stream);
  if (s != DWG_OK) return s;
  // queries that are the references themselves (same array, same count) run in cell order
  const bool self = self_skip && Q == R && m == nr;
  return knn_query(Q, m, 0, m, w, self_skip ? 1 : 0, 1, k, idx, dist, stream, self);
}

dwg_status delta_from_knn(const float* dist, int64_t n, int k, float scale, float* delta,
                          hipStream_t stream) {
  hipLaunchKernelGGL(k_delta, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, stream, dist, n, k, scale, delta);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

size_t anchor_ws_bytes(int64_t n, int64_t chunk, int64_t n_anchor) {
  Carver c(nullptr);
  AnchorCtx x;
  carve_anchor(c, n, chunk, n_anchor, &x);
  return c.used;
}

size_t carve_anchor(Carver& c, int64_t n, int64_t chunk, int64_t n_anchor, AnchorCtx* out) {
  const size_t s0 = c.used;
  AnchorCtx x;
  x.stride = std::max<int64_t>(1, n / std::max<int64_t>(n_anchor, 1));
  x.na = cdiv(n, x.stride);
  x.chunk = chunk;
  x.A = c.take<float>(3 * (size_t)x.na);
  x.idx = c.take<int32_t>((size_t)chunk * DWG_FEAT_K);
  x.dist = c.take<float>((size_t)chunk * DWG_FEAT_K);
  x.feat = c.take<float>((size_t)chunk * DWG_MLP_IN);
  carve_knn(c, x.na, chunk, &x.w);
  if (out) *out = x;
  return c.used - s0;
}

dwg_status pca_normals(const float* P, int64_t n, int k, float* N, void* ws, hipStream_t stream) {
  Carver c(ws);
  int32_t* idx = c.take<int32_t>((size_t)n * k);
  float* dist = c.take<float>((size_t)n * k);
  dwg_status s = knn_run(P, n, P, n, 1, nullptr, k, idx, dist, static_cast<char*>(ws) + c.used, 0, stream);
  if (s != DWG_OK) return s;
  hipLaunchKernelGGL(k_pca_normals, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, stream, P, n, idx, k, N);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status voronoi_area(const float* P, int64_t n, int m, float* area, void* ws, hipStream_t stream) {
  Carver c(ws);
  int32_t* idx = c.take<int32_t>((size_t)n * m);
  float* dist = c.take<float>((size_t)n * m);
  dwg_status s = knn_run(P, n, P, n, 1, nullptr, m, idx, dist, static_cast<char*>(ws) + c.used, 0, stream);
  if (s != DWG_OK) return s;
  hipLaunchKernelGGL(k_voronoi_area, dim3((unsigned)cdiv(n, 128)), dim3(128), 0, stream, P, n, idx, m, area);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status delta_window(const float* P, int64_t n, int k, float vmin, float vmax, float* delta, void* ws,
                        hipStream_t stream) {
  Carver c(ws);
  int32_t* idx = c.take<int32_t>((size_t)n * k);
  float* dist = c.take<float>((size_t)n * k);
  dwg_status s = knn_run(P, n, P, n, 1, nullptr, k, idx, dist, static_cast<char*>(ws) + c.used, 0, stream);
  if (s != DWG_OK) return s;
  hipLaunchKernelGGL(k_delta_window, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, stream, dist, n, k, vmin, vmax,
                     delta);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status gauss_normals(const float* P, int64_t n, float* N, hipStream_t stream) {
  hipLaunchKernelGGL(k_gauss_normals, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, stream, P, n, N);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

// Anchors: every stride-th point, stride = max(1, n / n_anchor); grid over the anchors.
dwg_status anchor_build(const float* P, int64_t n, const AnchorCtx& x, hipStream_t stream) {
  hipLaunchKernelGGL(k_gather_anchors, dim3((unsigned)cdiv(x.na, 256)), dim3(256), 0, stream, P, n, x.stride,
                     x.na, x.A);
  DWG_TRY_LAUNCH();
  return build_grid(x.A, x.na, x.w, stream);
}

// Features of the points q0 .. q0 + m - 1 (m <= chunk) into feat [m][48].
dwg_status anchor_features(const float* P, int64_t n, int64_t q0, int64_t m, const AnchorCtx& x, float* feat,
                           hipStream_t stream) {
  dwg_status s = knn_query(P, n, q0, m, x.w, 2, x.stride, DWG_FEAT_K, x.idx, x.dist, stream);
  if (s != DWG_OK) return s;
  hipLaunchKernelGGL(k_features, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, stream, P, n, q0, m, x.A, x.na,
                     x.idx, x.dist, feat);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

// delta_i = scale x mean distance from p_i to its k nearest anchors (the anchor i itself
// excluded), for all points in chunks of x.chunk.
dwg_status anchor_delta(const float* P, int64_t n, const AnchorCtx& x, int k, float scale, float* delta,
                        hipStream_t stream) {
  for (int64_t q0 = 0; q0 < n; q0 += x.chunk) {
    const int64_t cnt = std::min<int64_t>(x.chunk, n - q0);
    dwg_status s = knn_query(P, n, q0, cnt, x.w, 2, x.stride, k, x.idx, x.dist, stream);
    if (s != DWG_OK) return s;
    s = delta_from_knn(x.dist, cnt, k, scale, delta + q0, stream);
    if (s != DWG_OK) return s;
  }
  return DWG_OK;
}

dwg_status features_run(const float* P, int64_t n, int64_t n_anchor, float* feat, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
  (void)ws_bytes;
  Carver c(ws);
  AnchorCtx x;
  carve_anchor(c, n, n, n_anchor, &x);
  dwg_status s = anchor_build(P, n, x, stream);
  if (s != DWG_OK) return s;
  return anchor_features(P, n, 0, n, x, feat, stream);
}

}  // namespace dwg
