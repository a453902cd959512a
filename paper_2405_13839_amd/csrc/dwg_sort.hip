// Spatial order of the points for the all-pairs kernel.
//
// Sort key = (radius class, Morton code of the point's cell in a 128^3 grid over the bounding
// box). Radius class 1 holds points whose kernel radius max(delta, eps) exceeds 4 x the mean
// radius (outliers, sparse regions): grouped at the end, their large radii do not spoil the
// near/far test of the tiles of dense surface points. Counting sort over 2 x 2^21 bins with
// atomic cursors, then every bin's indices are put in ascending order, so the permutation does
// not depend on the order in which atomics were served.
#include <cmath>

#include "dwg_internal.h"

namespace dwg {
namespace {

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x7fu;
  v = (v | (v << 8)) & 0x0000f00fu;
  v = (v | (v << 4)) & 0x000c30c3u;
  v = (v | (v << 2)) & 0x00249249u;
  return v;
}

__device__ __forceinline__ float radius_of(const float* D, int64_t j, float eps) {
  const float d = D ? D[j] : 0.0f;
  return d > eps ? d : eps;
}

__global__ __launch_bounds__(256) void k_radius_partial(const float* __restrict__ D, int64_t n, float eps,
                                                        double* __restrict__ part) {
  __shared__ double lds[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += (double)radius_of(D, i, eps);
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) lds[threadIdx.x] += lds[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = lds[0];
}

__global__ void k_radius_mean(const double* __restrict__ part, int nb, int64_t n, float* __restrict__ box) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[b];
  box[6] = (float)(s / (double)n);
}

__global__ void k_sort_keys(const float* __restrict__ P, int64_t n, const float* __restrict__ D, float eps,
                            const float* __restrict__ box, uint32_t* __restrict__ key, int32_t* __restrict__ bins) {
  const float ox = box[0], oy = box[1], oz = box[2];
  const float ext = fmaxf(fmaxf(box[3] - ox, box[4] - oy), fmaxf(box[5] - oz, 1e-30f));
  const float sc = 128.0f / ext;
  const float thr = 4.0f * box[6];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t cx = (uint32_t)min(max((int)((P[i] - ox) * sc), 0), 127);
    const uint32_t cy = (uint32_t)min(max((int)((P[n + i] - oy) * sc), 0), 127);
    const uint32_t cz = (uint32_t)min(max((int)((P[2 * n + i] - oz) * sc), 0), 127);
    const uint32_t cls = radius_of(D, i, eps) > thr ? 1u : 0u;
    const uint32_t k = (cls << 21) | (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
    key[i] = k;
    atomicAdd(&bins[k], 1);
  }
}

__global__ void k_zero(int32_t* __restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

__global__ void k_sort_scatter(const uint32_t* __restrict__ key, int64_t n, const int32_t* __restrict__ start,
                               int32_t* __restrict__ cursor, int32_t* __restrict__ perm) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = key[i];
    perm[start[k] + atomicAdd(&cursor[k], 1)] = (int32_t)i;
  }
}

// Ascending indices inside every bin (insertion sort; bins hold few points).
__global__ void k_bin_sort(const int32_t* __restrict__ start, int64_t nbins, int32_t* __restrict__ perm) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nbins; b += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = start[b], e = start[b + 1];
    for (int32_t i = s + 1; i < e; ++i) {
      const int32_t v = perm[i];
      int32_t j = i - 1;
      while (j >= s && perm[j] > v) {
        perm[j + 1] = perm[j];
        --j;
      }
      perm[j + 1] = v;
    }
  }
}

unsigned grid_n(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 16384)); }

}  // namespace

size_t carve_sort(Carver& c, int64_t n, SortWork* out) {
  const size_t s0 = c.used;
  SortWork w;
  w.part = c.take<float>(kBboxParts);
  w.box = c.take<float>(8);
  w.rpart = c.take<double>(256);
  w.key = c.take<uint32_t>((size_t)n);
  w.bins = c.take<int32_t>((size_t)kSortBins + 1);
  w.cursor = c.take<int32_t>((size_t)kSortBins);
  w.sums = c.take<int32_t>(scan_sums_len(kSortBins));
  if (out) *out = w;
  return c.used - s0;
}

dwg_status spatial_sort(const float* P, int64_t n, const float* delta, float eps, const SortWork& w,
                        int32_t* perm, hipStream_t st) {
  dwg_status s = launch_bbox(P, n, w.part, w.box, st);
  if (s != DWG_OK) return s;
  hipLaunchKernelGGL(k_radius_partial, dim3(256), dim3(256), 0, st, delta, n, eps, w.rpart);
  hipLaunchKernelGGL(k_radius_mean, dim3(1), dim3(64), 0, st, w.rpart, 256, n, w.box);
  hipLaunchKernelGGL(k_zero, dim3(grid_n(kSortBins + 1)), dim3(256), 0, st, w.bins, kSortBins + 1);
  hipLaunchKernelGGL(k_zero, dim3(grid_n(kSortBins)), dim3(256), 0, st, w.cursor, kSortBins);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_sort_keys, dim3(grid_n(n)), dim3(256), 0, st, P, n, delta, eps, w.box, w.key, w.bins);
  DWG_TRY_LAUNCH();
  s = exclusive_scan(w.bins, kSortBins, w.sums, st);
  if (s != DWG_OK) return s;
  hipLaunchKernelGGL(k_sort_scatter, dim3(grid_n(n)), dim3(256), 0, st, w.key, n, w.bins, w.cursor, perm);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_bin_sort, dim3(grid_n(kSortBins)), dim3(256), 0, st, w.bins, kSortBins, perm);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

}  // namespace dwg
