// Spatial order of the points for the all-pairs kernel.
//
// Sort key = (radius class, Morton code of the point's cell in a 128^3 grid over the bounding
// box). Radius class 1 holds points whose kernel radius max(delta, eps) exceeds 4 x the mean
// radius (outliers, sparse regions): grouped at the end, their large radii do not spoil the
// near/far test of the tiles of dense surface points. The (key, index) pairs go through the
// stable LSD radix sort (3 passes of 8 bits over the 22-bit key): equal keys keep ascending
// indices, so the permutation is deterministic, and the cost is linear in n whatever the
// distribution (every point in one cell included).
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
                            const float* __restrict__ box, uint64_t* __restrict__ key, int32_t* __restrict__ val) {
  const float ox = box[0], oy = box[1], oz = box[2];
  const float ext = fmaxf(fmaxf(box[3] - ox, box[4] - oy), fmaxf(box[5] - oz, 1e-30f));
  const float sc = 128.0f / ext;
  const float thr = 4.0f * box[6];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t cx = (uint32_t)min(max((int)((P[i] - ox) * sc), 0), 127);
    const uint32_t cy = (uint32_t)min(max((int)((P[n + i] - oy) * sc), 0), 127);
    const uint32_t cz = (uint32_t)min(max((int)((P[2 * n + i] - oz) * sc), 0), 127);
    const uint32_t cls = radius_of(D, i, eps) > thr ? 1u : 0u;
    key[i] = (uint64_t)((cls << 21) | (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz));
    val[i] = (int32_t)i;
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
  w.key[0] = c.take<uint64_t>((size_t)n);
  w.key[1] = c.take<uint64_t>((size_t)n);
  w.val = c.take<int32_t>((size_t)n);
  w.hist = c.take<int32_t>(radix_hist_len(n));
  w.hsums = c.take<int32_t>(scan_sums_len((int64_t)radix_hist_len(n)));
  if (out) *out = w;
  return c.used - s0;
}

dwg_status spatial_sort(const float* P, int64_t n, const float* delta, float eps, const SortWork& w,
                        int32_t* perm, hipStream_t st) {
  dwg_status s = launch_bbox(P, n, w.part, w.box, st);
  if (s != DWG_OK) return s;
  hipLaunchKernelGGL(k_radius_partial, dim3(256), dim3(256), 0, st, delta, n, eps, w.rpart);
  hipLaunchKernelGGL(k_radius_mean, dim3(1), dim3(64), 0, st, w.rpart, 256, n, w.box);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_sort_keys, dim3(grid_n(n)), dim3(256), 0, st, P, n, delta, eps, w.box, w.key[0], w.val);
  DWG_TRY_LAUNCH();
  // three passes (a 22-bit key) leave the sorted pairs in the second buffers: perm
  static_assert((kSortKeyBits + 7) / 8 == 3, "an odd number of passes ends in the second buffers");
  int32_t* const vals[2] = {w.val, perm};
  int res = 0;
  return radix_sort_pairs(w.key, vals, n, kSortKeyBits, w.hist, w.hsums, &res, st);
}

}  // namespace dwg
