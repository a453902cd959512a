// 63-bit Morton codes of the octree frame shared by the octree and the grid code: the cell
// of a point at level 21 is floor((x - lo) * 2^21 / side) per axis (FP64, explicit rounding
// so that no multiply-add is fused), clamped to [0, 2^21 - 1]; x is the most significant
// bit of each interleaved triple.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dwg {
namespace morton {

constexpr int kDepth = 21;

__device__ __forceinline__ uint64_t spread21(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ int compact21(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x1fffffull;
  return (int)x;
}

__device__ __forceinline__ uint64_t code3(uint64_t x, uint64_t y, uint64_t z) {
  return (spread21(x) << 2) | (spread21(y) << 1) | spread21(z);
}

// Level-21 cell of point i of the planar [3][n] array P; frame = (lo xyz, 2^21 / side), a
// zero scale (all points equal) gives cell 0.
__device__ __forceinline__ void cell21(const float* __restrict__ P, int64_t n, int64_t i,
                                       const double* __restrict__ frame, int c[3]) {
  const double sc = frame[3];
  for (int d = 0; d < 3; ++d) {
    double f = 0.0;
    if (sc > 0.0) {
      f = floor(__dmul_rn(__dsub_rn((double)P[d * n + i], frame[d]), sc));
      f = f < 0.0 ? 0.0 : (f > 2097151.0 ? 2097151.0 : f);
    }
    c[d] = (int)f;
  }
}

}  // namespace morton
}  // namespace dwg
