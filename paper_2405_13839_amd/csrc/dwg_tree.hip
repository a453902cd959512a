// Octree evaluation of the (screened) GWN and its gradient (Sec. 5.2 "Octree Traversal",
// after the fast winding numbers of Barill et al. 2018).
//
// Octree. The root cell is the cube [lo, lo + ext]^3 (lo = per-axis minimum of the sources,
// ext = largest per-axis extent). A source's cell at the deepest level D = 21 has integer
// coordinates floor((x - lo) * 2^21 / ext) clamped to [0, 2^21 - 1], computed in FP64; its
// 63-bit Morton code interleaves them with x the most significant bit of each triple.
// Sources are sorted by (code, index). A node is a non-empty cell, a leaf when it holds at
// most `leaf` sources or sits at level D; a cell whose sources all lie in one child cell is
// represented by the deepest cell of that chain (same sources, so the same summaries and
// decisions), which bounds the node count by 2n - 1. Nodes are numbered in depth-first
// pre-order; a node's first child is the next node and `skip` is the first node after its
// subtree.
//
// Build (once per source set), all flat and deterministic:
//   codes -> stable LSD radix sort (8 passes of 8 bits; ranks inside a block from wave
//   ballots) -> per sorted source, the range of levels of the nodes that start there ->
//   exclusive scan -> nodes in pre-order. A node at level L starting at sorted position i
//   exists iff i starts its level-L cell and the parent cell holds more than `leaf`
//   sources; the deepest level at which the cell of i holds more than `leaf` sources is the
//   largest shared prefix of the codes at positions (j, j + leaf) over windows containing i.
// Node summaries (Sec. 5.2): area A and area-weighted centre c.m, FP64 sums over chunks of
// 256 sorted sources added in chunk order; r = largest |p_j - c.m| (FP64, max over chunks);
// dmax = largest kernel radius max(delta_j, eps); opening radius crit = max(beta r, r + dmax)
// (the second term keeps every source of a far node outside its clamp radius). Per
// iteration, the moment M = sum m_j (m_j = a_j n_j / 4 pi, FP64 prefix sums of the staged
// FP32 moments).
//
// Traversal. One wavefront walks the pre-order node list with one node index for all 64 of
// its queries (sorted, so they are neighbours) and per-lane "skip until" indices: a lane
// for which node i is far adds the node's dipole and ignores the rest of its subtree; the
// wave descends (i + 1) when any active lane must open node i, sums a leaf's sources for the
// lanes that opened it, and otherwise jumps to skip. Every query thus sees exactly the
// per-query decisions of the paper's depth-first traversal; node loads are wave-uniform.
// A leaf opened by at most half of the lanes is spread over the idle ones (groups of lanes
// each take every k-th source for one query; partial sums return through LDS).
// The FP64 criterion |q - c.m|^2 > crit^2 decides (unscaled); the far dipole and the leaf
// pairs use the FP32 pair arithmetic of the all-pairs kernel in its scaled coordinates (leaf
// pairs from positions staged relative to the leaf's centre).
#include <cmath>

#include "dwg_internal.h"
#include "dwg_morton.h"
#include "dwg_pair.h"

namespace dwg {
namespace {

using namespace pairk;
using morton::kDepth;
constexpr int kSortTile = 2048;  // elements per block of the radix sort (256 threads x 8 rounds)
constexpr int kScanTile = 2048;  // elements per block of the FP64 scans (256 threads x 8)
constexpr int kChunk = 256;      // sources per work item of the radius pass

// Node count written by the build, never above the carved capacity.
__device__ __forceinline__ int64_t node_count(const int32_t* total_p, int64_t cap) {
  const int64_t t = *total_p;
  return t < cap ? t : cap;
}

unsigned grid_cap(int64_t n, int64_t cap = 16384) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), cap));
}

// Number of levels 1..D at which codes a and b share their cell (D when equal).
__device__ __forceinline__ int shared_levels(uint64_t a, uint64_t b) {
  const uint64_t x = a ^ b;
  if (x == 0) return kDepth;
  const int h = 63 - __clzll((long long)x);
  return kDepth - h / 3 - 1;
}

// End (exclusive) of the level-L cell that contains sorted position i.
__device__ int64_t cell_end(const uint64_t* __restrict__ code, int64_t n, int64_t i, int L) {
  if (L == 0) return n;
  const int sh = 3 * (kDepth - L);
  const uint64_t pre = code[i] >> sh;
  int64_t lo = i + 1, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((code[mid] >> sh) == pre)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// frame = (lo x, lo y, lo z, 2^21 / ext), ext = the largest extent (scale 0 when ext == 0).
__global__ void k_tree_frame(const float* __restrict__ box, double* __restrict__ frame) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double ex = (double)box[3] - (double)box[0];
  const double ey = (double)box[4] - (double)box[1];
  const double ez = (double)box[5] - (double)box[2];
  double ext = ex;
  if (ey > ext) ext = ey;
  if (ez > ext) ext = ez;
  frame[0] = box[0];
  frame[1] = box[1];
  frame[2] = box[2];
  frame[3] = ext > 0.0 ? 2097152.0 / ext : 0.0;
}

__global__ void k_tree_keys(const float* __restrict__ P, int64_t n, const double* __restrict__ frame,
                            uint64_t* __restrict__ key, int32_t* __restrict__ val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int c[3];
    morton::cell21(P, n, i, frame, c);
    key[i] = morton::code3(c[0], c[1], c[2]);
    val[i] = (int32_t)i;
  }
}

// Radix sort pass, part 1: per-block digit counts, digit-major: hist[d * nb + b].
__global__ __launch_bounds__(256) void k_rs_hist(const uint64_t* __restrict__ key, int64_t n, int shift,
                                                 int32_t* __restrict__ hist, int64_t nb) {
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kSortTile / 256; ++k) {
    const int64_t i = b0 + k * 256 + threadIdx.x;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Radix sort pass, part 2: stable scatter. Elements of a block are ranked in index order:
// rounds of 256, inside a round by wave, inside a wave by lane (peers with the same digit
// found by 8 ballots).
__global__ __launch_bounds__(256) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                    const int32_t* __restrict__ vin, int64_t n, int shift,
                                                    const int32_t* __restrict__ hist, int64_t nb,
                                                    uint64_t* __restrict__ kout, int32_t* __restrict__ vout) {
  __shared__ int32_t base[256];
  __shared__ int32_t wcnt[4][256];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  base[tid] = hist[(int64_t)tid * nb + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t b0 = (int64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kSortTile / 256; ++k) {
    const int64_t i = b0 + k * 256 + tid;
    const bool valid = i < n;
    uint64_t key = 0;
    int32_t val = 0;
    uint32_t d = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
      d = (uint32_t)(key >> shift) & 255u;
    }
    uint64_t peers = __ballot(valid);
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t bb = __ballot(valid && on);
      peers &= on ? bb : ~bb;
    }
    const int rank = __popcll(peers & lt);
    for (int t = tid; t < 4 * 256; t += 256) (&wcnt[0][0])[t] = 0;
    __syncthreads();
    if (valid && rank == 0) wcnt[wv][d] = __popcll(peers);
    __syncthreads();
    {
      int run = base[tid];
      for (int w = 0; w < 4; ++w) {
        const int c = wcnt[w][tid];
        wcnt[w][tid] = run;
        run += c;
      }
      base[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const int pos = wcnt[wv][d] + rank;
      if (pos < n) {
        kout[pos] = key;
        vout[pos] = val;
      }
    }
    __syncthreads();
  }
}

// Per sorted source i: the levels [ldiff, lend] of the uncompressed nodes starting at i and
// the number of kept (deepest-of-chain) nodes among them.
__global__ void k_tree_mark(const uint64_t* __restrict__ code, int64_t n, int leaf, int32_t* __restrict__ lev,
                            int32_t* __restrict__ cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int ldiff = i == 0 ? 0 : shared_levels(code[i - 1], code[i]) + 1;
    int deep = -1;
    const int64_t j0 = i - leaf > 0 ? i - leaf : 0;
    const int64_t j1 = i < n - 1 - leaf ? i : n - 1 - leaf;
    for (int64_t j = j0; j <= j1; ++j) {
      const int s = shared_levels(code[j], code[j + leaf]);
      deep = s > deep ? s : deep;
    }
    const int lend = deep + 1 < kDepth ? deep + 1 : kDepth;
    int c = 0;
    if (ldiff <= lend) {
      int64_t e = cell_end(code, n, i, ldiff);
      for (int L = ldiff; L < lend; ++L) {
        const int64_t e2 = cell_end(code, n, i, L + 1);
        if (e2 != e) ++c;
        e = e2;
      }
      ++c;
    }
    lev[i] = ldiff | (lend << 8);
    cnt[i] = c;
  }
}

// Writes the kept nodes: (start, end, skip, level | leaf << 8).
__global__ void k_tree_emit(const uint64_t* __restrict__ code, int64_t n, int leaf, const int32_t* __restrict__ lev,
                            const int32_t* __restrict__ off, int64_t cap, int4* __restrict__ node) {
  const int32_t total = off[n];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int ldiff = lev[i] & 255, lend = lev[i] >> 8;
    if (ldiff > lend) continue;
    int64_t k = off[i];
    int64_t e = cell_end(code, n, i, ldiff);
    for (int L = ldiff; L <= lend; ++L) {
      const int64_t e2 = L < lend ? cell_end(code, n, i, L + 1) : -1;
      if (L == lend || e2 != e) {
        if (k < cap) {
          const int skip = e == n ? total : off[e];
          const int lf = (e - i <= leaf || L == kDepth) ? 1 : 0;
          node[k] = make_int4((int)i, (int)e, skip, L | (lf << 8));
        }
        ++k;
      }
      e = e2;
    }
  }
}

// FP64 prefix sums of the staged moments m (K = 3 components) in sorted order: block-local
// exclusive scan.
template <int K>
__global__ __launch_bounds__(256) void k_scan_local(const float4* __restrict__ src, int64_t n,
                                                    double* __restrict__ S, double* __restrict__ blk, int64_t nblk) {
  __shared__ double lds[K][256];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * 8;
  double v[8][K];
  double tot[K];
  for (int c = 0; c < K; ++c) tot[c] = 0.0;
  for (int t = 0; t < 8; ++t) {
    const int64_t j = base + t;
    for (int c = 0; c < K; ++c) v[t][c] = 0.0;
    if (j < n) {
      const float4 b = src[2 * j + 1];
      v[t][0] = b.x;
      v[t][1] = b.y;
      v[t][2] = b.z;
    }
    for (int c = 0; c < K; ++c) tot[c] += v[t][c];
  }
  for (int c = 0; c < K; ++c) lds[c][tid] = tot[c];
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    double add[K];
    for (int c = 0; c < K; ++c) add[c] = tid >= off ? lds[c][tid - off] : 0.0;
    __syncthreads();
    for (int c = 0; c < K; ++c) lds[c][tid] += add[c];
    __syncthreads();
  }
  for (int c = 0; c < K; ++c) {
    double run = tid > 0 ? lds[c][tid - 1] : 0.0;  // exclusive prefix of this thread in the block
    for (int t = 0; t < 8; ++t) {
      const int64_t j = base + t;
      if (j < n) S[c * (n + 1) + j] = run;
      run += v[t][c];
    }
  }
  if (tid == 255)
    for (int c = 0; c < K; ++c) blk[c * nblk + blockIdx.x] = lds[c][255];
}

// Exclusive scan of the block totals (one block, fixed order); S[c][n] = grand total.
template <int K>
__global__ __launch_bounds__(256) void k_scan_tops(double* __restrict__ blk, int64_t nblk, double* __restrict__ S,
                                                   int64_t n) {
  __shared__ double lds[K][256];
  const int tid = threadIdx.x;
  double carry[K];
  for (int c = 0; c < K; ++c) carry[c] = 0.0;
  for (int64_t b0 = 0; b0 < nblk; b0 += 256) {
    const int64_t b = b0 + tid;
    double x[K];
    for (int c = 0; c < K; ++c) {
      x[c] = b < nblk ? blk[c * nblk + b] : 0.0;
      lds[c][tid] = x[c];
    }
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      double add[K];
      for (int c = 0; c < K; ++c) add[c] = tid >= off ? lds[c][tid - off] : 0.0;
      __syncthreads();
      for (int c = 0; c < K; ++c) lds[c][tid] += add[c];
      __syncthreads();
    }
    for (int c = 0; c < K; ++c) {
      const double excl = (tid > 0 ? lds[c][tid - 1] : 0.0);
      if (b < nblk) blk[c * nblk + b] = carry[c] + excl;
    }
    double last[K];
    for (int c = 0; c < K; ++c) last[c] = lds[c][255];
    __syncthreads();
    for (int c = 0; c < K; ++c) carry[c] += last[c];
  }
  if (tid == 0)
    for (int c = 0; c < K; ++c) S[c * (n + 1) + n] = carry[c];
}

template <int K>
__global__ void k_scan_add(double* __restrict__ S, int64_t n, const double* __restrict__ blk, int64_t nblk) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = j / kScanTile;
    for (int c = 0; c < K; ++c) S[c * (n + 1) + j] += blk[c * nblk + b];
  }
}

// Radius-pass chunks per node (0 past the last node) and cleared maxima.
__global__ void k_tree_count(const int4* __restrict__ node, const int32_t* __restrict__ total_p, int64_t cap,
                             unsigned long long* __restrict__ rbits, uint32_t* __restrict__ dbits,
                             int32_t* __restrict__ chunks) {
  const int64_t total = node_count(total_p, cap);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cap; k += (int64_t)gridDim.x * blockDim.x) {
    if (k >= total) {
      chunks[k] = 0;
      continue;
    }
    const int4 nd = node[k];
    rbits[k] = 0ull;
    dbits[k] = 0u;
    chunks[k] = (nd.y - nd.x + kChunk - 1) / kChunk;
  }
}

// Last node k with coff[k] <= c (coff ascending, coff[total] > c).
__device__ __forceinline__ int64_t chunk_node(const int32_t* __restrict__ coff, int64_t total, int64_t c) {
  int64_t lo = 0, hi = total;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (coff[mid] <= c)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// FP64 sums of (a, a px, a py, a pz) over each chunk, in sorted order.
__global__ void k_tree_chunk_sums(const int4* __restrict__ node, const int32_t* __restrict__ total_p, int64_t cap,
                                  const int32_t* __restrict__ coff, const float* __restrict__ P,
                                  const float* __restrict__ area, const int32_t* __restrict__ perm, int64_t n,
                                  double4* __restrict__ csum) {
  const int64_t total = node_count(total_p, cap);
  const int64_t nch = coff[total];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nch; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = chunk_node(coff, total, c);
    const int4 nd = node[k];
    const int64_t s = nd.x + (c - coff[k]) * kChunk;
    const int64_t e = s + kChunk < nd.y ? s + kChunk : nd.y;
    double a = 0.0, x = 0.0, y = 0.0, z = 0.0;
    for (int64_t j = s; j < e; ++j) {
      const int64_t o = perm[j];
      const double aj = area[o];
      a += aj;
      x += aj * (double)P[o];
      y += aj * (double)P[n + o];
      z += aj * (double)P[2 * n + o];
    }
    csum[c] = make_double4(a, x, y, z);
  }
}

// Node area and area-weighted centre from its chunks in order (the node's first source when
// the area is 0).
__global__ void k_tree_centre(const int4* __restrict__ node, const int32_t* __restrict__ total_p, int64_t cap,
                              const int32_t* __restrict__ coff, const double4* __restrict__ csum,
                              const float* __restrict__ P, const int32_t* __restrict__ perm, int64_t n,
                              double4* __restrict__ geo) {
  const int64_t total = node_count(total_p, cap);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
    double a = 0.0, x = 0.0, y = 0.0, z = 0.0;
    for (int64_t c = coff[k]; c < coff[k + 1]; ++c) {
      const double4 v = csum[c];
      a += v.x;
      x += v.y;
      y += v.z;
      z += v.w;
    }
    double4 g;
    if (a != 0.0) {
      g = make_double4(x / a, y / a, z / a, 0.0);
    } else {
      const int64_t o = perm[node[k].x];
      g = make_double4(P[o], P[n + o], P[2 * n + o], 0.0);
    }
    geo[k] = g;
  }
}

// r (FP64) and dmax over chunks of kChunk sources: atomic max of the bit patterns, which
// order like unsigned integers for non-negative values.
__global__ void k_tree_radius(const int4* __restrict__ node, const int32_t* __restrict__ total_p, int64_t cap,
                              const int32_t* __restrict__ coff, const float* __restrict__ P,
                              const float* __restrict__ D, float eps, const int32_t* __restrict__ perm, int64_t n,
                              const double4* __restrict__ geo, unsigned long long* __restrict__ rbits,
                              uint32_t* __restrict__ dbits) {
  const int64_t total = node_count(total_p, cap);
  const int64_t nch = coff[total];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nch; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = chunk_node(coff, total, c);
    const int4 nd = node[k];
    const double4 g = geo[k];
    const int64_t s = nd.x + (c - coff[k]) * kChunk;
    const int64_t e = s + kChunk < nd.y ? s + kChunk : nd.y;
    double r = 0.0;
    float dm = 0.0f;
    for (int64_t j = s; j < e; ++j) {
      const int64_t o = perm[j];
      const double ex = (double)P[o] - g.x, ey = (double)P[n + o] - g.y, ez = (double)P[2 * n + o] - g.z;
      const double dd = sqrt(ex * ex + ey * ey + ez * ez);
      r = dd > r ? dd : r;
      const float dj = D ? D[o] : 0.0f;
      const float fl = dj > eps ? dj : eps;
      dm = fl > dm ? fl : dm;
    }
    atomicMax(&rbits[k], (unsigned long long)__double_as_longlong(r));
    atomicMax(&dbits[k], __float_as_uint(dm));
  }
}

__global__ void k_tree_crit(const int32_t* __restrict__ total_p, int64_t cap, double beta,
                            const unsigned long long* __restrict__ rbits, const uint32_t* __restrict__ dbits,
                            double4* __restrict__ geo) {
  const int64_t total = node_count(total_p, cap);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
    const double r = __longlong_as_double((long long)rbits[k]);
    const double dm = (double)__uint_as_float(dbits[k]);
    double crit = beta * r;
    if (r + dm > crit) crit = r + dm;
    geo[k].w = crit * crit;
  }
}

// Node moments for the current normals: M = sum of the staged m_j over the node (FP64).
__global__ void k_tree_mom(const int4* __restrict__ node, const int32_t* __restrict__ total_p, int64_t cap,
                           const double* __restrict__ S, int64_t n, float4* __restrict__ mom) {
  const int64_t total = node_count(total_p, cap);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
    const int4 nd = node[k];
    float m[3];
    for (int d = 0; d < 3; ++d) m[d] = (float)(S[d * (n + 1) + nd.y] - S[d * (n + 1) + nd.x]);
    mom[k] = make_float4(m[0], m[1], m[2], 0.0f);
  }
}

template <int NA, bool KAHAN>
__device__ __forceinline__ void fold(float* sum, float* cmp, const float* acc) {
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    if (KAHAN) {
      const float y = acc[a] - cmp[a];
      const float t = sum[a] + y;
      cmp[a] = (t - sum[a]) - y;
      sum[a] = t;
    } else {
      sum[a] += acc[a];
    }
  }
}

// Leaf-relative staging of the source positions for the leaf pairs, in place: kappa (p_j - c)
// with c the leaf's centre rounded to FP32, which the traversal also subtracts from the
// query, so a near pair's difference is rounded relative to the leaf's neighbourhood, not to
// |p|. Every sorted source lies in exactly one leaf (one writer per source); .w keeps the
// staged 1/(kappa max(delta, eps)), and the moments beside it are untouched.
__global__ void k_tree_leafpos(const int4* __restrict__ node, const int32_t* __restrict__ total_p, int64_t cap,
                               const double4* __restrict__ geo, float4* __restrict__ src, int64_t n, float kappa) {
  const int64_t total = node_count(total_p, cap);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
    const int4 nd = node[k];
    if (!(nd.w >> 8)) continue;
    const double4 g = geo[k];
    const float cx = (float)g.x, cy = (float)g.y, cz = (float)g.z;
    const int64_t e = nd.y < n ? nd.y : n;
    for (int64_t j = nd.x; j < e; ++j) {
      const float4 a = src[2 * j];
      src[2 * j] = make_float4(kappa * (a.x - cx), kappa * (a.y - cy), kappa * (a.z - cz), a.w);
    }
  }
}

// Traversal: one thread per sorted query, one node index per wavefront (see the file head).
// Contributions are summed in FP32 into `acc` and folded into the (Kahan-compensated when
// KAHAN) running sums after every kFoldLeaves leaf visits of the wavefront and at the end
// (a fold is 4 VALU per accumulator; folding after every visit was ~2% slower at 1M). The
// next node is usually i + 1 (a node opened, or a leaf, whose skip is i + 1), so its data is
// loaded one step ahead.
constexpr int kFoldLeaves = 4;
// Threads per block of the traversal: its wavefronts share no data and never wait for each
// other (each has its own LDS area and no barrier).
constexpr int kTreeBlock = 256;
constexpr int kTreeWaves = kTreeBlock / 64;
// A leaf visit is spread over the idle lanes when that saves at least this many iterations.
constexpr int kSplitMinSaved = 2;

// A leaf of ns sources opened by na lanes of a wavefront: the log2 of the number k of lane
// groups its loop is spread over (0 = not spread), the largest power of two with k na <= 64
// and k <= ns, kept only when ceil(ns / k) saves at least kSplitMinSaved iterations.
__device__ __forceinline__ int leaf_split_log2(int na, int ns) {
  if (na < 1 || ns < 2) return 0;
  const int by_lanes = __clz((unsigned)(na - 1)) - 26;  // 6 - ceil(log2 na): 2^j na <= 64
  const int by_sources = 31 - __clz((unsigned)ns);      // floor(log2 ns): 2^j <= ns
  int lk = by_lanes < by_sources ? by_lanes : by_sources;
  if (lk > 0 && ns - ((ns + (1 << lk) - 1) >> lk) < kSplitMinSaved) lk = 0;
  return lk > 0 ? lk : 0;
}

// Workgroups are dealt to the 8 XCDs in turn (block b to XCD b mod 8), and each XCD has an L2
// of its own. Block b evaluates the (b mod 8)-th contiguous run of query blocks instead of
// query block b, so the blocks resident on one XCD hold neighbouring queries, which visit
// nearly the same nodes and leaf sources, and that XCD's L2 holds one region of the tree
// rather than every eighth block's share of all of it. A bijection of [0, nb) onto itself.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned q = nb / 8, r = nb % 8, x = b % 8, k = b / 8;
  return x * q + (x < r ? x : r) + k;
}

template <bool GRAD, bool SCREENED, bool KAHAN>
__global__ __launch_bounds__(kTreeBlock) void k_tree_eval(const float* __restrict__ Q, int64_t m,
                                                   const int32_t* __restrict__ qperm, const int4* __restrict__ node,
                                                   const double4* __restrict__ geo, const float4* __restrict__ mom,
                                                   const int32_t* __restrict__ total_p, int64_t cap,
                                                   const float4* __restrict__ src, int64_t n_src, Scr sk,
                                                   float kappa, float* __restrict__ part, int64_t mpad) {
  constexpr int NA = GRAD ? kNAcc : 1;
  // per wavefront: the queries of a split leaf visit by rank, and the lanes' partial sums
  __shared__ float4 lds_q[kTreeWaves][64];
  __shared__ float lds_p[kTreeWaves][64][NA == 1 ? 1 : 8];
  const int wv = (int)(threadIdx.x >> 6);
  const int64_t qi = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t o = qperm[qi < m ? qi : m - 1];
  const float ux = Q[o], uy = Q[m + o], uz = Q[2 * m + o];
  const double dqx = ux, dqy = uy, dqz = uz;  // the opening test runs in unscaled FP64
  const double dk = kappa;
  float sum[NA], cmp[NA], acc[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) sum[a] = cmp[a] = acc[a] = 0.0f;
  int nn = __builtin_amdgcn_readfirstlane(*total_p);
  if (nn > cap) nn = (int)cap;
  int skip_to = 0;
  int i = 0;
  int visits = 0;  // leaf visits of the wavefront since the last fold
  int4 nd = node[0];
  double4 g = geo[0];
  float4 mm = mom[0];
  while (i < nn) {
    const int nskip = __builtin_amdgcn_readfirstlane(nd.z);
    bool open = false, direct = false;
    if (i >= skip_to) {
      const double dx = g.x - dqx, dy = g.y - dqy, dz = g.z - dqz;
      const double d2 = dx * dx + dy * dy + dz * dz;
      if (d2 > g.w) {
        const float fx = (float)(dk * dx), fy = (float)(dk * dy), fz = (float)(dk * dz);
        if (SCREENED)
          pair_screened_d<GRAD, true>(fx, fy, fz, 0.0f, mm, sk, acc);
        else
          pair_plain_d<GRAD, true>(fx, fy, fz, 0.0f, mm, acc);
        skip_to = nskip;
      } else if (nd.w >> 8) {
        direct = true;
      } else {
        open = true;
      }
    }
    // The next node is loaded only now: scalar loads return out of order, so the wait in
    // front of this step's test covered every scalar load in flight; issued after the test,
    // the next node's loads have the rest of this step to arrive. (Loading the node after
    // this one's subtree too, the other possible successor, cost more registers than it
    // saved.)
    __asm__ __volatile__("" ::: "memory");
    const int nxt = i + 1 < nn ? i + 1 : i;
    const int4 nd1 = node[nxt];
    const double4 g1 = geo[nxt];
    const float4 mm1 = mom[nxt];
    int next;
    if (__any(open)) {
      next = i + 1;
    } else {
      if (__any(direct)) {
        const int s0 = __builtin_amdgcn_readfirstlane(nd.x);
        int s1 = __builtin_amdgcn_readfirstlane(nd.y);
        if (s1 > n_src) s1 = (int)n_src;
        // the query relative to the leaf's centre, as its sources are staged (k_tree_leafpos)
        const float lx = kappa * (ux - (float)g.x), ly = kappa * (uy - (float)g.y), lz = kappa * (uz - (float)g.z);
        // With a lanes opening the leaf, k = 2^lk groups of a lanes (k a <= 64) can take an
        // interleaved k-th of its sources each for one query, in ceil(s / k) iterations
        // instead of s; the groups' partial sums then go back to the querying lanes.
        const uint64_t dmask = __ballot(direct);
        const int lk = __builtin_amdgcn_readfirstlane(leaf_split_log2(__popcll(dmask), s1 - s0));
        if (lk == 0) {
          if (direct) {
            // the lanes that did not open the leaf sit the whole loop out (one exec mask for
            // the loop, not one per source). Two sources per iteration: their scalar loads
            // are waited for once and their rsq and exp issue in pairs (1-3.5% faster than one
            // per iteration at beta 2.3-32); the spread loop below keeps one, as two there
            // take the kernel to 78 VGPRs and 6 wavefronts per SIMD, which ran slower.
            int j = s0;
#pragma unroll 1
            for (; j + 1 < s1; j += 2) {  // two independent sources per iteration
              const float4 a0 = src[2 * (int64_t)j], b0 = src[2 * (int64_t)j + 1];
              const float4 a1 = src[2 * (int64_t)j + 2], b1 = src[2 * (int64_t)j + 3];
              if (SCREENED) {
                pair_screened<GRAD, false>(a0, b0, lx, ly, lz, sk, acc);
                pair_screened<GRAD, false>(a1, b1, lx, ly, lz, sk, acc);
              } else {
                pair_plain<GRAD, false>(a0, b0, lx, ly, lz, acc);
                pair_plain<GRAD, false>(a1, b1, lx, ly, lz, acc);
              }
            }
            if (j < s1) {
              const float4 a = src[2 * (int64_t)j], b = src[2 * (int64_t)j + 1];
              if (SCREENED)
                pair_screened<GRAD, false>(a, b, lx, ly, lz, sk, acc);
              else
                pair_plain<GRAD, false>(a, b, lx, ly, lz, acc);
            }
          }
        } else {
          const int lane = (int)(threadIdx.x & 63);
          const int rank = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(dmask >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((unsigned)dmask, 0u));
          float4* qs = lds_q[wv];
          if (direct) qs[rank] = make_float4(lx, ly, lz, 0.0f);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const int grp = lane & ((1 << lk) - 1), who = lane >> lk;
          float pac[NA];
#pragma unroll
          for (int a = 0; a < NA; ++a) pac[a] = 0.0f;
          if (who < __popcll(dmask)) {
            const float4 qq = qs[who];
#pragma unroll 1
            for (int j = s0 + grp; j < s1; j += 1 << lk) {
              const float4 a = src[2 * (int64_t)j], b = src[2 * (int64_t)j + 1];
              if (SCREENED)
                pair_screened<GRAD, false>(a, b, qq.x, qq.y, qq.z, sk, pac);
              else
                pair_plain<GRAD, false>(a, b, qq.x, qq.y, qq.z, pac);
            }
          }
          float* ps = lds_p[wv][lane];
#pragma unroll
          for (int a = 0; a < NA; ++a) ps[a] = pac[a];
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (direct) {
#pragma unroll 1
            for (int gi = 0; gi < (1 << lk); ++gi) {
              const float* pg = lds_p[wv][(rank << lk) + gi];
#pragma unroll
              for (int a = 0; a < NA; ++a) acc[a] += pg[a];
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (++visits == kFoldLeaves) {
          visits = 0;
          fold<NA, KAHAN>(sum, cmp, acc);
#pragma unroll
          for (int a = 0; a < NA; ++a) acc[a] = 0.0f;
        }
      }
      next = nskip > i ? nskip : i + 1;  // pre-order: skip > i always; guards the loop regardless
    }
    if (next == i + 1) {
      nd = nd1;
      g = g1;
      mm = mm1;
    } else if (next < nn) {
      nd = node[next];
      g = geo[next];
      mm = mom[next];
    }
    i = __builtin_amdgcn_readfirstlane(next);
  }
  fold<NA, KAHAN>(sum, cmp, acc);
#pragma unroll
  for (int a = 0; a < NA; ++a) part[a * mpad + qi] = KAHAN ? sum[a] - cmp[a] : sum[a];
}

// Work of the traversal (the counts of dwg_octree_work). The decisions are those of
// k_tree_eval (the same FP64 opening test, the same wave-wide walk over the same wavefronts of
// 64 sorted queries), without its arithmetic. Per-query counts leave out lanes past m (they
// repeat query m - 1, which sits in the same wavefront, so they change no wave-wide step);
// wavefront counts come from lane 0 of each wavefront with a query below m. Integer atomics
// make the totals independent of the order of the blocks.
__global__ __launch_bounds__(256) void k_tree_work(const float* __restrict__ Q, int64_t m,
                                                   const int32_t* __restrict__ qperm, const int4* __restrict__ node,
                                                   const double4* __restrict__ geo,
                                                   const int32_t* __restrict__ total_p, int64_t cap, int64_t n_src,
                                                   unsigned long long* __restrict__ out) {
  __shared__ unsigned long long red[kTreeWorkCounts][4];
  const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = qi < m;
  const int64_t o = qperm[live ? qi : m - 1];
  const double dqx = Q[o], dqy = Q[m + o], dqz = Q[2 * m + o];
  int nn = __builtin_amdgcn_readfirstlane(*total_p);
  if (nn > cap) nn = (int)cap;
  unsigned long long nfar = 0, npair = 0, wfar = 0, wleaf = 0;
  int skip_to = 0;
  int i = 0;
  while (i < nn) {
    const int4 nd = node[i];
    const double4 g = geo[i];
    const int nskip = __builtin_amdgcn_readfirstlane(nd.z);
    bool far = false, open = false, direct = false;
    if (i >= skip_to) {
      const double dx = g.x - dqx, dy = g.y - dqy, dz = g.z - dqz;
      const double d2 = dx * dx + dy * dy + dz * dz;
      if (d2 > g.w) {
        far = true;
        ++nfar;
        skip_to = nskip;
      } else if (nd.w >> 8) {
        direct = true;
      } else {
        open = true;
      }
    }
    if (__any(far)) ++wfar;
    int next;
    if (__any(open)) {
      next = i + 1;
    } else {
      const int s1 = nd.y < n_src ? nd.y : (int)n_src;
      if (direct) npair += (unsigned long long)(s1 - nd.x);
      const uint64_t dmask = __ballot(direct);
      if (dmask) {
        const int ns = s1 - __builtin_amdgcn_readfirstlane(nd.x);
        const int lk = leaf_split_log2(__popcll(dmask), ns);
        wleaf += (unsigned long long)((ns + (1 << lk) - 1) >> lk);
      }
      next = nskip > i ? nskip : i + 1;
    }
    i = __builtin_amdgcn_readfirstlane(next);
  }
  if (!live) nfar = npair = 0;
  for (int off = 32; off > 0; off >>= 1) {
    nfar += __shfl_xor(nfar, off, 64);
    npair += __shfl_xor(npair, off, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    // lane 0 is live whenever any lane of its wavefront is
    red[0][wv] = nfar;
    red[1][wv] = npair;
    red[2][wv] = live ? wfar : 0;
    red[3][wv] = live ? wleaf : 0;
  }
  __syncthreads();
  if (threadIdx.x < kTreeWorkCounts)
    atomicAdd(&out[threadIdx.x], red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3]);
}

__global__ void k_zero_u64(unsigned long long* __restrict__ a, int k) {
  if ((int)threadIdx.x < k) a[threadIdx.x] = 0ull;
}

__global__ void k_copy_i32(const int32_t* __restrict__ a, int64_t n, int32_t* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// (start, end, level, skip) per node for dwg_octree.
__global__ void k_tree_export(const int4* __restrict__ node, const int32_t* __restrict__ total_p, int64_t cap,
                              int32_t* __restrict__ out) {
  const int64_t total = node_count(total_p, cap);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
    const int4 nd = node[k];
    out[4 * k + 0] = nd.x;
    out[4 * k + 1] = nd.y;
    out[4 * k + 2] = nd.w & 255;
    out[4 * k + 3] = nd.z;
  }
}

template <int K>
dwg_status scan_f64(const float4* src, int64_t n, const TreeWork& t, hipStream_t st) {
  const int64_t nblk = cdiv(n, kScanTile);
  hipLaunchKernelGGL((k_scan_local<K>), dim3((unsigned)nblk), dim3(256), 0, st, src, n, t.scan, t.sblk, nblk);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL((k_scan_tops<K>), dim3(1), dim3(256), 0, st, t.sblk, nblk, t.scan, n);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL((k_scan_add<K>), dim3(grid_cap(n)), dim3(256), 0, st, t.scan, n, t.sblk, nblk);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

template <bool GRAD, bool SCREENED, bool KAHAN>
void launch_eval_t(const float* Q, int64_t m, const int32_t* qperm, const GwnWork& w, const TreeWork& t,
                   float kappa, hipStream_t st) {
  hipLaunchKernelGGL((k_tree_eval<GRAD, SCREENED, KAHAN>), dim3((unsigned)(w.mpad / kTreeBlock)), dim3(kTreeBlock), 0,
                     st, Q, m, qperm, t.node, t.geo, t.mom, t.off + t.n, t.cap, w.src, t.n, kScaledScr, kappa,
                     w.part, w.mpad);
}

}  // namespace

int64_t tree_cap(int64_t n) { return 2 * n + 1; }

size_t radix_hist_len(int64_t n) { return (size_t)(256 * cdiv(n, kSortTile) + 1); }

dwg_status radix_sort_pairs(uint64_t* const key[2], int32_t* const val[2], int64_t n, int bits, int32_t* hist,
                            int32_t* hsums, int* result, hipStream_t st) {
  const int64_t nsb = cdiv(n, kSortTile);
  const int passes = (bits + 7) / 8;
  for (int pass = 0; pass < passes; ++pass) {
    const int a = pass & 1, b = a ^ 1;
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nsb), dim3(256), 0, st, key[a], n, 8 * pass, hist, nsb);
    DWG_TRY_LAUNCH();
    dwg_status s = exclusive_scan(hist, 256 * nsb, hsums, st);
    if (s != DWG_OK) return s;
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nsb), dim3(256), 0, st, key[a], val[a], n, 8 * pass, hist, nsb,
                       key[b], val[b]);
    DWG_TRY_LAUNCH();
  }
  *result = passes & 1;
  return DWG_OK;
}

dwg_status morton_frame(const float* P, int64_t n, float* bpart, float* box, double* frame, hipStream_t st) {
  dwg_status s = launch_bbox(P, n, bpart, box, st);
  if (s != DWG_OK) return s;
  hipLaunchKernelGGL(k_tree_frame, dim3(1), dim3(64), 0, st, box, frame);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

size_t carve_tree(Carver& c, int64_t n, int leaf, double beta, TreeWork* out) {
  const size_t s0 = c.used;
  TreeWork t{};
  t.n = n;
  t.cap = tree_cap(n);
  t.leaf = leaf;
  t.beta = beta;
  t.nsb = cdiv(n, kSortTile);
  t.nscan = cdiv(n, kScanTile);
  t.bpart = c.take<float>(kBboxParts);
  t.box = c.take<float>(8);
  t.frame = c.take<double>(4);
  t.key[0] = c.take<uint64_t>((size_t)n);
  t.key[1] = c.take<uint64_t>((size_t)n);
  t.val[0] = c.take<int32_t>((size_t)n);
  t.val[1] = c.take<int32_t>((size_t)n);
  t.hist = c.take<int32_t>((size_t)(256 * t.nsb + 1));
  t.hsums = c.take<int32_t>(scan_sums_len(256 * t.nsb));
  t.lev = c.take<int32_t>((size_t)n);
  t.off = c.take<int32_t>((size_t)n + 1);
  t.osums = c.take<int32_t>(scan_sums_len(n));
  t.node = c.take<int4>((size_t)t.cap);
  t.geo = c.take<double4>((size_t)t.cap);
  t.mom = c.take<float4>((size_t)t.cap);
  t.rbits = c.take<unsigned long long>((size_t)t.cap);
  t.dbits = c.take<uint32_t>((size_t)t.cap);
  t.coff = c.take<int32_t>((size_t)t.cap + 1);
  t.csums = c.take<int32_t>(scan_sums_len(t.cap));
  // chunks: at most one partial chunk per node plus sum(node sizes) / kChunk, and every
  // source lies in at most kDepth + 1 nodes
  t.ccap = t.cap + cdiv(n * (kDepth + 1), kChunk);
  t.csum = c.take<double4>((size_t)t.ccap);
  t.scan = c.take<double>(3 * ((size_t)n + 1));
  t.sblk = c.take<double>(3 * (size_t)t.nscan);
  if (out) *out = t;
  return c.used - s0;
}

dwg_status tree_build(const float* P, const float* area, const float* delta, int64_t n, float eps,
                      const TreeWork& t, int32_t* perm, hipStream_t st) {
  dwg_status s = morton_frame(P, n, t.bpart, t.box, t.frame, st);
  if (s != DWG_OK) return s;
  hipLaunchKernelGGL(k_tree_keys, dim3(grid_cap(n)), dim3(256), 0, st, P, n, t.frame, t.key[0], t.val[0]);
  DWG_TRY_LAUNCH();
  int res = 0;
  s = radix_sort_pairs(t.key, t.val, n, 64, t.hist, t.hsums, &res, st);
  if (s != DWG_OK) return s;
  // eight passes: the sorted codes and indices are back in buffer 0
  hipLaunchKernelGGL(k_tree_mark, dim3(grid_cap(n)), dim3(256), 0, st, t.key[0], n, t.leaf, t.lev, t.off);
  DWG_TRY_LAUNCH();
  s = exclusive_scan(t.off, n, t.osums, st);
  if (s != DWG_OK) return s;
  hipLaunchKernelGGL(k_tree_emit, dim3(grid_cap(n)), dim3(256), 0, st, t.key[0], n, t.leaf, t.lev, t.off, t.cap,
                     t.node);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_copy_i32, dim3(grid_cap(n)), dim3(256), 0, st, t.val[0], n, perm);
  DWG_TRY_LAUNCH();
  if (!area) return DWG_OK;  // topology only (dwg_octree)
  const int32_t* total = t.off + n;
  hipLaunchKernelGGL(k_tree_count, dim3(grid_cap(t.cap)), dim3(256), 0, st, t.node, total, t.cap, t.rbits, t.dbits,
                     t.coff);
  DWG_TRY_LAUNCH();
  s = exclusive_scan(t.coff, t.cap, t.csums, st);
  if (s != DWG_OK) return s;
  hipLaunchKernelGGL(k_tree_chunk_sums, dim3(grid_cap(t.ccap)), dim3(256), 0, st, t.node, total, t.cap, t.coff, P,
                     area, perm, n, t.csum);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_tree_centre, dim3(grid_cap(t.cap)), dim3(256), 0, st, t.node, total, t.cap, t.coff, t.csum,
                     P, perm, n, t.geo);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_tree_radius, dim3(grid_cap(t.cap)), dim3(256), 0, st, t.node, total, t.cap, t.coff, P, delta, eps,
                     perm, n, t.geo, t.rbits, t.dbits);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_tree_crit, dim3(grid_cap(t.cap)), dim3(256), 0, st, total, t.cap, t.beta, t.rbits, t.dbits,
                     t.geo);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status tree_stage_leaves(const GwnWork& w, const TreeWork& t, float kappa, hipStream_t st) {
  hipLaunchKernelGGL(k_tree_leafpos, dim3(grid_cap(t.cap)), dim3(256), 0, st, t.node, t.off + t.n, t.cap, t.geo, w.src,
                     t.n, kappa);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status tree_moments(const GwnWork& w, const TreeWork& t, hipStream_t st) {
  dwg_status s = scan_f64<3>(w.src, t.n, t, st);
  if (s != DWG_OK) return s;
  hipLaunchKernelGGL(k_tree_mom, dim3(grid_cap(t.cap)), dim3(256), 0, st, t.node, t.off + t.n, t.cap, t.scan, t.n,
                     t.mom);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status tree_eval(const float* Q, int64_t m, const dwg_kernel_params& kp, bool grad, const GwnWork& w,
                     const TreeWork& t, hipStream_t st) {
  const bool scr = kp.lambda > 0.0f;
  const bool kah = kp.compensated != 0;
  const float kappa = position_scale(kp);
#define DWG_TREE_CASE(G, S, K) \
  if (grad == G && scr == S && kah == K) launch_eval_t<G, S, K>(Q, m, w.perm_q, w, t, kappa, st);
  DWG_TREE_CASE(true, false, true)
  DWG_TREE_CASE(true, false, false)
  DWG_TREE_CASE(true, true, true)
  DWG_TREE_CASE(true, true, false)
  DWG_TREE_CASE(false, false, true)
  DWG_TREE_CASE(false, false, false)
  DWG_TREE_CASE(false, true, true)
  DWG_TREE_CASE(false, true, false)
#undef DWG_TREE_CASE
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status tree_work(const float* Q, int64_t m, const int32_t* qperm, const TreeWork& t, unsigned long long* out,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, out, kTreeWorkCounts);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_tree_work, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, st, Q, m, qperm, t.node, t.geo,
                     t.off + t.n, t.cap, t.n, out);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status tree_export(const TreeWork& t, int32_t* nodes_out, int64_t cap_out, int64_t* count_host,
                       hipStream_t st) {
  int32_t total = 0;
  DWG_TRY_HIP(hipMemcpyAsync(&total, t.off + t.n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  DWG_TRY_HIP(hipStreamSynchronize(st));
  *count_host = total;
  if (total > cap_out) {
    set_error("octree has %d nodes, output holds %lld", total, (long long)cap_out);
    return DWG_E_INVALID;
  }
  hipLaunchKernelGGL(k_tree_export, dim3(grid_cap(total)), dim3(256), 0, st, t.node, t.off + t.n, cap_out, nodes_out);
  DWG_TRY_LAUNCH();
  DWG_TRY_HIP(hipStreamSynchronize(st));
  return DWG_OK;
}

}  // namespace dwg
