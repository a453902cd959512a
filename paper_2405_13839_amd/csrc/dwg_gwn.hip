// All-pairs GWN / gradient kernels, the normal-update epilogue and the FP64 statistics of
// one DWG iteration (Sec. 3 Eq. 2-3, Sec. 4.2 Eq. 5, Sec. 4.3 Eq. 6-7, Sec. 5.1-5.2).
//
// Data layout in HBM (all carved from the caller's workspace; "sorted" = the spatial order
// of dwg_sort.hip, perm[i] = original index of sorted position i):
//   src   [2*npad] float4  sorted sources: (p_j, 1/(kappa max(delta_j, eps))), (m_j, 0) with
//                          m_j = a_j n_j / (4 pi); padding sources are all zero, which makes
//                          their contribution exactly zero in the general path.
//   kk    [npad]           a_j / (4 pi) per sorted source (restaging after the update)
//   tbox  [2*ntiles]       per source tile: (min xyz, max radius), (max xyz, 0)
//   qbox  [2*nqblk]        per block of kQBlock sorted queries: (min xyz, 0), (max xyz, 0)
//   part  [split][7][mpad] per-split partial sums of w, A, B per sorted query
//   theta [m] double       angle between consecutive normals (degrees), sorted order
// Positions and boxes are in the caller's units; kappa = s log2(e) for the screened kernel
// (1 for the plain one) is applied to pair differences inside the kernels.
// Queries are gathered from the caller's planar [3][m] array through the query permutation.
#include <cmath>

#include "dwg_internal.h"
#include "dwg_pair.h"

namespace dwg {
namespace {

using namespace pairk;

constexpr double kRadToDeg = 57.295779513082320876798;

// Tile classes of the all-pairs kernel: general (clamp and coincidence handled), far (no pair
// clamped or coincident) and separated (far, and every pair at least as long as the largest
// distance of a query from the block's centre), each with its own pair loop.
enum TileKind { kGeneral = 0, kFar = 1, kSeparated = 2 };

// One LDS tile of sources against the thread's QPT queries. The tile holds the separated
// form (a = (-2 p, |p|^2), b = (m, m . p), iw apart); the general and far loops recover the
// difference p - q exactly as fma(-2 p, -1/2, -q).
template <int QPT, int NS, bool GRAD, bool SCREENED, int KIND>
__device__ __forceinline__ void tile_loop(const float4* sa, const float4* sb, const float* sw, const float* qx,
                                          const float* qy, const float* qz, const float* qq, const Scr k,
                                          float (*acc)[NS]) {
#pragma unroll 2
  for (int j = 0; j < kTile; ++j) {
    const float4 a = sa[j];
    const float4 b = sb[j];
    const float iw = KIND == kGeneral ? sw[j] : 0.0f;
    if (KIND == kSeparated) {
      // Every query's r^2 and rsq first, then the rest: the rsq latency is then covered by
      // the work that does not depend on it (m . q). Left to itself the compiler interleaves
      // the queries' chains and issues each rsq right before its first use (measured 568 ms
      // per 1M x 1M screened launch against 524 ms in this order).
      float r2[QPT], ir[QPT];
#pragma unroll
      for (int q = 0; q < QPT; ++q) r2[q] = sep_r2(a, qx[q], qy[q], qz[q], qq[q]);
#pragma unroll
      for (int q = 0; q < QPT; ++q) ir[q] = rsq(r2[q]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < QPT; ++q) {
        if (SCREENED)
          pair_screened_sep<GRAD>(a, b, qx[q], qy[q], qz[q], r2[q], ir[q], k, acc[q]);
        else
          pair_plain_sep<GRAD>(a, b, qx[q], qy[q], qz[q], ir[q], acc[q]);
      }
    } else {
#pragma unroll
      for (int q = 0; q < QPT; ++q) {
        const float dx = fmaf(a.x, -0.5f, -qx[q]), dy = fmaf(a.y, -0.5f, -qy[q]), dz = fmaf(a.z, -0.5f, -qz[q]);
        if (SCREENED)
          pair_screened_d<GRAD, KIND == kFar>(dx, dy, dz, iw, b, k, acc[q]);
        else
          pair_plain_d<GRAD, KIND == kFar>(dx, dy, dz, iw, b, acc[q]);
      }
      if (KIND == kFar && SCREENED && GRAD) {
        // Instruction order of one source against the QPT = 2 queries (scheduling only): the
        // two LDS reads, the 12 VALU of both differences and r^2, both rsq, 8 VALU, both exp,
        // then the rest. Left to itself the compiler issues the four rsq (and four exp) of the
        // unrolled pair of sources back to back; this order measured 528-531 ms against
        // 546-551 ms per 1M x 1M launch when every far tile took this loop.
        __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);   // DS read
        __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);  // VALU
        __builtin_amdgcn_sched_group_barrier(0x400, 2, 0);   // transcendental
        __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);
        __builtin_amdgcn_sched_group_barrier(0x400, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 34, 0);
      }
    }
  }
}

// All-pairs kernel. Block = 256 threads holding QPT queries each (sorted query
// q0 + k*256 + tid); grid.y = source split. Source tiles of 256 are staged in LDS and read
// back as broadcasts. Per tile, the block decides (uniformly) whether the tile is far from
// all of its queries -- box distance above the tile's largest radius, so no pair can be
// clamped or coincident -- and then runs the shorter far-pair loop; a far tile whose box
// distance is also at least the largest distance of a query from the block's centre takes
// the separated far loop (r^2 and m . (p - q) from per-source |p|^2 and m . p).
// Each tile's contributions go to FP32 partials, folded into running sums
// (Kahan-compensated when KAHAN). The compensation terms live in LDS, one column per
// thread: they are touched once per tile, and the 14 registers they would take hold the
// screened kernel at 4 waves per SIMD instead of 5 (the kernel asks for 5, which it fits
// without spills).
// Positions enter the pair arithmetic relative to a point c of the block and scaled by kappa:
// kappa (x - c), formed when the tile is filled (with |p|^2 and m . p in the fourth
// components). The rounding of a near pair's difference is then relative to the pair's
// distance from c, not to |x| (kappa x rounded in FP32 would move r by up to |x| 2^-24,
// enough to flip the clamp branch of pairs within ~1e-5 of r = delta in a scene of size 2).
// c is the block's middle query (sorted position q0 + 256), not the centre of its box:
// where the spatial order jumps inside a block (a lone point far from the rest of its
// block), the box centre lies far from every query and all of the block's near pairs lose
// precision; the middle query keeps the block's bulk exact relative to itself, and the far
// query's pairs are long.
template <int QPT, bool GRAD, bool SCREENED, bool KAHAN>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_gwn(const float* __restrict__ Q, int64_t m,
                                                 const int32_t* __restrict__ qperm,
                                                 const float4* __restrict__ src, int64_t ntiles,
                                                 int64_t nfull, int64_t tiles_per_split,
                                                 const float4* __restrict__ tbox,
                                                 const float4* __restrict__ qbox, Scr sk, float kappa,
                                                 float* __restrict__ part, int64_t mpad) {
  constexpr int NA = GRAD ? kNAcc : 1;
  constexpr int NS = GRAD ? kNAcc + 1 : 1;  // + sum of t in the separated loop
  __shared__ float4 sa[kTile];
  __shared__ float4 sb[kTile];
  __shared__ float sw[kTile];
  const int tid = threadIdx.x;
  const int64_t q0 = (int64_t)blockIdx.x * (kBlock * QPT);
  const float4 qlo = qbox[2 * blockIdx.x], qhi = qbox[2 * blockIdx.x + 1];
  const int64_t oc = qperm[min(q0 + (kBlock * QPT) / 2, m - 1)];
  const float cx = Q[oc], cy = Q[m + oc], cz = Q[2 * m + oc];
  // largest distance of a query of the block from c (the query box's farthest corner)
  const float rx = fmaxf(qhi.x - cx, cx - qlo.x), ry = fmaxf(qhi.y - cy, cy - qlo.y),
              rz = fmaxf(qhi.z - cz, cz - qlo.z);
  const float rq2 = rx * rx + ry * ry + rz * rz;
  float qx[QPT], qy[QPT], qz[QPT], qq[QPT];
#pragma unroll
  for (int k = 0; k < QPT; ++k) {
    int64_t qi = q0 + k * kBlock + tid;
    if (qi >= m) qi = m - 1;
    const int64_t o = qperm[qi];
    qx[k] = kappa * (Q[o] - cx);
    qy[k] = kappa * (Q[m + o] - cy);
    qz[k] = kappa * (Q[2 * m + o] - cz);
    qq[k] = fmaf(qz[k], qz[k], fmaf(qy[k], qy[k], qx[k] * qx[k]));
  }
  __shared__ float cmp[KAHAN ? QPT * NA : 1][kBlock];  // thread-private columns
  float sum[QPT][NA];
#pragma unroll
  for (int k = 0; k < QPT; ++k)
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      sum[k][a] = 0.0f;
      if (KAHAN) cmp[k * NA + a][tid] = 0.0f;
    }

  const int64_t t0 = (int64_t)blockIdx.y * tiles_per_split;
  const int64_t t1 = min(t0 + tiles_per_split, ntiles);
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    {
      const float4 a = src[2 * (t * kTile + tid)];
      const float4 b = src[2 * (t * kTile + tid) + 1];
      const float px = kappa * (a.x - cx), py = kappa * (a.y - cy), pz = kappa * (a.z - cz);
      sa[tid] = make_float4(-2.0f * px, -2.0f * py, -2.0f * pz, fmaf(pz, pz, fmaf(py, py, px * px)));
      sb[tid] = make_float4(b.x, b.y, b.z, fmaf(b.z, pz, fmaf(b.y, py, b.x * px)));
      sw[tid] = a.w;
    }
    const float4 tlo = tbox[2 * t], thi = tbox[2 * t + 1];
    const float gx = fmaxf(0.0f, fmaxf(qlo.x - thi.x, tlo.x - qhi.x));
    const float gy = fmaxf(0.0f, fmaxf(qlo.y - thi.y, tlo.y - qhi.y));
    const float gz = fmaxf(0.0f, fmaxf(qlo.z - thi.z, tlo.z - qhi.z));
    const float gap2 = gx * gx + gy * gy + gz * gz;
    // tiles with padding (t >= nfull) always take the general path
    const bool far = t < nfull && gap2 > 0.0f && gap2 > 1.0001f * tlo.w * tlo.w;
    const bool sep = far && gap2 >= rq2;
    __syncthreads();
    float acc[QPT][NS];
#pragma unroll
    for (int k = 0; k < QPT; ++k)
#pragma unroll
      for (int a = 0; a < NS; ++a) acc[k][a] = 0.0f;
    if (sep) {
      tile_loop<QPT, NS, GRAD, SCREENED, kSeparated>(sa, sb, sw, qx, qy, qz, qq, sk, acc);
      if (GRAD) {
#pragma unroll
        for (int k = 0; k < QPT; ++k) {  // A = -sum(t P) / 2 - q sum(t)
          acc[k][1] = fmaf(-0.5f, acc[k][1], -qx[k] * acc[k][NS - 1]);
          acc[k][2] = fmaf(-0.5f, acc[k][2], -qy[k] * acc[k][NS - 1]);
          acc[k][3] = fmaf(-0.5f, acc[k][3], -qz[k] * acc[k][NS - 1]);
        }
      }
    } else if (far) {
      tile_loop<QPT, NS, GRAD, SCREENED, kFar>(sa, sb, sw, qx, qy, qz, qq, sk, acc);
    } else {
      tile_loop<QPT, NS, GRAD, SCREENED, kGeneral>(sa, sb, sw, qx, qy, qz, qq, sk, acc);
    }
#pragma unroll
    for (int k = 0; k < QPT; ++k)
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        if (KAHAN) {
          const float y = acc[k][a] - cmp[k * NA + a][tid];
          const float tt = sum[k][a] + y;
          cmp[k * NA + a][tid] = (tt - sum[k][a]) - y;
          sum[k][a] = tt;
        } else {
          sum[k][a] += acc[k][a];
        }
      }
  }
  float* out = part + (int64_t)blockIdx.y * NA * mpad;
#pragma unroll
  for (int k = 0; k < QPT; ++k) {
    const int64_t qi = q0 + k * kBlock + tid;  // < mpad by construction of mpad
#pragma unroll
    for (int a = 0; a < NA; ++a) out[a * mpad + qi] = KAHAN ? sum[k][a] - cmp[k * NA + a][tid] : sum[k][a];
  }
}

// Stage the sources in spatial order: (p, 1/(kappa max(delta,eps))) and m = a n / (4 pi)
// (kappa = the position scale of the kernel, 1 when plain; positions stay unscaled, the
// evaluation kernels scale differences).
// A NaN delta poisons the source's m so that the result is NaN as in the definition.
__global__ void k_stage(const float* __restrict__ P, const float* __restrict__ N,
                        const float* __restrict__ A, const float* __restrict__ D, int64_t n,
                        int64_t npad, float eps, float kappa, const int32_t* __restrict__ perm,
                        float4* __restrict__ src, float* __restrict__ kk) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= npad) return;
  float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = make_float4(0.f, 0.f, 0.f, 0.f);
  float k = 0.0f;
  if (j < n) {
    const int64_t o = perm[j];
    const float d = D ? D[o] : 0.0f;
    const float fl = kappa * (d > eps ? d : eps);
    const float id = fl > 0.0f ? 1.0f / fl : INFINITY;
    k = A[o] * kInv4Pi;
    if (d != d) k = NAN;
    a = make_float4(P[o], P[n + o], P[2 * n + o], id);
    b = make_float4(k * N[o], k * N[n + o], k * N[2 * n + o], 0.0f);
  }
  src[2 * j] = a;
  src[2 * j + 1] = b;
  kk[j] = k;
}

// Box of each source tile (real sources only) and its largest radius max(delta, eps), in the
// unscaled units of the positions (the staged 1/radius carries kappa).
__global__ __launch_bounds__(kTile) void k_tile_box(const float4* __restrict__ src, int64_t n, float kappa,
                                                    float4* __restrict__ tbox) {
  __shared__ float lds[7][kTile];
  const int64_t j = (int64_t)blockIdx.x * kTile + threadIdx.x;
  float v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0f};
  if (j < n) {
    const float4 a = src[2 * j];
    v[0] = v[3] = a.x;
    v[1] = v[4] = a.y;
    v[2] = v[5] = a.z;
    v[6] = 1.0f / (kappa * a.w);  // radius (0 when 1/radius is +inf)
    if (!(v[6] == v[6])) v[6] = INFINITY;
  }
  for (int d = 0; d < 7; ++d) lds[d][threadIdx.x] = v[d];
  __syncthreads();
  for (int s = kTile / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int d = 0; d < 3; ++d) lds[d][threadIdx.x] = fminf(lds[d][threadIdx.x], lds[d][threadIdx.x + s]);
      for (int d = 3; d < 7; ++d) lds[d][threadIdx.x] = fmaxf(lds[d][threadIdx.x], lds[d][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tbox[2 * blockIdx.x] = make_float4(lds[0][0], lds[1][0], lds[2][0], lds[6][0]);
    tbox[2 * blockIdx.x + 1] = make_float4(lds[3][0], lds[4][0], lds[5][0], 0.0f);
  }
}

// Box of each block of kQBlock sorted queries.
__global__ __launch_bounds__(kBlock) void k_query_box(const float* __restrict__ Q, int64_t m,
                                                      const int32_t* __restrict__ qperm,
                                                      float4* __restrict__ qbox) {
  __shared__ float lds[6][kBlock];
  float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int k = 0; k < kQpt; ++k) {
    int64_t qi = (int64_t)blockIdx.x * kQBlock + k * kBlock + threadIdx.x;
    if (qi >= m) qi = m - 1;  // the kernel evaluates the clamped query there as well
    const int64_t o = qperm[qi];
    const float x = Q[o], y = Q[m + o], z = Q[2 * m + o];
    v[0] = fminf(v[0], x);
    v[1] = fminf(v[1], y);
    v[2] = fminf(v[2], z);
    v[3] = fmaxf(v[3], x);
    v[4] = fmaxf(v[4], y);
    v[5] = fmaxf(v[5], z);
  }
  for (int d = 0; d < 6; ++d) lds[d][threadIdx.x] = v[d];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int d = 0; d < 3; ++d) lds[d][threadIdx.x] = fminf(lds[d][threadIdx.x], lds[d][threadIdx.x + s]);
      for (int d = 3; d < 6; ++d) lds[d][threadIdx.x] = fmaxf(lds[d][threadIdx.x], lds[d][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    qbox[2 * blockIdx.x] = make_float4(lds[0][0], lds[1][0], lds[2][0], 0.0f);
    qbox[2 * blockIdx.x + 1] = make_float4(lds[3][0], lds[4][0], lds[5][0], 0.0f);
  }
}

// Sum of `split` partials of accumulator `a` for sorted query i, in split order.
__device__ __forceinline__ float combine(const float* part, int split, int64_t mpad, int na, int a, int64_t i,
                                         bool kahan) {
  float s = 0.0f, c = 0.0f;
  for (int p = 0; p < split; ++p) {
    const float x = part[((int64_t)p * na + a) * mpad + i];
    if (kahan) {
      const float y = x - c;
      const float t = s + y;
      c = (t - s) - y;
      s = t;
    } else {
      s += x;
    }
  }
  return kahan ? s - c : s;
}

// Block-wide FP64 sum (deterministic: fixed shuffle tree, then fixed LDS order).
__device__ double block_sum(double v, double* lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += lds[k];
  return r;  // valid on thread 0
}

// Output scaling of the accumulators: w = ws w', grad = as A - bs B'.
struct Scale {
  float ws, as, bs;
};
Scale scale_of(const dwg_kernel_params& kp) {
  if (!(kp.lambda > 0.0f)) return Scale{1.0f, 3.0f, 1.0f};
  // screened sums in scaled coordinates: w' carries 1/kappa^2, A and B' carry 1/kappa^3
  const double k = position_scale(kp);
  return Scale{(float)(k * k / 3.0), (float)(k * k * k), (float)(k * k * k / 3.0)};
}

// Evaluation epilogue: combine splits; write w and grad at the query's original index;
// FP64 block partial of w.
__global__ __launch_bounds__(kRedBlock) void k_combine(const float* __restrict__ part, int split,
                                                       int64_t mpad, int64_t m, bool grad, Scale sc,
                                                       bool kahan, const int32_t* __restrict__ qperm,
                                                       float* __restrict__ wout,
                                                       float* __restrict__ gout,
                                                       double* __restrict__ blk) {
  __shared__ double lds[kRedBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double wv = 0.0;
  if (i < m) {
    const int na = grad ? kNAcc : 1;
    const int64_t o = qperm[i];
    const float w = sc.ws * combine(part, split, mpad, na, 0, i, kahan);
    if (grad) {
      for (int d = 0; d < 3; ++d) {
        const float A = combine(part, split, mpad, na, 1 + d, i, kahan);
        const float B = combine(part, split, mpad, na, 4 + d, i, kahan);
        gout[d * m + o] = fmaf(sc.as, A, -sc.bs * B);
      }
    }
    if (wout) wout[o] = w;
    wv = (double)w;
  }
  const double bs = block_sum(wv, lds);
  if (threadIdx.x == 0) blk[blockIdx.x] = bs;
}

// Iteration epilogue (Eq. 7): n_new = -grad/|grad| (kept when |grad| is 0 or not finite),
// written in place at the point's original index; restage m for the next iteration;
// theta_i (degrees, FP64); FP64 block partials of w and of the chord |n_new - n_old|.
__global__ __launch_bounds__(kRedBlock) void k_update(const float* __restrict__ part, int split,
                                                      int64_t mpad, int64_t n, Scale sc, bool kahan,
                                                      const int32_t* __restrict__ perm,
                                                      const float* __restrict__ kk,
                                                      float* __restrict__ N,
                                                      float4* __restrict__ src,
                                                      double* __restrict__ theta,
                                                      double* __restrict__ blk, int nblk) {
  __shared__ double lds[kRedBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double wv = 0.0, cv = 0.0;
  if (i < n) {
    const float w = sc.ws * combine(part, split, mpad, kNAcc, 0, i, kahan);
    float g[3];
    for (int d = 0; d < 3; ++d) {
      const float A = combine(part, split, mpad, kNAcc, 1 + d, i, kahan);
      const float B = combine(part, split, mpad, kNAcc, 4 + d, i, kahan);
      g[d] = fmaf(sc.as, A, -sc.bs * B);
    }
    const int64_t o = perm[i];
    const float o0 = N[o], o1 = N[n + o], o2 = N[2 * n + o];
    const double gl = sqrt((double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2]);
    float n0 = o0, n1 = o1, n2 = o2;
    if (gl > 0.0 && gl <= 1.7976931348623157e308) {
      n0 = (float)(-(double)g[0] / gl);
      n1 = (float)(-(double)g[1] / gl);
      n2 = (float)(-(double)g[2] / gl);
    }
    const double e0 = (double)n0 - o0, e1 = (double)n1 - o1, e2 = (double)n2 - o2;
    const double ch = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    const double h = 0.5 * ch;
    theta[i] = 2.0 * asin(h < 1.0 ? h : 1.0) * kRadToDeg;
    N[o] = n0;
    N[n + o] = n1;
    N[2 * n + o] = n2;
    const float k = kk[i];
    src[2 * i + 1] = make_float4(k * n0, k * n1, k * n2, 0.0f);
    wv = (double)w;
    cv = ch;
  }
  const double bw = block_sum(wv, lds);
  const double bc = block_sum(cv, lds);
  if (threadIdx.x == 0) {
    blk[blockIdx.x] = bw;
    blk[nblk + blockIdx.x] = bc;
  }
}

// Fixed-order sum of the block partials: stats[0] = sum w / n, stats[2] = sum chord / n;
// also resets the radix-select state for k largest values.
__global__ __launch_bounds__(kRedBlock) void k_sums(const double* __restrict__ blk, int nblk,
                                                    int64_t n, int64_t k, int with_chord,
                                                    double* __restrict__ stats,
                                                    uint32_t* __restrict__ hist,
                                                    uint64_t* __restrict__ sel) {
  __shared__ double lds[kRedBlock / 64];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
    a += blk[i];
    if (with_chord) b += blk[nblk + i];
  }
  const double sa = block_sum(a, lds);
  const double sb = block_sum(b, lds);
  if (threadIdx.x == 0) {
    stats[0] = sa / (double)n;
    stats[2] = sb / (double)n;
    sel[0] = 0;
    sel[1] = (uint64_t)k;
  }
  for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
}

// One radix-select pass over the FP64 bit patterns (non-negative doubles order like
// unsigned integers): histogram of digit (bits >> shift) & 255 among values whose higher
// bits equal the prefix selected so far.
__global__ __launch_bounds__(kRedBlock) void k_radix_hist(const double* __restrict__ theta,
                                                          int64_t n, int shift,
                                                          const uint64_t* __restrict__ sel,
                                                          uint32_t* __restrict__ hist) {
  __shared__ uint32_t lh[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) lh[i] = 0;
  __syncthreads();
  const uint64_t prefix = sel[0];
  const uint64_t hmask = shift >= 56 ? 0ull : (~0ull << (shift + 8));
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t bits = (uint64_t)__double_as_longlong(theta[i]);
    if ((bits & hmask) == (prefix & hmask)) atomicAdd(&lh[(bits >> shift) & 255u], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x)
    if (lh[i]) atomicAdd(&hist[i], lh[i]);
}

// Picks the digit holding the k-th largest value, extends the prefix, clears the histogram.
// One block of 256 threads, one per digit: with cum[d] = the count of digits >= d (a suffix
// scan in LDS), the digit taken is the largest d with cum[d] >= krem, and krem drops by
// cum[d + 1] -- what walking the digits down from 255 and subtracting their counts until
// krem <= count gives. If no digit qualifies the prefix is kept and krem drops by the total.
__global__ __launch_bounds__(256) void k_radix_select(int shift, uint64_t* __restrict__ sel,
                                                      uint32_t* __restrict__ hist) {
  __shared__ uint64_t cum[257];
  __shared__ int found;
  const int t = threadIdx.x;
  cum[t] = hist[t];
  if (t == 0) {
    cum[256] = 0;
    found = -1;
  }
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive suffix scan
    const uint64_t x = t + off < 256 ? cum[t + off] : 0;
    __syncthreads();
    cum[t] += x;
    __syncthreads();
  }
  const uint64_t krem = sel[1];
  if (cum[t] >= krem && (t == 255 || cum[t + 1] < krem)) found = t;  // the largest such digit
  __syncthreads();
  if (t == 0) {
    if (found >= 0) {
      sel[0] |= (uint64_t)found << shift;
      sel[1] = krem - cum[found + 1];
    } else {
      sel[1] = krem - cum[0];
    }
  }
  hist[t] = 0;
}

// FP64 block partials of the sum of theta_i strictly above the selected k-th largest value.
__global__ __launch_bounds__(kRedBlock) void k_top_partial(const double* __restrict__ theta, int64_t n,
                                                           const uint64_t* __restrict__ sel,
                                                           double* __restrict__ blk) {
  __shared__ double lds[kRedBlock / 64];
  const uint64_t thr = sel[0];
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double x = theta[i];
    if ((uint64_t)__double_as_longlong(x) > thr) v += x;
  }
  const double b = block_sum(v, lds);
  if (threadIdx.x == 0) blk[blockIdx.x] = b;
}

__global__ __launch_bounds__(kRedBlock) void k_top_final(const double* __restrict__ blk, int nblk,
                                                         int64_t k, const uint64_t* __restrict__ sel,
                                                         double* __restrict__ stats) {
  __shared__ double lds[kRedBlock / 64];
  double a = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) a += blk[i];
  const double s = block_sum(a, lds);
  if (threadIdx.x == 0) {
    const double t = __longlong_as_double((long long)sel[0]);
    stats[1] = (s + (double)sel[1] * t) / (double)k;
  }
}

// SplitMix64 output number t of the stream started at `seed` (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t t) {
  uint64_t z = seed + (t + 1ull) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void k_random_normals(uint64_t seed, int64_t n, float* __restrict__ N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float u0 = (float)(splitmix64(seed, 2ull * i) >> 40) * 0x1p-24f;
  const float u1 = (float)(splitmix64(seed, 2ull * i + 1ull) >> 40) * 0x1p-24f;
  const float z = 1.0f - 2.0f * u0;                 // exact
  const float rr = sqrtf((1.0f - z) * (1.0f + z));  // one rounding before the sqrt
  float sn, cs;
  sincosf(6.28318530717958647692f * u1, &sn, &cs);
  N[i] = rr * cs;
  N[n + i] = rr * sn;
  N[2 * n + i] = z;
}

template <int QPT, bool GRAD, bool SCREENED, bool KAHAN>
void launch_gwn_t(dim3 grid, hipStream_t st, const float* Q, int64_t m, const int32_t* qperm,
                  const GwnWork& w, int64_t tps, float kappa) {
  const int64_t nfull = w.n_src / kTile;  // tiles without padding
  hipLaunchKernelGGL((k_gwn<QPT, GRAD, SCREENED, KAHAN>), grid, dim3(kBlock), 0, st, Q, m, qperm, w.src,
                     w.ntiles, nfull, tps, w.tbox, w.qbox, kScaledScr, kappa, w.part, w.mpad);
}

}  // namespace

float position_scale(const dwg_kernel_params& kp) {
  return kp.lambda > 0.0f ? (float)(std::sqrt((double)kp.lambda) * 1.4426950408889634) : 1.0f;
}

int choose_split(int64_t n_src, int64_t n_qry, int requested) {
  const int64_t ntiles = cdiv(n_src, kTile);
  if (requested > 0) return (int)std::min<int64_t>(std::min<int64_t>(requested, kMaxSplit), ntiles);
  const int64_t qblocks = cdiv(n_qry, kQBlock);
  // Aim for >= 32768 blocks (128 per CU, ~25 rounds of resident blocks) while every split keeps
  // >= 8 tiles: blocks differ in cost (near tiles take the longer path), and the last round of
  // a launch with few rounds leaves CUs idle. Measured: 1M x 1M 2 splits 599 ms, 6 splits
  // 556 ms, 16 splits 550 ms; 100K x 100K 16 splits 6.14 ms, 48 splits 5.70 ms. The partial
  // sums (28 B per query and split) are held to kAutoSplitBytes, or 16 splits if that is more.
  int64_t s = cdiv(32768, qblocks);
  s = std::min<int64_t>(s, std::max<int64_t>(1, ntiles / 8));
  const int64_t mem_cap =
      std::max<int64_t>(16, (int64_t)(kAutoSplitBytes / ((int64_t)kNAcc * 4 * qblocks * kQBlock)));
  s = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(s, mem_cap), kMaxSplit));
  return (int)s;
}

size_t carve_gwn(Carver& c, int64_t n_src, int64_t n_qry, int split, bool same, GwnWork* out) {
  GwnWork w{};
  w.n_src = n_src;
  w.ntiles = cdiv(n_src, kTile);
  w.npad = w.ntiles * kTile;
  w.mpad = cdiv(n_qry, kQBlock) * kQBlock;
  w.split = split;
  w.nblk = (int)cdiv(std::max(n_src, n_qry), kRedBlock);
  const size_t start = c.used;
  w.src = c.take<float4>(2 * (size_t)w.npad);
  w.part = c.take<float>((size_t)split * kNAcc * (size_t)w.mpad);
  w.kk = c.take<float>((size_t)w.npad);
  w.theta = c.take<double>((size_t)std::max(n_src, n_qry));
  w.blk = c.take<double>(2 * (size_t)w.nblk);
  w.stats = c.take<double>(4);
  w.hist = c.take<uint32_t>(256);
  w.sel = c.take<uint64_t>(2);
  w.tbox = c.take<float4>(2 * (size_t)w.ntiles);
  w.qbox = c.take<float4>(2 * (size_t)(w.mpad / kQBlock));
  w.perm_s = c.take<int32_t>((size_t)w.npad);
  w.perm_q = same ? w.perm_s : c.take<int32_t>((size_t)w.mpad);
  carve_sort(c, std::max(n_src, n_qry), &w.sort);
  if (out) *out = w;
  return c.used - start;
}

dwg_status launch_stage(const float* P, const float* N, const float* area, const float* delta,
                        int64_t n, float eps, float kappa, const GwnWork& w, hipStream_t stream) {
  hipLaunchKernelGGL(k_stage, dim3((unsigned)cdiv(w.npad, 256)), dim3(256), 0, stream, P, N, area,
                     delta, n, w.npad, eps, kappa, w.perm_s, w.src, w.kk);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_tile_box, dim3((unsigned)w.ntiles), dim3(kTile), 0, stream, w.src, n, kappa, w.tbox);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status launch_order(const float* P, int64_t n, const float* delta, float eps, float kappa, const float* Q,
                        int64_t m, bool same, const GwnWork& w, hipStream_t stream) {
  dwg_status s = spatial_sort(P, n, delta, eps, w.sort, w.perm_s, stream);
  if (s != DWG_OK) return s;
  if (!same) {
    s = spatial_sort(Q, m, nullptr, 0.0f, w.sort, w.perm_q, stream);
    if (s != DWG_OK) return s;
  }
  hipLaunchKernelGGL(k_query_box, dim3((unsigned)(w.mpad / kQBlock)), dim3(kBlock), 0, stream, Q, m, w.perm_q,
                     w.qbox);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status launch_gwn(const float* Q, int64_t m, const dwg_kernel_params& kp, bool grad,
                      const GwnWork& w, hipStream_t stream) {
  const int64_t qblocks = cdiv(m, kQBlock);
  const int64_t tps = cdiv(w.ntiles, w.split);
  dim3 grid((unsigned)qblocks, (unsigned)w.split);
  const bool scr = kp.lambda > 0.0f;
  const bool kah = kp.compensated != 0;
  const float kappa = position_scale(kp);
#define DWG_GWN_CASE(G, S, K) \
  if (grad == G && scr == S && kah == K) launch_gwn_t<kQpt, G, S, K>(grid, stream, Q, m, w.perm_q, w, tps, kappa);
  DWG_GWN_CASE(true, false, true)
  DWG_GWN_CASE(true, false, false)
  DWG_GWN_CASE(true, true, true)
  DWG_GWN_CASE(true, true, false)
  DWG_GWN_CASE(false, false, true)
  DWG_GWN_CASE(false, false, false)
  DWG_GWN_CASE(false, true, true)
  DWG_GWN_CASE(false, true, false)
#undef DWG_GWN_CASE
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status launch_combine(int64_t m, const dwg_kernel_params& kp, bool grad, float* wout,
                          float* gout, double* wmean, const GwnWork& w, hipStream_t stream) {
  const int nb = (int)cdiv(m, kRedBlock);
  hipLaunchKernelGGL(k_combine, dim3(nb), dim3(kRedBlock), 0, stream, w.part, w.split, w.mpad, m, grad,
                     scale_of(kp), kp.compensated != 0, w.perm_q, wout, gout, w.blk);
  DWG_TRY_LAUNCH();
  if (wmean) {
    hipLaunchKernelGGL(k_sums, dim3(1), dim3(kRedBlock), 0, stream, w.blk, nb, m, (int64_t)1, 0,
                       w.stats, w.hist, w.sel);
    DWG_TRY_LAUNCH();
    DWG_TRY_HIP(hipMemcpyAsync(wmean, w.stats, sizeof(double), hipMemcpyDeviceToDevice, stream));
  }
  return DWG_OK;
}

dwg_status launch_update(int64_t n, const dwg_kernel_params& kp, float* N, const GwnWork& w,
                         hipStream_t stream) {
  const int nb = (int)cdiv(n, kRedBlock);
  hipLaunchKernelGGL(k_update, dim3(nb), dim3(kRedBlock), 0, stream, w.part, w.split, w.mpad, n, scale_of(kp),
                     kp.compensated != 0, w.perm_s, w.kk, N, w.src, w.theta, w.blk, nb);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

static int64_t top_count(int64_t n, double top_frac) {
  int64_t k = (int64_t)std::ceil(top_frac * (double)n);
  if (k < 1) k = 1;
  if (k > n) k = n;
  return k;
}

dwg_status launch_stats(int64_t n, double top_frac, const GwnWork& w, hipStream_t stream) {
  const int nb = (int)cdiv(n, kRedBlock);
  const int64_t k = top_count(n, top_frac);
  hipLaunchKernelGGL(k_sums, dim3(1), dim3(kRedBlock), 0, stream, w.blk, nb, n, k, 1, w.stats, w.hist,
                     w.sel);
  DWG_TRY_LAUNCH();
  const int hb = (int)std::min<int64_t>(cdiv(n, kRedBlock), 1024);
  for (int shift = 56; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(hb), dim3(kRedBlock), 0, stream, w.theta, n, shift, w.sel,
                       w.hist);
    DWG_TRY_LAUNCH();
    hipLaunchKernelGGL(k_radix_select, dim3(1), dim3(256), 0, stream, shift, w.sel, w.hist);
    DWG_TRY_LAUNCH();
  }
  hipLaunchKernelGGL(k_top_partial, dim3(hb), dim3(kRedBlock), 0, stream, w.theta, n, w.sel, w.blk);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_top_final, dim3(1), dim3(kRedBlock), 0, stream, w.blk, hb, k, w.sel, w.stats);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status launch_random_normals(uint64_t seed, int64_t n, float* N, hipStream_t stream) {
  hipLaunchKernelGGL(k_random_normals, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, stream, seed, n, N);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

}  // namespace dwg
