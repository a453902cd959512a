// Per-pair arithmetic of the (screened) GWN kernel shared by the all-pairs and the octree
// kernels (Sec. 3 Eq. 2-3, Sec. 4.2 Eq. 5, Sec. 5.2 modified Poisson kernel). Accumulators:
// acc[0] = w (x3 when screened), acc[1..3] = A, acc[4..6] = B (x3 when screened); the
// gradient is 3A - B (plain) or A - B/3 (screened), scaled by the evaluation epilogue.
#pragma once

#include <hip/hip_runtime.h>

namespace dwg {
namespace pairk {

constexpr float kInv4Pi = 0.0795774715459476678844f;
// 2^126: r2 * kCoincide is 0 exactly when r2 == 0 and larger than 1/r for every pair with
// r2 >= 2^-84; it is the third operand of the min that zeroes coincident pairs.
constexpr float kCoincide = 8.507059173023462e37f;
// Added to r2 before rsqrt in the general screened path so that r = r2 * rsqrt(r2 + tiny) is
// 0 (not 0 * inf) for coincident pairs; below half an ulp of any r2 >= 2^-84.
constexpr float kTiny = 1e-37f;

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }

// min of three non-negative floats (+inf allowed) through their bit patterns, which order
// like unsigned integers for non-negative IEEE values: one v_min3_u32, no NaN handling.
__device__ __forceinline__ float min3_nonneg(float a, float b, float c) {
  const unsigned x = __float_as_uint(a), y = __float_as_uint(b), z = __float_as_uint(c);
  return __uint_as_float(min(min(x, y), z));
}

// Per-pair constants of the screened kernel. The screened kernel works in scaled coordinates
// x' = kappa x with kappa = s log2(e) (the sources are staged and the queries loaded that
// way), so that e^{-s r} = 2^{-r'} needs no multiply; then s r = ln(2) r' and the s^2 term
// becomes ln(2)^2 in units of 1/r'^2. The epilogue multiplies the sums by the powers of kappa.
struct Scr {
  float s3;  // 3 s / kappa = 3 ln 2
  float s2;  // s^2 / kappa^2 = (ln 2)^2
};
constexpr Scr kScaledScr{2.0794415416798359f, 0.48045301391820144f};

// One (query, source) pair of the plain kernel (Eq. 2-3 with the modified Poisson kernel).
//   ip = 1/rho = min(1/r, 1/max(delta,eps)), and 0 when r == 0 (pair skipped).
//   w += c ip^3;  B += ip^3 m;  A += [rho == r] c ip^5 d;  grad = 3 A - B.
// FAR: the caller guarantees r > max(delta_j, eps) > = 0 and r > 0, so ip = 1/r.
// dx, dy, dz = p_j - q; iw = 1/max(delta_j, eps) (unused when FAR); b = (m_j, -).
template <bool GRAD, bool FAR>
__device__ __forceinline__ void pair_plain_d(float dx, float dy, float dz, float iw, const float4 b,
                                             float* acc) {
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  const float ir = rsq(r2);
  const float ip = FAR ? ir : min3_nonneg(ir, iw, r2 * kCoincide);
  const float ip2 = ip * ip;
  const float ip3 = ip2 * ip;
  const float c = fmaf(dz, b.z, fmaf(dy, b.y, dx * b.x));
  if (!GRAD) {
    acc[0] = fmaf(c, ip3, acc[0]);
  } else {
    const float e = c * ip3;
    acc[0] += e;
    acc[4] = fmaf(ip3, b.x, acc[4]);
    acc[5] = fmaf(ip3, b.y, acc[5]);
    acc[6] = fmaf(ip3, b.z, acc[6]);
    const float t = (FAR || ir <= iw) ? e * ip2 : 0.0f;
    acc[1] = fmaf(t, dx, acc[1]);
    acc[2] = fmaf(t, dy, acc[2]);
    acc[3] = fmaf(t, dz, acc[3]);
  }
}

template <bool GRAD, bool FAR>
__device__ __forceinline__ void pair_plain(const float4 a, const float4 b, float qx, float qy,
                                           float qz, float* acc) {
  pair_plain_d<GRAD, FAR>(a.x - qx, a.y - qy, a.z - qz, a.w, b, acc);
}

// One pair of the screened kernel (Eq. 5), in the scaled coordinates above (r is r'):
// E = e^{-s r} = 2^{-r'}, o3 = 3 (1 + s r), f = E ip^3.
//   w' += c f o3            (= 3 w)
//   B' += f o3 m            (= 3 B with B = sum phi ip^3 m)
//   A  += c f (o3 ip^2 [rho == r] + s^2) d
//   grad = A - B' / 3,  w = w' / 3.
template <bool GRAD, bool FAR>
__device__ __forceinline__ void pair_screened_d(float dx, float dy, float dz, float iw, const float4 b,
                                                const Scr k, float* acc) {
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  const float ir = rsq(FAR ? r2 : r2 + kTiny);
  const float ip = FAR ? ir : min3_nonneg(ir, iw, r2 * kCoincide);
  const float ip2 = ip * ip;
  const float ip3 = ip2 * ip;
  const float r = r2 * ir;
  const float E = exp2_hw(-r);
  const float o3 = fmaf(k.s3, r, 3.0f);
  const float f = E * ip3;
  const float c = fmaf(dz, b.z, fmaf(dy, b.y, dx * b.x));
  const float e0 = c * f;
  acc[0] = fmaf(e0, o3, acc[0]);
  if (GRAD) {
    const float g = f * o3;
    acc[4] = fmaf(g, b.x, acc[4]);
    acc[5] = fmaf(g, b.y, acc[5]);
    acc[6] = fmaf(g, b.z, acc[6]);
    const float h = fmaf(o3, ip2, k.s2);
    const float t = e0 * ((FAR || ir <= iw) ? h : k.s2);
    acc[1] = fmaf(t, dx, acc[1]);
    acc[2] = fmaf(t, dy, acc[2]);
    acc[3] = fmaf(t, dz, acc[3]);
  }
}

template <bool GRAD, bool FAR>
__device__ __forceinline__ void pair_screened(const float4 a, const float4 b, float qx, float qy,
                                              float qz, const Scr k, float* acc) {
  pair_screened_d<GRAD, FAR>(a.x - qx, a.y - qy, a.z - qz, a.w, b, k, acc);
}

// Far pairs in separated form, for a source tile well separated from a block of queries that
// are all close to one centre c. Positions are relative to c; the source is staged as
// a = (P, pp) with P = -2 p and pp = |p|^2, b = (m, mp) with mp = m . p, and the query brings
// qq = |q|^2. Then r^2 = pp + qq + P . q and c = m . (p - q) = mp - m . q need no difference
// vector, and the A sums collect t P and t; the caller forms A = -sum(t P) / 2 - q sum(t)
// (acc[7] = sum t) once per tile. This is one issue slot per pair fewer than the difference
// form (three differences against the qq add and the sum of t). The rounding of r^2 and c
// is relative to (|p| + |q|)^2 and |m| (|p| + |q|) rather than to r^2 and |m| r, so the caller
// takes this form only where r >= max|q|: then |p| + |q| <= 3 r, which bounds both ratios by
// 9 and 3.
// The caller computes r^2 (sep_r2) and ir = 1/sqrt(r^2) of all its queries first.
__device__ __forceinline__ float sep_r2(const float4 a, float qx, float qy, float qz, float qq) {
  return fmaf(a.z, qz, fmaf(a.y, qy, fmaf(a.x, qx, a.w + qq)));
}

template <bool GRAD>
__device__ __forceinline__ void pair_plain_sep(const float4 a, const float4 b, float qx, float qy,
                                               float qz, float ip, float* acc) {
  const float c = fmaf(-b.z, qz, fmaf(-b.y, qy, fmaf(-b.x, qx, b.w)));
  const float ip2 = ip * ip;
  const float ip3 = ip2 * ip;
  if (!GRAD) {
    acc[0] = fmaf(c, ip3, acc[0]);
  } else {
    const float e = c * ip3;
    acc[0] += e;
    acc[4] = fmaf(ip3, b.x, acc[4]);
    acc[5] = fmaf(ip3, b.y, acc[5]);
    acc[6] = fmaf(ip3, b.z, acc[6]);
    const float t = e * ip2;
    acc[1] = fmaf(t, a.x, acc[1]);
    acc[2] = fmaf(t, a.y, acc[2]);
    acc[3] = fmaf(t, a.z, acc[3]);
    acc[7] += t;
  }
}

template <bool GRAD>
__device__ __forceinline__ void pair_screened_sep(const float4 a, const float4 b, float qx, float qy,
                                                  float qz, float r2, float ir, const Scr k, float* acc) {
  const float c = fmaf(-b.z, qz, fmaf(-b.y, qy, fmaf(-b.x, qx, b.w)));
  const float ip2 = ir * ir;
  const float ip3 = ip2 * ir;
  const float r = r2 * ir;
  const float E = exp2_hw(-r);
  const float o3 = fmaf(k.s3, r, 3.0f);
  const float f = E * ip3;
  const float e0 = c * f;
  acc[0] = fmaf(e0, o3, acc[0]);
  if (GRAD) {
    const float g = f * o3;
    acc[4] = fmaf(g, b.x, acc[4]);
    acc[5] = fmaf(g, b.y, acc[5]);
    acc[6] = fmaf(g, b.z, acc[6]);
    const float t = e0 * fmaf(o3, ip2, k.s2);
    acc[1] = fmaf(t, a.x, acc[1]);
    acc[2] = fmaf(t, a.y, acc[2]);
    acc[3] = fmaf(t, a.z, acc[3]);
    acc[7] += t;
  }
}

}  // namespace pairk
}  // namespace dwg
