// FP64 device math for the response kernels.  Phases are carried in cycles and
// reduced exactly (x - rint(x) is exact in binary floating point) before a
// short polynomial, so no general-purpose transcendental with its
// large-argument reduction sits in the hot loop.
#pragma once
#include <hip/hip_runtime.h>

#include "pes_poly.hpp"

namespace pes {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.141592653589793238462643383279503;

template <int N>
__device__ __forceinline__ double horner(const double (&c)[N], double t) {
  double p = c[0];
#pragma unroll
  for (int i = 1; i < N; ++i) p = fma(p, t, c[i]);
  return p;
}

// sin(2 pi x), cos(2 pi x) for any finite x given in cycles.
// r = x - rint(x) in [-1/2, 1/2], quadrant q = rint(4 r) in {-2, ..., 2},
// y = r - q/4 in [-1/8, 1/8] (all exact), then the fitted polynomials and the
// rotation by q quarter turns, (cos, sin)(q pi/2) = (1 - |q|, q (2 - |q|)):
// products with 0 and +-1, so exact, and FP64 arithmetic instead of integer
// selects.
__device__ __forceinline__ void sincos_cycles(double x, double& s, double& c) {
  const double r = x - rint(x);
  const double q = rint(4.0 * r);
  const double y = fma(-0.25, q, r);
  const double t = y * y;
  const double sy = y * horner(kSin2pi, t);
  const double cy = horner(kCos2pi, t);
  const double aq = fabs(q);
  const double cq = 1.0 - aq;
  const double sq = q * (2.0 - aq);
  s = fma(sy, cq, cy * sq);
  c = fma(cy, cq, -(sy * sq));
}

// sin(b)/b as a polynomial in b^2.  LONG selects the fit valid to b = 4
// (12 terms) instead of b^2 <= 4.9 (10 terms); the host picks the short one
// whenever every detector's largest argument 2 pi f_max L allows it.
template <bool LONG>
__device__ __forceinline__ double sinc(double b) {
  const double t = b * b;
  return LONG ? horner(kSincLong, t) : horner(kSincShort, t);
}

// sin(x), cos(x) for |x| <= 0.7 without argument reduction.
__device__ __forceinline__ void sincos_small(double x, double& s, double& c) {
  const double t = x * x;
  s = x * horner(kSinSmall, t);
  c = horner(kCosSmall, t);
}

// ---- FP32 versions for the single-precision log-likelihood kernel (fits at
// FP32 accuracy, fewer terms).
template <int N>
__device__ __forceinline__ float horner(const float (&c)[N], float t) {
  float p = c[0];
#pragma unroll
  for (int i = 1; i < N; ++i) p = fmaf(p, t, c[i]);
  return p;
}

// sin(2 pi x), cos(2 pi x) for x in cycles given as the FP32 residue r of an
// exact FP64 reduction (|r| <= 1/2): quadrant and polynomial as in the FP64
// version.
__device__ __forceinline__ void sincos_rev_f(float r, float& s, float& c) {
  const float q = rintf(4.0f * r);
  const float y = fmaf(-0.25f, q, r);
  const float t = y * y;
  const float sy = y * horner(kSin2piF, t);
  const float cy = horner(kCos2piF, t);
  const float aq = fabsf(q);
  const float cq = 1.0f - aq;
  const float sq = q * (2.0f - aq);
  s = fmaf(sy, cq, cy * sq);
  c = fmaf(cy, cq, -(sy * sq));
}
// The same for any FP64 argument: the integer part is removed exactly in FP64.
__device__ __forceinline__ void sincos_cycles_f(double x, float& s, float& c) {
  sincos_rev_f((float)(x - rint(x)), s, c);
}
template <bool LONG>
__device__ __forceinline__ float sinc_f(float b) {
  const float t = b * b;
  return LONG ? horner(kSincLongF, t) : horner(kSincShortF, t);
}
__device__ __forceinline__ void sincos_small_f(float x, float& s, float& c) {
  const float t = x * x;
  s = x * horner(kSinSmallF, t);
  c = horner(kCosSmallF, t);
}

// Derivative-carrying versions for the tangent (forward-mode) kernels.
template <int N> struct Dual;

template <int N, int M>
__device__ __forceinline__ void horner_d(const double (&c)[M], double t, double& p, double& dp) {
  // p = P(t), dp = P'(t) in one pass
  p = c[0];
  dp = 0.0;
#pragma unroll
  for (int i = 1; i < M; ++i) {
    dp = fma(dp, t, p);
    p = fma(p, t, c[i]);
  }
}

// Exact split of a product: p + e == a * b exactly (e from one fused multiply-add).
__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = fma(a, b, -p);
}

// 64-lane wavefront sum (butterfly over the full wave; every lane ends with the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// 64-lane wavefront maximum (every lane ends with it).
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// One DPP lane permutation of a double (two 32-bit moves).  Rows outside
// ROW_MASK receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// 64-lane wavefront sum with data-parallel-primitive moves: pairs, quads
// (quad_perm), 8 lanes (row_half_mirror), rows of 16 (row_mirror), then the
// row broadcasts of lanes 15 and 31; lane 63 holds the total, returned to the
// whole wave.  Fixed order, so results are bitwise repeatable.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
  v += dpp_f64<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
  v += dpp_f64<0x141, 0xf>(v);   // row_half_mirror
  v += dpp_f64<0x140, 0xf>(v);   // row_mirror
  v += dpp_f64<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

}  // namespace pes
