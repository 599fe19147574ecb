// Forward-mode dual numbers for the derivative kernels: Dual<N> carries a value
// and N tangents.  Used with N = 11 in the per-walker setup (derivatives of
// every walker constant with respect to theta) and N = 1 in the per-bin
// evaluation (one tangent direction per pass).
#pragma once
#include <hip/hip_runtime.h>

namespace pes {

// The double-precision functions stay visible next to the dual overloads below.
using ::cbrt;
using ::cos;
using ::fma;
using ::log;
using ::sin;
using ::sqrt;

template <int N>
struct Dual {
  double v;
  double d[N];
  __device__ Dual() {}
  __device__ Dual(double x) : v(x) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
};

template <int N>
__device__ __forceinline__ Dual<N> mk(double v, const Dual<N>& a, double s) {  // f(a), f'(a) = s
  Dual<N> r;
  r.v = v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = s * a.d[i];
  return r;
}
template <int N> __device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N> __device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N> __device__ __forceinline__ Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N> __device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = fma(a.d[i], b.v, a.v * b.d[i]);
  return r;
}
template <int N> __device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <int N> __device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, double b) {
  Dual<N> r = a; r.v += b; return r;
}
template <int N> __device__ __forceinline__ Dual<N> operator+(double b, const Dual<N>& a) { return a + b; }
template <int N> __device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, double b) {
  Dual<N> r = a; r.v -= b; return r;
}
template <int N> __device__ __forceinline__ Dual<N> operator-(double b, const Dual<N>& a) { return -(a - b); }
template <int N> __device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r; r.v = a.v * b;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <int N> __device__ __forceinline__ Dual<N> operator*(double b, const Dual<N>& a) { return a * b; }
template <int N> __device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> __device__ __forceinline__ Dual<N> operator/(double a, const Dual<N>& b) {
  const double r = a / b.v;
  return mk(r, b, -r / b.v);
}
template <int N> __device__ __forceinline__ Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }
template <int N> __device__ __forceinline__ Dual<N>& operator*=(Dual<N>& a, const Dual<N>& b) { a = a * b; return a; }
template <int N> __device__ __forceinline__ Dual<N>& operator*=(Dual<N>& a, double b) { a = a * b; return a; }

// a * b + c
template <int N> __device__ __forceinline__ Dual<N> fma(const Dual<N>& a, const Dual<N>& b, const Dual<N>& c) {
  Dual<N> r; r.v = ::fma(a.v, b.v, c.v);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = ::fma(a.d[i], b.v, ::fma(a.v, b.d[i], c.d[i]));
  return r;
}
template <int N> __device__ __forceinline__ Dual<N> fma(double a, const Dual<N>& b, const Dual<N>& c) {
  Dual<N> r; r.v = ::fma(a, b.v, c.v);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = ::fma(a, b.d[i], c.d[i]);
  return r;
}
template <int N> __device__ __forceinline__ Dual<N> fma(const Dual<N>& a, double b, const Dual<N>& c) {
  return fma(b, a, c);
}
template <int N> __device__ __forceinline__ Dual<N> fma(const Dual<N>& a, const Dual<N>& b, double c) {
  Dual<N> r; r.v = ::fma(a.v, b.v, c);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = ::fma(a.d[i], b.v, a.v * b.d[i]);
  return r;
}
template <int N> __device__ __forceinline__ Dual<N> fma(const Dual<N>& a, double b, double c) {
  Dual<N> r; r.v = ::fma(a.v, b, c);
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <int N> __device__ __forceinline__ Dual<N> fma(double a, const Dual<N>& b, double c) {
  return fma(b, a, c);
}
template <int N> __device__ __forceinline__ Dual<N> fma(double a, double b, const Dual<N>& c) {
  Dual<N> r = c; r.v = ::fma(a, b, c.v); return r;
}

template <int N> __device__ __forceinline__ Dual<N> sin(const Dual<N>& a) { return mk(::sin(a.v), a, ::cos(a.v)); }
template <int N> __device__ __forceinline__ Dual<N> cos(const Dual<N>& a) { return mk(::cos(a.v), a, -::sin(a.v)); }
template <int N> __device__ __forceinline__ Dual<N> log(const Dual<N>& a) { return mk(::log(a.v), a, 1.0 / a.v); }
template <int N> __device__ __forceinline__ Dual<N> sqrt(const Dual<N>& a) {
  const double s = ::sqrt(a.v);
  return mk(s, a, 0.5 / s);
}
template <int N> __device__ __forceinline__ Dual<N> cbrt(const Dual<N>& a) {
  const double c = ::cbrt(a.v);
  return mk(c, a, 1.0 / (3.0 * c * c));
}

__device__ __forceinline__ double val(double x) { return x; }
template <int N> __device__ __forceinline__ double val(const Dual<N>& x) { return x.v; }

}  // namespace pes
