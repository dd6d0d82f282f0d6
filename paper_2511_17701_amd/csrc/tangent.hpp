// tangent.hpp -- FP64 value with N directional derivatives (forward-mode
// tangents), for the per-step Jacobian of the adjoint.  The templated metric,
// tetrad and Boris code of geometry.hpp / particles.hpp runs on it unchanged.
#pragma once

#include "geometry.hpp"

namespace grpic {

// the FP64 library functions stay visible next to the overloads below
using ::exp;
using ::sincos;
using ::sqrt;

template <int N>
struct Tan {
  double v;
  double d[N];
  Tan() = default;
  __host__ __device__ Tan(double x) : v(x) {  // a constant: zero tangents
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = 0.0;
  }
};

// the k-th input variable with value x
template <int N>
__device__ inline Tan<N> seed(double x, int k) {
  Tan<N> t(x);
  t.d[k] = 1.0;
  return t;
}

template <int N>
__device__ inline Tan<N> operator+(const Tan<N>& a, const Tan<N>& b) {
  Tan<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int N>
__device__ inline Tan<N> operator-(const Tan<N>& a, const Tan<N>& b) {
  Tan<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int N>
__device__ inline Tan<N> operator-(const Tan<N>& a) {
  Tan<N> r;
  r.v = -a.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int N>
__device__ inline Tan<N> operator*(const Tan<N>& a, const Tan<N>& b) {
  Tan<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
// x -> f(x) with f' = df at the value
template <int N>
__device__ inline Tan<N> chain(const Tan<N>& a, double f, double df) {
  Tan<N> r;
  r.v = f;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = df * a.d[k];
  return r;
}
template <int N>
__device__ inline Tan<N> rcp(const Tan<N>& a) {
  const double y = 1.0 / a.v;
  return chain(a, y, -y * y);
}
template <int N>
__device__ inline Tan<N> operator/(const Tan<N>& a, const Tan<N>& b) {
  return a * rcp(b);
}
template <int N>
__device__ inline Tan<N> sqrt(const Tan<N>& a) {
  const double y = ::sqrt(a.v);
  return chain(a, y, 0.5 / y);
}
template <int N>
__device__ inline Tan<N> rsqrt(const Tan<N>& a) {
  const double y = 1.0 / ::sqrt(a.v);
  return chain(a, y, -0.5 * y / a.v);
}
template <int N>
__device__ inline Tan<N> exp(const Tan<N>& a) {
  const double y = ::exp(a.v);
  return chain(a, y, y);
}
template <int N>
__device__ inline void sincos(const Tan<N>& a, Tan<N>* s, Tan<N>* c) {
  double sv, cv;
  ::sincos(a.v, &sv, &cv);
  *s = chain(a, sv, cv);
  *c = chain(a, cv, -sv);
}

}  // namespace grpic
