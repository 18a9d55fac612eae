// Dual numbers v + d eps (eps^2 = 0) for forward-mode derivatives of the
// pointwise terms of the element kernels, and the reciprocal / reciprocal
// square root used there (hardware estimates refined by Newton steps).
#pragma once

#include "pf_element.h"

namespace pf {

// 1/sqrt(x), x > 0: hardware estimate refined by two Newton steps
__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x * r, r, 1.5);
  return r * fma(-0.5 * x * r, r, 1.5);
}

// Dual number v + d eps (eps^2 = 0) for forward-mode derivatives.
struct Dual {
  double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, fma(a.d, b.v, a.v * b.d)}; }
__device__ __forceinline__ Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
__device__ __forceinline__ Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }

__device__ __forceinline__ double rcp_t(double x) { return rcp_nr(x); }
__device__ __forceinline__ Dual rcp_t(Dual x) {
  const double r = rcp_nr(x.v);
  return {r, -x.d * r * r};
}
__device__ __forceinline__ double rsqrt_t(double x) { return rsqrt_nr(x); }
__device__ __forceinline__ Dual rsqrt_t(Dual x) {
  const double r = rsqrt_nr(x.v);
  return {r, -0.5 * x.d * r * r * r};
}
__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ double val(Dual x) { return x.v; }

}  // namespace pf
