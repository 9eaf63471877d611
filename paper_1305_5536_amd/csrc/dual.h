// Forward-mode dual numbers for the discrete adjoints: the Jacobian-vector
// products of the face and volume fluxes and of the limiter, one direction at
// a time, through the same templated device code the forward kernels run.
#pragma once

#include <hip/hip_runtime.h>

#include "dg_math.h"

namespace dg {

// Forward-mode dual number: value and one tangent.  The arithmetic the HLLD
// solver and the limiter use is defined as hidden friends, so it is found by
// argument-dependent lookup only and hides nothing of the plain overloads.
template <typename T>
struct Dual {
  T v, d;
  __device__ __forceinline__ Dual() : v(T(0)), d(T(0)) {}
  __device__ __forceinline__ Dual(double a) : v(T(a)), d(T(0)) {}
  __device__ __forceinline__ Dual(T a, T b) : v(a), d(b) {}

  friend __device__ __forceinline__ Dual operator+(Dual a, Dual b) {
    return Dual(a.v + b.v, a.d + b.d);
  }
  friend __device__ __forceinline__ Dual operator-(Dual a, Dual b) {
    return Dual(a.v - b.v, a.d - b.d);
  }
  friend __device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
  friend __device__ __forceinline__ Dual operator*(Dual a, Dual b) {
    return Dual(a.v * b.v, a.d * b.v + a.v * b.d);
  }
  friend __device__ __forceinline__ bool operator<(Dual a, Dual b) { return a.v < b.v; }
  friend __device__ __forceinline__ bool operator>(Dual a, Dual b) { return a.v > b.v; }
  friend __device__ __forceinline__ bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
  friend __device__ __forceinline__ bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
  friend __device__ __forceinline__ Dual fma(Dual a, Dual b, Dual c) {
    return Dual(fma(a.v, b.v, c.v), a.d * b.v + a.v * b.d + c.d);
  }
  // min / max return the first argument on ties
  friend __device__ __forceinline__ Dual fmin(Dual a, Dual b) { return b.v < a.v ? b : a; }
  friend __device__ __forceinline__ Dual fmax(Dual a, Dual b) { return b.v > a.v ? b : a; }
  friend __device__ __forceinline__ Dual fabs(Dual a) { return a.v < T(0) ? -a : a; }
  friend __device__ __forceinline__ Dual rcp(Dual a) {
    const T r = rcp(a.v);
    return Dual(r, -a.d * r * r);
  }
  friend __device__ __forceinline__ Dual sqrt_pos(Dual a) {
    const T s = sqrt_pos(a.v);
    return Dual(s, a.d * T(0.5) * rcp(s));
  }
  friend __device__ __forceinline__ Dual div_small(Dual a, Dual b) {
    const T q = div_small(a.v, b.v);
    return Dual(q, div_small(a.d - q * b.d, b.v));
  }
};

}  // namespace dg
