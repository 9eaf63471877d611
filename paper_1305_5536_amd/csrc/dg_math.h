// Device arithmetic helpers shared by the stage kernels (gfx950).
//
// Reciprocal and square root.  The kernels need 1/rho, 1/(S_R - S_L), the
// limiter ratio and sound speeds at every quadrature point; IEEE-exact FP64
// division and sqrt expand to long scaled sequences.  Inputs here are positive
// and far from the denormal range (rho, p > 0 are checked separately), so the
// hardware estimates refined by Newton-Raphson (reciprocal) and Goldschmidt
// (square root) iterations give results within an ulp or two, which the parity
// tolerances absorb.
#pragma once

#include <hip/hip_runtime.h>

namespace dg {

__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ float rcp(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  float e = fmaf(-x, r, 1.0f);
  return fmaf(r, e, r);
}

// sqrt(x) for x > 0: Goldschmidt iterations on g ~ sqrt(x), h ~ 1/(2 sqrt(x))
// seeded by the hardware reciprocal square root, then one residual correction.
__device__ __forceinline__ double sqrt_pos(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  return fma(d, h, g);
}

__device__ __forceinline__ float sqrt_pos(float x) {
  float y = __builtin_amdgcn_rsqf(x);
  float g = x * y, h = 0.5f * y;
  float d = fmaf(-g, g, x);
  return fmaf(d, h, g);
}

// a / b for b > 0 that may be tiny, down to the denormal range (the limiter's
// D / dm of a nearly flat cell): the reciprocal of such a b overflows, so both
// operands are first scaled by a power of two (exactly).  For b above the
// threshold this is a * rcp(b).
__device__ __forceinline__ double div_small(double a, double b) {
  const double s = b < 0x1p-900 ? 0x1p+1000 : 1.0;
  return (a * s) * rcp(b * s);
}
__device__ __forceinline__ float div_small(float a, float b) {
  const float s = b < 0x1p-100f ? 0x1p+100f : 1.0f;
  return (a * s) * rcp(b * s);
}

// sqrt of a value that may be exactly zero.
template <typename T>
__device__ __forceinline__ T sqrt_nn(T x) {
  return x > T(0) ? sqrt_pos(x) : T(0);
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip; remap the
// block index so each XCD receives a contiguous range of tiles (neighbouring
// tiles, and the halo rows they share, then hit the same L2).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  int per = nb >> 3;
  if (b < (per << 3)) return (b & 7) * per + (b >> 3);
  return b;
}

// Neighbour-lane exchange along the whole wave with DPP (wave_shr:1 and
// wave_shl:1), a VALU move with no LDS round trip: lane_up(v) gives lane l the
// value of lane l-1, lane_down(v) that of lane l+1; the end lane (0, resp. 63)
// keeps its own value.  Doubles move as two 32-bit halves.
__device__ __forceinline__ int dpp_shr1(int v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_shl1(int v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ float lane_up(float v) {
  return __int_as_float(dpp_shr1(__float_as_int(v)));
}
__device__ __forceinline__ float lane_down(float v) {
  return __int_as_float(dpp_shl1(__float_as_int(v)));
}
__device__ __forceinline__ double lane_up(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_shr1((int)(b & 0xffffffffLL)), hi = dpp_shr1((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_down(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_shl1((int)(b & 0xffffffffLL)), hi = dpp_shl1((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave-wide minimum of a double (lanes exchange through DPP/permute).
__device__ __forceinline__ double wave_min(double d) {
  for (int o = 32; o > 0; o >>= 1) d = fmin(d, __shfl_xor(d, o));
  return d;
}

}  // namespace dg
