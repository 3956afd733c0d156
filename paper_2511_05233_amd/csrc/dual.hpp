// Forward-mode dual numbers for device code.
//
// A Dual<S> carries a value and one directional derivative.  Evaluating the
// residual body on duals seeded with (u, v) returns (R(u), J(u) v): the exact
// tangent-linear operator of the same arithmetic, with zero derivative
// wherever a clamp or a guard selects a constant branch (comparisons look at
// values only).
#pragma once

#include <hip/hip_runtime.h>

namespace lsbdg {

// Arithmetic kernels of the dual numbers.  Double: IEEE operations and the
// device library.  Float (the tangent inside the FP32 Krylov solve, whose
// root is set by the FP64 residual): hardware reciprocal, exp2 and log2
// (about 1 ulp; a few instructions instead of the exact-division and
// library sequences).
__device__ __forceinline__ double dual_div(double a, double b) { return a / b; }
__device__ __forceinline__ double dual_exp(double a) { return ::exp(a); }
__device__ __forceinline__ double dual_log(double a) { return ::log(a); }
__device__ __forceinline__ float dual_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float dual_exp(float a) { return __expf(a); }
__device__ __forceinline__ float dual_log(float a) { return __logf(a); }

template <typename S>
struct Dual {
  S v, d;
  __host__ __device__ Dual() = default;
  __host__ __device__ constexpr Dual(double x) : v(S(x)), d(S(0)) {}
  __host__ __device__ constexpr Dual(S x, S dx) : v(x), d(dx) {}

  friend __device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
  friend __device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
  friend __device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
  friend __device__ __forceinline__ Dual operator*(Dual a, Dual b) {
    return {a.v * b.v, a.v * b.d + a.d * b.v};
  }
  friend __device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    const S q = dual_div(a.v, b.v);
    return {q, dual_div(a.d - q * b.d, b.v)};
  }
  __device__ __forceinline__ Dual& operator+=(Dual b) { v += b.v; d += b.d; return *this; }
  __device__ __forceinline__ Dual& operator-=(Dual b) { v -= b.v; d -= b.d; return *this; }
  __device__ __forceinline__ Dual& operator*=(Dual b) { *this = *this * b; return *this; }
  friend __device__ __forceinline__ bool operator>(Dual a, Dual b) { return a.v > b.v; }
  friend __device__ __forceinline__ bool operator<(Dual a, Dual b) { return a.v < b.v; }
  friend __device__ __forceinline__ Dual exp(Dual a) {
    const S e = dual_exp(a.v);
    return {e, e * a.d};
  }
  friend __device__ __forceinline__ Dual log(Dual a) { return {dual_log(a.v), dual_div(a.d, a.v)}; }
  friend __device__ __forceinline__ Dual sqrt(Dual a) {
    const S s = ::sqrt(a.v);
    return {s, a.d * S(0.5) / s};
  }
};

// value / derivative accessors that also work on plain scalars
template <typename S>
__device__ __forceinline__ S value_of(S x) { return x; }
template <typename S>
__device__ __forceinline__ S value_of(Dual<S> x) { return x.v; }
template <typename S>
__device__ __forceinline__ S deriv_of(Dual<S> x) { return x.d; }

}  // namespace lsbdg
