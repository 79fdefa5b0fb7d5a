// Forward-mode dual numbers (value + one directional derivative) used by
// the adjoint kernels to differentiate the equilibrium moments and the
// energy-flux modification through the very code the step uses.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

struct Dual {
  double v, d;
  __host__ __device__ Dual() : v(0.0), d(0.0) {}
  __host__ __device__ Dual(double x) : v(x), d(0.0) {}
  __host__ __device__ Dual(double x, double dx) : v(x), d(dx) {}
};

__host__ __device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__host__ __device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__host__ __device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__host__ __device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__host__ __device__ __forceinline__ Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
__host__ __device__ __forceinline__ Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
__host__ __device__ __forceinline__ Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
__host__ __device__ __forceinline__ Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
__host__ __device__ __forceinline__ Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
__host__ __device__ __forceinline__ Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
__host__ __device__ __forceinline__ Dual operator/(double a, Dual b) {
  const double r = 1.0 / b.v;
  return Dual(a * r, -a * b.d * r * r);
}
__host__ __device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const double r = 1.0 / b.v;
  const double q = a.v * r;
  return Dual(q, (a.d - q * b.d) * r);
}
__host__ __device__ __forceinline__ Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
__host__ __device__ __forceinline__ Dual& operator+=(Dual& a, Dual b) {
  a = a + b;
  return a;
}
__host__ __device__ __forceinline__ Dual sexp(Dual a) {
  const double e = ::exp(a.v);
  return Dual(e, e * a.d);
}

}  // namespace lbm
