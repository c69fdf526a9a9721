// Scalar helpers shared by the device code: real (double) and complex
// (double2, interleaved) elements through one interface.
#pragma once
#include "common.hpp"

namespace chase {

// ------------------------------------------------------- scalar helpers --
template <typename E> struct Num;
template <> struct Num<double> {
  __device__ static double zero() { return 0.0; }
  __device__ static double mul(double a, double b) { return a * b; }
  __device__ static double cj(double a) { return a; }
  __device__ static double abs2(double a) { return a * a; }
  __device__ static double re(double a) { return a; }
  __device__ static double im(double) { return 0.0; }
  __device__ static double real(double r) { return r; }
  __device__ static double scale(double a, double s) { return a * s; }
  // a + (the value of lane ^ m)
  __device__ static double add_xor(double a, int m) { return a + __shfl_xor(a, m); }
  __device__ static double sel(bool p, double a, double b) { return p ? a : b; }
};
template <> struct Num<double2> {
  __device__ static double2 zero() { return make_double2(0.0, 0.0); }
  __device__ static double2 mul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
  }
  __device__ static double2 cj(double2 a) { return make_double2(a.x, -a.y); }
  __device__ static double abs2(double2 a) { return a.x * a.x + a.y * a.y; }
  __device__ static double re(double2 a) { return a.x; }
  __device__ static double im(double2 a) { return a.y; }
  __device__ static double2 real(double r) { return make_double2(r, 0.0); }
  __device__ static double2 scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
  __device__ static double2 add_xor(double2 a, int m) {
    return make_double2(a.x + __shfl_xor(a.x, m), a.y + __shfl_xor(a.y, m));
  }
  // p ? a : b by components (a select of the vector struct goes through memory)
  __device__ static double2 sel(bool p, double2 a, double2 b) {
    return make_double2(p ? a.x : b.x, p ? a.y : b.y);
  }
};
// 1 / sqrt(d) for a positive normal d: the hardware estimate (about 2^-24
// relative) refined by two Newton steps, y <- y + y (1 - d y^2) / 2, to
// about an ulp (1.24 ulp at most measured over 1e-300 .. 1e300): seven
// dependent operations where the correctly rounded square root and the
// division after it take about twenty
__device__ __forceinline__ double rsqrt_refined(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double r = __builtin_fma(-d * y, y, 1.0);
    y = __builtin_fma(0.5 * y, r, y);
  }
  return y;
}

__device__ __forceinline__ double2 operator+(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 operator-(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 operator-(double2 a) { return make_double2(-a.x, -a.y); }

}  // namespace chase
