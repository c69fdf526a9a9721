// Shared host/device definitions of the gfx950 library (types, error
// handling, small helpers).  Nothing here depends on PyTorch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

namespace chase {

// Storage element of a matrix: real T, or an interleaved complex pair.
template <typename T, bool CPLX> struct Elem { typedef T type; };
template <> struct Elem<double, true> { typedef double2 type; };
template <> struct Elem<float, true> { typedef float2 type; };

__device__ __forceinline__ double re_of(double v) { return v; }
__device__ __forceinline__ float re_of(float v) { return v; }
__device__ __forceinline__ double re_of(double2 v) { return v.x; }
__device__ __forceinline__ float re_of(float2 v) { return v.x; }
__device__ __forceinline__ double im_of(double) { return 0.0; }
__device__ __forceinline__ float im_of(float) { return 0.0f; }
__device__ __forceinline__ double im_of(double2 v) { return v.y; }
__device__ __forceinline__ float im_of(float2 v) { return v.y; }

template <typename E> __device__ __forceinline__ E make_elem(double r, double i);
template <> __device__ __forceinline__ double make_elem<double>(double r, double) { return r; }
template <> __device__ __forceinline__ float make_elem<float>(double r, double) { return (float)r; }
template <> __device__ __forceinline__ double2 make_elem<double2>(double r, double i) { return make_double2(r, i); }
template <> __device__ __forceinline__ float2 make_elem<float2>(double r, double i) { return make_float2((float)r, (float)i); }

// Thread-local last error message (exposed through chase_last_error()).
void set_error(const std::string &msg);
const char *get_error();

}  // namespace chase

#define CHASE_HIP(call)                                                        \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::chase::set_error(std::string(#call) + ": " + hipGetErrorString(e_));  \
      throw ::chase::DeviceError();                                            \
    }                                                                          \
  } while (0)

namespace chase {
struct DeviceError {};
struct InvalidArg {};
struct OutOfMemory {};
}  // namespace chase
