// Shared device helpers and launch utilities for the condensed-space IPM library (gfx950).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>

namespace cmpc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;

typedef unsigned short bf16_t;  // bfloat16 bit pattern

__device__ inline bf16_t f2bf(float x) {  // round to nearest, ties to even
  unsigned int b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (bf16_t)(b >> 16);
}
__device__ inline float bf2f(bf16_t h) { return __uint_as_float(((unsigned int)h) << 16); }

// Thread-local message of the last error (set by the C ABI layer).
void set_error(const std::string& msg);

#define CMPC_HIP(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::cmpc::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));         \
      return CMPC_ERR_HIP;                                                          \
    }                                                                               \
  } while (0)

#define CMPC_LAUNCH_CHECK()                                                         \
  do {                                                                              \
    hipError_t e_ = hipGetLastError();                                              \
    if (e_ != hipSuccess) {                                                         \
      ::cmpc::set_error(std::string("kernel launch: ") + hipGetErrorString(e_));    \
      return CMPC_ERR_HIP;                                                          \
    }                                                                               \
  } while (0)

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// ---- wavefront reductions (64 lanes, fixed butterfly order: deterministic) ----
__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}
__device__ inline double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, kWave));
  return x;
}
__device__ inline double wave_min(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, kWave));
  return x;
}

// Block reductions for blockDim.x == 256 (4 waves); result valid in every thread.
__device__ inline double block_sum256(double x, double* sh /* >= 4 */) {
  x = wave_sum(x);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = x;
  __syncthreads();
  double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}
__device__ inline double block_max256(double x, double* sh) {
  x = wave_max(x);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = x;
  __syncthreads();
  double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  __syncthreads();
  return r;
}
__device__ inline double block_min256(double x, double* sh) {
  x = wave_min(x);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = x;
  __syncthreads();
  double r = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
  __syncthreads();
  return r;
}

}  // namespace cmpc
