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

// x from another lane by the DPP control CTRL (quad_perm, row rotation; no LDS round trip).
template <int CTRL>
__device__ inline double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// x of lane `lane` (a constant or wavefront-uniform index) in every lane.
__device__ inline double readlane_f64(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ---- wavefront reductions (all 64 lanes active; fixed order: deterministic) ----
// Within each 16-lane row by DPP (lane ^ 1, lane ^ 2, rotations by 4 and 8: every lane of
// the row ends with the row's value), then the four rows through scalar reads.
template <typename Op>
__device__ inline double wave_reduce(double x, Op op) {
  x = op(x, dpp_f64<0xB1>(x));
  x = op(x, dpp_f64<0x4E>(x));
  x = op(x, dpp_f64<0x124>(x));
  x = op(x, dpp_f64<0x128>(x));
  return op(op(readlane_f64(x, 0), readlane_f64(x, 16)),
            op(readlane_f64(x, 32), readlane_f64(x, 48)));
}
__device__ inline double wave_sum(double x) {
  return wave_reduce(x, [](double a, double b) { return a + b; });
}
__device__ inline double wave_max(double x) {
  return wave_reduce(x, [](double a, double b) { return fmax(a, b); });
}
__device__ inline double wave_min(double x) {
  return wave_reduce(x, [](double a, double b) { return fmin(a, b); });
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

// K workgroup reductions (blockDim.x == 256) through one exchange of the wavefronts' results;
// op[k]: 0 = sum, 1 = max, 2 = min.  Each value is reduced and combined exactly as by
// block_sum256 / block_max256 / block_min256, so the results are the same bits.
enum : int { kRedSum = 0, kRedMax = 1, kRedMin = 2 };
template <int K>
__device__ inline void block_multi256(double (&x)[K], const int (&op)[K], double (*sh)[4]) {
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double r = op[k] == kRedSum ? wave_sum(x[k])
                                      : (op[k] == kRedMax ? wave_max(x[k]) : wave_min(x[k]));
    if ((threadIdx.x & 63) == 0) sh[k][w] = r;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double* q = sh[k];
    x[k] = op[k] == kRedSum ? (q[0] + q[1]) + (q[2] + q[3])
                            : (op[k] == kRedMax ? fmax(fmax(q[0], q[1]), fmax(q[2], q[3]))
                                                : fmin(fmin(q[0], q[1]), fmin(q[2], q[3])));
  }
  __syncthreads();
}

}  // namespace cmpc
