// Kernels of the learned surrogate policy x0 -> u (a library extension that the
// interior-point method of Section 3 judges): the multilayer perceptron's forward and
// backward passes, its loss and AdamW update, and the FP64 judge of an answer
// (simulation of eqn. (dyn), bound violation, objective, and the lambda = 0 dual bound).
//
// Precision: weights and activations are stored as T = bfloat16 (training and inference)
// or float (the test mode); products accumulate in float32 on MFMA
// (v_mfma_f32_16x16x32_bf16 / v_mfma_f32_16x16x4f32); master weights, Adam moments,
// pre-activations and gradients of the weights are float32.  The rounding points are the
// ones the CPU oracle of the surrogate applies.
//
// Shapes: every matrix dimension is padded to a multiple of 64 (zero rows and columns that
// stay zero), so the GEMM tiles need no bounds tests.
#include "surrogate.hpp"

namespace cmpc {

template <typename T>
struct Cvt;
template <>
struct Cvt<float> {
  __device__ static inline float from(float x) { return x; }
  __device__ static inline float to(float x) { return x; }
};
template <>
struct Cvt<bf16_t> {
  __device__ static inline bf16_t from(float x) { return f2bf(x); }
  __device__ static inline float to(bf16_t x) { return bf2f(x); }
};

// gelu(x) = x Phi(x) (exact form) and its derivative Phi(x) + x phi(x), in float32
__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
         x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// 8 consecutive elements (16-byte aligned for bf16; two float4 for float)
__device__ inline void load8(const bf16_t* p, bf16_t (&v)[8]) {
  const uint4 q = *reinterpret_cast<const uint4*>(p);
  const unsigned int w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    v[2 * e] = (bf16_t)(w[e] & 0xFFFFu);
    v[2 * e + 1] = (bf16_t)(w[e] >> 16);
  }
}
__device__ inline void load8(const float* p, float (&v)[8]) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

template <typename T>
struct Mma;
template <>
struct Mma<bf16_t> {
  static constexpr int kPad = 8;  // LDS row of 40 bf16 (80 bytes, 16-byte aligned rows)
  // acc += A(16 x 32) B(16 x 32)' for one 32-deep slab; lane l supplies row l%16,
  // elements 8 (l/16) .. 8 (l/16) + 7 of both operands
  template <int W>
  __device__ static inline f4 slab(const bf16_t (*As)[W], const bf16_t (*Bs)[W], int ra, int rb,
                                   int li, int lk, f4 acc) {
    const s8 a = *reinterpret_cast<const s8*>(&As[ra + li][8 * lk]);
    const s8 b = *reinterpret_cast<const s8*>(&Bs[rb + li][8 * lk]);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
};
template <>
struct Mma<float> {
  static constexpr int kPad = 1;
  template <int W>
  __device__ static inline f4 slab(const float (*As)[W], const float (*Bs)[W], int ra, int rb,
                                   int li, int lk, f4 acc) {
#pragma unroll
    for (int s = 0; s < 8; ++s)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(As[ra + li][4 * s + lk], Bs[rb + li][4 * s + lk],
                                                 acc, 0, 0, 0);
    return acc;
  }
};

// C(i, j) = sum_r A(i, r) B(j, r) over r < K for one 64 x 64 tile of C; A(i, r) is
// A[i lda + r] when AK = 1 and A[r lda + i] when AK = 0 (same for B with BK, ldb).
// 4 wavefronts, each a 32 x 32 quadrant (2 x 2 MFMA blocks); 32-deep slabs staged in LDS
// (transposed on the way in when the operand is not r-contiguous), the next slab's global
// loads in flight behind the current slab's MFMAs.  The epilogue (EPI) is fused.
template <typename T, int AK, int BK, int EPI>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(const T* __restrict__ A, int lda,
                                                       const T* __restrict__ B, int ldb, int K,
                                                       MlpEpi e) {
  constexpr int W = 32 + Mma<T>::kPad;
  __shared__ __attribute__((aligned(16))) T As[64][W];
  __shared__ __attribute__((aligned(16))) T Bs[64][W];
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wi = wave >> 1, wj = wave & 1, li = lane & 15, lk = lane >> 4;
  // staging coordinates: r-contiguous -> (row t/4, 8 elements from 8 (t%4));
  //                      i-contiguous -> (slab row t/8, 8 elements from 8 (t%8))
  const int ra = AK ? (t >> 2) : (t >> 3), ca = AK ? 8 * (t & 3) : 8 * (t & 7);
  const int rb = BK ? (t >> 2) : (t >> 3), cb = BK ? 8 * (t & 3) : 8 * (t & 7);
  auto gptr_a = [&](int r0) {
    return AK ? A + (long long)(i0 + ra) * lda + r0 + ca : A + (long long)(r0 + ra) * lda + i0 + ca;
  };
  auto gptr_b = [&](int r0) {
    return BK ? B + (long long)(j0 + rb) * ldb + r0 + cb : B + (long long)(r0 + rb) * ldb + j0 + cb;
  };
  T va[8], vb[8];
  auto stage = [&]() {
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      if (AK) As[ra][ca + x] = va[x]; else As[ca + x][ra] = va[x];
      if (BK) Bs[rb][cb + x] = vb[x]; else Bs[cb + x][rb] = vb[x];
    }
  };
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  load8(gptr_a(0), va);
  load8(gptr_b(0), vb);
  stage();
  __syncthreads();
  for (int r0 = 0; r0 < K; r0 += 32) {
    const bool more = r0 + 32 < K;
    if (more) {
      load8(gptr_a(r0 + 32), va);
      load8(gptr_b(r0 + 32), vb);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = Mma<T>::template slab<W>(As, Bs, 32 * wi + 16 * a, 32 * wj + 16 * b, li, lk,
                                             acc[a][b]);
    __syncthreads();
    if (more) {
      stage();
      __syncthreads();
    }
  }
  // epilogue: element v of block (a, b) sits at row 4 (l/16) + v, column l%16
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 32 * wi + 16 * a + 4 * lk + v;
        const int j = j0 + 32 * wj + 16 * b + li;
        const float c = acc[a][b][v];
        if (EPI == kEpiGelu) {
          const float z = c + e.bias[j];
          e.z[(long long)i * e.ldz + j] = z;
          reinterpret_cast<T*>(e.h)[(long long)i * e.ldh + j] = Cvt<T>::from(gelu_f(z));
        } else if (EPI == kEpiLinear) {
          e.z[(long long)i * e.ldz + j] = c + e.bias[j];
        } else if (EPI == kEpiDGelu) {
          const float g = c * gelu_grad_f(e.zin[(long long)i * e.ldzi + j]);
          reinterpret_cast<T*>(e.h)[(long long)i * e.ldh + j] = Cvt<T>::from(g);
        } else {
          e.z[(long long)i * e.ldz + j] = c;
        }
      }
}

template <typename T, int AK, int BK, int EPI>
static int gemm_go(hipStream_t s, const T* A, int lda, const T* B, int ldb, int M, int N, int K,
                   const MlpEpi& e) {
  hipLaunchKernelGGL((mlp_gemm_kernel<T, AK, BK, EPI>), dim3(N / 64, M / 64), dim3(256), 0, s, A,
                     lda, B, ldb, K, e);
  CMPC_LAUNCH_CHECK();
  return 0;
}

template <typename T>
int launch_mlp_gemm(hipStream_t s, int kind, const T* A, int lda, const T* B, int ldb, int M,
                    int N, int K, const MlpEpi& e) {
  if (M % 64 || N % 64 || K % 32 || M <= 0 || N <= 0 || K <= 0) {
    set_error("MLP GEMM shapes must be multiples of 64 (K of 32)");
    return CMPC_ERR_INVALID;
  }
  switch (kind) {
    case kGemmFwdGelu: return gemm_go<T, 1, 1, kEpiGelu>(s, A, lda, B, ldb, M, N, K, e);
    case kGemmFwdLinear: return gemm_go<T, 1, 1, kEpiLinear>(s, A, lda, B, ldb, M, N, K, e);
    case kGemmBwdData: return gemm_go<T, 1, 0, kEpiDGelu>(s, A, lda, B, ldb, M, N, K, e);
    case kGemmBwdWeight: return gemm_go<T, 0, 0, kEpiF32>(s, A, lda, B, ldb, M, N, K, e);
    default: set_error("unknown MLP GEMM kind"); return CMPC_ERR_INVALID;
  }
}
template int launch_mlp_gemm<bf16_t>(hipStream_t, int, const bf16_t*, int, const bf16_t*, int, int,
                                     int, int, const MlpEpi&);
template int launch_mlp_gemm<float>(hipStream_t, int, const float*, int, const float*, int, int, int,
                                    int, const MlpEpi&);

// ---------------------------------------------------------------- elementwise kernels
// a0 (Mp x ldp) = T(x0 rows idx[r]) for r < rows, zero elsewhere (columns >= ns are zero).
template <typename T>
__global__ void stage_rows_kernel(const double* __restrict__ X, int ld_x, int ncols,
                                  const int* __restrict__ idx, int rows, T* __restrict__ out,
                                  int ldo, int Mp) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)Mp * ldo) return;
  const int r = (int)(e / ldo), c = (int)(e - (long long)r * ldo);
  float v = 0.f;
  if (r < rows && c < ncols) {
    const long long src = idx ? idx[r] : r;
    v = (float)X[src * ld_x + c];
  }
  out[e] = Cvt<T>::from(v);
}

template <typename T>
int launch_stage_rows(hipStream_t s, const double* X, int ld_x, int ncols, const int* idx,
                      int rows, T* out, int ldo, int Mp) {
  const long long len = (long long)Mp * ldo;
  hipLaunchKernelGGL(stage_rows_kernel<T>, dim3(ceil_div(len, 256)), dim3(256), 0, s, X, ld_x,
                     ncols, idx, rows, out, ldo, Mp);
  CMPC_LAUNCH_CHECK();
  return 0;
}
template int launch_stage_rows<bf16_t>(hipStream_t, const double*, int, int, const int*, int,
                                       bf16_t*, int, int);
template int launch_stage_rows<float>(hipStream_t, const double*, int, int, const int*, int, float*,
                                      int, int);

// g = T(2 (y - u) / (rows ncols)) on the valid block, 0 on the padding; per-block partial
// sums of (y - u)^2 (fixed order) for the loss.
template <typename T>
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* __restrict__ Y, int ldy,
                                                       const float* __restrict__ U, int ldu,
                                                       int rows, int ncols, T* __restrict__ G,
                                                       int ldg, int Mp,
                                                       double* __restrict__ part) {
  __shared__ double sh[4];
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  double sq = 0.0;
  if (e < (long long)Mp * ldg) {
    const int r = (int)(e / ldg), c = (int)(e - (long long)r * ldg);
    float g = 0.f;
    if (r < rows && c < ncols) {
      const float d = Y[(long long)r * ldy + c] - U[(long long)r * ldu + c];
      g = 2.0f * d / ((float)rows * (float)ncols);
      sq = (double)d * (double)d;
    }
    G[e] = Cvt<T>::from(g);
  }
  sq = block_sum256(sq, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = sq;
}

template <typename T>
int launch_mse_grad(hipStream_t s, const float* Y, int ldy, const float* U, int ldu, int rows,
                    int ncols, T* G, int ldg, int Mp, double* part, int* nparts) {
  const long long len = (long long)Mp * ldg;
  *nparts = ceil_div(len, 256);
  hipLaunchKernelGGL(mse_grad_kernel<T>, dim3(*nparts), dim3(256), 0, s, Y, ldy, U, ldu, rows,
                     ncols, G, ldg, Mp, part);
  CMPC_LAUNCH_CHECK();
  return 0;
}
template int launch_mse_grad<bf16_t>(hipStream_t, const float*, int, const float*, int, int, int,
                                     bf16_t*, int, int, double*, int*);
template int launch_mse_grad<float>(hipStream_t, const float*, int, const float*, int, int, int,
                                    float*, int, int, double*, int*);

// out[0] = sum of part[0..n) / denom (one workgroup, fixed order)
__global__ __launch_bounds__(256) void sum_parts_kernel(const double* __restrict__ part, int n,
                                                        double denom, double* __restrict__ out) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  acc = block_sum256(acc, sh);
  if (threadIdx.x == 0) *out = acc / denom;
}

int launch_sum_parts(hipStream_t s, const double* part, int n, double denom, double* out) {
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, s, part, n, denom, out);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// db[j] = sum over rows of G[i][j] (float), 64 columns x 4 row groups per workgroup
template <typename T>
__global__ __launch_bounds__(256) void colsum_kernel(const T* __restrict__ G, int ldg, int rows,
                                                     float* __restrict__ db) {
  __shared__ float sh[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  float acc = 0.f;
  for (int r = g; r < rows; r += 4) acc += Cvt<T>::to(G[(long long)r * ldg + c]);
  sh[g][threadIdx.x & 63] = acc;
  __syncthreads();
  if (g == 0) db[c] = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}

template <typename T>
int launch_colsum(hipStream_t s, const T* G, int ldg, int rows, int ncols, float* db) {
  hipLaunchKernelGGL(colsum_kernel<T>, dim3(ncols / 64), dim3(256), 0, s, G, ldg, rows, db);
  CMPC_LAUNCH_CHECK();
  return 0;
}
template int launch_colsum<bf16_t>(hipStream_t, const bf16_t*, int, int, int, float*);
template int launch_colsum<float>(hipStream_t, const float*, int, int, int, float*);

// AdamW on float32 master values, then the low-precision copy used by the GEMMs.
// c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t) (bias corrections of step t).
template <typename T>
__global__ void adamw_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                             const float* __restrict__ g, T* __restrict__ wlow, long long len,
                             float lr, float b1, float b2, float eps, float wd, float c1,
                             float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * ((mi * c1) / (sqrtf(vi * c2) + eps) + wd * w[i]);
  w[i] = wi;
  if (wlow) wlow[i] = Cvt<T>::from(wi);
}

template <typename T>
int launch_adamw(hipStream_t s, float* w, float* m, float* v, const float* g, T* wlow,
                 long long len, float lr, float b1, float b2, float eps, float wd, float c1,
                 float c2) {
  hipLaunchKernelGGL(adamw_kernel<T>, dim3(ceil_div(len, 256)), dim3(256), 0, s, w, m, v, g, wlow,
                     len, lr, b1, b2, eps, wd, c1, c2);
  CMPC_LAUNCH_CHECK();
  return 0;
}
template int launch_adamw<bf16_t>(hipStream_t, float*, float*, float*, const float*, bf16_t*,
                                  long long, float, float, float, float, float, float, float);
template int launch_adamw<float>(hipStream_t, float*, float*, float*, const float*, float*,
                                 long long, float, float, float, float, float, float, float);

// low-precision copy of a float32 array
template <typename T>
__global__ void to_low_kernel(const float* __restrict__ in, T* __restrict__ out, long long len) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) out[i] = Cvt<T>::from(in[i]);
}
template <typename T>
int launch_to_low(hipStream_t s, const float* in, T* out, long long len) {
  hipLaunchKernelGGL(to_low_kernel<T>, dim3(ceil_div(len, 256)), dim3(256), 0, s, in, out, len);
  CMPC_LAUNCH_CHECK();
  return 0;
}
template int launch_to_low<bf16_t>(hipStream_t, const float*, bf16_t*, long long);
template int launch_to_low<float>(hipStream_t, const float*, float*, long long);

// u[r][c] = clip(y[r][c], ul[c % nu], uu[c % nu]) in float64, r < rows, c < n
__global__ void clip_out_kernel(const float* __restrict__ Y, int ldy, int rows, int n, int nu,
                                const double* __restrict__ ul, const double* __restrict__ uu,
                                double* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)rows * n) return;
  const int r = (int)(e / n), c = (int)(e - (long long)r * n);
  const int k = c % nu;
  out[e] = fmin(fmax((double)Y[(long long)r * ldy + c], ul[k]), uu[k]);
}

int launch_clip_out(hipStream_t s, const float* Y, int ldy, int rows, int n, int nu,
                    const double* ul, const double* uu, double* out) {
  const long long len = (long long)rows * n;
  if (len == 0) return 0;
  hipLaunchKernelGGL(clip_out_kernel, dim3(ceil_div(len, 256)), dim3(256), 0, s, Y, ldy, rows, n,
                     nu, ul, uu, out);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// ---------------------------------------------------------------- FP64 judge
// One workgroup per query: simulate x_{t+1} = A x_t + B u_t (eqn. (dyn)) with A in CSR
// (or dense when arp == NULL), accumulate the objective of eqn. (sparse) with diagonal
// weights q (Q) and qf (Q_f) and dense R, and the largest bound violation of the states
// x_1..x_N (infinite bounds ignored; the controls are clipped, so they are inside).
__global__ __launch_bounds__(256) void judge_sim_kernel(
    const double* __restrict__ X0, const double* __restrict__ Uq, int ns, int nu, int N,
    const int* __restrict__ arp, const int* __restrict__ acol, const double* __restrict__ aval,
    const double* __restrict__ Adense, const double* __restrict__ B, const double* __restrict__ q,
    const double* __restrict__ qf, const double* __restrict__ R, const double* __restrict__ xl,
    const double* __restrict__ xu, double* __restrict__ fout, double* __restrict__ vout) {
  extern __shared__ double xs[];  // 2 ns (ping-pong) + nu
  __shared__ double sh[4];
  const int qi = blockIdx.x;
  const int n = nu * N;
  double* xa = xs;
  double* xb = xs + ns;
  double* ut = xs + 2 * ns;
  const double* x0 = X0 + (long long)qi * ns;
  const double* u = Uq + (long long)qi * n;
  double f = 0.0, vio = 0.0;
  for (int i = threadIdx.x; i < ns; i += 256) {
    xa[i] = x0[i];
    f += 0.5 * q[i] * x0[i] * x0[i];
  }
  for (int t = 0; t < N; ++t) {
    __syncthreads();
    if (threadIdx.x < nu) ut[threadIdx.x] = u[t * nu + threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
      double ru = 0.0;
      for (int a = 0; a < nu; ++a) {
        double ra = 0.0;
        for (int b = 0; b < nu; ++b) ra += R[a * nu + b] * ut[b];
        ru += ut[a] * ra;
      }
      f += 0.5 * ru;
    }
    const double* w = (t == N - 1) ? qf : q;
    for (int i = threadIdx.x; i < ns; i += 256) {
      double acc = 0.0;
      if (arp) {
        for (int k = arp[i]; k < arp[i + 1]; ++k) acc += aval[k] * xa[acol[k]];
      } else {
        for (int k = 0; k < ns; ++k) acc += Adense[(long long)i * ns + k] * xa[k];
      }
      for (int c = 0; c < nu; ++c) acc += B[(long long)i * nu + c] * ut[c];
      xb[i] = acc;
      f += 0.5 * w[i] * acc * acc;
      if (!isinf(xu[i])) vio = fmax(vio, acc - xu[i]);
      if (!isinf(xl[i])) vio = fmax(vio, xl[i] - acc);
    }
    double* tmp = xa;
    xa = xb;
    xb = tmp;
  }
  f = block_sum256(f, sh);
  vio = block_max256(vio, sh);
  if (threadIdx.x == 0) {
    fout[qi] = f;
    vout[qi] = vio;
  }
}

int launch_judge_sim(hipStream_t s, const double* X0, const double* U, int count, int ns, int nu,
                     int N, const int* arp, const int* acol, const double* aval,
                     const double* Adense, const double* B, const double* q, const double* qf,
                     const double* R, const double* xl, const double* xu, double* f,
                     double* vio) {
  if (count <= 0) return 0;
  const size_t lds = sizeof(double) * (2 * (size_t)ns + nu);
  hipLaunchKernelGGL(judge_sim_kernel, dim3(count), dim3(256), lds, s, X0, U, ns, nu, N, arp, acol,
                     aval, Adense, B, q, qf, R, xl, xu, f, vio);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// lb[q] = 1/2 x0_q' P x0_q for 4 queries per workgroup (P symmetric ns x ns, read once per
// 4 queries); P is the unconstrained cost-to-go of the Riccati recursion, so this is the
// minimum of the unconstrained QP, h0 - 1/2 h' H^-1 h.
__global__ __launch_bounds__(256) void judge_lb_kernel(const double* __restrict__ X0, int count,
                                                       int ns, const double* __restrict__ P,
                                                       double* __restrict__ lb) {
  __shared__ double sh[4];
  const int q0 = blockIdx.x * 4;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < ns; i += 256) {
    double pi[4] = {0.0, 0.0, 0.0, 0.0};
    const double* row = P + (long long)i * ns;
    for (int k = 0; k < ns; ++k) {
      const double pk = row[k];
#pragma unroll
      for (int g = 0; g < 4; ++g)
        if (q0 + g < count) pi[g] = fma(pk, X0[(long long)(q0 + g) * ns + k], pi[g]);
    }
#pragma unroll
    for (int g = 0; g < 4; ++g)
      if (q0 + g < count) acc[g] += X0[(long long)(q0 + g) * ns + i] * pi[g];
  }
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const double v = block_sum256(acc[g], sh);
    if (threadIdx.x == 0 && q0 + g < count) lb[q0 + g] = 0.5 * v;
  }
}

int launch_judge_lb(hipStream_t s, const double* X0, int count, int ns, const double* P,
                    double* lb) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(judge_lb_kernel, dim3(ceil_div(count, 4)), dim3(256), 0, s, X0, count, ns, P,
                     lb);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// accept[q] = violation <= vtol and (f - LB) / |LB| <= gtol; gap[q] = (f - LB) / |LB|
__global__ void judge_decide_kernel(const double* __restrict__ f, const double* __restrict__ vio,
                                    const double* __restrict__ lb, int count, double vtol,
                                    double gtol, int* __restrict__ accept,
                                    double* __restrict__ gap) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const double l = lb[q];
  const double g = l != 0.0 ? (f[q] - l) / fabs(l) : (f[q] == l ? 0.0 : INFINITY);
  gap[q] = g;
  accept[q] = (vio[q] <= vtol && g <= gtol) ? 1 : 0;
}

int launch_judge_decide(hipStream_t s, const double* f, const double* vio, const double* lb,
                        int count, double vtol, double gtol, int* accept, double* gap) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(judge_decide_kernel, dim3(ceil_div(count, 256)), dim3(256), 0, s, f, vio, lb,
                     count, vtol, gtol, accept, gap);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// ---------------------------------------------------------------- Riccati helpers
// K = S^-1 T for the small SPD S (nu x nu, nu <= 64) and T (nu x ns): one workgroup factors S
// in LDS (Cholesky, column by column) and then solves for the ns columns of T.
__global__ __launch_bounds__(256) void small_spd_solve_kernel(const double* __restrict__ S, int nu,
                                                              const double* __restrict__ T, int ns,
                                                              double* __restrict__ K,
                                                              int* __restrict__ fail) {
  __shared__ double L[64][65];
  for (int e = threadIdx.x; e < nu * nu; e += 256) L[e / nu][e % nu] = S[e];
  __syncthreads();
  for (int j = 0; j < nu; ++j) {
    if (threadIdx.x == 0) {
      double d = L[j][j];
      for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
      if (!(d > 0.0)) *fail = 1;
      L[j][j] = sqrt(fmax(d, 1e-300));
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < nu; i += 256) {
      double v = L[i][j];
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / L[j][j];
    }
    __syncthreads();
  }
  for (int c = threadIdx.x; c < ns; c += 256) {
    double y[64];
    for (int i = 0; i < nu; ++i) {
      double v = T[(long long)i * ns + c];
      for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
      y[i] = v / L[i][i];
    }
    for (int i = nu - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < nu; ++k) v -= L[k][i] * y[k];
      y[i] = v / L[i][i];
    }
    for (int i = 0; i < nu; ++i) K[(long long)i * ns + c] = y[i];
  }
}

int launch_small_spd_solve(hipStream_t s, const double* S, int nu, const double* T, int ns,
                           double* K, int* fail) {
  if (nu > 64) {
    set_error("surrogate judge: nu > 64 is not supported");
    return CMPC_ERR_INVALID;
  }
  hipLaunchKernelGGL(small_spd_solve_kernel, dim3(1), dim3(256), 0, s, S, nu, T, ns, K, fail);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// P = 1/2 (P + P') in place (removes the rounding asymmetry of the recursion)
__global__ void symmetrize_kernel(double* __restrict__ P, int n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * n) return;
  const int i = (int)(e / n), j = (int)(e - (long long)i * n);
  if (j >= i) return;
  const double v = 0.5 * (P[(long long)i * n + j] + P[(long long)j * n + i]);
  P[(long long)i * n + j] = v;
  P[(long long)j * n + i] = v;
}

int launch_symmetrize(hipStream_t s, double* P, int n) {
  const long long len = (long long)n * n;
  hipLaunchKernelGGL(symmetrize_kernel, dim3(ceil_div(len, 256)), dim3(256), 0, s, P, n);
  CMPC_LAUNCH_CHECK();
  return 0;
}

}  // namespace cmpc
