// Setup kernels: the state elimination of Section 2 (eqn. (x_def)) and the x0-dependent
// data of eqn. (dense).  They run once per problem or once per initial state, not per
// interior-point iteration.
#include <algorithm>

#include "problem.hpp"

namespace cmpc {

// C (M x Nc, leading dimension ldc) = alpha * op(A) op(B) + beta * C with strided operands:
// op(A)(i, k) = A[i * a_i + k * a_k], op(B)(k, j) = B[k * b_k + j * b_j].  16 x 16 output
// tiles, 16-deep slabs staged in LDS.  Setup only (G_k = A G_{k-1}, general-Q Hessian).
__global__ __launch_bounds__(256) void gemm_f64_kernel(int M, int Nc, int Kd, double alpha,
                                                       const double* __restrict__ A, long long a_i,
                                                       long long a_k, const double* __restrict__ B,
                                                       long long b_k, long long b_j, double beta,
                                                       double* __restrict__ C, long long ldc) {
  __shared__ double As[16][17];
  __shared__ double Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < Kd; k0 += 16) {
    const int ia = blockIdx.y * 16 + ty, ka = k0 + tx;
    As[ty][tx] = (ia < M && ka < Kd) ? A[ia * a_i + ka * a_k] : 0.0;
    const int kb = k0 + ty, jb = blockIdx.x * 16 + tx;
    Bs[ty][tx] = (kb < Kd && jb < Nc) ? B[kb * b_k + jb * b_j] : 0.0;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) acc = fma(As[ty][kk], Bs[kk][tx], acc);
    __syncthreads();
  }
  if (i < M && j < Nc) {
    double* cp = C + i * ldc + j;
    *cp = alpha * acc + (beta == 0.0 ? 0.0 : beta * *cp);
  }
}

int launch_gemm_f64(hipStream_t s, int M, int Nc, int Kd, double alpha, const double* A,
                    long long a_i, long long a_k, const double* B, long long b_k, long long b_j,
                    double beta, double* C, long long ldc) {
  if (M <= 0 || Nc <= 0) return 0;
  dim3 grid(ceil_div(Nc, 16), ceil_div(M, 16));
  hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, s, M, Nc, Kd, alpha, A, a_i, a_k, B,
                     b_k, b_j, beta, C, ldc);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// Row block t (1..N) of Gamma: rows (t-1) ns + i, columns a = j nu + k < t nu, entry
// G_{t-1-j}[i][k] = (A^(t-1-j) B)[i][k] (eqn. (x_def) with K = 0), written ns x (t nu)
// row-major.  Setup only: the general-Q Hessian takes one block at a time.
__global__ void gamma_block_kernel(const double* __restrict__ G, double* __restrict__ out,
                                   int t, int ns, int nu) {
  const long long len = (long long)t * nu;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)ns * len) return;
  const int i = (int)(e / len);
  const int a = (int)(e - (long long)i * len);
  const int j = a / nu, k = a - j * nu;
  out[e] = G[((long long)(t - 1 - j) * ns + i) * nu + k];
}

int launch_gamma_block(Problem& p, int t, double* out) {
  hipLaunchKernelGGL(gamma_block_kernel, dim3(ceil_div((long long)p.ns * t * p.nu, 256)),
                     dim3(256), 0, p.stream, p.G, out, t, p.ns, p.nu);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// Gt[(m nu + k) ns + i] = G[(m ns + i) nu + k]: the blocks of Gamma with the state index
// fastest, so that the Gamma products read them in coalesced rows.
__global__ void transpose_g_kernel(const double* __restrict__ G, double* __restrict__ Gt, int ns,
                                   int nu) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // index into Gt
  const int m = blockIdx.y;
  if (e >= (long long)ns * nu) return;
  const int k = (int)(e / ns), i = (int)(e - (long long)k * ns);
  Gt[(long long)m * ns * nu + e] = G[((long long)m * ns + i) * nu + k];
}

int launch_transpose_g(Problem& p) {
  dim3 grid(ceil_div((long long)p.ns * p.nu, 256), p.N);
  hipLaunchKernelGGL(transpose_g_kernel, grid, dim3(256), 0, p.stream, p.G, p.Gt, p.ns, p.nu);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// y = A x (A rows x cols, row-major): one wavefront per row, lanes stride the row.
__global__ __launch_bounds__(256) void gemv_kernel(const double* __restrict__ A,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y, int rows, int cols) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  const double* a = A + (long long)row * cols;
  double acc = 0.0;
  for (int j = lane; j < cols; j += 64) acc = fma(a[j], x[j], acc);
  acc = wave_sum(acc);
  if (lane == 0) y[row] = acc;
}

int launch_gemv(hipStream_t s, const double* A, const double* x, double* y, int rows, int cols) {
  hipLaunchKernelGGL(gemv_kernel, dim3(ceil_div(rows, 4)), dim3(256), 0, s, A, x, y, rows, cols);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// out = Qbar in, Qbar = blockdiag(Q, ..., Q, Q_f) over t = 1..N (ns N rows).
__global__ __launch_bounds__(256) void block_diag_kernel(const double* __restrict__ Q,
                                                         const double* __restrict__ Qf,
                                                         const double* __restrict__ in,
                                                         double* __restrict__ out, int ns, int N) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= ns * N) return;
  const int t = row / ns + 1, i = row - (t - 1) * ns;
  const double* W = (t == N ? Qf : Q) + (long long)i * ns;
  const double* x = in + (long long)(t - 1) * ns;
  double acc = 0.0;
  for (int j = lane; j < ns; j += 64) acc = fma(W[j], x[j], acc);
  acc = wave_sum(acc);
  if (lane == 0) out[row] = acc;
}

__global__ void diag_weight_kernel(const double* __restrict__ q, const double* __restrict__ in,
                                   double* __restrict__ out, int mx) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < mx) out[r] = q[r] * in[r];
}

int launch_block_diag_weight(Problem& p, const double* in, double* out) {
  if (p.q_diag) {
    hipLaunchKernelGGL(diag_weight_kernel, dim3(ceil_div(p.mx, 256)), dim3(256), 0, p.stream,
                       p.qdiag, in, out, p.mx);
  } else {
    hipLaunchKernelGGL(block_diag_kernel, dim3(ceil_div(p.mx, 4)), dim3(256), 0, p.stream, p.Q,
                       p.Qf, in, out, p.ns, p.N);
  }
  CMPC_LAUNCH_CHECK();
  return 0;
}

// d = [xu - c; c - xl; uu; -ul]; an infinite bound gives an infinite entry (dropped row).
__global__ void make_d_kernel(const double* __restrict__ c, const double* __restrict__ xl,
                              const double* __restrict__ xu, const double* __restrict__ ul,
                              const double* __restrict__ uu, double* __restrict__ d, int ns,
                              int nu, int mx, int n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < mx) {
    const int i = r % ns;
    d[r] = isinf(xu[i]) ? INFINITY : xu[i] - c[r];
    d[mx + r] = isinf(xl[i]) ? INFINITY : c[r] - xl[i];
  }
  if (r < n) {
    const int k = r % nu;
    d[2 * mx + r] = isinf(uu[k]) ? INFINITY : uu[k];
    d[2 * mx + n + r] = isinf(ul[k]) ? INFINITY : -ul[k];
  }
}

int launch_make_d(Problem& p) {
  const int len = p.mx > p.n ? p.mx : p.n;
  hipLaunchKernelGGL(make_d_kernel, dim3(ceil_div(len, 256)), dim3(256), 0, p.stream, p.c, p.xl,
                     p.xu, p.ul, p.uu, p.d, p.ns, p.nu, p.mx, p.n);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// h0 = 1/2 x0' (Q x0) + 1/2 c' (Qbar c) in two stages: per-block partial sums of c' qc,
// then one workgroup adds them (fixed order) to x0' (Q x0).
__global__ __launch_bounds__(256) void dot_partial_kernel(const double* __restrict__ a,
                                                          const double* __restrict__ b,
                                                          long long len,
                                                          double* __restrict__ part) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < len;
       i += (long long)gridDim.x * 256)
    acc = fma(a[i], b[i], acc);
  acc = block_sum256(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void h0_kernel(const double* __restrict__ x0,
                                                 const double* __restrict__ qx0,
                                                 const double* __restrict__ part, int nparts,
                                                 int ns, IpmState* st) {
  __shared__ double sh[4];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < ns; i += 256) a = fma(x0[i], qx0[i], a);
  for (int i = threadIdx.x; i < nparts; i += 256) b += part[i];
  a = block_sum256(a, sh);
  b = block_sum256(b, sh);
  if (threadIdx.x == 0) st->h0 = 0.5 * a + 0.5 * b;
}

int launch_h0(Problem& p) {
  // tmpn2 has room for max(n, ns) doubles; red_part for 1024
  if (launch_gemv(p.stream, p.Q, p.x0, p.tmpn2, p.ns, p.ns)) return CMPC_ERR_HIP;
  const int nparts = std::min(1024, ceil_div(p.mx, 256));
  hipLaunchKernelGGL(dot_partial_kernel, dim3(nparts), dim3(256), 0, p.stream, p.c, p.qc,
                     (long long)p.mx, p.red_part);
  CMPC_LAUNCH_CHECK();
  hipLaunchKernelGGL(h0_kernel, dim3(1), dim3(256), 0, p.stream, p.x0, p.tmpn2, p.red_part, nparts,
                     p.ns, p.st);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// Free response c_t = A^t x0, t = 1..N, for a sparse A (CSR): one workgroup keeps the
// state in LDS and steps through the horizon.
__global__ __launch_bounds__(1024) void free_response_csr_kernel(
    const int* __restrict__ rowptr, const int* __restrict__ col, const double* __restrict__ val,
    const double* __restrict__ x0, double* __restrict__ c, int ns, int N,
    const double* __restrict__ w) {
  extern __shared__ double buf[];  // 2 ns
  double* cur = buf;
  double* nxt = buf + ns;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) cur[i] = x0[i];
  __syncthreads();
  for (int t = 1; t <= N; ++t) {
    for (int i = threadIdx.x; i < ns; i += blockDim.x) {
      double acc = 0.0;
      for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) acc = fma(val[e], cur[col[e]], acc);
      if (w != nullptr) acc += w[(long long)(t - 1) * ns + i];
      nxt[i] = acc;
      c[(long long)(t - 1) * ns + i] = acc;
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
}

// The same with each thread's rows of A (R rows, at most kRowNnz nonzeros each) held in
// registers for the whole horizon, so a step reads only the state in LDS; each row's sum is
// formed over its own entries in the CSR order, as above.
constexpr int kRowNnz = 8;
template <int R>
__global__ __launch_bounds__(1024) void free_response_reg_kernel(
    const int* __restrict__ rowptr, const int* __restrict__ col, const double* __restrict__ val,
    const double* __restrict__ x0, double* __restrict__ c, int ns, int N,
    const double* __restrict__ w) {
  extern __shared__ double buf[];  // 2 ns
  double* cur = buf;
  double* nxt = buf + ns;
  double a[R][kRowNnz];
  int ac[R][kRowNnz], cnt[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = threadIdx.x + 1024 * r;
    const int b = i < ns ? rowptr[i] : 0, e = i < ns ? rowptr[i + 1] : 0;
    cnt[r] = e - b;
#pragma unroll
    for (int k = 0; k < kRowNnz; ++k) {
      a[r][k] = b + k < e ? val[b + k] : 0.0;
      ac[r][k] = b + k < e ? col[b + k] : 0;
    }
  }
  for (int i = threadIdx.x; i < ns; i += 1024) cur[i] = x0[i];
  __syncthreads();
  for (int t = 1; t <= N; ++t) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = threadIdx.x + 1024 * r;
      if (i < ns) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kRowNnz; ++k)
          if (k < cnt[r]) acc = fma(a[r][k], cur[ac[r][k]], acc);
        if (w != nullptr) acc += w[(long long)(t - 1) * ns + i];
        nxt[i] = acc;
        c[(long long)(t - 1) * ns + i] = acc;
      }
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
}

__global__ void add_into_kernel(double* __restrict__ y, const double* __restrict__ w, int len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) y[i] += w[i];
}

// c_t = A c_{t-1} + w_{t-1} (w = NULL: 0), c_0 = x0, t = 1..N (eqn. (dyn) with v = 0).
int launch_free_response(Problem& p) {
  if (p.a_rowptr != nullptr && p.a_maxnnz <= kRowNnz) {
    const size_t lds = sizeof(double) * 2 * (size_t)p.ns;
    const int R = ceil_div(p.ns, 1024);  // 1..4: the CSR copy exists for ns <= 4096
    const double* w = p.wdist;
    switch (R) {
      case 1: hipLaunchKernelGGL(free_response_reg_kernel<1>, dim3(1), dim3(1024), lds, p.stream,
                                 p.a_rowptr, p.a_col, p.a_val, p.x0, p.c, p.ns, p.N, w); break;
      case 2: hipLaunchKernelGGL(free_response_reg_kernel<2>, dim3(1), dim3(1024), lds, p.stream,
                                 p.a_rowptr, p.a_col, p.a_val, p.x0, p.c, p.ns, p.N, w); break;
      case 3: hipLaunchKernelGGL(free_response_reg_kernel<3>, dim3(1), dim3(1024), lds, p.stream,
                                 p.a_rowptr, p.a_col, p.a_val, p.x0, p.c, p.ns, p.N, w); break;
      default: hipLaunchKernelGGL(free_response_reg_kernel<4>, dim3(1), dim3(1024), lds, p.stream,
                                  p.a_rowptr, p.a_col, p.a_val, p.x0, p.c, p.ns, p.N, w); break;
    }
    CMPC_LAUNCH_CHECK();
    return 0;
  }
  if (p.a_rowptr != nullptr) {
    hipLaunchKernelGGL(free_response_csr_kernel, dim3(1), dim3(1024),
                       sizeof(double) * 2 * (size_t)p.ns, p.stream, p.a_rowptr, p.a_col, p.a_val,
                       p.x0, p.c, p.ns, p.N, (const double*)p.wdist);
    CMPC_LAUNCH_CHECK();
    return 0;
  }
  for (int t = 1; t <= p.N; ++t) {
    double* ct = p.c + (size_t)(t - 1) * p.ns;
    if (launch_gemv(p.stream, p.A, t == 1 ? p.x0 : ct - p.ns, ct, p.ns, p.ns)) return CMPC_ERR_HIP;
    if (p.wdist != nullptr) {
      hipLaunchKernelGGL(add_into_kernel, dim3(ceil_div(p.ns, 256)), dim3(256), 0, p.stream, ct,
                         p.wdist + (size_t)(t - 1) * p.ns, p.ns);
      CMPC_LAUNCH_CHECK();
    }
  }
  return 0;
}

// Validity of a device-resident x0: 1 = outside [xl, xu], 2 = not finite.
__global__ void check_x0_kernel(const double* __restrict__ x0, const double* __restrict__ xl,
                                const double* __restrict__ xu, int ns, IpmState* st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) st->x0_flag = 0;
  __syncthreads();
  if (blockIdx.x != 0) return;
  int flag = 0;
  for (int j = threadIdx.x; j < ns; j += blockDim.x) {
    const double x = x0[j];
    if (!isfinite(x)) flag = max(flag, 2);
    else if (x < xl[j] || x > xu[j]) flag = max(flag, 1);
  }
  if (flag) atomicMax(&st->x0_flag, flag);
}

int launch_check_x0(Problem& p) {
  hipLaunchKernelGGL(check_x0_kernel, dim3(1), dim3(256), 0, p.stream, p.x0, p.xl, p.xu,
                     p.ns_real, p.st);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// ---- the cross weight S~ of the stage cost (general data, see fold_general in capi.hip):
// 1/2 x_t'Q~x_t + x_t'S~ v_t + 1/2 v_t'R v_t with x_t = c_t + Gamma_t v adds
// H(j, t) += G_{t-1-j}' S~ (and the transposed block at (t, j)) for j < t <= N-1, and
// h(stage t) += S~' c_t for t = 0..N-1 (c_0 = x0).
__global__ void cross_blocks_kernel(const double* __restrict__ G, const double* __restrict__ S,
                                    double* __restrict__ C, int ns, int nu, int N) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // (m, a, b)
  if (e >= (long long)N * nu * nu) return;
  const int m = (int)(e / ((long long)nu * nu));
  const int ab = (int)(e - (long long)m * nu * nu), a = ab / nu, b = ab - a * nu;
  const double* Gm = G + (long long)m * ns * nu;
  double acc = 0.0;
  for (int i = 0; i < ns; ++i) acc = fma(Gm[(long long)i * nu + a], S[(long long)i * nu + b], acc);
  C[e] = acc;  // C_m = G_m' S~ (nu x nu)
}

__global__ void add_cross_kernel(const double* __restrict__ C, double* __restrict__ H, int nu,
                                 int N) {
  const int n = nu * N;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * n) return;
  const int r = (int)(e / n), c = (int)(e - (long long)r * n);
  const int j = r / nu, t = c / nu, a = r - j * nu, b = c - t * nu;
  if (j < t && t <= N - 1)
    H[e] += C[((long long)(t - 1 - j) * nu + a) * nu + b];
  else if (t < j && j <= N - 1)
    H[e] += C[((long long)(j - 1 - t) * nu + b) * nu + a];
}

int launch_cross_hessian(Problem& p, const double* S) {
  double* C = nullptr;
  CMPC_HIP(hipMalloc(&C, sizeof(double) * (size_t)p.N * p.nu * p.nu));
  hipLaunchKernelGGL(cross_blocks_kernel, dim3(ceil_div((long long)p.N * p.nu * p.nu, 256)),
                     dim3(256), 0, p.stream, p.G, S, C, p.ns, p.nu, p.N);
  hipLaunchKernelGGL(add_cross_kernel, dim3(ceil_div((long long)p.n * p.n, 256)), dim3(256), 0,
                     p.stream, C, p.H, p.nu, p.N);
  const hipError_t e = hipGetLastError();
  hipStreamSynchronize(p.stream);
  hipFree(C);
  if (e != hipSuccess) {
    set_error(std::string("cross-weight Hessian: ") + hipGetErrorString(e));
    return CMPC_ERR_HIP;
  }
  return 0;
}

__global__ void h_cross_kernel(const double* __restrict__ S, const double* __restrict__ x0,
                               const double* __restrict__ c, double* __restrict__ h, int ns,
                               int nu, int N) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;  // (t, b)
  if (e >= nu * N) return;
  const int t = e / nu, b = e - t * nu;
  const double* ct = t == 0 ? x0 : c + (long long)(t - 1) * ns;
  double acc = 0.0;
  for (int i = 0; i < ns; ++i) acc = fma(S[(long long)i * nu + b], ct[i], acc);
  h[e] += acc;
}

int launch_h_cross(Problem& p) {
  hipLaunchKernelGGL(h_cross_kernel, dim3(ceil_div(p.n, 256)), dim3(256), 0, p.stream, p.Sx,
                     p.x0, p.c, p.h, p.ns, p.nu, p.N);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// The problem's own states and inputs from xa = c + Gamma v (states x_1..x_N with the extra
// stage rows): x_t = the first ns_real components of xa_t; with a feedback the inputs are the
// first nu extra components of xa_{t+1} (they hold K x_t + v_t), else u = v.
__global__ void unfold_solution_kernel(const double* __restrict__ xa, const double* __restrict__ v,
                                       double* __restrict__ u, double* __restrict__ x, int ns,
                                       int ns_real, int nu, int N, int feedback) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x != nullptr && e < (long long)ns_real * N) {
    const int t = (int)(e / ns_real), i = (int)(e - (long long)t * ns_real);
    x[e] = xa[(long long)t * ns + i];
  }
  if (u != nullptr && e < (long long)nu * N) {
    const int t = (int)(e / nu), k = (int)(e - (long long)t * nu);
    u[e] = feedback ? xa[(long long)t * ns + ns_real + k] : v[e];
  }
}

int launch_unfold_solution(Problem& p, const double* xa, double* u, double* x) {
  const long long len = std::max<long long>((long long)p.ns_real * p.N, p.n);
  hipLaunchKernelGGL(unfold_solution_kernel, dim3(ceil_div(len, 256)), dim3(256), 0, p.stream,
                     xa, p.v, u, x, p.ns, p.ns_real, p.nu, p.N, p.feedback ? 1 : 0);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// Hb = Rbar = blockdiag(R, ..., R) (n x n, full).
__global__ void rbar_kernel(const double* __restrict__ R, double* __restrict__ Hb, int nu, int n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * n) return;
  const int i = (int)(e / n), j = (int)(e - (long long)i * n);
  double v = 0.0;
  if (i / nu == j / nu) v = R[(i % nu) * nu + (j % nu)];
  Hb[e] = v;
}

int launch_rbar(Problem& p, double* Hb) {
  hipLaunchKernelGGL(rbar_kernel, dim3(ceil_div((long long)p.n * p.n, 256)), dim3(256), 0,
                     p.stream, p.R, Hb, p.nu, p.n);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// H[j][i] = H[i][j] for i > j.
__global__ void mirror_lower_kernel(double* __restrict__ H, int n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * n) return;
  const int i = (int)(e / n), j = (int)(e - (long long)i * n);
  if (j > i) H[e] = H[(long long)j * n + i];
}

int launch_mirror_lower(hipStream_t s, double* H, int n) {
  hipLaunchKernelGGL(mirror_lower_kernel, dim3(ceil_div((long long)n * n, 256)), dim3(256), 0, s,
                     H, n);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// Dense Gamma (mx x n) from the blocks G_m, structural zeros written.
__global__ void dense_gamma_kernel(const double* __restrict__ G, double* __restrict__ out,
                                   int ns, int nu, int N) {
  const int n = nu * N;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)ns * N * n) return;
  const long long r = e / n;
  const int a = (int)(e - r * n);
  const int t = (int)(r / ns) + 1, i = (int)(r - (long long)(t - 1) * ns);
  const int j = a / nu, k = a - j * nu;
  out[e] = a < t * nu ? G[((long long)(t - 1 - j) * ns + i) * nu + k] : 0.0;
}

int launch_dense_gamma(Problem& p, double* dense) {
  hipLaunchKernelGGL(dense_gamma_kernel, dim3(ceil_div((long long)p.mx * p.n, 256)), dim3(256), 0,
                     p.stream, p.G, dense, p.ns, p.nu, p.N);
  CMPC_LAUNCH_CHECK();
  return 0;
}

}  // namespace cmpc
