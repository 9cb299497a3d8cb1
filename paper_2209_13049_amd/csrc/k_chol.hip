// Dense Cholesky factorisation K = L L' and the two triangular solves (Section 3: the
// condensed matrix is positive definite, so it is factored by Cholesky and p_v follows by
// triangular solves).  Row-major, lower triangle, leading dimension ld.
//
// Blocked right-looking factorisation with 64-column panels:
//   potrf_diag   one workgroup factors the 64 x 64 diagonal block in LDS;
//   trsm_panel   the rows below solve X L_kk' = A_ik, one row per thread, L_kk in LDS;
//   syrk_update  every 64 x 64 tile of the trailing lower triangle subtracts L_ik L_jk'
//                with v_mfma_f64_16x16x4f64 from LDS-staged panels.
// The triangular solves run in one workgroup: 64-row blocks, wavefront-wide dot products
// for the off-diagonal part, a shuffle-broadcast substitution inside each diagonal block.
#include "problem.hpp"

namespace cmpc {

__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ K, int ld, int k0,
                                                         int nb, int* done, int* info,
                                                         int* status) {
  __shared__ double a[64][65];
  if (*done) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < 4096; e += 256) {
    const int i = e >> 6, j = e & 63;
    a[i][j] = (i < nb && j <= i) ? K[(long long)(k0 + i) * ld + k0 + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double piv = a[j][j];
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (tid == 0) {
        *info = k0 + j + 1;
        *status = CMPC_ERR_CHOLESKY;
        *done = 1;
      }
      return;
    }
    const double inv = 1.0 / piv;
    for (int e = tid; e < 4096; e += 256) {
      const int i = e >> 6, k = e & 63;
      if (k > j && k <= i && i < nb) a[i][k] -= a[i][j] * a[k][j] * inv;
    }
    __syncthreads();
  }
  for (int e = tid; e < 4096; e += 256) {
    const int i = e >> 6, j = e & 63;
    if (i < nb && j <= i) {
      const double r = sqrt(a[j][j]);
      K[(long long)(k0 + i) * ld + k0 + j] = (i == j) ? r : a[i][j] / r;
    }
  }
}

__global__ __launch_bounds__(256) void trsm_panel_kernel(double* __restrict__ K, int ld, int k0,
                                                         int nb, int n, const int* done) {
  __shared__ double L[64][65];
  if (*done) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < 4096; e += 256) {
    const int i = e >> 6, j = e & 63;
    L[i][j] = (i < nb && j <= i) ? K[(long long)(k0 + i) * ld + k0 + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  const int row = k0 + nb + blockIdx.x * 256 + tid;
  if (row >= n) return;
  double* rp = K + (long long)row * ld + k0;
  double x[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) x[j] = (j < nb) ? rp[j] : 0.0;
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    double sum = x[j];
#pragma unroll
    for (int k = 0; k < j; ++k) sum = fma(-x[k], L[j][k], sum);
    x[j] = sum / L[j][j];
  }
#pragma unroll
  for (int j = 0; j < 64; ++j)
    if (j < nb) rp[j] = x[j];
}

__global__ __launch_bounds__(256) void syrk_update_kernel(double* __restrict__ K, int ld, int k0,
                                                          int nb, int n, const int* done) {
  __shared__ double PI[64][65];
  __shared__ double PJ[64][65];
  if (*done) return;
  const int k1 = k0 + nb;
  // lower-triangular tile index -> (I, J), I >= J
  const int b = blockIdx.x;
  int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= b) ++I;
  while (I * (I + 1) / 2 > b) --I;
  const int J = b - I * (I + 1) / 2;
  const int r0 = k1 + 64 * I, c0 = k1 + 64 * J;
  const int tid = threadIdx.x;
  for (int e = tid; e < 4096; e += 256) {
    const int i = e >> 6, k = e & 63;
    PI[i][k] = (r0 + i < n && k < nb) ? K[(long long)(r0 + i) * ld + k0 + k] : 0.0;
    PJ[i][k] = (c0 + i < n && k < nb) ? K[(long long)(c0 + i) * ld + k0 + k] : 0.0;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int wr = wave >> 1, wc = wave & 1;
  if (I == J && wc > wr) return;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0, 0, 0, 0};
  for (int ks = 0; ks < 16; ++ks) {
    double xa[2], xb[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      xa[q] = PI[32 * wr + 16 * q + li][4 * ks + lk];
      xb[q] = PJ[32 * wc + 16 * q + li][4 * ks + lk];
    }
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
        acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[ib], xb[jb], acc[ib][jb], 0, 0, 0);
  }
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = r0 + 32 * wr + 16 * ib + lk + 4 * v;
        const int gj = c0 + 32 * wc + 16 * jb + li;
        if (gi < n && gj <= gi) K[(long long)gi * ld + gj] -= acc[ib][jb][v];
      }
}

int launch_potrf(hipStream_t s, double* K, int n, int ld, int* done, int* info, int* status) {
  for (int k0 = 0; k0 < n; k0 += 64) {
    const int nb = n - k0 < 64 ? n - k0 : 64;
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, K, ld, k0, nb, done, info,
                       status);
    CMPC_LAUNCH_CHECK();
    const int rest = n - k0 - nb;
    if (rest > 0) {
      hipLaunchKernelGGL(trsm_panel_kernel, dim3(ceil_div(rest, 256)), dim3(256), 0, s, K, ld, k0,
                         nb, n, done);
      CMPC_LAUNCH_CHECK();
      const int nt = ceil_div(rest, 64);
      hipLaunchKernelGGL(syrk_update_kernel, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, K, ld, k0,
                         nb, n, done);
      CMPC_LAUNCH_CHECK();
    }
  }
  return 0;
}

// Solve L L' x = b in place, one workgroup, n <= 8192.
__global__ __launch_bounds__(256) void potrs_kernel(const double* __restrict__ L, int n, int ld,
                                                    double* __restrict__ b, const int* done) {
  __shared__ double y[8192];
  if (done != nullptr && *done) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int i = tid; i < n; i += 256) y[i] = b[i];
  __syncthreads();
  // forward: L y = b, blocks of 64 rows, left-looking
  for (int k0 = 0; k0 < n; k0 += 64) {
    const int nb = n - k0 < 64 ? n - k0 : 64;
    for (int q = wave; q < nb; q += 4) {
      const double* rp = L + (long long)(k0 + q) * ld;
      double acc = 0.0;
      for (int j = lane; j < k0; j += 64) acc = fma(rp[j], y[j], acc);
      acc = wave_sum(acc);
      if (lane == 0) y[k0 + q] -= acc;
    }
    __syncthreads();
    if (wave == 0) {
      double yr = lane < nb ? y[k0 + lane] : 0.0;
      for (int j = 0; j < nb; ++j) {
        const double ljj = L[(long long)(k0 + j) * ld + k0 + j];
        const double yj = __shfl(yr, j, 64) / ljj;
        if (lane == j) yr = yj;
        else if (lane > j && lane < nb) yr = fma(-L[(long long)(k0 + lane) * ld + k0 + j], yj, yr);
      }
      if (lane < nb) y[k0 + lane] = yr;
    }
    __syncthreads();
  }
  // backward: L' x = y, blocks from the bottom, right-looking updates of the rows above
  const int last0 = ((n - 1) / 64) * 64;
  for (int k0 = last0; k0 >= 0; k0 -= 64) {
    const int nb = n - k0 < 64 ? n - k0 : 64;
    if (wave == 0) {
      double xr = lane < nb ? y[k0 + lane] : 0.0;
      for (int j = nb - 1; j >= 0; --j) {
        const double ljj = L[(long long)(k0 + j) * ld + k0 + j];
        const double xj = __shfl(xr, j, 64) / ljj;
        if (lane == j) xr = xj;
        else if (lane < j) xr = fma(-L[(long long)(k0 + j) * ld + k0 + lane], xj, xr);
      }
      if (lane < nb) y[k0 + lane] = xr;
    }
    __syncthreads();
    for (int i = tid; i < k0; i += 256) {
      double acc = 0.0;
      for (int j = 0; j < nb; ++j) acc = fma(L[(long long)(k0 + j) * ld + i], y[k0 + j], acc);
      y[i] -= acc;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += 256) b[i] = y[i];
}

int launch_potrs(hipStream_t s, const double* L, int n, int ld, double* b, const int* done) {
  if (n > 8192) {
    set_error("potrs: n > 8192 not supported");
    return CMPC_ERR_INVALID;
  }
  hipLaunchKernelGGL(potrs_kernel, dim3(1), dim3(256), 0, s, L, n, ld, b, done);
  CMPC_LAUNCH_CHECK();
  return 0;
}

}  // namespace cmpc
