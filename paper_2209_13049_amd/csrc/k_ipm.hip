// Interior-point iteration kernels (Algorithm 1 of the paper) other than the formation and
// factorisation of K.  All of them read the device-side IpmState and return at entry once
// the solve is done, so a whole iteration can be queued (or graph-replayed) without a host
// round trip.
//
// Rows of the inequality system J v <= d, with J = [Gamma; -Gamma; I; -I], are kept in the
// order [x <= xu (mx) | -x <= -xl (mx) | u <= uu (n) | -u <= -ul (n)].  A "pair" is the
// upper/lower couple of one bounded quantity: pair p < mx is state row p, pair mx + c is
// control c.  Because the two rows of a pair share one row of Gamma (with opposite sign),
// J' diag(sigma) J = Gamma' diag(sigma_up + sigma_lo) Gamma + diag(sigma_up + sigma_lo)_u
// and J' y = Gamma' (y_up - y_lo) + (y_up - y_lo)_u.  A row whose bound is infinite has
// d = +inf and takes no part (s = 1, lambda = z = 0, sigma = 0).
#include "problem.hpp"

namespace cmpc {

constexpr double kKappaEps = 10.0, kKappaMu = 0.2, kThetaMu = 1.5, kKappaSigma = 1e10;
constexpr double kTauMin = 0.99, kMuInit = 0.1, kSInitMin = 1e-2, kAlphaMin = 1e-14;

int ipm_alloc_work(Problem& p) {
  const size_t n = p.n, m = p.m, mx = p.mx;
  const size_t nmax = (size_t)(p.n > p.ns ? p.n : p.ns);
  double** vecs_n[] = {&p.v, &p.pv, &p.rhs, &p.Du, &p.Hv, &p.h, &p.tmpn, &p.eqs};
  for (double** q : vecs_n) CMPC_HIP(hipMalloc(q, sizeof(double) * n));
  CMPC_HIP(hipMalloc(&p.tmpn2, sizeof(double) * nmax));
  double** vecs_r[] = {&p.ref_res, &p.ref_dlt};
  for (double** q : vecs_r) CMPC_HIP(hipMalloc(q, sizeof(double) * n));
  double** vecs_m[] = {&p.s, &p.lam, &p.z, &p.ps, &p.plam, &p.pz, &p.d};
  for (double** q : vecs_m) CMPC_HIP(hipMalloc(q, sizeof(double) * m));
  double** vecs_mx[] = {&p.gv, &p.gpv, &p.c, &p.qc, &p.Dx, &p.tmpmx};
  for (double** q : vecs_mx) CMPC_HIP(hipMalloc(q, sizeof(double) * mx));
  CMPC_HIP(hipMalloc(&p.x0, sizeof(double) * p.ns));
  CMPC_HIP(hipMalloc(&p.wx, sizeof(double) * 3 * mx));
  CMPC_HIP(hipMalloc(&p.wu, sizeof(double) * 3 * n));
  CMPC_HIP(hipMalloc(&p.gt, sizeof(double) * 3 * n));
  p.n_prep_blocks = ceil_div((long long)mx + n, 256);
  p.n_step_blocks = p.n_prep_blocks;
  CMPC_HIP(hipMalloc(&p.norm_part, sizeof(double) * 5 * p.n_prep_blocks));
  CMPC_HIP(hipMalloc(&p.alpha_part, sizeof(double) * 2 * p.n_step_blocks));
  p.gt_chunks = gt_chunk_count(p.ns, p.nu, p.N);
  CMPC_HIP(hipMalloc(&p.gt_part, sizeof(double) * 3 * kGtJ * (size_t)p.gt_chunks));
  CMPC_HIP(hipMalloc(&p.red_part, sizeof(double) * 1024));
  CMPC_HIP(hipMalloc(&p.Wdiag, sizeof(double) * wall_doubles(p.n)));
  CMPC_HIP(hipMalloc(&p.st, sizeof(IpmState)));
  CMPC_HIP(hipMemset(p.st, 0, sizeof(IpmState)));
  return 0;
}

// ---------------------------------------------------------------- Gamma' W  (NV vectors)
// out[v][j nu + k] = sum_{m < N-j} sum_i G_m[i][k] W[v][(m + j) ns + i]  (W[v] = w_1 .. w_N),
// through Gt: Gamma is block Toeplitz (block (t, j) = G_{t-1-j}).  Workgroup (jr, k, ic): the
// column blocks j = kGtJ jr .. +kGtJ-1, column k, rows i = 256 ic + thread.  A thread walks m
// upward; G_m[i][k] is read once for all kGtJ column blocks of the range, and the blocks of W
// it meets, w_{m+j+1} for j in the range, form a window that slides by one block per m (each
// block of W read once per range).  kGtJ steps of m are loaded together (the window's
// earlier blocks are kept in registers, the step's new ones loaded with the Gt entries), then
// consumed in m order.  The workgroup adds its 256 rows in a fixed pattern (quad sums by DPP,
// then the 64 quads in order) into its partial; a second pass adds the partials in order.
// Each workgroup takes one of kGtMs consecutive parts of the range of m (shorter chains).
template <int NV>
__device__ __forceinline__ void gamma_t_partial_body(int bid, const double* __restrict__ Gt,
                                                     const double* __restrict__ W,
                                                     long long wstride, double* __restrict__ part,
                                                     int ns, int nu, int N,
                                                     const int* __restrict__ done) {
  constexpr int J = kGtJ;
  __shared__ double red[J * NV][65];
  if (done != nullptr && *done) return;
  const int nic = gt_row_chunks(ns);
  const int mh = bid % kGtMs, r2 = bid / kGtMs;
  const int ic = r2 % nic, rest = r2 / nic;
  const int k = rest % nu, jr = rest / nu;
  const int j0 = J * jr;
  const int mend = N - j0;  // m < N - j0 reaches the range's first column block
  const int half = ((mend + J - 1) / J + kGtMs - 1) / kGtMs;  // steps of J per part
  const int ms0 = mh * half * J, ms1 = min(mend, (mh + 1) * half * J);
  const int tid = threadIdx.x;
  const int i = 256 * ic + tid;
  const int icl = i < ns ? i : ns - 1;
  const double* __restrict__ wi = W + icl;
  auto wblock = [&](int s, double (&x)[NV]) {  // w_{s+1}[i] of the NV vectors, s clamped
    const long long o = (long long)(s < N ? s : N - 1) * ns;
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = wi[v * wstride + o];
  };
  double acc[J][NV], old[J - 1][NV];
#pragma unroll
  for (int q = 0; q < J; ++q)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[q][v] = 0.0;
#pragma unroll
  for (int q = 0; q < J - 1; ++q) wblock(ms0 + j0 + q, old[q]);
  for (int m0 = ms0; m0 < ms1; m0 += J) {
    double g[J], nw[J][NV];
#pragma unroll
    for (int u = 0; u < J; ++u) {
      const int mc = m0 + u < ms1 ? m0 + u : ms1 - 1;
      g[u] = Gt[((long long)mc * nu + k) * ns + icl];
      wblock(m0 + j0 + J - 1 + u, nw[u]);
    }
#pragma unroll
    for (int u = 0; u < J; ++u) {
      if (m0 + u < ms1) {  // uniform
#pragma unroll
        for (int jj = 0; jj < J; ++jj) {
          if (m0 + u + j0 + jj <= N - 1) {  // block m + j within the horizon (uniform)
            const int q = u + jj;  // window position: block m0 + j0 + q
#pragma unroll
            for (int v = 0; v < NV; ++v)
              acc[jj][v] = fma(g[u], q < J - 1 ? old[q < J - 1 ? q : 0][v]
                                               : nw[q >= J - 1 ? q - (J - 1) : 0][v],
                               acc[jj][v]);
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < J - 1; ++q)
#pragma unroll
      for (int v = 0; v < NV; ++v) old[q][v] = nw[q + 1][v];
  }
  const int lane = tid & 63;
#pragma unroll
  for (int jj = 0; jj < J; ++jj)
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double x = i < ns ? acc[jj][v] : 0.0;
      x += dpp_f64<0xB1>(x);  // lane ^ 1
      x += dpp_f64<0x4E>(x);  // lane ^ 2: the quad's sum (the same in its 4 lanes)
      if ((lane & 3) == 0) red[jj * NV + v][tid >> 2] = x;
    }
  __syncthreads();
  if (tid < J * NV) {
    double sum = 0.0;
#pragma unroll 16
    for (int q = 0; q < 64; ++q) sum += red[tid][q];
    part[(long long)bid * J * NV + tid] = sum;
  }
}

template <int NV>
__global__ __launch_bounds__(256) void gamma_t_partial_kernel(
    const double* __restrict__ Gt, const double* __restrict__ W, long long wstride,
    double* __restrict__ part, int ns, int nu, int N, const int* __restrict__ done) {
  gamma_t_partial_body<NV>(blockIdx.x, Gt, W, wstride, part, ns, nu, N, done);
}

// (Gamma' W)[v][a] from the pass's partials: the (row chunk, part of m) partials of column a
// added in order.
template <int NV>
__device__ __forceinline__ void gamma_t_column(const double* __restrict__ part, int a, int ns,
                                               int nu, double (&out)[NV]) {
  const int j = a / nu, k = a - j * nu;
  const int jr = j / kGtJ, jj = j - jr * kGtJ;
  const int nparts = gt_row_chunks(ns) * kGtMs;
  const long long base = ((long long)jr * nu + k) * nparts;
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = 0.0;
#pragma unroll 8
  for (int c = 0; c < nparts; ++c)
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] += part[((base + c) * kGtJ + jj) * NV + v];
}

// out[v][a] for 256 columns a per workgroup.
template <int NV>
__device__ __forceinline__ void gamma_t_reduce_body(int bid, const double* __restrict__ part,
                                                    double* __restrict__ out, int n, int ns,
                                                    int nu, const int* __restrict__ done) {
  if (done != nullptr && *done) return;
  const int a = bid * 256 + threadIdx.x;
  if (a >= n) return;
  double g[NV];
  gamma_t_column<NV>(part, a, ns, nu, g);
#pragma unroll
  for (int v = 0; v < NV; ++v) out[(long long)v * n + a] = g[v];
}

template <int NV>
__global__ __launch_bounds__(256) void gamma_t_reduce_kernel(const double* __restrict__ part,
                                                             double* __restrict__ out, int n,
                                                             int ns, int nu,
                                                             const int* __restrict__ done) {
  gamma_t_reduce_body<NV>(blockIdx.x, part, out, n, ns, nu, done);
}

int launch_gamma_t(Problem& p, const double* w, int nvec, double* out, const int* done) {
  if (nvec == 3) {
    hipLaunchKernelGGL(gamma_t_partial_kernel<3>, dim3(p.gt_chunks), dim3(256), 0, p.stream,
                       p.Gt, w, (long long)p.mx, p.gt_part, p.ns, p.nu, p.N, done);
    CMPC_LAUNCH_CHECK();
    hipLaunchKernelGGL(gamma_t_reduce_kernel<3>, dim3(ceil_div(p.n, 256)), dim3(256), 0,
                       p.stream, p.gt_part, out, p.n, p.ns, p.nu, done);
  } else {
    hipLaunchKernelGGL(gamma_t_partial_kernel<1>, dim3(p.gt_chunks), dim3(256), 0, p.stream,
                       p.Gt, w, (long long)p.mx, p.gt_part, p.ns, p.nu, p.N, done);
    CMPC_LAUNCH_CHECK();
    hipLaunchKernelGGL(gamma_t_reduce_kernel<1>, dim3(ceil_div(p.n, 256)), dim3(256), 0,
                       p.stream, p.gt_part, out, p.n, p.ns, p.nu, done);
  }
  CMPC_LAUNCH_CHECK();
  return 0;
}

// ---------------------------------------------------------------- y = Gamma x
// y[(t-1) ns + i] = sum_{e < t nu} Gt[e][i] x[(t-1-m) nu + k]  (e = m nu + k).  One
// workgroup per (group of MT row blocks t = t_hi, t_hi - 1, ..., larger first; 64 rows):
// lane = row i (coalesced rows of Gt).  The range of e is cut into chunks of 16; wavefront w
// takes the chunks c = w, w + 4, w + 8, ... in order (each row of Gt read once for the whole
// group) and keeps one sum per row block of the group, and the four wavefronts' sums are added
// in order.  Which wavefront adds which term, and in which order, depends only on e, so the
// result does not depend on MT.  The x entries, the same in every lane, come through the
// scalar cache, loaded with the rows (MT = 1), or, for the groups' four times as many, from a
// copy of x in LDS read where each product needs it (broadcast reads; n <= kMvXs), which keeps
// the registers, and so the waves in flight, of a single block's pass; the copy measured
// slower for MT = 1.
constexpr int kMvXs = 2048;
template <int MT>
__device__ __forceinline__ void gamma_mv_body(int bid, const double* __restrict__ Gt,
                                              const double* __restrict__ xg,
                                              double* __restrict__ y, int ns, int nu, int N,
                                              const int* __restrict__ done,
                                              const double* __restrict__ scale = nullptr) {
  __shared__ double red[4][MT][64];
  __shared__ double xs[MT > 1 ? kMvXs : 1];
  if (done != nullptr && *done) return;
  const int n = N * nu;
  const bool in_lds = MT > 1 && n <= kMvXs;  // uniform
  if (in_lds) {
    for (int c = threadIdx.x; c < n; c += 256) xs[c] = xg[c];
    __syncthreads();
  }
  const double* x = in_lds ? xs : xg;
  const int nbx = (ns + 63) >> 6;
  const int tb = bid / nbx, bx = bid - tb * nbx;
  const int t_hi = N - MT * tb;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int i = 64 * bx + lane, ic = i < ns ? i : ns - 1;
  const int T = t_hi * nu;
  double acc[MT];
#pragma unroll
  for (int u = 0; u < MT; ++u) acc[u] = 0.0;
  if constexpr (MT > 1) {  // x read where it is used (from LDS if it fits): few registers,
                           // many waves in flight (loading the next chunk's rows ahead measured
                           // slower: fewer waves)
    for (int e0 = 16 * w; e0 < T; e0 += 64) {
      double gv[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = e0 + q < T ? e0 + q : T - 1;
        gv[q] = Gt[(long long)e * ns + ic];
      }
      int m = e0 / nu, k = e0 - m * nu;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        if (e0 + q < T) {
#pragma unroll
          for (int u = 0; u < MT; ++u)
            if (m < t_hi - u) acc[u] = fma(gv[q], x[(t_hi - u - 1 - m) * nu + k], acc[u]);
        }
        if (++k == nu) {
          k = 0;
          ++m;
        }
      }
    }
  } else {
    for (int e0 = 16 * w; e0 < T; e0 += 64) {
      double gv[16], xv[16][MT];
      const int m0 = e0 / nu, k0 = e0 - m0 * nu;
      int mq = m0, kq = k0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = e0 + q < T ? e0 + q : T - 1;
        gv[q] = Gt[(long long)e * ns + ic];
#pragma unroll
        for (int u = 0; u < MT; ++u) {
          const int xi = (t_hi - u - 1 - mq) * nu + kq;
          xv[q][u] = x[xi > 0 ? xi : 0];
        }
        if (++kq == nu) {
          kq = 0;
          ++mq;
        }
      }
      int m = m0, k = k0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        if (e0 + q < T) {
#pragma unroll
          for (int u = 0; u < MT; ++u)
            if (m < t_hi - u) acc[u] = fma(gv[q], xv[q][u], acc[u]);
        }
        if (++k == nu) {
          k = 0;
          ++m;
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < MT; ++u) red[w][u][lane] = acc[u];
  __syncthreads();
  if (w < MT) {  // wavefront w writes row block t_hi - w
    const int t = t_hi - w;
    if (t >= 1 && i < ns) {
      const long long r = (long long)(t - 1) * ns + i;
      const double val = ((red[0][w][lane] + red[1][w][lane]) + red[2][w][lane]) + red[3][w][lane];
      y[r] = scale != nullptr ? val * scale[r] : val;
    }
  }
}

// y = Gamma x, or with scale != NULL y = scale o (Gamma x)
__global__ __launch_bounds__(256) void gamma_mv_kernel(const double* __restrict__ Gt,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y, int ns, int nu,
                                                       int N, const int* __restrict__ done,
                                                       const double* __restrict__ scale) {
  gamma_mv_body<kMvT>(blockIdx.x, Gt, x, y, ns, nu, N, done, scale);
}

int launch_gamma_mv(Problem& p, const double* x, double* y, const int* done,
                    const double* scale) {
  hipLaunchKernelGGL(gamma_mv_kernel, dim3(gmv_blocks(p.ns, p.N)), dim3(256), 0, p.stream, p.Gt,
                     x, y, p.ns, p.nu, p.N, done, scale);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// ---------------------------------------------------------------- y = H x (H symmetric)
// One wavefront per row, lanes stride the (contiguous) row.
__device__ __forceinline__ void hv_body(int bid, const double* __restrict__ H,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ y, int n,
                                                 const int* __restrict__ done) {
  if (done != nullptr && *done) return;
  const int c = bid * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= n) return;
  const double* row = H + (long long)c * n;
  double acc = 0.0;
  for (int j = lane; j < n; j += 64) acc = fma(row[j], x[j], acc);
  acc = wave_sum(acc);
  if (lane == 0) y[c] = acc;
}

__global__ __launch_bounds__(256) void hv_kernel(const double* __restrict__ H,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ y, int n,
                                                 const int* __restrict__ done) {
  hv_body(blockIdx.x, H, x, y, n, done);
}

static int launch_hv(Problem& p, const double* x, double* y, const int* done) {
  hipLaunchKernelGGL(hv_kernel, dim3(ceil_div(p.n, 4)), dim3(256), 0, p.stream, p.H, x, y, p.n,
                     done);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// ---------------------------------------------------------------- start point
// Start point.  Cold (warm = 0): v = 0, s = max(d, 1e-2), lambda = z = mu0 / s with
// mu0 = 0.1.  Warm (warm = 1, the receding-horizon start): v and gv = Gamma v are given, so
// s = max(d - J v, 1e-2) with J v = [Gamma v; -Gamma v; v; -v], and lambda = z = mu0 / s.
__device__ __forceinline__ void ipm_init_body(int bid, const double* __restrict__ d, double* __restrict__ s,
                                double* __restrict__ lam, double* __restrict__ z,
                                double* __restrict__ v, double* __restrict__ gv, int m, int n,
                                int mx, IpmState* st, double tol, int max_iter, int low,
                                double mu_switch, double contract, int warm = 0,
                                double mu0 = kMuInit) {
  const long long i = (long long)bid * blockDim.x + threadIdx.x;
  if (i < m) {
    const double di = d[i];
    if (isinf(di)) {
      s[i] = 1.0;
      lam[i] = 0.0;
      z[i] = 0.0;
    } else {
      double jv = 0.0;
      if (warm) {
        if (i < mx) jv = gv[i];
        else if (i < 2LL * mx) jv = -gv[i - mx];
        else if (i < 2LL * mx + n) jv = v[i - 2LL * mx];
        else jv = -v[i - 2LL * mx - n];
      }
      const double si = fmax(di - jv, kSInitMin);
      s[i] = si;
      lam[i] = mu0 / si;
      z[i] = mu0 / si;
    }
  }
  if (!warm) {
    if (i < n) v[i] = 0.0;
    if (i < mx) gv[i] = 0.0;
  }
  if (i == 0) {
    const int xf = st->x0_flag;
    st->mu = mu0;
    st->tau = fmax(kTauMin, 1.0 - mu0);
    st->alpha = st->alpha_z = 0.0;
    st->tol = tol;
    st->mu_min = tol / 10.0;
    st->iter = 0;
    st->status = xf == 2 ? CMPC_ERR_NONFINITE : (xf == 1 ? CMPC_ERR_X0_BOUNDS : kRunning);
    st->done = xf != 0;
    st->info = 0;
    st->max_iter = max_iter;
    st->switch_iter = -1;
    st->refine_steps = 0;
    st->nonc = 0;
    st->use_low = low;
    st->mixed = low;
    st->mu_switch = mu_switch;
    st->contract = contract;
    st->ref_skip = 1;
    st->res_prev = INFINITY;
  }
}

__global__ void ipm_init_kernel(const double* __restrict__ d, double* __restrict__ s,
                                double* __restrict__ lam, double* __restrict__ z,
                                double* __restrict__ v, double* __restrict__ gv, int m, int n,
                                int mx, IpmState* st, double tol, int max_iter, int low,
                                double mu_switch, double contract, int warm, double mu0) {
  ipm_init_body(blockIdx.x, d, s, lam, z, v, gv, m, n, mx, st, tol, max_iter, low, mu_switch,
                contract, warm, mu0);
}

int launch_ipm_init(Problem& p, const cmpc_options& o, int warm, double mu0) {
  const long long len = p.m;
  const int low = o.precision == CMPC_BF16_SYRK ? 2 : (o.precision == CMPC_FP32_SYRK ? 1 : 0);
  if (warm && launch_gamma_mv(p, p.v, p.gv, nullptr)) return CMPC_ERR_HIP;
  hipLaunchKernelGGL(ipm_init_kernel, dim3(ceil_div(len, 256)), dim3(256), 0, p.stream, p.d, p.s,
                     p.lam, p.z, p.v, p.gv, p.m, p.n, p.mx, p.st, o.tol, o.max_iter, low,
                     o.mu_switch, o.refine_contract, warm, warm ? mu0 : kMuInit);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// Receding-horizon shift of the controls (reading of Section 1): stage t of the result is
// stage t + 1 of v (t = 0..N-2), the last stage repeats stage N-1.  out must not alias v.
__global__ void shift_controls_kernel(const double* __restrict__ v, double* __restrict__ out,
                                      int nu, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int src = i + nu < n ? i + nu : i;  // the last stage (i >= n - nu) keeps its value
  out[i] = v[src];
}

int launch_shift_controls(Problem& p) {
  hipLaunchKernelGGL(shift_controls_kernel, dim3(ceil_div(p.n, 256)), dim3(256), 0, p.stream,
                     p.v, p.tmpn, p.nu, p.n);
  CMPC_LAUNCH_CHECK();
  CMPC_HIP(hipMemcpyAsync(p.v, p.tmpn, sizeof(double) * p.n, hipMemcpyDeviceToDevice, p.stream));
  return 0;
}

// ---------------------------------------------------------------- per-pair helpers
struct PairRows {
  long long up, lo;
  double jv;  // (J v) of the upper row; the lower row has -jv
};

__device__ inline PairRows pair_rows(int p, int mx, int n, const double* gv, const double* v) {
  PairRows pr;
  if (p < mx) {
    pr.up = p;
    pr.lo = (long long)mx + p;
    pr.jv = gv[p];
  } else {
    const int c = p - mx;
    pr.up = 2LL * mx + c;
    pr.lo = 2LL * mx + n + c;
    pr.jv = v[c];
  }
  return pr;
}

// sigma, folded weights, Gamma' right-hand sides and the residual norms of the iterate.
__device__ __forceinline__ void prep_body(int bid, 
    const double* __restrict__ d, const double* __restrict__ s, const double* __restrict__ lam,
    const double* __restrict__ z, const double* __restrict__ gv, const double* __restrict__ v,
    double* __restrict__ Dx, double* __restrict__ Du, double* __restrict__ wx,
    double* __restrict__ wu, double* __restrict__ norm_part, int mx, int n,
    const int* __restrict__ done) {
  __shared__ double sh5[5][4];
  if (*done) return;
  const int p = bid * 256 + threadIdx.x;
  double nr3 = 0.0, nlz = 0.0, szmax = 0.0, szmin = INFINITY, gap = 0.0;
  if (p < mx + n) {
    const PairRows pr = pair_rows(p, mx, n, gv, v);
    double sig[2] = {0.0, 0.0}, dl[2] = {0.0, 0.0}, inv[2] = {0.0, 0.0}, y3[2] = {0.0, 0.0};
    const long long rows[2] = {pr.up, pr.lo};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const long long r = rows[q];
      const double dr = d[r];
      if (!isinf(dr)) {
        const double sr = s[r], zr = z[r], lr = lam[r];
        const double jv = q == 0 ? pr.jv : -pr.jv;
        const double r3 = jv - dr + sr;
        sig[q] = zr / sr;
        inv[q] = 1.0 / sr;
        y3[q] = sig[q] * r3;
        dl[q] = lr;
        nr3 = fmax(nr3, fabs(r3));
        nlz = fmax(nlz, fabs(lr - zr));
        const double sz = sr * zr;
        szmax = fmax(szmax, sz);
        szmin = fmin(szmin, sz);
        gap += sz;
      }
    }
    const double D = sig[0] + sig[1];
    if (p < mx) {
      Dx[p] = D;
      wx[p] = dl[0] - dl[1];
      wx[(long long)mx + p] = inv[0] - inv[1];
      wx[2LL * mx + p] = y3[0] - y3[1];
    } else {
      const int c = p - mx;
      Du[c] = D;
      wu[c] = dl[0] - dl[1];
      wu[n + c] = inv[0] - inv[1];
      wu[2 * n + c] = y3[0] - y3[1];
    }
  }
  {
    double r[5] = {nr3, nlz, szmax, szmin, gap};
    constexpr int op[5] = {kRedMax, kRedMax, kRedMax, kRedMin, kRedSum};
    block_multi256(r, op, sh5);
    nr3 = r[0];
    nlz = r[1];
    szmax = r[2];
    szmin = r[3];
    gap = r[4];
  }
  if (threadIdx.x == 0) {
    double* np = norm_part + 5LL * bid;
    np[0] = nr3;
    np[1] = nlz;
    np[2] = szmax;
    np[3] = szmin;
    np[4] = gap;
  }
}

__global__ __launch_bounds__(256) void prep_kernel(
    const double* __restrict__ d, const double* __restrict__ s, const double* __restrict__ lam,
    const double* __restrict__ z, const double* __restrict__ gv, const double* __restrict__ v,
    double* __restrict__ Dx, double* __restrict__ Du, double* __restrict__ wx,
    double* __restrict__ wu, double* __restrict__ norm_part, int mx, int n,
    const int* __restrict__ done) {
  prep_body(blockIdx.x, d, s, lam, z, gv, v, Dx, Du, wx, wu, norm_part, mx, n, done);
}

int launch_prep(Problem& p) {
  hipLaunchKernelGGL(prep_kernel, dim3(p.n_prep_blocks), dim3(256), 0, p.stream, p.d, p.s, p.lam,
                     p.z, p.gv, p.v, p.Dx, p.Du, p.wx, p.wu, p.norm_part, p.mx, p.n, &p.st->done);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// Termination test, barrier update and right-hand side of eqn. (cond_KKT):
//   r1 = H v + h + J' lambda,   E_0 = max(|r1|, |r3|, |lambda - z|, |s z|),
//   while E_mu <= kappa_eps mu: mu <- max(mu_min, min(kappa_mu mu, mu^theta_mu)),
//   rhs = -r1 + J' r2 - J' Sigma r3 = -(H v + h) - mu J' S^-1 1 - J' Sigma r3.
// fixed_mu != 0: no test and no update (used for a single step from a given iterate).
// gt_part != NULL: gt = Gamma' [wx] is first formed from the Gamma' pass's partials (each
// thread its own columns, in gamma_t_reduce_body's order) and stored, instead of read.
__device__ __forceinline__ void mu_rhs_body(int bid, 
    const double* __restrict__ Hv, const double* __restrict__ h, double* gt,
    const double* __restrict__ wu, const double* __restrict__ norm_part, int nparts,
    const double* __restrict__ v, double* __restrict__ rhs, int n, IpmState* st, int fixed_mu,
    const double* __restrict__ gt_part = nullptr, int ns = 0, int nu = 0) {
  if (st->done) return;
  // The barrier parameter of the previous iteration, read by every thread before the
  // exchange barrier below: thread 0 stores the new one at the end, and a wavefront reading
  // st->mu after the barrier could see it.
  const double mu_prev = st->mu;
  double nr1 = 0.0, f = 0.0;
  for (int c = threadIdx.x; c < n; c += 256) {
    if (gt_part != nullptr) {
      double g[3];
      gamma_t_column<3>(gt_part, c, ns, nu, g);
      gt[c] = g[0];
      gt[n + c] = g[1];
      gt[2 * n + c] = g[2];
    }
    const double r1 = Hv[c] + h[c] + (gt[c] + wu[c]);
    nr1 = fmax(nr1, fabs(r1));
    f += v[c] * (0.5 * Hv[c] + h[c]);
  }
  double nr3 = 0.0, nlz = 0.0, szmax = 0.0, szmin = INFINITY, gap = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 256) {
    nr3 = fmax(nr3, norm_part[5LL * b]);
    nlz = fmax(nlz, norm_part[5LL * b + 1]);
    szmax = fmax(szmax, norm_part[5LL * b + 2]);
    szmin = fmin(szmin, norm_part[5LL * b + 3]);
    gap += norm_part[5LL * b + 4];
  }
  // the seven workgroup reductions through one exchange of the wavefronts' results (the
  // same wavefront reductions and the same order of the four as block_*256)
  __shared__ double shr[7][4];
  {
    const double wr[7] = {wave_max(nr1), wave_sum(f),    wave_sum(gap),  wave_max(nr3),
                          wave_max(nlz), wave_max(szmax), wave_min(szmin)};
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int k = 0; k < 7; ++k) shr[k][w] = wr[k];
    }
  }
  __syncthreads();
  nr1 = fmax(fmax(shr[0][0], shr[0][1]), fmax(shr[0][2], shr[0][3]));
  f = (shr[1][0] + shr[1][1]) + (shr[1][2] + shr[1][3]);
  gap = (shr[2][0] + shr[2][1]) + (shr[2][2] + shr[2][3]);
  nr3 = fmax(fmax(shr[3][0], shr[3][1]), fmax(shr[3][2], shr[3][3]));
  nlz = fmax(fmax(shr[4][0], shr[4][1]), fmax(shr[4][2], shr[4][3]));
  szmax = fmax(fmax(shr[5][0], shr[5][1]), fmax(shr[5][2], shr[5][3]));
  szmin = fmin(fmin(shr[6][0], shr[6][1]), fmin(shr[6][2], shr[6][3]));
  __syncthreads();  // shr is written again by a workgroup's next item (batch lists)
  double mu = mu_prev;
  bool stop = false;
  if (!fixed_mu) {
    const double e0 = fmax(fmax(nr1, nr3), fmax(nlz, szmax));
    if (threadIdx.x == 0) {
      st->nr1 = nr1;
      st->nr3 = nr3;
      st->nlz = nlz;
      st->szmax = szmax;
      st->szmin = szmin;
      st->err0 = e0;
      st->obj = f + st->h0;
      st->gap = gap;
    }
    if (e0 <= st->tol) {
      if (threadIdx.x == 0) {
        st->status = CMPC_OK;
        st->done = 1;
        st->ref_skip = 1;  // no refinement work in iterations queued after the stop
      }
      stop = true;
    } else if (st->iter >= st->max_iter) {
      if (threadIdx.x == 0) {
        st->status = CMPC_MAX_ITER;
        st->done = 1;
        st->ref_skip = 1;
      }
      stop = true;
    } else {
      const double base = fmax(fmax(nr1, nr3), nlz);
      while (mu > st->mu_min) {
        const double emu = fmax(base, fmax(szmax - mu, mu - szmin));
        if (emu > kKappaEps * mu) break;
        mu = fmax(st->mu_min, fmin(kKappaMu * mu, pow(mu, kThetaMu)));
      }
    }
  }
  if (stop) return;
  for (int c = threadIdx.x; c < n; c += 256)
    rhs[c] = -(Hv[c] + h[c]) - mu * (gt[n + c] + wu[n + c]) - (gt[2 * n + c] + wu[2 * n + c]);
  if (threadIdx.x == 0 && !fixed_mu) {
    st->mu = mu;
    st->tau = fmax(kTauMin, 1.0 - mu);
    if (st->use_low && mu < st->mu_switch) st->use_low = 0;  // late iterations: FP64 SYRK
    if (st->mixed && !st->use_low && st->switch_iter < 0) st->switch_iter = st->iter;
    st->ref_skip = st->use_low ? 0 : 1;
    st->res_prev = INFINITY;
  }
}

__global__ __launch_bounds__(256) void mu_rhs_kernel(
    const double* __restrict__ Hv, const double* __restrict__ h, double* gt,
    const double* __restrict__ wu, const double* __restrict__ norm_part, int nparts,
    const double* __restrict__ v, double* __restrict__ rhs, int n, IpmState* st, int fixed_mu,
    const double* __restrict__ gt_part, int ns, int nu) {
  mu_rhs_body(blockIdx.x, Hv, h, gt, wu, norm_part, nparts, v, rhs, n, st, fixed_mu, gt_part, ns,
              nu);
}

// Gamma' [wx] partial sums (the first gt_chunks workgroups) and Hv = H v (the rest, 4 rows
// each) in one launch: the two are independent.
template <int NV>
__global__ __launch_bounds__(256) void gamma_t_hv_kernel(
    const double* __restrict__ Gt, const double* __restrict__ W, long long wstride,
    double* __restrict__ part, int ns, int nu, int N, int nchunks, const double* __restrict__ H,
    const double* __restrict__ x, double* __restrict__ y, int n, const int* __restrict__ done) {
  if ((int)blockIdx.x < nchunks)
    gamma_t_partial_body<NV>(blockIdx.x, Gt, W, wstride, part, ns, nu, N, done);
  else
    hv_body(blockIdx.x - nchunks, H, x, y, n, done);
}

int launch_mu_rhs(Problem& p) {
  const int* done = &p.st->done;
  hipLaunchKernelGGL(gamma_t_hv_kernel<3>, dim3(p.gt_chunks + ceil_div(p.n, 4)), dim3(256), 0,
                     p.stream, p.Gt, p.wx, (long long)p.mx, p.gt_part, p.ns, p.nu, p.N,
                     p.gt_chunks, p.H, p.v, p.Hv, p.n, done);
  CMPC_LAUNCH_CHECK();
  // the one-workgroup mu / rhs kernel adds the pass's partials itself (no reduction launch)
  hipLaunchKernelGGL(mu_rhs_kernel, dim3(1), dim3(256), 0, p.stream, p.Hv, p.h, p.gt, p.wu,
                     p.norm_part, p.n_prep_blocks, p.v, p.rhs, p.n, p.st, 0, p.gt_part, p.ns,
                     p.nu);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// ---------------------------------------------------------------- step recovery
// p_s = -r3 - J p_v;  p_lambda = -r2 + Sigma r3 + Sigma J p_v = -r2 - Sigma p_s;
// p_z = mu S^-1 1 - z - Sigma p_s;  per-block minima of the fraction-to-boundary ratios.
__device__ __forceinline__ void step_body(int bid, 
    const double* __restrict__ d, const double* __restrict__ s, const double* __restrict__ lam,
    const double* __restrict__ z, const double* __restrict__ gv, const double* __restrict__ v,
    const double* __restrict__ gpv, const double* __restrict__ pv, double* __restrict__ ps,
    double* __restrict__ plam, double* __restrict__ pz, double* __restrict__ alpha_part, int mx,
    int n, const IpmState* st) {
  __shared__ double sh2[2][4];
  if (st->done) return;
  const double mu = st->mu, tau = st->tau;
  const int p = bid * 256 + threadIdx.x;
  double amin = INFINITY, azmin = INFINITY;
  if (p < mx + n) {
    const PairRows pr = pair_rows(p, mx, n, gv, v);
    const double jp = p < mx ? gpv[p] : pv[p - mx];
    const long long rows[2] = {pr.up, pr.lo};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const long long r = rows[q];
      const double dr = d[r];
      double a = 0.0, b = 0.0, c = 0.0;
      if (!isinf(dr)) {
        const double sr = s[r], zr = z[r], lr = lam[r];
        const double jv = q == 0 ? pr.jv : -pr.jv;
        const double jpv = q == 0 ? jp : -jp;
        const double r3 = jv - dr + sr;
        const double sig = zr / sr;
        const double r2 = lr - mu / sr;
        a = -r3 - jpv;
        b = -r2 - sig * a;
        c = mu / sr - zr - sig * a;
        if (a < 0.0) amin = fmin(amin, -tau * sr / a);
        if (c < 0.0) azmin = fmin(azmin, -tau * zr / c);
      }
      ps[r] = a;
      plam[r] = b;
      pz[r] = c;
    }
  }
  {
    double r[2] = {amin, azmin};
    constexpr int op[2] = {kRedMin, kRedMin};
    block_multi256(r, op, sh2);
    amin = r[0];
    azmin = r[1];
  }
  if (threadIdx.x == 0) {
    alpha_part[2LL * bid] = amin;
    alpha_part[2LL * bid + 1] = azmin;
  }
}

__global__ __launch_bounds__(256) void step_kernel(
    const double* __restrict__ d, const double* __restrict__ s, const double* __restrict__ lam,
    const double* __restrict__ z, const double* __restrict__ gv, const double* __restrict__ v,
    const double* __restrict__ gpv, const double* __restrict__ pv, double* __restrict__ ps,
    double* __restrict__ plam, double* __restrict__ pz, double* __restrict__ alpha_part, int mx,
    int n, const IpmState* st) {
  step_body(blockIdx.x, d, s, lam, z, gv, v, gpv, pv, ps, plam, pz, alpha_part, mx, n, st);
}

int launch_step(Problem& p, int refine) {
  const int* done = &p.st->done;
  // the factorisation ran the forward substitution of rhs into tmpn (one-workgroup sizes)
  if (launch_potrs(p.stream, p.K, p.n, p.n, p.Wdiag, p.rhs, p.pv, p.tmpn, done,
                   p.eq_on ? p.eqs : nullptr, p.n <= kPotrsSingleMax ? p.tmpn : nullptr))
    return CMPC_ERR_HIP;
  for (int r = 0; r < refine; ++r)
    if (launch_refine_step(p)) return CMPC_ERR_HIP;
  if (launch_gamma_mv(p, p.pv, p.gpv, done)) return CMPC_ERR_HIP;
  hipLaunchKernelGGL(step_kernel, dim3(p.n_step_blocks), dim3(256), 0, p.stream, p.d, p.s, p.lam,
                     p.z, p.gv, p.v, p.gpv, p.pv, p.ps, p.plam, p.pz, p.alpha_part, p.mx, p.n,
                     p.st);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// ---------------------------------------------------------------- update
// Every workgroup reduces the step-length partials itself (min is order independent), then
// v += alpha p_v, s += alpha p_s, lambda += alpha p_lambda, z += alpha_z p_z, and z is
// safeguarded into [mu/(kappa s), kappa mu/s].  apply == 0 only records alpha, alpha_z.
// Returns whether the step was applied (the same in every workgroup: each reduces all partials).
__device__ __forceinline__ bool update_body(int bid, 
    const double* __restrict__ d, double* __restrict__ s, double* __restrict__ lam,
    double* __restrict__ z, double* __restrict__ gv, double* __restrict__ v,
    const double* __restrict__ gpv, const double* __restrict__ pv, const double* __restrict__ ps,
    const double* __restrict__ plam, const double* __restrict__ pz,
    const double* __restrict__ alpha_part, int nparts, int mx, int n, IpmState* st, int apply) {
  __shared__ double sh2[2][4];
  __shared__ int sdone;
  // done is read once per workgroup: workgroup 0 sets it during this launch on a small step,
  // and every wavefront of a workgroup must take the same path through the barriers below.
  if (threadIdx.x == 0) sdone = st->done;
  __syncthreads();
  const bool stopped = sdone != 0;
  __syncthreads();
  if (stopped) return false;
  double amin = 1.0, azmin = 1.0;
  for (int b = threadIdx.x; b < nparts; b += 256) {
    amin = fmin(amin, alpha_part[2LL * b]);
    azmin = fmin(azmin, alpha_part[2LL * b + 1]);
  }
  double r[2] = {amin, azmin};
  constexpr int op[2] = {kRedMin, kRedMin};
  block_multi256(r, op, sh2);
  const double alpha = r[0], alpha_z = r[1];
  const double mu = st->mu;
  if (bid == 0 && threadIdx.x == 0) {
    st->alpha = alpha;
    st->alpha_z = alpha_z;
  }
  if (!apply) return false;
  if (alpha < kAlphaMin) {
    if (bid == 0 && threadIdx.x == 0) {
      st->status = CMPC_SMALL_STEP;
      st->done = 1;
    }
    return false;
  }
  const int p = bid * 256 + threadIdx.x;
  if (p < mx + n) {
    long long rows[2];
    if (p < mx) {
      rows[0] = p;
      rows[1] = (long long)mx + p;
      gv[p] += alpha * gpv[p];
    } else {
      const int c = p - mx;
      rows[0] = 2LL * mx + c;
      rows[1] = 2LL * mx + n + c;
      v[c] += alpha * pv[c];
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const long long r = rows[q];
      if (isinf(d[r])) continue;
      const double sn = s[r] + alpha * ps[r];
      const double ln = lam[r] + alpha * plam[r];
      double zn = z[r] + alpha_z * pz[r];
      zn = fmin(fmax(zn, mu / (kKappaSigma * sn)), kKappaSigma * mu / sn);
      s[r] = sn;
      lam[r] = ln;
      z[r] = zn;
    }
  }
  if (bid == 0 && threadIdx.x == 0) st->iter += 1;
  return true;
}

__global__ __launch_bounds__(256) void update_kernel(
    const double* __restrict__ d, double* __restrict__ s, double* __restrict__ lam,
    double* __restrict__ z, double* __restrict__ gv, double* __restrict__ v,
    const double* __restrict__ gpv, const double* __restrict__ pv, const double* __restrict__ ps,
    const double* __restrict__ plam, const double* __restrict__ pz,
    const double* __restrict__ alpha_part, int nparts, int mx, int n, IpmState* st, int apply) {
  update_body(blockIdx.x, d, s, lam, z, gv, v, gpv, pv, ps, plam, pz, alpha_part, nparts, mx, n, st, apply);
}

// End-of-iteration flag for the host: 1 = still running, 2 = done, written with a
// system-scope release into mapped pinned memory (the host polls it; no copy, no event).
__global__ void publish_kernel(IpmState* st, int* flag, IterLog* log) {
  const int d = st->done;
  if (log != nullptr) {  // ordered before the flag by the release store
    IterLog e;
    e.iter = st->iter;
    e.level = st->use_low;
    e.done = d;
    e.pad = st->status;
    e.mu = st->mu;
    e.err0 = st->err0;
    e.nr1 = st->nr1;
    e.nr3 = st->nr3;
    e.nlz = st->nlz;
    e.szmax = st->szmax;
    e.alpha = st->alpha;
    e.alpha_z = st->alpha_z;
    *log = e;
  }
  if (d == 2) st->done = 0;  // the iteration was skipped for a retry one level up
  const int v = d == 1 ? 2 : 1;
  __hip_atomic_store(flag, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The update followed, in the same threads, by the next iteration's prep: both map thread p to
// the pair of rows p (n_step_blocks == n_prep_blocks), so each thread re-reads only what it has
// just written.  Runs only where the step was applied; a skipped or final iteration leaves the
// previous prep outputs, which still describe the unchanged iterate.
__global__ __launch_bounds__(256) void update_prep_kernel(
    const double* __restrict__ d, double* __restrict__ s, double* __restrict__ lam,
    double* __restrict__ z, double* __restrict__ gv, double* __restrict__ v,
    const double* __restrict__ gpv, const double* __restrict__ pv, const double* __restrict__ ps,
    const double* __restrict__ plam, const double* __restrict__ pz,
    const double* __restrict__ alpha_part, int nparts, int mx, int n, IpmState* st,
    double* __restrict__ Dx, double* __restrict__ Du, double* __restrict__ wx,
    double* __restrict__ wu, double* __restrict__ norm_part) {
  if (update_body(blockIdx.x, d, s, lam, z, gv, v, gpv, pv, ps, plam, pz, alpha_part, nparts, mx,
                  n, st, 1))
    prep_body(blockIdx.x, d, s, lam, z, gv, v, Dx, Du, wx, wu, norm_part, mx, n, &st->done);
}

// The update (with the next iteration's prep) and the host flag of ring slot `slot` (two
// launches: the flag needs every workgroup of the update finished, which a last-workgroup tail
// could only see through a device-scope fence per workgroup, an L2 write-back each, measured
// slower).  The first iteration's prep is launched by the caller.
int launch_update_publish(Problem& p, int slot) {
  hipLaunchKernelGGL(update_prep_kernel, dim3(p.n_step_blocks), dim3(256), 0, p.stream, p.d,
                     p.s, p.lam, p.z, p.gv, p.v, p.gpv, p.pv, p.ps, p.plam, p.pz, p.alpha_part,
                     p.n_step_blocks, p.mx, p.n, p.st, p.Dx, p.Du, p.wx, p.wu, p.norm_part);
  CMPC_LAUNCH_CHECK();
  hipLaunchKernelGGL(publish_kernel, dim3(1), dim3(1), 0, p.stream, p.st, p.dflags + slot,
                     p.dlog != nullptr ? p.dlog + slot : nullptr);
  CMPC_LAUNCH_CHECK();
  return 0;
}


// ---------------------------------------------------------------- sigma folding (testing)
__global__ void sigma_fold_kernel(const double* __restrict__ sigma, const double* __restrict__ xl,
                                  const double* __restrict__ xu, const double* __restrict__ ul,
                                  const double* __restrict__ uu, double* __restrict__ Dx,
                                  double* __restrict__ Du, int ns, int nu, int mx, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < mx) {
    const int i = p % ns;
    Dx[p] = (isinf(xu[i]) ? 0.0 : sigma[p]) + (isinf(xl[i]) ? 0.0 : sigma[(long long)mx + p]);
  } else if (p < mx + n) {
    const int c = p - mx, k = c % nu;
    Du[c] = (isinf(uu[k]) ? 0.0 : sigma[2LL * mx + c]) +
            (isinf(ul[k]) ? 0.0 : sigma[2LL * mx + n + c]);
  }
}

int launch_sigma_fold(Problem& p, const double* sigma) {
  hipLaunchKernelGGL(sigma_fold_kernel, dim3(ceil_div((long long)p.mx + p.n, 256)), dim3(256), 0,
                     p.stream, sigma, p.xl, p.xu, p.ul, p.uu, p.Dx, p.Du, p.ns, p.nu, p.mx, p.n);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// ---------------------------------------------------------------- iterative refinement
// Mixed modes: p_v solved with the factor of the low-precision K is corrected against the
// exact FP64 operator  K p = H p + Gamma'(D_x o Gamma p) + D_u o p:
//   res = rhs - K p;  stop when |res| <= 1e-12 |rhs|;  else p += (L L')^-1 res.
// A step that does not shrink |res| by 10x counts as not contracting; after two the SYRK
// moves one precision level up (BF16 -> FP32 -> FP64) from the next iteration on.  Every kernel is gated by st->ref_skip.
__device__ __forceinline__ void axpy_gated_body(int bid, double* __restrict__ y, const double* __restrict__ x, int len,
                                  const int* __restrict__ skip) {
  if (*skip) return;
  const int i = bid * blockDim.x + threadIdx.x;
  if (i < len) y[i] += x[i];
}

__global__ void axpy_gated_kernel(double* __restrict__ y, const double* __restrict__ x, int len,
                                  const int* __restrict__ skip) {
  axpy_gated_body(blockIdx.x, y, x, len, skip);
}

// gt_part != NULL: Gamma'(D_x o Gamma p) is added up here from the Gamma' pass's partials (the
// order of gamma_t_reduce), instead of being read from gtp.
// Gamma'(D_x o Gamma p) enters as the Gamma' pass's per-chunk partials, added up here.
__device__ __forceinline__ void refine_check_body(int bid, 
    const double* __restrict__ rhs, const double* __restrict__ Hp,
    const double* __restrict__ Du, const double* __restrict__ p, double* __restrict__ res, int n,
    IpmState* st, const double* __restrict__ gt_part, int ns, int nu) {
  __shared__ double sh2[2][4];
  if (st->ref_skip || st->done) return;
  double nr = 0.0, nb = 0.0;
  for (int c = threadIdx.x; c < n; c += 256) {
    double g[1];
    gamma_t_column<1>(gt_part, c, ns, nu, g);
    const double r = rhs[c] - (Hp[c] + g[0] + Du[c] * p[c]);
    res[c] = r;
    nr = fmax(nr, fabs(r));
    nb = fmax(nb, fabs(rhs[c]));
  }
  {
    double r[2] = {nr, nb};
    constexpr int op[2] = {kRedMax, kRedMax};
    block_multi256(r, op, sh2);
    nr = r[0];
    nb = r[1];
  }
  if (threadIdx.x == 0) {
    if (nr <= 1e-12 * nb) {
      st->ref_skip = 1;
    } else {
      if (nr > st->contract * st->res_prev) {
        st->nonc += 1;
        if (st->nonc >= 2 && st->use_low > 0) {  // next iteration one precision level up
          st->use_low -= 1;
          st->nonc = 0;
        }
      }
      st->res_prev = nr;
      st->refine_steps += 1;
    }
  }
}

__global__ __launch_bounds__(256) void refine_check_kernel(
    const double* __restrict__ rhs, const double* __restrict__ Hp,
    const double* __restrict__ Du, const double* __restrict__ p, double* __restrict__ res, int n,
    IpmState* st, const double* __restrict__ gt_part, int ns, int nu) {
  refine_check_body(blockIdx.x, rhs, Hp, Du, p, res, n, st, gt_part, ns, nu);
}

// One refinement step in four launches (the batch form's five carry the same arithmetic):
// D_x o Gamma p (the scaling fused into the Gamma pass); the Gamma' pass's partials beside
// H p; the residual with the partials added up in the check; p += (L L')^-1 res in the solve.
int launch_refine_step(Problem& p) {
  const int* skip = &p.st->ref_skip;
  if (launch_gamma_mv(p, p.pv, p.gpv, skip, p.Dx)) return CMPC_ERR_HIP;
  hipLaunchKernelGGL(gamma_t_hv_kernel<1>, dim3(p.gt_chunks + ceil_div(p.n, 4)), dim3(256), 0,
                     p.stream, p.Gt, p.gpv, (long long)p.mx, p.gt_part, p.ns, p.nu, p.N,
                     p.gt_chunks, p.H, p.pv, p.Hv, p.n, skip);
  CMPC_LAUNCH_CHECK();
  hipLaunchKernelGGL(refine_check_kernel, dim3(1), dim3(256), 0, p.stream, p.rhs, p.Hv,
                     p.Du, p.pv, p.ref_res, p.n, p.st, p.gt_part, p.ns, p.nu);
  CMPC_LAUNCH_CHECK();
  if (p.n <= kPotrsSingleMax)  // pv += the correction, in the solve's own store
    return launch_potrs(p.stream, p.K, p.n, p.n, p.Wdiag, p.ref_res, p.pv, p.tmpn, skip,
                        p.eq_on ? p.eqs : nullptr, nullptr, 1);
  if (launch_potrs(p.stream, p.K, p.n, p.n, p.Wdiag, p.ref_res, p.ref_dlt, p.tmpn, skip,
                   p.eq_on ? p.eqs : nullptr))
    return CMPC_ERR_HIP;
  hipLaunchKernelGGL(axpy_gated_kernel, dim3(ceil_div(p.n, 256)), dim3(256), 0, p.stream, p.pv,
                     p.ref_dlt, p.n, skip);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// ---------------------------------------------------------------- one step from an iterate
__global__ void set_step_state_kernel(IpmState* st, double mu, double tau) {
  st->mu = mu;
  st->tau = tau;
  st->done = 0;
  st->status = kRunning;
  st->info = 0;
}

int launch_step_given(Problem& p, const double* v, const double* s, const double* lam,
                      const double* z, double mu, double tau) {
  const size_t m = p.m;
  p.eq_on = false;  // plain FP64 step
  CMPC_HIP(hipMemcpyAsync(p.v, v, sizeof(double) * p.n, hipMemcpyDeviceToDevice, p.stream));
  CMPC_HIP(hipMemcpyAsync(p.s, s, sizeof(double) * m, hipMemcpyDeviceToDevice, p.stream));
  CMPC_HIP(hipMemcpyAsync(p.lam, lam, sizeof(double) * m, hipMemcpyDeviceToDevice, p.stream));
  CMPC_HIP(hipMemcpyAsync(p.z, z, sizeof(double) * m, hipMemcpyDeviceToDevice, p.stream));
  hipLaunchKernelGGL(set_step_state_kernel, dim3(1), dim3(1), 0, p.stream, p.st, mu, tau);
  CMPC_LAUNCH_CHECK();
  const int* done = &p.st->done;
  if (launch_gamma_mv(p, p.v, p.gv, done)) return CMPC_ERR_HIP;
  if (launch_prep(p)) return CMPC_ERR_HIP;
  if (launch_gamma_t(p, p.wx, 3, p.gt, done)) return CMPC_ERR_HIP;
  if (launch_hv(p, p.v, p.Hv, done)) return CMPC_ERR_HIP;
  hipLaunchKernelGGL(mu_rhs_kernel, dim3(1), dim3(256), 0, p.stream, p.Hv, p.h, p.gt, p.wu,
                     p.norm_part, p.n_prep_blocks, p.v, p.rhs, p.n, p.st, 1,
                     (const double*)nullptr, 0, 0);
  CMPC_LAUNCH_CHECK();
  if (launch_syrk(p, CMPC_FP64, p.Dx, p.H, p.Du, p.K)) return CMPC_ERR_HIP;
  if (launch_potrf(p.stream, p.K, p.n, p.n, p.Wdiag, &p.st->done, &p.st->info, &p.st->status,
                   nullptr, nullptr, nullptr, p.rhs, nullptr, p.tmpn))
    return CMPC_ERR_HIP;
  if (launch_step(p, 0)) return CMPC_ERR_HIP;
  hipLaunchKernelGGL(update_kernel, dim3(1), dim3(256), 0, p.stream, p.d, p.s, p.lam, p.z, p.gv,
                     p.v, p.gpv, p.pv, p.ps, p.plam, p.pz, p.alpha_part, p.n_step_blocks, p.mx,
                     p.n, p.st, 0);
  CMPC_LAUNCH_CHECK();
  return 0;
}


// ================================================================ work-list (batched) forms
// Each kernel walks a list of (instance, block) items; the per-item work is the body of the
// single-instance kernel above with the same block decomposition, so every instance of a
// batch computes bit for bit what it computes alone.  Workgroups loop over the list with
// stride gridDim.x (persistent when the grid is smaller than the list); the barrier at the
// top of the loop separates the LDS use of consecutive items.  Items of a finished instance
// return at entry (their st->done is set).


__global__ __launch_bounds__(256) void ipm_init_batch_kernel(const InstView* __restrict__ views,
                                                             const WorkItem* __restrict__ items,
                                                             int nitems, double tol, int max_iter,
                                                             int low, double mu_switch,
                                                             double contract, int warm,
                                                             double mu0) {
  CMPC_ITEMS_BEGIN
  ipm_init_body(bid, V.d, V.s, V.lam, V.z, V.v, V.gv, V.m, V.n, V.mx, V.st, tol, max_iter, low,
                mu_switch, contract, warm, mu0);
  CMPC_ITEMS_END
}

__global__ __launch_bounds__(256) void prep_batch_kernel(const InstView* __restrict__ views,
                                                         const WorkItem* __restrict__ items,
                                                         int nitems) {
  CMPC_ITEMS_BEGIN
  prep_body(bid, V.d, V.s, V.lam, V.z, V.gv, V.v, V.Dx, V.Du, V.wx, V.wu, V.norm_part, V.mx, V.n,
            &V.st->done);
  CMPC_ITEMS_END
}

// which = 0: Gamma' [wx] (3 vectors) -> partials under st->done; which = 1: Gamma' gpv ->
// partials under st->ref_skip (added up in the refinement check).
template <int NV>
__global__ __launch_bounds__(256) void gamma_t_partial_batch_kernel(
    const InstView* __restrict__ views, const WorkItem* __restrict__ items, int nitems) {
  CMPC_ITEMS_BEGIN
  gamma_t_partial_body<NV>(bid, V.Gt, NV == 3 ? V.wx : V.gpv, (long long)V.mx, V.gt_part,
                           V.ns, V.nu, V.N, gate_of(V, NV == 3 ? 0 : 1));
  CMPC_ITEMS_END
}

// gate 0: Hv = H v; gate 1: Hv = H pv (refinement)
__global__ __launch_bounds__(256) void hv_batch_kernel(const InstView* __restrict__ views,
                                                       const WorkItem* __restrict__ items,
                                                       int nitems, int gate) {
  CMPC_ITEMS_BEGIN
  hv_body(bid, V.H, gate ? V.pv : V.v, V.Hv, V.n, gate_of(V, gate));
  CMPC_ITEMS_END
}

__global__ __launch_bounds__(256) void mu_rhs_batch_kernel(const InstView* __restrict__ views,
                                                           const WorkItem* __restrict__ items,
                                                           int nitems) {
  CMPC_ITEMS_BEGIN
  mu_rhs_body(bid, V.Hv, V.h, V.gt, V.wu, V.norm_part, V.nblk, V.v, V.rhs, V.n, V.st, 0,
              V.gt_part, V.ns, V.nu);
  CMPC_ITEMS_END
}

// gpv = Gamma pv (gate 0: the step; gate 1: the refinement product); gate 2: gv = Gamma v
// for every instance (the warm start, before the start point is formed)
__global__ __launch_bounds__(256) void gamma_mv_batch_kernel(const InstView* __restrict__ views,
                                                             const WorkItem* __restrict__ items,
                                                             int nitems, int gate) {
  CMPC_ITEMS_BEGIN
  if (gate == 2)
    gamma_mv_body<kMvTBatch>(bid, V.Gt, V.v, V.gv, V.ns, V.nu, V.N, nullptr);
  else  // the refinement's pass (gate 1) is scaled by D_x, as in the single-instance step
    gamma_mv_body<kMvTBatch>(bid, V.Gt, V.pv, V.gpv, V.ns, V.nu, V.N, gate_of(V, gate),
                  gate == 1 ? V.Dx : nullptr);
  CMPC_ITEMS_END
}

__global__ __launch_bounds__(256) void step_batch_kernel(const InstView* __restrict__ views,
                                                         const WorkItem* __restrict__ items,
                                                         int nitems) {
  CMPC_ITEMS_BEGIN
  step_body(bid, V.d, V.s, V.lam, V.z, V.gv, V.v, V.gpv, V.pv, V.ps, V.plam, V.pz, V.alpha_part,
            V.mx, V.n, V.st);
  CMPC_ITEMS_END
}

// The update, then (where it was applied) the next iteration's prep of the same pairs, as in
// update_prep_kernel; the items are the 256-pair blocks of both.
__global__ __launch_bounds__(256) void update_batch_kernel(const InstView* __restrict__ views,
                                                           const WorkItem* __restrict__ items,
                                                           int nitems) {
  CMPC_ITEMS_BEGIN
  if (update_body(bid, V.d, V.s, V.lam, V.z, V.gv, V.v, V.gpv, V.pv, V.ps, V.plam, V.pz,
                  V.alpha_part, V.nblk, V.mx, V.n, V.st, 1))
    prep_body(bid, V.d, V.s, V.lam, V.z, V.gv, V.v, V.Dx, V.Du, V.wx, V.wu, V.norm_part, V.mx,
              V.n, &V.st->done);
  CMPC_ITEMS_END
}

__global__ __launch_bounds__(256) void refine_check_batch_kernel(
    const InstView* __restrict__ views, const WorkItem* __restrict__ items, int nitems) {
  CMPC_ITEMS_BEGIN
  refine_check_body(bid, V.rhs, V.Hv, V.Du, V.pv, V.ref_res, V.n, V.st, V.gt_part,
                    V.ns, V.nu);
  CMPC_ITEMS_END
}

// refinement: pv += ref_dlt (items over 256-entry blocks of n)
__global__ __launch_bounds__(256) void axpy_batch_kernel(const InstView* __restrict__ views,
                                                         const WorkItem* __restrict__ items,
                                                         int nitems) {
  CMPC_ITEMS_BEGIN
  axpy_gated_body(bid, V.pv, V.ref_dlt, V.n, &V.st->ref_skip);
  CMPC_ITEMS_END
}

// End of a batch iteration: instances whose low-precision Cholesky failed (done = 2) are
// re-armed, the running ones are counted, and count + 1 is stored with a system-scope
// release into slot (iteration % ring) of the host-mapped ring.  One workgroup.
__global__ __launch_bounds__(256) void publish_batch_kernel(const InstView* __restrict__ views,
                                                            int count, int* __restrict__ iter,
                                                            int* __restrict__ flags, int ring) {
  __shared__ double sh[4];
  double running = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) {
    IpmState* st = views[i].st;
    int d = st->done;
    if (d == 2) {
      st->done = 0;
      d = 0;
    }
    running += d == 0 ? 1.0 : 0.0;
  }
  running = block_sum256(running, sh);
  if (threadIdx.x == 0) {
    const int k = *iter;
    *iter = k + 1;
    __hip_atomic_store(flags + (k % ring), (int)running + 1, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ void batch_reset_kernel(int* iter) { *iter = 0; }

// Gather the per-instance states into one array (one device-to-host copy at the end).
__global__ void gather_state_kernel(const InstView* __restrict__ views, int count,
                                    IpmState* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = *views[i].st;
}

int launch_b_init(const ListArg& L, double tol, int max_iter, int low, double mu_switch,
                  double contract, int warm, double mu0) {
  CMPC_LAUNCH_LIST(ipm_init_batch_kernel, L, tol, max_iter, low, mu_switch, contract, warm,
                   warm ? mu0 : kMuInit);
}
int launch_b_prep(const ListArg& L) { CMPC_LAUNCH_LIST(prep_batch_kernel, L); }
int launch_b_gamma_t_partial(const ListArg& L, int nv) {
  if (nv == 3) CMPC_LAUNCH_LIST(gamma_t_partial_batch_kernel<3>, L);
  CMPC_LAUNCH_LIST(gamma_t_partial_batch_kernel<1>, L);
}
int launch_b_hv(const ListArg& L, int gate) { CMPC_LAUNCH_LIST(hv_batch_kernel, L, gate); }
int launch_b_mu_rhs(const ListArg& L) { CMPC_LAUNCH_LIST(mu_rhs_batch_kernel, L); }
int launch_b_gamma_mv(const ListArg& L, int gate) {
  CMPC_LAUNCH_LIST(gamma_mv_batch_kernel, L, gate);
}
int launch_b_step(const ListArg& L) { CMPC_LAUNCH_LIST(step_batch_kernel, L); }
int launch_b_update(const ListArg& L) { CMPC_LAUNCH_LIST(update_batch_kernel, L); }
int launch_b_refine_check(const ListArg& L) { CMPC_LAUNCH_LIST(refine_check_batch_kernel, L); }
int launch_b_axpy(const ListArg& L) { CMPC_LAUNCH_LIST(axpy_batch_kernel, L); }

int launch_b_publish(hipStream_t s, const InstView* views, int count, int* iter, int* flags,
                     int ring) {
  hipLaunchKernelGGL(publish_batch_kernel, dim3(1), dim3(256), 0, s, views, count, iter, flags,
                     ring);
  CMPC_LAUNCH_CHECK();
  return 0;
}
int launch_b_reset(hipStream_t s, int* iter) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, s, iter);
  CMPC_LAUNCH_CHECK();
  return 0;
}
int launch_b_gather(hipStream_t s, const InstView* views, int count, IpmState* out) {
  hipLaunchKernelGGL(gather_state_kernel, dim3(ceil_div(count, 64)), dim3(64), 0, s, views, count,
                     out);
  CMPC_LAUNCH_CHECK();
  return 0;
}

}  // namespace cmpc
