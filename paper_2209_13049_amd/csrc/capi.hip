// C ABI (include/condmpc.h) and the host-side interior-point driver (Algorithm 1).
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "problem.hpp"

namespace cmpc {

static thread_local std::string g_error;
void set_error(const std::string& msg) { g_error = msg; }

int launch_convert_gamma(Problem& p, int precision);

// ---- the scratch of cmpc_potrf_noalloc: the tile inverses W_k of the factorisation and
// their condition figures (4104 doubles per 64-column block) and three status flags, in one
// file-scope device array of fixed size.  Host code never passes the array's name to a kernel or a copy: it is a
// host-side stand-in, not a device address.  Each device's copy is looked up once with
// hipGetSymbolAddress (that device current) and that address is used from then on.
constexpr size_t kNoAllocWallDoubles = (4096 + 8) * (size_t)((CMPC_POTRF_NOALLOC_MAX_N + 63) / 64);
static __device__ __align__(256) double scratch[kNoAllocWallDoubles + 8];

namespace {
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;  // device ordinal -> address of that device's scratch
}  // namespace

__global__ void zero_ints_kernel(int* __restrict__ p, int count) {
  if ((int)threadIdx.x < count) p[threadIdx.x] = 0;
}

// Address of the scratch array on the device that runs `s` (set up once per device).
static int potrf_scratch(hipStream_t s, double** out) {
  int dev = 0;
  if (s != nullptr) {
    if (hipStreamGetDevice(s, &dev) != hipSuccess) {
      set_error("cmpc_potrf_noalloc: cannot tell the stream's device");
      return CMPC_ERR_HIP;
    }
  } else if (hipGetDevice(&dev) != hipSuccess) {
    set_error("cmpc_potrf_noalloc: no current device");
    return CMPC_ERR_HIP;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return 0;
  }
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || (cur != dev && hipSetDevice(dev) != hipSuccess)) {
    set_error("cmpc_potrf_noalloc: cannot make the stream's device current");
    return CMPC_ERR_HIP;
  }
  double* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (cur != dev) hipSetDevice(cur);
  if (e != hipSuccess || ptr == nullptr) {
    set_error(std::string("cmpc_potrf_noalloc: hipGetSymbolAddress failed: ") +
              hipGetErrorString(e));
    return CMPC_ERR_HIP;
  }
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return 0;
}

__global__ void add_vec_kernel(const double* __restrict__ a, const double* __restrict__ b,
                               double* __restrict__ out, int len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) out[i] = a[i] + b[i];
}

void free_problem(Problem* p) {
  if (!p) return;
  if (p->stream) hipStreamSynchronize(p->stream);
  else hipDeviceSynchronize();
  double** bufs[] = {&p->A,  &p->B,   &p->Q,    &p->Qf,    &p->R,    &p->xl,   &p->xu,
                     &p->ul, &p->uu,  &p->qdiag, &p->G,    &p->Gt,   &p->H,    &p->K,
                     &p->x0, &p->c,   &p->qc,   &p->h,     &p->d,    &p->v,    &p->s,
                     &p->lam, &p->z,  &p->gv,   &p->pv,    &p->ps,   &p->plam, &p->pz,
                     &p->gpv, &p->rhs, &p->Dx,  &p->Du,    &p->wx,   &p->wu,   &p->gt,
                     &p->Hv, &p->tmpn, &p->tmpn2, &p->tmpmx, &p->norm_part, &p->alpha_part,
                     &p->gt_part, &p->Wdiag, &p->ref_res, &p->ref_dlt, &p->eqs};
  for (double** b : bufs) {
    if (*b) hipFree(*b);
    *b = nullptr;
  }
  if (p->a_rowptr) hipFree(p->a_rowptr);
  if (p->a_col) hipFree(p->a_col);
  if (p->a_val) hipFree(p->a_val);
  if (p->red_part) hipFree(p->red_part);
  if (p->Sx) hipFree(p->Sx);
  if (p->wdist) hipFree(p->wdist);
  if (p->G32) hipFree(p->G32);
  if (p->G16) hipFree(p->G16);
  if (p->st) hipFree(p->st);
  for (hipEvent_t e : p->prof_ev) hipEventDestroy(e);
  if (p->hflags) hipHostFree(p->hflags);
  if (p->hlog) hipHostFree(p->hlog);
  if (p->ev0) hipEventDestroy(p->ev0);
  if (p->ev1) hipEventDestroy(p->ev1);
  syrk_free(p->syrk);
  delete p;
}

static bool all_finite(const double* a, size_t len) {
  for (size_t i = 0; i < len; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

static int upload(double** dst, const double* src, size_t len, hipStream_t s) {
  CMPC_HIP(hipMalloc(dst, sizeof(double) * std::max<size_t>(1, len)));
  CMPC_HIP(hipMemcpyAsync(*dst, src, sizeof(double) * len, hipMemcpyHostToDevice, s));
  return 0;
}

static int create_standard(const cmpc_lq_desc* desc, hipStream_t stream, Problem** out) {
  if (!desc || !out) {
    set_error("NULL argument");
    return CMPC_ERR_INVALID;
  }
  *out = nullptr;
  const int ns = desc->ns, nu = desc->nu, N = desc->N;
  if (ns <= 0 || nu <= 0 || N <= 0) {
    set_error("ns, nu and N must be positive");
    return CMPC_ERR_INVALID;
  }
  if ((long long)nu * N > 8192) {
    set_error("nu * N > 8192 is not supported");
    return CMPC_ERR_INVALID;
  }
  if (!desc->A || !desc->B || !desc->Q || !desc->R || !desc->xl || !desc->xu || !desc->ul ||
      !desc->uu) {
    set_error("NULL problem data");
    return CMPC_ERR_INVALID;
  }
  const double* Qf = desc->Qf ? desc->Qf : desc->Q;
  if (!all_finite(desc->A, (size_t)ns * ns) || !all_finite(desc->B, (size_t)ns * nu) ||
      !all_finite(desc->Q, (size_t)ns * ns) || !all_finite(Qf, (size_t)ns * ns) ||
      !all_finite(desc->R, (size_t)nu * nu)) {
    set_error("non-finite entry in A, B, Q, Q_f or R");
    return CMPC_ERR_NONFINITE;
  }
  for (int i = 0; i < ns; ++i)
    if (std::isnan(desc->xl[i]) || std::isnan(desc->xu[i]) || desc->xl[i] > desc->xu[i] ||
        desc->xu[i] == -INFINITY || desc->xl[i] == INFINITY) {
      set_error("invalid state bounds");
      return std::isnan(desc->xl[i]) || std::isnan(desc->xu[i]) ? CMPC_ERR_NONFINITE
                                                                 : CMPC_ERR_INVALID;
    }
  for (int k = 0; k < nu; ++k)
    if (std::isnan(desc->ul[k]) || std::isnan(desc->uu[k]) || desc->ul[k] >= desc->uu[k] ||
        desc->uu[k] == -INFINITY || desc->ul[k] == INFINITY) {
      set_error("invalid control bounds (need ul < uu)");
      return std::isnan(desc->ul[k]) || std::isnan(desc->uu[k]) ? CMPC_ERR_NONFINITE
                                                                 : CMPC_ERR_INVALID;
    }
  {  // R symmetric positive definite (host Cholesky, nu is small)
    std::vector<double> L(desc->R, desc->R + (size_t)nu * nu);
    for (int i = 0; i < nu; ++i)
      for (int j = 0; j < i; ++j)
        if (std::fabs(L[i * nu + j] - L[j * nu + i]) >
            1e-12 * (std::fabs(L[i * nu + j]) + std::fabs(L[j * nu + i]) + 1e-300)) {
          set_error("R is not symmetric");
          return CMPC_ERR_INVALID;
        }
    for (int j = 0; j < nu; ++j) {
      double dj = L[j * nu + j];
      for (int k = 0; k < j; ++k) dj -= L[j * nu + k] * L[j * nu + k];
      if (!(dj > 0)) {
        set_error("R is not positive definite");
        return CMPC_ERR_INVALID;
      }
      dj = std::sqrt(dj);
      L[j * nu + j] = dj;
      for (int i = j + 1; i < nu; ++i) {
        double v = L[i * nu + j];
        for (int k = 0; k < j; ++k) v -= L[i * nu + k] * L[j * nu + k];
        L[i * nu + j] = v / dj;
      }
    }
  }
  Problem* p = new Problem();
  p->ns = ns;
  p->ns_real = ns;
  p->nu = nu;
  p->N = N;
  p->n = nu * N;
  p->mx = ns * N;
  p->m = 2 * p->mx + 2 * p->n;
  p->stream = stream;
  int rc = 0;
#define TRY(x)              \
  do {                      \
    rc = (x);               \
    if (rc) {               \
      free_problem(p);      \
      return rc;            \
    }                       \
  } while (0)
  TRY(upload(&p->A, desc->A, (size_t)ns * ns, stream));
  TRY(upload(&p->B, desc->B, (size_t)ns * nu, stream));
  TRY(upload(&p->Q, desc->Q, (size_t)ns * ns, stream));
  TRY(upload(&p->Qf, Qf, (size_t)ns * ns, stream));
  TRY(upload(&p->R, desc->R, (size_t)nu * nu, stream));
  TRY(upload(&p->xl, desc->xl, ns, stream));
  TRY(upload(&p->xu, desc->xu, ns, stream));
  TRY(upload(&p->ul, desc->ul, nu, stream));
  TRY(upload(&p->uu, desc->uu, nu, stream));
  {  // sparse copy of A for the free response, when A is sparse enough
    std::vector<int> rowptr(ns + 1, 0), col;
    std::vector<double> val;
    for (int i = 0; i < ns; ++i) {
      for (int j = 0; j < ns; ++j) {
        const double a = desc->A[(size_t)i * ns + j];
        if (a != 0.0) {
          col.push_back(j);
          val.push_back(a);
        }
      }
      rowptr[i + 1] = (int)col.size();
    }
    int maxnnz = 0;
    for (int i = 0; i < ns; ++i) maxnnz = std::max(maxnnz, rowptr[i + 1] - rowptr[i]);
    if ((double)col.size() <= 0.25 * (double)ns * ns && ns <= 4096 && !col.empty()) {
      p->a_maxnnz = maxnnz;
      if (hipMalloc(&p->a_rowptr, sizeof(int) * (ns + 1)) != hipSuccess ||
          hipMalloc(&p->a_col, sizeof(int) * col.size()) != hipSuccess) {
        free_problem(p);
        return CMPC_ERR_NOMEM;
      }
      TRY(upload(&p->a_val, val.data(), val.size(), stream));
      if (hipMemcpyAsync(p->a_rowptr, rowptr.data(), sizeof(int) * (ns + 1), hipMemcpyHostToDevice,
                         stream) != hipSuccess ||
          hipMemcpyAsync(p->a_col, col.data(), sizeof(int) * col.size(), hipMemcpyHostToDevice,
                         stream) != hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess) {
        free_problem(p);
        return CMPC_ERR_HIP;
      }
    }
  }
  bool qd = true;
  for (int i = 0; i < ns && qd; ++i)
    for (int j = 0; j < ns; ++j)
      if (i != j && (desc->Q[(size_t)i * ns + j] != 0.0 || Qf[(size_t)i * ns + j] != 0.0)) {
        qd = false;
        break;
      }
  p->q_diag = qd;
  std::vector<double> qdiag;
  if (qd) {
    qdiag.resize(p->mx);
    for (int t = 1; t <= N; ++t)
      for (int i = 0; i < ns; ++i)
        qdiag[(size_t)(t - 1) * ns + i] = (t == N ? Qf : desc->Q)[(size_t)i * ns + i];
    TRY(upload(&p->qdiag, qdiag.data(), p->mx, stream));
  }
  // G_k = A^k B (eqn. (x_def) with K = 0)
  if (hipMalloc(&p->G, sizeof(double) * (size_t)N * ns * nu) != hipSuccess) {
    set_error("out of device memory (G)");
    free_problem(p);
    return CMPC_ERR_NOMEM;
  }
  if (hipMemcpyAsync(p->G, p->B, sizeof(double) * ns * nu, hipMemcpyDeviceToDevice, stream) !=
      hipSuccess) {
    free_problem(p);
    return CMPC_ERR_HIP;
  }
  for (int k = 1; k < N; ++k)
    TRY(launch_gemm_f64(stream, ns, nu, ns, 1.0, p->A, ns, 1, p->G + (size_t)(k - 1) * ns * nu,
                        nu, 1, 0.0, p->G + (size_t)k * ns * nu, nu));
  if (hipMalloc(&p->Gt, sizeof(double) * (size_t)N * ns * nu) != hipSuccess) {
    set_error("out of device memory (Gt)");
    free_problem(p);
    return CMPC_ERR_NOMEM;
  }
  TRY(launch_transpose_g(*p));
  if ((long long)N * ns * nu * (long long)sizeof(double) >= (1LL << 32)) {
    // the SYRK addresses G with 32-bit byte offsets
    set_error("ns * nu * N too large (G must stay below 4 GiB)");
    free_problem(p);
    return CMPC_ERR_INVALID;
  }
  TRY(ipm_alloc_work(*p));
  if (hipMalloc(&p->H, sizeof(double) * (size_t)p->n * p->n) != hipSuccess ||
      hipMalloc(&p->K, sizeof(double) * (size_t)p->n * p->n) != hipSuccess) {
    set_error("out of device memory (H, K)");
    free_problem(p);
    return CMPC_ERR_NOMEM;
  }
  TRY(syrk_plan(*p));
  // H = Gamma' Qbar Gamma + Rbar
  TRY(launch_rbar(*p, p->H));
  if (qd) {
    TRY(launch_syrk(*p, CMPC_FP64, p->qdiag, p->H, nullptr, p->H));
  } else {
    // one row block Gamma_t of Gamma at a time: H += Gamma_t' (W Gamma_t)
    double *Y = nullptr, *Gb = nullptr;
    if (hipMalloc(&Y, sizeof(double) * (size_t)ns * p->n) != hipSuccess ||
        hipMalloc(&Gb, sizeof(double) * (size_t)ns * p->n) != hipSuccess) {
      if (Y) hipFree(Y);
      free_problem(p);
      return CMPC_ERR_NOMEM;
    }
    for (int t = 1; t <= N && rc == 0; ++t) {
      const int len = t * nu;
      const double* W = (t == N) ? p->Qf : p->Q;
      rc = launch_gamma_block(*p, t, Gb);
      if (!rc) rc = launch_gemm_f64(stream, ns, len, ns, 1.0, W, ns, 1, Gb, len, 1, 0.0, Y, len);
      if (!rc) rc = launch_gemm_f64(stream, len, len, ns, 1.0, Gb, 1, len, Y, len, 1, 1.0, p->H, p->n);
    }
    hipStreamSynchronize(stream);
    hipFree(Y);
    hipFree(Gb);
    if (rc) {
      free_problem(p);
      return rc;
    }
  }
  TRY(launch_mirror_lower(stream, p->H, p->n));
  if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess) {
    free_problem(p);
    return CMPC_ERR_HIP;
  }
  if (hipStreamSynchronize(stream) != hipSuccess) {
    set_error(std::string("problem build: ") + hipGetErrorString(hipGetLastError()));
    free_problem(p);
    return CMPC_ERR_HIP;
  }
#undef TRY
  *out = p;
  return 0;
}

// ---- general data of eqn. (sparse) (cross weight S, rows gl <= E x + F u <= gu, disturbance
// w, feedback u = K x + v of eqn. (K_constraint)) folded into the form the kernels solve.
// With v the decision variable, x_{t+1} = A_K x_t + B v_t + w_t (A_K = A + B K), and every
// stage row that is not a bound on x_t -- the input bounds under a feedback (u_t = K x_t +
// v_t) and E x_t + F u_t = (E + F K) x_t + F v_t -- is the value y_{t+1} = M x_t + P v_t of
// nz extra state components, M = [K; E + F K], P = [I; F].  Their bounds [ul; gl], [uu; gu]
// on y_1..y_N are exactly those rows for t = 0..N-1, so J and the condensed matrix are the
// paper's (rows reordered).  The stage cost in (x, v) is 1/2 x'Q~x + x'S~v + 1/2 v'Rv with
// Q~ = Q + S K + K'S' + K'R K and S~ = S + K'R; the extra components carry no cost.
struct GeneralData {
  bool any = false, feedback = false;
  int ns_real = 0, nz = 0;
  std::vector<double> A, B, Q, Qf, R, xl, xu, ul, uu, S, w;
  cmpc_lq_desc std_desc{};
};

static int host_copy(const double* src, size_t len, bool on_device, std::vector<double>& dst) {
  dst.resize(len);
  if (len == 0) return 0;
  if (on_device) {
    CMPC_HIP(hipMemcpy(dst.data(), src, sizeof(double) * len, hipMemcpyDeviceToHost));
  } else {
    std::memcpy(dst.data(), src, sizeof(double) * len);
  }
  return 0;
}

static int fold_general(const cmpc_lq_desc& d, GeneralData& g) {
  const int ns = d.ns, nu = d.nu, N = d.N, nc = d.nc;
  const bool dev = d.data_on_device != 0;
  g.any = dev || d.S || d.w || d.Kfb || nc > 0;
  if (!g.any) return 0;
  if (ns <= 0 || nu <= 0 || N <= 0 || nc < 0) {
    set_error("ns, nu and N must be positive and nc >= 0");
    return CMPC_ERR_INVALID;
  }
  if (!d.A || !d.B || !d.Q || !d.R || !d.xl || !d.xu || !d.ul || !d.uu ||
      (nc > 0 && (!d.E || !d.F || !d.gl || !d.gu))) {
    set_error("NULL problem data");
    return CMPC_ERR_INVALID;
  }
  std::vector<double> A, B, Q, Qf, R, xl, xu, ul, uu, S, E, F, gl, gu, w, K;
  int rc = 0;
  rc = rc ? rc : host_copy(d.A, (size_t)ns * ns, dev, A);
  rc = rc ? rc : host_copy(d.B, (size_t)ns * nu, dev, B);
  rc = rc ? rc : host_copy(d.Q, (size_t)ns * ns, dev, Q);
  rc = rc ? rc : host_copy(d.Qf ? d.Qf : d.Q, (size_t)ns * ns, dev, Qf);
  rc = rc ? rc : host_copy(d.R, (size_t)nu * nu, dev, R);
  rc = rc ? rc : host_copy(d.xl, ns, dev, xl);
  rc = rc ? rc : host_copy(d.xu, ns, dev, xu);
  rc = rc ? rc : host_copy(d.ul, nu, dev, ul);
  rc = rc ? rc : host_copy(d.uu, nu, dev, uu);
  if (d.S) rc = rc ? rc : host_copy(d.S, (size_t)ns * nu, dev, S);
  if (nc > 0) {
    rc = rc ? rc : host_copy(d.E, (size_t)nc * ns, dev, E);
    rc = rc ? rc : host_copy(d.F, (size_t)nc * nu, dev, F);
    rc = rc ? rc : host_copy(d.gl, nc, dev, gl);
    rc = rc ? rc : host_copy(d.gu, nc, dev, gu);
  }
  if (d.w) rc = rc ? rc : host_copy(d.w, (size_t)N * ns, dev, w);
  if (d.Kfb) rc = rc ? rc : host_copy(d.Kfb, (size_t)nu * ns, dev, K);
  if (rc) return rc;
  for (const std::vector<double>* v : {&S, &E, &F, &w, &K})
    if (!all_finite(v->data(), v->size())) {
      set_error("non-finite entry in S, E, F, w or Kfb");
      return CMPC_ERR_NONFINITE;
    }
  for (int k = 0; k < nc; ++k)
    if (std::isnan(gl[k]) || std::isnan(gu[k]) || gl[k] > gu[k]) {
      set_error("invalid bounds of the rows E x + F u (need gl <= gu)");
      return std::isnan(gl[k]) || std::isnan(gu[k]) ? CMPC_ERR_NONFINITE : CMPC_ERR_INVALID;
    }
  g.feedback = !K.empty();
  if (K.empty()) K.assign((size_t)nu * ns, 0.0);
  if (S.empty()) S.assign((size_t)ns * nu, 0.0);
  const int nz = (g.feedback ? nu : 0) + nc, na = ns + nz;
  g.ns_real = ns;
  g.nz = nz;
  auto at = [](std::vector<double>& M, int ld, int i, int j) -> double& {
    return M[(size_t)i * ld + j];
  };
  // A_K = A + B K, M = [K; E + F K] (nz x ns), P = [I; F] (nz x nu)
  std::vector<double> AK(A), Mz((size_t)nz * ns, 0.0), Pz((size_t)nz * nu, 0.0);
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < ns; ++j) {
      double acc = 0.0;
      for (int k = 0; k < nu; ++k) acc += B[(size_t)i * nu + k] * K[(size_t)k * ns + j];
      at(AK, ns, i, j) += acc;
    }
  int r0 = 0;
  if (g.feedback) {
    for (int k = 0; k < nu; ++k) {
      for (int j = 0; j < ns; ++j) at(Mz, ns, k, j) = K[(size_t)k * ns + j];
      at(Pz, nu, k, k) = 1.0;
    }
    r0 = nu;
  }
  for (int c = 0; c < nc; ++c) {
    for (int j = 0; j < ns; ++j) {
      double acc = E[(size_t)c * ns + j];
      for (int k = 0; k < nu; ++k) acc += F[(size_t)c * nu + k] * K[(size_t)k * ns + j];
      at(Mz, ns, r0 + c, j) = acc;
    }
    for (int k = 0; k < nu; ++k) at(Pz, nu, r0 + c, k) = F[(size_t)c * nu + k];
  }
  // augmented A' = [[A_K, 0], [M, 0]], B' = [B; P]
  g.A.assign((size_t)na * na, 0.0);
  g.B.assign((size_t)na * nu, 0.0);
  for (int i = 0; i < ns; ++i) {
    for (int j = 0; j < ns; ++j) at(g.A, na, i, j) = at(AK, ns, i, j);
    for (int k = 0; k < nu; ++k) at(g.B, nu, i, k) = B[(size_t)i * nu + k];
  }
  for (int r = 0; r < nz; ++r) {
    for (int j = 0; j < ns; ++j) at(g.A, na, ns + r, j) = at(Mz, ns, r, j);
    for (int k = 0; k < nu; ++k) at(g.B, nu, ns + r, k) = at(Pz, nu, r, k);
  }
  // Q~ = Q + S K + K'S' + K'R K, S~ = S + K'R (ns x nu); Q' = blkdiag(Q~, 0), Qf' likewise
  g.Q.assign((size_t)na * na, 0.0);
  g.Qf.assign((size_t)na * na, 0.0);
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < ns; ++j) {
      double sk = 0.0, ks = 0.0, krk = 0.0;
      for (int k = 0; k < nu; ++k) {
        sk += S[(size_t)i * nu + k] * K[(size_t)k * ns + j];
        ks += K[(size_t)k * ns + i] * S[(size_t)j * nu + k];
        double rk = 0.0;
        for (int l = 0; l < nu; ++l) rk += R[(size_t)k * nu + l] * K[(size_t)l * ns + j];
        krk += K[(size_t)k * ns + i] * rk;
      }
      at(g.Q, na, i, j) = Q[(size_t)i * ns + j] + sk + ks + krk;
      at(g.Qf, na, i, j) = Qf[(size_t)i * ns + j];
    }
  g.S.assign((size_t)na * nu, 0.0);
  bool cross = false;
  for (int i = 0; i < ns; ++i)
    for (int k = 0; k < nu; ++k) {
      double v = S[(size_t)i * nu + k];
      for (int l = 0; l < nu; ++l) v += K[(size_t)l * ns + i] * R[(size_t)l * nu + k];
      at(g.S, nu, i, k) = v;
      cross = cross || v != 0.0;
    }
  if (!cross) g.S.clear();
  // bounds: x' in [xl; ul (feedback); gl], v free under a feedback
  g.xl = xl;
  g.xu = xu;
  if (g.feedback) {
    g.xl.insert(g.xl.end(), ul.begin(), ul.end());
    g.xu.insert(g.xu.end(), uu.begin(), uu.end());
    g.ul.assign(nu, -INFINITY);
    g.uu.assign(nu, INFINITY);
  } else {
    g.ul = ul;
    g.uu = uu;
  }
  g.xl.insert(g.xl.end(), gl.begin(), gl.end());
  g.xu.insert(g.xu.end(), gu.begin(), gu.end());
  g.R = R;
  if (!w.empty()) {
    g.w.assign((size_t)N * na, 0.0);
    for (int t = 0; t < N; ++t)
      for (int i = 0; i < ns; ++i) g.w[(size_t)t * na + i] = w[(size_t)t * ns + i];
  }
  cmpc_lq_desc& sd = g.std_desc;
  std::memset(&sd, 0, sizeof(sd));
  sd.ns = na;
  sd.nu = nu;
  sd.N = N;
  sd.A = g.A.data();
  sd.B = g.B.data();
  sd.Q = g.Q.data();
  sd.Qf = g.Qf.data();
  sd.R = g.R.data();
  sd.xl = g.xl.data();
  sd.xu = g.xu.data();
  sd.ul = g.ul.data();
  sd.uu = g.uu.data();
  return 0;
}


int create(const cmpc_lq_desc* desc, hipStream_t stream, Problem** out) {
  if (!desc || !out) {
    set_error("NULL argument");
    return CMPC_ERR_INVALID;
  }
  *out = nullptr;
  GeneralData g;
  int rc = fold_general(*desc, g);
  if (rc) return rc;
  if (!g.any) return create_standard(desc, stream, out);
  Problem* p = nullptr;
  rc = create_standard(&g.std_desc, stream, &p);
  if (rc) return rc;
  p->ns_real = g.ns_real;
  p->nz = g.nz;
  p->feedback = g.feedback;
  if (!g.S.empty()) {
    rc = upload(&p->Sx, g.S.data(), g.S.size(), stream);
    if (!rc) rc = launch_cross_hessian(*p, p->Sx);
  }
  if (!rc && !g.w.empty()) rc = upload(&p->wdist, g.w.data(), g.w.size(), stream);
  if (!rc && hipStreamSynchronize(stream) != hipSuccess) rc = CMPC_ERR_HIP;
  if (rc) {
    free_problem(p);
    return rc;
  }
  *out = p;
  return 0;
}

int set_x0(Problem& p, const double* x0, int on_device) {
  const int nr = p.ns_real;  // the problem's own states; the extra stage rows start at 0
  if (!on_device) {
    for (int i = 0; i < nr; ++i)
      if (!std::isfinite(x0[i])) {
        set_error("x0 has a non-finite entry");
        return CMPC_ERR_NONFINITE;
      }
    if (p.xl_host.empty()) {
      p.xl_host.resize(nr);
      p.xu_host.resize(nr);
      CMPC_HIP(hipMemcpy(p.xl_host.data(), p.xl, sizeof(double) * nr, hipMemcpyDeviceToHost));
      CMPC_HIP(hipMemcpy(p.xu_host.data(), p.xu, sizeof(double) * nr, hipMemcpyDeviceToHost));
    }
    for (int i = 0; i < nr; ++i)
      if (x0[i] < p.xl_host[i] || x0[i] > p.xu_host[i]) {
        set_error("x0 violates a state bound");
        return CMPC_ERR_X0_BOUNDS;
      }
  }
  CMPC_HIP(hipMemcpyAsync(p.x0, x0, sizeof(double) * nr,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p.stream));
  if (nr < p.ns)
    CMPC_HIP(hipMemsetAsync(p.x0 + nr, 0, sizeof(double) * (p.ns - nr), p.stream));
  // device x0: validated on the device; a bad x0 makes the next solve return the error
  if (launch_check_x0(p)) return CMPC_ERR_HIP;
  if (launch_free_response(p)) return CMPC_ERR_HIP;  // c_t = A c_{t-1} + w_{t-1}, c_0 = x0
  if (launch_block_diag_weight(p, p.c, p.qc)) return CMPC_ERR_HIP;
  if (launch_gamma_t(p, p.qc, 1, p.h, nullptr)) return CMPC_ERR_HIP;
  if (p.Sx != nullptr && launch_h_cross(p)) return CMPC_ERR_HIP;  // + S~' c_t on stage t
  if (launch_h0(p)) return CMPC_ERR_HIP;
  if (launch_make_d(p)) return CMPC_ERR_HIP;
  if (!on_device) CMPC_HIP(hipStreamSynchronize(p.stream));  // host x0 buffer may be reused
  p.have_x0 = true;
  return 0;
}

int solve(Problem& p, const cmpc_options& o, cmpc_result* res, int warm) {
  if (!p.have_x0) {
    set_error("cmpc_set_x0 must be called before cmpc_solve");
    return CMPC_ERR_INVALID;
  }
  if (!(o.tol > 0) || o.max_iter < 0) {
    set_error("invalid options");
    return CMPC_ERR_INVALID;
  }
  const int check = std::max(1, o.check_every);
  const bool prof = o.profile != 0;
  // mixed: starting precision level of the SYRK (2 BF16, 1 FP32), 0 = plain FP64
  const int mixed = o.precision == CMPC_BF16_SYRK ? 2 : (o.precision == CMPC_FP32_SYRK ? 1 : 0);
  {
    bool changed = false;
    const int rc = ensure_plan(p, o.precision, &changed);
    if (rc) return rc;
  }
  if (mixed) {
    const int rc = launch_convert_gamma(p, o.precision);
    if (rc) return rc;
  }
  p.eq_on = o.equilibrate < 0 ? mixed > 0 : o.equilibrate != 0;
  if (prof) {
    const size_t need = 4 * (size_t)(o.max_iter + 1);
    while (p.prof_ev.size() < need) {
      hipEvent_t e;
      CMPC_HIP(hipEventCreate(&e));
      p.prof_ev.push_back(e);
    }
  }
  CMPC_HIP(hipEventRecord(p.ev0, p.stream));
  if (launch_ipm_init(p, o, warm, o.warm_mu)) return CMPC_ERR_HIP;
  // Convergence is read back without stalling the queue: the last kernel of iteration it
  // stores 1 (running) or 2 (done) into slot it % R of a mapped pinned ring; before queueing
  // iteration it + depth the host polls slot it only.
  const int depth = std::max(1, check);
  constexpr int R = 16;
  if (p.hflags == nullptr) {
    CMPC_HIP(hipHostMalloc((void**)&p.hflags, sizeof(int) * R, hipHostMallocMapped));
    CMPC_HIP(hipHostGetDevicePointer((void**)&p.dflags, p.hflags, 0));
  }
  if (o.log != nullptr && p.hlog == nullptr) {
    CMPC_HIP(hipHostMalloc((void**)&p.hlog, sizeof(IterLog) * R, hipHostMallocMapped));
    CMPC_HIP(hipHostGetDevicePointer((void**)&p.dlog, p.hlog, 0));
  }
  IterLog* const dlog_keep = p.dlog;
  if (o.log == nullptr) p.dlog = nullptr;  // the iteration kernels write no snapshot
  volatile int* hf = p.hflags;
  int rc = 0;
  // log callback: iteration j's snapshot is read once its flag is set, in order
  int logged = 0, queued = 0;
  bool log_done = o.log == nullptr;
  auto emit = [&](int j) {
    if (log_done || j != logged) return;
    const volatile IterLog& e = p.hlog[j % R];
    char line[320];
    if (e.done == 2)
      std::snprintf(line, sizeof line, "iter %d: Cholesky of the low-precision K failed, "
                    "iteration redone at level %d", j, e.level);
    else if (e.done == 1)
      std::snprintf(line, sizeof line, "stop after %d iterations: %s, E0 %.3e, mu %.3e", e.iter,
                    cmpc_status_str(e.pad), e.err0, e.mu);
    else
      std::snprintf(line, sizeof line, "iter %d: mu %.3e E0 %.3e |r1| %.3e |r3| %.3e "
                    "|lam-z| %.3e max sz %.3e alpha %.3e alpha_z %.3e level %d", j, e.mu, e.err0,
                    e.nr1, e.nr3, e.nlz, e.szmax, e.alpha, e.alpha_z, e.level);
    o.log(line, o.log_ctx);
    ++logged;
    if (e.done == 1) log_done = true;
  };
  for (int it = 0; it <= o.max_iter && rc == 0; ++it) {
    if (it >= depth) {
      const int slot = (it - depth) % R;
      long long spins = 0;
      while (hf[slot] == 0) {
        if ((++spins & 1023) == 0) {
          const hipError_t q = hipStreamQuery(p.stream);
          if (q == hipSuccess && hf[slot] == 0) {  // queue drained but the flag never came
            set_error("solve: iteration flag missing");
            rc = CMPC_ERR_HIP;
            break;
          }
          if (q != hipSuccess && q != hipErrorNotReady) {
            set_error(std::string("solve: ") + hipGetErrorString(q));
            rc = CMPC_ERR_HIP;
            break;
          }
        }
      }
      if (rc) break;
      emit(it - depth);
      if (hf[slot] == 2) break;
    }
    const int slot = it % R;
    hf[slot] = 0;
    hipEvent_t e0 = prof ? p.prof_ev[4 * it] : nullptr, e1 = prof ? p.prof_ev[4 * it + 1] : nullptr;
    hipEvent_t e2 = prof ? p.prof_ev[4 * it + 2] : nullptr, e3 = prof ? p.prof_ev[4 * it + 3] : nullptr;
    if (it == 0) rc = launch_prep(p);  // later iterations' prep runs in the update kernel
    if (!rc) rc = launch_mu_rhs(p);
    if (!rc) rc = launch_syrk(p, CMPC_FP64, p.Dx, p.H, p.Du, p.K, e0, e1, mixed);
    if (!rc && p.eq_on) rc = launch_equilibrate(p.stream, p.K, p.n, p.n, p.eqs, &p.st->done);
    if (!rc) rc = launch_potrf(p.stream, p.K, p.n, p.n, p.Wdiag, &p.st->done, &p.st->info,
                               &p.st->status, e2, e3, mixed ? &p.st->use_low : nullptr, p.rhs,
                               p.eq_on ? p.eqs : nullptr, p.tmpn);
    if (!rc) rc = launch_step(p, mixed ? o.max_refine : 0);
    if (!rc) rc = launch_update_publish(p, slot);
    if (!rc) queued = it + 1;
  }
  p.dlog = dlog_keep;
  if (rc) return rc;
  CMPC_HIP(hipEventRecord(p.ev1, p.stream));
  IpmState hs;
  CMPC_HIP(hipMemcpyAsync(&hs, p.st, sizeof(IpmState), hipMemcpyDeviceToHost, p.stream));
  CMPC_HIP(hipStreamSynchronize(p.stream));
  for (int j = logged; j < queued && !log_done; ++j) emit(j);  // the last published ones
  const double gap = hs.gap;
  float ms = 0.f;
  hipEventElapsedTime(&ms, p.ev0, p.ev1);
  double ms_syrk = 0.0, ms_form = 0.0, ms_potrf = 0.0;
  if (prof)
    for (int it = 0; it < hs.iter && 4 * it + 3 < (int)p.prof_ev.size(); ++it) {
      float a = 0.f, b = 0.f, c = 0.f;
      hipEventElapsedTime(&a, p.prof_ev[4 * it], p.prof_ev[4 * it + 1]);
      hipEventElapsedTime(&b, p.prof_ev[4 * it], p.prof_ev[4 * it + 2]);
      hipEventElapsedTime(&c, p.prof_ev[4 * it + 2], p.prof_ev[4 * it + 3]);
      ms_syrk += a;
      ms_form += b;
      ms_potrf += c;
    }
  const int status = hs.done ? hs.status : CMPC_MAX_ITER;
  p.have_solution = status >= 0;
  if (res) {
    res->status = status;
    res->iters = hs.iter;
    res->precision_switch_iter = hs.switch_iter;
    res->refine_steps = hs.refine_steps;
    res->obj = hs.obj;
    res->primal_res = hs.nr3;
    res->dual_res = hs.nr1;
    res->compl_res = hs.szmax;
    res->mu = hs.mu;
    res->gap = gap;
    res->ms_total = ms;
    res->ms_syrk = ms_syrk;
    res->ms_form = ms_form;
    res->ms_potrf = ms_potrf;
  }
  if (status == CMPC_ERR_CHOLESKY) set_error("Cholesky breakdown at column " + std::to_string(hs.info));
  return status;
}

}  // namespace cmpc

using namespace cmpc;

extern "C" {

void cmpc_default_options(cmpc_options* o) {
  if (!o) return;
  o->tol = 1e-8;
  o->max_iter = 200;
  o->precision = CMPC_FP64;
  o->max_refine = 5;
  o->mu_switch = 1e-6;
  o->refine_contract = 0.1;
  o->log = nullptr;
  o->log_ctx = nullptr;
  o->warm_mu = 1e-3;
  o->check_every = 2;
  o->profile = 0;
  o->equilibrate = -1;
}

int cmpc_problem_info(const cmpc_problem* h, cmpc_info* info) {
  if (!h || !info) {
    set_error("NULL argument");
    return CMPC_ERR_INVALID;
  }
  const Problem& p = *h->p;
  info->n = p.n;
  info->mx = p.mx;
  info->m = p.m;
  info->gamma_nnz = (long long)p.ns * p.nu * ((long long)p.N * (p.N + 1) / 2);
  info->syrk_flops = p.syrk.flops_structural;
  info->potrf_flops = (double)p.n * p.n * p.n / 3.0;
  info->syrk_workgroups = p.syrk.nwg;
  info->syrk_partial_slots = p.syrk.nslots;
  const double gsz = (double)p.N * p.ns * p.nu;  // G and its transpose; Gamma is not stored
  double b = 0.0;
  if (p.G32) b += 4.0 * gsz;
  if (p.G16) b += 2.0 * gsz;
  b += 8.0 * (2.0 * p.n * p.n + 2.0 * gsz + 2.0 * p.ns * p.ns);
  b += 8.0 * 4096.0 * p.syrk.nslots + 8.0 * 3.0 * kGtJ * (double)p.gt_chunks;
  b += 8.0 * (7.0 * p.m + 12.0 * p.mx + 16.0 * p.n);
  info->device_bytes = b;
  return 0;
}

int cmpc_problem_create(const cmpc_lq_desc* desc, void* stream, cmpc_problem** out) {
  if (!out) {
    set_error("NULL output");
    return CMPC_ERR_INVALID;
  }
  *out = nullptr;
  Problem* p = nullptr;
  const int rc = create(desc, (hipStream_t)stream, &p);
  if (rc) return rc;
  *out = new cmpc_problem{p, false};
  return 0;
}

void cmpc_problem_destroy(cmpc_problem* h) {
  if (!h || h->borrowed) return;  // instances of a batch belong to the batch
  free_problem(h->p);
  delete h;
}

int cmpc_problem_dims(const cmpc_problem* h, int* n, int* mx, int* m) {
  if (!h) {
    set_error("NULL problem");
    return CMPC_ERR_INVALID;
  }
  if (n) *n = h->p->n;
  if (mx) *mx = h->p->mx;
  if (m) *m = h->p->m;
  return 0;
}

int cmpc_set_x0(cmpc_problem* h, const double* x0, int on_device) {
  if (!h || !x0) {
    set_error("NULL argument");
    return CMPC_ERR_INVALID;
  }
  return set_x0(*h->p, x0, on_device);
}

static int solve_options(const cmpc_options* opts, cmpc_options* o) {
  cmpc_default_options(o);
  if (opts) *o = *opts;
  if (o->precision != CMPC_FP64 && o->precision != CMPC_FP32_SYRK &&
      o->precision != CMPC_BF16_SYRK) {
    set_error("unsupported precision mode");
    return CMPC_ERR_INVALID;
  }
  if (o->max_refine < 0 || o->max_refine > 20) {
    set_error("max_refine must lie in [0, 20]");
    return CMPC_ERR_INVALID;
  }
  return 0;
}

int cmpc_solve(cmpc_problem* h, const cmpc_options* opts, cmpc_result* res) {
  if (!h) {
    set_error("NULL problem");
    return CMPC_ERR_INVALID;
  }
  cmpc_options o;
  const int rc = solve_options(opts, &o);
  if (rc) return rc;
  return solve(*h->p, o, res);
}

int cmpc_solve_warm(cmpc_problem* h, const cmpc_options* opts, const double* v0, int on_device,
                    cmpc_result* res) {
  if (!h) {
    set_error("NULL problem");
    return CMPC_ERR_INVALID;
  }
  cmpc_options o;
  int rc = solve_options(opts, &o);
  if (rc) return rc;
  if (!(o.warm_mu > 0) || !std::isfinite(o.warm_mu)) {
    set_error("warm_mu must be positive and finite");
    return CMPC_ERR_INVALID;
  }
  Problem& p = *h->p;
  if (!p.have_x0) {
    set_error("cmpc_set_x0 must be called before cmpc_solve_warm");
    return CMPC_ERR_INVALID;
  }
  if (v0 == nullptr) {
    if (!p.have_solution) {
      set_error("cmpc_solve_warm with v0 = NULL needs an earlier solve of this problem");
      return CMPC_ERR_INVALID;
    }
    rc = launch_shift_controls(p);
  } else if (on_device) {
    CMPC_HIP(hipMemcpyAsync(p.v, v0, sizeof(double) * p.n, hipMemcpyDeviceToDevice, p.stream));
  } else {
    if (!all_finite(v0, (size_t)p.n)) {
      set_error("non-finite entry in v0");
      return CMPC_ERR_NONFINITE;
    }
    CMPC_HIP(hipMemcpyAsync(p.v, v0, sizeof(double) * p.n, hipMemcpyHostToDevice, p.stream));
    CMPC_HIP(hipStreamSynchronize(p.stream));  // v0 is host memory the caller may reuse
  }
  if (rc) return rc;
  return solve(p, o, res, 1);
}

int cmpc_get_solution(const cmpc_problem* h, double* u, double* x, int on_device) {
  if (!h) {
    set_error("NULL problem");
    return CMPC_ERR_INVALID;
  }
  Problem& p = *h->p;
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const bool folded = p.ns_real != p.ns || p.feedback;
  if (!folded) {
    if (u) CMPC_HIP(hipMemcpyAsync(u, p.v, sizeof(double) * p.n, k, p.stream));
    if (x) {
      if (launch_gamma_mv(p, p.v, p.tmpmx, nullptr)) return CMPC_ERR_HIP;
      hipLaunchKernelGGL(add_vec_kernel, dim3(ceil_div(p.mx, 256)), dim3(256), 0, p.stream, p.c,
                         p.tmpmx, p.tmpmx, p.mx);
      CMPC_LAUNCH_CHECK();
      CMPC_HIP(hipMemcpyAsync(x, p.tmpmx, sizeof(double) * p.mx, k, p.stream));
    }
  } else if (u || x) {
    // the states with the extra stage rows, then the problem's own states and inputs
    if (launch_gamma_mv(p, p.v, p.tmpmx, nullptr)) return CMPC_ERR_HIP;
    hipLaunchKernelGGL(add_vec_kernel, dim3(ceil_div(p.mx, 256)), dim3(256), 0, p.stream, p.c,
                       p.tmpmx, p.tmpmx, p.mx);
    CMPC_LAUNCH_CHECK();
    double* ud = u ? (on_device ? u : p.tmpn) : nullptr;
    double* xd = x ? (on_device ? x : p.gpv) : nullptr;
    if (launch_unfold_solution(p, p.tmpmx, ud, xd)) return CMPC_ERR_HIP;
    if (u && !on_device)
      CMPC_HIP(hipMemcpyAsync(u, p.tmpn, sizeof(double) * p.n, hipMemcpyDeviceToHost, p.stream));
    if (x && !on_device)
      CMPC_HIP(hipMemcpyAsync(x, p.gpv, sizeof(double) * (size_t)p.ns_real * p.N,
                              hipMemcpyDeviceToHost, p.stream));
  }
  CMPC_HIP(hipStreamSynchronize(p.stream));
  return 0;
}

int cmpc_get_iterate(const cmpc_problem* h, double* v, double* s, double* lam, double* z,
                     int on_device) {
  if (!h) {
    set_error("NULL problem");
    return CMPC_ERR_INVALID;
  }
  Problem& p = *h->p;
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (v) CMPC_HIP(hipMemcpyAsync(v, p.v, sizeof(double) * p.n, k, p.stream));
  if (s) CMPC_HIP(hipMemcpyAsync(s, p.s, sizeof(double) * p.m, k, p.stream));
  if (lam) CMPC_HIP(hipMemcpyAsync(lam, p.lam, sizeof(double) * p.m, k, p.stream));
  if (z) CMPC_HIP(hipMemcpyAsync(z, p.z, sizeof(double) * p.m, k, p.stream));
  CMPC_HIP(hipStreamSynchronize(p.stream));
  return 0;
}

int cmpc_export_dense(const cmpc_problem* h, double* H, double* hv, double* h0, double* d,
                      double* c, double* Gamma) {
  if (!h) {
    set_error("NULL problem");
    return CMPC_ERR_INVALID;
  }
  Problem& p = *h->p;
  const hipMemcpyKind k = hipMemcpyDeviceToHost;
  if (H) CMPC_HIP(hipMemcpyAsync(H, p.H, sizeof(double) * p.n * p.n, k, p.stream));
  if ((hv || h0 || d || c) && !p.have_x0) {
    set_error("x0-dependent data requested before cmpc_set_x0");
    return CMPC_ERR_INVALID;
  }
  if (hv) CMPC_HIP(hipMemcpyAsync(hv, p.h, sizeof(double) * p.n, k, p.stream));
  if (h0) CMPC_HIP(hipMemcpyAsync(h0, &p.st->h0, sizeof(double), k, p.stream));
  if (d) CMPC_HIP(hipMemcpyAsync(d, p.d, sizeof(double) * p.m, k, p.stream));
  if (c) CMPC_HIP(hipMemcpyAsync(c, p.c, sizeof(double) * p.mx, k, p.stream));
  if (Gamma) {
    double* tmp = nullptr;
    CMPC_HIP(hipMalloc(&tmp, sizeof(double) * (size_t)p.mx * p.n));
    int rc = launch_dense_gamma(p, tmp);
    if (!rc && hipMemcpyAsync(Gamma, tmp, sizeof(double) * (size_t)p.mx * p.n, k, p.stream) !=
                   hipSuccess)
      rc = CMPC_ERR_HIP;
    hipStreamSynchronize(p.stream);
    hipFree(tmp);
    if (rc) return rc;
  }
  CMPC_HIP(hipStreamSynchronize(p.stream));
  return 0;
}

int cmpc_form_condensed(cmpc_problem* h, const double* sigma, double* K, int precision) {
  if (!h || !sigma || !K) {
    set_error("NULL argument");
    return CMPC_ERR_INVALID;
  }
  if (precision != CMPC_FP64 && precision != CMPC_FP32_SYRK && precision != CMPC_BF16_SYRK) {
    set_error("unsupported precision");
    return CMPC_ERR_INVALID;
  }
  Problem& p = *h->p;
  if (precision != CMPC_FP64 && launch_convert_gamma(p, precision)) return CMPC_ERR_HIP;
  CMPC_HIP(hipMemsetAsync(&p.st->done, 0, sizeof(int), p.stream));
  if (launch_sigma_fold(p, sigma)) return CMPC_ERR_HIP;
  if (launch_syrk(p, precision, p.Dx, p.H, p.Du, K)) return CMPC_ERR_HIP;
  CMPC_HIP(hipStreamSynchronize(p.stream));
  return 0;
}

int cmpc_newton_step(cmpc_problem* h, const double* v, const double* s, const double* lam,
                     const double* z, double mu, double tau, double* pv, double* ps, double* plam,
                     double* pz, double* alphas) {
  if (!h || !v || !s || !lam || !z) {
    set_error("NULL argument");
    return CMPC_ERR_INVALID;
  }
  Problem& p = *h->p;
  if (!p.have_x0) {
    set_error("cmpc_set_x0 must be called first");
    return CMPC_ERR_INVALID;
  }
  if (!(mu > 0) || !(tau > 0) || !(tau <= 1)) {
    set_error("need mu > 0 and 0 < tau <= 1");
    return CMPC_ERR_INVALID;
  }
  if (launch_step_given(p, v, s, lam, z, mu, tau)) return CMPC_ERR_HIP;
  const hipMemcpyKind k = hipMemcpyDeviceToDevice;
  if (pv) CMPC_HIP(hipMemcpyAsync(pv, p.pv, sizeof(double) * p.n, k, p.stream));
  if (ps) CMPC_HIP(hipMemcpyAsync(ps, p.ps, sizeof(double) * p.m, k, p.stream));
  if (plam) CMPC_HIP(hipMemcpyAsync(plam, p.plam, sizeof(double) * p.m, k, p.stream));
  if (pz) CMPC_HIP(hipMemcpyAsync(pz, p.pz, sizeof(double) * p.m, k, p.stream));
  IpmState hs;
  CMPC_HIP(hipMemcpyAsync(&hs, p.st, sizeof(IpmState), hipMemcpyDeviceToHost, p.stream));
  CMPC_HIP(hipStreamSynchronize(p.stream));
  if (hs.done && hs.status == CMPC_ERR_CHOLESKY) {
    set_error("Cholesky breakdown at column " + std::to_string(hs.info));
    return CMPC_ERR_CHOLESKY;
  }
  if (alphas) {
    alphas[0] = hs.alpha;
    alphas[1] = hs.alpha_z;
  }
  return 0;
}

int cmpc_potrf(double* K, int n, int ld, void* stream, int* info) {
  if (!K || n <= 0 || ld < n) {
    set_error("invalid argument");
    return CMPC_ERR_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  int* flags = nullptr;  // done, info, status
  double* Wall = nullptr;
  CMPC_HIP(hipMalloc(&flags, 3 * sizeof(int)));
  if (hipMalloc(&Wall, sizeof(double) * wall_doubles(n)) != hipSuccess) {
    hipFree(flags);
    set_error("out of device memory");
    return CMPC_ERR_NOMEM;
  }
  int rc = 0;
  if (hipMemsetAsync(flags, 0, 3 * sizeof(int), s) != hipSuccess) rc = CMPC_ERR_HIP;
  if (!rc) rc = launch_potrf(s, K, n, ld, Wall, flags, flags + 1, flags + 2);
  int hf[3] = {0, 0, 0};
  if (!rc && (hipMemcpyAsync(hf, flags, 3 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess))
    rc = CMPC_ERR_HIP;
  hipFree(flags);
  hipFree(Wall);
  if (rc) return rc;
  if (info) *info = hf[1];
  if (hf[0]) {
    set_error("matrix is not positive definite (column " + std::to_string(hf[1]) + ")");
    return CMPC_ERR_CHOLESKY;
  }
  return 0;
}

int cmpc_potrf_noalloc(double* K, int n, int ld, void* stream, int* info) {
  if (!K || n <= 0 || ld < n) {
    set_error("invalid argument");
    return CMPC_ERR_INVALID;
  }
  if (n > CMPC_POTRF_NOALLOC_MAX_N) {
    set_error("cmpc_potrf_noalloc: n = " + std::to_string(n) + " exceeds its maximum " +
              std::to_string(CMPC_POTRF_NOALLOC_MAX_N) + " (use cmpc_potrf)");
    return CMPC_ERR_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  double* base = nullptr;
  int rc = potrf_scratch(s, &base);
  if (rc) return rc;
  double* Wall = base;
  int* flags = (int*)(base + kNoAllocWallDoubles);  // done, info, status
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, s, flags, 3);
  if (hipGetLastError() != hipSuccess) {
    set_error("cmpc_potrf_noalloc: launch failed");
    return CMPC_ERR_HIP;
  }
  rc = launch_potrf(s, K, n, ld, Wall, flags, flags + 1, flags + 2);
  int hf[3] = {0, 0, 0};
  if (!rc && (hipMemcpyAsync(hf, flags, 3 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess))
    rc = CMPC_ERR_HIP;
  if (rc) return rc;
  if (info) *info = hf[1];
  if (hf[0]) {
    set_error("matrix is not positive definite (column " + std::to_string(hf[1]) + ")");
    return CMPC_ERR_CHOLESKY;
  }
  return 0;
}

int cmpc_potrs(const double* L, int n, int ld, double* b, void* stream) {
  if (!L || !b || n <= 0 || ld < n) {
    set_error("invalid argument");
    return CMPC_ERR_INVALID;
  }
  if (n > 8192) {
    set_error("n > 8192 is not supported");
    return CMPC_ERR_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  double* Wall = nullptr;
  CMPC_HIP(hipMalloc(&Wall, sizeof(double) * (wall_doubles(n) + n)));
  int rc = launch_tri_inv(s, L, n, ld, Wall);
  if (!rc) rc = launch_potrs(s, L, n, ld, Wall, b, b, Wall + wall_doubles(n), nullptr);
  if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = CMPC_ERR_HIP;
  hipFree(Wall);
  return rc;
}

const char* cmpc_last_error(void) { return g_error.c_str(); }

const char* cmpc_status_str(int status) {
  switch (status) {
    case CMPC_OK: return "converged";
    case CMPC_MAX_ITER: return "iteration limit";
    case CMPC_SMALL_STEP: return "step too small";
    case CMPC_ERR_INVALID: return "invalid argument";
    case CMPC_ERR_NONFINITE: return "non-finite input";
    case CMPC_ERR_X0_BOUNDS: return "x0 outside the state bounds";
    case CMPC_ERR_CHOLESKY: return "Cholesky breakdown";
    case CMPC_ERR_HIP: return "HIP error";
    case CMPC_ERR_NOMEM: return "out of device memory";
    default: return "unknown status";
  }
}

}  // extern "C"
