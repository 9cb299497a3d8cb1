// C ABI (include/condmpc.h) and the host-side interior-point driver (Algorithm 1).
#include <algorithm>
#include <cstring>
#include <vector>

#include "problem.hpp"

namespace cmpc {

static thread_local std::string g_error;
void set_error(const std::string& msg) { g_error = msg; }

int launch_convert_gamma(Problem& p, int precision);

__global__ void add_vec_kernel(const double* __restrict__ a, const double* __restrict__ b,
                               double* __restrict__ out, int len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) out[i] = a[i] + b[i];
}

static void free_problem(Problem* p) {
  if (!p) return;
  if (p->stream) hipStreamSynchronize(p->stream);
  else hipDeviceSynchronize();
  double** bufs[] = {&p->A,  &p->B,   &p->Q,    &p->Qf,    &p->R,    &p->xl,   &p->xu,
                     &p->ul, &p->uu,  &p->qdiag, &p->G,    &p->Gam,  &p->H,    &p->K,
                     &p->x0, &p->c,   &p->qc,   &p->h,     &p->d,    &p->v,    &p->s,
                     &p->lam, &p->z,  &p->gv,   &p->pv,    &p->ps,   &p->plam, &p->pz,
                     &p->gpv, &p->rhs, &p->Dx,  &p->Du,    &p->wx,   &p->wu,   &p->gt,
                     &p->Hv, &p->tmpn, &p->tmpn2, &p->tmpmx, &p->norm_part, &p->alpha_part,
                     &p->gt_part};
  for (double** b : bufs) {
    if (*b) hipFree(*b);
    *b = nullptr;
  }
  if (p->goff) hipFree(p->goff);
  if (p->Gam32) hipFree(p->Gam32);
  if (p->Gam16) hipFree(p->Gam16);
  if (p->st) hipFree(p->st);
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

static int create(const cmpc_lq_desc* desc, hipStream_t stream, Problem** out) {
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
  // packed Gamma
  p->off.resize(N + 1);
  for (int t = 1; t <= N + 1; ++t) p->off[t - 1] = (long long)ns * nu * (long long)t * (t - 1) / 2;
  if (hipMalloc(&p->Gam, sizeof(double) * (size_t)p->off[N]) != hipSuccess) {
    set_error("out of device memory (Gamma)");
    free_problem(p);
    return CMPC_ERR_NOMEM;
  }
  if (hipMalloc(&p->goff, sizeof(long long) * (N + 1)) != hipSuccess) {
    free_problem(p);
    return CMPC_ERR_NOMEM;
  }
  if (hipMemcpyAsync(p->goff, p->off.data(), sizeof(long long) * (N + 1), hipMemcpyHostToDevice,
                     stream) != hipSuccess) {
    free_problem(p);
    return CMPC_ERR_HIP;
  }
  TRY(launch_pack_gamma(*p));
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
    double* Y = nullptr;
    if (hipMalloc(&Y, sizeof(double) * (size_t)ns * p->n) != hipSuccess) {
      free_problem(p);
      return CMPC_ERR_NOMEM;
    }
    for (int t = 1; t <= N && rc == 0; ++t) {
      const int len = t * nu;
      const double* Gt = p->Gam + p->off[t - 1];
      const double* W = (t == N) ? p->Qf : p->Q;
      rc = launch_gemm_f64(stream, ns, len, ns, 1.0, W, ns, 1, Gt, len, 1, 0.0, Y, len);
      if (!rc) rc = launch_gemm_f64(stream, len, len, ns, 1.0, Gt, 1, len, Y, len, 1, 1.0, p->H, p->n);
    }
    hipStreamSynchronize(stream);
    hipFree(Y);
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

static int set_x0(Problem& p, const double* x0, int on_device) {
  std::vector<double> hx(p.ns);
  if (on_device) {
    CMPC_HIP(hipMemcpyAsync(hx.data(), x0, sizeof(double) * p.ns, hipMemcpyDeviceToHost, p.stream));
    CMPC_HIP(hipStreamSynchronize(p.stream));
  } else {
    std::memcpy(hx.data(), x0, sizeof(double) * p.ns);
  }
  if (!all_finite(hx.data(), p.ns)) {
    set_error("x0 has a non-finite entry");
    return CMPC_ERR_NONFINITE;
  }
  std::vector<double> xl(p.ns), xu(p.ns);
  CMPC_HIP(hipMemcpyAsync(xl.data(), p.xl, sizeof(double) * p.ns, hipMemcpyDeviceToHost, p.stream));
  CMPC_HIP(hipMemcpyAsync(xu.data(), p.xu, sizeof(double) * p.ns, hipMemcpyDeviceToHost, p.stream));
  CMPC_HIP(hipStreamSynchronize(p.stream));
  for (int i = 0; i < p.ns; ++i)
    if (hx[i] < xl[i] || hx[i] > xu[i]) {
      set_error("x0 violates a state bound");
      return CMPC_ERR_X0_BOUNDS;
    }
  CMPC_HIP(hipMemcpyAsync(p.x0, x0, sizeof(double) * p.ns,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p.stream));
  // c_t = A^t x0, t = 1..N
  if (launch_gemv(p.stream, p.A, p.x0, p.c, p.ns, p.ns)) return CMPC_ERR_HIP;
  for (int t = 2; t <= p.N; ++t)
    if (launch_gemv(p.stream, p.A, p.c + (size_t)(t - 2) * p.ns, p.c + (size_t)(t - 1) * p.ns,
                    p.ns, p.ns))
      return CMPC_ERR_HIP;
  if (launch_block_diag_weight(p, p.c, p.qc)) return CMPC_ERR_HIP;
  if (launch_gamma_t(p, p.qc, 1, p.h, nullptr)) return CMPC_ERR_HIP;
  if (launch_h0(p)) return CMPC_ERR_HIP;
  if (launch_make_d(p)) return CMPC_ERR_HIP;
  p.have_x0 = true;
  return 0;
}

static int solve(Problem& p, const cmpc_options& o, cmpc_result* res) {
  if (!p.have_x0) {
    set_error("cmpc_set_x0 must be called before cmpc_solve");
    return CMPC_ERR_INVALID;
  }
  if (!(o.tol > 0) || o.max_iter < 0) {
    set_error("invalid options");
    return CMPC_ERR_INVALID;
  }
  const int check = std::max(1, o.check_every);
  CMPC_HIP(hipEventRecord(p.ev0, p.stream));
  if (launch_ipm_init(p, o)) return CMPC_ERR_HIP;
  int* hflag = nullptr;
  CMPC_HIP(hipHostMalloc((void**)&hflag, sizeof(int)));
  *hflag = 0;
  int rc = 0;
  for (int it = 0; it <= o.max_iter && rc == 0; ++it) {
    rc = launch_prep(p);
    if (!rc) rc = launch_mu_rhs(p);
    if (!rc) rc = launch_syrk(p, CMPC_FP64, p.Dx, p.H, p.Du, p.K);
    if (!rc) rc = launch_potrf(p.stream, p.K, p.n, p.n, &p.st->done, &p.st->info, &p.st->status);
    if (!rc) rc = launch_step(p);
    if (!rc) rc = launch_update(p);
    if (rc) break;
    if ((it + 1) % check == 0 || it == o.max_iter) {
      if (hipMemcpyAsync(hflag, &p.st->done, sizeof(int), hipMemcpyDeviceToHost, p.stream) !=
              hipSuccess ||
          hipStreamSynchronize(p.stream) != hipSuccess) {
        set_error(std::string("solve: ") + hipGetErrorString(hipGetLastError()));
        rc = CMPC_ERR_HIP;
        break;
      }
      if (*hflag) break;
    }
  }
  hipHostFree(hflag);
  if (rc) return rc;
  if (launch_finalize(p)) return CMPC_ERR_HIP;
  CMPC_HIP(hipEventRecord(p.ev1, p.stream));
  IpmState hs;
  double gap = 0;
  CMPC_HIP(hipMemcpyAsync(&hs, p.st, sizeof(IpmState), hipMemcpyDeviceToHost, p.stream));
  CMPC_HIP(hipMemcpyAsync(&gap, p.tmpn, sizeof(double), hipMemcpyDeviceToHost, p.stream));
  CMPC_HIP(hipStreamSynchronize(p.stream));
  float ms = 0.f;
  hipEventElapsedTime(&ms, p.ev0, p.ev1);
  const int status = hs.done ? hs.status : CMPC_MAX_ITER;
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
  }
  if (status == CMPC_ERR_CHOLESKY) set_error("Cholesky breakdown at column " + std::to_string(hs.info));
  return status;
}

}  // namespace cmpc

using namespace cmpc;

struct cmpc_problem {
  Problem* p;
};

extern "C" {

void cmpc_default_options(cmpc_options* o) {
  if (!o) return;
  o->tol = 1e-8;
  o->max_iter = 200;
  o->precision = CMPC_FP64;
  o->max_refine = 5;
  o->mu_switch = 1e-6;
  o->check_every = 1;
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
  *out = new cmpc_problem{p};
  return 0;
}

void cmpc_problem_destroy(cmpc_problem* h) {
  if (!h) return;
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

int cmpc_solve(cmpc_problem* h, const cmpc_options* opts, cmpc_result* res) {
  if (!h) {
    set_error("NULL problem");
    return CMPC_ERR_INVALID;
  }
  cmpc_options o;
  cmpc_default_options(&o);
  if (opts) o = *opts;
  if (o.precision != CMPC_FP64) {
    set_error("mixed-precision modes are not available in this build");
    return CMPC_ERR_INVALID;
  }
  return solve(*h->p, o, res);
}

int cmpc_get_solution(const cmpc_problem* h, double* u, double* x, int on_device) {
  if (!h) {
    set_error("NULL problem");
    return CMPC_ERR_INVALID;
  }
  Problem& p = *h->p;
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (u) CMPC_HIP(hipMemcpyAsync(u, p.v, sizeof(double) * p.n, k, p.stream));
  if (x) {
    if (launch_gamma_mv(p, p.v, p.tmpmx, nullptr)) return CMPC_ERR_HIP;
    hipLaunchKernelGGL(add_vec_kernel, dim3(ceil_div(p.mx, 256)), dim3(256), 0, p.stream, p.c,
                       p.tmpmx, p.tmpmx, p.mx);
    CMPC_LAUNCH_CHECK();
    CMPC_HIP(hipMemcpyAsync(x, p.tmpmx, sizeof(double) * p.mx, k, p.stream));
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
  if (precision != CMPC_FP64 && precision != CMPC_FP32_SYRK) {
    set_error("unsupported precision");
    return CMPC_ERR_INVALID;
  }
  Problem& p = *h->p;
  if (precision == CMPC_FP32_SYRK && launch_convert_gamma(p, precision)) return CMPC_ERR_HIP;
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
  CMPC_HIP(hipMalloc(&flags, 3 * sizeof(int)));
  int rc = 0;
  if (hipMemsetAsync(flags, 0, 3 * sizeof(int), s) != hipSuccess) rc = CMPC_ERR_HIP;
  if (!rc) rc = launch_potrf(s, K, n, ld, flags, flags + 1, flags + 2);
  int hf[3] = {0, 0, 0};
  if (!rc && (hipMemcpyAsync(hf, flags, 3 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess))
    rc = CMPC_ERR_HIP;
  hipFree(flags);
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
  hipStream_t s = (hipStream_t)stream;
  if (launch_potrs(s, L, n, ld, b, nullptr)) return CMPC_ERR_HIP;
  CMPC_HIP(hipStreamSynchronize(s));
  return 0;
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
