// Host driver of the surrogate policy (library extension): a multilayer perceptron that
// maps x0 to the control sequence of the condensed QP of Section 2, trained on the
// interior-point method's own solutions with the MLP kernels (k_mlp.hip), and a judge that
// certifies each answer (bounds on the simulated states within 1e-4, objective within 1e-3
// of the lambda = 0 dual bound) and hands every answer it cannot certify to Algorithm 1.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "surrogate.hpp"

namespace cmpc {

constexpr int kMlpRows = 4096;  // activation rows held on the device (queries per chunk)

static int pad64(int x) { return (x + 63) / 64 * 64; }

struct Mlp {
  int precision = CMPC_MLP_BF16;
  int ns = 0, nu = 0, N = 0, n = 0, depth = 0, hidden = 0;
  std::vector<int> w, wp;          // true and padded widths, L + 2 entries
  std::vector<float*> W, b, mW, vW, mb, vb, dW, db;  // index l = 1..L+1 (0 unused)
  std::vector<void*> Wlow;         // T copies of W
  std::vector<void*> a;            // activations a_0..a_L (T, kMlpRows x wp[l])
  std::vector<float*> z;           // pre-activations z_1..z_L (float)
  float* y = nullptr;              // output (float, kMlpRows x wp[L+1])
  float* ut = nullptr;             // targets (float, kMlpRows x wp[L+1])
  void* g[2] = {nullptr, nullptr}; // gradient ping-pong (T, kMlpRows x max width)
  int* idx = nullptr;              // minibatch row indices (device)
  int idx_cap = 0;
  double* part = nullptr;          // loss partial sums
  int part_cap = 0;
  double* steploss = nullptr;      // per-step loss (device)
  int steploss_cap = 0;
  long long step = 0;              // AdamW step counter
  hipStream_t stream = nullptr;
  // judge (FP64): diagonal weights and the unconstrained cost-to-go P0
  double *q = nullptr, *qf = nullptr, *P0 = nullptr;
  double *jf = nullptr, *jv = nullptr, *jl = nullptr, *jg = nullptr;
  int* jacc = nullptr;
  int jcap = 0;
  Problem* prob = nullptr;         // the problem the policy answers (not owned)
  cmpc_batch* fb = nullptr;        // fallback batch of copies of prob (not owned), or NULL
  int fb_warm = 0;                 // fallback solves start from the network's answer
  size_t tsize() const { return precision == CMPC_MLP_BF16 ? 2 : 4; }
};

static void free_mlp(Mlp* m) {
  if (!m) return;
  if (m->stream) hipStreamSynchronize(m->stream);
  for (auto* vec : {&m->W, &m->b, &m->mW, &m->vW, &m->mb, &m->vb, &m->dW, &m->db})
    for (float* p : *vec)
      if (p) hipFree(p);
  for (void* p : m->Wlow)
    if (p) hipFree(p);
  for (void* p : m->a)
    if (p) hipFree(p);
  for (float* p : m->z)
    if (p) hipFree(p);
  void* rest[] = {m->y, m->ut, m->g[0], m->g[1], m->idx, m->part, m->steploss, m->q, m->qf,
                  m->P0, m->jf, m->jv, m->jl, m->jg, m->jacc};
  for (void* p : rest)
    if (p) hipFree(p);
  delete m;
}

template <typename T>
static T* dalloc(size_t count, int* rc) {
  T* p = nullptr;
  if (*rc) return nullptr;
  if (hipMalloc(&p, sizeof(T) * std::max<size_t>(1, count)) != hipSuccess) {
    set_error("out of device memory (surrogate)");
    *rc = CMPC_ERR_NOMEM;
    return nullptr;
  }
  if (hipMemset(p, 0, sizeof(T) * std::max<size_t>(1, count)) != hipSuccess) *rc = CMPC_ERR_HIP;
  return p;
}

static long long param_count(const Mlp& m) {
  long long c = 0;
  for (size_t l = 1; l < m.w.size(); ++l) c += (long long)m.w[l] * m.w[l - 1] + m.w[l];
  return c;
}

// Copy packed host parameters (W_1, b_1, ..., W_{L+1}, b_{L+1}, unpadded, row-major) into the
// padded master arrays and their low-precision copies.
static int set_params(Mlp& m, const float* host) {
  size_t off = 0;
  for (size_t l = 1; l < m.w.size(); ++l) {
    const int dout = m.w[l], din = m.w[l - 1], ldp = m.wp[l - 1];
    std::vector<float> Wp((size_t)m.wp[l] * ldp, 0.f), bp(m.wp[l], 0.f);
    for (int i = 0; i < dout; ++i)
      std::memcpy(&Wp[(size_t)i * ldp], host + off + (size_t)i * din, sizeof(float) * din);
    off += (size_t)dout * din;
    std::memcpy(bp.data(), host + off, sizeof(float) * dout);
    off += dout;
    CMPC_HIP(hipMemcpy(m.W[l], Wp.data(), sizeof(float) * Wp.size(), hipMemcpyHostToDevice));
    CMPC_HIP(hipMemcpy(m.b[l], bp.data(), sizeof(float) * bp.size(), hipMemcpyHostToDevice));
    const long long len = (long long)Wp.size();
    CMPC_HIP(hipMemset(m.mW[l], 0, sizeof(float) * len));
    CMPC_HIP(hipMemset(m.vW[l], 0, sizeof(float) * len));
    CMPC_HIP(hipMemset(m.mb[l], 0, sizeof(float) * m.wp[l]));
    CMPC_HIP(hipMemset(m.vb[l], 0, sizeof(float) * m.wp[l]));
    int rc = m.precision == CMPC_MLP_BF16
                 ? launch_to_low<bf16_t>(m.stream, m.W[l], (bf16_t*)m.Wlow[l], len)
                 : launch_to_low<float>(m.stream, m.W[l], (float*)m.Wlow[l], len);
    if (rc) return rc;
  }
  m.step = 0;
  CMPC_HIP(hipStreamSynchronize(m.stream));
  return 0;
}

static int get_padded(const Mlp& m, const std::vector<float*>& Ws, const std::vector<float*>& bs,
                      float* host) {
  size_t off = 0;
  for (size_t l = 1; l < m.w.size(); ++l) {
    const int dout = m.w[l], din = m.w[l - 1], ldp = m.wp[l - 1];
    std::vector<float> Wp((size_t)m.wp[l] * ldp), bp(m.wp[l]);
    CMPC_HIP(hipMemcpy(Wp.data(), Ws[l], sizeof(float) * Wp.size(), hipMemcpyDeviceToHost));
    CMPC_HIP(hipMemcpy(bp.data(), bs[l], sizeof(float) * bp.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < dout; ++i)
      std::memcpy(host + off + (size_t)i * din, &Wp[(size_t)i * ldp], sizeof(float) * din);
    off += (size_t)dout * din;
    std::memcpy(host + off, bp.data(), sizeof(float) * dout);
    off += dout;
  }
  return 0;
}

template <typename T>
static int forward_t(Mlp& m, int Mp) {
  const int L = m.depth;
  for (int l = 1; l <= L + 1; ++l) {
    MlpEpi e;
    e.bias = m.b[l];
    if (l <= L) {
      e.z = m.z[l];
      e.ldz = m.wp[l];
      e.h = m.a[l];
      e.ldh = m.wp[l];
    } else {
      e.z = m.y;
      e.ldz = m.wp[l];
    }
    const int rc = launch_mlp_gemm<T>(m.stream, l <= L ? kGemmFwdGelu : kGemmFwdLinear,
                                      (const T*)m.a[l - 1], m.wp[l - 1], (const T*)m.Wlow[l],
                                      m.wp[l - 1], Mp, m.wp[l], m.wp[l - 1], e);
    if (rc) return rc;
  }
  return 0;
}

// Gradient of the mean squared error over rows [0, rows) and outputs [0, n) of the last
// forward pass, into dW, db; the loss goes to *loss_dev.
template <typename T>
static int backward_t(Mlp& m, int Mp, int rows, double* loss_dev) {
  const int L = m.depth;
  int nparts = 0;
  const long long need = ((long long)Mp * m.wp[L + 1] + 255) / 256;
  if (need > m.part_cap) {
    set_error("surrogate: loss buffer too small");
    return CMPC_ERR_INVALID;
  }
  int rc = launch_mse_grad<T>(m.stream, m.y, m.wp[L + 1], m.ut, m.wp[L + 1], rows, m.n,
                              (T*)m.g[0], m.wp[L + 1], Mp, m.part, &nparts);
  if (!rc && loss_dev)
    rc = launch_sum_parts(m.stream, m.part, nparts, (double)rows * m.n, loss_dev);
  int cur = 0;
  for (int l = L + 1; l >= 1 && !rc; --l) {
    MlpEpi ew;
    ew.z = m.dW[l];
    ew.ldz = m.wp[l - 1];
    rc = launch_mlp_gemm<T>(m.stream, kGemmBwdWeight, (const T*)m.g[cur], m.wp[l],
                            (const T*)m.a[l - 1], m.wp[l - 1], m.wp[l], m.wp[l - 1], Mp, ew);
    if (!rc) rc = launch_colsum<T>(m.stream, (const T*)m.g[cur], m.wp[l], Mp, m.wp[l], m.db[l]);
    if (!rc && l > 1) {
      MlpEpi ed;
      ed.zin = m.z[l - 1];
      ed.ldzi = m.wp[l - 1];
      ed.h = m.g[1 - cur];
      ed.ldh = m.wp[l - 1];
      rc = launch_mlp_gemm<T>(m.stream, kGemmBwdData, (const T*)m.g[cur], m.wp[l],
                              (const T*)m.Wlow[l], m.wp[l - 1], Mp, m.wp[l - 1], m.wp[l], ed);
      cur = 1 - cur;
    }
  }
  return rc;
}

static int forward(Mlp& m, int Mp) {
  return m.precision == CMPC_MLP_BF16 ? forward_t<bf16_t>(m, Mp) : forward_t<float>(m, Mp);
}
static int backward(Mlp& m, int Mp, int rows, double* loss_dev) {
  return m.precision == CMPC_MLP_BF16 ? backward_t<bf16_t>(m, Mp, rows, loss_dev)
                                      : backward_t<float>(m, Mp, rows, loss_dev);
}

// Stage rows idx[0..rows) (or 0..rows) of the x0 matrix (and of the targets) into a_0 / ut.
static int stage(Mlp& m, const double* X, const double* U, const int* idx, int rows, int Mp) {
  int rc = m.precision == CMPC_MLP_BF16
               ? launch_stage_rows<bf16_t>(m.stream, X, m.ns, m.ns, idx, rows, (bf16_t*)m.a[0],
                                           m.wp[0], Mp)
               : launch_stage_rows<float>(m.stream, X, m.ns, m.ns, idx, rows, (float*)m.a[0],
                                          m.wp[0], Mp);
  if (!rc && U)
    rc = launch_stage_rows<float>(m.stream, U, m.n, m.n, idx, rows, m.ut, m.wp[m.depth + 1], Mp);
  return rc;
}

static int adamw_all(Mlp& m, float lr, const cmpc_train_opts& o) {
  m.step += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)o.beta1, (double)m.step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)o.beta2, (double)m.step)));
  for (size_t l = 1; l < m.w.size(); ++l) {
    const long long lw = (long long)m.wp[l] * m.wp[l - 1];
    int rc = m.precision == CMPC_MLP_BF16
                 ? launch_adamw<bf16_t>(m.stream, m.W[l], m.mW[l], m.vW[l], m.dW[l],
                                        (bf16_t*)m.Wlow[l], lw, lr, o.beta1, o.beta2, o.eps,
                                        o.weight_decay, c1, c2)
                 : launch_adamw<float>(m.stream, m.W[l], m.mW[l], m.vW[l], m.dW[l],
                                       (float*)m.Wlow[l], lw, lr, o.beta1, o.beta2, o.eps,
                                       o.weight_decay, c1, c2);
    if (rc) return rc;
    rc = launch_adamw<float>(m.stream, m.b[l], m.mb[l], m.vb[l], m.db[l], (float*)nullptr,
                             m.wp[l], lr, o.beta1, o.beta2, o.eps, 0.0f, c1, c2);
    if (rc) return rc;
  }
  return 0;
}

// P0 of the backward Riccati recursion of the unconstrained problem:
//   P_N = Q_f;  S = R + B'P B;  T = B'P A;  K = S^-1 T;  P <- Q + A'P A - T'K.
// 1/2 x0'P_0 x0 is the minimum of the unconstrained QP, i.e. h0 - 1/2 h'H^-1 h.
static int riccati_p0(Mlp& m, const Problem& p) {
  const int ns = p.ns, nu = p.nu;
  int rc = 0;
  double* P = dalloc<double>((size_t)ns * ns, &rc);
  double* Pn = dalloc<double>((size_t)ns * ns, &rc);
  double* PA = dalloc<double>((size_t)ns * ns, &rc);
  double* PB = dalloc<double>((size_t)ns * nu, &rc);
  double* S = dalloc<double>((size_t)nu * nu, &rc);
  double* T = dalloc<double>((size_t)nu * ns, &rc);
  double* K = dalloc<double>((size_t)nu * ns, &rc);
  int* fail = dalloc<int>(1, &rc);
  hipStream_t s = m.stream;
  if (!rc && hipMemcpyAsync(P, p.Qf, sizeof(double) * ns * ns, hipMemcpyDeviceToDevice, s) !=
                 hipSuccess)
    rc = CMPC_ERR_HIP;
  for (int t = p.N - 1; t >= 0 && !rc; --t) {
    rc = launch_gemm_f64(s, ns, ns, ns, 1.0, P, ns, 1, p.A, ns, 1, 0.0, PA, ns);
    if (!rc) rc = launch_gemm_f64(s, ns, nu, ns, 1.0, P, ns, 1, p.B, nu, 1, 0.0, PB, nu);
    if (!rc && hipMemcpyAsync(S, p.R, sizeof(double) * nu * nu, hipMemcpyDeviceToDevice, s) !=
                   hipSuccess)
      rc = CMPC_ERR_HIP;
    if (!rc) rc = launch_gemm_f64(s, nu, nu, ns, 1.0, p.B, 1, nu, PB, nu, 1, 1.0, S, nu);
    if (!rc) rc = launch_gemm_f64(s, nu, ns, ns, 1.0, p.B, 1, nu, PA, ns, 1, 0.0, T, ns);
    if (!rc) rc = launch_small_spd_solve(s, S, nu, T, ns, K, fail);
    if (!rc && hipMemcpyAsync(Pn, p.Q, sizeof(double) * ns * ns, hipMemcpyDeviceToDevice, s) !=
                   hipSuccess)
      rc = CMPC_ERR_HIP;
    if (!rc) rc = launch_gemm_f64(s, ns, ns, ns, 1.0, p.A, 1, ns, PA, ns, 1, 1.0, Pn, ns);
    if (!rc) rc = launch_gemm_f64(s, ns, ns, nu, -1.0, T, 1, ns, K, ns, 1, 1.0, Pn, ns);
    if (!rc) rc = launch_symmetrize(s, Pn, ns);
    std::swap(P, Pn);
  }
  int hf = 0;
  if (!rc && (hipMemcpyAsync(&hf, fail, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess))
    rc = CMPC_ERR_HIP;
  if (!rc && hf) {
    set_error("surrogate judge: R + B'PB not positive definite");
    rc = CMPC_ERR_INVALID;
  }
  hipStreamSynchronize(s);
  for (double* x : {Pn, PA, PB, S, T, K}) hipFree(x);
  hipFree(fail);
  if (rc) {
    hipFree(P);
    return rc;
  }
  m.P0 = P;
  return 0;
}

__global__ void diag_of_kernel(const double* __restrict__ M, int n, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = M[(long long)i * n + i];
}

static int create_mlp(Problem* p, int hidden, int depth, int precision, const float* init,
                      Mlp** out) {
  if (!p || !init || !out || hidden <= 0 || hidden % 64 || depth < 1 || depth > 16) {
    set_error("surrogate: need a problem, initial parameters, hidden % 64 == 0, 1 <= depth <= 16");
    return CMPC_ERR_INVALID;
  }
  if (precision != CMPC_MLP_BF16 && precision != CMPC_MLP_FP32) {
    set_error("surrogate: precision must be CMPC_MLP_BF16 or CMPC_MLP_FP32");
    return CMPC_ERR_INVALID;
  }
  if (p->ns_real != p->ns || p->feedback || p->Sx != nullptr || p->wdist != nullptr) {
    set_error("surrogate judge: problems with S, E/F rows, w or a feedback are not supported");
    return CMPC_ERR_INVALID;
  }
  if (!p->q_diag) {
    set_error("surrogate judge: Q and Q_f must be diagonal");
    return CMPC_ERR_INVALID;
  }
  if (p->nu > 64 || p->ns > 3500) {
    set_error("surrogate judge: needs nu <= 64 and ns <= 3500");
    return CMPC_ERR_INVALID;
  }
  Mlp* m = new Mlp();
  m->precision = precision;
  m->ns = p->ns;
  m->nu = p->nu;
  m->N = p->N;
  m->n = p->n;
  m->depth = depth;
  m->hidden = hidden;
  m->prob = p;
  m->stream = p->stream;
  m->w.push_back(p->ns);
  for (int l = 0; l < depth; ++l) m->w.push_back(hidden);
  m->w.push_back(p->n);
  for (int x : m->w) m->wp.push_back(pad64(x));
  const int L1 = depth + 1;
  int rc = 0;
  for (auto* vec : {&m->W, &m->b, &m->mW, &m->vW, &m->mb, &m->vb, &m->dW, &m->db})
    vec->assign(L1 + 1, nullptr);
  m->Wlow.assign(L1 + 1, nullptr);
  m->z.assign(depth + 1, nullptr);
  int maxw = 0;
  for (int x : m->wp) maxw = std::max(maxw, x);
  for (int l = 1; l <= L1; ++l) {
    const size_t lw = (size_t)m->wp[l] * m->wp[l - 1];
    m->W[l] = dalloc<float>(lw, &rc);
    m->mW[l] = dalloc<float>(lw, &rc);
    m->vW[l] = dalloc<float>(lw, &rc);
    m->dW[l] = dalloc<float>(lw, &rc);
    m->b[l] = dalloc<float>(m->wp[l], &rc);
    m->mb[l] = dalloc<float>(m->wp[l], &rc);
    m->vb[l] = dalloc<float>(m->wp[l], &rc);
    m->db[l] = dalloc<float>(m->wp[l], &rc);
    m->Wlow[l] = dalloc<char>(lw * m->tsize(), &rc);
  }
  for (int l = 0; l <= depth; ++l) {
    m->a.push_back(dalloc<char>((size_t)kMlpRows * m->wp[l] * m->tsize(), &rc));
    if (l >= 1) m->z[l] = dalloc<float>((size_t)kMlpRows * m->wp[l], &rc);
  }
  m->y = dalloc<float>((size_t)kMlpRows * m->wp[L1], &rc);
  m->ut = dalloc<float>((size_t)kMlpRows * m->wp[L1], &rc);
  m->g[0] = dalloc<char>((size_t)kMlpRows * maxw * m->tsize(), &rc);
  m->g[1] = dalloc<char>((size_t)kMlpRows * maxw * m->tsize(), &rc);
  m->part_cap = (int)(((long long)kMlpRows * m->wp[L1] + 255) / 256);
  m->part = dalloc<double>(m->part_cap, &rc);
  m->q = dalloc<double>(p->ns, &rc);
  m->qf = dalloc<double>(p->ns, &rc);
  if (rc) {
    free_mlp(m);
    return rc;
  }
  hipLaunchKernelGGL(diag_of_kernel, dim3(ceil_div(p->ns, 256)), dim3(256), 0, m->stream, p->Q,
                     p->ns, m->q);
  hipLaunchKernelGGL(diag_of_kernel, dim3(ceil_div(p->ns, 256)), dim3(256), 0, m->stream, p->Qf,
                     p->ns, m->qf);
  if (hipGetLastError() != hipSuccess) rc = CMPC_ERR_HIP;
  if (!rc) rc = set_params(*m, init);
  if (!rc) rc = riccati_p0(*m, *p);
  if (rc) {
    free_mlp(m);
    return rc;
  }
  *out = m;
  return 0;
}

static int ensure_judge_cap(Mlp& m, int count) {
  if (count <= m.jcap) return 0;
  for (double** x : {&m.jf, &m.jv, &m.jl, &m.jg})
    if (*x) hipFree(*x);
  if (m.jacc) hipFree(m.jacc);
  int rc = 0;
  m.jf = dalloc<double>(count, &rc);
  m.jv = dalloc<double>(count, &rc);
  m.jl = dalloc<double>(count, &rc);
  m.jg = dalloc<double>(count, &rc);
  m.jacc = dalloc<int>(count, &rc);
  if (rc) {
    m.jcap = 0;
    return rc;
  }
  m.jcap = count;
  return 0;
}

// Judge answers U (device, count x n) for initial states X0 (device, count x ns).
static int judge(Mlp& m, const double* X0, const double* U, int count) {
  int rc = ensure_judge_cap(m, count);
  if (rc) return rc;
  const Problem& p = *m.prob;
  rc = launch_judge_sim(m.stream, X0, U, count, p.ns, p.nu, p.N, p.a_rowptr, p.a_col, p.a_val,
                        p.A, p.B, m.q, m.qf, p.R, p.xl, p.xu, m.jf, m.jv);
  if (!rc) rc = launch_judge_lb(m.stream, X0, count, p.ns, m.P0, m.jl);
  if (!rc)
    rc = launch_judge_decide(m.stream, m.jf, m.jv, m.jl, count, CMPC_JUDGE_VIOLATION,
                             CMPC_JUDGE_GAP, m.jacc, m.jg);
  return rc;
}

static int predict(Mlp& m, const double* X0, int count, double* U) {
  const Problem& p = *m.prob;
  for (int c0 = 0; c0 < count; c0 += kMlpRows) {
    const int rows = std::min(kMlpRows, count - c0);
    const int Mp = pad64(rows);
    int rc = stage(m, X0 + (size_t)c0 * m.ns, nullptr, nullptr, rows, Mp);
    if (!rc) rc = forward(m, Mp);
    if (!rc)
      rc = launch_clip_out(m.stream, m.y, m.wp[m.depth + 1], rows, m.n, m.nu, p.ul, p.uu,
                           U + (size_t)c0 * m.n);
    if (rc) return rc;
  }
  return 0;
}

static int train(Mlp& m, const double* X, const double* U, int count, const cmpc_train_opts& o,
                 const int* order, double* epoch_loss) {
  if (count <= 0 || o.batch <= 0 || o.batch > kMlpRows || o.epochs < 0) {
    set_error("surrogate training: need count > 0 and 0 < batch <= 4096");
    return CMPC_ERR_INVALID;
  }
  const int steps_per_epoch = (count + o.batch - 1) / o.batch;
  const long long total = (long long)steps_per_epoch * o.epochs;
  int rc = 0;
  if (count > m.idx_cap) {
    if (m.idx) hipFree(m.idx);
    m.idx = dalloc<int>(count, &rc);
    if (rc) return rc;
    m.idx_cap = count;
  }
  if (steps_per_epoch > m.steploss_cap) {
    if (m.steploss) hipFree(m.steploss);
    m.steploss = dalloc<double>(steps_per_epoch, &rc);
    if (rc) return rc;
    m.steploss_cap = steps_per_epoch;
  }
  std::vector<int> seq(count);
  for (int i = 0; i < count; ++i) seq[i] = i;
  std::vector<double> sl(steps_per_epoch);
  long long k = 0;
  for (int ep = 0; ep < o.epochs; ++ep) {
    const int* ord = order ? order + (size_t)ep * count : seq.data();
    for (int i = 0; i < count; ++i)
      if (ord[i] < 0 || ord[i] >= count) {
        set_error("surrogate training: order holds an index outside [0, count)");
        return CMPC_ERR_INVALID;
      }
    CMPC_HIP(hipMemcpyAsync(m.idx, ord, sizeof(int) * count, hipMemcpyHostToDevice, m.stream));
    for (int st = 0; st < steps_per_epoch; ++st, ++k) {
      const int r0 = st * o.batch, rows = std::min(o.batch, count - r0);
      const int Mp = pad64(rows);
      // cosine decay from lr to lr_final over all steps
      const double frac = total > 1 ? (double)k / (double)(total - 1) : 0.0;
      const float lr = (float)(o.lr_final + 0.5 * (o.lr - o.lr_final) * (1.0 + std::cos(M_PI * frac)));
      rc = stage(m, X, U, m.idx + r0, rows, Mp);
      if (!rc) rc = forward(m, Mp);
      if (!rc) rc = backward(m, Mp, rows, m.steploss + st);
      if (!rc) rc = adamw_all(m, lr, o);
      if (rc) return rc;
    }
    CMPC_HIP(hipMemcpyAsync(sl.data(), m.steploss, sizeof(double) * steps_per_epoch,
                            hipMemcpyDeviceToHost, m.stream));
    CMPC_HIP(hipStreamSynchronize(m.stream));  // the host order buffer may be reused
    if (epoch_loss) {
      double s = 0.0;
      for (int st = 0; st < steps_per_epoch; ++st) {
        const int rows = std::min(o.batch, count - st * o.batch);
        s += sl[st] * rows;
      }
      epoch_loss[ep] = s / count;
    }
  }
  return 0;
}

}  // namespace cmpc

using namespace cmpc;

struct cmpc_mlp {
  Mlp* m;
};

extern "C" {

void cmpc_default_train_opts(cmpc_train_opts* o) {
  if (!o) return;
  o->batch = 512;
  o->epochs = 20;
  o->lr = 1e-3f;
  o->lr_final = 1e-5f;
  o->beta1 = 0.9f;
  o->beta2 = 0.999f;
  o->eps = 1e-8f;
  o->weight_decay = 1e-4f;
}

int cmpc_mlp_create(cmpc_problem* p, int hidden, int depth, int precision, const float* init,
                    cmpc_mlp** out) {
  if (!out) {
    set_error("NULL output");
    return CMPC_ERR_INVALID;
  }
  *out = nullptr;
  if (!p) {
    set_error("NULL problem");
    return CMPC_ERR_INVALID;
  }
  Mlp* m = nullptr;
  const int rc = create_mlp(p->p, hidden, depth, precision, init, &m);
  if (rc) return rc;
  *out = new cmpc_mlp{m};
  return 0;
}

void cmpc_mlp_destroy(cmpc_mlp* h) {
  if (!h) return;
  free_mlp(h->m);
  delete h;
}

long long cmpc_mlp_param_count(const cmpc_mlp* h) { return h ? param_count(*h->m) : 0; }

int cmpc_mlp_get_params(const cmpc_mlp* h, float* params) {
  if (!h || !params) {
    set_error("NULL argument");
    return CMPC_ERR_INVALID;
  }
  CMPC_HIP(hipStreamSynchronize(h->m->stream));
  return get_padded(*h->m, h->m->W, h->m->b, params);
}

int cmpc_mlp_set_params(cmpc_mlp* h, const float* params) {
  if (!h || !params) {
    set_error("NULL argument");
    return CMPC_ERR_INVALID;
  }
  return set_params(*h->m, params);
}

int cmpc_mlp_gradients(cmpc_mlp* h, const double* x0s, const double* ustars, int count,
                       float* grads, double* loss, float* y) {
  if (!h || !x0s || !ustars || count <= 0 || count > kMlpRows) {
    set_error("need 0 < count <= 4096 and device inputs");
    return CMPC_ERR_INVALID;
  }
  Mlp& m = *h->m;
  const int Mp = pad64(count);
  double* dl = nullptr;
  CMPC_HIP(hipMalloc(&dl, sizeof(double)));
  int rc = stage(m, x0s, ustars, nullptr, count, Mp);
  if (!rc) rc = forward(m, Mp);
  if (!rc) rc = backward(m, Mp, count, dl);
  double hl = 0.0;
  if (!rc && (hipMemcpyAsync(&hl, dl, sizeof(double), hipMemcpyDeviceToHost, m.stream) !=
                  hipSuccess ||
              hipStreamSynchronize(m.stream) != hipSuccess))
    rc = CMPC_ERR_HIP;
  hipFree(dl);
  if (rc) return rc;
  if (loss) *loss = hl;
  if (grads) rc = get_padded(m, m.dW, m.db, grads);
  if (!rc && y) {
    const int ld = m.wp[m.depth + 1];
    std::vector<float> yp((size_t)count * ld);
    CMPC_HIP(hipMemcpy(yp.data(), m.y, sizeof(float) * yp.size(), hipMemcpyDeviceToHost));
    for (int r = 0; r < count; ++r)
      std::memcpy(y + (size_t)r * m.n, &yp[(size_t)r * ld], sizeof(float) * m.n);
  }
  return rc;
}

int cmpc_mlp_train(cmpc_mlp* h, const double* x0s, const double* ustars, int count,
                   const cmpc_train_opts* opts, const int* order, double* epoch_loss) {
  if (!h || !x0s || !ustars) {
    set_error("NULL argument");
    return CMPC_ERR_INVALID;
  }
  cmpc_train_opts o;
  cmpc_default_train_opts(&o);
  if (opts) o = *opts;
  return train(*h->m, x0s, ustars, count, o, order, epoch_loss);
}

int cmpc_mlp_predict(cmpc_mlp* h, const double* x0s, int count, double* u) {
  if (!h || !x0s || !u || count < 0) {
    set_error("invalid argument");
    return CMPC_ERR_INVALID;
  }
  const int rc = predict(*h->m, x0s, count, u);
  if (rc) return rc;
  CMPC_HIP(hipStreamSynchronize(h->m->stream));
  return 0;
}

int cmpc_judge(cmpc_mlp* h, const double* x0s, const double* u, int count, int* accepted,
               double* violation, double* f, double* lb) {
  if (!h || !x0s || !u || count < 0) {
    set_error("invalid argument");
    return CMPC_ERR_INVALID;
  }
  Mlp& m = *h->m;
  int rc = judge(m, x0s, u, count);
  if (rc) return rc;
  const hipStream_t s = m.stream;
  if (accepted)
    CMPC_HIP(hipMemcpyAsync(accepted, m.jacc, sizeof(int) * count, hipMemcpyDeviceToHost, s));
  if (violation)
    CMPC_HIP(hipMemcpyAsync(violation, m.jv, sizeof(double) * count, hipMemcpyDeviceToHost, s));
  if (f) CMPC_HIP(hipMemcpyAsync(f, m.jf, sizeof(double) * count, hipMemcpyDeviceToHost, s));
  if (lb) CMPC_HIP(hipMemcpyAsync(lb, m.jl, sizeof(double) * count, hipMemcpyDeviceToHost, s));
  CMPC_HIP(hipStreamSynchronize(s));
  return 0;
}

int cmpc_mlp_set_fallback(cmpc_mlp* h, cmpc_batch* batch, int warm) {
  if (!h) {
    set_error("NULL network");
    return CMPC_ERR_INVALID;
  }
  Mlp& m = *h->m;
  if (batch != nullptr) {
    const int R = cmpc_batch_size(batch);
    if (R <= 0) {
      set_error("cmpc_mlp_set_fallback: empty batch");
      return CMPC_ERR_INVALID;
    }
    for (int i = 0; i < R; ++i) {
      const Problem& q = *cmpc_batch_instance(batch, i)->p;
      if (q.ns != m.prob->ns || q.nu != m.prob->nu || q.N != m.prob->N) {
        set_error("cmpc_mlp_set_fallback: instance " + std::to_string(i) +
                  " is not a copy of the network's problem (ns, nu, N differ)");
        return CMPC_ERR_INVALID;
      }
    }
  }
  m.fb = batch;
  m.fb_warm = warm != 0;
  return 0;
}

int cmpc_surrogate_solve(cmpc_mlp* h, const double* x0s, int count, double* u, int* accepted,
                         cmpc_surrogate_report* rep) {
  if (!h || !x0s || !u || count < 0) {
    set_error("invalid argument");
    return CMPC_ERR_INVALID;
  }
  Mlp& m = *h->m;
  Problem& p = *m.prob;
  const hipStream_t s = m.stream;
  hipEvent_t e0, e1, e2;
  CMPC_HIP(hipEventCreate(&e0));
  CMPC_HIP(hipEventCreate(&e1));
  CMPC_HIP(hipEventCreate(&e2));
  const auto t0 = std::chrono::steady_clock::now();
  int rc = hipEventRecord(e0, s) == hipSuccess ? 0 : CMPC_ERR_HIP;
  if (!rc) rc = predict(m, x0s, count, u);
  if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = CMPC_ERR_HIP;
  if (!rc) rc = judge(m, x0s, u, count);
  if (!rc && hipEventRecord(e2, s) != hipSuccess) rc = CMPC_ERR_HIP;
  std::vector<int> acc(std::max(1, count));
  std::vector<double> vio(std::max(1, count)), gap(std::max(1, count));
  if (!rc && (hipMemcpyAsync(acc.data(), m.jacc, sizeof(int) * count, hipMemcpyDeviceToHost, s) !=
                  hipSuccess ||
              hipMemcpyAsync(vio.data(), m.jv, sizeof(double) * count, hipMemcpyDeviceToHost, s) !=
                  hipSuccess ||
              hipMemcpyAsync(gap.data(), m.jg, sizeof(double) * count, hipMemcpyDeviceToHost, s) !=
                  hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess))
    rc = CMPC_ERR_HIP;
  float ms_inf = 0.f, ms_judge = 0.f;
  if (!rc) {
    hipEventElapsedTime(&ms_inf, e0, e1);
    hipEventElapsedTime(&ms_judge, e1, e2);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipEventDestroy(e2);
  if (rc) return rc;
  const auto t1 = std::chrono::steady_clock::now();
  int n_acc = 0, fb_ok = 0, fb_fail = 0;
  double max_vio = 0.0, max_gap = 0.0;
  cmpc_options o;
  cmpc_default_options(&o);
  std::vector<int> rejected;
  for (int q = 0; q < count; ++q) {
    if (acc[q]) {
      ++n_acc;
      max_vio = std::max(max_vio, vio[q]);
      max_gap = std::max(max_gap, gap[q]);
    } else {
      rejected.push_back(q);
    }
  }
  if (m.fb == nullptr) {
    // Algorithm 1 from each rejected x0 (FP64) on the network's problem, one after another;
    // its controls replace the answer
    for (int q : rejected) {
      rc = set_x0(p, x0s + (size_t)q * p.ns, 1);
      if (rc) return rc;
      cmpc_result r;
      if (m.fb_warm)
        CMPC_HIP(hipMemcpyAsync(p.v, u + (size_t)q * p.n, sizeof(double) * p.n,
                                hipMemcpyDeviceToDevice, p.stream));
      const int st = solve(p, o, &r, m.fb_warm);
      if (st == CMPC_OK) {
        ++fb_ok;
        CMPC_HIP(hipMemcpyAsync(u + (size_t)q * p.n, p.v, sizeof(double) * p.n,
                                hipMemcpyDeviceToDevice, p.stream));
      } else {
        ++fb_fail;
        if (st < 0) return st;
      }
    }
  } else {
    // the rejected queries in groups of count(batch), one batched solve per group (the last
    // group's empty places repeat its last query; their results are not used)
    const int R = cmpc_batch_size(m.fb);
    std::vector<const double*> v0s(R);
    std::vector<cmpc_result> res(R);
    for (size_t g0 = 0; g0 < rejected.size(); g0 += R) {
      const int len = (int)std::min<size_t>(R, rejected.size() - g0);
      for (int i = 0; i < R; ++i) {
        const int q = rejected[g0 + std::min(i, len - 1)];
        cmpc_problem* inst = cmpc_batch_instance(m.fb, i);
        rc = set_x0(*inst->p, x0s + (size_t)q * p.ns, 1);
        if (rc) return rc;
        v0s[i] = u + (size_t)q * p.n;
      }
      const int st = m.fb_warm ? cmpc_batch_solve_warm(m.fb, &o, v0s.data(), 1, res.data())
                               : cmpc_batch_solve(m.fb, &o, res.data());
      if (st < 0 && st != CMPC_ERR_CHOLESKY) return st;
      for (int i = 0; i < len; ++i) {
        const int q = rejected[g0 + i];
        if (res[i].status == CMPC_OK) {
          ++fb_ok;
          Problem& ip = *cmpc_batch_instance(m.fb, i)->p;
          CMPC_HIP(hipMemcpyAsync(u + (size_t)q * p.n, ip.v, sizeof(double) * p.n,
                                  hipMemcpyDeviceToDevice, ip.stream));
        } else {
          ++fb_fail;
        }
      }
      CMPC_HIP(hipStreamSynchronize(cmpc_batch_instance(m.fb, 0)->p->stream));
    }
  }
  CMPC_HIP(hipStreamSynchronize(p.stream));
  const auto t2 = std::chrono::steady_clock::now();
  if (accepted) std::memcpy(accepted, acc.data(), sizeof(int) * count);
  if (rep) {
    rep->count = count;
    rep->accepted = n_acc;
    rep->fallback_solved = fb_ok;
    rep->fallback_failed = fb_fail;
    rep->max_violation_accepted = max_vio;
    rep->max_gap_accepted = max_gap;
    rep->ms_infer = ms_inf;
    rep->ms_judge = ms_judge;
    rep->ms_fallback = std::chrono::duration<double, std::milli>(t2 - t1).count();
    rep->ms_total = std::chrono::duration<double, std::milli>(t2 - t0).count();
  }
  return fb_fail ? CMPC_MAX_ITER : 0;
}

}  // extern "C"
