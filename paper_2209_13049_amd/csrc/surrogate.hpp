// Surrogate policy: kernel launchers (k_mlp.hip) shared with the host driver (surrogate.hip).
#pragma once

#include "problem.hpp"

namespace cmpc {

// GEMM kinds of the multilayer perceptron (C(i, j) = sum_r A(i, r) B(j, r)):
//   FwdGelu   Z = A W' + b, H = T(gelu(Z))    (A: activations, B: weights, both r-contiguous)
//   FwdLinear Y = A W' + b                    (last layer, float output)
//   BwdData   G = T((G_next W) * gelu'(Z))    (A: G_next r-contiguous, B: W i-contiguous)
//   BwdWeight dW = G' A                       (both operands i-contiguous, float output)
enum { kGemmFwdGelu = 0, kGemmFwdLinear = 1, kGemmBwdData = 2, kGemmBwdWeight = 3 };
enum { kEpiGelu = 0, kEpiLinear = 1, kEpiDGelu = 2, kEpiF32 = 3 };

struct MlpEpi {
  const float* bias = nullptr;  // FwdGelu, FwdLinear
  float* z = nullptr;           // FwdGelu: pre-activation; FwdLinear: output; BwdWeight: dW
  int ldz = 0;
  void* h = nullptr;            // FwdGelu: activation (T); BwdData: gradient (T)
  int ldh = 0;
  const float* zin = nullptr;   // BwdData: pre-activation of the layer the gradient enters
  int ldzi = 0;
};

template <typename T>
int launch_mlp_gemm(hipStream_t s, int kind, const T* A, int lda, const T* B, int ldb, int M,
                    int N, int K, const MlpEpi& e);
template <typename T>
int launch_stage_rows(hipStream_t s, const double* X, int ld_x, int ncols, const int* idx,
                      int rows, T* out, int ldo, int Mp);
template <typename T>
int launch_mse_grad(hipStream_t s, const float* Y, int ldy, const float* U, int ldu, int rows,
                    int ncols, T* G, int ldg, int Mp, double* part, int* nparts);
int launch_sum_parts(hipStream_t s, const double* part, int n, double denom, double* out);
template <typename T>
int launch_colsum(hipStream_t s, const T* G, int ldg, int rows, int ncols, float* db);
template <typename T>
int launch_adamw(hipStream_t s, float* w, float* m, float* v, const float* g, T* wlow,
                 long long len, float lr, float b1, float b2, float eps, float wd, float c1,
                 float c2);
template <typename T>
int launch_to_low(hipStream_t s, const float* in, T* out, long long len);
int launch_clip_out(hipStream_t s, const float* Y, int ldy, int rows, int n, int nu,
                    const double* ul, const double* uu, double* out);
int launch_judge_sim(hipStream_t s, const double* X0, const double* U, int count, int ns, int nu,
                     int N, const int* arp, const int* acol, const double* aval,
                     const double* Adense, const double* B, const double* q, const double* qf,
                     const double* R, const double* xl, const double* xu, double* f,
                     double* vio);
int launch_judge_lb(hipStream_t s, const double* X0, int count, int ns, const double* P,
                    double* lb);
int launch_judge_decide(hipStream_t s, const double* f, const double* vio, const double* lb,
                        int count, double vtol, double gtol, int* accept, double* gap);
int launch_small_spd_solve(hipStream_t s, const double* S, int nu, const double* T, int ns,
                           double* K, int* fail);
int launch_symmetrize(hipStream_t s, double* P, int n);

}  // namespace cmpc
