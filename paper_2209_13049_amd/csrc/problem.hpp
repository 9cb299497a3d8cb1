// Device-resident problem, IPM workspace and the launchers of every kernel family.
#pragma once

#include <vector>

#include "common.hpp"
#include "condmpc.h"

namespace cmpc {

// Interior-point scalars kept on the device so that one iteration needs no host round trip.
struct IpmState {
  double mu, tau, alpha, alpha_z;
  double nr1, nr3, nlz, szmax, szmin, err0;  // norms at the top of the current iteration
  double tol, mu_min, h0, obj, gap;
  int iter;      // steps taken
  int status;    // CMPC_* outcome once done
  int done;      // nonzero: every later kernel of the solve returns at entry
  int info;      // Cholesky: 1-based failing column
  int max_iter;
  int use_low;   // mixed modes: precision level of the SYRK (2 BF16, 1 FP32, 0 FP64)
  int switch_iter;
  int refine_steps;
  int nonc;      // mixed modes: refinement failures so far
  int x0_flag;   // device x0 check: 1 = outside the bounds, 2 = not finite
  int ref_skip;  // mixed modes: nonzero = no (more) refinement in this iteration
  int mixed;     // starting precision level of the solve (0 = plain FP64)
  double mu_switch, res_prev;
  double contract;  // mixed modes: a refinement step must shrink |res| below contract x the last
};

constexpr int kRunning = 100;

// Snapshot of one iteration for the host's log callback (written by the iteration's last
// kernel into a mapped pinned ring next to its flag).
struct IterLog {
  int iter, level, done, pad;
  double mu, err0, nr1, nr3, nlz, szmax, alpha, alpha_z;
};

// One split-K job of the SYRK: rows [r0, r1) of row block t (1-based) contribute to
// output tile `tile`; slot >= 0 means the accumulator is written to partial slot `slot`
// after this job and cleared.
struct SyrkJob {
  int tile, t, r0, r1, slot;
};

struct SyrkPlan {
  int nt = 0, ntiles = 0, nwg = 0, nslots = 0;
  int quantum = 0;               // least work per workgroup (row x 16-block units, see syrk_plan)
  int2* tiles = nullptr;         // (I, J) tile coordinates, I >= J, 64 x 64 tiles
  SyrkJob* jobs = nullptr;
  int* wg_begin = nullptr;       // nwg + 1
  int* slot_begin = nullptr;     // ntiles + 1 (CSR of partial slots per tile)
  int* slots = nullptr;
  double* partials = nullptr;    // nslots x 4096
  double flops_structural = 0;   // algorithmic FLOPs of one SYRK (structural nonzeros)
};

struct Problem {
  int ns = 0, nu = 0, N = 0, n = 0, mx = 0, m = 0;
  // general data folded in (capi.hip: fold_general): ns counts the problem's own ns_real
  // states and nz extra stage rows (input bounds under a feedback, E x + F u)
  int ns_real = 0, nz = 0;
  bool feedback = false;          // u = K x + v: the inputs are the first nu extra rows
  double* Sx = nullptr;           // cross weight S~ (ns x nu) of the stage cost, or NULL
  double* wdist = nullptr;        // disturbance w_t (N x ns), or NULL
  hipStream_t stream = nullptr;
  bool q_diag = false;
  // problem data (device)
  double *A = nullptr, *B = nullptr, *Q = nullptr, *Qf = nullptr, *R = nullptr;
  double *xl = nullptr, *xu = nullptr, *ul = nullptr, *uu = nullptr;
  double *qdiag = nullptr;       // diag(Qbar), length mx (diagonal weights only)
  // Gamma is never formed: it is block Toeplitz (block (t, j) = G_{t-1-j}), so every pass
  // over it reads only the N blocks G_m.
  double *G = nullptr;           // G_m = A^m B, m = 0..N-1: N x ns x nu (the SYRK's operand)
  double *Gt = nullptr;          // Gt[(m nu + k) ns + i] = G_m[i][k]: n x ns (Gamma products)
  float* G32 = nullptr;          // FP32 copy of G (mixed modes)
  unsigned short* G16 = nullptr; // BF16 copy of G (mixed modes)
  double *H = nullptr;           // n x n, full symmetric
  double *Wdiag = nullptr;       // inverses of the diagonal 64 x 64 factor tiles
  double *eqs = nullptr;         // equilibration scales diag(K)^-1/2 (n)
  double *K = nullptr;           // n x n workspace (lower triangle = condensed matrix / factor)
  int *a_rowptr = nullptr, *a_col = nullptr;  // CSR copy of A when it is sparse
  double* a_val = nullptr;
  int a_maxnnz = 0;  // most nonzeros in a row of that copy
  double *red_part = nullptr;    // 1024 partial sums
  double *x0 = nullptr, *c = nullptr, *qc = nullptr, *h = nullptr, *d = nullptr;
  bool have_x0 = false;
  bool have_solution = false;     // p.v holds the controls of a finished solve
  // iterate
  double *v = nullptr, *s = nullptr, *lam = nullptr, *z = nullptr, *gv = nullptr;
  // step and work vectors
  double *pv = nullptr, *ps = nullptr, *plam = nullptr, *pz = nullptr, *gpv = nullptr;
  double *rhs = nullptr, *Dx = nullptr, *Du = nullptr, *wx = nullptr, *wu = nullptr;
  double *gt = nullptr, *Hv = nullptr, *tmpn = nullptr, *tmpn2 = nullptr, *tmpmx = nullptr;
  double *ref_res = nullptr, *ref_dlt = nullptr;  // refinement vectors (n)
  double *norm_part = nullptr, *alpha_part = nullptr, *gt_part = nullptr;
  int n_prep_blocks = 0, n_step_blocks = 0, gt_chunks = 0;
  bool eq_on = false;               // this solve factors the equilibrated S K S
  IpmState* st = nullptr;
  SyrkPlan syrk;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<hipEvent_t> prof_ev;  // per iteration: SYRK begin/end, Cholesky begin/end
  int* hflags = nullptr;            // mapped pinned ring: 0 pending, 1 running, 2 done
  int* dflags = nullptr;            // device alias of hflags
  IterLog* hlog = nullptr;          // mapped pinned ring of iteration snapshots (log callback)
  IterLog* dlog = nullptr;          // device alias of hlog
  std::vector<double> xl_host, xu_host;
};

// ---- host driver (capi.hip) and tuning table (batch.hip) ----
int create(const cmpc_lq_desc* desc, hipStream_t stream, Problem** out);
void free_problem(Problem* p);
int set_x0(Problem& p, const double* x0, int on_device);
int solve(Problem& p, const cmpc_options& o, cmpc_result* res, int warm = 0);
// Rebuild the SYRK plan if the tuning table holds another work quantum for
// (n, mx, precision); *changed tells whether it did.
int ensure_plan(Problem& p, int precision, bool* changed);

// ---- batches ----
// One instance as the work-list kernels see it (an array of these lives in device memory).
struct InstView {
  int ns, nu, N, n, mx, m;
  int nblk;                      // 256-pair blocks of the vector kernels
  int gt_chunks;
  int nt;                        // ceil(n / 64)
  int syrk_nwg;
  const double* G;
  const double* Gt;
  const float* G32;
  const bf16_t* G16;
  const double *H, *d, *h;
  double *K, *Wdiag, *eqs;
  double *v, *s, *lam, *z, *gv, *pv, *ps, *plam, *pz, *gpv;
  double *rhs, *Dx, *Du, *wx, *wu, *gt, *Hv, *tmpn;
  double *ref_res, *ref_dlt;
  double *norm_part, *alpha_part, *gt_part;
  IpmState* st;
  const SyrkJob* jobs;
  const int* wg_begin;
  const int2* tiles;
  double* partials;
  const int *slot_begin, *slots;
};

// Gamma' passes through Gt (Gamma block (t, j) = G_{t-1-j}, so (Gamma' w)_j = sum_{m<N-j} G_m' w_{m+j+1}):
// one workgroup per (range of kGtJ column blocks j, column k within a block, 256 rows i, part
// of the range of m).
// Each workgroup's range of m is split in kGtMs parts (shorter dependent chains).
constexpr int kGtJ = 8;
constexpr int kGtMs = 2;
__host__ __device__ inline int gt_row_chunks(int ns) { return (ns + 255) / 256; }
inline int gt_chunk_count(int ns, int nu, int N) {
  return ((N + kGtJ - 1) / kGtJ) * nu * gt_row_chunks(ns) * kGtMs;
}
// Gamma x through the blocks of Gamma: block (t, j) is G_{t-1-j} = A^(t-1-j) B (zero for
// j >= t), so Gamma is block Toeplitz and (Gamma x)_t = sum_{m<t} G_m x_{t-1-m}, read from Gt
// (n x ns, rows e = m nu + k).  One workgroup per (group of MT row blocks, 64 rows); the
// blocks of a group share the rows of Gt.  A single solve uses MT = kMvT = 1 (groups of 2 and
// 4 were measured slower at n = 500: longer chains per wavefront); a batch, whose instances
// already fill the chip, uses kMvTBatch = 4 and reads a quarter of the rows.  The order of
// every sum does not depend on MT, so both give the same bits.
constexpr int kMvT = 1;
constexpr int kMvTBatch = 4;
template <int MT = kMvT>
__host__ __device__ inline int gmv_blocks(int ns, int N) {
  return ((ns + 63) / 64) * ((N + MT - 1) / MT);
}

// One entry of a work list: block `local` of instance `inst`.
struct WorkItem {
  int inst, local;
};

// Gate of a work-list kernel: 0 = the solve (st->done), 1 = the refinement (st->ref_skip).
__device__ inline const int* gate_of(const InstView& V, int gate) {
  return gate ? &V.st->ref_skip : &V.st->done;
}

// Loop of a work-list kernel over items[0, nitems) with stride gridDim.x (persistent when
// the grid is smaller than the list).  The barrier at the top separates the LDS use of
// consecutive items; V is the item's instance and bid its block index in that instance.
#define CMPC_ITEMS_BEGIN                                                  \
  for (int w_ = blockIdx.x; w_ < nitems; w_ += gridDim.x) {              \
    __syncthreads();                                                      \
    const WorkItem it_ = items[w_];                                       \
    const InstView& V = views[it_.inst];                                  \
    const int bid = it_.local;
#define CMPC_ITEMS_END }

// A work list as handed to a launcher: items [0, count) of the batch's device list; grid =
// count, or (persistent) at most the resident workgroups of the kernel on `cus` CUs.
struct ListArg {
  const InstView* views;
  const WorkItem* items;
  int count;
  int persistent;
  int cus;
  hipStream_t stream;
};
int occupancy_per_cu(const void* kernel);  // resident 256-thread workgroups per CU
inline int grid_for(const ListArg& L, const void* kernel) {
  if (!L.persistent) return L.count;
  const int cap = occupancy_per_cu(kernel) * L.cus;
  return L.count < cap ? L.count : (cap > 0 ? cap : 1);
}

// Launch a work-list kernel (arguments: views, items, count, then the extra ones) and return.
#define CMPC_LAUNCH_LIST(kernel, L, ...)                                                   \
  do {                                                                                     \
    if ((L).count > 0) {                                                                   \
      hipLaunchKernelGGL(kernel, dim3(grid_for((L), (const void*)(kernel))), dim3(256), 0, \
                         (L).stream, (L).views, (L).items, (L).count, ##__VA_ARGS__);      \
      CMPC_LAUNCH_CHECK();                                                                 \
    }                                                                                      \
    return 0;                                                                              \
  } while (0)

// ---- work-list launchers (k_ipm.hip, k_syrk.hip, k_chol.hip); a list of length 0 launches
// nothing.  gate / which: 0 = the solve, 1 = the refinement (see gate_of).
int launch_b_init(const ListArg& L, double tol, int max_iter, int low, double mu_switch,
                  double contract, int warm = 0, double mu0 = 0.0);
int launch_b_prep(const ListArg& L);
int launch_b_gamma_t_partial(const ListArg& L, int nv);
int launch_b_hv(const ListArg& L, int gate);
int launch_b_mu_rhs(const ListArg& L);
// gate 0: gpv = Gamma pv under st->done; 1: the same under st->ref_skip; 2: gv = Gamma v for
// every instance (the warm start)
int launch_b_gamma_mv(const ListArg& L, int gate);
int launch_b_step(const ListArg& L);
int launch_b_update(const ListArg& L);
int launch_b_refine_check(const ListArg& L);
int launch_b_axpy(const ListArg& L);
int launch_b_publish(hipStream_t s, const InstView* views, int count, int* iter, int* flags,
                     int ring);
int launch_b_reset(hipStream_t s, int* iter);
int launch_b_gather(hipStream_t s, const InstView* views, int count, IpmState* out);
int launch_b_syrk(const ListArg& L, int fp32, int mixed, int want_low);
int launch_b_finish(const ListArg& L);
int launch_b_equilibrate(const ListArg& Ln256, const ListArg& Ln4);
int launch_b_chol_first(const ListArg& L, int mixed);
int launch_b_chol_step(const ListArg& L, int k, int mixed, int fused, int eq);
int launch_b_potrs_copy(const ListArg& L, int which, int dir, int eq);
// the whole solve of each instance of the list (one item per instance) in one workgroup;
// nmax: the largest n of the batch (LDS size)
int launch_b_potrs_single(const ListArg& L, int which, int eq, int nmax, int fused);
int launch_b_trsv_fwd(const ListArg& L, int k, int which);
int launch_b_trsv_bwd(const ListArg& L, int k, int which);

// ---- setup kernels (k_build.hip) ----
int launch_gemm_f64(hipStream_t s, int M, int Nc, int Kd, double alpha, const double* A,
                    long long a_i, long long a_k, const double* B, long long b_k, long long b_j,
                    double beta, double* C, long long ldc);
// Row block t (1..N) of Gamma, ns x (t nu) row-major, into out (setup only).
int launch_gamma_block(Problem& p, int t, double* out);
int launch_transpose_g(Problem& p);
int launch_gemv(hipStream_t s, const double* A, const double* x, double* y, int rows, int cols);
int launch_block_diag_weight(Problem& p, const double* in, double* out);
int launch_make_d(Problem& p);
int launch_h0(Problem& p);
int launch_free_response(Problem& p);
int launch_check_x0(Problem& p);
// h += S~' c_t on the block of stage t (t = 0..N-1, c_0 = x0): the linear part of the cross
// term of the stage cost
int launch_h_cross(Problem& p);
// H(j, t) += G_{t-1-j}' S~ and its transpose (0 <= j < t <= N-1): the quadratic part
int launch_cross_hessian(Problem& p, const double* S);
// u (inputs, nu N) and x (the problem's own states, ns_real N) from v and xa = c + Gamma v
int launch_unfold_solution(Problem& p, const double* xa, double* u, double* x);
int launch_rbar(Problem& p, double* Hb);
int launch_mirror_lower(hipStream_t s, double* H, int n);
int launch_dense_gamma(Problem& p, double* dense);

// ---- SYRK (k_syrk.hip) ----
constexpr int kSyrkQuantumDefault = 12000;
int syrk_plan(Problem& p, int quantum = kSyrkQuantumDefault);
void syrk_free(SyrkPlan& sp);
// K(lower) = Hbase(lower) + Gamma' diag(Drow) Gamma + diag(Ddiag)   (Ddiag may be NULL)
// ev_start / ev_stop (optional): timing events attached to the split-K kernel's dispatch.
// precision CMPC_FP64 or CMPC_FP32_SYRK; mixed != 0 queues both variants, each running only
// when the device flag st->use_low selects it.
int launch_syrk(Problem& p, int precision, const double* Drow, const double* Hbase,
                const double* Ddiag, double* K, hipEvent_t ev_start = nullptr,
                hipEvent_t ev_stop = nullptr, int mixed = 0);
int launch_convert_gamma(Problem& p, int precision);

// ---- Cholesky (k_chol.hip) ----
// Wall: wall_doubles(n) doubles: the inverses of the diagonal factor tiles (ceil(n/64) x 64 x
// 64), then 8 per tile of condition figures (per wavefront max |L_kk| and max |W_k|) that
// decide whether the panel of that tile column is refined
// ev_start / ev_stop (optional): timing events attached to the first and last dispatch.
// lowflag (optional): if it is set when a pivot fails, it is cleared and *done = 2 (redo the
// iteration in FP64) instead of reporting the breakdown.
// fb != NULL (n <= kPotrsSingleMax): the launches also run the forward substitution
// L y = S fb (S = diag(feq), or 1) for every row block but the last two, one extra workgroup
// per launch (fwd_block_at) as soon as the block's row of L is complete, into fy (n doubles);
// launch_potrs with yf = fy then finishes the last two blocks and the backward substitution.
int launch_potrf(hipStream_t s, double* K, int n, int ld, double* Wall, int* done, int* info,
                 int* status, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr,
                 int* lowflag = nullptr, const double* fb = nullptr, const double* feq = nullptr,
                 double* fy = nullptr);
constexpr int kPotrsSingleMax = 4096;  // one-workgroup solves (and the fused forward) up to here
inline size_t wall_doubles(int n) { return (4096 + 8) * (size_t)((n + 63) / 64); }
// Row block whose forward substitution Cholesky launch k (0 <= k < nt) runs, or -1: row block
// j's row of L is complete after launch j (panel L_j,j-1), so block 0 runs in launch 0 and
// block j >= 1 in launch j + 1; the last two blocks are left to the solve kernel.
__host__ __device__ inline int fwd_block_at(int k, int nt) {
  const int j = k == 0 ? 0 : k - 1;
  return (k != 1 && j <= nt - 3) ? j : -1;
}
// x = (L L')^-1 b with n doubles of scratch `work` (distinct from b and x); x may alias b.
// eq != NULL: L is the factor of the equilibrated S K S (S = diag(eq)) and x = S (L L')^-1 S b.
// yf != NULL (n <= kPotrsSingleMax): y of every row block but the last two is already in yf
// (launch_potrf's fused forward substitution with the same b and eq).
// accumulate (n <= kPotrsSingleMax, x distinct from b): x += (L L')^-1 b instead.
int launch_potrs(hipStream_t s, const double* L, int n, int ld, const double* Wall,
                 const double* b, double* x, double* work, const int* done,
                 const double* eq = nullptr, const double* yf = nullptr, int accumulate = 0);
// Diagonal equilibration in place: eq_i = K_ii^-1/2, K_ij <- eq_i K_ij eq_j (lower triangle).
int launch_equilibrate(hipStream_t s, double* K, int n, int ld, double* eq, const int* done);
int launch_tri_inv(hipStream_t s, const double* L, int n, int ld, double* Wall);

// ---- IPM vector kernels (k_ipm.hip) ----
int ipm_alloc_work(Problem& p);
int launch_gamma_t(Problem& p, const double* w, int nvec, double* out, const int* done);
// y = Gamma x (scale != NULL: y = scale o Gamma x)
int launch_gamma_mv(Problem& p, const double* x, double* y, const int* done,
                    const double* scale = nullptr);
// warm = 0: the cold start; warm = 1: start from the controls already in p.v with barrier
// parameter mu0 (Gamma v is formed first).
int launch_ipm_init(Problem& p, const cmpc_options& o, int warm = 0, double mu0 = 0.0);
// p.v <- p.v shifted one stage earlier, the last stage repeated (receding horizon).
int launch_shift_controls(Problem& p);
int launch_prep(Problem& p);
int launch_mu_rhs(Problem& p);
int launch_step(Problem& p, int refine);  // refine: refinement steps queued (mixed modes)
int launch_update_publish(Problem& p, int slot);  // update + the host flag of ring slot `slot`
int launch_refine_step(Problem& p);
int launch_sigma_fold(Problem& p, const double* sigma);
int launch_step_given(Problem& p, const double* v, const double* s, const double* lam,
                      const double* z, double mu, double tau);

}  // namespace cmpc

// Handle behind the C ABI's cmpc_problem; instances of a batch are borrowed (the batch owns
// them and cmpc_problem_destroy leaves them alone).
struct cmpc_problem {
  cmpc::Problem* p;
  bool borrowed;
};
