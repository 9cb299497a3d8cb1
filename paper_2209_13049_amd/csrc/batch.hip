// Ragged batches of independent MPC instances, and the SYRK tuning table.
//
// A batch runs every stage of an interior-point iteration (Algorithm 1) for all of its
// instances in one launch over a work list of (instance, block) items, so many problems of
// uneven nu N share the GPU without one launch sequence per problem.  Each item is the body
// of the single-instance kernel with the instance's own block decomposition, reductions
// and SYRK plan, so an FP64 batch reproduces each instance's own solve bit for bit.  The
// launches of one iteration are captured once as a HIP graph and replayed; instances that
// have converged are predicated off (their items return at entry) until all are done.
//
// The tuning table maps (n, mx, precision) to the SYRK work quantum (least work per
// split-K workgroup) and the grid policy of the work-list launches; cmpc_batch_tune fills
// it by timing the batched SYRK over candidate settings, and every later solve of a
// problem with that key (batched or not) builds its plan from it.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "problem.hpp"

namespace cmpc {

// ------------------------------------------------------------------ tuning table
namespace {
struct TuneKey {
  int n, mx, precision;
  bool operator<(const TuneKey& o) const {
    if (n != o.n) return n < o.n;
    if (mx != o.mx) return mx < o.mx;
    return precision < o.precision;
  }
};
struct TuneVal {
  int quantum;
  int persistent;
  double us;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
std::mutex g_occ_mu;
std::map<const void*, int> g_occ;
}  // namespace

static bool tune_lookup(int n, int mx, int precision, TuneVal* out) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(TuneKey{n, mx, precision});
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

static void tune_store(int n, int mx, int precision, const TuneVal& v) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[TuneKey{n, mx, precision}] = v;
}

int ensure_plan(Problem& p, int precision, bool* changed) {
  TuneVal tv;
  int q = kSyrkQuantumDefault;
  if (tune_lookup(p.n, p.mx, precision, &tv)) q = tv.quantum;
  if (changed) *changed = false;
  if (q == p.syrk.quantum) return 0;
  CMPC_HIP(hipStreamSynchronize(p.stream));  // queued work may still read the old plan
  syrk_free(p.syrk);
  const int rc = syrk_plan(p, q);
  if (rc) return rc;
  if (changed) *changed = true;
  return 0;
}

int occupancy_per_cu(const void* kernel) {
  std::lock_guard<std::mutex> g(g_occ_mu);
  auto it = g_occ.find(kernel);
  if (it != g_occ.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess || nb < 1)
    nb = 1;
  g_occ[kernel] = nb;
  return nb;
}

// ------------------------------------------------------------------ batch
struct List {
  int off = 0, count = 0;
};

struct Batch {
  int count = 0;
  std::vector<Problem*> inst;
  std::vector<cmpc_problem> handles;
  hipStream_t user = nullptr;    // stream of creation, x0 uploads and instance calls
  hipStream_t stream = nullptr;  // the batch's own stream (graph capture and replay)
  int cus = 256;
  int persistent = 1;
  InstView* views = nullptr;
  std::vector<InstView> hviews;  // host copy of `views` as uploaded by build_lists
  WorkItem* items = nullptr;
  size_t items_cap = 0;
  List init, blk, gt, n4, one, syrk, fin, n256, gmv;
  std::vector<List> chol, fwd, bwd;
  int ntmax = 0, nmax = 0;
  bool lists_valid = false;
  int* d_iter = nullptr;
  int* hflags = nullptr;
  int* dflags = nullptr;
  IpmState* d_states = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_mixed = -1, graph_refine = -1, graph_eq = -1;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

constexpr int kRing = 16;

static void drop_graph(Batch& b) {
  if (b.exec) hipGraphExecDestroy(b.exec);
  if (b.graph) hipGraphDestroy(b.graph);
  b.exec = nullptr;
  b.graph = nullptr;
  b.graph_mixed = b.graph_refine = b.graph_eq = -1;
}

static void free_batch(Batch* b) {
  if (!b) return;
  if (b->stream) hipStreamSynchronize(b->stream);
  if (b->user) hipStreamSynchronize(b->user);
  drop_graph(*b);
  for (Problem* p : b->inst) free_problem(p);
  if (b->views) hipFree(b->views);
  if (b->items) hipFree(b->items);
  if (b->d_iter) hipFree(b->d_iter);
  if (b->d_states) hipFree(b->d_states);
  if (b->hflags) hipHostFree(b->hflags);
  if (b->ev0) hipEventDestroy(b->ev0);
  if (b->ev1) hipEventDestroy(b->ev1);
  if (b->stream) hipStreamDestroy(b->stream);
  delete b;
}

static InstView view_of(const Problem& p) {
  InstView v;
  std::memset(&v, 0, sizeof(v));  // padding too: views are compared bytewise
  v.ns = p.ns;
  v.nu = p.nu;
  v.N = p.N;
  v.n = p.n;
  v.mx = p.mx;
  v.m = p.m;
  v.nblk = p.n_prep_blocks;
  v.gt_chunks = p.gt_chunks;
  v.nt = ceil_div(p.n, 64);
  v.syrk_nwg = p.syrk.nwg;
  v.G = p.G;
  v.Gt = p.Gt;
  v.G32 = p.G32;
  v.G16 = (const bf16_t*)p.G16;
  v.H = p.H;
  v.d = p.d;
  v.h = p.h;
  v.K = p.K;
  v.Wdiag = p.Wdiag;
  v.eqs = p.eqs;
  v.v = p.v;
  v.s = p.s;
  v.lam = p.lam;
  v.z = p.z;
  v.gv = p.gv;
  v.pv = p.pv;
  v.ps = p.ps;
  v.plam = p.plam;
  v.pz = p.pz;
  v.gpv = p.gpv;
  v.rhs = p.rhs;
  v.Dx = p.Dx;
  v.Du = p.Du;
  v.wx = p.wx;
  v.wu = p.wu;
  v.gt = p.gt;
  v.Hv = p.Hv;
  v.tmpn = p.tmpn;
  v.ref_res = p.ref_res;
  v.ref_dlt = p.ref_dlt;
  v.norm_part = p.norm_part;
  v.alpha_part = p.alpha_part;
  v.gt_part = p.gt_part;
  v.st = p.st;
  v.jobs = p.syrk.jobs;
  v.wg_begin = p.syrk.wg_begin;
  v.tiles = p.syrk.tiles;
  v.partials = p.syrk.partials;
  v.slot_begin = p.syrk.slot_begin;
  v.slots = p.syrk.slots;
  return v;
}

// Instance views and every work list (instance-major item order).
static int build_lists(Batch& b) {
  std::vector<InstView> hv;
  for (Problem* p : b.inst) hv.push_back(view_of(*p));
  if (!b.views) CMPC_HIP(hipMalloc(&b.views, sizeof(InstView) * b.count));
  CMPC_HIP(hipMemcpy(b.views, hv.data(), sizeof(InstView) * b.count, hipMemcpyHostToDevice));
  b.hviews = hv;
  std::vector<WorkItem> all;
  auto add = [&](List& L, auto per) {
    L.off = (int)all.size();
    for (int i = 0; i < b.count; ++i) {
      const int c = per(hv[i]);
      for (int j = 0; j < c; ++j) all.push_back(WorkItem{i, j});
    }
    L.count = (int)all.size() - L.off;
  };
  add(b.init, [](const InstView& v) { return ceil_div(v.m, 256); });
  add(b.blk, [](const InstView& v) { return v.nblk; });
  add(b.gt, [](const InstView& v) { return v.gt_chunks; });
  add(b.n4, [](const InstView& v) { return ceil_div(v.n, 4); });
  add(b.one, [](const InstView&) { return 1; });
  add(b.syrk, [](const InstView& v) { return v.syrk_nwg; });
  add(b.fin, [&](const InstView& v) { return v.nt * (v.nt + 1) / 2 * 16; });
  add(b.n256, [](const InstView& v) { return ceil_div(v.n, 256); });
  add(b.gmv, [](const InstView& v) { return gmv_blocks<kMvTBatch>(v.ns, v.N); });
  b.ntmax = 0;
  b.nmax = 0;
  for (const InstView& v : hv) {
    b.ntmax = std::max(b.ntmax, v.nt);
    b.nmax = std::max(b.nmax, v.n);
  }
  b.chol.assign(b.ntmax, List());
  b.fwd.assign(b.ntmax, List());
  b.bwd.assign(b.ntmax, List());
  for (int k = 0; k < b.ntmax; ++k) {
    // the launch sequence of one instance: chol_step k for k < nt when nt > 1, with
    // npanel + rows (rows + 1) / 2 workgroups; trsv steps with max(1, nt-k-1) / max(1, k)
    // (+ 1 where the fused forward substitution has a block: one-workgroup solves)
    const bool fused = b.nmax <= kPotrsSingleMax;
    add(b.chol[k], [k, fused](const InstView& v) {
      if (v.nt <= 1 || k >= v.nt) return 0;
      const int npanel = k >= 1 ? v.nt - k : 0, rows = v.nt - 1 - k;
      return npanel + rows * (rows + 1) / 2 + (fused && fwd_block_at(k, v.nt) >= 0 ? 1 : 0);
    });
    add(b.fwd[k], [k](const InstView& v) { return k < v.nt ? std::max(1, v.nt - k - 1) : 0; });
    add(b.bwd[k], [k](const InstView& v) { return k < v.nt ? std::max(1, k) : 0; });
  }
  if (all.size() > b.items_cap) {
    if (b.items) hipFree(b.items);
    b.items = nullptr;
    CMPC_HIP(hipMalloc(&b.items, sizeof(WorkItem) * all.size()));
    b.items_cap = all.size();
  }
  CMPC_HIP(hipMemcpy(b.items, all.data(), sizeof(WorkItem) * all.size(), hipMemcpyHostToDevice));
  b.lists_valid = true;
  return 0;
}

static ListArg arg(const Batch& b, const List& L) {
  return ListArg{b.views, b.items + L.off, L.count, b.persistent, b.cus, b.stream};
}

// (L L')^-1 applied to rhs -> pv (which = 0) or ref_res -> ref_dlt (which = 1); eq: the
// factor is that of the equilibrated S K S.
static int enqueue_potrs(Batch& b, int which, int eq) {
  if (b.nmax <= kPotrsSingleMax)  // which = 0 follows the factorisation's fused forward pass
    return launch_b_potrs_single(arg(b, b.one), which, eq, b.nmax, 1);
  if (launch_b_potrs_copy(arg(b, b.n256), which, 0, eq)) return CMPC_ERR_HIP;
  for (int k = 0; k < b.ntmax; ++k)
    if (launch_b_trsv_fwd(arg(b, b.fwd[k]), k, which)) return CMPC_ERR_HIP;
  for (int k = b.ntmax - 1; k >= 0; --k)
    if (launch_b_trsv_bwd(arg(b, b.bwd[k]), k, which)) return CMPC_ERR_HIP;
  if (launch_b_potrs_copy(arg(b, b.n256), which, 1, eq)) return CMPC_ERR_HIP;
  return 0;
}

// mixed: starting precision level (2 BF16, 1 FP32); every level down to FP64 is queued and
// runs only for the instances currently at that level.
static int enqueue_syrk(Batch& b, int mixed) {
  if (mixed) {
    for (int lev = mixed; lev >= 0; --lev)
      if (launch_b_syrk(arg(b, b.syrk), lev, 1, lev)) return CMPC_ERR_HIP;
  } else if (launch_b_syrk(arg(b, b.syrk), 0, 0, 0)) {
    return CMPC_ERR_HIP;
  }
  return launch_b_finish(arg(b, b.fin));
}

// One interior-point iteration of every instance, in the order of the single-instance
// driver (residuals and rhs, K, Cholesky, solve and refinement, step, update with the next
// iteration's prep); the first iteration's prep is launched before the first replay.
static int enqueue_iteration(Batch& b, int mixed, int refine, int eq) {
  if (launch_b_gamma_t_partial(arg(b, b.gt), 3)) return CMPC_ERR_HIP;
  if (launch_b_hv(arg(b, b.n4), 0)) return CMPC_ERR_HIP;
  if (launch_b_mu_rhs(arg(b, b.one))) return CMPC_ERR_HIP;
  if (enqueue_syrk(b, mixed)) return CMPC_ERR_HIP;
  if (eq && launch_b_equilibrate(arg(b, b.n256), arg(b, b.n4))) return CMPC_ERR_HIP;
  if (launch_b_chol_first(arg(b, b.one), mixed)) return CMPC_ERR_HIP;
  for (int k = 0; k < b.ntmax; ++k)
    if (launch_b_chol_step(arg(b, b.chol[k]), k, mixed, b.nmax <= kPotrsSingleMax, eq))
      return CMPC_ERR_HIP;
  if (enqueue_potrs(b, 0, eq)) return CMPC_ERR_HIP;
  // refinement rounds in the single-instance step's arithmetic: D_x o Gamma p in the Gamma
  // pass, the Gamma' partials added up in the check, and (one-workgroup solves) the
  // correction added to p in the solve's store
  for (int r = 0; r < refine; ++r) {
    if (launch_b_gamma_mv(arg(b, b.gmv), 1)) return CMPC_ERR_HIP;
    if (launch_b_gamma_t_partial(arg(b, b.gt), 1)) return CMPC_ERR_HIP;
    if (launch_b_hv(arg(b, b.n4), 1)) return CMPC_ERR_HIP;
    if (launch_b_refine_check(arg(b, b.one))) return CMPC_ERR_HIP;
    if (enqueue_potrs(b, 1, eq)) return CMPC_ERR_HIP;
    if (b.nmax > kPotrsSingleMax && launch_b_axpy(arg(b, b.n256))) return CMPC_ERR_HIP;
  }
  if (launch_b_gamma_mv(arg(b, b.gmv), 0)) return CMPC_ERR_HIP;
  if (launch_b_step(arg(b, b.blk))) return CMPC_ERR_HIP;
  if (launch_b_update(arg(b, b.blk))) return CMPC_ERR_HIP;
  return launch_b_publish(b.stream, b.views, b.count, b.d_iter, b.dflags, kRing);
}

static int capture(Batch& b, int mixed, int refine, int eq) {
  drop_graph(b);
  CMPC_HIP(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue_iteration(b, mixed, refine, eq);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b.stream, &g);
  if (rc || e != hipSuccess) {
    if (g) hipGraphDestroy(g);
    if (!rc) set_error(std::string("graph capture: ") + hipGetErrorString(e));
    return rc ? rc : CMPC_ERR_HIP;
  }
  b.graph = g;
  if (hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0) != hipSuccess) {
    b.exec = nullptr;
    set_error("graph instantiation failed");
    return CMPC_ERR_HIP;
  }
  b.graph_mixed = mixed;
  b.graph_refine = refine;
  b.graph_eq = eq;
  return 0;
}

static int check_options(const cmpc_options& o) {
  if (!(o.tol > 0) || o.max_iter < 0) {
    set_error("invalid options");
    return CMPC_ERR_INVALID;
  }
  if (o.precision != CMPC_FP64 && o.precision != CMPC_FP32_SYRK &&
      o.precision != CMPC_BF16_SYRK) {
    set_error("unsupported precision mode");
    return CMPC_ERR_INVALID;
  }
  if (o.max_refine < 0 || o.max_refine > 20) {
    set_error("max_refine must lie in [0, 20]");
    return CMPC_ERR_INVALID;
  }
  return 0;
}

// Plans follow the tuning table; the FP32 copy of Gamma exists when needed; lists, views and
// the graph are rebuilt when anything they point to changed.
static int prepare(Batch& b, int precision) {
  bool any = false;
  for (Problem* p : b.inst) {
    if (!p->have_x0) {
      set_error("every instance needs an x0 (cmpc_set_x0) before the batch is solved");
      return CMPC_ERR_INVALID;
    }
    bool ch = false;
    const int rc = ensure_plan(*p, precision, &ch);
    if (rc) return rc;
    any = any || ch;
    if ((precision == CMPC_FP32_SYRK && p->G32 == nullptr) ||
        (precision == CMPC_BF16_SYRK && (p->G16 == nullptr || p->G32 == nullptr))) {
      const int rc2 = launch_convert_gamma(*p, precision);
      if (rc2) return rc2;
      any = true;
    }
  }
  CMPC_HIP(hipStreamSynchronize(b.user));  // creation, x0 and conversion work is done
  // Calls on an instance handle between batch solves (a single solve at another precision
  // rebuilds that instance's SYRK plan and frees the old one; a first BF16 solve allocates
  // its bfloat16 copy of Gamma) change what its view points to: the device views, the work
  // lists and the captured graph are rebuilt whenever any view differs from the uploaded one.
  for (int i = 0; i < b.count && !any && b.lists_valid; ++i) {
    const InstView v = view_of(*b.inst[i]);
    any = std::memcmp(&v, &b.hviews[i], sizeof(InstView)) != 0;
  }
  if (any || !b.lists_valid) {
    drop_graph(b);
    const int rc = build_lists(b);
    if (rc) return rc;
  }
  return 0;
}

// warm: start each instance from controls (v0s[i], or with v0s / v0s[i] NULL its last
// solution shifted one stage) instead of the cold start.
static int batch_solve(Batch& b, const cmpc_options& o, cmpc_result* res, int warm = 0,
                       const double* const* v0s = nullptr, int on_device = 0) {
  int rc = check_options(o);
  if (rc) return rc;
  if (warm && (!(o.warm_mu > 0) || !std::isfinite(o.warm_mu))) {
    set_error("warm_mu must be positive and finite");
    return CMPC_ERR_INVALID;
  }
  rc = prepare(b, o.precision);
  if (rc) return rc;
  if (warm) {
    for (int i = 0; i < b.count; ++i) {
      Problem& p = *b.inst[i];
      const double* v0 = v0s ? v0s[i] : nullptr;
      if (v0 == nullptr) {
        if (!p.have_solution) {
          set_error("instance " + std::to_string(i) + ": a warm start from the last solution "
                    "needs an earlier solve");
          return CMPC_ERR_INVALID;
        }
        rc = launch_shift_controls(p);
        if (rc) return rc;
      } else {
        CMPC_HIP(hipMemcpyAsync(p.v, v0, sizeof(double) * p.n,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                p.stream));
      }
    }
    CMPC_HIP(hipStreamSynchronize(b.user));
  }
  const int mixed = o.precision == CMPC_BF16_SYRK ? 2 : (o.precision == CMPC_FP32_SYRK ? 1 : 0);
  const int refine = mixed ? o.max_refine : 0;
  const int eq = o.equilibrate < 0 ? (mixed > 0) : (o.equilibrate != 0);
  if (!b.exec || b.graph_mixed != mixed || b.graph_refine != refine || b.graph_eq != eq) {
    rc = capture(b, mixed, refine, eq);
    if (rc) return rc;
  }
  CMPC_HIP(hipEventRecord(b.ev0, b.stream));
  if (warm && launch_b_gamma_mv(arg(b, b.gmv), 2)) return CMPC_ERR_HIP;  // gv = Gamma v0
  if (launch_b_init(arg(b, b.init), o.tol, o.max_iter, mixed, o.mu_switch,
                    o.refine_contract, warm, o.warm_mu)) return CMPC_ERR_HIP;
  if (launch_b_prep(arg(b, b.blk))) return CMPC_ERR_HIP;  // later ones run in the update
  if (launch_b_reset(b.stream, b.d_iter)) return CMPC_ERR_HIP;
  // The publish kernel of iteration it stores (running instances + 1) into ring slot
  // it % kRing; the host keeps `depth` iterations queued ahead of the last slot it read.
  const int depth = std::max(1, o.check_every);
  volatile int* hf = b.hflags;
  for (int it = 0; it <= o.max_iter && rc == 0; ++it) {
    if (it >= depth) {
      const int slot = (it - depth) % kRing;
      long long spins = 0;
      while (hf[slot] == 0) {
        if ((++spins & 1023) == 0) {
          const hipError_t q = hipStreamQuery(b.stream);
          if (q == hipSuccess && hf[slot] == 0) {
            set_error("batch solve: iteration flag missing");
            rc = CMPC_ERR_HIP;
            break;
          }
          if (q != hipSuccess && q != hipErrorNotReady) {
            set_error(std::string("batch solve: ") + hipGetErrorString(q));
            rc = CMPC_ERR_HIP;
            break;
          }
        }
      }
      if (rc) break;
      if (hf[slot] == 1) break;  // no instance running
    }
    hf[it % kRing] = 0;
    if (hipGraphLaunch(b.exec, b.stream) != hipSuccess) {
      set_error("graph launch failed");
      rc = CMPC_ERR_HIP;
    }
  }
  if (rc) {
    hipStreamSynchronize(b.stream);
    return rc;
  }
  CMPC_HIP(hipEventRecord(b.ev1, b.stream));
  if (launch_b_gather(b.stream, b.views, b.count, b.d_states)) return CMPC_ERR_HIP;
  std::vector<IpmState> hs(b.count);
  CMPC_HIP(hipMemcpyAsync(hs.data(), b.d_states, sizeof(IpmState) * b.count,
                          hipMemcpyDeviceToHost, b.stream));
  CMPC_HIP(hipStreamSynchronize(b.stream));
  float ms = 0.f;
  hipEventElapsedTime(&ms, b.ev0, b.ev1);
  int worst = CMPC_OK;
  for (int i = 0; i < b.count; ++i) {
    const IpmState& s = hs[i];
    const int status = s.done ? s.status : CMPC_MAX_ITER;
    b.inst[i]->have_solution = status >= 0;
    if (status != CMPC_OK && (worst == CMPC_OK || status < 0)) worst = status;
    if (res) {
      cmpc_result& r = res[i];
      std::memset(&r, 0, sizeof(r));
      r.status = status;
      r.iters = s.iter;
      r.precision_switch_iter = s.switch_iter;
      r.refine_steps = s.refine_steps;
      r.obj = s.obj;
      r.primal_res = s.nr3;
      r.dual_res = s.nr1;
      r.compl_res = s.szmax;
      r.mu = s.mu;
      r.gap = s.gap;
      r.ms_total = ms;
    }
  }
  if (worst != CMPC_OK) set_error("at least one instance did not converge (see its result)");
  return worst;
}

// Time the batched SYRK (+ finish) for every candidate (quantum, grid policy) and keep the
// fastest.  The instances must have an x0; their iterates are reset to the start point.
static int batch_tune(Batch& b, int precision, cmpc_tune_report* rep) {
  if (precision != CMPC_FP64 && precision != CMPC_FP32_SYRK && precision != CMPC_BF16_SYRK) {
    set_error("unsupported precision mode");
    return CMPC_ERR_INVALID;
  }
  static const int quanta[] = {3000, 6000, 12000, 24000, 48000, 96000};
  const int mixed = precision == CMPC_BF16_SYRK ? 2 : (precision == CMPC_FP32_SYRK ? 1 : 0);
  int rc = prepare(b, precision);
  if (rc) return rc;
  double best_us = 1e300, default_us = 0.0;
  int best_q = kSyrkQuantumDefault, best_p = 1, ncand = 0;
  const int reps = 3;
  for (int q : quanta) {
    for (Problem* p : b.inst) {
      syrk_free(p->syrk);
      rc = syrk_plan(*p, q);
      if (rc) return rc;
    }
    drop_graph(b);
    rc = build_lists(b);
    if (rc) return rc;
    // valid Sigma: the start point of the method, then its fold
    cmpc_options o;
    cmpc_default_options(&o);
    if (launch_b_init(arg(b, b.init), o.tol, o.max_iter, mixed, o.mu_switch,
                    o.refine_contract)) return CMPC_ERR_HIP;
    if (launch_b_prep(arg(b, b.blk))) return CMPC_ERR_HIP;
    for (int pers = 0; pers <= 1; ++pers) {
      b.persistent = pers;
      if (enqueue_syrk(b, mixed)) return CMPC_ERR_HIP;  // warm-up
      CMPC_HIP(hipEventRecord(b.ev0, b.stream));
      for (int r = 0; r < reps; ++r)
        if (enqueue_syrk(b, mixed)) return CMPC_ERR_HIP;
      CMPC_HIP(hipEventRecord(b.ev1, b.stream));
      CMPC_HIP(hipEventSynchronize(b.ev1));
      float ms = 0.f;
      CMPC_HIP(hipEventElapsedTime(&ms, b.ev0, b.ev1));
      const double us = 1e3 * ms / reps;
      ++ncand;
      if (q == kSyrkQuantumDefault && pers == 1) default_us = us;
      if (us < best_us) {
        best_us = us;
        best_q = q;
        best_p = pers;
      }
    }
  }
  for (Problem* p : b.inst) tune_store(p->n, p->mx, precision, TuneVal{best_q, best_p, best_us});
  b.persistent = best_p;
  for (Problem* p : b.inst) {
    syrk_free(p->syrk);
    rc = syrk_plan(*p, best_q);
    if (rc) return rc;
  }
  drop_graph(b);
  rc = build_lists(b);
  if (rc) return rc;
  if (rep) {
    rep->quantum = best_q;
    rep->persistent = best_p;
    rep->syrk_us = best_us;
    rep->default_us = default_us;
    rep->candidates = ncand;
  }
  return 0;
}

static int batch_create(int count, const cmpc_lq_desc* descs, const double* const* x0s,
                        hipStream_t stream, Batch** out) {
  if (count <= 0 || !descs || !out) {
    set_error("need count > 0, descriptors and an output pointer");
    return CMPC_ERR_INVALID;
  }
  Batch* b = new Batch();
  b->count = count;
  b->user = stream;
  for (int i = 0; i < count; ++i) {
    Problem* p = nullptr;
    int rc = create(&descs[i], stream, &p);
    if (!rc && x0s && x0s[i]) {
      rc = set_x0(*p, x0s[i], 0);
      if (rc) free_problem(p);
    }
    if (rc) {
      set_error("instance " + std::to_string(i) + ": " + cmpc_last_error());
      free_batch(b);
      return rc;
    }
    b->inst.push_back(p);
  }
  b->handles.resize(count);
  for (int i = 0; i < count; ++i) b->handles[i] = cmpc_problem{b->inst[i], true};
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
      hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc(&b->d_iter, sizeof(int)) != hipSuccess ||
      hipMalloc(&b->d_states, sizeof(IpmState) * count) != hipSuccess ||
      hipHostMalloc((void**)&b->hflags, sizeof(int) * kRing, hipHostMallocMapped) != hipSuccess ||
      hipHostGetDevicePointer((void**)&b->dflags, b->hflags, 0) != hipSuccess ||
      hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) {
    set_error("batch: HIP setup failed");
    free_batch(b);
    return CMPC_ERR_HIP;
  }
  b->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  *out = b;
  return 0;
}

}  // namespace cmpc

using namespace cmpc;

struct cmpc_batch {
  Batch* b;
};

extern "C" {

int cmpc_batch_create(int count, const cmpc_lq_desc* descs, const double* const* x0s,
                      void* stream, cmpc_batch** out) {
  if (!out) {
    set_error("NULL output");
    return CMPC_ERR_INVALID;
  }
  *out = nullptr;
  Batch* b = nullptr;
  const int rc = batch_create(count, descs, x0s, (hipStream_t)stream, &b);
  if (rc) return rc;
  *out = new cmpc_batch{b};
  return 0;
}

void cmpc_batch_destroy(cmpc_batch* h) {
  if (!h) return;
  free_batch(h->b);
  delete h;
}

int cmpc_batch_size(const cmpc_batch* h) { return h ? h->b->count : 0; }

cmpc_problem* cmpc_batch_instance(cmpc_batch* h, int i) {
  if (!h || i < 0 || i >= h->b->count) {
    set_error("no such instance");
    return nullptr;
  }
  return &h->b->handles[i];
}

int cmpc_batch_solve(cmpc_batch* h, const cmpc_options* opts, cmpc_result* results) {
  if (!h) {
    set_error("NULL batch");
    return CMPC_ERR_INVALID;
  }
  cmpc_options o;
  cmpc_default_options(&o);
  if (opts) o = *opts;
  return batch_solve(*h->b, o, results);
}

int cmpc_batch_solve_warm(cmpc_batch* h, const cmpc_options* opts, const double* const* v0s,
                          int on_device, cmpc_result* results) {
  if (!h) {
    set_error("NULL batch");
    return CMPC_ERR_INVALID;
  }
  cmpc_options o;
  cmpc_default_options(&o);
  if (opts) o = *opts;
  return batch_solve(*h->b, o, results, 1, v0s, on_device);
}

int cmpc_batch_tune(cmpc_batch* h, int precision, cmpc_tune_report* rep) {
  if (!h) {
    set_error("NULL batch");
    return CMPC_ERR_INVALID;
  }
  return batch_tune(*h->b, precision, rep);
}

int cmpc_tune_lookup(int n, int mx, int precision, int* quantum, int* persistent) {
  TuneVal tv;
  if (!tune_lookup(n, mx, precision, &tv)) return 1;
  if (quantum) *quantum = tv.quantum;
  if (persistent) *persistent = tv.persistent;
  return 0;
}

int cmpc_tune_store(int n, int mx, int precision, int quantum, int persistent) {
  if (n <= 0 || mx <= 0 || quantum < 256 || (persistent != 0 && persistent != 1) ||
      (precision != CMPC_FP64 && precision != CMPC_FP32_SYRK && precision != CMPC_BF16_SYRK)) {
    set_error("cmpc_tune_store: need n, mx > 0, quantum >= 256, persistent 0 or 1 and a "
              "supported precision");
    return CMPC_ERR_INVALID;
  }
  tune_store(n, mx, precision, TuneVal{quantum, persistent, 0.0});
  return 0;
}

void cmpc_tune_clear(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.clear();
}

}  // extern "C"
