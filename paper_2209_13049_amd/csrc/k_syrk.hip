// Formation of the condensed matrix K = Hbase + Gamma' diag(D) Gamma + diag(Ddiag)
// (left-hand side of eqn. (cond_KKT) after folding the two-sided bound rows; the paper's
// Section 5 names this condensation as the step whose cost grows with the row count of J).
//
// Design (gfx950):
//  * Gamma is never stored: it is block Toeplitz (block (t, j) = G_{t-1-j}, G_m = A^m B), so
//    entry (row i of block t, column j nu + k) is read from G_{t-1-j}[i][k] (N x ns x nu,
//    4 MB at K 500 x 500), which stays in the L2 / Infinity Cache while HBM is hardly
//    touched; only structural nonzeros are read, and tile (I, J) of K receives row block t
//    only if t nu > 64 I.
//  * Split-K: each 64 x 64 output tile's rows (its row blocks, t descending, all ns rows
//    of each) are cut into pieces, and the pieces packed into workgroups of equal cost
//    under a measured time model, all workgroups resident at once (at most 512, 2 per CU).
//    Pieces that cover the same rows of different tiles run together on one XCD.
//  * Each of the 4 wavefronts of a workgroup accumulates the whole tile over every 4th
//    group of 4 rows with v_mfma_f64_16x16x4f64 (v_mfma_f32_16x16x4f32 for FP32 and for
//    bfloat16 storage), operands loaded straight from memory in the MFMA lane layout
//    through a register prefetch ring and scaled by D on the fly; structurally zero columns
//    (>= t nu) enter as zeros, and a diagonal tile computes only its 10 blocks on or below
//    the diagonal.
//  * At the end of its piece a workgroup sums the 4 accumulators in LDS and writes a
//    partial slot; a second kernel adds the slots of each tile in a fixed order to Hbase
//    (deterministic, no atomics).
#include <algorithm>

#include "problem.hpp"

namespace cmpc {

static int nblocks16(int I, int J, int len) {
  const int a0 = 64 * I, b0 = 64 * J;
  if (len <= a0) return 0;
  const int nib = std::min(4, ceil_div(len - a0, 16));
  const int njb = std::min(4, ceil_div(len - b0, 16));
  if (I != J) return nib * njb;
  int c = 0;
  for (int ib = 0; ib < nib; ++ib)
    for (int jb = 0; jb < njb; ++jb)
      if (jb <= ib) ++c;
  return c;
}

void syrk_free(SyrkPlan& sp) {
  hipFree(sp.tiles);
  hipFree(sp.jobs);
  hipFree(sp.wg_begin);
  hipFree(sp.slot_begin);
  hipFree(sp.slots);
  hipFree(sp.partials);
  sp = SyrkPlan();
}

int syrk_plan(Problem& p, int quantum) {
  SyrkPlan& sp = p.syrk;
  const int ns = p.ns, nu = p.nu, N = p.N, n = p.n;
  sp.nt = ceil_div(n, 64);
  std::vector<int2> tiles;
  for (int I = 0; I < sp.nt; ++I)
    for (int J = 0; J <= I; ++J) tiles.push_back(make_int2(I, J));
  sp.ntiles = (int)tiles.size();
  sp.flops_structural = 0.0;
  for (int t = 1; t <= N; ++t) {
    const double len = (double)t * nu;
    sp.flops_structural += (double)ns * len * (len + 1.0);
  }
  // Tile q receives row blocks t = N, N-1, ..., t_q (a tile is reached once t nu > 64 I, so
  // its blocks are the last ones); its work is the row sequence of those blocks, t
  // descending, rows ascending.  A row of block t costs the 16 x 16 blocks the kernel
  // computes for it: the row blocks of the tile's 64 rows that t nu reaches (nib of 4),
  // times 4 column blocks, or, on a diagonal tile, the nib (nib + 1) / 2 blocks on or below
  // the diagonal.
  auto row_cost = [&](int q, int t) {
    const int len = t * nu, a0 = 64 * tiles[q].x;
    if (len <= a0) return 0;
    const int nib = std::min(4, ceil_div(len - a0, 16));
    return tiles[q].x == tiles[q].y ? nib * (nib + 1) / 2 : 4 * nib;
  };
  // Pieces: tile q's sequence cut into runs of cost at most C (whole groups of 16 rows) and
  // wherever the row cost changes (the kernel specialises a piece's loop on it); the pieces
  // are packed into workgroups of cost at most C, C the least (at least quantum) for which
  // all workgroups fit one resident round of kMaxWg (2 per CU).
  constexpr int kMaxWg = 512;
  // Time model in block units (measured): a row also costs 4 for its loads, masking and
  // address arithmetic, and a piece 800 for its prologue (the first groups' load latency)
  // and its flush.
  const long long kRowOverhead = 4, kPieceOverhead = 800;
  auto cut = [&](int q, long long C, std::vector<std::vector<SyrkJob>>* out) {
    long long npieces = 0, used = 0;
    bool open = false;
    std::vector<SyrkJob> cur;
    auto close = [&]() {
      if (!open) return;
      ++npieces;
      if (out) out->push_back(cur);
      cur.clear();
      used = 0;
      open = false;
    };
    for (int t = N; t >= 1; --t) {
      const int c = row_cost(q, t);
      if (c == 0) break;
      const long long w = c + kRowOverhead;
      if (open && c != row_cost(q, cur.back().t)) close();
      int r = 0;
      while (r < ns) {
        if (open && C - used < 16 * w) close();
        if (!open) {
          open = true;
          used = kPieceOverhead;
        }
        long long take = std::max<long long>(16, (C - used) / w / 16 * 16);
        take = std::min<long long>(take, ns - r);
        cur.push_back({q, t, r, r + (int)take, -1});
        used += take * w;
        r += (int)take;
      }
    }
    close();
    return npieces;
  };
  struct Piece {
    int q;
    size_t j;  // index of the piece within its tile's sequence
    long long cost;
    std::vector<SyrkJob> jobs;
  };
  auto make_pieces = [&](long long C) {
    std::vector<Piece> ps;
    for (int q = 0; q < sp.ntiles; ++q) {
      std::vector<std::vector<SyrkJob>> v;
      cut(q, C, &v);
      for (size_t j = 0; j < v.size(); ++j) {
        long long c = kPieceOverhead;
        for (const SyrkJob& jb : v[j]) c += (row_cost(q, jb.t) + kRowOverhead) * (jb.r1 - jb.r0);
        ps.push_back({q, j, c, std::move(v[j])});
      }
    }
    return ps;
  };
  // Workgroups: the pieces packed first-fit decreasing into bins of cost at most C (the
  // tails of the tiles' sequences fill up the workgroups of other tiles' tails).
  auto pack = [&](const std::vector<Piece>& ps, long long C, std::vector<std::vector<int>>* bins) {
    std::vector<int> order(ps.size());
    for (size_t i = 0; i < ps.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return ps[a].cost > ps[b].cost; });
    std::vector<long long> load;
    bins->clear();
    for (int i : order) {
      size_t b = 0;
      while (b < load.size() && load[b] + ps[i].cost > C) ++b;
      if (b == load.size()) {
        load.push_back(0);
        bins->emplace_back();
      }
      load[b] += ps[i].cost;
      (*bins)[b].push_back(i);
    }
    return (long long)bins->size();
  };
  long long total = 0;
  for (int q = 0; q < sp.ntiles; ++q)
    for (int t = N; t >= 1 && row_cost(q, t) > 0; --t)
      total += (row_cost(q, t) + kRowOverhead) * ns;
  long long C = std::max<long long>({(long long)quantum, 16LL * 16, (total + kMaxWg - 1) / kMaxWg});
  std::vector<Piece> ps;
  std::vector<std::vector<int>> bins;
  for (;;) {
    ps = make_pieces(C);
    if (pack(ps, C, &bins) <= kMaxWg) break;
    C += std::max<long long>(16, C / 200);
  }
  // Workgroups in the order of their largest piece's (index, tile): the full-length pieces
  // with the same index cover the same rows of every tile, and consecutive workgroups run on
  // the same XCD, so that those rows are fetched from HBM once into that XCD's L2 and
  // re-read there by each tile.
  auto key = [&](const std::vector<int>& bn) { return std::make_pair(ps[bn[0]].j, ps[bn[0]].q); };
  std::stable_sort(bins.begin(), bins.end(),
                   [&](const std::vector<int>& a, const std::vector<int>& b) { return key(a) < key(b); });
  std::vector<SyrkJob> jobs;
  std::vector<int> wg_begin;
  std::vector<int> slot_tile;
  for (const std::vector<int>& bn : bins) {
    wg_begin.push_back((int)jobs.size());
    for (int i : bn) {
      for (const SyrkJob& jb : ps[i].jobs) jobs.push_back(jb);
      jobs.back().slot = (int)slot_tile.size();
      slot_tile.push_back(ps[i].q);
    }
  }
  int nwg = std::max(8, ((int)wg_begin.size() + 7) / 8 * 8);
  wg_begin.resize(nwg + 1, (int)jobs.size());
  sp.nslots = (int)slot_tile.size();
  std::vector<int> slot_begin(sp.ntiles + 1, 0), slots(std::max(1, sp.nslots));
  for (int s = 0; s < sp.nslots; ++s) slot_begin[slot_tile[s] + 1]++;
  for (int q = 0; q < sp.ntiles; ++q) slot_begin[q + 1] += slot_begin[q];
  {
    std::vector<int> fill(slot_begin.begin(), slot_begin.end() - 1);
    for (int s = 0; s < sp.nslots; ++s) slots[fill[slot_tile[s]]++] = s;
  }
  sp.nwg = nwg;
  sp.quantum = quantum;
  CMPC_HIP(hipMalloc(&sp.tiles, sizeof(int2) * tiles.size()));
  CMPC_HIP(hipMalloc(&sp.jobs, sizeof(SyrkJob) * std::max<size_t>(1, jobs.size())));
  CMPC_HIP(hipMalloc(&sp.wg_begin, sizeof(int) * (nwg + 1)));
  CMPC_HIP(hipMalloc(&sp.slot_begin, sizeof(int) * (sp.ntiles + 1)));
  CMPC_HIP(hipMalloc(&sp.slots, sizeof(int) * std::max(1, sp.nslots)));
  CMPC_HIP(hipMalloc(&sp.partials, sizeof(double) * 4096 * (size_t)std::max(1, sp.nslots)));
  CMPC_HIP(hipMemcpy(sp.tiles, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice));
  CMPC_HIP(hipMemcpy(sp.jobs, jobs.data(), sizeof(SyrkJob) * jobs.size(), hipMemcpyHostToDevice));
  CMPC_HIP(hipMemcpy(sp.wg_begin, wg_begin.data(), sizeof(int) * (nwg + 1), hipMemcpyHostToDevice));
  CMPC_HIP(hipMemcpy(sp.slot_begin, slot_begin.data(), sizeof(int) * (sp.ntiles + 1),
                     hipMemcpyHostToDevice));
  CMPC_HIP(hipMemcpy(sp.slots, slots.data(), sizeof(int) * sp.nslots, hipMemcpyHostToDevice));
  return 0;
}

// ---------------------------------------------------------------------------------------

template <typename TIn>
struct MfmaOps;

template <>
struct MfmaOps<double> {
  typedef d4 acc_t;
  typedef double comp_t, scale_t;
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline comp_t scaled(double x, double d) { return x * d; }
  __device__ static inline comp_t plain(double x) { return x; }
  // output element v of lane l sits at row l/16 + 4v, column l%16 of the 16 x 16 block
  __device__ static inline int out_row(int lk, int v) { return lk + 4 * v; }
};

template <>
struct MfmaOps<float> {
  typedef f4 acc_t;
  typedef float comp_t, scale_t;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline comp_t scaled(float x, float d) { return x * d; }
  __device__ static inline comp_t plain(float x) { return x; }
  // output element v of lane l sits at row 4 (l/16) + v, column l%16
  __device__ static inline int out_row(int lk, int v) { return 4 * lk + v; }
};

// bfloat16: the real bfloat16 MFMA (v_mfma_f32_16x16x32_bf16, float32 accumulation); the
// element type only selects the interleaved row loop below.
template <>
struct MfmaOps<bf16_t> {
  typedef f4 acc_t;
  __device__ static inline int out_row(int lk, int v) { return 4 * lk + v; }
};

// The low-precision copies of G are interleaved by rows: element (m, r, k) sits at
// ((m RV + r / V) nu + k) V + r % V with RV = ceil(ns / V) and the rows past ns zero, so that
// V consecutive rows of one column of Gamma are one 16-byte load.  float: V = 4, and the
// 4 rows of a lane feed 4 steps of v_mfma_f32_16x16x4f32 (one row per step, the 4 lanes of
// a column group contracting 4 rows per step); bfloat16: V = 8, the 8 rows feed one
// v_mfma_f32_16x16x32_bf16 (lane group g supplies contraction elements 8 g .. 8 g + 7).
template <typename TIn>
struct VecRows;
template <>
struct VecRows<float> {
  static constexpr int V = 4;
  typedef f4 vec_t;
};
template <>
struct VecRows<bf16_t> {
  static constexpr int V = 8;
  typedef s8 vec_t;
};

// Rows [r0, r1) of one row block against one tile.  Every wavefront takes every 4th group
// of 4 rows; operands are loaded straight into the MFMA lane layout (lane l: column l%16 of
// a 16-column block, row l/16 of the 4-row group) through a PF-deep register ring (3 groups
// in FP64, 12 in FP32), so PF-1 groups of loads are in flight behind the MFMAs of the current
// group.  Columns >= t nu
// (structural zeros) and rows >= r1 enter as 0.  Only the first NIB row blocks of the tile
// (those that t nu reaches: NIB = min(4, ceil((t nu - a0) / 16))) are loaded and computed.
// DIAG (a diagonal tile, a0 == b0): both operands come from the same columns, loaded once,
// and only the blocks on or below the diagonal are computed.
template <typename TIn, bool DIAG, int NIB>
__device__ __forceinline__ void syrk_rows(typename MfmaOps<TIn>::acc_t (&acc)[4][4],
                                          const TIn* __restrict__ G,
                                          const double* __restrict__ Dt, int t, int ns, int nu,
                                          int a0, int b0, int r0, int r1, int wave, int li,
                                          int lk) {
  typedef MfmaOps<TIn> Ops;
  typedef typename Ops::comp_t TC;
  typedef typename Ops::scale_t TS;
  // Ring depth: the groups in flight must cover the load latency, and an FP32 group takes half
  // the MFMA time and half the registers of an FP64 one (measured at K 1500 x 1500, 549,250
  // rows: FP32 launch 8.7 ms at depth 3, 6.6 at 8, 5.2 at 12; 16 spills; FP64 no better at 4, 5).
  // BF16 storage needs a few more registers for the conversions: 10 (12 spills in the batch form).
  constexpr int PF = sizeof(TIn) == 8 ? 3 : (sizeof(TIn) == 4 ? 12 : 10);
  const int len = t * nu;
  bool va[4], vb[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    va[q] = a0 + 16 * q + li < len;
    vb[q] = b0 + 16 * q + li < len;
  }
  const int nsteps = (r1 - r0 + 15) >> 4;
  TIn ra[PF][4], rb[PF][4];
  TS rd[PF];
  // Every load is issued unconditionally from an in-bounds address (row r0, column 0 for
  // lanes outside the rows or columns), and the ring keeps the raw values; rows and columns
  // outside the piece are zeroed where a group is consumed.  With no branch around a load
  // and no use of a value before its group is due, the compiler waits for exactly that
  // group instead of draining every load in flight.
  // Column c = j nu + k of row block t is column k of G_{t-1-j}, and row r of that block is
  // row r of G_{t-1-j}: element ((t-1-j) ns + r) nu + k of G.  Each lane's column offset is
  // fixed for the job and a row adds r nu elements.  Byte offsets are 32-bit (G is far below
  // 4 GiB; the problem's creation checks it), so every load takes the uniform base in SGPRs
  // plus one offset VGPR.
  auto col_off = [&](int c) {
    const int j = c / nu, k = c - j * nu;
    return ((unsigned)(t - 1 - j) * (unsigned)ns * (unsigned)nu + (unsigned)k) *
           (unsigned)sizeof(TIn);
  };
  unsigned ca[4], cb[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ca[q] = va[q] ? col_off(a0 + 16 * q + li) : 0u;
    cb[q] = vb[q] ? col_off(b0 + 16 * q + li) : 0u;
  }
  const char* __restrict__ gb = (const char*)G;
  const unsigned rowbytes = (unsigned)nu * (unsigned)sizeof(TIn);
  auto load = [&](int step, TIn (&xa)[4], TIn (&xb)[4], TS& xd) {
    const int r = r0 + 16 * step + 4 * wave + lk;
    const int rr = r < r1 ? r : r0;
    const unsigned ro = (unsigned)rr * rowbytes;
    xd = (TS)Dt[rr];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q < NIB) xa[q] = *(const TIn*)(gb + (ro + ca[q]));
      if (!DIAG) xb[q] = *(const TIn*)(gb + (ro + cb[q]));
    }
  };
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    load(u, ra[u], rb[u], rd[u]);
    asm volatile("" ::: "memory");  // groups issued in ring order (see below)
    __builtin_amdgcn_sched_barrier(0);
  }
  for (int step = 0; step < nsteps; step += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const bool vr = r0 + 16 * (step + u) + 4 * wave + lk < r1;
      const TS d = vr ? rd[u] : (TS)0;
      TC sa[4], sb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < NIB) sa[q] = va[q] ? Ops::scaled(ra[u][q], d) : (TC)0;
        if (!DIAG) sb[q] = vb[q] ? Ops::plain(rb[u][q]) : (TC)0;
        else if (q < NIB) sb[q] = vb[q] ? Ops::plain(ra[u][q]) : (TC)0;
      }
#pragma unroll
      for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
          if (!DIAG || jb <= ib) acc[ib][jb] = Ops::mma(sa[ib], sb[jb], acc[ib][jb]);
      load(step + u + PF, ra[u], rb[u], rd[u]);
      // Keep each group's loads here, PF - 1 groups ahead of their use, and each group's
      // masking with its MFMAs: without the fences the compiler moves the loads down to
      // the iteration that consumes them and hoists the masking of later groups, and either
      // way every load in flight is waited for at the top of the loop.
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Rows [r0, r1) of row block t against one tile, from an interleaved copy of G (see
// VecRows): the wavefronts take every 4th group of 4 V rows (lane group lk: rows
// R + V lk .. R + V lk + V - 1), operands loaded 16 bytes per lane straight into the MFMA
// lane layout through a PF-deep register ring; the A operand is scaled by D per row (for
// bfloat16 rounded back to bfloat16, so each product is one of two bfloat16 values), rows
// >= r1 scaled by 0, columns >= t nu zero.  r0 is a multiple of 16 (the planner cuts rows in
// groups of 16), so every lane's V rows are one chunk of the copy.
template <typename TIn, bool DIAG, int NIB>
__device__ __forceinline__ void syrk_rows_vec(f4 (&acc)[4][4], const TIn* __restrict__ Gv,
                                              const double* __restrict__ Dt, int t, int ns,
                                              int nu, int a0, int b0, int r0, int r1, int wave,
                                              int li, int lk) {
  constexpr int V = VecRows<TIn>::V, GR = 4 * V;
  typedef typename VecRows<TIn>::vec_t vec_t;
  constexpr int PF = 2;
  const int len = t * nu;
  const int RV = (ns + V - 1) / V;
  bool va[4], vb[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    va[q] = a0 + 16 * q + li < len;
    vb[q] = b0 + 16 * q + li < len;
  }
  // column c = j nu + k of row block t: column k of G_{t-1-j}; 32-bit byte offsets (the copy
  // is smaller than G, which creation keeps below 4 GiB)
  auto col_off = [&](int c) {
    const int j = c / nu, k = c - j * nu;
    return (((unsigned)(t - 1 - j) * (unsigned)RV * (unsigned)nu + (unsigned)k) * (unsigned)V) *
           (unsigned)sizeof(TIn);
  };
  unsigned ca[4], cb[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ca[q] = va[q] ? col_off(a0 + 16 * q + li) : 0u;
    cb[q] = vb[q] ? col_off(b0 + 16 * q + li) : 0u;
  }
  const char* __restrict__ gb = (const char*)Gv;
  const unsigned chunkbytes = (unsigned)nu * (unsigned)V * (unsigned)sizeof(TIn);
  const int nsteps = (r1 - r0 + 4 * GR - 1) / (4 * GR);
  vec_t ra[PF][4], rb[PF][4];
  double rd[PF][V];
  // loads from in-bounds addresses only: a lane whose rows lie past r1 reads chunk r0 / V
  // (its rows are scaled by 0 when consumed), D rows past ns read row ns - 1
  auto load = [&](int step, vec_t (&xa)[4], vec_t (&xb)[4], double (&xd)[V]) {
    const int rc = r0 + 4 * GR * step + GR * wave + V * lk;
    const int rr = rc < r1 ? rc : r0;
    const unsigned ro = (unsigned)(rr / V) * chunkbytes;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q < NIB) xa[q] = *(const vec_t*)(gb + (ro + ca[q]));
      if (!DIAG) xb[q] = *(const vec_t*)(gb + (ro + cb[q]));
    }
#pragma unroll
    for (int e = 0; e < V; ++e) xd[e] = Dt[rr + e < ns ? rr + e : ns - 1];
  };
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    load(u, ra[u], rb[u], rd[u]);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  }
  for (int step = 0; step < nsteps; step += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int rc = r0 + 4 * GR * (step + u) + GR * wave + V * lk;
      float d[V];
#pragma unroll
      for (int e = 0; e < V; ++e) d[e] = rc + e < r1 ? (float)rd[u][e] : 0.0f;
      if constexpr (V == 4) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float sa[4], sb[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (q < NIB) sa[q] = va[q] ? ra[u][q][e] * d[e] : 0.0f;
            if (!DIAG) sb[q] = vb[q] ? rb[u][q][e] : 0.0f;
            else if (q < NIB) sb[q] = vb[q] ? ra[u][q][e] : 0.0f;
          }
#pragma unroll
          for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
            for (int jb = 0; jb < 4; ++jb)
              if (!DIAG || jb <= ib)
                acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(sa[ib], sb[jb], acc[ib][jb],
                                                                   0, 0, 0);
        }
      } else {
        s8 sa[4], sb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (q < NIB) {
            if (va[q]) {
#pragma unroll
              for (int e = 0; e < 8; ++e) {
                const __bf16 x = (__bf16)(bf2f((bf16_t)ra[u][q][e]) * d[e]);
                sa[q][e] = __builtin_bit_cast(short, x);
              }
            } else {
              sa[q] = s8{0, 0, 0, 0, 0, 0, 0, 0};
            }
          }
          if (!DIAG) sb[q] = vb[q] ? rb[u][q] : s8{0, 0, 0, 0, 0, 0, 0, 0};
          else if (q < NIB) sb[q] = vb[q] ? ra[u][q] : s8{0, 0, 0, 0, 0, 0, 0, 0};
        }
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
          for (int jb = 0; jb < 4; ++jb)
            if (!DIAG || jb <= ib)
              acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sa[ib], sb[jb], acc[ib][jb],
                                                                    0, 0, 0);
      }
      load(step + u + PF, ra[u], rb[u], rd[u]);
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// The jobs [j0, j1) of one workgroup (all on one tile, all with the same number NIB of row
// blocks reached): accumulate, and at a job that carries a slot sum the 4 wavefronts'
// accumulators in LDS and write the partial tile.
template <typename TIn, bool DIAG, int NIB>
__device__ __forceinline__ void syrk_jobs(const TIn* __restrict__ G,
                                          const double* __restrict__ D,
                                          const SyrkJob* __restrict__ jobs, int j0, int j1,
                                          const int2* __restrict__ tiles,
                                          double* __restrict__ partials, int ns, int nu,
                                          double* red) {
  typedef MfmaOps<TIn> Ops;
  typedef typename Ops::acc_t acc_t;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  for (int jj = j0; jj < j1; ++jj) {
    const SyrkJob job = jobs[jj];
    const int2 tl = tiles[job.tile];
    const int a0 = tl.x * 64, b0 = tl.y * 64;
    const double* __restrict__ Dt = D + (long long)(job.t - 1) * ns;
    if constexpr (sizeof(TIn) == 8)
      syrk_rows<TIn, DIAG, NIB>(acc, G, Dt, job.t, ns, nu, a0, b0, job.r0, job.r1, wave, li, lk);
    else
      syrk_rows_vec<TIn, DIAG, NIB>(acc, G, Dt, job.t, ns, nu, a0, b0, job.r0, job.r1, wave, li,
                                    lk);
    if (job.slot >= 0) {
      __syncthreads();
      for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
          for (int ib = 0; ib < 4; ++ib)
#pragma unroll
            for (int jb = 0; jb < 4; ++jb)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int idx = (16 * ib + Ops::out_row(lk, v)) * 64 + 16 * jb + li;
                const double x = (double)acc[ib][jb][v];
                red[idx] = (w == 0) ? x : red[idx] + x;
              }
        }
        __syncthreads();
      }
      double* dst = partials + (long long)job.slot * 4096;
      for (int e = threadIdx.x; e < 4096; e += 256) dst[e] = red[e];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    }
  }
}

template <typename TIn>
__device__ __forceinline__ void syrk_splitk_body(int bid, 
    const TIn* __restrict__ G, const double* __restrict__ D,
    const SyrkJob* __restrict__ jobs, const int* __restrict__ wg_begin,
    const int2* __restrict__ tiles, double* __restrict__ partials, int ns, int nu, int nwg,
    const int* __restrict__ done, const int* __restrict__ lowflag, int want_low) {
  __shared__ double red[64 * 64];
  if (done != nullptr && *done) return;
  if (lowflag != nullptr && *lowflag != want_low) return;
  const int j0 = wg_begin[bid], j1 = wg_begin[bid + 1];
  if (j0 >= j1) return;
  // A workgroup runs one or more pieces, each ending at a job that carries a slot.  Every
  // job of a piece is on the same tile and reaches the same number of the tile's row blocks
  // (the planner cuts pieces per tile and where that number changes), so one specialised
  // loop serves the whole piece.
  for (int pj = j0; pj < j1;) {
    int pe = pj;
    while (pe < j1 - 1 && jobs[pe].slot < 0) ++pe;
    const int2 tl = tiles[jobs[pj].tile];
    const int nib = min(4, (jobs[pj].t * nu - 64 * tl.x + 15) >> 4);  // >= 1 (t nu > 64 I)
#define CMPC_SYRK_JOBS(DIAG, NIB) \
  syrk_jobs<TIn, DIAG, NIB>(G, D, jobs, pj, pe + 1, tiles, partials, ns, nu, red)
    if (tl.x == tl.y) {
      switch (nib) {
        case 1: CMPC_SYRK_JOBS(true, 1); break;
        case 2: CMPC_SYRK_JOBS(true, 2); break;
        case 3: CMPC_SYRK_JOBS(true, 3); break;
        default: CMPC_SYRK_JOBS(true, 4); break;
      }
    } else {
      switch (nib) {
        case 1: CMPC_SYRK_JOBS(false, 1); break;
        case 2: CMPC_SYRK_JOBS(false, 2); break;
        case 3: CMPC_SYRK_JOBS(false, 3); break;
        default: CMPC_SYRK_JOBS(false, 4); break;
      }
    }
    pj = pe + 1;
  }
#undef CMPC_SYRK_JOBS
}

template <typename TIn>
__global__ __launch_bounds__(256, 2) void syrk_splitk_kernel(
    const TIn* __restrict__ G, const double* __restrict__ D,
    const SyrkJob* __restrict__ jobs, const int* __restrict__ wg_begin,
    const int2* __restrict__ tiles, double* __restrict__ partials, int ns, int nu, int nwg,
    const int* __restrict__ done, const int* __restrict__ lowflag, int want_low) {
  syrk_splitk_body<TIn>((blockIdx.x & 7) * (nwg >> 3) + (blockIdx.x >> 3), G, D, jobs, wg_begin,
                        tiles, partials, ns, nu, nwg, done, lowflag, want_low);
}

// K(lower) = Hb(lower) + sum of the tile's partial slots (fixed order) + diag(Ddiag).
// 16 workgroups per tile, one element per thread.
__device__ __forceinline__ void syrk_finish_body(int bid, 
    const double* __restrict__ partials, const int* __restrict__ slot_begin,
    const int* __restrict__ slots, const int2* __restrict__ tiles, const double* __restrict__ Hb,
    const double* __restrict__ Ddiag, double* __restrict__ K, int n, const int* __restrict__ done) {
  if (done != nullptr && *done) return;
  const int tile = bid >> 4;
  const int e = ((bid & 15) << 8) + threadIdx.x;
  const int2 tl = tiles[tile];
  const int gi = tl.x * 64 + (e >> 6), gj = tl.y * 64 + (e & 63);
  if (gi >= n || gj > gi) return;
  const int q0 = slot_begin[tile], q1 = slot_begin[tile + 1];
  double sum = 0.0;  // fixed order; unrolled so that the loads are in flight together
#pragma unroll 8
  for (int q = q0; q < q1; ++q) sum += partials[(long long)slots[q] * 4096 + e];
  double val = Hb[(long long)gi * n + gj] + sum;
  if (gi == gj && Ddiag != nullptr) val += Ddiag[gi];
  K[(long long)gi * n + gj] = val;
}

__global__ __launch_bounds__(256) void syrk_finish_kernel(
    const double* __restrict__ partials, const int* __restrict__ slot_begin,
    const int* __restrict__ slots, const int2* __restrict__ tiles, const double* __restrict__ Hb,
    const double* __restrict__ Ddiag, double* __restrict__ K, int n, const int* __restrict__ done) {
  syrk_finish_body(blockIdx.x, partials, slot_begin, slots, tiles, Hb, Ddiag, K, n, done);
}

// ---- work-list forms (batches): one item = one split-K workgroup (or one finish block) of
// one instance, with that instance's own plan, so the result is the single-instance one.
// mixed != 0: the item runs only when the instance's precision level st->use_low equals
// want_low (2 = BF16, 1 = FP32, 0 = FP64).
template <typename TIn>
__global__ __launch_bounds__(256, 2) void syrk_batch_kernel(const InstView* __restrict__ views,
                                                            const WorkItem* __restrict__ items,
                                                            int nitems, int mixed, int want_low) {
  CMPC_ITEMS_BEGIN
  const TIn* G = sizeof(TIn) == 8 ? (const TIn*)V.G
                                   : (sizeof(TIn) == 4 ? (const TIn*)V.G32 : (const TIn*)V.G16);
  syrk_splitk_body<TIn>(bid, G, V.Dx, V.jobs, V.wg_begin, V.tiles, V.partials, V.ns,
                         V.nu, V.syrk_nwg, &V.st->done, mixed ? &V.st->use_low : nullptr,
                         want_low);
  CMPC_ITEMS_END
}

__global__ __launch_bounds__(256) void syrk_finish_batch_kernel(const InstView* __restrict__ views,
                                                                const WorkItem* __restrict__ items,
                                                                int nitems) {
  CMPC_ITEMS_BEGIN
  syrk_finish_body(bid, V.partials, V.slot_begin, V.slots, V.tiles, V.H, V.Du, V.K, V.n,
                   &V.st->done);
  CMPC_ITEMS_END
}

template __global__ void syrk_batch_kernel<double>(const InstView*, const WorkItem*, int, int, int);
template __global__ void syrk_batch_kernel<float>(const InstView*, const WorkItem*, int, int, int);
template __global__ void syrk_batch_kernel<bf16_t>(const InstView*, const WorkItem*, int, int, int);

int launch_b_syrk(const ListArg& L, int level, int mixed, int want_low) {
  if (level == 2) CMPC_LAUNCH_LIST(syrk_batch_kernel<bf16_t>, L, mixed, want_low);
  if (level == 1) CMPC_LAUNCH_LIST(syrk_batch_kernel<float>, L, mixed, want_low);
  CMPC_LAUNCH_LIST(syrk_batch_kernel<double>, L, mixed, want_low);
}
int launch_b_finish(const ListArg& L) { CMPC_LAUNCH_LIST(syrk_finish_batch_kernel, L); }

int launch_syrk(Problem& p, int precision, const double* Drow, const double* Hbase,
                const double* Ddiag, double* K, hipEvent_t ev_start, hipEvent_t ev_stop,
                int mixed) {
  SyrkPlan& sp = p.syrk;
  const int* done = p.st ? &p.st->done : nullptr;
  const int* low = mixed ? &p.st->use_low : nullptr;
  // levels queued: mixed -> every level from the starting one down to FP64, each gated on
  // st->use_low; otherwise only the requested precision
  const int top = mixed ? mixed : (precision == CMPC_BF16_SYRK ? 2 : (precision == CMPC_FP32_SYRK ? 1 : 0));
  const int bottom = mixed ? 0 : top;
  if ((top >= 1 && bottom <= 1 && p.G32 == nullptr) || (top == 2 && p.G16 == nullptr)) {
    set_error("low-precision copy of G not allocated");
    return CMPC_ERR_INVALID;
  }
  for (int lev = top; lev >= bottom; --lev) {
    hipEvent_t e0 = lev == top ? ev_start : nullptr, e1 = lev == bottom ? ev_stop : nullptr;
    if (lev == 2)
      hipExtLaunchKernelGGL(syrk_splitk_kernel<bf16_t>, dim3(sp.nwg), dim3(256), 0, p.stream, e0,
                            e1, 0, (const bf16_t*)p.G16, Drow,
                            (const SyrkJob*)sp.jobs, (const int*)sp.wg_begin,
                            (const int2*)sp.tiles, sp.partials, p.ns, p.nu, sp.nwg, done, low, 2);
    else if (lev == 1)
      hipExtLaunchKernelGGL(syrk_splitk_kernel<float>, dim3(sp.nwg), dim3(256), 0, p.stream, e0,
                            e1, 0, (const float*)p.G32, Drow,
                            (const SyrkJob*)sp.jobs, (const int*)sp.wg_begin,
                            (const int2*)sp.tiles, sp.partials, p.ns, p.nu, sp.nwg, done, low, 1);
    else
      hipExtLaunchKernelGGL(syrk_splitk_kernel<double>, dim3(sp.nwg), dim3(256), 0, p.stream, e0,
                            e1, 0, (const double*)p.G, Drow,
                            (const SyrkJob*)sp.jobs, (const int*)sp.wg_begin,
                            (const int2*)sp.tiles, sp.partials, p.ns, p.nu, sp.nwg, done, low, 0);
    CMPC_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(syrk_finish_kernel, dim3(sp.ntiles * 16), dim3(256), 0, p.stream, sp.partials,
                     sp.slot_begin, sp.slots, sp.tiles, Hbase, Ddiag, K, p.n, done);
  CMPC_LAUNCH_CHECK();
  return 0;
}

}  // namespace cmpc

namespace cmpc {

// The interleaved low-precision copy of G (see VecRows): out element
// ((m RV + rv) nu + k) V + e = G[(m ns + V rv + e) nu + k], zero for rows V rv + e >= ns.
template <typename TOut, int V>
__global__ void convert_interleaved_kernel(const double* __restrict__ G, TOut* __restrict__ out,
                                           int ns, int nu, int N) {
  const int RV = (ns + V - 1) / V;
  const long long len = (long long)N * RV * nu * V;
  const long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= len) return;
  const int e = (int)(o % V);
  long long q = o / V;
  const int k = (int)(q % nu);
  q /= nu;
  const int rv = (int)(q % RV);
  const int m = (int)(q / RV);
  const int r = V * rv + e;
  const double x = r < ns ? G[((long long)m * ns + r) * nu + k] : 0.0;
  if constexpr (sizeof(TOut) == 4)
    out[o] = (TOut)x;
  else
    out[o] = f2bf((float)x);
}

// Low-precision copies of G for the mixed-precision SYRK (made once): CMPC_FP32_SYRK makes
// the float copy, CMPC_BF16_SYRK both (a BF16 solve may step to FP32).
int launch_convert_gamma(Problem& p, int precision) {
  if (precision == CMPC_BF16_SYRK && p.G16 == nullptr) {
    const long long len = (long long)p.N * ceil_div(p.ns, 8) * p.nu * 8;
    if (hipMalloc(&p.G16, sizeof(bf16_t) * (size_t)len) != hipSuccess) {
      p.G16 = nullptr;
      set_error("out of device memory (BF16 copy of G)");
      return CMPC_ERR_NOMEM;
    }
    hipLaunchKernelGGL((convert_interleaved_kernel<bf16_t, 8>), dim3(ceil_div(len, 256)),
                       dim3(256), 0, p.stream, p.G, (bf16_t*)p.G16, p.ns, p.nu, p.N);
    CMPC_LAUNCH_CHECK();
  }
  if (precision == CMPC_BF16_SYRK) precision = CMPC_FP32_SYRK;
  if (precision == CMPC_FP32_SYRK && p.G32 == nullptr) {
    const long long len = (long long)p.N * ceil_div(p.ns, 4) * p.nu * 4;
    if (hipMalloc(&p.G32, sizeof(float) * (size_t)len) != hipSuccess) {
      p.G32 = nullptr;
      set_error("out of device memory (FP32 copy of G)");
      return CMPC_ERR_NOMEM;
    }
    hipLaunchKernelGGL((convert_interleaved_kernel<float, 4>), dim3(ceil_div(len, 256)),
                       dim3(256), 0, p.stream, p.G, p.G32, p.ns, p.nu, p.N);
    CMPC_LAUNCH_CHECK();
  }
  return 0;
}

}  // namespace cmpc
