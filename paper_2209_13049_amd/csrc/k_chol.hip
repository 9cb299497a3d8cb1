// Dense Cholesky factorisation K = L L' and the two triangular solves (Section 3: the
// condensed matrix is positive definite, so it is factored by Cholesky and p_v follows by
// triangular solves).  Row-major, lower triangle, leading dimension ld.
//
// Right-looking blocked factorisation with 64 x 64 tiles and one launch per block column:
//   chol_first  factors the first diagonal tile and forms its inverse W_0 = L_00^-1;
//   chol_step k every workgroup owns one tile (i, j), i > k, k <= j <= i:
//                 X_i = A_ik W_k'  (the panel block L_ik, v_mfma_f64_16x16x4f64 from LDS);
//                 j == k : writes L_ik;
//                 j > k  : A_ij -= X_i X_j'  (also MFMA);
//                 (k+1, k+1) additionally factors its updated tile at once and forms W_{k+1},
//                 so the next launch finds the next pivot block ready (look-ahead).
// Where a diagonal tile is ill-conditioned (max|L_kk| max|W_k| above kRefineCond, figures
// stored beside W_k by the workgroup that formed it) every panel product of that tile column
// takes one step of iterative refinement against L_kk (refine_panel), so that the panel is as
// accurate as a triangular solve; the redundant copies of a panel in different workgroups stay
// identical.
// A diagonal tile is factored by 4 wavefronts in 16 panels of 4 columns dealt round robin
// (lane = row, one barrier per panel: chol_panels) and inverted in 16 x 16 blocks (inv64:
// substitution for the diagonal blocks, MFMA products for the rest).  The inverses W_k are
// kept (nt x 64 x 64) so that the triangular solves become block matrix-vector products.
#include "problem.hpp"

namespace cmpc {

typedef double Tile[64][65];

// 1/x from the hardware estimate refined by two Newton-Raphson steps (quadratic convergence
// from the estimate's ~2^-26 relative error to full double precision).
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/x from the hardware estimate and one Newton-Raphson step (relative error ~2^-52: the
// elimination's pivot reciprocals, whose columns are rescaled exactly at the end).
__device__ inline double recip1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// All 16 loads of a thread are issued before the first LDS store, so their latencies overlap
// (a load-store-load loop waits for each load in turn).
__device__ inline void load_tile(const double* __restrict__ K, int ld, int n, int r0, int c0,
                                 Tile& T) {
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int i = e >> 6, j = e & 63;
    v[q] = (r0 + i < n && c0 + j < n) ? K[(long long)(r0 + i) * ld + c0 + j] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    T[e >> 6][e & 63] = v[q];
  }
}

// Wt <- W_k (64 x 64, contiguous), A <- tile (ra, ca) of K, B <- tile (rb, cb) if wantB (entries
// past n as 0): all of a thread's loads are issued before its first LDS store.
__device__ inline void load_w_tiles(const double* __restrict__ Wk, Tile& Wt,
                                    const double* __restrict__ K, int ld, int n, int ra, int ca,
                                    Tile& A, bool wantB, int rb, int cb, Tile& B) {
  double vw[16], va[16], vb[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int i = e >> 6, j = e & 63;
    vw[q] = Wk[e];
    va[q] = (ra + i < n && ca + j < n) ? K[(long long)(ra + i) * ld + ca + j] : 0.0;
    vb[q] = (wantB && rb + i < n && cb + j < n) ? K[(long long)(rb + i) * ld + cb + j] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    Wt[e >> 6][e & 63] = vw[q];
    A[e >> 6][e & 63] = va[q];
    if (wantB) B[e >> 6][e & 63] = vb[q];
  }
}

// acc (per wavefront: its 32 x 32 quadrant, 2 x 2 blocks of 16 x 16) += A B' (neg: -= A B')
__device__ inline void mma_abt_add(const Tile& A, const Tile& B, d4 (&acc)[2][2], int wr, int wc,
                                   int li, int lk, bool neg = false) {
  for (int ks = 0; ks < 16; ++ks) {
    double xa[2], xb[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      xa[q] = A[32 * wr + 16 * q + li][4 * ks + lk];
      xb[q] = B[32 * wc + 16 * q + li][4 * ks + lk];
      if (neg) xa[q] = -xa[q];
    }
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
        acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[ib], xb[jb], acc[ib][jb], 0, 0, 0);
  }
}

// acc = A B'
__device__ inline void mma_abt(const Tile& A, const Tile& B, d4 (&acc)[2][2], int wr, int wc,
                               int li, int lk) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0, 0, 0, 0};
  mma_abt_add(A, B, acc, wr, wc, li, lk);
}

// Store a quadrant accumulator into an LDS tile (row = 32 wr + 16 ib + lk + 4 v).
__device__ inline void store_acc(Tile& T, const d4 (&acc)[2][2], int wr, int wc, int li, int lk) {
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        T[32 * wr + 16 * ib + lk + 4 * v][32 * wc + 16 * jb + li] = acc[ib][jb][v];
}

// 16 x 16 product C = A B of LDS blocks (row-major, padded stride 65) on one wavefront with
// v_mfma_f64_16x16x4f64; returns the accumulator (element v of lane l is C[l/16 + 4v][l%16]).
__device__ inline d4 mma16(const double* A, const double* B, d4 c, int li, int lk) {
#pragma unroll
  for (int ks = 0; ks < 4; ++ks)
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(A[li * 65 + 4 * ks + lk], B[(4 * ks + lk) * 65 + li],
                                             c, 0, 0, 0);
  return c;
}


// Inverse W = L^-1 of the lower-triangular tile T, given rdiag[j] = 1 / T[j][j] (T and rdiag
// visible to the whole workgroup), in 16 x 16 blocks W_ij.  Phase 1: wavefront b inverts the
// diagonal block b by forward substitution (4 lanes per column, the block's entries loaded into
// registers first).  Then, with W = [[W_A, 0], [W_BA, W_B]] for the 32 x 32 halves A, B:
// W_BA = -W_B (L_BA W_A), whose 2 x 2 blocks of products run on the four wavefronts in three
// phases separated by barriers (phase 2: W_10 = -W_11 L_10 W_00, W_32 = -W_33 L_32 W_22 and the
// parts of L_BA W_A that need only W_00, W_11; phase 3: the rest of L_BA W_A; phase 4: the four
// blocks of W_BA), a dependent chain of five 16 x 16 products instead of nine.  The products
// L_BA W_A are kept in the upper blocks of W, which W does not use (write_w emits them as zeros).
__device__ void inv64(const Tile& T, Tile& W, const double* rdiag) {
  __shared__ double S[2][16 * 65];  // per-wavefront 16 x 16 scratch (wavefronts 0, 1)
  __shared__ double S8[4][64];       // per-wavefront 8 x 8 scratch of phase 1
  const int t = threadIdx.x, w = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
  {  // phase 1: diagonal block w as two 8 x 8 halves by substitution (lanes 0-31 the upper
     // left one, lanes 32-63 the lower right one; 4 lanes per column), then the 8 x 8 block
     // between them, W_BA = -W_B L_BA W_A, one entry per lane
    const int h = lane >> 5, q = lane & 31, c = q >> 2, p = q & 3, o = 16 * w + 8 * h;
    double lv[8][2];  // L[o + ii][o + 4 kk + p] for 4 kk + p < ii
#pragma unroll
    for (int ii = 0; ii < 8; ++ii)
#pragma unroll
      for (int kk = 0; kk <= (ii >> 2); ++kk) {
        const int k = 4 * kk + p;
        lv[ii][kk] = k < ii ? T[o + ii][o + k] : 0.0;
      }
    double rd[8];
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) rd[ii] = rdiag[o + ii];
    double wv[2] = {0.0, 0.0};
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) {
      double part = 0.0;
#pragma unroll
      for (int kk = 0; kk <= (ii >> 2); ++kk) part = fma(lv[ii][kk], wv[kk], part);
      part += dpp_f64<0xB1>(part);  // lane ^ 1 within the quad
      part += dpp_f64<0x4E>(part);  // lane ^ 2
      const double val = (ii >= c) ? (((ii == c) ? 1.0 : 0.0) - part) * rd[ii] : 0.0;
      if (p == (ii & 3)) wv[ii >> 2] = val;
    }
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) W[o + 4 * kk + p][o + c] = wv[kk];
    const int b0 = 16 * w, r = lane >> 3, cc = lane & 7;
    W[b0 + r][b0 + 8 + cc] = 0.0;  // the diagonal block's upper right 8 x 8
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    double sacc = 0.0;  // (L_BA W_A)[r][cc]
#pragma unroll
    for (int k = 0; k < 8; ++k) sacc = fma(T[b0 + 8 + r][b0 + k], W[b0 + k][b0 + cc], sacc);
    S8[w][r * 8 + cc] = sacc;
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    double wacc = 0.0;  // (W_B S)[r][cc]
#pragma unroll
    for (int k = 0; k < 8; ++k) wacc = fma(W[b0 + 8 + r][b0 + 8 + k], S8[w][k * 8 + cc], wacc);
    W[b0 + 8 + r][b0 + cc] = -wacc;
  }
  __syncthreads();
  const int li = lane & 15, lk = lane >> 4;
  const d4 zero = d4{0, 0, 0, 0};
  // the blocks of L_BA W_A: P20 -> W(0,1), P21 -> W(0,2), P30 -> W(0,3), P31 -> W(1,2)
  double* P20 = &W[0][16];
  double* P21 = &W[0][32];
  double* P30 = &W[0][48];
  double* P31 = &W[16][32];
  auto store = [&](double* dst, const d4& acc, double sign) {
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[(lk + 4 * v) * 65 + li] = sign * acc[v];
  };
  d4 keep = zero;  // wavefronts 2, 3: L_20 W_00 or L_30 W_00, completed in phase 3
  // phase 2
  if (w <= 1) {
    const int i = w == 0 ? 1 : 3, j = w == 0 ? 0 : 2;  // W_ij = -W_ii L_ij W_jj
    double* Sw = S[w];
    store(Sw, mma16(&T[16 * i][16 * j], &W[16 * j][16 * j], zero, li, lk), 1.0);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    store(&W[16 * i][16 * j], mma16(&W[16 * i][16 * i], Sw, zero, li, lk), -1.0);
  } else {
    const int r = w == 2 ? 2 : 3;  // row block of L_BA
    keep = mma16(&T[16 * r][0], &W[0][0], zero, li, lk);                      // L_r0 W_00
    store(w == 2 ? P21 : P31, mma16(&T[16 * r][16], &W[16][16], zero, li, lk), 1.0);  // L_r1 W_11
  }
  __syncthreads();
  // phase 3: P_r0 = L_r0 W_00 + L_r1 W_10
  if (w >= 2) {
    const int r = w == 2 ? 2 : 3;
    store(w == 2 ? P20 : P30, mma16(&T[16 * r][16], &W[16][0], keep, li, lk), 1.0);
  }
  __syncthreads();
  // phase 4: W_BA = -W_B P: W_20 = -W_22 P20, W_21 = -W_22 P21, W_30 = -(W_32 P20 + W_33 P30),
  // W_31 = -(W_32 P21 + W_33 P31)
  {
    const int col = w & 1;  // 0: column block 0, 1: column block 1
    const double* Pa = col == 0 ? P20 : P21;
    d4 acc;
    if (w <= 1) {
      acc = mma16(&W[32][32], Pa, zero, li, lk);
      store(&W[32][16 * col], acc, -1.0);
    } else {
      acc = mma16(&W[48][32], Pa, zero, li, lk);
      acc = mma16(&W[48][48], col == 0 ? P30 : P31, acc, li, lk);
      store(&W[48][16 * col], acc, -1.0);
    }
  }
  __syncthreads();
}

// Right-looking factorisation of the tile in 16 panels of 4 columns, one barrier per panel.
// Panels are dealt round robin: wavefront W holds panels W, W+4, W+8, W+12 (local panel m =
// global panel 4m + W, columns 16m + 4W .. 16m + 4W + 3) of row i (lane i) in registers
// (r[4m + c]), so consecutive panels have different owners.  Between barriers P and P+1 (panel P published
// in LDS): the owner of panel P+1 applies panel P to that panel only, eliminates it
// (pivots and panel entries broadcast by readlane) and publishes it; its update of its other
// columns by panel P waits for the next interval, where it is not the owner; every other
// wavefront applies panel P (and a panel it deferred) to its later columns meanwhile.  The
// critical path per panel is one 4-column update, the elimination and the barrier.  Panels
// are published unscaled with their pivot reciprocals (LDL'-like updates, the scaling by
// 1/sqrt(pivot) follows at the end); entries above the diagonal are updated too (they never
// feed an entry on or below it and are discarded), so the only tests are static.
constexpr int kPW = 4;        // panel width (8 measured slower: longer eliminations)
constexpr int kNP = 64 / kPW;  // panels per tile
constexpr int kLP = kNP / 4;   // panels per wavefront
template <int W>
__device__ __forceinline__ void chol_panels(double (&r)[16], double* pan /* 3 x 64 x PW */,
                                            double* pinv /* 3 x PW */, double* piv, int i,
                                            int t) {
  // eliminate global panel P (owned by this wavefront: P % 4 == W)
  auto eliminate = [&](int P) {
    const int m = P >> 2;
    double* pb = pan + (P % 3) * 64 * kPW;
    double* ib = pinv + (P % 3) * kPW;
    double pv[kPW], ipv[kPW];
#pragma unroll
    for (int jj = 0; jj < kPW; ++jj) {
      const double p = readlane_f64(r[kPW * m + jj], kPW * P + jj);
      const double ip = recip1(p);
      const double lij = r[kPW * m + jj] * ip;
#pragma unroll
      for (int kk = jj + 1; kk < kPW; ++kk)
        r[kPW * m + kk] =
            fma(-lij, readlane_f64(r[kPW * m + jj], kPW * P + kk), r[kPW * m + kk]);
      pv[jj] = p;
      ipv[jj] = ip;
    }
#pragma unroll
    for (int jj = 0; jj < kPW; ++jj) pb[kPW * i + jj] = r[kPW * m + jj];
    if (t == 64 * W) {
#pragma unroll
      for (int jj = 0; jj < kPW; ++jj) {
        piv[kPW * P + jj] = pv[jj];
        ib[jj] = ipv[jj];
      }
    }
  };
  // apply published panel Q to this wavefront's panels g with lo <= g <= hi (global indices)
  auto apply = [&](int Q, int lo, int hi) {
    const double* pb = pan + (Q % 3) * 64 * kPW;
    const double* ib = pinv + (Q % 3) * kPW;
    double li[kPW];
#pragma unroll
    for (int jj = 0; jj < kPW; ++jj) li[jj] = pb[kPW * i + jj] * ib[jj];
#pragma unroll
    for (int m = 0; m < kLP; ++m) {
      const int g = 4 * m + W;
      if (g >= lo && g <= hi) {
#pragma unroll
        for (int c = 0; c < kPW; ++c) {
          const double* pk = pb + kPW * (kPW * g + c);
          double acc = r[kPW * m + c];
#pragma unroll
          for (int jj = 0; jj < kPW; ++jj) acc = fma(-li[jj], pk[jj], acc);
          r[kPW * m + c] = acc;
        }
      }
    }
  };
  if (W == 0) eliminate(0);
  __syncthreads();
#pragma unroll
  for (int P = 0; P < kNP - 1; ++P) {
    if (W == (P + 1) % 4) {  // owner of panel P+1
      apply(P, P + 1, P + 1);
      eliminate(P + 1);
    } else {
      if (P >= 1 && W == P % 4) apply(P - 1, P + 1, kNP - 1);  // deferred while owning panel P
      apply(P, P + 1, kNP - 1);
    }
    __syncthreads();
  }
}

// Factor the SPD tile T in place (lower triangle -> L, strict upper -> 0) and write its
// inverse to W.  Rows >= nvalid are identity padding.  Returns false (uniformly) and the
// 0-based failing column in *bad if a pivot is not positive and finite.
__device__ inline void write_tile_lower(double* __restrict__ K, int ld, int n, int r0, int c0,
                                        const Tile& T, bool diag);

// ... and stores the factor tile to K at (r0, c0) (lower triangle) as soon as it is scaled,
// so that the stores drain while the inverse is formed.
__device__ __forceinline__ bool chol_inv64(Tile& T, Tile& W, double* colb, double* piv, int nvalid,
                                           int* bad, double* __restrict__ K, int ld, int n, int r0,
                                           int c0, double* __restrict__ cslot) {
  __shared__ double pan[3 * 64 * kPW], pinv[3 * kPW];
  const int t = threadIdx.x, w = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
  // ---- factorisation: wavefront w holds panels w, w+4, ... of row `lane` in registers
  // (r[PW m + c]: column 4 PW m + PW w + c).  T is not written again before the panel
  // loop's barriers, so the loads need no barrier of their own.
  const int i = lane;
  double r[16];
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int k = 4 * kPW * (kk / kPW) + kPW * w + (kk % kPW);
    double x = (k <= i) ? T[i][k] : 0.0;
    if (i >= nvalid) x = (k == i) ? 1.0 : 0.0;
    r[kk] = x;
  }
  switch (w) {  // wavefront-uniform: column indices become compile-time constants
    case 0: chol_panels<0>(r, pan, pinv, piv, i, t); break;
    case 1: chol_panels<1>(r, pan, pinv, piv, i, t); break;
    case 2: chol_panels<2>(r, pan, pinv, piv, i, t); break;
    default: chol_panels<3>(r, pan, pinv, piv, i, t); break;
  }
  // (the panel loop ends with a barrier: every pivot is in piv)
  // A pivot that is not positive and finite leaves garbage behind it; it is reported here
  // (the first such column), after the loop, so the loop itself carries no test.  Every
  // wavefront tests all 64 pivots, so the outcome is uniform without a barrier.
  const double pj = piv[lane];
  const unsigned long long badm = __ballot(!(pj > 0.0) || !isfinite(pj));
  if (badm != 0ull) {
    if (t == 0) *bad = __ffsll((long long)badm) - 1;
    return false;
  }
  const double cb = recip(sqrt(pj));  // 1 / L_jj of column `lane`
  if (w == 0) colb[lane] = cb;
  double ml = 0.0;
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int k = 4 * kPW * (kk / kPW) + kPW * w + (kk % kPW);
    const double x = (k <= i) ? r[kk] * readlane_f64(cb, k) : 0.0;
    T[i][k] = x;
    ml = fmax(ml, fabs(x));
  }
  ml = wave_max(ml);
  if (lane == 0) cslot[2 * w] = ml;
  __syncthreads();
  write_tile_lower(K, ld, n, r0, c0, T, true);
  inv64(T, W, colb);
  return true;
}

// All 16 LDS reads of a thread are issued before its first store.
__device__ inline void write_tile_lower(double* __restrict__ K, int ld, int n, int r0, int c0,
                                        const Tile& T, bool diag) {
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    v[q] = T[e >> 6][e & 63];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int i = e >> 6, j = e & 63;
    if (r0 + i < n && c0 + j < n && (!diag || j <= i)) K[(long long)(r0 + i) * ld + c0 + j] = v[q];
  }
}

// W_k to global memory; its 16 x 16 blocks above the diagonal are zero by definition and are
// written as zeros without being read.  Wavefront w stores the largest |entry| it wrote to
// cslot[2w + 1].
__device__ inline void write_w(double* __restrict__ Wk, const Tile& W, double* __restrict__ cslot) {
  double v[16], mw = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int i = e >> 6, j = e & 63;
    v[q] = (j >> 4) <= (i >> 4) ? W[i][j] : 0.0;
    mw = fmax(mw, fabs(v[q]));
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) Wk[threadIdx.x + 256 * q] = v[q];
  mw = wave_max(mw);
  if ((threadIdx.x & 63) == 0) cslot[2 * (threadIdx.x >> 6) + 1] = mw;
}

__device__ inline void load_w(const double* __restrict__ Wk, Tile& W) {
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = Wk[threadIdx.x + 256 * q];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    W[e >> 6][e & 63] = v[q];
  }
}

// A factor tile (lower triangle of K at (r0, r0); the rest of the tile as 0) into T.
__device__ inline void load_lower_tile(const double* __restrict__ K, int ld, int n, int r0,
                                       Tile& T) {
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int i = e >> 6, j = e & 63;
    v[q] = (j <= i && r0 + i < n) ? K[(long long)(r0 + i) * ld + r0 + j] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    T[e >> 6][e & 63] = v[q];
  }
}

// Condition figures of a factored diagonal tile, 8 doubles beside the inverses: wavefront w
// stores the largest |L_ij| among the factor entries it scales (slot[2w], chol_inv64) and the
// largest |W_ij| among the inverse entries it writes (slot[2w+1], write_w).  A panel formed
// with the explicit inverse, A W', has a relative error up to about 64 eps max|L| max|W|; a
// triangular solve's error does not grow with that product.
// Panels of a tile column whose max|L| max|W| exceeds this are refined (refine_panel): below
// it the inverse-based panel loses at most about three digits more than a triangular solve.
constexpr double kRefineCond = 1e3;

__device__ inline bool panel_needs_refine(const double* __restrict__ slot) {
  const double ml = fmax(fmax(slot[0], slot[2]), fmax(slot[4], slot[6]));
  const double mw = fmax(fmax(slot[1], slot[3]), fmax(slot[5], slot[7]));
  return ml * mw > kRefineCond;
}

// One step of iterative refinement of the panel X = A W' of tile column k0 / 64 (W = L_kk^-1,
// L_kk the factor tile at (k0, k0) of K): X <- X + (A - X L_kk') W'.  On entry acc holds X,
// the product of Xa (= A) with Wt (= W), and likewise accb for Xb when two is set; on exit
// acc (accb) hold the refined panel, Wt holds W again and Xa, Xb hold scratch.  The step
// brings the panel's error down to that of a triangular solve (Higham, Accuracy and
// Stability of Numerical Algorithms, Ch. 12: one step of refinement in the working
// precision makes a solver with a small enough forward error backward stable).
__device__ __forceinline__ void refine_panel(const double* __restrict__ K, int ld, int n, int k0,
                             const double* __restrict__ Wk, Tile& Wt, Tile& Xa,
                             d4 (&acc)[2][2], Tile& Xb, d4 (&accb)[2][2], bool two, int wr,
                             int wc, int li, int lk) {
  d4 r[2][2], rb[2][2];  // A at this thread's accumulator positions, then the residual
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 32 * wr + 16 * ib + lk + 4 * v, j = 32 * wc + 16 * jb + li;
        r[ib][jb][v] = Xa[i][j];
        rb[ib][jb][v] = two ? Xb[i][j] : 0.0;
      }
  __syncthreads();  // the products that read Xa, Xb and Wt are complete
  store_acc(Xa, acc, wr, wc, li, lk);
  if (two) store_acc(Xb, accb, wr, wc, li, lk);
  load_lower_tile(K, ld, n, k0, Wt);
  __syncthreads();
  mma_abt_add(Xa, Wt, r, wr, wc, li, lk, true);  // R = A - X L_kk'
  if (two) mma_abt_add(Xb, Wt, rb, wr, wc, li, lk, true);
  __syncthreads();
  store_acc(Xa, r, wr, wc, li, lk);
  if (two) store_acc(Xb, rb, wr, wc, li, lk);
  load_w(Wk, Wt);
  __syncthreads();
  mma_abt_add(Xa, Wt, acc, wr, wc, li, lk);  // X += R W'
  if (two) mma_abt_add(Xb, Wt, accb, wr, wc, li, lk);
}

// Pivot failure: a low-precision K (mixed modes) is formed again one precision level higher
// (done = 2 skips the rest of the iteration); otherwise the breakdown is reported.
__device__ inline void chol_fail(int col, int* done, int* info, int* status, int* lowflag) {
  if (lowflag != nullptr && *lowflag) {
    *lowflag -= 1;  // one precision level up (BF16 -> FP32 -> FP64) and redo the iteration
    *done = 2;
    return;
  }
  *info = col;
  *status = CMPC_ERR_CHOLESKY;
  *done = 1;
}

__device__ __forceinline__ void chol_first_body(int bid, double* __restrict__ K, int ld, int n,
                                                         double* __restrict__ Wall, int* done,
                                                         int* info, int* status, int* lowflag) {
  __shared__ Tile T, W;
  __shared__ double colb[128], piv[64];
  __shared__ int bad;
  if (*done) return;
  load_tile(K, ld, n, 0, 0, T);
  __syncthreads();
  const int nvalid = n < 64 ? n : 64;
  double* cslot = Wall + 4096 * (long long)((n + 63) >> 6);  // tile 0's condition figures
  if (!chol_inv64(T, W, colb, piv, nvalid, &bad, K, ld, n, 0, 0, cslot)) {
    if (threadIdx.x == 0) chol_fail(bad + 1, done, info, status, lowflag);
    return;
  }
  write_w(Wall, W, cslot);
}

__global__ __launch_bounds__(256) void chol_first_kernel(double* __restrict__ K, int ld, int n,
                                                         double* __restrict__ Wall, int* done,
                                                         int* info, int* status, int* lowflag) {
  chol_first_body(blockIdx.x, K, ld, n, Wall, done, info, status, lowflag);
}

// Forward substitution for row block j on one 256-thread workgroup (4 lanes per row):
// y_j = W_j (S b_j - sum_{m<j} L_jm y_m), the y_m of earlier blocks read from y.  Where the
// diagonal tile is ill-conditioned (its condition figures, as for the panels) the block takes
// one step of refinement, y_j += W_j (r - L_jj y_j), so that its error is that of a
// substitution with L_jj.
__device__ __forceinline__ void fwd_block_body(int j, const double* __restrict__ L, int ld, int n,
                                               const double* __restrict__ Wall,
                                               const double* __restrict__ b,
                                               const double* __restrict__ eq,
                                               double* __restrict__ y) {
  __shared__ double rs[64], yj[64];
  const int t = threadIdx.x, i = t >> 2, g = t & 3;
  const int j0 = 64 * j, rows = min(64, n - j0);
  const bool refine = panel_needs_refine(Wall + 4096 * (long long)((n + 63) >> 6) + 8 * j);
  double acc = 0.0;
  if (i < rows) {
    const double* row = L + (long long)(j0 + i) * ld;
    double acc2 = 0.0;
    int c = g;
#pragma unroll 4
    for (; c + 4 < j0; c += 8) {
      acc = fma(row[c], y[c], acc);
      acc2 = fma(row[c + 4], y[c + 4], acc2);
    }
    if (c < j0) acc = fma(row[c], y[c], acc);
    acc += acc2;
  }
  acc += dpp_f64<0xB1>(acc);  // quad sum
  acc += dpp_f64<0x4E>(acc);
  if (g == 0) rs[i] = i < rows ? (eq ? eq[j0 + i] * b[j0 + i] : b[j0 + i]) - acc : 0.0;
  __syncthreads();
  const double* W = Wall + (long long)j * 4096 + i * 64;
  double v = 0.0;
#pragma unroll
  for (int q = g; q < 64; q += 4) v = fma(W[q], rs[q], v);
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  if (refine) {  // uniform
    if (g == 0) yj[i] = v;
    __syncthreads();
    double e = 0.0;  // (L_jj y_j)_i, lower triangle
    if (i < rows) {
      const double* row = L + (long long)(j0 + i) * ld + j0;
      for (int q = g; q <= i; q += 4) e = fma(row[q], yj[q], e);
    }
    e += dpp_f64<0xB1>(e);
    e += dpp_f64<0x4E>(e);
    if (g == 0) rs[i] = i < rows ? rs[i] - e : 0.0;  // every read of rs preceded the barrier
    __syncthreads();
    double d = 0.0;
#pragma unroll
    for (int q = g; q < 64; q += 4) d = fma(W[q], rs[q], d);
    d += dpp_f64<0xB1>(d);
    d += dpp_f64<0x4E>(d);
    v += d;
  }
  if (g == 0 && i < rows) y[j0 + i] = v;
}

// Launch k: (A) the panel of block column k-1, L_i,k-1 = A_i,k-1 W_k-1' for i >= k, written
// now because launch k-1 still read A_i,k-1 while forming its updates; (B) for k <= nt-2 the
// trailing update with block column k, and the factorisation of the next pivot tile.
// (C) with fb != NULL, the workgroup after the tiles (launched when fwd_block_at(k, nt) >= 0)
// runs the forward substitution of that row block, whose row of L the earlier launches
// completed.
__device__ __forceinline__ void chol_step_body(int bid, double* __restrict__ K, int ld, int n,
                                                        int k, int nt, double* __restrict__ Wall,
                                                        int* done, int* info, int* status,
                                                        int* lowflag, const double* fb,
                                                        const double* feq, double* fy) {
  __shared__ Tile Wt, Xi, Xj;
  __shared__ double colb[128], piv[64];
  __shared__ int bad;
  if (*done) return;
  if (fb != nullptr) {
    const int rows_t = nt - 1 - k;
    if (bid == (k >= 1 ? nt - k : 0) + rows_t * (rows_t + 1) / 2) {
      fwd_block_body(fwd_block_at(k, nt), K, ld, n, Wall, fb, feq, fy);
      return;
    }
  }
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int wr = wave >> 1, wc = wave & 1;
  double* cond = Wall + 4096 * (long long)nt;  // condition figures, 8 per tile
  int b = bid;
  d4 acc[2][2];
  const int npanel = k >= 1 ? nt - k : 0;
  if (b < npanel) {  // (A) panel tile (k + b, k - 1)
    const int r0 = 64 * (k + b), c0 = 64 * (k - 1);
    load_w(Wall + (long long)(k - 1) * 4096, Wt);
    load_tile(K, ld, n, r0, c0, Xi);
    __syncthreads();
    mma_abt(Xi, Wt, acc, wr, wc, li, lk);
    if (panel_needs_refine(cond + 8 * (k - 1)))  // uniform: one value for the workgroup
      refine_panel(K, ld, n, c0, Wall + (long long)(k - 1) * 4096, Wt, Xi, acc, Xj, acc, false,
                   wr, wc, li, lk);
    __syncthreads();
    store_acc(Xi, acc, wr, wc, li, lk);
    __syncthreads();
    write_tile_lower(K, ld, n, r0, c0, Xi, false);
    return;
  }
  b -= npanel;
  // (B) update tile (ti, tj), k+1 <= tj <= ti: lower-triangular index b
  int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= b) ++I;
  while (I > 0 && I * (I + 1) / 2 > b) --I;
  const int J = b - I * (I + 1) / 2;
  const int ti = k + 1 + I, tj = k + 1 + J;
  const int r0 = 64 * ti, c0 = 64 * tj, k0 = 64 * k;
  const bool diag = ti == tj;
  const bool pivot = diag && ti == k + 1;
  // Xj: tile (tj, k) for an off-diagonal tile; for the next pivot tile its own A_ij, loaded
  // now with the rest (a diagonal tile's product uses Xi twice)
  load_w_tiles(Wall + (long long)k * 4096, Wt, K, ld, n, r0, k0, Xi, !diag || pivot,
               diag ? r0 : c0, diag ? c0 : k0, Xj);
  __syncthreads();
  mma_abt(Xi, Wt, acc, wr, wc, li, lk);  // X_i = A_ik W_k'
  d4 accj[2][2];
  if (!diag) mma_abt(Xj, Wt, accj, wr, wc, li, lk);  // X_j
  if (panel_needs_refine(cond + 8 * k))  // the same decision as the panel's own launch
    refine_panel(K, ld, n, k0, Wall + (long long)k * 4096, Wt, Xi, acc, Xj, accj, !diag, wr, wc,
                 li, lk);
  __syncthreads();
  store_acc(Xi, acc, wr, wc, li, lk);
  if (!diag) store_acc(Xj, accj, wr, wc, li, lk);
  __syncthreads();
  mma_abt(Xi, diag ? Xi : Xj, acc, wr, wc, li, lk);  // X_i X_j'
  __syncthreads();
  if (!pivot) {
    if (diag && wc > wr) return;
    double old[2][2][4];
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gi = r0 + 32 * wr + 16 * ib + lk + 4 * v;
          const int gj = c0 + 32 * wc + 16 * jb + li;
          old[ib][jb][v] = (gi < n && gj <= gi) ? K[(long long)gi * ld + gj] : 0.0;
        }
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gi = r0 + 32 * wr + 16 * ib + lk + 4 * v;
          const int gj = c0 + 32 * wc + 16 * jb + li;
          if (gi < n && gj <= gi) K[(long long)gi * ld + gj] = old[ib][jb][v] - acc[ib][jb][v];
        }
    return;
  }
  // the next pivot tile (already in Xj): update in LDS, factor, invert, publish
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Xj[32 * wr + 16 * ib + lk + 4 * v][32 * wc + 16 * jb + li] -= acc[ib][jb][v];
  __syncthreads();
  const int nvalid = n - r0 < 64 ? n - r0 : 64;
  if (!chol_inv64(Xj, Xi, colb, piv, nvalid, &bad, K, ld, n, r0, c0, cond + 8 * (k + 1))) {
    if (threadIdx.x == 0) chol_fail(r0 + bad + 1, done, info, status, lowflag);
    return;
  }
  write_w(Wall + (long long)(k + 1) * 4096, Xi, cond + 8 * (k + 1));
}

__global__ __launch_bounds__(256) void chol_step_kernel(double* __restrict__ K, int ld, int n,
                                                        int k, int nt, double* __restrict__ Wall,
                                                        int* done, int* info, int* status,
                                                        int* lowflag, const double* fb,
                                                        const double* feq, double* fy) {
  chol_step_body(blockIdx.x, K, ld, n, k, nt, Wall, done, info, status, lowflag, fb, feq, fy);
}

int launch_potrf(hipStream_t s, double* K, int n, int ld, double* Wall, int* done, int* info,
                 int* status, hipEvent_t ev_start, hipEvent_t ev_stop, int* lowflag,
                 const double* fb, const double* feq, double* fy) {
  if (n > kPotrsSingleMax) fb = nullptr;
  const int nt = ceil_div(n, 64);
  hipExtLaunchKernelGGL(chol_first_kernel, dim3(1), dim3(256), 0, s, ev_start,
                        nt == 1 ? ev_stop : nullptr, 0, K, ld, n, Wall, done, info, status,
                        lowflag);
  CMPC_LAUNCH_CHECK();
  for (int k = 0; k < nt && nt > 1; ++k) {
    const int npanel = k >= 1 ? nt - k : 0;
    const int rows = nt - 1 - k;
    const int tiles = npanel + rows * (rows + 1) / 2 + (fb != nullptr && fwd_block_at(k, nt) >= 0);
    hipExtLaunchKernelGGL(chol_step_kernel, dim3(tiles), dim3(256), 0, s, (hipEvent_t) nullptr,
                          k == nt - 1 ? ev_stop : nullptr, 0, K, ld, n, k, nt, Wall, done, info,
                          status, lowflag, fb, feq, fy);
    CMPC_LAUNCH_CHECK();
  }
  return 0;
}

// Inverses of the diagonal tiles of an existing factor and their condition figures (for a
// standalone solve; one workgroup per tile, grid = ceil(n / 64)).
__global__ __launch_bounds__(256) void tri_inv_kernel(const double* __restrict__ L, int ld, int n,
                                                      double* __restrict__ Wall) {
  __shared__ Tile T, W;
  const int r0 = 64 * blockIdx.x;
  const int nvalid = n - r0 < 64 ? n - r0 : 64;
  load_tile(L, ld, n, r0, r0, T);
  __syncthreads();
  __shared__ double rdiag[64];
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int i = e >> 6, j = e & 63;
    if (j > i) T[i][j] = 0.0;
    if (i >= nvalid) T[i][j] = (i == j) ? 1.0 : 0.0;
  }
  // the diagonal entries of valid rows are not rewritten above
  if (threadIdx.x < 64) rdiag[threadIdx.x] = threadIdx.x < nvalid ? recip(T[threadIdx.x][threadIdx.x]) : 1.0;
  __syncthreads();
  double* cslot = Wall + 4096 * (long long)gridDim.x + 8 * blockIdx.x;
  double ml = 0.0;
  for (int e = threadIdx.x; e < 4096; e += 256) ml = fmax(ml, fabs(T[e >> 6][e & 63]));
  ml = wave_max(ml);
  if ((threadIdx.x & 63) == 0) cslot[2 * (threadIdx.x >> 6)] = ml;
  inv64(T, W, rdiag);
  write_w(Wall + (long long)blockIdx.x * 4096, W, cslot);
}

int launch_tri_inv(hipStream_t s, const double* L, int n, int ld, double* Wall) {
  hipLaunchKernelGGL(tri_inv_kernel, dim3(ceil_div(n, 64)), dim3(256), 0, s, L, ld, n, Wall);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// Triangular solves with the factor L and the diagonal-tile inverses W_k, one launch per
// 64-row block, many workgroups per launch.
//   forward step k:  y_k = W_k b_k  (b_k already holds b_k - sum_{j<k} L_kj y_j), and the
//                    workgroup for block i > k applies b_i -= L_ik y_k;
//   backward step k: x_k = W_k' y_k  (y_k already reduced by the blocks below), and the
//                    workgroup for block j < k applies y_j -= L_kj' x_k.
// Every workgroup recomputes the 64-long block solution (a 64 x 64 product) itself, so the
// launch needs no inter-workgroup synchronisation; workgroup 0 stores it.

// v = M u (trans = false) or M' u (trans = true) for the 64 x 64 tile M (row-major, ld 64);
// u, v in LDS.  4 lanes per output entry.
__device__ inline void tile_mv64(const double* __restrict__ M, const double* u, double* v,
                                 bool trans) {
  const int r = threadIdx.x >> 2, p = threadIdx.x & 3;
  double acc = 0.0;
  if (!trans) {
    for (int m = p; m < 64; m += 4) acc = fma(M[r * 64 + m], u[m], acc);
  } else {
    for (int m = p; m < 64; m += 4) acc = fma(M[m * 64 + r], u[m], acc);
  }
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  if (p == 0) v[r] = acc;
}

// v = L_kk^-1 u (trans: L_kk^-T u) for diagonal block k (rows k0 .. k0 + 63 of L, the part
// past n as identity) with its inverse W_k: v = W u, and where the tile is ill-conditioned one
// step of refinement v += W (u - L_kk v).  u, v, e (scratch) in LDS; ends with a barrier.
__device__ inline void tile_solve64(const double* __restrict__ Wk, const double* __restrict__ L,
                                    int ld, int n, int k0, bool refine, double* u, double* v,
                                    double* e, bool trans) {
  tile_mv64(Wk, u, v, trans);
  __syncthreads();
  if (!refine) return;
  const int r = threadIdx.x >> 2, p = threadIdx.x & 3;
  double acc = 0.0;  // (L_kk v)_r or (L_kk' v)_r over the valid rows
  if (k0 + r < n) {
    if (!trans) {
      for (int m = p; m <= r; m += 4) acc = fma(L[(long long)(k0 + r) * ld + k0 + m], v[m], acc);
    } else {
      for (int m = r + p; m < 64 && k0 + m < n; m += 4)
        acc = fma(L[(long long)(k0 + m) * ld + k0 + r], v[m], acc);
    }
  }
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  if (p == 0) e[r] = k0 + r < n ? u[r] - acc : 0.0;
  __syncthreads();
  double d = 0.0;
  if (!trans) {
    for (int m = p; m < 64; m += 4) d = fma(Wk[r * 64 + m], e[m], d);
  } else {
    for (int m = p; m < 64; m += 4) d = fma(Wk[m * 64 + r], e[m], d);
  }
  d += __shfl_xor(d, 1, 64);
  d += __shfl_xor(d, 2, 64);
  if (p == 0) v[r] += d;
  __syncthreads();
}

__device__ __forceinline__ void trsv_fwd_step_body(int bid, const double* __restrict__ L, int ld,
                                                           int n, const double* __restrict__ Wall,
                                                           double* __restrict__ b,
                                                           double* __restrict__ y, int k,
                                                           const int* __restrict__ done) {
  __shared__ double bk[64], yk[64], ek[64];
  if (done != nullptr && *done) return;
  const int k0 = 64 * k, t = threadIdx.x;
  const bool refine = panel_needs_refine(Wall + 4096 * (long long)((n + 63) >> 6) + 8 * k);
  if (t < 64) bk[t] = (k0 + t < n) ? b[k0 + t] : 0.0;
  __syncthreads();
  tile_solve64(Wall + (long long)k * 4096, L, ld, n, k0, refine, bk, yk, ek, false);
  if (bid == 0 && t < 64 && k0 + t < n) y[k0 + t] = yk[t];
  const int i0 = k0 + 64 * (1 + (int)bid);
  if (i0 >= n) return;
  // b_i -= L_ik y_k: 4 lanes per row of block i
  const int r = t >> 2, p = t & 3;
  double acc = 0.0;
  if (i0 + r < n) {
    const double* rp = L + (long long)(i0 + r) * ld + k0;
    for (int m = p; m < 64; m += 4) acc = fma(rp[m], yk[m], acc);
  }
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  if (p == 0 && i0 + r < n) b[i0 + r] -= acc;
}

__global__ __launch_bounds__(256) void trsv_fwd_step_kernel(const double* __restrict__ L, int ld,
                                                           int n, const double* __restrict__ Wall,
                                                           double* __restrict__ b,
                                                           double* __restrict__ y, int k,
                                                           const int* __restrict__ done) {
  trsv_fwd_step_body(blockIdx.x, L, ld, n, Wall, b, y, k, done);
}

__device__ __forceinline__ void trsv_bwd_step_body(int bid, const double* __restrict__ L, int ld,
                                                           int n, const double* __restrict__ Wall,
                                                           double* __restrict__ y,
                                                           double* __restrict__ x, int k,
                                                           const int* __restrict__ done) {
  __shared__ double ykk[64], xk[64], ek[64];
  if (done != nullptr && *done) return;
  const int k0 = 64 * k, t = threadIdx.x;
  const bool refine = panel_needs_refine(Wall + 4096 * (long long)((n + 63) >> 6) + 8 * k);
  if (t < 64) ykk[t] = (k0 + t < n) ? y[k0 + t] : 0.0;
  __syncthreads();
  tile_solve64(Wall + (long long)k * 4096, L, ld, n, k0, refine, ykk, xk, ek, true);
  if (bid == 0 && t < 64 && k0 + t < n) x[k0 + t] = xk[t];
  const int j = bid;
  if (j >= k) return;
  // y_j -= L_kj' x_k: column c of block j gets sum_r L[k0 + r][64 j + c] x_k[r]
  const int c = t & 63, g = t >> 6;
  double acc = 0.0;
  for (int r = g; r < 64; r += 4)
    if (k0 + r < n) acc = fma(L[(long long)(k0 + r) * ld + 64 * j + c], xk[r], acc);
  __shared__ double red[4][64];
  red[g][c] = acc;
  __syncthreads();
  if (g == 0) y[64 * j + c] -= (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

__global__ __launch_bounds__(256) void trsv_bwd_step_kernel(const double* __restrict__ L, int ld,
                                                           int n, const double* __restrict__ Wall,
                                                           double* __restrict__ y,
                                                           double* __restrict__ x, int k,
                                                           const int* __restrict__ done) {
  trsv_bwd_step_body(blockIdx.x, L, ld, n, Wall, y, x, k, done);
}

// dst = eq o src (eq == NULL: plain copy); returns at entry when *gate is set
__global__ void scale_copy_kernel(double* __restrict__ dst, const double* __restrict__ src,
                                  const double* __restrict__ eq, int n,
                                  const int* __restrict__ gate) {
  if (gate != nullptr && *gate) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = eq ? eq[i] * src[i] : src[i];
}

// Diagonal equilibration of the lower triangle of K before the factorisation (mixed
// modes): eq_i = K_ii^-1/2 (1 if K_ii is not positive: the factorisation reports it), then
// K_ij <- eq_i K_ij eq_j.  The solution of K p = r is p = S (S K S)^-1 S r, S = diag(eq).
__device__ __forceinline__ void equil_diag_body(int bid, const double* __restrict__ K, int n,
                                                int ld, double* __restrict__ eq,
                                                const int* __restrict__ done) {
  if (done != nullptr && *done) return;
  const int i = bid * 256 + threadIdx.x;
  if (i < n) {
    const double d = K[(long long)i * ld + i];
    eq[i] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
  }
}

// one wavefront per row (4 rows per workgroup)
__device__ __forceinline__ void equil_scale_body(int bid, double* __restrict__ K, int n, int ld,
                                                 const double* __restrict__ eq,
                                                 const int* __restrict__ done) {
  if (done != nullptr && *done) return;
  const int i = bid * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const double ei = eq[i];
  double* row = K + (long long)i * ld;
  for (int j = threadIdx.x & 63; j <= i; j += 64) row[j] *= ei * eq[j];
}

__global__ __launch_bounds__(256) void equil_diag_kernel(const double* __restrict__ K, int n,
                                                         int ld, double* __restrict__ eq,
                                                         const int* __restrict__ done) {
  equil_diag_body(blockIdx.x, K, n, ld, eq, done);
}
__global__ __launch_bounds__(256) void equil_scale_kernel(double* __restrict__ K, int n, int ld,
                                                          const double* __restrict__ eq,
                                                          const int* __restrict__ done) {
  equil_scale_body(blockIdx.x, K, n, ld, eq, done);
}

int launch_equilibrate(hipStream_t s, double* K, int n, int ld, double* eq, const int* done) {
  hipLaunchKernelGGL(equil_diag_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, K, n, ld, eq,
                     done);
  CMPC_LAUNCH_CHECK();
  hipLaunchKernelGGL(equil_scale_kernel, dim3(ceil_div(n, 4)), dim3(256), 0, s, K, n, ld, eq,
                     done);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// Bit k set: diagonal tile k is ill-conditioned (its condition figures exceed kRefineCond), and
// the substitutions with it take one step of refinement.  nt <= 64.  Wavefront 0 forms the
// mask and lane 0 stores it; it is read after the caller's next barrier.
__device__ inline void refine_mask(const double* __restrict__ Wall, int nt,
                                   unsigned long long* mask) {
  if (threadIdx.x < 64) {
    const int k = threadIdx.x;
    const bool f = k < nt && panel_needs_refine(Wall + 4096 * (long long)nt + 8 * k);
    const unsigned long long m = __ballot(f);
    if (k == 0) *mask = m;
  }
}

// The 16 lanes of each DPP row get the sum of the row's values.
__device__ inline double rowsum16(double x) {
  x += dpp_f64<0xB1>(x);   // quad_perm: lane ^ 1
  x += dpp_f64<0x4E>(x);   // quad_perm: lane ^ 2
  x += dpp_f64<0x124>(x);  // row_ror:4
  x += dpp_f64<0x128>(x);  // row_ror:8
  return x;
}

// One step of refinement of the forward block y_k = W_k r (r in rs, y_k in ys[k0 ..]) on 1024
// threads, row i of the block on the 16 lanes g of a DPP row: y_k += W_k (r - L_kk y_k); wrow:
// the lane's entries (i, g + 16 q) of W_k.  Begins and ends after a barrier.
__device__ inline void refine_fwd_block(const double* __restrict__ L, int ld, int n, int k0,
                                        const double (&wrow)[4], double* ys, const double* rs,
                                        double* es) {
  const int t = threadIdx.x, i = t >> 4, g = t & 15;
  const bool valid = k0 + i < n;
  double a = 0.0;
  if (valid) {
    const double* row = L + (long long)(k0 + i) * ld + k0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (g + 16 * q <= i) a = fma(row[g + 16 * q], ys[k0 + g + 16 * q], a);
  }
  a = rowsum16(a);
  if (g == 0) es[i] = valid ? rs[i] - a : 0.0;
  __syncthreads();
  double d = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) d = fma(wrow[q], es[g + 16 * q], d);
  d = rowsum16(d);
  if (g == 0 && valid) ys[k0 + i] += d;
  __syncthreads();
}

// The same for the backward block x_k = W_k' r, column i of the block on lane i of wavefront
// g: x_k += W_k' (r - L_kk' x_k); wcol: the lane's entries (g + 16 q, i) of W_k.
__device__ inline void refine_bwd_block(const double* __restrict__ L, int ld, int n, int k0,
                                        const double (&wcol)[4], double* ys, const double* rs,
                                        double* es, double (*red)[65]) {
  const int t = threadIdx.x, i = t & 63, g = t >> 6;
  double a = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = g + 16 * q;
    if (m >= i && k0 + m < n) a = fma(L[(long long)(k0 + m) * ld + k0 + i], ys[k0 + m], a);
  }
  red[g][i] = a;
  __syncthreads();
  if (g == 0) {
    double sum = 0.0;
    for (int q = 0; q < 16; ++q) sum += red[q][i];
    es[i] = k0 + i < n ? rs[i] - sum : 0.0;
  }
  __syncthreads();
  double d = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) d = fma(wcol[q], es[g + 16 * q], d);
  red[g][i] = d;
  __syncthreads();
  if (g == 0 && k0 + i < n) {
    double sum = 0.0;
    for (int q = 0; q < 16; ++q) sum += red[q][i];
    ys[k0 + i] += sum;
  }
  __syncthreads();
}

// The one-workgroup solves' start: ys <- S b (zero past n; the fused forward pass's y below
// block kf) and the refinement mask (no barrier: the caller's next one publishes both).
__device__ inline void potrs_prologue(const double* __restrict__ Wall, const double* __restrict__ b,
                                      const double* __restrict__ eq,
                                      const double* __restrict__ yf, int n, int nt, int kf,
                                      double* ys, unsigned long long* mask) {
  refine_mask(Wall, nt, mask);
  for (int i = threadIdx.x; i < 64 * nt; i += 1024)
    ys[i] = i < 64 * kf ? yf[i] : (i < n ? (eq ? eq[i] * b[i] : b[i]) : 0.0);
}

// Both triangular solves in one workgroup of 1024 threads (16 wavefronts), the vector held in
// LDS (ys, filled by the caller; blocks below kf already hold y): forward, for each 64-row
// block k, r = b_k - L_k,<k y_<k (16 lanes per row, a row segment of 16 consecutive columns per
// load) and y_k = W_k r; backward, for k from the last block down, r = y_k - L_>k,k' x_>k (a
// wavefront per 16th of the rows, 64 consecutive columns per load) and x_k = W_k' r.  Blocks
// whose bit is set in refm take one step of refinement after each product.  Partial sums are
// reduced in a fixed order.  One launch replaces 2 ceil(n/64) + 2 launches of the block-step
// kernels.  eq != NULL: x = S (..)^-1 S b.
__device__ __forceinline__ void potrs_single_body(const double* __restrict__ L, int ld, int n,
                                                  const double* __restrict__ Wall,
                                                  double* __restrict__ x,
                                                  const double* __restrict__ eq, double* ys,
                                                  double* rs, double (*red)[65], int kf,
                                                  unsigned long long refm, double* es,
                                                  int accumulate) {
  const int t = threadIdx.x;
  const int nt = (n + 63) >> 6;
  // ---- forward: L y = b
  {
    const int i = t >> 4, g = t & 15;  // row of the block, column phase
    for (int k = kf; k < nt; ++k) {
      const int k0 = 64 * k;
      const int rows = min(64, n - k0);
      const double* W = Wall + (long long)k * 4096;
      double wv[4];  // this lane's entries of row i of W_k, loaded behind the dot product
#pragma unroll
      for (int q = 0; q < 4; ++q) wv[q] = W[i * 64 + g + 16 * q];
      double acc = 0.0;
      if (i < rows) {
        const double* row = L + (long long)(k0 + i) * ld;
        double acc2 = 0.0;  // two chains; 16 loads in flight per lane
        int c = g;
#pragma unroll 8
        for (; c + 16 < k0; c += 32) {
          acc = fma(row[c], ys[c], acc);
          acc2 = fma(row[c + 16], ys[c + 16], acc2);
        }
        if (c < k0) acc = fma(row[c], ys[c], acc);
        acc += acc2;
      }
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      acc += __shfl_xor(acc, 4, 64);
      acc += __shfl_xor(acc, 8, 64);
      if (g == 0) rs[i] = i < rows ? ys[k0 + i] - acc : 0.0;
      __syncthreads();
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) v = fma(wv[q], rs[g + 16 * q], v);
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      if (g == 0 && i < rows) ys[k0 + i] = v;
      __syncthreads();
      if ((refm >> k) & 1ull) refine_fwd_block(L, ld, n, k0, wv, ys, rs, es);
    }
  }
  // ---- backward: L' x = y (x overwrites y block by block)
  {
    const int i = t & 63, g = t >> 6;  // column of the block, row phase (one wavefront each)
    for (int k = nt - 1; k >= 0; --k) {
      const int k0 = 64 * k;
      const int rows = min(64, n - k0);
      const double* W = Wall + (long long)k * 4096;
      double wv[4];  // entries (m, i) of W_k for m = g + 16 q
#pragma unroll
      for (int q = 0; q < 4; ++q) wv[q] = W[(g + 16 * q) * 64 + i];
      double acc = 0.0;
      if (i < rows) {
        double acc2 = 0.0;
        int r = k0 + 64 + g;
#pragma unroll 8
        for (; r + 16 < n; r += 32) {
          acc = fma(L[(long long)r * ld + k0 + i], ys[r], acc);
          acc2 = fma(L[(long long)(r + 16) * ld + k0 + i], ys[r + 16], acc2);
        }
        if (r < n) acc = fma(L[(long long)r * ld + k0 + i], ys[r], acc);
        acc += acc2;
      }
      red[g][i] = acc;
      __syncthreads();
      if (g == 0) {
        double sum = 0.0;
        for (int q = 0; q < 16; ++q) sum += red[q][i];
        rs[i] = i < rows ? ys[k0 + i] - sum : 0.0;
      }
      __syncthreads();
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) v = fma(wv[q], rs[g + 16 * q], v);
      red[g][i] = v;
      __syncthreads();
      if (g == 0 && i < rows) {
        double sum = 0.0;
        for (int q = 0; q < 16; ++q) sum += red[q][i];
        ys[k0 + i] = sum;
      }
      __syncthreads();
      if ((refm >> k) & 1ull) refine_bwd_block(L, ld, n, k0, wv, ys, rs, es, red);
    }
  }
  for (int i = t; i < n; i += 1024) {
    const double v = eq ? eq[i] * ys[i] : ys[i];
    x[i] = accumulate ? x[i] + v : v;
  }
}

// The same two substitutions for n <= 64 NT with NT <= 8 block steps, unrolled so that the
// loads of the next step are issued early: while step k reduces, multiplies by W_k and passes
// its barriers, the rows of L (forward: row block k+1 left of the diagonal; backward: column
// block k-1 below it) and then the next W tile are already in flight to registers.  ys holds
// 64 NT doubles, zero past n, so rows past n contribute nothing.
template <int NT>
__device__ __forceinline__ void potrs_pipe_body(const double* __restrict__ L, int ld, int n,
                                                const double* __restrict__ Wall,
                                                const double* __restrict__ b,
                                                double* __restrict__ x,
                                                const double* __restrict__ eq, double* ys,
                                                double* rs, double (*red)[65],
                                                const double* __restrict__ yf, double* es,
                                                unsigned long long* mask, int accumulate) {
  const int t = threadIdx.x;
  const int kf = yf ? (NT > 2 ? NT - 2 : 0) : 0;  // blocks done by the fused forward pass
  potrs_prologue(Wall, b, eq, yf, n, NT, kf, ys, mask);
  double lr[4 * NT];
  double wv[4];
  {  // ---- forward: L y = b, row i of block k on 16 lanes (a DPP row), column phase g; with
     // yf only the blocks from kf on (their loads still issued one step ahead)
    const int i = t >> 4, g = t & 15;
#pragma unroll
    for (int q = 0; q < 4; ++q) wv[q] = Wall[(long long)kf * 4096 + i * 64 + g + 16 * q];
    __syncthreads();
    if (*mask != 0ull) {  // a tile to refine: the looped form (uniform)
      potrs_single_body(L, ld, n, Wall, x, eq, ys, rs, red, kf, *mask, es, accumulate);
      return;
    }
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const int k0 = 64 * k;
      const bool run = k >= kf;  // uniform
      const bool next = k + 1 < NT && k + 1 >= kf;
      double acc = 0.0;
      if (run) {
#pragma unroll
        for (int m = 0; m < 4 * k; ++m) acc = fma(lr[m], ys[g + 16 * m], acc);
      }
      if (next) {
        const double* row = L + (long long)min(k0 + 64 + i, n - 1) * ld + g;
#pragma unroll
        for (int m = 0; m < 4 * (k + 1); ++m) lr[m] = row[16 * m];
      }
      double v = 0.0;
      const bool valid = k0 + i < n;
      if (run) {
        acc = rowsum16(acc);
        if (g == 0) rs[i] = valid ? ys[k0 + i] - acc : 0.0;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) v = fma(wv[q], rs[g + 16 * q], v);
      }
      if (next) {
#pragma unroll
        for (int q = 0; q < 4; ++q) wv[q] = Wall[(long long)(k + 1) * 4096 + i * 64 + g + 16 * q];
      }
      if (run) {
        v = rowsum16(v);
        if (g == 0 && valid) ys[k0 + i] = v;
        __syncthreads();
      }
    }
  }
  {  // ---- backward: L' x = y, column i of block k, row phase g (one wavefront each)
    const int i = t & 63, g = t >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) wv[q] = Wall[(long long)(NT - 1) * 4096 + (g + 16 * q) * 64 + i];
#pragma unroll
    for (int kk = 0; kk < NT; ++kk) {
      const int k = NT - 1 - kk, k0 = 64 * k;
      double acc = 0.0;  // rows k0 + 64 + g + 16 m below the block
#pragma unroll
      for (int m = 0; m < 4 * kk; ++m) acc = fma(lr[m], ys[k0 + 64 + g + 16 * m], acc);
      if (k > 0) {
#pragma unroll
        for (int m = 0; m < 4 * (kk + 1); ++m)
          lr[m] = L[(long long)min(k0 + g + 16 * m, n - 1) * ld + k0 - 64 + i];
      }
      red[g][i] = acc;
      __syncthreads();
      if (g == 0) {
        double sum = 0.0;
        for (int q = 0; q < 16; ++q) sum += red[q][i];
        rs[i] = k0 + i < n ? ys[k0 + i] - sum : 0.0;
      }
      __syncthreads();
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) v = fma(wv[q], rs[g + 16 * q], v);
      if (k > 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) wv[q] = Wall[(long long)(k - 1) * 4096 + (g + 16 * q) * 64 + i];
      }
      red[g][i] = v;
      __syncthreads();
      if (g == 0 && k0 + i < n) {
        double sum = 0.0;
        for (int q = 0; q < 16; ++q) sum += red[q][i];
        ys[k0 + i] = sum;
      }
      __syncthreads();
    }
  }
  for (int i = t; i < n; i += 1024) {
    const double v = eq ? eq[i] * ys[i] : ys[i];
    x[i] = accumulate ? x[i] + v : v;
  }
}

// One workgroup solves: the pipelined form up to 8 block steps, the looped form beyond (and
// wherever a diagonal tile needs refinement).
__device__ __forceinline__ void potrs_one_body(const double* __restrict__ L, int ld, int n,
                                               const double* __restrict__ Wall,
                                               const double* __restrict__ b,
                                               double* __restrict__ x,
                                               const double* __restrict__ eq,
                                               const int* __restrict__ gate,
                                               const double* __restrict__ yf, int accumulate) {
  extern __shared__ double ys[];  // 64 ceil(n / 64)
  __shared__ double rs[64], es[64];
  __shared__ double red[16][65];
  __shared__ unsigned long long mask;
  if (gate != nullptr && *gate) return;
  switch ((n + 63) >> 6) {
    case 1: potrs_pipe_body<1>(L, ld, n, Wall, b, x, eq, ys, rs, red, yf, es, &mask, accumulate); break;
    case 2: potrs_pipe_body<2>(L, ld, n, Wall, b, x, eq, ys, rs, red, yf, es, &mask, accumulate); break;
    case 3: potrs_pipe_body<3>(L, ld, n, Wall, b, x, eq, ys, rs, red, yf, es, &mask, accumulate); break;
    case 4: potrs_pipe_body<4>(L, ld, n, Wall, b, x, eq, ys, rs, red, yf, es, &mask, accumulate); break;
    case 5: potrs_pipe_body<5>(L, ld, n, Wall, b, x, eq, ys, rs, red, yf, es, &mask, accumulate); break;
    case 6: potrs_pipe_body<6>(L, ld, n, Wall, b, x, eq, ys, rs, red, yf, es, &mask, accumulate); break;
    case 7: potrs_pipe_body<7>(L, ld, n, Wall, b, x, eq, ys, rs, red, yf, es, &mask, accumulate); break;
    case 8: potrs_pipe_body<8>(L, ld, n, Wall, b, x, eq, ys, rs, red, yf, es, &mask, accumulate); break;
    default: {
      const int nt = (n + 63) >> 6, kf = yf ? nt - 2 : 0;
      potrs_prologue(Wall, b, eq, yf, n, nt, kf, ys, &mask);
      __syncthreads();
      potrs_single_body(L, ld, n, Wall, x, eq, ys, rs, red, kf, mask, es, accumulate);
    }
  }
}

__global__ __launch_bounds__(1024) void potrs_single_kernel(const double* __restrict__ L, int ld,
                                                            int n, const double* __restrict__ Wall,
                                                            const double* __restrict__ b,
                                                            double* __restrict__ x,
                                                            const double* __restrict__ eq,
                                                            const int* __restrict__ gate,
                                                            const double* __restrict__ yf,
                                                            int accumulate) {
  potrs_one_body(L, ld, n, Wall, b, x, eq, gate, yf, accumulate);
}

// x = (L L')^-1 b (eq != NULL: x = S (L L')^-1 S b).  work: n doubles of scratch (the reduced
// right-hand side) for the block-step form; x may alias b.  n <= 4096 takes the one-launch
// form (the vector in LDS, at most 32 KB).
int launch_potrs(hipStream_t s, const double* L, int n, int ld, const double* Wall,
                 const double* b, double* x, double* work, const int* done, const double* eq,
                 const double* yf, int accumulate) {
  if (n <= kPotrsSingleMax) {
    hipLaunchKernelGGL(potrs_single_kernel, dim3(1), dim3(1024),
                       sizeof(double) * 64 * (size_t)ceil_div(n, 64), s, L,
                       ld, n, Wall, b, x, eq, done, yf, accumulate);
    CMPC_LAUNCH_CHECK();
    return 0;
  }
  const int nt = ceil_div(n, 64);
  if (work != b || eq != nullptr) {
    hipLaunchKernelGGL(scale_copy_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, work, b, eq, n,
                       done);
    CMPC_LAUNCH_CHECK();
  }
  for (int k = 0; k < nt; ++k) {  // forward: y (into x) from work
    hipLaunchKernelGGL(trsv_fwd_step_kernel, dim3(nt - k - 1 > 0 ? nt - k - 1 : 1), dim3(256), 0,
                       s, L, ld, n, Wall, work, x, k, done);
    CMPC_LAUNCH_CHECK();
  }
  for (int k = nt - 1; k >= 0; --k) {  // backward: x from y (x reduced in place)
    hipLaunchKernelGGL(trsv_bwd_step_kernel, dim3(k > 0 ? k : 1), dim3(256), 0, s, L, ld, n, Wall,
                       x, work, k, done);
    CMPC_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(scale_copy_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, x, work, eq, n,
                     done);
  CMPC_LAUNCH_CHECK();
  return 0;
}

// ---- work-list forms (batches).  Step k of every instance runs in one launch; an instance
// takes part in chol_step k when it has more than one tile column and k < nt, exactly as its
// own launch sequence would.  The factorisation kernels take one item per workgroup (grid =
// list length): their fully unrolled tile code does not fit the registers inside an item
// loop, and one step's list is short.  which = 0: solve rhs -> pv (gate st->done); which = 1: solve
// ref_res -> ref_dlt (gate st->ref_skip).  tmpn is the reduced right-hand side.
__global__ __launch_bounds__(256) void chol_first_batch_kernel(const InstView* __restrict__ views,
                                                               const WorkItem* __restrict__ items,
                                                               int nitems, int mixed) {
  if ((int)blockIdx.x >= nitems) return;
  const WorkItem it = items[blockIdx.x];
  const InstView& V = views[it.inst];
  chol_first_body(it.local, V.K, V.n, V.n, V.Wdiag, &V.st->done, &V.st->info, &V.st->status,
                  mixed ? &V.st->use_low : nullptr);
}

// fused: the list holds one more item per instance where fwd_block_at(k, nt) >= 0: the
// forward substitution of that row block of L y = S rhs into tmpn.
__global__ __launch_bounds__(256) void chol_step_batch_kernel(const InstView* __restrict__ views,
                                                              const WorkItem* __restrict__ items,
                                                              int nitems, int k, int mixed,
                                                              int fused, int eq) {
  if ((int)blockIdx.x >= nitems) return;
  const WorkItem it = items[blockIdx.x];
  const InstView& V = views[it.inst];
  chol_step_body(it.local, V.K, V.n, V.n, k, V.nt, V.Wdiag, &V.st->done, &V.st->info,
                 &V.st->status, mixed ? &V.st->use_low : nullptr, fused ? V.rhs : nullptr,
                 eq ? V.eqs : nullptr, V.tmpn);
}

// dir 0: tmpn = b (b = rhs or ref_res); dir 1: x = tmpn (x = pv or ref_dlt).  Items over
// 256-entry blocks of n.
__global__ __launch_bounds__(256) void potrs_copy_batch_kernel(const InstView* __restrict__ views,
                                                               const WorkItem* __restrict__ items,
                                                               int nitems, int which, int dir,
                                                               int eq) {
  CMPC_ITEMS_BEGIN
  if (*gate_of(V, which) == 0) {
    const int i = bid * 256 + threadIdx.x;
    if (i < V.n) {
      const double sc = eq ? V.eqs[i] : 1.0;
      if (dir == 0)
        V.tmpn[i] = eq ? sc * (which ? V.ref_res[i] : V.rhs[i]) : (which ? V.ref_res[i] : V.rhs[i]);
      else
        (which ? V.ref_dlt : V.pv)[i] = eq ? sc * V.tmpn[i] : V.tmpn[i];
    }
  }
  CMPC_ITEMS_END
}

__global__ __launch_bounds__(256) void equil_diag_batch_kernel(const InstView* __restrict__ views,
                                                               const WorkItem* __restrict__ items,
                                                               int nitems) {
  CMPC_ITEMS_BEGIN
  equil_diag_body(bid, V.K, V.n, V.n, V.eqs, &V.st->done);
  CMPC_ITEMS_END
}

__global__ __launch_bounds__(256) void equil_scale_batch_kernel(const InstView* __restrict__ views,
                                                                const WorkItem* __restrict__ items,
                                                                int nitems) {
  CMPC_ITEMS_BEGIN
  equil_scale_body(bid, V.K, V.n, V.n, V.eqs, &V.st->done);
  CMPC_ITEMS_END
}

__global__ __launch_bounds__(256) void trsv_fwd_batch_kernel(const InstView* __restrict__ views,
                                                             const WorkItem* __restrict__ items,
                                                             int nitems, int k, int which) {
  CMPC_ITEMS_BEGIN
  trsv_fwd_step_body(bid, V.K, V.n, V.n, V.Wdiag, V.tmpn, which ? V.ref_dlt : V.pv, k,
                     gate_of(V, which));
  CMPC_ITEMS_END
}

__global__ __launch_bounds__(256) void trsv_bwd_batch_kernel(const InstView* __restrict__ views,
                                                             const WorkItem* __restrict__ items,
                                                             int nitems, int k, int which) {
  CMPC_ITEMS_BEGIN
  trsv_bwd_step_body(bid, V.K, V.n, V.n, V.Wdiag, which ? V.ref_dlt : V.pv, V.tmpn, k,
                     gate_of(V, which));
  CMPC_ITEMS_END
}

int launch_b_chol_first(const ListArg& L, int mixed) {
  ListArg M = L;
  M.persistent = 0;  // one item per workgroup
  CMPC_LAUNCH_LIST(chol_first_batch_kernel, M, mixed);
}
int launch_b_chol_step(const ListArg& L, int k, int mixed, int fused, int eq) {
  ListArg M = L;
  M.persistent = 0;
  CMPC_LAUNCH_LIST(chol_step_batch_kernel, M, k, mixed, fused, eq);
}
// Whole solve of one instance per workgroup (1024 threads, the instance's vector in LDS).
__global__ __launch_bounds__(1024) void potrs_single_batch_kernel(
    const InstView* __restrict__ views, const WorkItem* __restrict__ items, int nitems, int which,
    int eq, int fused) {
  if ((int)blockIdx.x >= nitems) return;
  const WorkItem it = items[blockIdx.x];
  const InstView& V = views[it.inst];
  // which = 1: pv += the correction (the refinement's axpy in the solve's own store)
  potrs_one_body(V.K, V.n, V.n, V.Wdiag, which ? V.ref_res : V.rhs, V.pv, eq ? V.eqs : nullptr,
                 gate_of(V, which), fused && !which ? V.tmpn : nullptr, which);
}

int launch_b_potrs_single(const ListArg& L, int which, int eq, int nmax, int fused) {
  if (L.count <= 0) return 0;
  hipLaunchKernelGGL(potrs_single_batch_kernel, dim3(L.count), dim3(1024),
                     sizeof(double) * 64 * (size_t)ceil_div(nmax, 64), L.stream, L.views, L.items,
                     L.count, which, eq, fused);
  CMPC_LAUNCH_CHECK();
  return 0;
}

int launch_b_potrs_copy(const ListArg& L, int which, int dir, int eq) {
  CMPC_LAUNCH_LIST(potrs_copy_batch_kernel, L, which, dir, eq);
}
static int launch_b_equil_diag(const ListArg& L) { CMPC_LAUNCH_LIST(equil_diag_batch_kernel, L); }
static int launch_b_equil_scale(const ListArg& L) {
  CMPC_LAUNCH_LIST(equil_scale_batch_kernel, L);
}
int launch_b_equilibrate(const ListArg& Ln256, const ListArg& Ln4) {
  if (launch_b_equil_diag(Ln256)) return CMPC_ERR_HIP;
  return launch_b_equil_scale(Ln4);
}
int launch_b_trsv_fwd(const ListArg& L, int k, int which) {
  CMPC_LAUNCH_LIST(trsv_fwd_batch_kernel, L, k, which);
}
int launch_b_trsv_bwd(const ListArg& L, int k, int which) {
  CMPC_LAUNCH_LIST(trsv_bwd_batch_kernel, L, k, which);
}

}  // namespace cmpc
