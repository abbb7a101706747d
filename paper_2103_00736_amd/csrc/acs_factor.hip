// Direct projection for gfx950: the normal matrix M = A_s A_s^T of the
// current scaling, formed and inverted in FP64 at each conditioning event.
//
// The projection of Alg. 2 step 17 needs w with M w = A_s (p - chat) - b_s.
// The CG path solves it approximately every iteration; this path factors M
// once per conditioning epoch (O, hence M, is fixed between events) and
// then applies M^{-1} to the residual r = A_s v - b_s of the warm start,
// w <- w + M^{-1} r, which is exact up to the accuracy of M^{-1}.
//
//   form   B = A_s in FP64 (dense, mp x ldb), M = B B^T by FP64 MFMA
//          (v_mfma_f64_16x16x4), lower 128 x 128 tiles only.
//   sweep  blocked Gauss-Jordan (the symmetric sweep operator) over pivot
//          blocks of 64: for block K with P = S_KK, Op = S_:K,
//              S_KK <- -P^{-1},  S_RK <- Op_R P^{-1},  S_RR <- S_RR - Op_R P^{-1} Op_R^T
//          for all other rows R.  After every block S = -M^{-1}.  M is
//          symmetric positive semidefinite with unit diagonal on live rows,
//          so no pivoting is needed.  P^{-1} is never multiplied in as an
//          explicit inverse: with P = L L^T (Cholesky of the pivot block),
//          W = Op L^{-T}, the update is S_RR -= W W^T and S_RK = W L^{-1}.
//          Multiplying by an explicit P^{-1} instead loses a factor of about
//          cond(P) (||I - M^{-1} M|| of 1e-7 instead of 1e-12 at cond 5e5 in
//          FP64).  A pivot at or below kFacPivotTol is a dependent (e.g.
//          empty) row and is skipped, which leaves zeros in its row and
//          column: the result is then the inverse on the other rows, with
//          the oracle's pseudo-inverse's projection.  The trailing update is
//          an FP64 MFMA product on the lower 64 x 64 tiles; steps are taken
//          in groups of four, so that one pass over S applies the rank-64
//          terms of four steps (each block row of the group is brought up to
//          date before its pivot), and the next group's pivots and panels
//          run on a second stream alongside the pass.
//   mirror S <- -S, both triangles.
//   apply  w += S r64 (FP64 rows, HBM-bound).
#include <algorithm>
#include <cmath>

#include "acs_kernels.h"

namespace acs {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kT = kFacTile;     // 64
constexpr int kSyrkTile = 128;   // output tile of the product B B^T
constexpr int kSyrkK = 32;       // k-depth of one LDS stage
constexpr int kSyrkLd = kSyrkK + 2;  // LDS row stride (doubles)

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// D += A B for one 16 x 16 x 4 FP64 MFMA.  Lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] and holds D[l / 16 + 4 v][l % 16], v = 0..3.
__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// t -> (I, J) with t = I (I + 1) / 2 + J, 0 <= J <= I (lower-triangular tiles)
__device__ __forceinline__ void tri_index(int t, int& I, int& J) {
  int i = int((sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  I = i;
  J = t - i * (i + 1) / 2;
}

// ----------------------------------------------------------------------------
// form
// ----------------------------------------------------------------------------
// B row i = diag(d) A O of a dense problem, in FP64 (hi + lo when stored)
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_fac_dense_b(Dev<VT> d, FacDev f) {
  const int i = blockIdx.x;
  double* __restrict__ row = f.B + size_t(i) * f.ldb;
  if (i >= d.m) {
    for (int j = threadIdx.x; j < f.ldb; j += kBlock) row[j] = 0.0;
    return;
  }
  const double di = d.dinv[i];
  const float* __restrict__ hi = d.dhi + size_t(i) * d.ld;
  const float* __restrict__ lo = d.dlo ? d.dlo + size_t(i) * d.ld : nullptr;
  for (int j = threadIdx.x; j < f.ldb; j += kBlock) {
    double a = 0.0;
    if (j < d.n) {
      a = double(hi[j]);
      if (lo) a += double(lo[j]);
      a = a * d.O[j] * di;
    }
    row[j] = a;
  }
}

__global__ __launch_bounds__(kBlock) void k_fac_zero(double* __restrict__ p, size_t n) {
  for (size_t k = size_t(blockIdx.x) * kBlock + threadIdx.x; k < n; k += size_t(gridDim.x) * kBlock) p[k] = 0.0;
}

// B row i = row i of the FP64 A_s of a sparse problem (B zero beforehand)
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_fac_sparse_b(Dev<VT> d, FacDev f) {
  const int i = blockIdx.x;
  double* __restrict__ row = f.B + size_t(i) * f.ldb;
  for (int k = d.a_rp[i] + threadIdx.x; k < d.a_rp[i + 1]; k += kBlock) row[d.a_col[k]] = d.a_val64[k];
}

// Lower 128 x 128 tiles of S = B B^T (k = ldb columns of B).  Eight waves
// in 2 x 4, each owning a 64 x 32 block as 4 x 2 MFMA tiles; stages of 32
// columns go through LDS, the next stage's loads held in registers during
// the current one's MFMAs.  Register budget: 128 a wave, so that two
// workgroups (4 waves a SIMD, with 68 KB of LDS each) share a CU with the
// prefetch in registers.  That is why each MFMA step reads its six operands
// from LDS just before use instead of holding a half stage of them (that
// layout needs about 150 registers: at 4 waves a SIMD the compiler moves
// the prefetch to scratch memory, at 2 waves a SIMD it runs 15% slower; the
// 4-wave, 64 x 64-block layout runs 55% slower).  The contraction index is
// permuted (lane slot q of MFMA step s is column 16 (s / 4) + 4 q + s % 4);
// both operands use the same order.
constexpr int kSyrkThreads = 512;

__global__ __launch_bounds__(kSyrkThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_fac_syrk(FacDev f) {
  const double* __restrict__ A = f.B;
  const int lda = f.ldb, kdim = f.ldb;
  __shared__ double As[kSyrkTile * kSyrkLd];
  __shared__ double Bs[kSyrkTile * kSyrkLd];
  const int tile = f.syrk_order[blockIdx.x];
  if (tile < 0) return;
  const int I = tile >> 16, J = tile & 0xffff;
  const int r0 = I * kSyrkTile, c0 = J * kSyrkTile;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 2, wc = wave & 3, li = lane & 15, kq = lane >> 4;
  const double* __restrict__ Ag = A + size_t(r0) * lda;
  const double* __restrict__ Bg = A + size_t(c0) * lda;
  const int sr = tid >> 4, sc = (tid & 15) * 2;  // staging: rows sr + 32 q, columns sc, sc + 1
  d4 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  // the next stage's loads, issued unconditionally (the last stage reloads
  // its own columns).  Eight named registers: written as arrays, the
  // compiler keeps them in scratch memory.
  auto ld = [&](const double* g, int row, int k) {
    return *reinterpret_cast<const double2*>(g + size_t(row) * lda + k + sc);
  };
  auto st = [&](double* l, int row, double2 v) { *reinterpret_cast<double2*>(l + row * kSyrkLd + sc) = v; };
  double2 pa0 = ld(Ag, sr, 0), pa1 = ld(Ag, sr + 32, 0), pa2 = ld(Ag, sr + 64, 0), pa3 = ld(Ag, sr + 96, 0);
  double2 pb0 = ld(Bg, sr, 0), pb1 = ld(Bg, sr + 32, 0), pb2 = ld(Bg, sr + 64, 0), pb3 = ld(Bg, sr + 96, 0);
  for (int k0 = 0; k0 < kdim; k0 += kSyrkK) {
    __syncthreads();
    st(As, sr, pa0);
    st(As, sr + 32, pa1);
    st(As, sr + 64, pa2);
    st(As, sr + 96, pa3);
    st(Bs, sr, pb0);
    st(Bs, sr + 32, pb1);
    st(Bs, sr + 64, pb2);
    st(Bs, sr + 96, pb3);
    __syncthreads();
    const int kn = (k0 + kSyrkK < kdim) ? k0 + kSyrkK : k0;
    pa0 = ld(Ag, sr, kn);
    pa1 = ld(Ag, sr + 32, kn);
    pa2 = ld(Ag, sr + 64, kn);
    pa3 = ld(Ag, sr + 96, kn);
    pb0 = ld(Bg, sr, kn);
    pb1 = ld(Bg, sr + 32, kn);
    pb2 = ld(Bg, sr + 64, kn);
    pb3 = ld(Bg, sr + 96, kn);
#pragma unroll
    for (int s = 0; s < kSyrkK / 4; ++s) {
      const int col = 16 * (s >> 2) + 4 * kq + (s & 3);
      double av[4], bv[2];
#pragma unroll
      for (int t = 0; t < 4; ++t) av[t] = As[(wr * 64 + t * 16 + li) * kSyrkLd + col];
#pragma unroll
      for (int t = 0; t < 2; ++t) bv[t] = Bs[(wc * 32 + t * 16 + li) * kSyrkLd + col];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a], bv[b], acc[a][b]);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + wr * 64 + a * 16 + kq + 4 * v, col = c0 + wc * 32 + b * 16 + li;
        f.S[size_t(row) * f.mp + col] = acc[a][b][v];
      }
}

// ----------------------------------------------------------------------------
// sweep
// ----------------------------------------------------------------------------
// Shared by the panel and the update: the W panels, and 64-row FP64 MFMA
// products of blocks staged in LDS (four waves in 2 x 2, each 32 x 32 as
// 2 x 2 MFMA tiles; lane slot q of MFMA step s in quarter h of the staged
// columns is column 16 h + 4 q + s).
constexpr int kWc = 32;         // columns of a W block staged in LDS at a time
constexpr int kWcLd = kWc + 2;  // LDS row stride of a staged chunk (doubles)
enum UpdMode { kUpdStrip = 0, kUpdPass = 1, kUpdPassNext = 2, kUpdPassRest = 3 };

// W = Op L^{-T} of sweep step K for row block I: kFacSlots slots of mp x 64,
// so that all steps of a group are available to its pass while the next
// group's panels write theirs
__device__ __forceinline__ double* w_block(const FacDev& f, int K, int I) {
  return f.C + size_t(K % kFacSlots) * f.mp * kT + size_t(I) * kT * kT;
}

// chunk q of the tile's W columns: term q / 2 (step K0 + q / 2), columns
// 32 (q % 2) .. + 32 of row block B
__device__ __forceinline__ const double* w_chunk(const FacDev& f, int K0, int q, int B) {
  return w_block(f, K0 + q / 2, B) + kWc * (q % 2);
}

// rows r + 16 q, columns c, c + 1 of a chunk, as one vector value (an array
// held across MFMAs is kept in scratch memory by the compiler; a vector
// stays in registers)
typedef double d8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ d8 w_fetch(const double* __restrict__ w, int r, int c) {
  d8 x;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double2 v = *reinterpret_cast<const double2*>(w + (r + 16 * q) * kT + c);
    x[2 * q] = v.x;
    x[2 * q + 1] = v.y;
  }
  return x;
}

__device__ __forceinline__ void w_stage(double* Ws, int r, int c, d8 x) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
    *reinterpret_cast<double2*>(Ws + (r + 16 * q) * kWcLd + c) = double2{x[2 * q], x[2 * q + 1]};
}

// acc += Wi Wj^T over kCols staged columns (LDS row stride kLd), on this
// wave's 32 x 32 block: rows 32 wr .., columns 32 wc ..
template <int kCols = kWc, int kLd = kWcLd>
__device__ __forceinline__ void w_product(const double* Wi, const double* Wj, int wr, int wc, int li, int kq,
                                          d4 (&acc)[2][2]) {
#pragma unroll
  for (int h = 0; h < kCols / 16; ++h) {
    double av[2][4], bv[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const double* pa = Wi + (wr * 32 + t * 16 + li) * kLd + h * 16 + kq * 4;
      const double* pb = Wj + (wc * 32 + t * 16 + li) * kLd + h * 16 + kq * 4;
      const double2 a0 = *reinterpret_cast<const double2*>(pa), a1 = *reinterpret_cast<const double2*>(pa + 2);
      const double2 b0 = *reinterpret_cast<const double2*>(pb), b1 = *reinterpret_cast<const double2*>(pb + 2);
      av[t][0] = a0.x;
      av[t][1] = a0.y;
      av[t][2] = a1.x;
      av[t][3] = a1.y;
      bv[t][0] = b0.x;
      bv[t][1] = b0.y;
      bv[t][2] = b1.x;
      bv[t][3] = b1.y;
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a][s4], bv[b][s4], acc[a][b]);
  }
}

// acc += A B over 64 staged columns, A row-major [row][k], B k-major
// [k][column] (LDS row stride kPLd), on this wave's 32 x 32 block
constexpr int kPLd = kT + 2;  // LDS row stride of the panel's 64 x 64 blocks

__device__ __forceinline__ void kn_product(const double* A, const double* B, int wr, int wc, int li, int kq,
                                           d4 (&acc)[2][2]) {
#pragma unroll
  for (int h = 0; h < kT / 16; ++h) {
    double av[2][4], bv[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const double* pa = A + (wr * 32 + t * 16 + li) * kPLd + h * 16 + kq * 4;
      const double2 a0 = *reinterpret_cast<const double2*>(pa), a1 = *reinterpret_cast<const double2*>(pa + 2);
      av[t][0] = a0.x;
      av[t][1] = a0.y;
      av[t][2] = a1.x;
      av[t][3] = a1.y;
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) bv[t][s4] = B[(h * 16 + kq * 4 + s4) * kPLd + wc * 32 + t * 16 + li];
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a][s4], bv[b][s4], acc[a][b]);
  }
}

// A 64 x 64 block, row stride ld, read by the workgroup: element e = tid +
// 256 u in v[u].  The loads are all issued before any is used (a loop that
// stores each element to LDS as it arrives waits for every load in turn).
constexpr int kPer = kT * kT / kBlock;  // 16

__device__ __forceinline__ void block_load(const double* __restrict__ src, size_t ld, double (&v)[kPer]) {
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = threadIdx.x + kBlock * u;
    v[u] = src[size_t(e / kT) * ld + e % kT];
  }
}

// Pivot block K, P = S_KK (the Schur complement of the rows not yet swept,
// positive semidefinite): right-looking Cholesky P = L L^T in LDS (a pivot at
// or below kFacPivotTol is skipped: its column of L is zero), with the
// forward substitution L X = I carried along in the same sweep (step j
// finishes row j of X = L^{-1}; skipped pivots leave zero rows and columns).
// Writes L^{-1} to f.P, S_KK <- -P^{-1} = -L^{-T} L^{-1}, and zero W blocks
// for block K of every step K0 .. K of its group (see the update).
__global__ __launch_bounds__(kBlock) void k_fac_pivot(FacDev f, int K, int K0) {
  __shared__ double P[kT][kT + 1];  // the trailing Schur complements; column j of L is P_:j / L_jj
  __shared__ double X[kT][kT + 1];  // L^{-1}: forward substitution of L X = I, row by row with L
  const int tid = threadIdx.x;
  double* __restrict__ Skk = f.S + size_t(K) * kT * f.mp + size_t(K) * kT;
  {
    double v[kPer];
    block_load(Skk, f.mp, v);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + kBlock * u, i = e / kT, k = e % kT;
      P[i][k] = v[u];
      X[i][k] = (i == k) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  // One barrier a column: every thread takes 1 / L_jj itself, scales the
  // column-j values of L and row j of X it reads in registers, and row j of
  // X is scaled in place one column later, when no thread reads it any more.
  double rprev = 0.0;
  const int k = tid & 63, w = tid >> 6;
  constexpr int kRows = kT / (kBlock / 64);  // rows i > j a wave takes at most
  for (int j = 0; j < kT; ++j) {
    if (j > 0 && tid < kT) X[j - 1][tid] *= rprev;  // row j - 1 of L^{-1} is final
    // rows i = j + 1 + w + 4 q > j, a wave per row, a lane per column k <= i:
    // X (nonzero for k <= j) and the trailing lower part of P (j < k <= i).
    // The lane's factor (row j of X or column j of P) is the same for every
    // row; the rows' column-j entries and the entries to update are all read
    // (at clamped rows) before any update, so the loads issue together and
    // only the stores are predicated.  The loads do not wait for 1 / L_jj,
    // which is computed without a branch (a skipped pivot multiplies by 0).
    const double d = P[j][j];
    const double pk = k <= j ? X[j][k] : P[k][j];
    double* __restrict__ dst = k <= j ? &X[0][k] : &P[0][k];
    double l[kRows], v[kRows];
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      const int ic = min(j + 1 + w + 4 * q, kT - 1);
      l[q] = P[ic][j];
      v[q] = dst[ic * (kT + 1)];
    }
    const double r = (1.0 / sqrt(fmax(d, kFacPivotTol))) * double(d > kFacPivotTol);  // 0: skipped pivot
    const double src = pk * r;
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      const int i = j + 1 + w + 4 * q;
      if (i < kT && k <= i) dst[i * (kT + 1)] = v[q] - (l[q] * r) * src;
    }
    __syncthreads();
    rprev = r;
  }
  if (tid < kT) X[kT - 1][tid] *= rprev;
  __syncthreads();
  // S_KK = -L^{-T} L^{-1}, 4 x 4 blocks per thread; L^{-1} is lower triangular
  const int a0 = (tid >> 4) * 4, b0 = (tid & 15) * 4;
  double acc[4][4] = {};
  for (int t = 0; t < kT; ++t) {
    double xa[4], xb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      xa[q] = X[t][a0 + q];
      xb[q] = X[t][b0 + q];
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[p][q] += xa[p] * xb[q];
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) Skk[size_t(a0 + p) * f.mp + b0 + q] = -acc[p][q];
  for (int e = tid; e < kT * kT; e += kBlock) f.P[e] = X[e / kT][e % kT];
  // W of this step on block K itself is zero: the paired update then adds
  // nothing from this step to block row and column K
  for (int s = K0; s <= K; ++s) {
    double* __restrict__ Wk = w_block(f, s, K);
    for (int e = tid; e < kT * kT; e += kBlock) Wk[e] = 0.0;
  }
}

// Panel of block K, one workgroup per other row block I: Op = S_IK (read
// from the lower tile S_KI^T when I < K), W = Op L^{-T} (kept for the
// update, in slot K mod kFacSlots), C = W L^{-1} = Op P^{-1} written back to S_IK
// (S_KI^T).
__global__ __launch_bounds__(kBlock) void k_fac_panel(FacDev f, int K) {
  __shared__ double T[kT * kPLd];   // Op, then W, then C
  __shared__ double Li[kT * kPLd];  // L^{-1}
  const int I = blockIdx.x < K ? blockIdx.x : blockIdx.x + 1;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, kq = lane >> 4;
  const bool below = I > K;
  {
    double vl[kPer], vt[kPer];
    block_load(f.P, kT, vl);
    block_load(below ? f.S + size_t(I) * kT * f.mp + size_t(K) * kT : f.S + size_t(K) * kT * f.mp + size_t(I) * kT,
               f.mp, vt);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + kBlock * u, a = e / kT, b = e % kT;
      Li[a * kPLd + b] = vl[u];
      if (below)
        T[a * kPLd + b] = vt[u];
      else
        T[b * kPLd + a] = vt[u];
    }
  }
  __syncthreads();
  // W = Op L^{-T}: W_ic = sum_e Op_ie Li_ce (FP64 MFMA, 4 waves of 32 x 32)
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  w_product<kT, kPLd>(T, Li, wr, wc, li, kq, acc);
  __syncthreads();
  double* __restrict__ Wg = w_block(f, K, I);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 32 + a * 16 + kq + 4 * v, col = wc * 32 + b * 16 + li;
        T[row * kPLd + col] = acc[a][b][v];
        Wg[row * kT + col] = acc[a][b][v];
        acc[a][b][v] = 0.0;
      }
  __syncthreads();
  // C = W L^{-1}: C_ic = sum_e W_ie Li_ec
  kn_product(T, Li, wr, wc, li, kq, acc);
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) T[(wr * 32 + a * 16 + kq + 4 * v) * kPLd + wc * 32 + b * 16 + li] = acc[a][b][v];
  __syncthreads();
  if (below) {
    double* __restrict__ dst = f.S + size_t(I) * kT * f.mp + size_t(K) * kT;
    for (int e = tid; e < kT * kT; e += kBlock) dst[size_t(e / kT) * f.mp + e % kT] = T[(e / kT) * kPLd + e % kT];
  } else {
    double* __restrict__ dst = f.S + size_t(K) * kT * f.mp + size_t(I) * kT;
    for (int e = tid; e < kT * kT; e += kBlock) dst[size_t(e / kT) * f.mp + e % kT] = T[(e % kT) * kPLd + e / kT];
  }
}

// Trailing update on the lower 64 x 64 tiles.  Sweep steps are taken in
// groups K0 .. K0 + cnt - 1 (cnt <= kFacGroup), so that one pass over S
// applies the rank-64 terms W_I W_J^T of all of them:
//   strip (after step K0 + g's panel, g + 1 < cnt): every tile of block row
//          and column B = K0 + g + 1 takes the terms of steps K0 .. K0 + g,
//          so that step B's pivot and panel see up-to-date values;
//   pass  (after the group's last panel): every tile outside block row and
//          column K0 + cnt - 1 takes the terms of all cnt steps.
// Each tile must take each step's term once, and none on the block row and
// column that step writes in final form.  Both follow from zero W blocks:
// W of step s on block K is zero for s = K (its own pivot) and for s < K in
// the group (zeroed by step K's pivot, after the strip that applied them to
// block row K).  So every tile takes every available term, with no case
// analysis.  The order was checked against the one-step sweep in a CPU
// emulation.
// The tile's S values are loaded first (their latency overlaps the staging
// of the W blocks in LDS).  W columns are staged 32 at a time (35 KB of LDS,
// three workgroups a CU at 164 registers), the next chunk fetched into
// registers while the current chunk's MFMAs run.
// S_IJ -= sum over kTerms steps K0, K0 + 1, .. of W_I W_J^T, the W columns
// staged 32 at a time, the next chunk fetched into registers during the
// current chunk's MFMAs
template <int kTerms>
__device__ __forceinline__ void update_tile(const FacDev& f, int I, int J, int K0, double* Wi, double* Wj) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, kq = lane >> 4;
  double* __restrict__ St = f.S + size_t(I) * kT * f.mp + size_t(J) * kT;
  double sv[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) sv[a][b][v] = St[size_t(wr * 32 + a * 16 + kq + 4 * v) * f.mp + wc * 32 + b * 16 + li];
  const int r = tid >> 4, c = (tid & 15) * 2;  // staging: rows r + 16 q, columns c, c + 1
  d8 xi = w_fetch(w_chunk(f, K0, 0, I), r, c), xj = w_fetch(w_chunk(f, K0, 0, J), r, c);
  w_stage(Wi, r, c, xi);
  w_stage(Wj, r, c, xj);
  __syncthreads();
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  constexpr int kChunks = 2 * kTerms;
#pragma unroll
  for (int q = 0; q < kChunks; ++q) {
    if (q + 1 < kChunks) {
      xi = w_fetch(w_chunk(f, K0, q + 1, I), r, c);
      xj = w_fetch(w_chunk(f, K0, q + 1, J), r, c);
    }
    w_product(Wi, Wj, wr, wc, li, kq, acc);
    if (q + 1 < kChunks) {
      __syncthreads();
      w_stage(Wi, r, c, xi);
      w_stage(Wj, r, c, xj);
      __syncthreads();
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        St[size_t(wr * 32 + a * 16 + kq + 4 * v) * f.mp + wc * 32 + b * 16 + li] = sv[a][b][v] - acc[a][b][v];
}

template <int kMode, int kTerms>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_fac_update(FacDev f, int K0,
                                                                                                 int nxt, int cntn) {
  __shared__ double Wi[kT * kWcLd];
  __shared__ double Wj[kT * kWcLd];
  int I, J;
  const int last = K0 + kTerms - 1;
  if (kMode == kUpdStrip) {  // block row and column B = K0 + kTerms, lower tiles (B, t) or (t, B)
    const int t = blockIdx.x, B = K0 + kTerms;
    I = max(t, B);
    J = min(t, B);
  } else if (kMode == kUpdPassNext) {  // block rows and columns b = nxt .. nxt + cntn - 1
    const int b = nxt + int(blockIdx.x) / f.nb, t = int(blockIdx.x) % f.nb;
    if (t >= nxt && t < nxt + cntn && t > b) return;  // a tile of two such blocks once
    I = max(t, b);
    J = min(t, b);
    if (I == last || J == last) return;
  } else {
    const int tile = f.upd_order[blockIdx.x];
    if (tile < 0) return;
    I = tile >> 16;
    J = tile & 0xffff;
    if (I == last || J == last) return;
    if (kMode == kUpdPassRest && ((I >= nxt && I < nxt + cntn) || (J >= nxt && J < nxt + cntn))) return;
  }
  update_tile<kTerms>(f, I, J, K0, Wi, Wj);
}

// S <- -S on both triangles from the lower tiles (diagonal tiles from their
// lower half, so the result is exactly symmetric)
__global__ __launch_bounds__(kBlock) void k_fac_mirror(FacDev f) {
  __shared__ double T[kT][kT + 1];
  int I, J;
  tri_index(blockIdx.x, I, J);
  const int tid = threadIdx.x;
  double* __restrict__ Sij = f.S + size_t(I) * kT * f.mp + size_t(J) * kT;
  for (int e = tid; e < kT * kT; e += kBlock) T[e / kT][e % kT] = Sij[size_t(e / kT) * f.mp + e % kT];
  __syncthreads();
  if (I == J) {
    for (int e = tid; e < kT * kT; e += kBlock) {
      const int i = e / kT, j = e % kT;
      Sij[size_t(i) * f.mp + j] = -(j <= i ? T[i][j] : T[j][i]);
    }
    return;
  }
  double* __restrict__ Sji = f.S + size_t(J) * kT * f.mp + size_t(I) * kT;
  for (int e = tid; e < kT * kT; e += kBlock) Sij[size_t(e / kT) * f.mp + e % kT] = -T[e / kT][e % kT];
  for (int e = tid; e < kT * kT; e += kBlock) Sji[size_t(e / kT) * f.mp + e % kT] = -T[e % kT][e / kT];
}

// ----------------------------------------------------------------------------
// apply: w_i += sum_j S_ij r64_j, four rows per wave
// ----------------------------------------------------------------------------
constexpr int kApplyRows = 4;

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_fac_apply(Dev<VT> d, FacDev f) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i0 = (blockIdx.x * (kBlock / 64) + wave) * kApplyRows;
  if (i0 >= f.m) return;
  const double* rows[kApplyRows];
  double s[kApplyRows];
#pragma unroll
  for (int r = 0; r < kApplyRows; ++r) {
    rows[r] = f.S + size_t(min(i0 + r, f.m - 1)) * f.mp;
    s[r] = 0.0;
  }
  const int ncol = f.nb * kT;
  const double* __restrict__ x = d.r64;
  for (int c = lane * 2; c < ncol; c += 128) {
    const double2 xv = *reinterpret_cast<const double2*>(x + c);
#pragma unroll
    for (int r = 0; r < kApplyRows; ++r) {
      const double2 a = *reinterpret_cast<const double2*>(rows[r] + c);
      s[r] += a.x * xv.x;
      s[r] += a.y * xv.y;
    }
  }
#pragma unroll
  for (int r = 0; r < kApplyRows; ++r) {
    double v = s[r];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    s[r] = v;
  }
  if (lane == 0)
    for (int r = 0; r < kApplyRows; ++r)
      if (i0 + r < f.m) d.w[i0 + r] += s[r];
}

}  // namespace

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
template <typename VT>
void launch_fac_copy(const Dev<VT>& d, const FacDev& f, hipStream_t st) {
  if (d.dense) {
    ACS_LAUNCH((k_fac_dense_b<VT>), dim3(f.mp), dim3(kBlock), 0, st, d, f);
  } else {
    const size_t n = size_t(f.mp) * f.ldb;
    const int nb = int(std::min<size_t>((n + kBlock - 1) / kBlock, 16384));
    ACS_LAUNCH(k_fac_zero, dim3(nb), dim3(kBlock), 0, st, f.B, n);
    ACS_LAUNCH((k_fac_sparse_b<VT>), dim3(d.m), dim3(kBlock), 0, st, d, f);
  }
}

std::vector<int32_t> fac_tile_order(int tiles) {
  constexpr int kXcds = 8;
  const int G = std::max(1, std::min(8, tiles / 8));  // small orders: squares small enough to spread
  std::vector<std::vector<int32_t>> lists(kXcds);
  int sq = 0;
  for (int P = 0; P * G < tiles; ++P)
    for (int Q = 0; Q <= P; ++Q, ++sq) {
      std::vector<int32_t>& L = lists[sq % kXcds];
      for (int I = P * G; I < std::min(tiles, P * G + G); ++I)
        for (int J = Q * G; J < std::min(I + 1, Q * G + G); ++J) L.push_back((I << 16) | J);
    }
  size_t len = 0;
  for (const auto& L : lists) len = std::max(len, L.size());
  std::vector<int32_t> out(len * kXcds, -1);
  for (int x = 0; x < kXcds; ++x)
    for (size_t k = 0; k < lists[x].size(); ++k) out[k * kXcds + x] = lists[x][k];
  return out;
}

void launch_fac_syrk(const FacDev& f, hipStream_t st) {
  ACS_LAUNCH(k_fac_syrk, dim3(f.syrk_blocks), dim3(kSyrkThreads), 0, st, f);
}

void launch_fac_pivot_panel(const FacDev& f, int K, int K0, hipStream_t st) {
  ACS_LAUNCH(k_fac_pivot, dim3(1), dim3(kBlock), 0, st, f, K, K0);
  if (f.nb > 1) ACS_LAUNCH(k_fac_panel, dim3(f.nb - 1), dim3(kBlock), 0, st, f, K);
}

void launch_fac_strip(const FacDev& f, int K0, int terms, hipStream_t st) {
  static_assert(kFacGroup == 4, "one strip instance per term count below the group size");
  const dim3 g(f.nb), b(kBlock);
  switch (terms) {
    case 1: ACS_LAUNCH((k_fac_update<kUpdStrip, 1>), g, b, 0, st, f, K0, 0, 0); break;
    case 2: ACS_LAUNCH((k_fac_update<kUpdStrip, 2>), g, b, 0, st, f, K0, 0, 0); break;
    case 3: ACS_LAUNCH((k_fac_update<kUpdStrip, 3>), g, b, 0, st, f, K0, 0, 0); break;
    default: throw AcsError(ACS_ERR_ARG, "sweep strip: term count out of range");
  }
}

namespace {
template <int kMode>
void launch_pass_mode(const FacDev& f, int K0, int terms, int nxt, int cntn, dim3 g, hipStream_t st) {
  const dim3 b(kBlock);
  switch (terms) {
    case 1: ACS_LAUNCH((k_fac_update<kMode, 1>), g, b, 0, st, f, K0, nxt, cntn); break;
    case 2: ACS_LAUNCH((k_fac_update<kMode, 2>), g, b, 0, st, f, K0, nxt, cntn); break;
    case 3: ACS_LAUNCH((k_fac_update<kMode, 3>), g, b, 0, st, f, K0, nxt, cntn); break;
    case 4: ACS_LAUNCH((k_fac_update<kMode, 4>), g, b, 0, st, f, K0, nxt, cntn); break;
    default: throw AcsError(ACS_ERR_ARG, "sweep pass: term count out of range");
  }
}

void check_next(const FacDev& f, int K0, int terms, int nxt, int cntn) {
  if (cntn < 1 || cntn > kFacGroup || nxt < K0 + terms || nxt + cntn > f.nb)
    throw AcsError(ACS_ERR_ARG, "sweep pass: next group out of range");
}
}  // namespace

void launch_fac_pass(const FacDev& f, int K0, int terms, hipStream_t st) {
  if (f.nb > 1) launch_pass_mode<kUpdPass>(f, K0, terms, f.nb, 0, dim3(f.upd_blocks), st);
}

void launch_fac_pass_next(const FacDev& f, int K0, int terms, int nxt, int cntn, hipStream_t st) {
  check_next(f, K0, terms, nxt, cntn);
  launch_pass_mode<kUpdPassNext>(f, K0, terms, nxt, cntn, dim3(cntn * f.nb), st);
}

void launch_fac_pass_rest(const FacDev& f, int K0, int terms, int nxt, int cntn, hipStream_t st) {
  check_next(f, K0, terms, nxt, cntn);
  launch_pass_mode<kUpdPassRest>(f, K0, terms, nxt, cntn, dim3(f.upd_blocks), st);
}

void launch_fac_mirror(const FacDev& f, hipStream_t st) {
  const int all = f.mp / kT;
  ACS_LAUNCH(k_fac_mirror, dim3(all * (all + 1) / 2), dim3(kBlock), 0, st, f);
}

template <typename VT>
void launch_fac_apply(const Dev<VT>& d, const FacDev& f, hipStream_t st) {
  const int nb = ceil_div(f.m, kApplyRows * (kBlock / 64));
  ACS_LAUNCH((k_fac_apply<VT>), dim3(nb), dim3(kBlock), 0, st, d, f);
}

template void launch_fac_copy<float>(const Dev<float>&, const FacDev&, hipStream_t);
template void launch_fac_copy<double>(const Dev<double>&, const FacDev&, hipStream_t);
template void launch_fac_apply<float>(const Dev<float>&, const FacDev&, hipStream_t);
template void launch_fac_apply<double>(const Dev<double>&, const FacDev&, hipStream_t);

}  // namespace acs
