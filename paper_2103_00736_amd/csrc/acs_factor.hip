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
//          a rank-64 FP64 MFMA product on the lower tiles.
//   mirror S <- -S, both triangles.
//   apply  w += S r64 (FP64 rows, HBM-bound).
#include <cmath>

#include "acs_kernels.h"

namespace acs {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kT = kFacTile;     // 64
constexpr int kSyrkTile = 128;   // output tile of the product B B^T
constexpr int kSyrkK = 16;       // k-depth of one LDS stage
constexpr int kSyrkLd = kSyrkK + 4;  // LDS row stride (doubles)

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

// Lower 128 x 128 tiles of S = B B^T.  Four waves in 2 x 2, each owning a
// 64 x 64 block as 4 x 4 MFMA tiles.  Stages of 16 columns of B go through
// LDS, the next stage's loads in flight during the current one's MFMAs.  The
// contraction index inside a stage is permuted (lane slot q of MFMA step s is
// column 4 q + s) so that each lane reads 4 consecutive doubles per tile.
__global__ __launch_bounds__(kBlock) void k_fac_syrk(FacDev f) {
  __shared__ double As[kSyrkTile * kSyrkLd];
  __shared__ double Bs[kSyrkTile * kSyrkLd];
  int I, J;
  tri_index(blockIdx.x, I, J);
  const int r0 = I * kSyrkTile, c0 = J * kSyrkTile;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, kq = lane >> 4;
  const double* __restrict__ Ag = f.B + size_t(r0) * f.ldb;
  const double* __restrict__ Bg = f.B + size_t(c0) * f.ldb;
  const int sr = tid >> 3, sc = (tid & 7) * 2;  // staging: rows sr + 32 q, columns sc, sc + 1
  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  double2 pa[4], pb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      pa[q] = *reinterpret_cast<const double2*>(Ag + size_t(sr + 32 * q) * f.ldb + k0 + sc);
      pb[q] = *reinterpret_cast<const double2*>(Bg + size_t(sr + 32 * q) * f.ldb + k0 + sc);
    }
  };
  gload(0);
  for (int k0 = 0; k0 < f.ldb; k0 += kSyrkK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<double2*>(As + (sr + 32 * q) * kSyrkLd + sc) = pa[q];
      *reinterpret_cast<double2*>(Bs + (sr + 32 * q) * kSyrkLd + sc) = pb[q];
    }
    __syncthreads();
    if (k0 + kSyrkK < f.ldb) gload(k0 + kSyrkK);
    double av[4][4], bv[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double* pa_ = As + (wr * 64 + t * 16 + li) * kSyrkLd + kq * 4;
      const double* pb_ = Bs + (wc * 64 + t * 16 + li) * kSyrkLd + kq * 4;
      const double2 a0 = *reinterpret_cast<const double2*>(pa_), a1 = *reinterpret_cast<const double2*>(pa_ + 2);
      const double2 b0 = *reinterpret_cast<const double2*>(pb_), b1 = *reinterpret_cast<const double2*>(pb_ + 2);
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
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma64(av[a][s], bv[b][s], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + wr * 64 + a * 16 + kq + 4 * v, col = c0 + wc * 64 + b * 16 + li;
        f.S[size_t(row) * f.mp + col] = acc[a][b][v];
      }
}

// ----------------------------------------------------------------------------
// sweep
// ----------------------------------------------------------------------------
// Pivot block K, P = S_KK (the Schur complement of the rows not yet swept,
// positive semidefinite): Cholesky P = L L^T in LDS (a pivot at or below
// kFacPivotTol is skipped: its column of L is zero), then L^{-1} by forward
// substitution (zero rows and columns for skipped pivots).  Writes L^{-1} to
// f.P and S_KK <- -P^{-1} = -L^{-T} L^{-1}.
__global__ __launch_bounds__(kBlock) void k_fac_pivot(FacDev f, int K) {
  __shared__ double P[kT][kT + 1];  // L in the lower triangle
  __shared__ double X[kT][kT + 1];  // L^{-1}
  __shared__ double rd[kT];         // 1 / L_jj, 0 for a skipped pivot
  const int tid = threadIdx.x;
  double* __restrict__ Skk = f.S + size_t(K) * kT * f.mp + size_t(K) * kT;
  for (int e = tid; e < kT * kT; e += kBlock) P[e / kT][e % kT] = Skk[size_t(e / kT) * f.mp + e % kT];
  __syncthreads();
  for (int j = 0; j < kT; ++j) {  // right-looking, lower triangle
    if (tid == 0) {
      const double d = P[j][j];
      const bool ok = d > kFacPivotTol;
      const double l = ok ? sqrt(d) : 0.0;
      P[j][j] = l;
      rd[j] = ok ? 1.0 / l : 0.0;
    }
    __syncthreads();
    if (tid > j && tid < kT) P[tid][j] *= rd[j];
    __syncthreads();
    for (int e = tid; e < kT * kT; e += kBlock) {
      const int i = e / kT, k = e % kT;
      if (k > j && i >= k) P[i][k] -= P[i][j] * P[k][j];
    }
    __syncthreads();
  }
  if (tid < kT) {  // column j of L^{-1}
    const int j = tid;
    for (int i = 0; i < kT; ++i) {
      double x = 0.0;
      if (i >= j && rd[i] != 0.0 && rd[j] != 0.0) {
        double acc = (i == j) ? 1.0 : 0.0;
        for (int t = j; t < i; ++t) acc -= P[i][t] * X[t][j];
        x = acc * rd[i];
      }
      X[i][j] = x;
    }
  }
  __syncthreads();
  for (int e = tid; e < kT * kT; e += kBlock) {
    const int a = e / kT, b = e % kT;
    double acc = 0.0;
    for (int t = a > b ? a : b; t < kT; ++t) acc += X[t][a] * X[t][b];
    f.P[e] = X[a][b];
    Skk[size_t(a) * f.mp + b] = -acc;
  }
}

// Panel of block K, one workgroup per other row block I: Op = S_IK (read
// from the lower tile S_KI^T when I < K), W = Op L^{-T} (kept for the
// update), C = W L^{-1} = Op P^{-1} written back to S_IK (S_KI^T).
__global__ __launch_bounds__(kBlock) void k_fac_panel(FacDev f, int K) {
  __shared__ double T[kT][kT + 1];
  __shared__ double Li[kT][kT + 1];
  const int I = blockIdx.x < K ? blockIdx.x : blockIdx.x + 1;
  const int tid = threadIdx.x;
  const bool below = I > K;
  for (int e = tid; e < kT * kT; e += kBlock) Li[e / kT][e % kT] = f.P[e];
  if (below) {
    const double* __restrict__ src = f.S + size_t(I) * kT * f.mp + size_t(K) * kT;
    for (int e = tid; e < kT * kT; e += kBlock) T[e / kT][e % kT] = src[size_t(e / kT) * f.mp + e % kT];
  } else {
    const double* __restrict__ src = f.S + size_t(K) * kT * f.mp + size_t(I) * kT;
    for (int e = tid; e < kT * kT; e += kBlock) T[e % kT][e / kT] = src[size_t(e / kT) * f.mp + e % kT];
  }
  __syncthreads();
  const int i0 = (tid >> 4) * 4, c0 = (tid & 15) * 4;  // this thread's 4 x 4 block
  double w[4][4] = {};
  for (int e = 0; e < kT; ++e) {  // W = Op L^{-T}: W_ic = sum_e Op_ie Li_ce
    double a[4], l[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = T[i0 + r][e];
#pragma unroll
    for (int q = 0; q < 4; ++q) l[q] = Li[c0 + q][e];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) w[r][q] += a[r] * l[q];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) T[i0 + r][c0 + q] = w[r][q];
  __syncthreads();
  double* __restrict__ Wg = f.C + size_t(I) * kT * kT;
  for (int e = tid; e < kT * kT; e += kBlock) Wg[e] = T[e / kT][e % kT];
  double c[4][4] = {};
  for (int e = 0; e < kT; ++e) {  // C = W L^{-1}: C_ic = sum_e W_ie Li_ec
    double a[4], l[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = T[i0 + r][e];
#pragma unroll
    for (int q = 0; q < 4; ++q) l[q] = Li[e][c0 + q];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) c[r][q] += a[r] * l[q];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) T[i0 + r][c0 + q] = c[r][q];
  __syncthreads();
  if (below) {
    double* __restrict__ dst = f.S + size_t(I) * kT * f.mp + size_t(K) * kT;
    for (int e = tid; e < kT * kT; e += kBlock) dst[size_t(e / kT) * f.mp + e % kT] = T[e / kT][e % kT];
  } else {
    double* __restrict__ dst = f.S + size_t(K) * kT * f.mp + size_t(I) * kT;
    for (int e = tid; e < kT * kT; e += kBlock) dst[size_t(e / kT) * f.mp + e % kT] = T[e % kT][e / kT];
  }
}

// Trailing update of block K on the lower tile (I, J), I, J != K:
// S_IJ -= W_I W_J^T (= Op_I P^{-1} Op_J^T), rank 64.  Four waves in 2 x 2, each 32 x 32 (2 x 2
// MFMA tiles); lane slot q of MFMA step (h, s) is column 16 q + 8 h + s.
__global__ __launch_bounds__(kBlock) void k_fac_update(FacDev f, int K) {
  int I, J;
  tri_index(blockIdx.x, I, J);
  if (I == K || J == K) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, kq = lane >> 4;
  double* __restrict__ St = f.S + size_t(I) * kT * f.mp + size_t(J) * kT;
  double sv[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        sv[a][b][v] = St[size_t(wr * 32 + a * 16 + kq + 4 * v) * f.mp + wc * 32 + b * 16 + li];
  const double* __restrict__ Cg = f.C + size_t(I) * kT * kT;
  const double* __restrict__ Og = f.C + size_t(J) * kT * kT;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double av[2][8], bv[2][8];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const double* pa = Cg + (wr * 32 + t * 16 + li) * kT + kq * 16 + h * 8;
      const double* pb = Og + (wc * 32 + t * 16 + li) * kT + kq * 16 + h * 8;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 x = *reinterpret_cast<const double2*>(pa + 2 * u);
        const double2 y = *reinterpret_cast<const double2*>(pb + 2 * u);
        av[t][2 * u] = x.x;
        av[t][2 * u + 1] = x.y;
        bv[t][2 * u] = y.x;
        bv[t][2 * u + 1] = y.y;
      }
    }
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a][s], bv[b][s], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        St[size_t(wr * 32 + a * 16 + kq + 4 * v) * f.mp + wc * 32 + b * 16 + li] = sv[a][b][v] - acc[a][b][v];
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

void launch_fac_syrk(const FacDev& f, hipStream_t st) {
  const int t = f.mp / kSyrkTile;
  ACS_LAUNCH(k_fac_syrk, dim3(t * (t + 1) / 2), dim3(kBlock), 0, st, f);
}

void launch_fac_sweep(const FacDev& f, hipStream_t st) {
  const int tiles = f.nb * (f.nb + 1) / 2;
  for (int K = 0; K < f.nb; ++K) {
    ACS_LAUNCH(k_fac_pivot, dim3(1), dim3(kBlock), 0, st, f, K);
    if (f.nb > 1) {
      ACS_LAUNCH(k_fac_panel, dim3(f.nb - 1), dim3(kBlock), 0, st, f, K);
      ACS_LAUNCH(k_fac_update, dim3(tiles), dim3(kBlock), 0, st, f, K);
    }
  }
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
