// HIP kernels for gfx950: one generic LDS-staged CSR row-block engine and the
// steps of Algorithm 2 built on it (see acs_kernels.h for the scaled form).
//
// Every kernel that sweeps a matrix processes one RowBlock per workgroup:
// products val[k] * x[col[k]] of the block's rows are staged in LDS with
// coalesced loads, then each row is summed by a group of G lanes (G adapts
// to the rows per block: 1 lane for very short rows, up to a wave64 per
// row) with a wavefront-shuffle reduction; a row longer than the stage gets
// a whole workgroup.  Row sums feed a per-kernel epilogue (the fused vector
// update of that step).  Grid-wide FP64 reductions are deterministic: each
// workgroup writes a partial, the last workgroup to arrive sums them in
// fixed order.  Workgroup ids are remapped so that each of the 8 XCDs gets a
// contiguous range of row blocks.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "acs_kernels.h"

namespace acs {

LaunchEvents*& launch_events() {
  static thread_local LaunchEvents* slot = nullptr;
  return slot;
}

// ----------------------------------------------------------------------------
// helpers
// ----------------------------------------------------------------------------

// Hardware places workgroup b on XCD b % 8; hand XCD x a contiguous range.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7;
  const int x = b & 7, i = b >> 3;
  return x * q + (x < rem ? x : rem) + i;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}

// Progress records in pinned host memory.  host_store releases at system
// scope: every earlier write of the kernel is visible to the host first, which
// costs a write-back of the L2 before the next kernel starts; it is used only
// where the host then reads other results (the KKT check).  host_post is a
// relaxed system-scope store for the CG progress records, which the host uses
// only to decide what to launch next.
template <typename T>
__device__ __forceinline__ void host_store(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <typename T>
__device__ __forceinline__ void host_post(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Per-block partial sums (N values) -> partials[blk * N + i].
template <int N, bool MIN = false>
__device__ __forceinline__ void block_store_partials(double (&acc)[N], double* partials, int blk) {
  __shared__ double sh[kBlock / 64][N];
#pragma unroll
  for (int i = 0; i < N; ++i) acc[i] = MIN ? wave_min(acc[i]) : wave_sum(acc[i]);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) sh[w][i] = acc[i];
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double s = sh[0][threadIdx.x];
    for (int k = 1; k < kBlock / 64; ++k) s = MIN ? fmin(s, sh[k][threadIdx.x]) : s + sh[k][threadIdx.x];
    partials[size_t(blk) * N + threadIdx.x] = s;
  }
}

// Sum (or min) of the partials of nb workgroups in fixed order, by one
// workgroup of a later kernel (the kernel boundary makes them visible);
// result on every thread.
template <int N, bool MIN = false>
__device__ __forceinline__ void sum_partials(const double* __restrict__ partials, int nb, double (&out)[N]) {
  __shared__ double sh[kBlock / 64][N];
  double acc[N];
#pragma unroll
  for (int i = 0; i < N; ++i) acc[i] = MIN ? INFINITY : 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double v = partials[size_t(b) * N + i];
      acc[i] = MIN ? fmin(acc[i], v) : acc[i] + v;
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) acc[i] = MIN ? wave_min(acc[i]) : wave_sum(acc[i]);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) sh[w][i] = acc[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double v = sh[0][i];
    for (int k = 1; k < kBlock / 64; ++k) v = MIN ? fmin(v, sh[k][i]) : v + sh[k][i];
    out[i] = v;
  }
}

// Sum over each row of prod(k) for the rows of one RowBlock; epi(row, sum)
// runs on one lane per row.  All threads of the workgroup must call it.
template <typename Acc, class Prod, class Epi>
__device__ __forceinline__ void rows_block(const int32_t* __restrict__ rp, RowBlock rb, Prod& prod, Epi& epi) {
  __shared__ Acc lds[kStageNnz];
  __shared__ Acc red[kBlock / 64];
  const int tid = threadIdx.x;
  const int r0 = rb.r0, r1 = rb.r1;
  const int k0 = rp[r0], k1 = rp[r1];
  if (k1 - k0 > kStageNnz) {  // a single long row: the whole workgroup
    Acc s = 0;
    for (int k = k0 + tid; k < k1; k += kBlock) s += prod(k);
    s = wave_sum(s);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
      Acc tot = red[0];
      for (int i = 1; i < kBlock / 64; ++i) tot += red[i];
      epi(r0, tot);
    }
    return;
  }
#pragma unroll
  for (int it = 0; it < kStageNnz / kBlock; ++it) {
    const int k = k0 + it * kBlock + tid;
    if (k < k1) lds[k - k0] = prod(k);
  }
  __syncthreads();
  const int nrows = r1 - r0;
  int G = 64;
  while (G > 1 && G * nrows > kBlock) G >>= 1;
  const int grp = tid / G, lane = tid & (G - 1), ngrp = kBlock / G;
  for (int r = r0 + grp; r < r1; r += ngrp) {
    const int a = rp[r] - k0, e = rp[r + 1] - k0;
    Acc s = 0;
    for (int k = a + lane; k < e; k += G) s += lds[k];
    for (int off = G >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) epi(r, s);
  }
}

// f(row, k) for every nonzero k of the block's rows.
template <class F>
__device__ __forceinline__ void rows_foreach(const int32_t* __restrict__ rp, RowBlock rb, F& f) {
  const int tid = threadIdx.x;
  const int r0 = rb.r0, r1 = rb.r1;
  const int k0 = rp[r0], k1 = rp[r1];
  if (r1 - r0 == 1) {
    for (int k = k0 + tid; k < k1; k += kBlock) f(r0, k);
    return;
  }
  const int nrows = r1 - r0;
  int G = 64;
  while (G > 1 && G * nrows > kBlock) G >>= 1;
  const int grp = tid / G, lane = tid & (G - 1), ngrp = kBlock / G;
  for (int r = r0 + grp; r < r1; r += ngrp) {
    const int e = rp[r + 1];
    for (int k = rp[r] + lane; k < e; k += G) f(r, k);
  }
}

// Dot products over strided SELL entries, s += v[e*stride] * vec[c[e*stride]]
// in order of e.  The loads of a group of entries are issued together
// (indices and values, then the gathers) so a lane keeps several requests in
// flight, and no load sits behind a branch (the compiler would wait for every
// outstanding load at the join).  Each entry is loaded once.

// exactly N entries
template <int N, typename VT, typename XT>
__device__ __forceinline__ void dot_exact(const int32_t* __restrict__ c, const VT* __restrict__ v, int stride,
                                          const XT* __restrict__ vec, VT& s) {
  int32_t cc[N];
  VT vv[N], g[N];
#pragma unroll
  for (int u = 0; u < N; ++u) {
    cc[u] = c[u * stride];
    vv[u] = v[u * stride];
  }
#pragma unroll
  for (int u = 0; u < N; ++u) g[u] = VT(vec[cc[u]]);
#pragma unroll
  for (int u = 0; u < N; ++u) s += vv[u] * g[u];
}

// count entries, count uniform across the wave: groups of 8, then the rest
template <typename VT, typename XT>
__device__ __forceinline__ VT dot_uniform(const int32_t* __restrict__ c, const VT* __restrict__ v, int count,
                                          int stride, const XT* __restrict__ vec) {
  VT s = 0;
  int e = 0;
  for (; e + 8 <= count; e += 8) dot_exact<8>(c + e * stride, v + e * stride, stride, vec, s);
  c += e * stride;
  v += e * stride;
  switch (count - e) {
    case 1: dot_exact<1>(c, v, stride, vec, s); break;
    case 2: dot_exact<2>(c, v, stride, vec, s); break;
    case 3: dot_exact<3>(c, v, stride, vec, s); break;
    case 4: dot_exact<4>(c, v, stride, vec, s); break;
    case 5: dot_exact<5>(c, v, stride, vec, s); break;
    case 6: dot_exact<6>(c, v, stride, vec, s); break;
    case 7: dot_exact<7>(c, v, stride, vec, s); break;
    default: break;
  }
  return s;
}

// a row of len >= 1 entries at c[0..len), v[0..len) shared by `lanes` lanes:
// lane l takes entries l, l + lanes, ...  Groups of up to 8 per lane, the
// count of groups uniform across the lanes; a lane past the row's end reads
// the row's last entry again and drops the product.
template <typename VT, typename XT>
__device__ __forceinline__ VT dot_row(const int32_t* __restrict__ c, const VT* __restrict__ v, int len, int lane,
                                      int lanes, const XT* __restrict__ vec) {
  const int per = (len + lanes - 1) / lanes;  // entries of the busiest lane
  VT s = 0;
  for (int e0 = 0; e0 < per; e0 += 8) {
    int32_t cc[8];
    VT vv[8], g[8];
    bool ok[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = lane + (e0 + u) * lanes;
      ok[u] = e0 + u < per && e < len;
      const int ec = ok[u] ? e : len - 1;
      cc[u] = c[ec];
      vv[u] = v[ec];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) g[u] = VT(vec[cc[u]]);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const VT prod = vv[u] * g[u];
      s += ok[u] ? prod : VT(0);
    }
  }
  return s;
}

// Rows of one slice x of a SELL layout for the workgroup's task lb (see Sell
// in acs_internal.h).  pre(row) runs on the lane owning a row before its
// product (to start loads the epilogue needs); epi(row, sum, pre_value) runs
// after it.  A long task uses the whole workgroup and a barrier, so lb must
// be uniform across the workgroup; waves without a task return at once.
// Entries are summed in storage order, so results are reproducible.
template <typename VT, typename XT, class Pre, class Epi>
__device__ __forceinline__ void sell_rows(const SellDev& S, const VT* __restrict__ val, int x, int lb,
                                          const XT* __restrict__ vec, Pre& pre, Epi& epi) {
  const int tid = threadIdx.x;
  const int nl = S.long_off[x + 1] - S.long_off[x];
  const int32_t* __restrict__ col = S.col;
  if (lb < nl) {
    __shared__ VT red[kBlock / 64];
    const int li = S.long_off[x] + lb;
    const int beg = S.long_beg[li], end = S.long_end[li];
    const int row = S.long_row[li];
    const VT pv = tid == 0 ? pre(row) : VT(0);
    VT s = dot_row(col + beg, val + beg, end - beg, tid, kBlock, vec);
    s = wave_sum(s);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
      VT tot = red[0];
      for (int i = 1; i < kBlock / 64; ++i) tot += red[i];
      epi(row, tot, pv);
    }
    return;
  }
  const int t = S.wt_off[x] + (lb - nl) * 4 + (tid >> 6);
  if (t >= S.wt_off[x + 1]) return;
  const int lane = tid & 63;
  const int ptr = S.wt_ptr[t], len = S.wt_len[t], row = S.wt_row[t];
  const int r = S.chunk_row[size_t(t) * kSellChunk + lane];  // independent of the loads above
  if (row >= 0) {  // one row per wave, lanes stride the row
    const VT pv = lane == 0 ? pre(row) : VT(0);
    VT s = dot_row(col + ptr, val + ptr, len, lane, 64, vec);
    s = wave_sum(s);
    if (lane == 0) epi(row, s, pv);
    return;
  }
  // chunk: one row per lane, entries column-major
  const VT pv = r >= 0 ? pre(r) : VT(0);
  const VT s = dot_uniform(col + ptr + lane, val + ptr + lane, len, kSellChunk, vec);
  if (r >= 0) epi(r, s, pv);
}

__device__ __forceinline__ double lorentz_dist2(double u0, double nb) {
  if (nb <= u0) return 0.0;
  if (nb <= -u0) return u0 * u0 + nb * nb;
  const double g = nb - u0;
  return 0.5 * g * g;
}

// ----------------------------------------------------------------------------
// step 18 (+19-20 on checks, +16 of the next iteration): rows j of A_s^T
// ----------------------------------------------------------------------------
// Per column j of A_s^T, given u = (A_s^T w)_j: steps 16-20 fused (see the
// header), and the check reductions.  Shared by the sparse and dense sweeps.
template <typename VT, int MODE, bool CHECK>
struct UpdateEpi {
  const Dev<VT>& d;
  const VT* __restrict__ s_cur;
  VT* __restrict__ s_new;
  double (&acc)[kUpdSums];
  __device__ __forceinline__ void operator()(int j, double u) const {
    const double mu = d.mu;
    const double zt = d.chat[j] + u;  // mu * (O z) implied by w
    const double s = double(s_cur[j]);
    const bool orth = j < d.n_orth;
    double sn = s;
    if (MODE != UPD_PROLOGUE) {
      const double pj = orth ? fabs(s) : double(d.p[j]);
      const VT snv = VT(0.5 * (s + pj) - zt);
      s_new[j] = snv;
      sn = double(snv);
      acc[0] += (sn - s) * (sn - s);
      if (CHECK) {
        const double Oj = d.O[j];
        const double xh = 0.5 * (pj + sn);
        const double x = Oj * xh;
        const double z = 0.5 * (pj - sn) / (mu * Oj);
        d.xout[j] = x;
        d.zout[j] = z;
        d.xhat[j] = xh;
        acc[1] += d.c[j] * x;
        acc[2] += x * x;
        acc[3] += z * z;
        if (orth) {
          const double mx = fmin(x, 0.0), mz = fmin(z, 0.0);
          acc[4] += mx * mx;
          acc[5] += mz * mz;
          acc[8] += fabs(x * z);  // |x_j z_j| of the objective-error estimate (cones: k_cone)
        }
        const double dr = (pj - sn - 2.0 * zt) / (2.0 * mu * Oj);  // (A^T y + z - c)_j
        acc[6] += dr * dr;
        acc[7] += x * dr;  // r_d^T x
      }
    }
    if (MODE != UPD_UPDATE_ONLY) {
      if (orth)
        d.v[j] = VT(fabs(sn) - zt);
      else
        d.zt[j] = zt;
    }
  }
};

template <typename VT, int MODE, bool CHECK>
__global__ __launch_bounds__(kBlock) void k_update(Dev<VT> d, const VT* __restrict__ s_cur, VT* __restrict__ s_new) {
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  double acc[kUpdSums] = {};
  UpdateEpi<VT, MODE, CHECK> upd{d, s_cur, s_new, acc};
  auto pre = [](int) -> double { return 0.0; };
  auto epi = [&](int j, double u, double) { upd(j, u); };
  sell_rows<double, double>(d.st, d.st_val64, 0, blk, d.w, pre, epi);
  // the sums are read only by the KKT check (k_fin_upd runs on check iterations)
  if (MODE != UPD_PROLOGUE && CHECK) block_store_partials<kUpdSums>(acc, d.partials, blk);
}

// ----------------------------------------------------------------------------
// step 16 on the Lorentz cones: one group of G lanes per cone
// ----------------------------------------------------------------------------
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_cone(Dev<VT> d, const VT* __restrict__ s, int check, int next, int G) {
  const int gpb = kBlock / G;
  const int grp = threadIdx.x / G, lane = threadIdx.x & (G - 1);
  const int cone = blockIdx.x * gpb + grp;
  double acc[3] = {0, 0, 0};
  if (cone < d.n_soc) {
    const int off = d.soc_off[cone], end = d.soc_off[cone + 1];
    if (check) {
      double nx = 0, nz = 0, xz = 0;
      for (int e = off + 1 + lane; e < end; e += G) {
        const double xe = d.xout[e], ze = d.zout[e];
        nx += xe * xe;
        nz += ze * ze;
        xz += xe * ze;
      }
      for (int o = G >> 1; o > 0; o >>= 1) {
        nx += __shfl_xor(nx, o);
        nz += __shfl_xor(nz, o);
        xz += __shfl_xor(xz, o);
      }
      if (lane == 0) {
        const double x0 = d.xout[off], z0 = d.zout[off];
        acc[0] = lorentz_dist2(x0, sqrt(nx));
        acc[1] = lorentz_dist2(z0, sqrt(nz));
        acc[2] = x0 * z0 + xz;  // x_C^T z_C: the estimate sums the cones with their signs
      }
    }
    if (next) {
      double n2 = 0;
      for (int e = off + 1 + lane; e < end; e += G) {
        const double se = double(s[e]);
        n2 += se * se;
      }
      for (int o = G >> 1; o > 0; o >>= 1) n2 += __shfl_xor(n2, o);
      const double s0 = double(s[off]);
      const double nv = sqrt(n2);
      double a0, f;  // proj = (a0, f * s_bar)
      if (nv <= s0) {
        a0 = s0;
        f = 1.0;
      } else if (nv <= -s0) {
        a0 = 0.0;
        f = 0.0;
      } else {
        const double a = 0.5 * (s0 + nv);
        a0 = a;
        f = a / nv;
      }
      for (int e = off + lane; e < end; e += G) {
        const double se = double(s[e]);
        const double pr = (e == off) ? a0 : f * se;
        const VT pv = VT(2.0 * pr - se);
        d.p[e] = pv;
        d.v[e] = VT(double(pv) - d.zt[e]);
      }
    }
  }
  if (check) block_store_partials<3>(acc, d.partials, blockIdx.x);
}

// ----------------------------------------------------------------------------
// CG start: r = A_s v - b_s (rows i of A_s), FP64 accumulation
// ----------------------------------------------------------------------------
// row i given (A_s v)_i: r in VT (and in FP64 for the direct projection), ||r||^2
template <typename VT>
__device__ __forceinline__ void resid_row(const Dev<VT>& d, int i, double sum, double& rr) {
  const double r64 = sum - d.bs[i];
  const VT ri = VT(r64);
  d.r[i] = ri;
  if (d.r64) d.r64[i] = r64;
  rr += double(ri) * double(ri);
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_resid_part(Dev<VT> d) {
  const int x = blockIdx.x % d.sa.slices, lb = blockIdx.x / d.sa.slices;
  if (lb >= d.sa.wg[x]) return;
  double* __restrict__ part = d.part64 + size_t(x) * d.m;
  auto pre = [](int) -> double { return 0.0; };
  auto epi = [&](int i, double sum, double) { part[i] = sum; };
  sell_rows<double, VT>(d.sa, d.sa_val64, x, lb, d.v, pre, epi);
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_resid_comb(Dev<VT> d) {
  double acc[1] = {0};
  const int m = d.m;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) {
    double sum = d.part64[i];
    for (int x = 1; x < d.sa.slices; ++x) sum += d.part64[size_t(x) * m + i];
    resid_row(d, i, sum, acc[0]);
  }
  block_store_partials<1>(acc, d.partials, blockIdx.x);
}

// One column slice: r = A_s v - b_s from whole rows, no partials to combine
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_resid_one(Dev<VT> d) {
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  double acc[1] = {0};
  auto pre = [](int) -> double { return 0.0; };
  auto epi = [&](int i, double sum, double) { resid_row(d, i, sum, acc[0]); };
  sell_rows<double, VT>(d.sa, d.sa_val64, 0, blk, d.v, pre, epi);
  block_store_partials<1>(acc, d.partials, blk);
}

// ----------------------------------------------------------------------------
// CG, first half: t = A_s^T q with q = r + beta q_old, kept as the recurrence
// t = A_s^T r + beta t_old (one gathered operand); alpha = rho / ||t||^2
// ----------------------------------------------------------------------------
// j >= 1 with the one-slice layout: every workgroup first finalizes step j-1
// from the second half's ||r||^2 partials, in the same order (as k_fin_cg_a
// does in one workgroup), so all agree on beta and on the stop test;
// workgroup 0 records the result.  It reads rho of step j-1 from the slot of
// that step and writes step j's into the other slot, so no workgroup of this
// kernel reads what another writes.  j < 0: k_fin_cg_a ran.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_cg_t(Dev<VT> d, int j, int rr_nb) {
  __shared__ int done_sh;
  if (threadIdx.x == 0) done_sh = d.ctl->done;
  __syncthreads();
  if (done_sh) return;
  double beta = d.ctl->beta;
  if (j >= 1) {
    double t[1];
    sum_partials<1>(d.partials, rr_nb, t);
    Ctl* c = d.ctl;
    const double rn = t[0];
    const bool bad = !(rn == rn) || isinf(rn);
    beta = bad ? 0.0 : rn / c->rho_step[(j - 1) & 1];
    const bool done = bad || rn <= c->tol2 || j >= c->cg_max;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      c->rho_step[j & 1] = rn;
      c->rho = rn;
      c->beta = beta;
      c->k = j;
      c->cg_total += 1;
      if (done) {
        c->done = 1;
        if (bad) host_post(&d.hs->numeric, 1);
        host_post(&d.hs->cg_done_iter, c->iter);
      }
    }
    if (done) return;
  }
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const VT vbeta = VT(beta);
  double acc[1] = {0};
  auto pre = [&](int j) -> VT { return beta != 0.0 ? d.t[j] : VT(0); };
  auto epi = [&](int j, VT sum, VT t_old) {
    const VT tj = (beta != 0.0) ? sum + vbeta * t_old : sum;
    d.t[j] = tj;
    acc[0] += double(tj) * double(tj);
  };
  sell_rows<VT, VT>(d.st_cg, d.st_cg_val, 0, blk, d.r, pre, epi);
  // one slice: the fused second half reads them while it writes d.partials
  block_store_partials<1>(acc, d.sa.slices == 1 ? d.partials2 : d.partials, blk);
}

// ----------------------------------------------------------------------------
// CG, second half, by column slices: workgroup b works on slice b % kSlices,
// i.e. on the XCD it is dispatched to, so its gathers of t touch 1/kSlices of
// t and stay in that XCD's L2; it writes partial row sums part[x][i].
// Workgroup 0 first turns the first half's partials into alpha = rho/||t||^2.
// ----------------------------------------------------------------------------
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_cg_a_part(Dev<VT> d, int t_nb) {
  __shared__ int done_sh;  // workgroup 0 may set done below: one read per workgroup
  if (threadIdx.x == 0) done_sh = d.ctl->done;
  __syncthreads();
  if (done_sh) return;
  if (blockIdx.x == 0) {
    double tt[1];
    sum_partials<1>(d.partials, t_nb, tt);
    if (threadIdx.x == 0) {
      Ctl* c = d.ctl;
      if (tt[0] > 0.0 && !isinf(tt[0])) {
        c->alpha = c->rho / tt[0];
      } else {
        c->alpha = 0.0;
        c->done = 1;
        if (!(tt[0] == tt[0])) host_post(&d.hs->numeric, 1);
        host_post(&d.hs->cg_done_iter, c->iter);
      }
    }
  }
  const int x = blockIdx.x % d.sa.slices, lb = blockIdx.x / d.sa.slices;
  if (lb >= d.sa.wg[x]) return;
  VT* __restrict__ part = d.part + size_t(x) * d.m;
  auto pre = [](int) -> VT { return VT(0); };
  auto epi = [&](int i, VT sum, VT) { part[i] = sum; };
  sell_rows<VT, VT>(d.sa_cg, d.sa_val, x, lb, d.t, pre, epi);
}

// CG update of row i given (M q)_i: q = r + beta q; w += alpha q; r -= alpha M q
template <typename VT>
__device__ __forceinline__ void cg_row_update(const Dev<VT>& d, int i, VT mq, double alpha, double beta, VT valpha,
                                              VT vbeta, double& rr) {
  const VT ri = d.r[i];
  const VT qi = (beta != 0.0) ? ri + vbeta * d.q[i] : ri;
  d.q[i] = qi;
  d.w[i] += alpha * double(qi);
  const VT rn = ri - valpha * mq;
  d.r[i] = rn;
  rr += double(rn) * double(rn);
}

// Mq_i = sum over slices (fixed order); q = r + beta q; w += alpha q; r -= alpha Mq
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_cg_a_comb(Dev<VT> d) {
  if (d.ctl->done) return;
  const double alpha = d.ctl->alpha, beta = d.ctl->beta;
  const VT valpha = VT(alpha), vbeta = VT(beta);
  double acc[1] = {0};
  const int m = d.m;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) {
    VT mq = d.part[i];
    for (int x = 1; x < d.sa.slices; ++x) mq += d.part[size_t(x) * m + i];
    cg_row_update(d, i, mq, alpha, beta, valpha, vbeta, acc[0]);
  }
  block_store_partials<1>(acc, d.partials, blockIdx.x);
}

// CG, second half with one column slice: whole rows of A_s t and the CG
// update of each row in one kernel.  Every workgroup turns the first half's
// partials into alpha in the same order (so all agree); workgroup 0 records it.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_cg_a_one(Dev<VT> d, int t_nb, long long launch_id) {
  __shared__ int bad_sh, done_sh;
  if (blockIdx.x == 0 && threadIdx.x == 0) host_post(&d.hs->launch_seq, launch_id);  // host's progress
  if (threadIdx.x == 0) done_sh = d.ctl->done;
  __syncthreads();
  if (done_sh) return;
  double tt[1];
  sum_partials<1>(d.partials2, t_nb, tt);
  if (threadIdx.x == 0) bad_sh = !(tt[0] > 0.0) || isinf(tt[0]);
  __syncthreads();
  if (bad_sh) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      Ctl* c = d.ctl;
      c->alpha = 0.0;
      c->done = 1;
      if (!(tt[0] == tt[0])) host_post(&d.hs->numeric, 1);
      host_post(&d.hs->cg_done_iter, c->iter);
    }
    return;
  }
  const double alpha = d.ctl->rho / tt[0], beta = d.ctl->beta;
  if (blockIdx.x == 0 && threadIdx.x == 0) d.ctl->alpha = alpha;
  const VT valpha = VT(alpha), vbeta = VT(beta);
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  double acc[1] = {0};
  auto pre = [](int) -> VT { return VT(0); };
  auto epi = [&](int i, VT mq, VT) { cg_row_update(d, i, mq, alpha, beta, valpha, vbeta, acc[0]); };
  sell_rows<VT, VT>(d.sa_cg, d.sa_val, 0, blk, d.t, pre, epi);
  block_store_partials<1>(acc, d.partials, blk);
}

// values of a SELL layout from the FP64 A_s (padding entries hold 0), in VT
// for the CG and in FP64 for the refinement sweeps (one array when VT = double;
// val64 == nullptr: VT values only)
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_sell_vals(const int32_t* __restrict__ src, int64_t count,
                                                      const double* __restrict__ a64, VT* __restrict__ val,
                                                      double* __restrict__ val64) {
  for (int64_t e = blockIdx.x * int64_t(kBlock) + threadIdx.x; e < count; e += int64_t(gridDim.x) * kBlock) {
    const int32_t k = src[e];
    const double a = k >= 0 ? a64[k] : 0.0;
    if constexpr (sizeof(VT) == sizeof(double)) {
      val64[e] = a;
    } else {
      val[e] = VT(a);
      if (val64) val64[e] = a;
    }
  }
}

// ----------------------------------------------------------------------------
// KKT check (rows i of A_s): ||A x - b||^2 = sum (d_i^-1 ((A_s xhat)_i - b_s,i))^2,
// y = -d w / mu, b^T y; the last workgroup assembles the relative errors
// ----------------------------------------------------------------------------
// check, row i given (A_s xhat)_i: ||A x - b||^2 term, y_i, b^T y term and
// y^T (A x - b) of the objective-error estimate
template <typename VT>
__device__ __forceinline__ void pres_row(const Dev<VT>& d, int i, double ax, double mu, double (&acc)[3]) {
  const double res = (ax - d.bs[i]) * d.dsq[i];
  acc[0] += res * res;
  const double yi = -d.dinv[i] * d.w[i] / mu;
  d.yout[i] = yi;
  acc[1] += d.b[i] * yi;
  acc[2] += yi * res;  // y^T r_p of the objective-error estimate
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_pres(Dev<VT> d) {
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const RowBlock rb = d.a_blk[blk];
  const double* __restrict__ av = d.a_val64;
  const int32_t* __restrict__ ac = d.a_col;
  const double* __restrict__ xh = d.xhat;
  auto prod = [&](int k) -> double { return av[k] * xh[ac[k]]; };
  double acc[3] = {0, 0, 0};
  const double mu = d.mu;
  auto epi = [&](int i, double ax) { pres_row(d, i, ax, mu, acc); };
  rows_block<double>(d.a_rp, rb, prod, epi);
  block_store_partials<3>(acc, d.partials, blk);
}

// ----------------------------------------------------------------------------
// conditioning, steps 5-11: ratio per cone unit, then O = o^alpha
// ----------------------------------------------------------------------------
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_cond_ratio(Dev<VT> d, const VT* __restrict__ s_prev,
                                                       const VT* __restrict__ s_cur) {
  const int units = d.n_orth + d.n_soc;
  const int u = blockIdx.x * kBlock + threadIdx.x;
  double acc[3] = {INFINITY, INFINITY, INFINITY};  // min log o, min -log o, min -valid
  const double mu = d.mu;
  if (u < units) {
    double num, den;
    if (u < d.n_orth) {
      const double sp = double(s_prev[u]), sc = double(s_cur[u]);
      const double pj = fabs(sp), Oj = d.O[u];
      const double x = Oj * 0.5 * (pj + sc);
      const double z = 0.5 * (pj - sc) / (mu * Oj);
      d.xc[u] = x;
      d.zc[u] = z;
      num = fabs(x);
      den = fabs(z);
    } else {
      const int cone = u - d.n_orth;
      const int off = d.soc_off[cone], end = d.soc_off[cone + 1];
      const double Ob = d.O[off];
      // p = abs_K(s_prev) on this cone, recomputed in FP64 (closed-form projection)
      double n2 = 0;
      for (int e = off + 1; e < end; ++e) {
        const double se = double(s_prev[e]);
        n2 += se * se;
      }
      const double s0 = double(s_prev[off]), nv = sqrt(n2);
      double a0, f;
      if (nv <= s0) {
        a0 = s0;
        f = 1.0;
      } else if (nv <= -s0) {
        a0 = 0.0;
        f = 0.0;
      } else {
        a0 = 0.5 * (s0 + nv);
        f = a0 / nv;
      }
      double nb = 0, x0 = 0, z0 = 0;
      for (int e = off; e < end; ++e) {
        const double spe = double(s_prev[e]);
        const double pe = 2.0 * ((e == off) ? a0 : f * spe) - spe;
        const double se = double(s_cur[e]);
        const double x = Ob * 0.5 * (pe + se);
        const double z = 0.5 * (pe - se) / (mu * Ob);
        d.xc[e] = x;
        d.zc[e] = z;
        if (e == off) {
          x0 = x;
          z0 = z;
        } else {
          nb += x * x;
        }
      }
      num = fabs(x0 - sqrt(nb));
      den = fabs(z0);
    }
    double o;
    if (num == 0.0 && den == 0.0)
      o = 1.0;
    else if (den == 0.0)
      o = INFINITY;
    else
      o = num / den;
    if (d.eq && o > 0.0 && !isinf(o) && !(num == 0.0 && den == 0.0)) {
      // equilibrated: the ratio of x_hat = x / E, z_hat = E z
      const double e = d.eq[u < d.n_orth ? u : d.soc_off[u - d.n_orth]];
      o = o / (e * e);
    }
    d.ounit[u] = o;
    if (o > 0.0 && !isinf(o) && o == o) {
      const double lo = log(o);
      acc[0] = lo;
      acc[1] = -lo;
      acc[2] = -1.0;
    }
  }
  block_store_partials<3, true>(acc, d.partials, blockIdx.x);
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_cond_scale(Dev<VT> d, VT* __restrict__ s_cur) {
  const int units = d.n_orth + d.n_soc;
  const int u = blockIdx.x * kBlock + threadIdx.x;
  if (u >= units) return;
  const Ctl* c = d.ctl;
  const bool any = c->cond[2] < 0.0;
  double Onew = 1.0;
  if (any) {
    double o = d.ounit[u];
    if (!(o == o)) o = 1.0;
    if (o == 0.0) o = exp(c->cond[0]);
    if (isinf(o)) o = exp(-c->cond[1]);
    Onew = pow(o, c->cond[3]);
  }
  int off, end;
  if (u < d.n_orth) {
    off = u;
    end = u + 1;
  } else {
    off = d.soc_off[u - d.n_orth];
    end = d.soc_off[u - d.n_orth + 1];
  }
  if (d.eq) Onew *= d.eq[off];  // equilibrated: the column scaling E O_hat
  const double mu = d.mu;
  for (int e = off; e < end; ++e) {
    d.O[e] = Onew;
    d.chat[e] = mu * Onew * d.c[e];
    s_cur[e] = VT(d.xc[e] / Onew - mu * Onew * d.zc[e]);  // step 14
  }
}

// ----------------------------------------------------------------------------
// step 12: rebuild A_s = diag(d) A O; d_i = (sum_j a_ij^2 O_j^2)^(-1/2)
// wmode: 0 keep w, 1 rescale w by d_old/d_new, 2 w holds unscaled w -> multiply by 1/d
// ----------------------------------------------------------------------------
// step 12, row i given D = sum_j a_ij^2 O_j^2: d_i, 1/d_i, b_s; w rescaled (wmode)
template <typename VT>
__device__ __forceinline__ void rowsum_row(const Dev<VT>& d, int i, double D, int wmode) {
  if (!(D > 0.0)) D = 1.0;  // empty row: unit diagonal
  const double ds = sqrt(D);
  if (wmode == 1) d.w[i] *= ds / d.dsq[i];
  if (wmode == 2) d.w[i] *= ds;
  d.dsq[i] = ds;
  d.dinv[i] = 1.0 / ds;
  d.bs[i] = d.b[i] / ds;
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_rowsum(Dev<VT> d, int wmode) {
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const RowBlock rb = d.a_blk[blk];
  const double* __restrict__ ao = d.a_orig;
  const int32_t* __restrict__ ac = d.a_col;
  const double* __restrict__ O = d.O;
  auto prod = [&](int k) -> double {
    const double g = ao[k] * O[ac[k]];
    return g * g;
  };
  auto epi = [&](int i, double D) { rowsum_row(d, i, D, wmode); };
  rows_block<double>(d.a_rp, rb, prod, epi);
}

// Row index of every staged nonzero of a row block (LDS), so that the
// per-nonzero rewrite below reads and writes with coalesced accesses.
__device__ __forceinline__ void stage_rows(const int32_t* __restrict__ rp, RowBlock rb, int k0, int32_t* rowof) {
  const int tid = threadIdx.x;
  const int nrows = rb.r1 - rb.r0;
  int G = 64;
  while (G > 1 && G * nrows > kBlock) G >>= 1;
  const int grp = tid / G, lane = tid & (G - 1), ngrp = kBlock / G;
  for (int r = rb.r0 + grp; r < rb.r1; r += ngrp) {
    const int e = rp[r + 1] - k0;
    for (int k = rp[r] - k0 + lane; k < e; k += G) rowof[k] = r;
  }
  __syncthreads();
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_scale_a(Dev<VT> d) {
  __shared__ int32_t rowof[kStageNnz];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const RowBlock rb = d.a_blk[blk];
  const int k0 = d.a_rp[rb.r0], k1 = d.a_rp[rb.r1];
  const bool one = (k1 - k0 > kStageNnz);
  if (!one) stage_rows(d.a_rp, rb, k0, rowof);
  for (int k = k0 + threadIdx.x; k < k1; k += kBlock) {
    const int i = one ? rb.r0 : rowof[k - k0];
    const double a = d.a_orig[k] * d.O[d.a_col[k]] * d.dinv[i];
    d.a_val64[k] = a;
  }
}

// ----------------------------------------------------------------------------
// Sinkhorn-Knopp l2 equilibration (Sec. III, A_hat = D A E), FP64: with
// u = D^2 and v = E^2 (eq holds v during the sweeps), each sweep sets
// u_i = 1 / sum_j a_ij^2 v_j and then, per Lorentz cone of k coordinates (an
// orthant coordinate is a cone of one), v = (m/n) k / sum over its columns of
// sum_i a_ij^2 u_i.  Rows and cones without a nonzero keep u = 1 / v = 1.
// ----------------------------------------------------------------------------
// squared values in the order of the A^T layout (into its FP64 value array,
// which the first rescale overwrites with A_s)
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_sk_sq(const int32_t* __restrict__ src, int64_t count,
                                                  const double* __restrict__ a, double* __restrict__ sq) {
  for (int64_t e = blockIdx.x * int64_t(kBlock) + threadIdx.x; e < count; e += int64_t(gridDim.x) * kBlock) {
    const int32_t k = src[e];
    const double v = k >= 0 ? a[k] : 0.0;
    sq[e] = v * v;
  }
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_sk_rows(Dev<VT> d) {
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const RowBlock rb = d.a_blk[blk];
  const double* __restrict__ ao = d.a_orig;
  const int32_t* __restrict__ ac = d.a_col;
  const double* __restrict__ v = d.eq;
  auto prod = [&](int k) -> double {
    const double a = ao[k];
    return a * a * v[ac[k]];
  };
  auto epi = [&](int i, double sum) { d.eq_u[i] = sum > 0.0 ? 1.0 / sum : 1.0; };
  rows_block<double>(d.a_rp, rb, prod, epi);
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_sk_cols(Dev<VT> d) {
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  auto pre = [](int) -> double { return 0.0; };
  auto epi = [&](int j, double sum, double) { d.eq_c[j] = sum; };
  sell_rows<double, double>(d.st, d.st_val64, 0, blk, d.eq_u, pre, epi);
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_sk_unit(Dev<VT> d, double target, int last) {
  const int units = d.n_orth + d.n_soc;
  const int u = blockIdx.x * kBlock + threadIdx.x;
  if (u >= units) return;
  int off, end;
  if (u < d.n_orth) {
    off = u;
    end = u + 1;
  } else {
    off = d.soc_off[u - d.n_orth];
    end = d.soc_off[u - d.n_orth + 1];
  }
  double tot = 0.0;
  for (int e = off; e < end; ++e) tot += d.eq_c[e];
  double v = tot > 0.0 ? target * double(end - off) / tot : 1.0;
  if (last) v = sqrt(v);
  for (int e = off; e < end; ++e) d.eq[e] = v;
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_chat(Dev<VT> d) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j < d.n) d.chat[j] = d.mu * d.O[j] * d.c[j];
}

// ----------------------------------------------------------------------------
// plain products with the current scaled matrix (tests, bandwidth timing)
// ----------------------------------------------------------------------------
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_spmv_t(Dev<VT> d, const VT* __restrict__ x, VT* __restrict__ y) {
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  auto pre = [](int) -> VT { return VT(0); };
  auto epi = [&](int j, VT s, VT) { y[j] = s; };
  sell_rows<VT, VT>(d.st, d.st_val, 0, blk, x, pre, epi);
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_spmv_a(Dev<VT> d, const VT* __restrict__ x) {
  const int xs = blockIdx.x % d.sa.slices, lb = blockIdx.x / d.sa.slices;
  if (lb >= d.sa.wg[xs]) return;
  VT* __restrict__ part = d.part + size_t(xs) * d.m;
  auto pre = [](int) -> VT { return VT(0); };
  auto epi = [&](int i, VT s, VT) { part[i] = s; };
  sell_rows<VT, VT>(d.sa, d.sa_val, xs, lb, x, pre, epi);
}

// y[row_perm[i]] = sum of the slice partials of row i (same order as the CG)
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_spmv_comb(Dev<VT> d, VT* __restrict__ y) {
  const int m = d.m;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) {
    VT s = d.part[i];
    for (int x = 1; x < d.sa.slices; ++x) s += d.part[size_t(x) * m + i];
    y[d.row_perm[i]] = s;
  }
}

// internal order of a caller's m-vector: mtmp[i] = x[row_perm[i]]
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_perm_in(Dev<VT> d, const VT* __restrict__ x) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < d.m) d.mtmp[i] = x[d.row_perm[i]];
}

// outputs into caller-owned device buffers: x, z as they are, y in the
// caller's row order (y[row_perm[i]] = yout[i])
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_out_device(Dev<VT> d, double* __restrict__ x, double* __restrict__ y,
                                                      double* __restrict__ z) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < d.n) {
    if (x) x[i] = d.xout[i];
    if (z) z[i] = d.zout[i];
  }
  if (y && i < d.m) y[d.row_perm[i]] = d.yout[i];
}

template <typename VT>
__global__ void k_ctl_reset(Dev<VT> d, int cg_max) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    Ctl* c = d.ctl;
    c->rho = c->rho0 = c->tol2 = c->alpha = c->beta = 0.0;
    c->rho_step[0] = c->rho_step[1] = 0.0;
    c->k = 0;
    c->done = 1;
    c->cg_max = cg_max;
    c->iter = 0;
    c->cg_total = 0;
    for (int i = 0; i < kUpdSums; ++i) c->upd[i] = 0.0;
    for (int i = 0; i < 4; ++i) c->cone[i] = 0.0;
    for (int i = 0; i < 4; ++i) c->cond[i] = 0.0;
    for (int i = 0; i < 9; ++i) c->kkt[i] = 0.0;
  }
}

// ----------------------------------------------------------------------------
// finalizers: one workgroup sums the per-workgroup partials of the kernel
// just before it and applies the scalar logic
// ----------------------------------------------------------------------------
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_fin_upd(Dev<VT> d, int nb) {
  double t[kUpdSums];
  sum_partials<kUpdSums>(d.partials, nb, t);
  if (threadIdx.x == 0)
    for (int i = 0; i < kUpdSums; ++i) d.ctl->upd[i] = t[i];
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_fin_cone(Dev<VT> d, int nb) {
  double t[3];
  sum_partials<3>(d.partials, nb, t);
  if (threadIdx.x == 0) {
    d.ctl->cone[0] = t[0];
    d.ctl->cone[1] = t[1];
    d.ctl->cone[2] = t[2];
  }
}

// CG start: rho_0, the stop threshold, zero-step exit
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_fin_resid(Dev<VT> d, int nb, int iter, double red2, double abs2,
                                                      int cg_max) {
  double t[1];
  sum_partials<1>(d.partials, nb, t);
  if (threadIdx.x == 0) {
    Ctl* c = d.ctl;
    const double rho = t[0];
    c->cg_max = cg_max;
    c->rho = rho;
    c->rho0 = rho;
    c->rho_step[0] = rho;
    c->tol2 = fmax(red2 * rho, abs2);
    c->alpha = 0.0;
    c->beta = 0.0;
    c->k = 0;
    c->iter = iter;
    const bool bad = !(rho == rho) || isinf(rho);
    const int done = (bad || rho <= c->tol2 || c->cg_max <= 0) ? 1 : 0;
    c->done = done;
    if (bad) host_post(&d.hs->numeric, 1);
    if (done) host_post(&d.hs->cg_done_iter, iter);
  }
}

// beta = ||r_new||^2 / rho, stop test, progress record for the host
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_fin_cg_a(Dev<VT> d, int nb, long long launch_id) {
  if (!d.ctl->done) {
    double t[1];
    sum_partials<1>(d.partials, nb, t);
    if (threadIdx.x == 0) {
      Ctl* c = d.ctl;
      const double rn = t[0];
      const bool bad = !(rn == rn) || isinf(rn);
      c->beta = bad ? 0.0 : rn / c->rho;
      c->rho = rn;
      c->k += 1;
      c->cg_total += 1;
      const int done = (bad || rn <= c->tol2 || c->k >= c->cg_max) ? 1 : 0;
      c->done = done;
      if (bad) host_post(&d.hs->numeric, 1);
      if (done) host_post(&d.hs->cg_done_iter, c->iter);
    }
  }
  if (threadIdx.x == 0) host_post(&d.hs->launch_seq, launch_id);
}

// KKT relative errors of the check iteration
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_fin_pres(Dev<VT> d, int nb, int iter, double bnorm, double cnorm,
                                                     int has_soc) {
  double t[3];
  sum_partials<3>(d.partials, nb, t);
  if (threadIdx.x == 0) {
    Ctl* c = d.ctl;
    const double* u = c->upd;
    const double ctx = u[1], bty = t[1];
    const double dx2 = u[4] + (has_soc ? c->cone[0] : 0.0);
    const double dz2 = u[5] + (has_soc ? c->cone[1] : 0.0);
    double e[9];
    e[0] = sqrt(t[0]) / (1.0 + bnorm);
    e[1] = sqrt(u[6]) / (1.0 + cnorm);
    e[2] = fabs(ctx - bty) / (1.0 + fabs(ctx) + fabs(bty));
    e[3] = fmax(sqrt(dx2), sqrt(dz2)) / (1.0 + fmax(sqrt(u[2]), sqrt(u[3])));
    e[4] = fmax(fmax(e[0], e[1]), fmax(e[2], e[3]));
    e[5] = ctx;
    e[6] = bty;
    e[7] = u[0];
    // estimate of |c^T x - p*| / (1 + |c^T x|): c^T x - p* = z*^T x + y*^T r_p,
    // at the current y, z: |x_j z_j| per orthant coordinate, the Lorentz
    // cones' x_C^T z_C summed with their signs, |y^T r_p|
    e[8] = (u[8] + (has_soc ? fabs(c->cone[2]) : 0.0) + fabs(t[2])) / (1.0 + fabs(ctx));
    bool bad = false;
    for (int i = 0; i < 9; ++i) {
      c->kkt[i] = e[i];
      d.hs->kkt[i] = e[i];
      if (!(e[i] == e[i]) || isinf(e[i])) bad = true;
    }
    d.hs->cg_total = c->cg_total;
    if (bad) host_store(&d.hs->numeric, 1);
    __threadfence_system();
    host_store(&d.hs->check_iter, iter);
  }
}

// step 11: alpha from the log range of the valid ratios
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_fin_cond(Dev<VT> d, int nb, double t_cap) {
  double t[3];
  sum_partials<3, true>(d.partials, nb, t);
  if (threadIdx.x == 0) {
    Ctl* c = d.ctl;
    c->cond[0] = t[0];
    c->cond[1] = t[1];
    c->cond[2] = t[2];
    const double span = -t[1] - t[0];
    c->cond[3] = (t[2] < 0.0 && span > 0.0) ? fmin(1.0, t_cap / span) : 1.0;
  }
}

// ----------------------------------------------------------------------------
// Dense A, row-major with leading dimension ld (Sec. V instances).  Products
// apply the scalings to vectors: (A_s x)_i = d_i sum_j a_ij (O_j x_j) and
// (A_s^T y)_j = O_j sum_i a_ij (d_i y_i), with d_i = 1/sqrt(D_i).  They stream
// A once each with 16-byte loads: rows of A by a wave per 4 rows (the x chunk
// loaded once for the 4 rows); columns by strips of 1024 columns (4 per lane)
// over chunks of rows into partial sums, added in fixed order by a second
// kernel.  FP64 sweeps add the FP32 low part of each value when present.
// ----------------------------------------------------------------------------
enum DenseKind { DK_CG = 0, DK_RESID = 1, DK_PRES = 2, DK_ROWSUM = 3, DK_SPMV = 4, DK_UPDATE = 5 };
constexpr int kDenseRows = 4;                      // rows per wave of the row products
constexpr int kDenseStrip = kBlock * 4;            // columns per workgroup of the column products

template <typename ACC, typename XT>
__device__ __forceinline__ void load_x4(const XT* __restrict__ x, int c, ACC (&xv)[4]) {
  if constexpr (sizeof(XT) == 4) {
    const float4 v = *reinterpret_cast<const float4*>(x + c);
    xv[0] = ACC(v.x);
    xv[1] = ACC(v.y);
    xv[2] = ACC(v.z);
    xv[3] = ACC(v.w);
  } else {
    const double2 v0 = *reinterpret_cast<const double2*>(x + c);
    const double2 v1 = *reinterpret_cast<const double2*>(x + c + 2);
    xv[0] = ACC(v0.x);
    xv[1] = ACC(v0.y);
    xv[2] = ACC(v1.x);
    xv[3] = ACC(v1.y);
  }
}

template <typename ACC, bool SQ>
__device__ __forceinline__ void fma4(ACC& s, const float4 a, const float4* lo, const ACC (&xv)[4]) {
  ACC a0 = ACC(a.x), a1 = ACC(a.y), a2 = ACC(a.z), a3 = ACC(a.w);
  if (lo) {
    a0 += ACC(lo->x);
    a1 += ACC(lo->y);
    a2 += ACC(lo->z);
    a3 += ACC(lo->w);
  }
  if (SQ) {
    a0 *= a0;
    a1 *= a1;
    a2 *= a2;
    a3 *= a3;
  }
  s += a0 * xv[0];
  s += a1 * xv[1];
  s += a2 * xv[2];
  s += a3 * xv[3];
}

// sum_j a_ij x_j (a_ij^2 x_j if SQ) for the wave's rows i0..i0+3 (clamped to
// m), in ACC; result on every lane.  x has ld entries (padding zero).
template <typename VT, typename ACC, typename XT, bool SQ>
__device__ __forceinline__ void dense_rows4(const Dev<VT>& d, int i0, const XT* __restrict__ x, bool use_lo,
                                            ACC (&s)[kDenseRows]) {
  const int lane = threadIdx.x & 63;
  const float* rows[kDenseRows];
  const float* rlo[kDenseRows];
#pragma unroll
  for (int r = 0; r < kDenseRows; ++r) {
    const size_t i = size_t(min(i0 + r, d.m - 1));
    rows[r] = d.dhi + i * d.ld;
    rlo[r] = use_lo ? d.dlo + i * d.ld : nullptr;
    s[r] = 0;
  }
  for (int c = lane * 4; c < d.ld; c += 256) {
    ACC xv[4];
    float4 a[kDenseRows];
#pragma unroll
    for (int r = 0; r < kDenseRows; ++r) a[r] = *reinterpret_cast<const float4*>(rows[r] + c);
    load_x4<ACC, XT>(x, c, xv);
    if (use_lo) {
      float4 l[kDenseRows];
#pragma unroll
      for (int r = 0; r < kDenseRows; ++r) l[r] = *reinterpret_cast<const float4*>(rlo[r] + c);
#pragma unroll
      for (int r = 0; r < kDenseRows; ++r) fma4<ACC, SQ>(s[r], a[r], &l[r], xv);
    } else {
#pragma unroll
      for (int r = 0; r < kDenseRows; ++r) fma4<ACC, SQ>(s[r], a[r], nullptr, xv);
    }
  }
#pragma unroll
  for (int r = 0; r < kDenseRows; ++r) s[r] = wave_sum(s[r]);
}

// Row products.  CG: (A_s t)_i from dx32 = O t, then the CG update of row i
// (alpha from the ||t||^2 partials, computed by every workgroup in the same
// order).  RESID: r = A_s v - b_s from dx64 = O v.  PRES: the check from
// dx64 = O xhat.  ROWSUM: D_i from dx64 = O^2 (wmode as k_rowsum).  SPMV:
// y = A_s x from dx32 = O x.
template <typename VT, int KIND>
__global__ __launch_bounds__(kBlock) void k_dense_rows(Dev<VT> d, int aux, VT* __restrict__ y) {
  __shared__ int bad_sh, done_sh;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i0 = (blockIdx.x * (kBlock / 64) + wave) * kDenseRows;
  double acc[3] = {0, 0, 0};
  double alpha = 0, beta = 0;
  if (KIND == DK_CG) {
    if (threadIdx.x == 0) done_sh = d.ctl->done;  // workgroup 0 may set done below
    __syncthreads();
    if (done_sh) return;
    double tt[1];
    sum_partials<1>(d.partials2, aux, tt);
    if (threadIdx.x == 0) bad_sh = !(tt[0] > 0.0) || isinf(tt[0]);
    __syncthreads();
    if (bad_sh) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        Ctl* c = d.ctl;
        c->alpha = 0.0;
        c->done = 1;
        if (!(tt[0] == tt[0])) host_post(&d.hs->numeric, 1);
        host_post(&d.hs->cg_done_iter, c->iter);
      }
      return;
    }
    alpha = d.ctl->rho / tt[0];
    beta = d.ctl->beta;
    if (blockIdx.x == 0 && threadIdx.x == 0) d.ctl->alpha = alpha;
  }
  if (KIND == DK_CG || KIND == DK_SPMV) {
    VT s[kDenseRows];  // FP64 mode keeps the exact values (the low part)
    dense_rows4<VT, VT, VT, false>(d, i0, d.dx32, sizeof(VT) == sizeof(double) && d.dlo != nullptr, s);
    if (lane == 0) {
      for (int r = 0; r < kDenseRows; ++r) {
        const int i = i0 + r;
        if (i >= d.m) break;
        const VT mq = VT(d.dinv[i]) * s[r];
        if (KIND == DK_CG)
          cg_row_update(d, i, mq, alpha, beta, VT(alpha), VT(beta), acc[0]);
        else
          y[i] = mq;
      }
    }
  } else {
    double s[kDenseRows];
    if (KIND == DK_ROWSUM)
      dense_rows4<VT, double, double, true>(d, i0, d.dx64, d.dlo != nullptr, s);
    else
      dense_rows4<VT, double, double, false>(d, i0, d.dx64, d.dlo != nullptr, s);
    if (lane == 0) {
      for (int r = 0; r < kDenseRows; ++r) {
        const int i = i0 + r;
        if (i >= d.m) break;
        if (KIND == DK_RESID) {
          const double r64 = d.dinv[i] * s[r] - d.bs[i];
          const VT ri = VT(r64);
          d.r[i] = ri;
          if (d.r64) d.r64[i] = r64;
          acc[0] += double(ri) * double(ri);
        } else if (KIND == DK_PRES) {
          pres_row(d, i, d.dinv[i] * s[r], d.mu, acc);
        } else {
          rowsum_row(d, i, s[r], aux);
        }
      }
    }
  }
  if (KIND == DK_CG || KIND == DK_RESID) {
    double a1[1] = {acc[0]};
    block_store_partials<1>(a1, d.partials, blockIdx.x);
  } else if (KIND == DK_PRES) {
    block_store_partials<3>(acc, d.partials, blockIdx.x);
  }
}

// Column products, partial sums over one chunk of rows: part[chunk][j] =
// sum_i a_ij y_i with y_i = d_i r_i (CG, VT), d_i w_i (UPDATE, FP64) or d_i
// x_i (SPMV, VT; x in the caller's order, which is the internal one here).
template <typename VT, int KIND>
__global__ __launch_bounds__(kBlock) void k_dense_cols(Dev<VT> d, const VT* __restrict__ xin) {
  using ACC = typename std::conditional<KIND == DK_UPDATE, double, VT>::type;
  if (KIND == DK_CG && d.ctl->done) return;
  const int c = (blockIdx.x * kBlock + threadIdx.x) * 4;
  if (c >= d.ld) return;
  const int r0 = blockIdx.y * d.dchunk, r1 = min(d.m, r0 + d.dchunk);
  const bool use_lo = sizeof(ACC) == sizeof(double) && d.dlo != nullptr;  // FP64 sums keep the exact values
  ACC s[4] = {0, 0, 0, 0};
  for (int i = r0; i < r1; ++i) {
    ACC yi;
    if (KIND == DK_CG)
      yi = ACC(d.dinv[i]) * ACC(d.r[i]);
    else if (KIND == DK_UPDATE)
      yi = d.dinv[i] * d.w[i];
    else
      yi = ACC(d.dinv[i]) * ACC(xin[i]);
    const float4 a = *reinterpret_cast<const float4*>(d.dhi + size_t(i) * d.ld + c);
    ACC a0 = ACC(a.x), a1 = ACC(a.y), a2 = ACC(a.z), a3 = ACC(a.w);
    if (use_lo) {
      const float4 l = *reinterpret_cast<const float4*>(d.dlo + size_t(i) * d.ld + c);
      a0 += ACC(l.x);
      a1 += ACC(l.y);
      a2 += ACC(l.z);
      a3 += ACC(l.w);
    }
    s[0] += a0 * yi;
    s[1] += a1 * yi;
    s[2] += a2 * yi;
    s[3] += a3 * yi;
  }
  ACC* part = reinterpret_cast<ACC*>(d.dpart) + size_t(blockIdx.y) * d.ld + c;
  if constexpr (sizeof(ACC) == 4) {
    *reinterpret_cast<float4*>(part) = make_float4(s[0], s[1], s[2], s[3]);
  } else {
    *reinterpret_cast<double2*>(part) = make_double2(s[0], s[1]);
    *reinterpret_cast<double2*>(part + 2) = make_double2(s[2], s[3]);
  }
}

// Column products, the chunk partials added in fixed order and the step of
// the column: CG t = O_j sum + beta t_old, dx32 = O t, ||t||^2 partials;
// UPDATE the fused update (UpdateEpi); SPMV y_j = O_j sum.
template <typename VT, int KIND, int MODE, bool CHECK>
__global__ __launch_bounds__(kBlock) void k_dense_cols_fin(Dev<VT> d, const VT* __restrict__ s_cur,
                                                           VT* __restrict__ s_new) {
  using ACC = typename std::conditional<KIND == DK_UPDATE, double, VT>::type;
  if (KIND == DK_CG && d.ctl->done) return;
  const int j = blockIdx.x * kBlock + threadIdx.x;
  const ACC* part = reinterpret_cast<const ACC*>(d.dpart);
  double acc[kUpdSums] = {};
  if (j < d.n) {
    ACC sum = part[j];
    for (int ch = 1; ch < d.dnchunk; ++ch) sum += part[size_t(ch) * d.ld + j];
    if (KIND == DK_CG) {
      const double beta = d.ctl->beta;
      const VT t = VT(d.O[j]) * sum;
      const VT tj = (beta != 0.0) ? t + VT(beta) * d.t[j] : t;
      d.t[j] = tj;
      d.dx32[j] = VT(d.O[j]) * tj;
      acc[0] = double(tj) * double(tj);
    } else if (KIND == DK_UPDATE) {
      UpdateEpi<VT, MODE, CHECK> upd{d, s_cur, s_new, acc};
      upd(j, d.O[j] * double(sum));
    } else {
      s_new[j] = VT(d.O[j]) * sum;
    }
  }
  if (KIND == DK_CG) {
    double a1[1] = {acc[0]};
    block_store_partials<1>(a1, d.partials2, blockIdx.x);
  } else if (KIND == DK_UPDATE && MODE != UPD_PROLOGUE && CHECK) {
    block_store_partials<kUpdSums>(acc, d.partials, blockIdx.x);
  }
}

// inputs of the row products: dx64 = O v (0), O xhat (1), O^2 (2); dx32 = O x (3)
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_dense_prep(Dev<VT> d, int what, const VT* __restrict__ x) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= d.n) return;
  const double o = d.O[j];
  if (what == 0)
    d.dx64[j] = o * double(d.v[j]);
  else if (what == 1)
    d.dx64[j] = o * d.xhat[j];
  else if (what == 2)
    d.dx64[j] = o * o;
  else
    d.dx32[j] = VT(o) * x[j];
}

static inline int dense_row_blocks(int m) { return (m + kDenseRows * (kBlock / 64) - 1) / (kDenseRows * (kBlock / 64)); }

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
static inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

template <typename VT>
static void launch_dense_update(const Dev<VT>& d, const VT* s_cur, VT* s_new, int mode, bool check, hipStream_t st) {
  const dim3 gc(ceil_div(d.ld, kDenseStrip), d.dnchunk), b(kBlock);
  ACS_LAUNCH((k_dense_cols<VT, DK_UPDATE>), gc, b, 0, st, d, static_cast<const VT*>(nullptr));
  const dim3 gf(ceil_div(d.n, kBlock));
  if (mode == UPD_PROLOGUE) {
    ACS_LAUNCH((k_dense_cols_fin<VT, DK_UPDATE, UPD_PROLOGUE, false>), gf, b, 0, st, d, s_cur, s_new);
    return;
  }
  if (mode == UPD_UPDATE) {
    if (check)
      ACS_LAUNCH((k_dense_cols_fin<VT, DK_UPDATE, UPD_UPDATE, true>), gf, b, 0, st, d, s_cur, s_new);
    else
      ACS_LAUNCH((k_dense_cols_fin<VT, DK_UPDATE, UPD_UPDATE, false>), gf, b, 0, st, d, s_cur, s_new);
  } else {
    if (check)
      ACS_LAUNCH((k_dense_cols_fin<VT, DK_UPDATE, UPD_UPDATE_ONLY, true>), gf, b, 0, st, d, s_cur, s_new);
    else
      ACS_LAUNCH((k_dense_cols_fin<VT, DK_UPDATE, UPD_UPDATE_ONLY, false>), gf, b, 0, st, d, s_cur, s_new);
  }
  if (check) ACS_LAUNCH((k_fin_upd<VT>), dim3(1), b, 0, st, d, int(gf.x));
}

template <typename VT>
void launch_update(const Dev<VT>& d, const VT* s_cur, VT* s_new, int mode, bool check, hipStream_t st) {
  if (d.dense) {
    launch_dense_update(d, s_cur, s_new, mode, check, st);
    return;
  }
  const dim3 g(d.st.wg[0]), b(kBlock);
  if (mode == UPD_PROLOGUE) {
    ACS_LAUNCH((k_update<VT, UPD_PROLOGUE, false>), g, b, 0, st, d, s_cur, s_new);
    return;
  }
  if (mode == UPD_UPDATE) {
    if (check)
      ACS_LAUNCH((k_update<VT, UPD_UPDATE, true>), g, b, 0, st, d, s_cur, s_new);
    else
      ACS_LAUNCH((k_update<VT, UPD_UPDATE, false>), g, b, 0, st, d, s_cur, s_new);
  } else {
    if (check)
      ACS_LAUNCH((k_update<VT, UPD_UPDATE_ONLY, true>), g, b, 0, st, d, s_cur, s_new);
    else
      ACS_LAUNCH((k_update<VT, UPD_UPDATE_ONLY, false>), g, b, 0, st, d, s_cur, s_new);
  }
  if (check) ACS_LAUNCH((k_fin_upd<VT>), dim3(1), b, 0, st, d, d.st.wg[0]);  // sums only the check reads
}

template <typename VT>
void launch_cone(const Dev<VT>& d, const VT* s, bool check, bool next, int group, hipStream_t st) {
  if (d.n_soc == 0) return;
  const int gpb = kBlock / group;
  const int nb = ceil_div(d.n_soc, gpb);
  ACS_LAUNCH((k_cone<VT>), dim3(nb), dim3(kBlock), 0, st, d, s, int(check), int(next), group);
  if (check) ACS_LAUNCH((k_fin_cone<VT>), dim3(1), dim3(kBlock), 0, st, d, nb);
}

static inline int comb_blocks(int m) { return std::min(ceil_div(m, kBlock), 2048); }

template <typename VT>
void launch_resid(const Dev<VT>& d, hipStream_t st) {
  if (d.dense) {
    ACS_LAUNCH((k_dense_prep<VT>), dim3(ceil_div(d.n, kBlock)), dim3(kBlock), 0, st, d, 0,
               static_cast<const VT*>(nullptr));
    ACS_LAUNCH((k_dense_rows<VT, DK_RESID>), dim3(dense_row_blocks(d.m)), dim3(kBlock), 0, st, d, 0,
               static_cast<VT*>(nullptr));
    return;
  }
  if (d.sa.slices == 1) {
    ACS_LAUNCH((k_resid_one<VT>), dim3(d.sa.wg[0]), dim3(kBlock), 0, st, d);
    return;
  }
  ACS_LAUNCH((k_resid_part<VT>), dim3(d.sa.slices * d.sa.wg_max), dim3(kBlock), 0, st, d);
  ACS_LAUNCH((k_resid_comb<VT>), dim3(comb_blocks(d.m)), dim3(kBlock), 0, st, d);
}

// workgroups whose ||r||^2 partials the finalize kernels of the CG sum
template <typename VT>
static int rr_blocks(const Dev<VT>& d) {
  return d.dense ? dense_row_blocks(d.m) : d.sa.slices == 1 ? d.sa.wg[0] : comb_blocks(d.m);
}

template <typename VT>
void launch_fin_resid(const Dev<VT>& d, int iter, double red2, double abs2, int cg_max, hipStream_t st) {
  const int nb = rr_blocks(d);
  ACS_LAUNCH((k_fin_resid<VT>), dim3(1), dim3(kBlock), 0, st, d, nb, iter, red2, abs2, cg_max);
}

template <typename VT>
void launch_cg_t(const Dev<VT>& d, int j, hipStream_t st) {
  if (d.dense) {
    ACS_LAUNCH((k_dense_cols<VT, DK_CG>), dim3(ceil_div(d.ld, kDenseStrip), d.dnchunk), dim3(kBlock), 0, st, d,
               static_cast<const VT*>(nullptr));
    ACS_LAUNCH((k_dense_cols_fin<VT, DK_CG, 0, false>), dim3(ceil_div(d.n, kBlock)), dim3(kBlock), 0, st, d,
               static_cast<const VT*>(nullptr), static_cast<VT*>(nullptr));
    return;
  }
  ACS_LAUNCH((k_cg_t<VT>), dim3(d.st_cg.wg[0]), dim3(kBlock), 0, st, d, cg_fin_folded(d) ? j : -1, rr_blocks(d));
}

template <typename VT>
void launch_cg_a(const Dev<VT>& d, long long launch_id, hipStream_t st) {
  if (d.dense) {  // the row product and the CG update of each row in one kernel
    ACS_LAUNCH((k_dense_rows<VT, DK_CG>), dim3(dense_row_blocks(d.m)), dim3(kBlock), 0, st, d, ceil_div(d.n, kBlock),
               static_cast<VT*>(nullptr));
    return;
  }
  if (d.sa.slices == 1) {  // the row product and the CG update of each row in one kernel
    ACS_LAUNCH((k_cg_a_one<VT>), dim3(d.sa.wg[0]), dim3(kBlock), 0, st, d, d.st_cg.wg[0], launch_id);
    return;
  }
  ACS_LAUNCH((k_cg_a_part<VT>), dim3(d.sa.slices * d.sa.wg_max), dim3(kBlock), 0, st, d, d.st_cg.wg[0]);
}

template <typename VT>
void launch_cg_comb(const Dev<VT>& d, hipStream_t st) {
  if (d.dense || d.sa.slices == 1) return;  // fused into the row product
  ACS_LAUNCH((k_cg_a_comb<VT>), dim3(comb_blocks(d.m)), dim3(kBlock), 0, st, d);
}

template <typename VT>
void launch_fin_cg_a(const Dev<VT>& d, long long launch_id, hipStream_t st) {
  const int nb = rr_blocks(d);
  ACS_LAUNCH((k_fin_cg_a<VT>), dim3(1), dim3(kBlock), 0, st, d, nb, launch_id);
}

template <typename VT>
void launch_pres(const Dev<VT>& d, int iter, double bnorm, double cnorm, hipStream_t st) {
  int nb = d.a_nblk;
  if (d.dense) {
    nb = dense_row_blocks(d.m);
    ACS_LAUNCH((k_dense_prep<VT>), dim3(ceil_div(d.n, kBlock)), dim3(kBlock), 0, st, d, 1,
               static_cast<const VT*>(nullptr));
    ACS_LAUNCH((k_dense_rows<VT, DK_PRES>), dim3(nb), dim3(kBlock), 0, st, d, 0, static_cast<VT*>(nullptr));
  } else {
    ACS_LAUNCH((k_pres<VT>), dim3(nb), dim3(kBlock), 0, st, d);
  }
  ACS_LAUNCH((k_fin_pres<VT>), dim3(1), dim3(kBlock), 0, st, d, nb, iter, bnorm, cnorm, int(d.n_soc > 0));
}

template <typename VT>
void launch_cond_ratio(const Dev<VT>& d, const VT* s_prev, const VT* s_cur, double t_cap, hipStream_t st) {
  const int units = d.n_orth + d.n_soc;
  const int nb = ceil_div(units, kBlock);
  ACS_LAUNCH((k_cond_ratio<VT>), dim3(nb), dim3(kBlock), 0, st, d, s_prev, s_cur);
  ACS_LAUNCH((k_fin_cond<VT>), dim3(1), dim3(kBlock), 0, st, d, nb, t_cap);
}

template <typename VT>
void launch_cond_scale(const Dev<VT>& d, VT* s_cur, hipStream_t st) {
  const int units = d.n_orth + d.n_soc;
  ACS_LAUNCH((k_cond_scale<VT>), dim3(ceil_div(units, kBlock)), dim3(kBlock), 0, st, d, s_cur);
}

template <typename VT>
void launch_rescale(const Dev<VT>& d, int wmode, hipStream_t st) {
  if (d.dense) {  // D from the stored A and O; the products scale on the fly
    ACS_LAUNCH((k_dense_prep<VT>), dim3(ceil_div(d.n, kBlock)), dim3(kBlock), 0, st, d, 2,
               static_cast<const VT*>(nullptr));
    ACS_LAUNCH((k_dense_rows<VT, DK_ROWSUM>), dim3(dense_row_blocks(d.m)), dim3(kBlock), 0, st, d, wmode,
               static_cast<VT*>(nullptr));
    ACS_LAUNCH((k_chat<VT>), dim3(ceil_div(d.n, kBlock)), dim3(kBlock), 0, st, d);
    return;
  }
  ACS_LAUNCH((k_rowsum<VT>), dim3(d.a_nblk), dim3(kBlock), 0, st, d, wmode);
  ACS_LAUNCH((k_scale_a<VT>), dim3(d.a_nblk), dim3(kBlock), 0, st, d);
  for (const auto* S : {&d.sa, &d.st}) {
    const int nb = int(std::max<int64_t>(1, std::min<int64_t>((S->entries + kBlock - 1) / kBlock, 8192)));
    const bool a = S == &d.sa;
    ACS_LAUNCH((k_sell_vals<VT>), dim3(nb), dim3(kBlock), 0, st, S->src, S->entries, d.a_val64,
                       a ? d.sa_val : d.st_val, a ? d.sa_val64 : d.st_val64);
  }
  if (d.st_cg_val != d.st_val) {  // the CG's own A_s^T values (sa_cg shares sa's)
    const int nb = int(std::max<int64_t>(1, std::min<int64_t>((d.st_cg.entries + kBlock - 1) / kBlock, 8192)));
    double* v64 = sizeof(VT) == sizeof(double) ? reinterpret_cast<double*>(d.st_cg_val) : nullptr;
    ACS_LAUNCH((k_sell_vals<VT>), dim3(nb), dim3(kBlock), 0, st, d.st_cg.src, d.st_cg.entries, d.a_val64,
               d.st_cg_val, v64);
  }
  ACS_LAUNCH((k_chat<VT>), dim3(ceil_div(d.n, kBlock)), dim3(kBlock), 0, st, d);
}

template <typename VT>
void launch_equilibrate(const Dev<VT>& d, int sweeps, hipStream_t st) {
  const int nb = int(std::max<int64_t>(1, std::min<int64_t>((d.st.entries + kBlock - 1) / kBlock, 8192)));
  ACS_LAUNCH((k_sk_sq<VT>), dim3(nb), dim3(kBlock), 0, st, d.st.src, d.st.entries, d.a_orig, d.st_val64);
  const int units = d.n_orth + d.n_soc;
  const double target = double(d.m) / double(d.n);
  for (int k = 0; k < sweeps; ++k) {
    ACS_LAUNCH((k_sk_rows<VT>), dim3(d.a_nblk), dim3(kBlock), 0, st, d);
    ACS_LAUNCH((k_sk_cols<VT>), dim3(d.st.wg[0]), dim3(kBlock), 0, st, d);
    ACS_LAUNCH((k_sk_unit<VT>), dim3(ceil_div(units, kBlock)), dim3(kBlock), 0, st, d, target,
               k + 1 == sweeps ? 1 : 0);
  }
}

template <typename VT>
void launch_spmv(const Dev<VT>& d, int which, const VT* x, VT* y, hipStream_t st) {
  if (d.dense) {
    if (which == 0) {
      ACS_LAUNCH((k_dense_prep<VT>), dim3(ceil_div(d.n, kBlock)), dim3(kBlock), 0, st, d, 3, x);
      ACS_LAUNCH((k_dense_rows<VT, DK_SPMV>), dim3(dense_row_blocks(d.m)), dim3(kBlock), 0, st, d, 0, y);
    } else {
      ACS_LAUNCH((k_dense_cols<VT, DK_SPMV>), dim3(ceil_div(d.ld, kDenseStrip), d.dnchunk), dim3(kBlock), 0, st,
                 d, x);
      ACS_LAUNCH((k_dense_cols_fin<VT, DK_SPMV, 0, false>), dim3(ceil_div(d.n, kBlock)), dim3(kBlock), 0, st, d,
                 static_cast<const VT*>(nullptr), y);
    }
    return;
  }
  if (which == 0) {
    ACS_LAUNCH((k_spmv_a<VT>), dim3(d.sa.slices * d.sa.wg_max), dim3(kBlock), 0, st, d, x);
    ACS_LAUNCH((k_spmv_comb<VT>), dim3(comb_blocks(d.m)), dim3(kBlock), 0, st, d, y);
  } else {
    ACS_LAUNCH((k_perm_in<VT>), dim3(ceil_div(d.m, kBlock)), dim3(kBlock), 0, st, d, x);
    ACS_LAUNCH((k_spmv_t<VT>), dim3(d.st.wg[0]), dim3(kBlock), 0, st, d, d.mtmp, y);
  }
}

template <typename VT>
void launch_out_device(const Dev<VT>& d, double* x, double* y, double* z, hipStream_t st) {
  ACS_LAUNCH((k_out_device<VT>), dim3(ceil_div(std::max(d.m, d.n), kBlock)), dim3(kBlock), 0, st, d, x, y, z);
}

template <typename VT>
void launch_ctl_reset(const Dev<VT>& d, int cg_max, hipStream_t st) {
  ACS_LAUNCH((k_ctl_reset<VT>), dim3(1), dim3(64), 0, st, d, cg_max);
}

#define ACS_INSTANTIATE(VT)                                                                            \
  template void launch_update<VT>(const Dev<VT>&, const VT*, VT*, int, bool, hipStream_t);            \
  template void launch_cone<VT>(const Dev<VT>&, const VT*, bool, bool, int, hipStream_t);            \
  template void launch_resid<VT>(const Dev<VT>&, hipStream_t);                                        \
  template void launch_fin_resid<VT>(const Dev<VT>&, int, double, double, int, hipStream_t);               \
  template void launch_cg_t<VT>(const Dev<VT>&, int, hipStream_t);                                    \
  template void launch_cg_a<VT>(const Dev<VT>&, long long, hipStream_t);                              \
  template void launch_cg_comb<VT>(const Dev<VT>&, hipStream_t);                                      \
  template void launch_fin_cg_a<VT>(const Dev<VT>&, long long, hipStream_t);                          \
  template void launch_pres<VT>(const Dev<VT>&, int, double, double, hipStream_t);                    \
  template void launch_cond_ratio<VT>(const Dev<VT>&, const VT*, const VT*, double, hipStream_t);     \
  template void launch_cond_scale<VT>(const Dev<VT>&, VT*, hipStream_t);                              \
  template void launch_rescale<VT>(const Dev<VT>&, int, hipStream_t);                                 \
  template void launch_spmv<VT>(const Dev<VT>&, int, const VT*, VT*, hipStream_t);                    \
  template void launch_ctl_reset<VT>(const Dev<VT>&, int, hipStream_t);                              \
  template void launch_equilibrate<VT>(const Dev<VT>&, int, hipStream_t);                             \
  template void launch_out_device<VT>(const Dev<VT>&, double*, double*, double*, hipStream_t);

ACS_INSTANTIATE(float)
ACS_INSTANTIATE(double)

}  // namespace acs
