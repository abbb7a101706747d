// Persistent batched kernel: one workgroup advances one instance through
// Algorithm 2 (same fused form and precision split as the one-instance
// kernels, see acs_kernels.h), taking instances from a device work queue.
// Rows are handled by groups of G lanes (G per instance and per matrix,
// chosen by the autotuner); all reductions are workgroup reductions in a
// fixed order, so a batch result does not depend on which workgroup ran it.
#include <cmath>

#include "acs_batch.h"

namespace acs {

namespace {

constexpr int kBB = 256;  // threads per workgroup of the batch kernel

template <typename T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ double wmin(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}

// Workgroup sum / min, result on every thread.
__device__ __forceinline__ double bsum(double v, double* sh) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = sh[0];
  for (int i = 1; i < kBB / 64; ++i) s += sh[i];
  return s;
}

__device__ __forceinline__ double bmin(double v, double* sh) {
  v = wmin(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = sh[0];
  for (int i = 1; i < kBB / 64; ++i) s = fmin(s, sh[i]);
  return s;
}

// Row sums of prod(k) with G lanes per row; epi(row, sum) on one lane.  A
// lane takes its entries four at a time, all four products' loads issued
// before the first add (the adds keep the order of k, so sums do not change).
template <typename Acc, class Prod, class Epi>
__device__ __forceinline__ void bspmv(const int32_t* __restrict__ rp, int nrows, int G, Prod& prod, Epi& epi) {
  const int tid = threadIdx.x, ngrp = kBB / G, grp = tid / G, lane = tid & (G - 1);
  for (int base = 0; base < nrows; base += ngrp) {
    const int r = base + grp;
    Acc s = 0;
    if (r < nrows) {
      const int e = rp[r + 1];
      int k = rp[r] + lane;
      for (; k + 3 * G < e; k += 4 * G) {
        const Acc p0 = prod(k), p1 = prod(k + G), p2 = prod(k + 2 * G), p3 = prod(k + 3 * G);
        s += p0;
        s += p1;
        s += p2;
        s += p3;
      }
      for (; k < e; k += G) s += prod(k);
    }
    for (int off = G >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0 && r < nrows) epi(r, s);
  }
}

// f(row, k) for every nonzero, G lanes per row
template <class F>
__device__ __forceinline__ void bforeach(const int32_t* __restrict__ rp, int nrows, int G, F& f) {
  const int tid = threadIdx.x, ngrp = kBB / G, grp = tid / G, lane = tid & (G - 1);
  for (int r = grp; r < nrows; r += ngrp) {
    const int e = rp[r + 1];
    for (int k = rp[r] + lane; k < e; k += G) f(r, k);
  }
}

__device__ __forceinline__ bool in_sched(const BInst& I, int l) {
  if (l == 1) return true;
  if (I.l_first <= 0 || l < I.l_first) return false;
  if (I.l_last >= 0 && l > I.l_last) return false;
  if (I.l_every <= 0) return l == I.l_first;
  return (l - I.l_first) % I.l_every == 0;
}

__device__ __forceinline__ double ldist2(double u0, double nb) {
  if (nb <= u0) return 0.0;
  if (nb <= -u0) return u0 * u0 + nb * nb;
  const double g = nb - u0;
  return 0.5 * g * g;
}

// closed-form Lorentz projection of v = (v0, vbar) with ||vbar|| = nv: proj = (a0, f vbar)
__device__ __forceinline__ void lproj(double v0, double nv, double& a0, double& f) {
  if (nv <= v0) {
    a0 = v0;
    f = 1.0;
  } else if (nv <= -v0) {
    a0 = 0.0;
    f = 0.0;
  } else {
    a0 = 0.5 * (v0 + nv);
    f = a0 / nv;
  }
}

constexpr int kStageMax = 1024;  // LDS stage of the staged schedule (nonzeros)

struct Shared {
  double red[kBB / 64];
  double stage[kStageMax];  // staged products (double, or float in the first half)
  BInst inst;               // the running instance's descriptor, kept in LDS
};

// One sweep over the rows of A_s (which = 0) or of A_s^T (which = 1) with the
// instance's schedule: direct (G lanes per row) or LDS-staged row blocks.
template <typename Acc, class Prod, class Epi>
__device__ __forceinline__ void bsweep(const BInst& I, int which, Prod& prod, Epi& epi, Shared& sh) {
  const int32_t* __restrict__ rp = which ? I.t_rp : I.a_rp;
  if (!(which ? I.st_t : I.st_a)) {
    bspmv<Acc>(rp, which ? I.n : I.m, which ? I.g_t : I.g_a, prod, epi);
    return;
  }
  const RowBlock* __restrict__ blk = which ? I.t_blk : I.a_blk;
  const int nb = which ? I.t_nblk : I.a_nblk;
  Acc* lds = reinterpret_cast<Acc*>(sh.stage);
  const int tid = threadIdx.x;
  for (int b = 0; b < nb; ++b) {
    const RowBlock rb = blk[b];
    const int k0 = rp[rb.r0], k1 = rp[rb.r1];
    if (k1 - k0 > kStageMax) {  // one row longer than the stage: the whole workgroup
      Acc s = 0;
      for (int k = k0 + tid; k < k1; k += kBB) s += prod(k);
      s = wsum(s);
      __syncthreads();  // a preceding bsum may still be reading sh.red
      if ((tid & 63) == 0) sh.red[tid >> 6] = double(s);
      __syncthreads();
      if (tid == 0) {
        double tot = sh.red[0];
        for (int i = 1; i < kBB / 64; ++i) tot += sh.red[i];
        epi(rb.r0, Acc(tot));
      }
      __syncthreads();
      continue;
    }
#pragma unroll
    for (int it = 0; it < kStageMax / kBB; ++it) {
      const int k = k0 + it * kBB + tid;
      if (k < k1) lds[k - k0] = prod(k);
    }
    __syncthreads();
    const int nrows = rb.r1 - rb.r0;
    int G = 64;
    while (G > 1 && G * nrows > kBB) G >>= 1;
    const int grp = tid / G, lane = tid & (G - 1), ngrp = kBB / G;
    for (int r = rb.r0 + grp; r < rb.r1; r += ngrp) {
      const int a = rp[r] - k0, e = rp[r + 1] - k0;
      Acc sacc = 0;
      for (int k = a + lane; k < e; k += G) sacc += lds[k];
      for (int off = G >> 1; off > 0; off >>= 1) sacc += __shfl_xor(sacc, off);
      if (lane == 0) epi(r, sacc);
    }
    __syncthreads();
  }
}

// p = abs_K(s), v = p - zt on the Lorentz cones of s (thread per cone)
__device__ void cones_next(BInst& I, const float* __restrict__ s) {
  for (int cone = threadIdx.x; cone < I.n_soc; cone += kBB) {
    const int off = I.soc_off[cone], end = I.soc_off[cone + 1];
    double n2 = 0;
    for (int e = off + 1; e < end; ++e) n2 += double(s[e]) * double(s[e]);
    double a0, f;
    lproj(double(s[off]), sqrt(n2), a0, f);
    for (int e = off; e < end; ++e) {
      const double se = double(s[e]);
      const float pv = float(2.0 * ((e == off) ? a0 : f * se) - se);
      I.p[e] = pv;
      I.v[e] = float(double(pv) - I.zt[e]);
    }
  }
}

// A_s^T w sweep: prologue (mode 0), update (1), update without next p/v (2)
__device__ void sweep_update(BInst& I, int mode, bool check, double (&acc)[10], Shared& sh) {
  const float* __restrict__ s = I.s_buf[I.cur];
  float* __restrict__ sn_out = I.s_buf[I.cur ^ 1];
  const double* __restrict__ tv = I.t_val64;
  const int32_t* __restrict__ tc = I.t_col;
  const double* __restrict__ w = I.w;
  const double mu = I.mu;
  auto prod = [&](int k) -> double { return tv[k] * w[tc[k]]; };
  auto epi = [&](int j, double u) {
    const double zt = I.chat[j] + u;
    const double sj = double(s[j]);
    const bool orth = j < I.n_orth;
    double sn = sj;
    if (mode != 0) {
      const double pj = orth ? fabs(sj) : double(I.p[j]);
      const float snv = float(0.5 * (sj + pj) - zt);
      sn_out[j] = snv;
      sn = double(snv);
      if (check) {
        const double Oj = I.O[j];
        const double xh = 0.5 * (pj + sn);
        const double x = Oj * xh;
        const double z = 0.5 * (pj - sn) / (mu * Oj);
        I.x[j] = x;
        I.z[j] = z;
        I.xhat[j] = xh;
        acc[0] += I.c[j] * x;
        acc[1] += x * x;
        acc[2] += z * z;
        if (orth) {
          const double mx = fmin(x, 0.0), mz = fmin(z, 0.0);
          acc[3] += mx * mx;
          acc[4] += mz * mz;
        }
        if (orth) acc[8] += fabs(x * z);  // |x_j z_j| of the objective-error estimate
        const double dr = (pj - sn - 2.0 * zt) / (2.0 * mu * Oj);
        acc[5] += dr * dr;
      }
    }
    if (mode != 2) {
      if (orth)
        I.v[j] = float(fabs(sn) - zt);
      else
        I.zt[j] = zt;
    }
  };
  bsweep<double>(I, 1, prod, epi, sh);
  __syncthreads();
  if (I.n_soc > 0) {
    if (check) {  // cone distances of x and z (written above)
      for (int cone = threadIdx.x; cone < I.n_soc; cone += kBB) {
        const int off = I.soc_off[cone], end = I.soc_off[cone + 1];
        double nx = 0, nz = 0, xz = I.x[off] * I.z[off];
        for (int e = off + 1; e < end; ++e) {
          nx += I.x[e] * I.x[e];
          nz += I.z[e] * I.z[e];
          xz += I.x[e] * I.z[e];
        }
        acc[6] += ldist2(I.x[off], sqrt(nx));
        acc[7] += ldist2(I.z[off], sqrt(nz));
        acc[9] += xz;  // x_C^T z_C, summed with signs over the cones
      }
    }
    if (mode != 2) cones_next(I, mode == 0 ? s : sn_out);
    __syncthreads();
  }
}

// steps 5-14 + 12 (rebuild A_s) at the start of iteration l
__device__ void condition(BInst& I, Shared& sh) {
  const float* __restrict__ sp = I.s_buf[I.cur ^ 1];
  float* __restrict__ sc = I.s_buf[I.cur];
  const double mu = I.mu;
  const int units = I.n_orth + I.n_soc;
  double mn = INFINITY, mnn = INFINITY, anyv = INFINITY;
  for (int u = threadIdx.x; u < units; u += kBB) {
    double num, den;
    if (u < I.n_orth) {
      const double pj = fabs(double(sp[u])), s = double(sc[u]), Oj = I.O[u];
      const double x = Oj * 0.5 * (pj + s), z = 0.5 * (pj - s) / (mu * Oj);
      I.x[u] = x;
      I.z[u] = z;
      num = fabs(x);
      den = fabs(z);
    } else {
      const int cone = u - I.n_orth;
      const int off = I.soc_off[cone], end = I.soc_off[cone + 1];
      const double Ob = I.O[off];
      double n2 = 0;
      for (int e = off + 1; e < end; ++e) n2 += double(sp[e]) * double(sp[e]);
      double a0, f;
      lproj(double(sp[off]), sqrt(n2), a0, f);
      double nb = 0, x0 = 0, z0 = 0;
      for (int e = off; e < end; ++e) {
        const double spe = double(sp[e]);
        const double pe = 2.0 * ((e == off) ? a0 : f * spe) - spe;
        const double se = double(sc[e]);
        const double x = Ob * 0.5 * (pe + se), z = 0.5 * (pe - se) / (mu * Ob);
        I.x[e] = x;
        I.z[e] = z;
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
    I.ounit[u] = o;
    if (o > 0.0 && !isinf(o) && o == o) {
      const double lo = log(o);
      mn = fmin(mn, lo);
      mnn = fmin(mnn, -lo);
      anyv = -1.0;
    }
  }
  mn = bmin(mn, sh.red);
  mnn = bmin(mnn, sh.red);
  anyv = bmin(anyv, sh.red);
  const bool any = anyv < 0.0;
  const double span = -mnn - mn;
  const double alpha = (any && span > 0.0) ? fmin(1.0, I.t_cap / span) : 1.0;
  for (int u = threadIdx.x; u < units; u += kBB) {
    double Onew = 1.0;
    if (any) {
      double o = I.ounit[u];
      if (!(o == o)) o = 1.0;
      if (o == 0.0) o = exp(mn);
      if (isinf(o)) o = exp(-mnn);
      Onew = pow(o, alpha);
    }
    int off = u, end = u + 1;
    if (u >= I.n_orth) {
      off = I.soc_off[u - I.n_orth];
      end = I.soc_off[u - I.n_orth + 1];
    }
    for (int e = off; e < end; ++e) {
      I.O[e] = Onew;
      I.chat[e] = mu * Onew * I.c[e];
      sc[e] = float(I.x[e] / Onew - mu * Onew * I.z[e]);
    }
  }
  __syncthreads();
  // D_i = sum_j a_ij^2 O_j^2 ; w keeps the unscaled multiplier
  auto prodD = [&](int k) -> double {
    const double g = I.a_orig[k] * I.O[I.a_col[k]];
    return g * g;
  };
  auto epiD = [&](int i, double D) {
    if (!(D > 0.0)) D = 1.0;
    const double ds = sqrt(D);
    I.w[i] *= ds / I.dsq[i];
    I.dsq[i] = ds;
    I.dinv[i] = 1.0 / ds;
    I.bs[i] = I.b[i] / ds;
  };
  bsweep<double>(I, 0, prodD, epiD, sh);
  __syncthreads();
  auto fa = [&](int i, int k) {
    const double a = I.a_orig[k] * I.O[I.a_col[k]] * I.dinv[i];
    I.a_val64[k] = a;
    I.a_val[k] = float(a);
  };
  bforeach(I.a_rp, I.m, I.st_a ? 16 : I.g_a, fa);
  auto ft = [&](int j, int k) {
    const double a = I.a_orig[I.t_perm[k]] * I.O[j] * I.dinv[I.t_col[k]];
    I.t_val64[k] = a;
    I.t_val[k] = float(a);
  };
  bforeach(I.t_rp, I.n, I.st_t ? 16 : I.g_t, ft);
  __syncthreads();
  if (threadIdx.x == 0) {
    I.conds += 1;
    I.kkt[7] = alpha;
  }
}

// Steps 17-18 projection of iteration l: residual r = A_s v - b_s (FP64
// accumulation), then warm-started CG on (A_s A_s^T) dw = r.  With LDS the two
// gathered vectors r (m) and t (n) live in the workgroup's LDS, so the CG's
// random reads cost an LDS access instead of an L2 request; q and w stay in
// global memory.  Returns the CG steps taken; `bad` reports a NaN/Inf.
template <bool LDS>
__device__ __forceinline__ int project(BInst& I, Shared& sh, float* __restrict__ lds, int l, bool& bad_out) {
  float* __restrict__ rv = LDS ? lds : I.r;
  float* __restrict__ tvec = LDS ? lds + I.m : I.t;
  // r = A_s v - b_s (FP64 accumulation)
  double acc = 0;
  {
    const double* __restrict__ av = I.a_val64;
    const int32_t* __restrict__ ac = I.a_col;
    const float* __restrict__ v = I.v;
    auto prod = [&](int k) -> double { return av[k] * double(v[ac[k]]); };
    auto epi = [&](int i, double s) {
      const float ri = float(s - I.bs[i]);
      rv[i] = ri;
      acc += double(ri) * double(ri);
    };
    bsweep<double>(I, 0, prod, epi, sh);
  }
  double rho = bsum(acc, sh.red);
  // x, z of this iteration set O at l + 1: project accurately
  const bool feeds_event = in_sched(I, l + 1);
  const double red2 = feeds_event ? fmin(I.cg_red2, kEventCgReduce * kEventCgReduce) : I.cg_red2;
  const int cg_max = feeds_event ? I.cg_max * kEventCgMaxFactor : I.cg_max;
  const double tol2 = fmax(red2 * rho, I.cg_abs2);
  double beta = 0.0;
  int k = 0;
  bool bad = !(rho == rho) || isinf(rho);
  while (!bad && k < cg_max && rho > tol2) {
    acc = 0;
    {
      const float* __restrict__ tv = I.t_val;
      const int32_t* __restrict__ tc = I.t_col;
      const float* __restrict__ r = rv;
      const float vb = float(beta);
      auto prod = [&](int kk) -> float { return tv[kk] * r[tc[kk]]; };
      auto epi = [&](int j, float s) {
        const float tj = (beta != 0.0) ? s + vb * tvec[j] : s;
        tvec[j] = tj;
        acc += double(tj) * double(tj);
      };
      bsweep<float>(I, 1, prod, epi, sh);
    }
    const double tt = bsum(acc, sh.red);
    if (!(tt > 0.0) || isinf(tt)) {
      bad = !(tt == tt);
      break;
    }
    const double alpha = rho / tt;
    acc = 0;
    {
      const float* __restrict__ av = I.a_val;
      const int32_t* __restrict__ ac = I.a_col;
      const float* __restrict__ t = tvec;
      const float va = float(alpha), vb = float(beta);
      auto prod = [&](int kk) -> float { return av[kk] * t[ac[kk]]; };
      auto epi = [&](int i, float mq) {
        const float ri = rv[i];
        const float qi = (beta != 0.0) ? ri + vb * I.q[i] : ri;
        I.q[i] = qi;
        I.w[i] += alpha * double(qi);
        const float rn = ri - va * mq;
        rv[i] = rn;
        acc += double(rn) * double(rn);
      };
      bsweep<float>(I, 0, prod, epi, sh);
    }
    const double rn = bsum(acc, sh.red);
    bad = !(rn == rn) || isinf(rn);
    beta = bad ? 0.0 : rn / rho;
    rho = rn;
    ++k;
  }
  bad_out = bad;
  return k;
}

__device__ void solve_one(BInst* gI, int budget, Shared& sh, float* __restrict__ lds, int lds_floats) {
  BInst& I = sh.inst;
  {
    const int words = int(sizeof(BInst) / sizeof(int));
    const int* src = reinterpret_cast<const int*>(gI);
    int* dst = reinterpret_cast<int*>(&I);
    for (int i = threadIdx.x; i < words; i += kBB) dst[i] = src[i];
  }
  __syncthreads();
  if (I.status >= 0) return;
  const int it_end = min(I.max_iter, I.l + budget);
  const double mu = I.mu;
  int status = -1;
  long long cgt = I.cg_total;
  while (I.l < it_end) {
    const int l = I.l + 1;
    if (in_sched(I, l)) {
      condition(I, sh);
      double dummy[10];
      sweep_update(I, 0, false, dummy, sh);
    }
    bool bad = false;
    const int k = (I.m + I.n <= lds_floats) ? project<true>(I, sh, lds, l, bad) : project<false>(I, sh, lds, l, bad);
    cgt += k;
    __syncthreads();
    const bool next_event = in_sched(I, l + 1);
    const bool check = (l % I.check_every == 0) || l == I.max_iter;
    double ac[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    sweep_update(I, next_event ? 2 : 1, check, ac, sh);
    __syncthreads();
    if (threadIdx.x == 0) {
      I.cur ^= 1;
      I.l = l;
    }
    __syncthreads();
    if (check) {
      double a2[3] = {0, 0, 0};
      const double* __restrict__ av = I.a_val64;
      const int32_t* __restrict__ acol = I.a_col;
      const double* __restrict__ xh = I.xhat;
      auto prod = [&](int kk) -> double { return av[kk] * xh[acol[kk]]; };
      auto epi = [&](int i, double ax) {
        const double res = (ax - I.bs[i]) * I.dsq[i];
        a2[0] += res * res;
        const double yi = -I.dinv[i] * I.w[i] / mu;
        I.y[i] = yi;
        a2[1] += I.b[i] * yi;
        a2[2] += yi * res;  // y^T r_p of the objective-error estimate
      };
      bsweep<double>(I, 0, prod, epi, sh);
      double tot[10];
      for (int i = 0; i < 10; ++i) tot[i] = bsum(ac[i], sh.red);
      const double pres2 = bsum(a2[0], sh.red), bty = bsum(a2[1], sh.red), ytrp = bsum(a2[2], sh.red);
      const double ctx = tot[0];
      double e[7];
      e[0] = sqrt(pres2) / (1.0 + I.bnorm);
      e[1] = sqrt(tot[5]) / (1.0 + I.cnorm);
      e[2] = fabs(ctx - bty) / (1.0 + fabs(ctx) + fabs(bty));
      e[3] = fmax(sqrt(tot[3] + tot[6]), sqrt(tot[4] + tot[7])) / (1.0 + fmax(sqrt(tot[1]), sqrt(tot[2])));
      e[4] = fmax(fmax(e[0], e[1]), fmax(e[2], e[3]));
      e[5] = ctx;
      e[6] = bty;
      // estimate of the objective's relative error (see acs.h)
      const double eobj = (tot[8] + fabs(tot[9]) + fabs(ytrp)) / (1.0 + fabs(ctx));
      bool nan = bad || !(eobj == eobj) || isinf(eobj);
      for (int i = 0; i < 7; ++i)
        if (!(e[i] == e[i]) || isinf(e[i])) nan = true;
      if (nan)
        status = ACS_NUMERIC;
      else if (e[4] <= I.eps && eobj * I.obj_stop <= I.eps)
        status = ACS_SOLVED;
      else if (l >= I.max_iter)
        status = ACS_MAX_ITER;
      __syncthreads();
      if (threadIdx.x == 0) {
        for (int i = 0; i < 7; ++i) I.kkt[i] = e[i];
        I.kkt[8] = eobj;
        I.checked = l;
      }
    } else if (bad) {
      status = ACS_NUMERIC;
    }
    __syncthreads();
    if (status >= 0) break;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    I.cg_total = cgt;
    I.status = status;
    gI->l = I.l;
    gI->cur = I.cur;
    gI->status = I.status;
    gI->conds = I.conds;
    gI->checked = I.checked;
    gI->cg_total = I.cg_total;
    for (int i = 0; i < 9; ++i) gI->kkt[i] = I.kkt[i];
  }
  __syncthreads();
}

}  // namespace

// 4 waves per SIMD (16 per CU, 4 workgroups): 128 registers, a few spilled to
// scratch.  Unconstrained the kernel takes 169 registers, 2 workgroups per CU;
// measured on the 4096-LP batch, 3 workgroups (168 registers) gave +23% and 4
// a further +23% on the same box, with the stage at 1024 nonzeros so that 4
// workgroups and the CG vectors fit the 160 KB of LDS.
__global__ __launch_bounds__(kBB) __attribute__((amdgpu_waves_per_eu(4))) void k_batch(
    BInst* inst, const int32_t* order, int count, unsigned int* queue, int budget, int lds_floats) {
  __shared__ Shared sh;
  __shared__ int idx;
  extern __shared__ float vec_lds[];  // lds_floats: r and t of instances with m + n <= lds_floats
  for (;;) {
    if (threadIdx.x == 0) idx = int(atomicAdd(queue, 1u));
    __syncthreads();
    const int i = idx;
    __syncthreads();
    if (i >= count) return;
    solve_one(&inst[order[i]], budget, sh, vec_lds, lds_floats);
  }
}

__global__ void k_queue_reset(unsigned int* queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0u;
}

void launch_batch(BInst* inst, const int32_t* order, int32_t count, unsigned int* queue, int32_t grid,
                  int32_t lds_floats, int32_t iter_budget, hipStream_t st) {
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBB), size_t(lds_floats) * sizeof(float), st, inst, order, count, queue,
                     iter_budget, lds_floats);
}

int batch_blocks_per_cu(int32_t lds_floats) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch, kBB, size_t(lds_floats) * sizeof(float)) != hipSuccess)
    nb = 1;
  return nb > 0 ? nb : 1;
}

void launch_queue_reset(unsigned int* queue, hipStream_t st) {
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, queue);
}

}  // namespace acs
