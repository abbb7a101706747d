// HIP kernels of one Algorithm-2 instance on gfx950 (wave64).
//
// Scaled quantities kept on the device (O: column scaling of Alg. 2 step 11;
// d_i = 1/sqrt(sum_j a_ij^2 O_j^2), the row normalisation that makes the
// normal matrix unit-diagonal):
//   A_s = diag(d) A O   (values in CSR of A and, transposed, in CSR of A^T)
//   b_s = diag(d) b,    chat = mu O c
// range(A_s^T) = range((A O)^T), so the projection of step 17 is unchanged by
// the row normalisation.  One iteration (steps 16-20) is evaluated as
//   p  = abs_K(s)
//   w  : (A_s A_s^T) w = A_s (p - chat) - b_s           (CG, warm started)
//   s+ = (s + p)/2 - chat - A_s^T w
//   x  = O (p + s+)/2,  z = (p - s+)/(2 mu O),  y = -diag(d) w / mu
// which equals the listing's r = abs_{A_hat}(p), s+ = s/2 - r/2 + d.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <vector>

#include "acs_internal.h"

namespace acs {

// Timing of kernel launches.  While a LaunchEvents slot is installed on the
// calling thread, the launchers start the first kernel with `start` and every
// kernel with `stop` through hipExtLaunchKernelGGL, which takes both
// timestamps from the kernel dispatch itself (as a profiler does), so
// stop - start spans exactly the kernels launched, without separate event
// records on the stream.
struct LaunchEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
  int launches = 0;
};
LaunchEvents*& launch_events();  // thread-local slot, nullptr when not timing

// hipLaunchKernelGGL, or the timed launch while a LaunchEvents slot is set
#define ACS_LAUNCH(kernel, grid, block, shmem, stream, ...)                                          \
  do {                                                                                                \
    LaunchEvents* ev_ = launch_events();                                                              \
    if (ev_) {                                                                                        \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ev_->launches == 0 ? ev_->start : nullptr, \
                            ev_->stop, 0u, __VA_ARGS__);                                               \
      ++ev_->launches;                                                                                \
    } else {                                                                                          \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                            \
    }                                                                                                 \
  } while (0)

// Sums of the update kernel: ||s+ - s||^2; on check iterations also c^T x,
// ||x||^2, ||z||^2, the squared orthant distances of x and z, ||r_d||^2,
// r_d^T x and sum |x_j z_j| over the orthant
constexpr int kUpdSums = 9;
// Partial sums a reducing workgroup may write (the most of any reduction)
constexpr int kMaxSums = kUpdSums;

// Device control block of one instance (CG scalars, reductions, flags).
struct Ctl {
  double rho;     // ||r||^2 of the current CG residual
  double rho_step[2];  // ||r||^2 at the start of CG step j, in slot j & 1 (one-slice CG)
  double rho0;    // ||r_0||^2 of this outer iteration
  double tol2;    // CG stops when rho <= tol2
  double alpha;   // CG step length
  double beta;    // CG direction update (0 = fresh start)
  int32_t k;      // CG steps taken in this outer iteration
  int32_t done;   // CG finished for this outer iteration
  int32_t cg_max;
  int32_t iter;   // outer iteration the CG belongs to
  long long cg_total;
  double upd[9];  // reductions of the update kernel (kUpdSums)
  double cone[4]; // reductions of the cone kernel
  double cond[4]; // conditioning: min log o, -max log o, -any valid, alpha
  double kkt[9];  // eps_p, eps_d, eps_gap, eps_cone, kkt, pobj, dobj, ds2, eps_obj
};

// Host-visible status written by kernels into pinned, mapped host memory.
struct HostStatus {
  long long launch_seq;  // id of the last CG step the GPU has finished (8 slices) or reached (1 slice)
  int32_t cg_done_iter;  // last outer iteration whose CG finished
  int32_t check_iter;    // last iteration whose KKT check finished
  double kkt[9];         // copy of Ctl::kkt of check_iter
  long long cg_total;
  int32_t numeric;       // NaN/Inf seen
  int32_t pad;
};

// Device view of a Sell layout (see acs_internal.h).
struct SellDev {
  const int32_t* long_row;
  const int32_t* long_beg;
  const int32_t* long_end;
  const int32_t* wt_ptr;
  const int32_t* wt_len;
  const int32_t* wt_row;
  const int32_t* chunk_row;
  const int32_t* col;
  const int32_t* src;
  int64_t entries;
  int32_t long_off[kSlices + 1];
  int32_t wt_off[kSlices + 1];
  int32_t wg[kSlices];
  int32_t wg_max;
  int32_t slices;
};

template <typename VT>
struct Dev {
  int32_t m, n, n_orth, n_soc;
  int32_t a_rp_nnz;  // nnz
  double mu;
  // CSR of A (rows i): the problem's values a_orig and FP64 A_s (source of
  // the SELL values, KKT check, conditioning)
  const int32_t* a_rp;
  const int32_t* a_col;
  const double* a_orig;
  double* a_val64;
  // SELL layouts of the products with A_s (column slices, one per XCD) and
  // A_s^T: values in VT for the CG and in FP64 for the once-per-iteration
  // residual and update sweeps (iterative refinement of the CG); the FP64
  // arrays alias the VT ones when VT = double
  SellDev sa, st;
  VT* sa_val;
  VT* st_val;
  double* sa_val64;
  double* st_val64;
  // the CG's layouts: with 8 slices the columns of A are renumbered within
  // each slice in the order sa first reads them, so the CG vector t is stored
  // in that order: sa_cg is sa with the renumbered column array (values
  // sa_val), st_cg the A_s^T layout with its rows in the new order and its
  // own VT values.  With one slice they are sa, st and st_val themselves.
  SellDev sa_cg, st_cg;
  VT* st_cg_val;
  VT* part;                // kSlices x m partial row sums of A_s t
  double* part64;          // kSlices x m partial row sums of the FP64 residual
  const int32_t* row_perm; // internal row -> caller's row
  VT* mtmp;                // m-vector scratch of the plain products
  // dense A (row-major, leading dimension ld, padding columns zero): FP32
  // values, dlo = FP32 rounding error of each value or nullptr; products
  // apply D and O to vectors.  Column products run over row chunks of dchunk
  // rows into dpart (dnchunk x ld partial sums), then a reduction kernel.
  int32_t dense;
  int32_t ld;
  int32_t dchunk, dnchunk;
  const float* dhi;
  const float* dlo;
  double* dpart;
  VT* dx32;      // ld-vector input of the FP32 row products (O t, O x)
  double* dx64;  // ld-vector input of the FP64 row products (O v, O xhat, O^2)
  double* partials2;  // ||t||^2 partials of the dense CG, read by the row product
  const RowBlock* a_blk;
  int32_t a_nblk;
  const int32_t* soc_off;  // n_soc + 1 absolute offsets
  const double* b;
  const double* c;
  // scaling
  double* O;
  double* chat;
  double* dsq;
  double* dinv;
  double* bs;
  // iterate and CG
  VT* p;     // abs_K(s) on SOC coordinates (orthant ones are recomputed)
  VT* v;     // p - chat - A_s^T w : the CG right-hand side before A_s
  double* zt;  // chat + A_s^T w on SOC coordinates
  double* w;
  VT* r;
  double* r64;  // FP64 copy of the residual for the direct projection, else nullptr
  VT* q;
  VT* t;
  // outputs
  double* xout;
  double* zout;
  double* yout;
  double* xhat;
  double* xc;
  double* zc;
  double* ounit;
  Ctl* ctl;
  double* partials;
  HostStatus* hs;
  // Sinkhorn-Knopp equilibration (settings.equilibrate), else nullptr: eq
  // holds E^2 during the sweeps, then E (per coordinate, constant on every
  // cone); eq_u (m) is D^2 of the current sweep, eq_c (n) the column sums
  double* eq;
  double* eq_u;
  double* eq_c;
};

// Direct projection: the normal matrix M = A_s A_s^T of the current scaling,
// formed and inverted in FP64 at each conditioning event; each iteration
// then corrects w by M^{-1} r instead of running the CG.
constexpr int kFacTile = 64;        // pivot block and tile of the inversion sweep
constexpr int kFacPad = 128;        // the order of M is padded to a multiple of this
constexpr int kFacGroup = 4;        // sweep steps applied by one pass over the inverse
constexpr int kFacSlots = 2 * kFacGroup;  // W panels: this group's and the next group's
constexpr int kFacMaxOrder = 32768; // largest padded order (8 GiB of FP64)
constexpr double kFacPivotTol = 1e-11;  // pivots at or below it (unit-diagonal M) count as dependent rows

struct FacDev {
  int32_t m;    // rows of A
  int32_t mp;   // padded order of M (multiple of kFacPad)
  int32_t ldb;  // leading dimension of B (multiple of 64)
  int32_t nb;   // pivot blocks swept: ceil(m / kFacTile)
  double* S;    // mp x mp: M, then -M^{-1} (lower tiles) during the sweep, then M^{-1} (full)
  double* B;    // mp x ldb: A_s in FP64, zero outside m x n
  double* C;    // kFacSlots x mp x kFacTile: W = Op L^{-T} of sweep step K in slot K mod kFacSlots (Op the pivot-column panel)
  double* P;    // kFacTile x kFacTile: L^{-1}, L the Cholesky factor of the current pivot block
  // workgroup -> tile tables (fac_tile_order) of the form step (128 x 128
  // tiles of mp) and of the sweep's update (64 x 64 tiles of nb blocks)
  const int32_t* syrk_order;
  const int32_t* upd_order;
  int32_t syrk_blocks, upd_blocks;
};

// Workgroup order over the lower-triangular tiles (I, J), J <= I < tiles:
// squares of up to 8 x 8 tiles, each handed whole to one XCD (workgroup b runs on
// XCD b % 8), so the 64 workgroups an XCD runs at once share 8 row and 8
// column panels in its L2.  Entry (I << 16) | J, or -1 for an idle workgroup.
std::vector<int32_t> fac_tile_order(int tiles);

enum UpdMode { UPD_PROLOGUE = 0, UPD_UPDATE = 1, UPD_UPDATE_ONLY = 2 };

// Launchers (all on `st`); grid sizes derive from the row-block counts.
template <typename VT> void launch_update(const Dev<VT>& d, const VT* s_cur, VT* s_new, int mode, bool check,
                                          hipStream_t st);
template <typename VT> void launch_cone(const Dev<VT>& d, const VT* s, bool check, bool next, int group,
                                        hipStream_t st);
// residual sweep and its finalizer (rho_0, threshold, zero-step exit)
template <typename VT> void launch_resid(const Dev<VT>& d, hipStream_t st);
template <typename VT> void launch_fin_resid(const Dev<VT>& d, int iter, double red2, double abs2, int cg_max,
                                             hipStream_t st);
// the two CG sweeps (alpha in the first workgroup of the sliced one), the
// combine with the CG update, and the finalizer (beta, stop test, host progress record)
// CG step j (0-based) of the outer iteration; the one-slice layout finalizes
// step j-1 inside k_cg_t and posts `launch_id` from k_cg_a_one
template <typename VT> void launch_cg_t(const Dev<VT>& d, int j, hipStream_t st);
template <typename VT> void launch_cg_a(const Dev<VT>& d, long long launch_id, hipStream_t st);
// whether the per-step finalize (k_fin_cg_a) is folded into the next step
template <typename VT> bool cg_fin_folded(const Dev<VT>& d) { return !d.dense && d.sa.slices == 1; }
template <typename VT> void launch_cg_comb(const Dev<VT>& d, hipStream_t st);
template <typename VT> void launch_fin_cg_a(const Dev<VT>& d, long long launch_id, hipStream_t st);
template <typename VT> void launch_pres(const Dev<VT>& d, int iter, double bnorm, double cnorm, hipStream_t st);
template <typename VT> void launch_cond_ratio(const Dev<VT>& d, const VT* s_prev, const VT* s_cur, double t_cap,
                                              hipStream_t st);
template <typename VT> void launch_cond_scale(const Dev<VT>& d, VT* s_cur, hipStream_t st);
template <typename VT> void launch_rescale(const Dev<VT>& d, int wmode, hipStream_t st);
// plain product with the current A_s through the CG's SELL kernels; m-vectors
// in the caller's row order
template <typename VT> void launch_spmv(const Dev<VT>& d, int which, const VT* x, VT* y, hipStream_t st);
template <typename VT> void launch_ctl_reset(const Dev<VT>& d, int cg_max, hipStream_t st);
// Sinkhorn-Knopp equilibration: `sweeps` sweeps from eq = 1 (set by the
// caller), leaving E in eq (sparse problems)
template <typename VT> void launch_equilibrate(const Dev<VT>& d, int sweeps, hipStream_t st);
// x, z (n) and y (m, caller's row order) of the last check into device buffers (any may be null)
template <typename VT> void launch_out_device(const Dev<VT>& d, double* x, double* y, double* z, hipStream_t st);
// direct projection: B = A_s (copy), M = B B^T (syrk), M -> M^{-1} (the
// sweep: for K = 0..nb-1 pivot_panel(K) then update(K); then mirror),
// w += M^{-1} r64 (apply)
template <typename VT> void launch_fac_copy(const Dev<VT>& d, const FacDev& f, hipStream_t st);
void launch_fac_syrk(const FacDev& f, hipStream_t st);
// Sweep steps in groups K0, .., K0 + cnt - 1 (K0 a multiple of kFacGroup,
// cnt <= kFacGroup).  The group's chain: for g = 0 .. cnt - 1,
// launch_fac_pivot_panel(K0 + g), then (g + 1 < cnt) launch_fac_strip with
// g + 1 terms.  Then its pass with cnt terms: launch_fac_pass for the last
// group; otherwise launch_fac_pass_next (the tiles of the next group's block
// rows and columns, nxt .. nxt + cntn - 1), after which the next group's
// chain may run on another stream alongside launch_fac_pass_rest (all other
// tiles).
void launch_fac_pivot_panel(const FacDev& f, int K, int K0, hipStream_t st);
void launch_fac_strip(const FacDev& f, int K0, int terms, hipStream_t st);
void launch_fac_pass(const FacDev& f, int K0, int terms, hipStream_t st);
void launch_fac_pass_next(const FacDev& f, int K0, int terms, int nxt, int cntn, hipStream_t st);
void launch_fac_pass_rest(const FacDev& f, int K0, int terms, int nxt, int cntn, hipStream_t st);
void launch_fac_mirror(const FacDev& f, hipStream_t st);
template <typename VT> void launch_fac_apply(const Dev<VT>& d, const FacDev& f, hipStream_t st);

}  // namespace acs
