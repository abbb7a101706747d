// Batched solving of many independent small instances: one persistent launch,
// one workgroup per instance at a time, instances taken from a device work
// queue (largest first).  Each workgroup runs the whole of Algorithm 2 for
// its instance with workgroup-level sweeps and reductions, so instances never
// synchronise with each other.
#pragma once

#include <hip/hip_runtime.h>

#include "acs_internal.h"

namespace acs {

// Per-instance descriptor and resident state (device memory).
// Sweep schedule of one matrix of an instance: `staged` = 0 sums each row
// with `param` lanes reading the matrix directly; `staged` = 1 walks
// host-built row blocks of at most `param` nonzeros staged through LDS.
struct Sched {
  int32_t staged;
  int32_t param;
};

struct BInst {
  int32_t m, n, nnz, n_orth, n_soc;
  int32_t g_a, g_t;  // lanes per row for rows of A_s and of A_s^T (direct schedule)
  int32_t st_a, st_t;  // 1: staged schedule for rows of A_s / of A_s^T
  int32_t a_nblk, t_nblk;
  const RowBlock* a_blk;
  const RowBlock* t_blk;
  const int32_t* a_rp;
  const int32_t* a_col;
  const double* a_orig;
  float* a_val;
  double* a_val64;
  const int32_t* t_rp;
  const int32_t* t_col;
  const int32_t* t_perm;
  float* t_val;
  double* t_val64;
  const int32_t* soc_off;
  const double* b;
  const double* c;
  double* O;
  double* chat;
  double* dsq;
  double* dinv;
  double* bs;
  double* w;
  float* s_buf[2];
  float* p;
  float* v;
  float* t;
  float* r;
  float* q;
  double* zt;
  double* x;
  double* y;
  double* z;
  double* xhat;
  double* ounit;
  double bnorm, cnorm;
  // settings
  double mu, t_cap, eps, cg_red2, cg_abs2;
  int32_t l_first, l_every, l_last, max_iter, check_every, cg_max;
  // resident state
  int32_t l;        // iterations done
  int32_t cur;      // s_buf[cur] is the current iterate
  int32_t status;   // -1 running, else ACS_SOLVED / ACS_MAX_ITER / ACS_NUMERIC
  int32_t conds;    // conditioning events run
  int32_t checked;  // iteration of the last check
  int32_t obj_stop; // a check also needs obj_stop * eps_obj <= eps (settings.obj_stop)
  long long cg_total;
  double kkt[9];    // eps_p, eps_d, eps_gap, eps_cone, kkt, pobj, dobj, alpha, eps_obj
};

// Byte offsets of one instance's arrays inside an arena (256-B aligned).
struct InstLayout {
  size_t a_rp, a_col, a_orig, t_rp, t_col, t_perm, soc_off, b, c, const_end;
  size_t a_val, a_val64, t_val, t_val64, O, chat, dsq, dinv, bs, w, s0, s1, p, v, t, r, q, zt, x, y, z, xhat, ounit;
  size_t a_blk, t_blk;  // room for the row blocks of the smallest stage
  size_t end;
};
constexpr int kBatchStageMin = 512;  // smallest stage the autotuner tries
// Lay out one instance starting at byte `base`.
InstLayout layout_instance(const Problem& p, size_t base);
// Copy the constant arrays (pattern, values, b, c, cones) into the arena.
void upload_instance_const(char* d_arena, const InstLayout& o, const Problem& p, hipStream_t st);
// Descriptor with device pointers, settings and the initial state (x = z = e_K, O = 1, w = 0);
// uploads the initial vectors.
void init_instance_state(BInst& I, char* d_arena, const InstLayout& o, const Problem& p, const acs_settings& s,
                         Sched sa, Sched st_sched, hipStream_t st);
// Lanes per row: next power of two of the mean row length, in [1, 64].
int default_lanes(double mean_row);
// Default schedules of an instance (staged, 1024-nonzero blocks).
Sched default_sched_a(const Problem& p);
Sched default_sched_t(const Problem& p);

// Launch the persistent kernel over `count` descriptors; `order` lists
// descriptor indices in the order workgroups take them; every instance runs
// until solved or until `iter_budget` more iterations (resumable).
// lds_floats: LDS (in floats) per workgroup for the CG's gathered vectors r
// and t; an instance with m + n <= lds_floats keeps them there, a larger one
// in global memory.
void launch_batch(BInst* inst, const int32_t* order, int32_t count, unsigned int* queue, int32_t grid,
                  int32_t lds_floats, int32_t iter_budget, hipStream_t st);
void launch_queue_reset(unsigned int* queue, hipStream_t st);
// Resident workgroups of the batch kernel per compute unit with that LDS.
int batch_blocks_per_cu(int32_t lds_floats);
// Most LDS floats a batch gives the gathered vectors (32 KB).
constexpr int32_t kBatchLdsMax = 8192;

}  // namespace acs
