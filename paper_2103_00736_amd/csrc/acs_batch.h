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
struct BInst {
  int32_t m, n, nnz, n_orth, n_soc;
  int32_t g_a, g_t;  // lanes per row for rows of A_s and of A_s^T (autotuned)
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
  int32_t pad;
  long long cg_total;
  double kkt[8];    // eps_p, eps_d, eps_gap, eps_cone, kkt, pobj, dobj, alpha
};

// Launch the persistent kernel over `count` descriptors; `order` lists
// descriptor indices in the order workgroups take them; every instance runs
// until solved or until `iter_budget` more iterations (resumable).
void launch_batch(BInst* inst, const int32_t* order, int32_t count, unsigned int* queue, int32_t grid,
                  int32_t block, int32_t iter_budget, hipStream_t st);
void launch_queue_reset(unsigned int* queue, hipStream_t st);
// Resident workgroups of the batch kernel per compute unit.
int batch_blocks_per_cu();

}  // namespace acs
