// Host side of the batched solver: one device arena for all instances,
// per-instance descriptors, largest-first work order, lanes-per-row choice
// (heuristic or timed autotuning with an on-disk cache), and the persistent
// launch captured in a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>
#include <cstdlib>
#include <cstdio>

#include "acs_batch.h"
#include "acs_internal.h"

namespace acs {

#define BHIP(expr)                                                                                          \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) throw AcsError(ACS_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

static int pow2_at_least(double x, int lo, int hi) {
  int g = lo;
  while (g < hi && g < x) g <<= 1;
  return g;
}

// Size class of an instance for the lanes-per-row choice: log2 buckets of the
// mean row lengths of A and of A^T.
static int size_class(const Problem& p) {
  const double ra = double(p.nnz) / std::max(1, p.m), rt = double(p.nnz) / std::max(1, p.n);
  const int ca = std::min(7, int(std::floor(std::log2(std::max(1.0, ra)))));
  const int ct = std::min(7, int(std::floor(std::log2(std::max(1.0, rt)))));
  return ca * 8 + ct;
}


int default_lanes(double mean_row) { return pow2_at_least(mean_row, 1, 64); }
Sched default_sched_a(const Problem&) { return Sched{1, 1024}; }
Sched default_sched_t(const Problem&) { return Sched{1, 1024}; }

static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

InstLayout layout_instance(const Problem& p, size_t base) {
  InstLayout o;
  size_t off = base;
  const size_t m = p.m, n = p.n, nnz = p.nnz, units = size_t(p.n_orth) + p.soc_size.size();
  auto take = [&](size_t bytes) {
    const size_t r = off;
    off += al256(std::max<size_t>(bytes, 4));
    return r;
  };
  o.a_rp = take(4 * (m + 1));
  o.a_col = take(4 * nnz);
  o.a_orig = take(8 * nnz);
  o.t_rp = take(4 * (n + 1));
  o.t_col = take(4 * nnz);
  o.t_perm = take(4 * nnz);
  o.soc_off = take(4 * (p.soc_off.size()));
  o.b = take(8 * m);
  o.c = take(8 * n);
  o.const_end = off;
  o.a_val = take(4 * nnz);
  o.a_val64 = take(8 * nnz);
  o.t_val = take(4 * nnz);
  o.t_val64 = take(8 * nnz);
  o.O = take(8 * n);
  o.chat = take(8 * n);
  o.dsq = take(8 * m);
  o.dinv = take(8 * m);
  o.bs = take(8 * m);
  o.w = take(8 * m);
  o.s0 = take(4 * n);
  o.s1 = take(4 * n);
  o.p = take(4 * n);
  o.v = take(4 * n);
  o.t = take(4 * n);
  o.r = take(4 * m);
  o.q = take(4 * m);
  o.zt = take(8 * n);
  o.x = take(8 * n);
  o.y = take(8 * m);
  o.z = take(8 * n);
  o.xhat = take(8 * n);
  o.ounit = take(8 * units);
  const size_t nba = make_row_blocks(p.row_ptr.data(), p.m, kBatchStageMin).size();
  const size_t nbt = make_row_blocks(p.t_row_ptr.data(), p.n, kBatchStageMin).size();
  o.a_blk = take(sizeof(RowBlock) * (nba + 1));
  o.t_blk = take(sizeof(RowBlock) * (nbt + 1));
  o.end = off;
  return o;
}

void upload_instance_const(char* d_arena, const InstLayout& o, const Problem& p, hipStream_t st) {
  const size_t base = o.a_rp, len = o.const_end - o.a_rp;
  std::vector<char> stage(len, 0);
  auto put = [&](size_t at, const void* src, size_t bytes) {
    if (bytes) std::memcpy(stage.data() + (at - base), src, bytes);
  };
  put(o.a_rp, p.row_ptr.data(), 4 * p.row_ptr.size());
  put(o.a_col, p.col.data(), 4 * p.col.size());
  put(o.a_orig, p.val.data(), 8 * p.val.size());
  put(o.t_rp, p.t_row_ptr.data(), 4 * p.t_row_ptr.size());
  put(o.t_col, p.t_col.data(), 4 * p.t_col.size());
  put(o.t_perm, p.t_perm.data(), 4 * p.t_perm.size());
  put(o.soc_off, p.soc_off.data(), 4 * p.soc_off.size());
  put(o.b, p.b.data(), 8 * p.b.size());
  put(o.c, p.c.data(), 8 * p.c.size());
  BHIP(hipMemcpyAsync(d_arena + base, stage.data(), len, hipMemcpyHostToDevice, st));
  BHIP(hipStreamSynchronize(st));
}

void init_instance_state(BInst& I, char* B, const InstLayout& o, const Problem& p, const acs_settings& s, Sched sa,
                         Sched stt, hipStream_t st) {
  std::memset(&I, 0, sizeof(I));
  const int g_a = sa.staged ? 1 : sa.param, g_t = stt.staged ? 1 : stt.param;
  I.st_a = sa.staged;
  I.st_t = stt.staged;
  I.a_blk = reinterpret_cast<RowBlock*>(B + o.a_blk);
  I.t_blk = reinterpret_cast<RowBlock*>(B + o.t_blk);
  if (sa.staged) {
    const std::vector<RowBlock> bl = make_row_blocks(p.row_ptr.data(), p.m, std::max(sa.param, kBatchStageMin));
    I.a_nblk = int32_t(bl.size());
    BHIP(hipMemcpyAsync(B + o.a_blk, bl.data(), sizeof(RowBlock) * bl.size(), hipMemcpyHostToDevice, st));
    BHIP(hipStreamSynchronize(st));
  }
  if (stt.staged) {
    const std::vector<RowBlock> bl = make_row_blocks(p.t_row_ptr.data(), p.n, std::max(stt.param, kBatchStageMin));
    I.t_nblk = int32_t(bl.size());
    BHIP(hipMemcpyAsync(B + o.t_blk, bl.data(), sizeof(RowBlock) * bl.size(), hipMemcpyHostToDevice, st));
    BHIP(hipStreamSynchronize(st));
  }
  I.m = p.m;
  I.n = p.n;
  I.nnz = int32_t(p.nnz);
  I.n_orth = p.n_orth;
  I.n_soc = int32_t(p.soc_size.size());
  I.g_a = g_a;
  I.g_t = g_t;
  I.a_rp = reinterpret_cast<int32_t*>(B + o.a_rp);
  I.a_col = reinterpret_cast<int32_t*>(B + o.a_col);
  I.a_orig = reinterpret_cast<double*>(B + o.a_orig);
  I.a_val = reinterpret_cast<float*>(B + o.a_val);
  I.a_val64 = reinterpret_cast<double*>(B + o.a_val64);
  I.t_rp = reinterpret_cast<int32_t*>(B + o.t_rp);
  I.t_col = reinterpret_cast<int32_t*>(B + o.t_col);
  I.t_perm = reinterpret_cast<int32_t*>(B + o.t_perm);
  I.t_val = reinterpret_cast<float*>(B + o.t_val);
  I.t_val64 = reinterpret_cast<double*>(B + o.t_val64);
  I.soc_off = reinterpret_cast<int32_t*>(B + o.soc_off);
  I.b = reinterpret_cast<double*>(B + o.b);
  I.c = reinterpret_cast<double*>(B + o.c);
  I.O = reinterpret_cast<double*>(B + o.O);
  I.chat = reinterpret_cast<double*>(B + o.chat);
  I.dsq = reinterpret_cast<double*>(B + o.dsq);
  I.dinv = reinterpret_cast<double*>(B + o.dinv);
  I.bs = reinterpret_cast<double*>(B + o.bs);
  I.w = reinterpret_cast<double*>(B + o.w);
  I.s_buf[0] = reinterpret_cast<float*>(B + o.s0);
  I.s_buf[1] = reinterpret_cast<float*>(B + o.s1);
  I.p = reinterpret_cast<float*>(B + o.p);
  I.v = reinterpret_cast<float*>(B + o.v);
  I.t = reinterpret_cast<float*>(B + o.t);
  I.r = reinterpret_cast<float*>(B + o.r);
  I.q = reinterpret_cast<float*>(B + o.q);
  I.zt = reinterpret_cast<double*>(B + o.zt);
  I.x = reinterpret_cast<double*>(B + o.x);
  I.y = reinterpret_cast<double*>(B + o.y);
  I.z = reinterpret_cast<double*>(B + o.z);
  I.xhat = reinterpret_cast<double*>(B + o.xhat);
  I.ounit = reinterpret_cast<double*>(B + o.ounit);
  I.bnorm = p.bnorm;
  I.cnorm = p.cnorm;
  I.mu = s.mu;
  I.t_cap = s.t;
  I.eps = s.eps_kkt;
  I.cg_red2 = s.cg_reduce * s.cg_reduce;
  I.cg_abs2 = s.cg_abs * s.cg_abs;
  I.l_first = s.l_first;
  I.l_every = s.l_every;
  I.l_last = s.l_last;
  I.max_iter = s.max_iter;
  I.check_every = s.check_every;
  I.cg_max = s.cg_max;
  I.obj_stop = s.obj_stop;
  I.l = 0;
  I.cur = 0;
  I.status = -1;
  // s_buf[0] = s = (1-mu) e_K, s_buf[1] = s_prev = (1+mu) e_K, O = 1, w = 0, sqrt(D) = 1
  std::vector<float> s0(p.n, 0.f), s1(p.n, 0.f);
  for (int j = 0; j < p.n_orth; ++j) {
    s0[j] = float(1.0 - s.mu);
    s1[j] = float(1.0 + s.mu);
  }
  for (size_t c = 0; c < p.soc_size.size(); ++c) {
    s0[p.soc_off[c]] = float(1.0 - s.mu);
    s1[p.soc_off[c]] = float(1.0 + s.mu);
  }
  std::vector<double> ones_n(p.n, 1.0), ones_m(p.m, 1.0), zeros_m(p.m, 0.0);
  BHIP(hipMemcpyAsync(I.s_buf[0], s0.data(), 4 * p.n, hipMemcpyHostToDevice, st));
  BHIP(hipMemcpyAsync(I.s_buf[1], s1.data(), 4 * p.n, hipMemcpyHostToDevice, st));
  BHIP(hipMemcpyAsync(I.O, ones_n.data(), 8 * p.n, hipMemcpyHostToDevice, st));
  BHIP(hipMemcpyAsync(I.dsq, ones_m.data(), 8 * p.m, hipMemcpyHostToDevice, st));
  BHIP(hipMemcpyAsync(I.w, zeros_m.data(), 8 * p.m, hipMemcpyHostToDevice, st));
  BHIP(hipStreamSynchronize(st));
}

class Batch {
 public:
  Batch(std::vector<std::shared_ptr<const Problem>> probs, const acs_settings& s, hipStream_t stream)
      : probs_(std::move(probs)) {
    ensure_device();
    if (stream) {
      st_ = stream;
    } else {
      BHIP(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
      own_ = true;
    }
    const int count = int(probs_.size());
    settings_.resize(count);
    for (int i = 0; i < count; ++i) {
      settings_[i] = resolve_settings(s, *probs_[i]);
      settings_[i].projection = ACS_PROJ_CG;  // the kernel projects by CG (ACS_PROJ_AUTO included)
    }
    layout_and_upload();
    // default schedules: LDS-staged row blocks of 1024 nonzeros
    g_.resize(count);
    for (int i = 0; i < count; ++i) {
      g_[i].first = default_sched_a(*probs_[i]);
      g_[i].second = default_sched_t(*probs_[i]);
    }
    order_.resize(count);
    std::iota(order_.begin(), order_.end(), 0);
    std::stable_sort(order_.begin(), order_.end(), [&](int a, int b) { return probs_[a]->nnz > probs_[b]->nnz; });
    BHIP(hipMalloc(&d_order_, sizeof(int32_t) * std::max(count, 1)));
    BHIP(hipMemcpyAsync(d_order_, order_.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, st_));
    BHIP(hipStreamSynchronize(st_));
    BHIP(hipMalloc(&d_queue_, sizeof(unsigned int)));
    hipDeviceProp_t prop;
    BHIP(hipGetDeviceProperties(&prop, 0));
    cus_ = prop.multiProcessorCount;
    // LDS for the gathered CG vectors: enough for the largest instance that fits
    for (const auto& p : probs_) {
      const int64_t need = int64_t(p->m) + p->n;
      if (need <= kBatchLdsMax) lds_floats_ = std::max<int32_t>(lds_floats_, int32_t(need));
    }
    per_cu_ = batch_blocks_per_cu(lds_floats_);
    reset_all();
  }

  ~Batch() {
    if (st_) (void)hipStreamSynchronize(st_);
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    (void)hipFree(d_arena_);
    (void)hipFree(d_inst_);
    (void)hipFree(d_order_);
    (void)hipFree(d_queue_);
    if (own_) (void)hipStreamDestroy(st_);
  }

  int count() const { return int(probs_.size()); }

  // Runs every unfinished instance for up to `budget` more iterations in one
  // graph-launched persistent kernel; returns the launch's wall time in ms.
  double run(int budget, bool use_graph = true) {
    if (use_graph && (!exec_ || budget != graph_budget_)) build_graph(budget);
    hipEvent_t a, b;
    BHIP(hipEventCreate(&a));
    BHIP(hipEventCreate(&b));
    BHIP(hipEventRecord(a, st_));
    if (use_graph) {
      BHIP(hipGraphLaunch(exec_, st_));
    } else {
      const int grid = std::max(1, std::min(count(), cus_ * per_cu_));
      launch_queue_reset(d_queue_, st_);
      launch_batch(d_inst_, d_order_, count(), d_queue_, grid, lds_floats_, budget, st_);
      BHIP(hipGetLastError());
    }
    BHIP(hipEventRecord(b, st_));
    BHIP(hipEventSynchronize(b));
    float ms = 0;
    BHIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    fetch_state();
    return ms;
  }

  void result(int i, double* x, double* y, double* z, acs_info* info) {
    if (i < 0 || i >= count()) throw AcsError(ACS_ERR_ARG, "instance index out of range");
    const Problem& p = *probs_[i];
    const BInst& h = host_inst_[i];
    // every copy is ordered after the work on the batch's stream
    if (x) BHIP(hipMemcpyAsync(x, h.x, sizeof(double) * p.n, hipMemcpyDeviceToHost, st_));
    if (z) BHIP(hipMemcpyAsync(z, h.z, sizeof(double) * p.n, hipMemcpyDeviceToHost, st_));
    std::vector<double> yi(y ? p.m : 0);
    if (y) BHIP(hipMemcpyAsync(yi.data(), h.y, sizeof(double) * p.m, hipMemcpyDeviceToHost, st_));
    BHIP(hipStreamSynchronize(st_));
    if (y)  // internal row order -> caller's
      for (int k = 0; k < p.m; ++k) y[p.row_perm[k]] = yi[k];
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->status = h.status < 0 ? ACS_MAX_ITER : h.status;
      info->iterations = h.status == ACS_SOLVED ? h.checked : h.l;
      info->cg_steps = h.cg_total;
      info->conditionings = h.conds;
      info->eps_p = h.kkt[0];
      info->eps_d = h.kkt[1];
      info->eps_gap = h.kkt[2];
      info->eps_cone = h.kkt[3];
      info->kkt = h.kkt[4];
      info->pobj = h.kkt[5];
      info->dobj = h.kkt[6];
      info->alpha = h.kkt[7];
      info->eps_obj = h.kkt[8];
      info->solve_ms = last_ms_;
    }
  }

  // Resident state of instance i (tests, checkpoints): l, s_prev, s, O (n),
  // w and the row norms sqrt(D) (m, caller's row order); w is unscaled
  // (y = -w / mu), as in acs_state_get.
  void state(int i, int32_t* l, double* s_prev, double* s, double* O, double* w, double* dsq) {
    if (i < 0 || i >= count()) throw AcsError(ACS_ERR_ARG, "instance index out of range");
    const Problem& p = *probs_[i];
    const BInst& h = host_inst_[i];
    std::vector<float> sp(p.n), sc(p.n);
    std::vector<double> wi(p.m), di(p.m), ds(p.m);
    BHIP(hipMemcpyAsync(sp.data(), h.s_buf[h.cur ^ 1], sizeof(float) * p.n, hipMemcpyDeviceToHost, st_));
    BHIP(hipMemcpyAsync(sc.data(), h.s_buf[h.cur], sizeof(float) * p.n, hipMemcpyDeviceToHost, st_));
    if (O) BHIP(hipMemcpyAsync(O, h.O, sizeof(double) * p.n, hipMemcpyDeviceToHost, st_));
    BHIP(hipMemcpyAsync(wi.data(), h.w, sizeof(double) * p.m, hipMemcpyDeviceToHost, st_));
    BHIP(hipMemcpyAsync(di.data(), h.dinv, sizeof(double) * p.m, hipMemcpyDeviceToHost, st_));
    BHIP(hipMemcpyAsync(ds.data(), h.dsq, sizeof(double) * p.m, hipMemcpyDeviceToHost, st_));
    BHIP(hipStreamSynchronize(st_));
    if (l) *l = h.l;
    for (int j = 0; j < p.n; ++j) {
      if (s_prev) s_prev[j] = double(sp[j]);
      if (s) s[j] = double(sc[j]);
    }
    for (int k = 0; k < p.m; ++k) {
      if (w) w[p.row_perm[k]] = wi[k] * di[k];
      if (dsq) dsq[p.row_perm[k]] = ds[k];
    }
  }

  // Timed autotuning of the sweep schedules per size class (coordinate
  // search: rows of A_s first, then rows of A_s^T) on a sample of each class,
  // `iters` iterations per trial; results merge into the on-disk cache.
  void autotune(int sample, int iters, const char* cache_path) {
    std::map<int, std::pair<Sched, Sched>> cache = load_cache(cache_path);
    std::map<int, std::vector<int>> classes;
    for (int i = 0; i < count(); ++i) classes[size_class(*probs_[i])].push_back(i);
    for (auto& kv : classes) {
      const int cls = kv.first;
      std::vector<int>& members = kv.second;
      if (cache.find(cls) == cache.end()) {
        std::vector<int> pick;
        for (size_t k = 0; k < members.size() && int(pick.size()) < sample;
             k += std::max<size_t>(1, members.size() / sample))
          pick.push_back(members[k]);
        const Problem& p0 = *probs_[pick[0]];
        auto candidates = [&](double mean_row) {
          const int g0 = default_lanes(mean_row);
          std::vector<Sched> c = {Sched{1, 512}, Sched{1, 1024}};
          for (int g : {std::max(1, g0 / 2), g0, std::min(64, g0 * 2)}) c.push_back(Sched{0, g});
          return c;
        };
        Sched best_a = default_sched_a(p0), best_t = default_sched_t(p0);
        double best = trial(pick, best_a, best_t, iters);
        for (const Sched& ca : candidates(double(p0.nnz) / std::max(1, p0.m))) {
          const double ms = trial(pick, ca, best_t, iters);
          if (ms < best) {
            best = ms;
            best_a = ca;
          }
        }
        for (const Sched& ct : candidates(double(p0.nnz) / std::max(1, p0.n))) {
          const double ms = trial(pick, best_a, ct, iters);
          if (ms < best) {
            best = ms;
            best_t = ct;
          }
        }
        cache[cls] = {best_a, best_t};
        tuned_.push_back({cls, best_a, best_t, best});
      }
      for (int i : members) g_[i] = cache[cls];
    }
    save_cache(cache_path, cache);
    reset_all();
  }

  const std::vector<std::pair<Sched, Sched>>& lanes() const { return g_; }

 private:
  struct Tuned {
    int cls;
    Sched a, t;
    double ms;
  };

  // cache lines: "gfx950 <class> <staged_a> <param_a> <staged_t> <param_t>"
  std::map<int, std::pair<Sched, Sched>> load_cache(const char* path) {
    std::map<int, std::pair<Sched, Sched>> c;
    if (!path || !*path) return c;
    std::ifstream f(path);
    int cls, sa, pa, stt, pt;
    std::string arch;
    while (f >> arch >> cls >> sa >> pa >> stt >> pt)
      if (arch == "gfx950") c[cls] = {Sched{sa, pa}, Sched{stt, pt}};
    return c;
  }
  void save_cache(const char* path, const std::map<int, std::pair<Sched, Sched>>& c) {
    if (!path || !*path) return;
    std::ofstream f(path);
    for (auto& kv : c)
      f << "gfx950 " << kv.first << " " << kv.second.first.staged << " " << kv.second.first.param << " "
        << kv.second.second.staged << " " << kv.second.second.param << "\n";
  }

  double trial(const std::vector<int>& pick, Sched sa, Sched stt, int iters) {
    for (int i : pick) init_instance_state(host_inst_[i], d_arena_, offs_[i], *probs_[i], settings_[i], sa, stt, st_);
    std::vector<int32_t> ord(pick.begin(), pick.end());
    int32_t* d_ord = nullptr;
    BHIP(hipMalloc(&d_ord, sizeof(int32_t) * ord.size()));
    BHIP(hipMemcpyAsync(d_ord, ord.data(), sizeof(int32_t) * ord.size(), hipMemcpyHostToDevice, st_));
    upload_desc();
    const int grid = std::max(1, std::min(int(ord.size()), cus_ * per_cu_));
    hipEvent_t a, b;
    BHIP(hipEventCreate(&a));
    BHIP(hipEventCreate(&b));
    launch_queue_reset(d_queue_, st_);
    BHIP(hipEventRecord(a, st_));
    launch_batch(d_inst_, d_ord, int(ord.size()), d_queue_, grid, lds_floats_, iters, st_);
    BHIP(hipGetLastError());
    BHIP(hipEventRecord(b, st_));
    BHIP(hipStreamSynchronize(st_));
    float ms = 0;
    BHIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(d_ord);
    return ms;
  }

  // Arena layout of all instances; constant arrays are staged per instance.
  void layout_and_upload() {
    const int count = int(probs_.size());
    offs_.resize(count);
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
      offs_[i] = layout_instance(*probs_[i], off);
      off = offs_[i].end;
    }
    bytes_ = off;
    hipError_t e = hipMalloc(&d_arena_, std::max<size_t>(bytes_, 256));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw AcsError(ACS_ERR_NOMEM, "batch arena of " + std::to_string(bytes_) + " bytes does not fit");
    }
    // zero-filled on the batch's stream, so that the uploads below (same
    // stream) land after it; the null stream does not order work on a
    // non-blocking stream
    BHIP(hipMemsetAsync(d_arena_, 0, bytes_, st_));
    for (int i = 0; i < count; ++i) upload_instance_const(d_arena_, offs_[i], *probs_[i], st_);
    host_inst_.resize(count);
    BHIP(hipMalloc(&d_inst_, sizeof(BInst) * std::max(count, 1)));
  }

  void init_instance(int i) {
    init_instance_state(host_inst_[i], d_arena_, offs_[i], *probs_[i], settings_[i],
                        g_.empty() ? default_sched_a(*probs_[i]) : g_[i].first,
                        g_.empty() ? default_sched_t(*probs_[i]) : g_[i].second, st_);
  }

  void upload_desc() {
    BHIP(hipMemcpyAsync(d_inst_, host_inst_.data(), sizeof(BInst) * host_inst_.size(), hipMemcpyHostToDevice,
                        st_));
    BHIP(hipStreamSynchronize(st_));
  }

  void reset_all() {
    for (int i = 0; i < count(); ++i) init_instance(i);
    upload_desc();
    if (exec_) {
      (void)hipGraphExecDestroy(exec_);
      exec_ = nullptr;
    }
    if (graph_) {
      (void)hipGraphDestroy(graph_);
      graph_ = nullptr;
    }
  }

  void fetch_state() {
    std::vector<BInst> tmp(host_inst_.size());
    BHIP(hipMemcpyAsync(tmp.data(), d_inst_, sizeof(BInst) * tmp.size(), hipMemcpyDeviceToHost, st_));
    BHIP(hipStreamSynchronize(st_));
    for (size_t i = 0; i < tmp.size(); ++i) {
      BInst& h = host_inst_[i];
      h.l = tmp[i].l;
      h.cur = tmp[i].cur;
      h.status = tmp[i].status;
      h.conds = tmp[i].conds;
      h.checked = tmp[i].checked;
      h.cg_total = tmp[i].cg_total;
      for (int k = 0; k < 9; ++k) h.kkt[k] = tmp[i].kkt[k];
    }
  }

  // queue reset (a fill kernel, no memset node) + persistent kernel, captured once
  void build_graph(int budget) {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    exec_ = nullptr;
    graph_ = nullptr;
    const int grid = std::max(1, std::min(count(), cus_ * per_cu_));
    BHIP(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
    launch_queue_reset(d_queue_, st_);
    launch_batch(d_inst_, d_order_, count(), d_queue_, grid, lds_floats_, budget, st_);
    BHIP(hipStreamEndCapture(st_, &graph_));
    BHIP(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
    graph_budget_ = budget;
  }

  std::vector<std::shared_ptr<const Problem>> probs_;
  std::vector<acs_settings> settings_;
  std::vector<InstLayout> offs_;
  std::vector<BInst> host_inst_;
  std::vector<std::pair<Sched, Sched>> g_;
  std::vector<int32_t> order_;
  std::vector<Tuned> tuned_;
  hipStream_t st_ = nullptr;
  bool own_ = false;
  char* d_arena_ = nullptr;
  size_t bytes_ = 0;
  BInst* d_inst_ = nullptr;
  int32_t* d_order_ = nullptr;
  unsigned int* d_queue_ = nullptr;
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t exec_ = nullptr;
  int graph_budget_ = -1;
  int cus_ = 256, per_cu_ = 1;
  int32_t lds_floats_ = 0;

 public:
  double last_ms_ = 0;
};

}  // namespace acs

using namespace acs;

struct acs_batch {
  std::unique_ptr<Batch> b;
};

extern "C" {

int64_t acs_batch_device_bytes(const acs_problem* p) {
  if (!p || p->p->dense) return -1;
  return int64_t(layout_instance(*p->p, 0).end);
}

int acs_batch_create(int32_t count, const acs_problem* const* probs, const acs_settings* s, void* stream,
                     acs_batch** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (count < 1 || !probs || !s || !out) throw AcsError(ACS_ERR_ARG, "bad argument");
    if (s->projection != ACS_PROJ_CG && s->projection != ACS_PROJ_AUTO)
      throw AcsError(ACS_ERR_ARG, "the batch kernel projects by CG only");
    if (s->equilibrate) throw AcsError(ACS_ERR_ARG, "the batch kernel does not equilibrate (acs_solve does)");
    std::vector<std::shared_ptr<const Problem>> v;
    v.reserve(count);
    for (int i = 0; i < count; ++i) {
      if (!probs[i]) throw AcsError(ACS_ERR_ARG, "null problem in batch");
      if (probs[i]->p->dense) throw AcsError(ACS_ERR_ARG, "dense problems are solved one at a time (acs_solve)");
      v.push_back(probs[i]->p);
    }
    auto b = std::make_unique<acs_batch>();
    b->b = std::make_unique<Batch>(std::move(v), *s, static_cast<hipStream_t>(stream));
    *out = b.release();
  });
}

void acs_batch_destroy(acs_batch* b) { delete b; }

int acs_batch_autotune(acs_batch* b, int32_t sample, int32_t iters, const char* cache_path) {
  return guarded([&] {
    if (!b || sample < 1 || iters < 1) throw AcsError(ACS_ERR_ARG, "bad argument");
    b->b->autotune(sample, iters, cache_path);
  });
}

int acs_batch_run(acs_batch* b, int32_t iter_budget, int32_t use_graph, double* ms) {
  return guarded([&] {
    if (!b || iter_budget < 1) throw AcsError(ACS_ERR_ARG, "bad argument");
    const double t = b->b->run(iter_budget, use_graph != 0);
    b->b->last_ms_ = t;
    if (ms) *ms = t;
  });
}

int acs_batch_result(acs_batch* b, int32_t i, double* x, double* y, double* z, acs_info* info) {
  return guarded([&] {
    if (!b) throw AcsError(ACS_ERR_ARG, "null batch");
    b->b->result(i, x, y, z, info);
  });
}

int acs_batch_state_get(acs_batch* b, int32_t i, int32_t* l, double* s_prev, double* s, double* O, double* w,
                        double* dsq) {
  return guarded([&] {
    if (!b) throw AcsError(ACS_ERR_ARG, "null batch");
    b->b->state(i, l, s_prev, s, O, w, dsq);
  });
}

int acs_batch_lanes(acs_batch* b, int32_t i, int32_t* g_a, int32_t* g_t) {
  return guarded([&] {
    if (!b || i < 0 || i >= b->b->count()) throw AcsError(ACS_ERR_ARG, "bad argument");
    const auto& g = b->b->lanes()[i];
    // staged schedules are reported as the negated stage size
    if (g_a) *g_a = g.first.staged ? -g.first.param : g.first.param;
    if (g_t) *g_t = g.second.staged ? -g.second.param : g.second.param;
  });
}

int acs_batch_solve(int32_t count, const acs_problem* const* probs, const acs_settings* s, double* const* x,
                    double* const* y, double* const* z, acs_info* infos, void* stream) {
  return guarded([&] {
    if (count < 1 || !probs || !s) throw AcsError(ACS_ERR_ARG, "bad argument");
    if (s->projection != ACS_PROJ_CG && s->projection != ACS_PROJ_AUTO)
      throw AcsError(ACS_ERR_ARG, "the batch kernel projects by CG only");
    if (s->equilibrate) throw AcsError(ACS_ERR_ARG, "the batch kernel does not equilibrate (acs_solve does)");
    std::vector<std::shared_ptr<const Problem>> v;
    for (int i = 0; i < count; ++i) {
      if (!probs[i]) throw AcsError(ACS_ERR_ARG, "null problem in batch");
      if (probs[i]->p->dense) throw AcsError(ACS_ERR_ARG, "dense problems are solved one at a time (acs_solve)");
      v.push_back(probs[i]->p);
    }
    Batch b(std::move(v), *s, static_cast<hipStream_t>(stream));
    int budget = 0;
    for (int i = 0; i < count; ++i) budget = std::max(budget, s->max_iter);
    b.last_ms_ = b.run(std::max(budget, 1));
    for (int i = 0; i < count; ++i)
      b.result(i, x ? x[i] : nullptr, y ? y[i] : nullptr, z ? z[i] : nullptr, infos ? &infos[i] : nullptr);
  });
}

}  // extern "C"
