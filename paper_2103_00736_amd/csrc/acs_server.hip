// Serving loop: continuous batching of LP/SOCP solve requests on one GPU.
//
// Requests are admitted in arrival order while a slot is free and their
// device footprint fits the HBM budget.  Admitted requests stay resident
// (iterates, scalings, scaled matrix) until they finish:
//   - small requests (nnz <= small_nnz) live in a slot pool; one launch of the
//     persistent batch kernel per tick advances every resident small request
//     by up to `tick_iters` iterations; requests that arrive meanwhile join at
//     the next tick, finished ones leave and free their slot and memory;
//   - larger requests run the one-instance kernels on worker streams, several
//     at once, overlapping with each other and with the pool's launches.
// Results do not depend on what else is resident: the pool kernel gives each
// instance its own workgroup and fixed-order reductions, and each worker runs
// the same code path as acs_solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "acs_batch.h"
#include "acs_internal.h"

namespace acs {

#define SHIP(expr)                                                                                          \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) throw AcsError(ACS_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id = 0;
  std::shared_ptr<const Problem> p;
  acs_settings s{};
  int64_t bytes = 0;
  bool small = false;
  enum State { QUEUED, RUNNING, DONE } state = QUEUED;
  bool cancel = false;
  int error = ACS_OK;
  std::string error_msg;
  std::vector<double> x, y, z;
  acs_info info{};
  Clock::time_point t_submit, t_admit, t_done;
};

class Server {
 public:
  Server(int64_t budget, int max_slots, int64_t small_nnz, int workers, int tick_iters)
      : budget_(budget), max_slots_(max_slots), small_nnz_(small_nnz), tick_iters_(tick_iters) {
    ensure_device();
    // all request memory comes from one device pool and one pinned record pool,
    // so serving never calls hipMalloc/hipFree (which waits for the whole device)
    mem_ = std::make_unique<SubAllocator>(size_t(budget) + size_t(budget) / 8 + (size_t(64) << 20));
    status_ = std::make_unique<StatusPool>(workers + 4);
    res_.mem = mem_.get();
    res_.status = status_.get();
    SHIP(hipStreamCreateWithFlags(&pool_stream_, hipStreamNonBlocking));
    SHIP(hipMalloc(&d_inst_, sizeof(BInst) * max_slots_));
    SHIP(hipMalloc(&d_order_, sizeof(int32_t) * max_slots_));
    SHIP(hipMalloc(&d_queue_, sizeof(unsigned int)));
    pool_.resize(max_slots_);
    hipDeviceProp_t prop;
    SHIP(hipGetDeviceProperties(&prop, 0));
    grid_cap_ = prop.multiProcessorCount * batch_blocks_per_cu(0);
    for (int w = 0; w < workers; ++w) {
      hipStream_t st;
      SHIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      streams_.push_back(st);
    }
    sched_ = std::thread([this] { sched_loop(); });
    for (int w = 0; w < workers; ++w) workers_.emplace_back([this, w] { worker_loop(w); });
  }

  ~Server() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    work_cv_.notify_all();
    if (sched_.joinable()) sched_.join();
    for (auto& t : workers_)
      if (t.joinable()) t.join();
    for (auto& sl : pool_)
      if (sl.arena) mem_->release(sl.arena);
    (void)hipFree(d_inst_);
    (void)hipFree(d_order_);
    (void)hipFree(d_queue_);
    for (auto st : streams_) (void)hipStreamDestroy(st);
    (void)hipStreamDestroy(pool_stream_);
  }

  uint64_t submit(std::shared_ptr<const Problem> p, const acs_settings& s) {
    auto r = std::make_shared<Request>();
    r->t_submit = Clock::now();  // the latency includes the layout build below
    r->p = std::move(p);
    r->s = resolve_settings(s, *r->p);
    // dense requests and those asking for the direct projection or the
    // equilibration run on the worker streams
    r->small = !r->p->dense && r->s.projection == ACS_PROJ_CG && !r->s.equilibrate && r->p->nnz <= small_nnz_;
    r->bytes = r->small ? int64_t(layout_instance(*r->p, 0).end)
                        : instance_device_bytes(*r->p, r->s.precision, r->s.projection, r->s.equilibrate,
                                                r->s.a_slices);
    if (r->bytes > budget_) throw AcsError(ACS_ERR_NOMEM, "request needs more device memory than the server budget");
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stop_) throw AcsError(ACS_ERR_STATE, "server is shutting down");
      r->id = ++next_id_;
      reqs_[r->id] = r;
      queue_.push_back(r);
      ++n_queued_;
    }
    cv_.notify_all();
    return r->id;
  }

  // ACS_OK with results, ACS_PENDING, or an error; a finished ticket is released.
  int poll(uint64_t id, double* x, double* y, double* z, acs_info* info, int timeout_ms) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(id);
    if (it == reqs_.end()) throw AcsError(ACS_ERR_ARG, "unknown ticket");
    std::shared_ptr<Request> r = it->second;
    if (timeout_ms != 0) {
      auto pred = [&] { return r->state == Request::DONE; };
      if (timeout_ms < 0)
        done_cv_.wait(lk, pred);
      else
        done_cv_.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
    }
    if (r->state != Request::DONE) return ACS_PENDING;
    reqs_.erase(it);
    lk.unlock();
    if (r->error != ACS_OK) throw AcsError(r->error, r->error_msg);
    if (x && !r->x.empty()) std::memcpy(x, r->x.data(), sizeof(double) * r->x.size());
    if (y && !r->y.empty()) std::memcpy(y, r->y.data(), sizeof(double) * r->y.size());
    if (z && !r->z.empty()) std::memcpy(z, r->z.data(), sizeof(double) * r->z.size());
    if (info) *info = r->info;
    return ACS_OK;
  }

  void cancel(uint64_t id) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(id);
    if (it == reqs_.end()) throw AcsError(ACS_ERR_ARG, "unknown ticket");
    it->second->cancel = true;
    cv_.notify_all();
  }

  void stats(acs_server_counters* st) {
    std::lock_guard<std::mutex> lk(mu_);
    std::memset(st, 0, sizeof(*st));
    st->queued = n_queued_;
    st->running = slots_used_;
    st->completed = n_done_;
    st->bytes_in_use = bytes_used_;
    st->ticks = ticks_;
    st->peak_running = peak_running_;
  }

 private:
  struct Slot {
    std::shared_ptr<Request> r;
    char* arena = nullptr;
    InstLayout lay{};
    BInst host{};
    bool active = false;
  };

  void finish(const std::shared_ptr<Request>& r, bool cancelled) {
    r->t_done = Clock::now();
    r->info.queue_ms = std::chrono::duration<double, std::milli>(r->t_admit - r->t_submit).count();
    r->info.latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    if (cancelled) r->info.status = ACS_CANCELLED;
    {
      std::lock_guard<std::mutex> lk(mu_);
      r->state = Request::DONE;
      bytes_used_ -= r->bytes;
      slots_used_ -= 1;
      ++n_done_;
    }
    done_cv_.notify_all();
    cv_.notify_all();
  }

  // admission: FIFO while a slot is free and the footprint fits the budget
  void admit(std::vector<std::shared_ptr<Request>>& to_pool) {
    while (!queue_.empty()) {
      std::shared_ptr<Request> r = queue_.front();
      if (r->cancel) {
        queue_.pop_front();
        --n_queued_;
        r->state = Request::DONE;
        r->info.status = ACS_CANCELLED;
        ++n_done_;
        done_cv_.notify_all();
        continue;
      }
      if (slots_used_ >= max_slots_ || bytes_used_ + r->bytes > budget_) break;
      queue_.pop_front();
      --n_queued_;
      slots_used_ += 1;
      bytes_used_ += r->bytes;
      peak_running_ = std::max(peak_running_, slots_used_);
      r->state = Request::RUNNING;
      r->t_admit = Clock::now();
      if (r->small) {
        to_pool.push_back(r);
      } else {
        large_.push_back(r);
        work_cv_.notify_one();
      }
    }
  }

  void sched_loop() {
    (void)hipSetDevice(0);
    while (true) {
      std::vector<std::shared_ptr<Request>> to_pool;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait_for(lk, std::chrono::milliseconds(2), [&] { return stop_ || !queue_.empty() || pool_active_ > 0; });
        if (stop_) return;
        admit(to_pool);
      }
      for (auto& r : to_pool) place(r);
      if (pool_active_ > 0) tick();
    }
  }

  void place(const std::shared_ptr<Request>& r) {
    int idx = -1;
    for (int i = 0; i < max_slots_; ++i)
      if (!pool_[i].active) {
        idx = i;
        break;
      }
    Slot& sl = pool_[idx];
    try {
      sl.lay = layout_instance(*r->p, 0);
      sl.arena = static_cast<char*>(mem_->alloc(std::max<size_t>(sl.lay.end, 256)));
      if (!sl.arena) throw AcsError(ACS_ERR_NOMEM, "device pool fragmented");
      SHIP(hipMemsetAsync(sl.arena, 0, sl.lay.end, pool_stream_));
      upload_instance_const(sl.arena, sl.lay, *r->p, pool_stream_);
      const Problem& p = *r->p;
      init_instance_state(sl.host, sl.arena, sl.lay, p, r->s, default_sched_a(p), default_sched_t(p), pool_stream_);
      SHIP(hipMemcpyAsync(d_inst_ + idx, &sl.host, sizeof(BInst), hipMemcpyHostToDevice, pool_stream_));
      SHIP(hipStreamSynchronize(pool_stream_));
      sl.r = r;
      sl.active = true;
      ++pool_active_;
    } catch (const AcsError& e) {
      if (sl.arena) mem_->release(sl.arena);
      sl.arena = nullptr;
      r->error = e.code;
      r->error_msg = e.what();
      finish(r, false);
    }
  }

  void tick() {
    std::vector<int32_t> order;
    for (int i = 0; i < max_slots_; ++i)
      if (pool_[i].active) order.push_back(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return pool_[a].r->p->nnz > pool_[b].r->p->nnz; });
    SHIP(hipMemcpyAsync(d_order_, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice,
                        pool_stream_));
    const int grid = std::max(1, std::min(int(order.size()), grid_cap_));
    launch_queue_reset(d_queue_, pool_stream_);
    launch_batch(d_inst_, d_order_, int(order.size()), d_queue_, grid, 0, tick_iters_, pool_stream_);
    SHIP(hipGetLastError());
    SHIP(hipStreamSynchronize(pool_stream_));
    {
      std::lock_guard<std::mutex> lk(mu_);
      ++ticks_;
    }
    for (int idx : order) {
      Slot& sl = pool_[idx];
      BInst st;
      SHIP(hipMemcpyAsync(&st, d_inst_ + idx, sizeof(BInst), hipMemcpyDeviceToHost, pool_stream_));
      SHIP(hipStreamSynchronize(pool_stream_));
      const bool cancelled = sl.r->cancel;
      if (st.status < 0 && !cancelled) continue;
      std::shared_ptr<Request> r = sl.r;
      const Problem& p = *r->p;
      r->x.resize(p.n);
      r->z.resize(p.n);
      r->y.resize(p.m);
      {
        std::vector<double> yi(p.m);  // internal row order -> caller's
        SHIP(hipMemcpyAsync(r->x.data(), sl.host.x, sizeof(double) * p.n, hipMemcpyDeviceToHost, pool_stream_));
        SHIP(hipMemcpyAsync(r->z.data(), sl.host.z, sizeof(double) * p.n, hipMemcpyDeviceToHost, pool_stream_));
        SHIP(hipMemcpyAsync(yi.data(), sl.host.y, sizeof(double) * p.m, hipMemcpyDeviceToHost, pool_stream_));
        SHIP(hipStreamSynchronize(pool_stream_));
        for (int k = 0; k < p.m; ++k) r->y[p.row_perm[k]] = yi[k];
      }
      acs_info& in = r->info;
      std::memset(&in, 0, sizeof(in));
      in.status = st.status < 0 ? ACS_MAX_ITER : st.status;
      in.iterations = st.status == ACS_SOLVED ? st.checked : st.l;
      in.cg_steps = st.cg_total;
      in.conditionings = st.conds;
      in.eps_p = st.kkt[0];
      in.eps_d = st.kkt[1];
      in.eps_gap = st.kkt[2];
      in.eps_cone = st.kkt[3];
      in.kkt = st.kkt[4];
      in.pobj = st.kkt[5];
      in.dobj = st.kkt[6];
      in.alpha = st.kkt[7];
      in.eps_obj = st.kkt[8];
      in.solve_ms = std::chrono::duration<double, std::milli>(Clock::now() - r->t_admit).count();
      mem_->release(sl.arena);
      sl.arena = nullptr;
      sl.active = false;
      sl.r.reset();
      --pool_active_;
      finish(r, cancelled);
    }
  }

  void worker_loop(int w) {
    (void)hipSetDevice(0);
    while (true) {
      std::shared_ptr<Request> r;
      {
        std::unique_lock<std::mutex> lk(mu_);
        work_cv_.wait(lk, [&] { return stop_ || !large_.empty(); });
        if (large_.empty()) {
          if (stop_) return;
          continue;
        }
        r = large_.front();
        large_.pop_front();
      }
      try {
        if (!r->cancel) {
          SolveOut out = solve_one_instance(r->p, r->s, static_cast<void*>(streams_[w]), res_);
          r->x = std::move(out.x);
          r->y = std::move(out.y);
          r->z = std::move(out.z);
          const double q = r->info.queue_ms;
          r->info = out.info;
          r->info.queue_ms = q;
        }
      } catch (const AcsError& e) {
        r->error = e.code;
        r->error_msg = e.what();
      } catch (const std::exception& e) {
        r->error = ACS_ERR_DEVICE;
        r->error_msg = e.what();
      }
      finish(r, r->cancel);
    }
  }

  std::unique_ptr<SubAllocator> mem_;
  std::unique_ptr<StatusPool> status_;
  InstanceResources res_;
  int64_t budget_;
  int max_slots_;
  int64_t small_nnz_;
  int tick_iters_;
  int grid_cap_ = 256;
  hipStream_t pool_stream_ = nullptr;
  std::vector<hipStream_t> streams_;
  BInst* d_inst_ = nullptr;
  int32_t* d_order_ = nullptr;
  unsigned int* d_queue_ = nullptr;
  std::vector<Slot> pool_;
  int pool_active_ = 0;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_, work_cv_;
  std::deque<std::shared_ptr<Request>> queue_, large_;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> reqs_;
  uint64_t next_id_ = 0;
  int64_t bytes_used_ = 0;
  int slots_used_ = 0, peak_running_ = 0;
  int64_t n_queued_ = 0, n_done_ = 0, ticks_ = 0;
  bool stop_ = false;
  std::thread sched_;
  std::vector<std::thread> workers_;
};

}  // namespace acs

using namespace acs;

struct acs_server {
  std::unique_ptr<Server> s;
};

extern "C" {

int acs_server_create(int64_t hbm_budget, int32_t max_slots, int64_t small_nnz, int32_t workers, int32_t tick_iters,
                      acs_server** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out || hbm_budget <= 0 || max_slots < 1 || workers < 1 || workers > 8 || tick_iters < 1 || small_nnz < 0)
      throw AcsError(ACS_ERR_ARG, "bad argument");
    auto s = std::make_unique<acs_server>();
    s->s = std::make_unique<Server>(hbm_budget, max_slots, small_nnz, workers, tick_iters);
    *out = s.release();
  });
}

void acs_server_destroy(acs_server* s) { delete s; }

int acs_server_submit(acs_server* srv, const acs_problem* p, const acs_settings* s, uint64_t* ticket) {
  return guarded([&] {
    if (!srv || !p || !s || !ticket) throw AcsError(ACS_ERR_ARG, "null argument");
    *ticket = srv->s->submit(p->p, *s);
  });
}

int acs_server_poll(acs_server* srv, uint64_t ticket, double* x, double* y, double* z, acs_info* info) {
  int rc = ACS_OK;
  const int g = guarded([&] {
    if (!srv) throw AcsError(ACS_ERR_ARG, "null server");
    rc = srv->s->poll(ticket, x, y, z, info, 0);
  });
  return g != ACS_OK ? g : rc;
}

int acs_server_wait(acs_server* srv, uint64_t ticket, int32_t timeout_ms, double* x, double* y, double* z,
                    acs_info* info) {
  int rc = ACS_OK;
  const int g = guarded([&] {
    if (!srv) throw AcsError(ACS_ERR_ARG, "null server");
    rc = srv->s->poll(ticket, x, y, z, info, timeout_ms < 0 ? -1 : std::max(timeout_ms, 1));
  });
  return g != ACS_OK ? g : rc;
}

int acs_server_cancel(acs_server* srv, uint64_t ticket) {
  return guarded([&] {
    if (!srv) throw AcsError(ACS_ERR_ARG, "null server");
    srv->s->cancel(ticket);
  });
}

int acs_server_stats(acs_server* srv, acs_server_counters* st) {
  return guarded([&] {
    if (!srv || !st) throw AcsError(ACS_ERR_ARG, "null argument");
    srv->s->stats(st);
  });
}

}  // extern "C"
