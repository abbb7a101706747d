// Solver core (host side of one Algorithm-2 instance) and the C ABI.
//
// The host drives the iteration as a sequence of kernel launches on one
// stream.  Data-dependent control (how many CG steps an outer iteration
// needs, whether a KKT check passed) is read back without stalling the
// stream: the last workgroup of the relevant kernel writes a progress record
// into pinned, device-mapped host memory; the host polls it and keeps at
// most one chunk of CG launches in flight beyond what it has seen finish.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "acs_internal.h"
#include "acs_kernels.h"

namespace acs {

// ----------------------------------------------------------------------------
// errors
// ----------------------------------------------------------------------------
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

#define HIP_CHECK(expr)                                                                                     \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess)                                                                                   \
      throw AcsError(ACS_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));                    \
  } while (0)

static void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw AcsError(ACS_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}

// ----------------------------------------------------------------------------
// conditioning schedule L (Alg. 2 step 4: l in L u {1})
// ----------------------------------------------------------------------------
struct Schedule {
  int first = 300, every = 100, last = -1;
  bool contains(int l) const {
    if (l == 1) return true;
    if (first <= 0 || l < first) return false;
    if (last >= 0 && l > last) return false;
    if (every <= 0) return l == first;
    return (l - first) % every == 0;
  }
};

acs_settings resolve_settings(const acs_settings& in, const Problem& p) {
  acs_settings s = in;
  if (s.auto_params) {
    if (p.is_socp()) {
      s.t = 1.7;
      s.l_first = 200;
    } else {
      s.t = 9.2;
      s.l_first = 300;
    }
    s.l_every = 100;
    s.l_last = -1;
  }
  // cg_reduce = 0 picks the per-class reduction: measured whole solves of the
  // SOCPs run fastest near 0.2, the row-scaled LPs need 0.1 or tighter
  if (s.cg_reduce == 0.0) s.cg_reduce = p.is_socp() ? kCgReduceSocp : kCgReduceLp;
  if (!(s.cg_reduce > 0)) throw AcsError(ACS_ERR_ARG, "settings: cg_reduce must be >= 0 (0 = per class)");
  if (!(s.mu > 0) || !(s.t > 0)) throw AcsError(ACS_ERR_ARG, "settings: mu and t must be > 0");
  if (s.max_iter < 0 || s.check_every < 1 || s.cg_max < 0 || s.obj_stop < 0)
    throw AcsError(ACS_ERR_ARG, "settings: bad counts");
  if (s.precision != ACS_PREC_MIXED && s.precision != ACS_PREC_FP64) throw AcsError(ACS_ERR_ARG, "settings: precision");
  if (s.projection == ACS_PROJ_AUTO) s.projection = p.m <= kAutoFactorMaxM ? ACS_PROJ_FACTOR : ACS_PROJ_CG;
  if (s.projection != ACS_PROJ_CG && s.projection != ACS_PROJ_FACTOR) throw AcsError(ACS_ERR_ARG, "settings: projection");
  if ((s.equilibrate != 0 && s.equilibrate != 1) || s.eq_sweeps < 0)
    throw AcsError(ACS_ERR_ARG, "settings: equilibrate must be 0 or 1 and eq_sweeps >= 0");
  if (s.equilibrate && p.dense) throw AcsError(ACS_ERR_ARG, "settings: equilibration takes sparse problems only");
  if (s.a_slices != 0 && s.a_slices != 1 && s.a_slices != kSlices)
    throw AcsError(ACS_ERR_ARG, "settings: a_slices must be 0, 1 or 8");
  if (!p.dense) s.a_slices = p.a_slices(s.a_slices);
  return s;
}

// ----------------------------------------------------------------------------
// device memory
// ----------------------------------------------------------------------------
struct SubAllocator::Impl {
  std::mutex mu;
  std::map<size_t, size_t> free_by_off;  // offset -> size
  std::map<size_t, size_t> used;         // offset -> size
};

SubAllocator::SubAllocator(size_t bytes) : impl_(new Impl) {
  size_ = (bytes + 255) & ~size_t(255);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&base_), size_);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete impl_;
    impl_ = nullptr;
    throw AcsError(ACS_ERR_NOMEM, "device pool of " + std::to_string(size_) + " bytes does not fit");
  }
  impl_->free_by_off[0] = size_;
}

SubAllocator::SubAllocator(void* base, size_t bytes)
    : impl_(new Impl), base_(static_cast<char*>(base)), size_(bytes & ~size_t(255)), own_(false) {
  impl_->free_by_off[0] = size_;
}

SubAllocator::~SubAllocator() {
  if (base_ && own_) (void)hipFree(base_);
  delete impl_;
}

void* SubAllocator::alloc(size_t bytes) {
  bytes = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
  std::lock_guard<std::mutex> lk(impl_->mu);
  for (auto it = impl_->free_by_off.begin(); it != impl_->free_by_off.end(); ++it) {
    if (it->second < bytes) continue;
    const size_t off = it->first, sz = it->second;
    impl_->free_by_off.erase(it);
    if (sz > bytes) impl_->free_by_off[off + bytes] = sz - bytes;
    impl_->used[off] = bytes;
    return base_ + off;
  }
  return nullptr;
}

void SubAllocator::release(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(impl_->mu);
  const size_t off = size_t(static_cast<char*>(p) - base_);
  auto u = impl_->used.find(off);
  if (u == impl_->used.end()) return;
  size_t start = off, sz = u->second;
  impl_->used.erase(u);
  auto next = impl_->free_by_off.lower_bound(start);
  if (next != impl_->free_by_off.end() && next->first == start + sz) {  // merge with the following range
    sz += next->second;
    impl_->free_by_off.erase(next);
  }
  auto it = impl_->free_by_off.lower_bound(start);
  if (it != impl_->free_by_off.begin()) {  // merge with the preceding range
    auto prev = std::prev(it);
    if (prev->first + prev->second == start) {
      start = prev->first;
      sz += prev->second;
      impl_->free_by_off.erase(prev);
    }
  }
  impl_->free_by_off[start] = sz;
}

struct StatusPool::Impl {
  std::mutex mu;
  HostStatus* base = nullptr;
  std::vector<HostStatus*> free_list;
};

StatusPool::StatusPool(int count) : impl_(new Impl) {
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&impl_->base), sizeof(HostStatus) * std::max(count, 1),
                               hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete impl_;
    impl_ = nullptr;
    throw AcsError(ACS_ERR_NOMEM, "pinned status records");
  }
  for (int i = count - 1; i >= 0; --i) impl_->free_list.push_back(impl_->base + i);
}

StatusPool::~StatusPool() {
  if (impl_ && impl_->base) (void)hipHostFree(impl_->base);
  delete impl_;
}

HostStatus* StatusPool::take() {
  std::lock_guard<std::mutex> lk(impl_->mu);
  if (impl_->free_list.empty()) return nullptr;
  HostStatus* h = impl_->free_list.back();
  impl_->free_list.pop_back();
  return h;
}

void StatusPool::give(HostStatus* h) {
  std::lock_guard<std::mutex> lk(impl_->mu);
  impl_->free_list.push_back(h);
}

class DeviceArena {
 public:
  explicit DeviceArena(SubAllocator* sa = nullptr) : sa_(sa) {}
  ~DeviceArena() { release(); }
  template <typename T>
  T* alloc(size_t count) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (sa_) {
      p = sa_->alloc(bytes);
      if (!p) throw AcsError(ACS_ERR_NOMEM, "device pool exhausted (" + std::to_string(bytes) + " bytes)");
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw AcsError(ACS_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
      }
    }
    ptrs_.push_back(p);
    bytes_ += bytes;
    return static_cast<T*>(p);
  }
  void release() {
    for (void* p : ptrs_) {
      if (sa_)
        sa_->release(p);
      else
        (void)hipFree(p);
    }
    ptrs_.clear();
    bytes_ = 0;
  }
  size_t bytes() const { return bytes_; }

 private:
  SubAllocator* sa_;
  std::vector<void*> ptrs_;
  size_t bytes_ = 0;
};

// rows per chunk of the dense column products: enough workgroups (strips x
// chunks) to fill the chip, at least 16 rows per chunk
static void dense_chunks(const Problem& p, int32_t* rows, int32_t* chunks) {
  const int64_t strips = (int64_t(p.ld) + 1023) / 1024;
  const int64_t want = std::max<int64_t>(1, 4096 / strips);
  int64_t r = std::max<int64_t>(16, (int64_t(p.m) + want - 1) / want);
  *rows = int32_t(r);
  *chunks = int32_t((int64_t(p.m) + r - 1) / r);
}

// Direct projection sizes: padded order of M and leading dimension of B
static void factor_shape(const Problem& p, int32_t* mp, int32_t* ldb) {
  *mp = int32_t((int64_t(p.m) + kFacPad - 1) / kFacPad * kFacPad);
  *ldb = p.dense ? p.ld : int32_t((int64_t(p.n) + 63) / 64 * 64);
}

static int64_t factor_bytes(const Problem& p) {
  int32_t mp, ldb;
  factor_shape(p, &mp, &ldb);
  const int64_t orders = 4 * int64_t(fac_tile_order(mp / 128).size() + fac_tile_order((p.m + kFacTile - 1) / kFacTile).size());
  return 8 * (int64_t(mp) * mp + int64_t(mp) * ldb + kFacSlots * int64_t(mp) * kFacTile + kFacTile * kFacTile + mp) +
         orders +
         7 * 256;
}

static void check_factor_fits(const Problem& p) {
  int32_t mp, ldb;
  factor_shape(p, &mp, &ldb);
  if (int64_t(p.m) > kFacMaxOrder || mp > kFacMaxOrder)
    throw AcsError(ACS_ERR_ARG, "direct projection: m = " + std::to_string(p.m) + " exceeds " +
                                    std::to_string(kFacMaxOrder));
  if (int64_t(mp) * ldb > (int64_t(1) << 31))
    throw AcsError(ACS_ERR_ARG, "direct projection: the dense copy of A (m x n) exceeds 2^31 entries");
}

static int64_t estimate_bytes(const Problem& p, int precision, int a_slices) {
  const int64_t vt = precision == ACS_PREC_FP64 ? 8 : 4;
  const int64_t nnz = p.nnz, m = p.m, n = p.n;
  if (p.dense) {
    int32_t rows, chunks;
    dense_chunks(p, &rows, &chunks);
    int64_t b = 4 * int64_t(p.dhi.size()) + 4 * int64_t(p.dlo.size()) + 8 * int64_t(chunks) * p.ld;
    b += (vt + 8) * p.ld + n * (3 * vt + 8 * 10) + m * (3 * vt + 8 * 7 + 4 + vt);
    b += 8 * kMaxSums * (m / 16 + n / kBlock + 4) + 8 * kBlock + 64 * 256;
    return b;
  }
  const int slices = p.a_slices(a_slices);
  const SellPair& sp = p.sell(slices);
  int64_t b = 0;
  b += 4 * (m + 1) + 4 * nnz + 8 * nnz + 8 * nnz;        // A pattern, original and FP64 scaled values
  const int64_t v64 = vt == 8 ? 0 : 8;                   // FP64 SELL values beside the VT ones
  for (const Sell* S : {&sp.a, &sp.t, &sp.t_cg}) {       // SELL layouts: entries, tasks, chunk rows
    const int64_t per = S == &sp.t_cg ? 8 + vt : 8 + vt + v64;  // the CG's A^T: VT values only
    b += per * int64_t(S->col.size()) + 12 * int64_t(S->wt_ptr.size() + S->long_row.size()) +
         4 * int64_t(S->chunk_row.size());
  }
  b += 4 * int64_t(sp.a_cg_col.size());                  // the CG's column numbers of the A layout
  // (the CG's own layouts are empty with one slice)
  b += (vt + 8) * slices * m + (4 + vt) * m;             // slice partials, row permutation, scratch
  b += 8 * int64_t(std::max(sp.t.wg_max, sp.t_cg.wg_max)) + 256;  // ||t||^2 partials of the one-slice CG
  b += 8 * int64_t(p.a_blocks.size());
  b += n * (3 * vt + 8 * 10) + m * (3 * vt + 8 * 7);
  const size_t parts = std::max<size_t>({p.a_blocks.size(), p.t_blocks.size(), size_t(sp.t.wg_max),
                                         size_t(sp.t_cg.wg_max), size_t(sp.a.wg_max),
                                         size_t(n / kBlock + 2)});
  b += 8 * kMaxSums * int64_t(parts) + 8 * kBlock + 96 * 256;  // partials, per-array alignment
  return b;
}

// ----------------------------------------------------------------------------
// one instance
// ----------------------------------------------------------------------------
class InstanceBase {
 public:
  virtual ~InstanceBase() = default;
  virtual void set_state(int l, const double* s_prev, const double* s, const double* O, const double* w) = 0;
  virtual void run(int iters, bool stop_on_converge) = 0;
  virtual void get(int* l, double* s_prev, double* s, double* O, double* w, double* x, double* y, double* z) = 0;
  virtual void get_device(double* x, double* y, double* z) = 0;
  virtual void spmv(int which, const void* x, void* y, int reps, double* avg_ms) = 0;
  virtual void check_now() = 0;
  virtual void profile(uint32_t mask) = 0;
  virtual void timing(int cls, int64_t* count, double* total_ms) = 0;
  virtual int current_l() const = 0;
  virtual void normal_inverse(double* out) = 0;
  acs_info info{};
  acs_settings S{};
};

enum KClass {
  KC_UPDATE = 0, KC_RESID = 1, KC_CG_T = 2, KC_CG_A = 3, KC_CONE = 4, KC_CHECK = 5, KC_COND = 6, KC_FIN = 7,
  KC_CG_COMB = 8, KC_FAC_SYRK = 9, KC_FAC_UPDATE = 10, KC_FAC_APPLY = 11, KC_FAC_PANEL = 12, KC_N = 13
};

template <typename VT>
class Instance final : public InstanceBase {
 public:
  Instance(std::shared_ptr<const Problem> prob, const acs_settings& settings, hipStream_t stream,
           const InstanceResources& res = InstanceResources())
      : P_(std::move(prob)), res_(res), arena_(res.mem) {
    const auto t0 = std::chrono::steady_clock::now();
    S = resolve_settings(settings, *P_);
    sched_.first = S.l_first;
    sched_.every = S.l_every;
    sched_.last = S.l_last;
    if (stream) {
      st_ = stream;
    } else {
      HIP_CHECK(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
      own_stream_ = true;
    }
    // a constructor that throws (e.g. ACS_ERR_NOMEM from the arena or the
    // server's pools) runs no destructor: release what was taken so far
    try {
      setup_device();
      if (S.equilibrate) equilibrate();
      set_initial();
      HIP_CHECK(hipStreamSynchronize(st_));
    } catch (...) {
      release();
      throw;
    }
    info.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }

  ~Instance() override { release(); }

  // streams, events, device memory and the status record; idempotent
  void release() {
    if (st_) (void)hipStreamSynchronize(st_);
    if (st2_) {
      (void)hipStreamSynchronize(st2_);
      (void)hipStreamDestroy(st2_);
      st2_ = nullptr;
    }
    if (fork_) (void)hipEventDestroy(fork_);
    if (join_) (void)hipEventDestroy(join_);
    fork_ = join_ = nullptr;
    for (auto* v : {&prof_pending_, &prof_free_}) {
      for (auto& e : *v) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
      }
      v->clear();
    }
    arena_.release();
    if (hs_) {
      if (res_.status)
        res_.status->give(hs_);
      else
        (void)hipHostFree(hs_);
      hs_ = nullptr;
    }
    if (own_stream_ && st_) (void)hipStreamDestroy(st_);
    st_ = nullptr;
    own_stream_ = false;
  }

  // -------------------------------------------------------------- setup
  // CSR of A (conditioning and check sweeps) and the SELL layouts of the products
  template <class Up>
  void setup_sparse(Up& up) {
    const Problem& p = *P_;
    Dev<VT>& d = d_;
    int32_t* a_rp = arena_.alloc<int32_t>(p.m + 1);
    int32_t* a_col = arena_.alloc<int32_t>(p.nnz);
    double* a_orig = arena_.alloc<double>(p.nnz);
    RowBlock* a_blk = arena_.alloc<RowBlock>(p.a_blocks.size());
    up(a_rp, p.row_ptr);
    if (p.nnz) {
      up(a_col, p.col);
      up(a_orig, p.val);
    }
    up(a_blk, p.a_blocks);
    d.a_rp = a_rp;
    d.a_col = a_col;
    d.a_orig = a_orig;
    d.a_val64 = arena_.alloc<double>(p.nnz);
    d.a_blk = a_blk;
    d.a_nblk = int(p.a_blocks.size());
    d.a_rp_nnz = int32_t(p.nnz);
    {
      const SellPair& sp = p.sell(S.a_slices);
      auto sell_dev = [&](const Sell& S, SellDev* D) {
        auto put = [&](const std::vector<int32_t>& v) -> const int32_t* {
          int32_t* ptr = arena_.alloc<int32_t>(std::max<size_t>(v.size(), 1));
          if (!v.empty()) up(ptr, v);
          return ptr;
        };
        std::memset(D, 0, sizeof(*D));
        D->long_row = put(S.long_row);
        D->long_beg = put(S.long_beg);
        D->long_end = put(S.long_end);
        D->wt_ptr = put(S.wt_ptr);
        D->wt_len = put(S.wt_len);
        D->wt_row = put(S.wt_row);
        D->chunk_row = put(S.chunk_row);
        D->col = put(S.col);
        D->src = put(S.src);
        D->entries = int64_t(S.col.size());
        D->slices = S.slices;
        for (int x = 0; x <= S.slices; ++x) {
          D->long_off[x] = S.long_off[x];
          D->wt_off[x] = S.wt_off[x];
        }
        for (int x = 0; x < S.slices; ++x) D->wg[x] = S.wg[x];
        D->wg_max = S.wg_max;
      };
      sell_dev(sp.a, &d.sa);
      sell_dev(sp.t, &d.st);
      d.sa_val = arena_.alloc<VT>(std::max<size_t>(sp.a.col.size(), 1));
      d.st_val = arena_.alloc<VT>(std::max<size_t>(sp.t.col.size(), 1));
      if (sizeof(VT) == sizeof(double)) {
        d.sa_val64 = reinterpret_cast<double*>(d.sa_val);
        d.st_val64 = reinterpret_cast<double*>(d.st_val);
      } else {
        d.sa_val64 = arena_.alloc<double>(std::max<size_t>(sp.a.col.size(), 1));
        d.st_val64 = arena_.alloc<double>(std::max<size_t>(sp.t.col.size(), 1));
      }
      // the CG's layouts (after the value arrays: with one slice they alias them)
      d.sa_cg = d.sa;
      if (sp.cg_own) {  // renumbered columns
        sell_dev(sp.t_cg, &d.st_cg);
        int32_t* c = arena_.alloc<int32_t>(std::max<size_t>(sp.a_cg_col.size(), 1));
        if (!sp.a_cg_col.empty()) up(c, sp.a_cg_col);
        d.sa_cg.col = c;
        d.st_cg_val = arena_.alloc<VT>(std::max<size_t>(sp.t_cg.col.size(), 1));
      } else {
        d.st_cg = d.st;
        d.st_cg_val = d.st_val;
      }
      if (!d.sa_val || !d.st_val || !d.st_cg_val || !d.sa_cg.col || !d.st_cg.col)
        throw AcsError(ACS_ERR_DEVICE, "internal error: a SELL array of the CG is unset");
      d.part = arena_.alloc<VT>(size_t(S.a_slices) * p.m);
      d.part64 = arena_.alloc<double>(size_t(S.a_slices) * p.m);
      // ||t||^2 partials of k_cg_t, read by the one-slice second half
      d.partials2 = arena_.alloc<double>(std::max<size_t>(size_t(d.st_cg.wg_max), 1));
    }
  }

  // dense A: FP32 values (+ low part), chunk partials, padded product inputs
  template <class Up>
  void setup_dense(Up& up) {
    const Problem& p = *P_;
    Dev<VT>& d = d_;
    d.dense = 1;
    d.ld = p.ld;
    float* hi = arena_.alloc<float>(p.dhi.size());
    up(hi, p.dhi);
    d.dhi = hi;
    if (!p.dlo.empty()) {
      float* lo = arena_.alloc<float>(p.dlo.size());
      up(lo, p.dlo);
      d.dlo = lo;
    }
    dense_chunks(p, &d.dchunk, &d.dnchunk);
    d.dpart = arena_.alloc<double>(size_t(d.dnchunk) * p.ld);
    d.dx32 = arena_.alloc<VT>(p.ld);
    d.dx64 = arena_.alloc<double>(p.ld);
    d.partials2 = arena_.alloc<double>(size_t(p.n) / kBlock + 2);
    // padding columns of the product inputs stay zero
    HIP_CHECK(hipMemsetAsync(d.dx32, 0, sizeof(VT) * p.ld, st_));
    HIP_CHECK(hipMemsetAsync(d.dx64, 0, sizeof(double) * p.ld, st_));
  }

  // direct projection: M (mp x mp), the FP64 copy of A_s, the sweep panels
  void setup_factor() {
    const Problem& p = *P_;
    check_factor_fits(p);
    fac_ = true;
    FacDev& f = f_;
    f.m = p.m;
    factor_shape(p, &f.mp, &f.ldb);
    f.nb = (p.m + kFacTile - 1) / kFacTile;
    f.S = arena_.alloc<double>(size_t(f.mp) * f.mp);
    f.B = arena_.alloc<double>(size_t(f.mp) * f.ldb);
    f.C = arena_.alloc<double>(size_t(kFacSlots) * f.mp * kFacTile);
    f.P = arena_.alloc<double>(kFacTile * kFacTile);
    {
      const std::vector<int32_t> so = fac_tile_order(f.mp / 128), uo = fac_tile_order(f.nb);
      int32_t* a = arena_.alloc<int32_t>(so.size());
      int32_t* b = arena_.alloc<int32_t>(uo.size());
      HIP_CHECK(hipMemcpyAsync(a, so.data(), 4 * so.size(), hipMemcpyHostToDevice, st_));
      HIP_CHECK(hipMemcpyAsync(b, uo.data(), 4 * uo.size(), hipMemcpyHostToDevice, st_));
      HIP_CHECK(hipStreamSynchronize(st_));
      f.syrk_order = a;
      f.upd_order = b;
      f.syrk_blocks = int32_t(so.size());
      f.upd_blocks = int32_t(uo.size());
    }
    d_.r64 = arena_.alloc<double>(f.mp);
    // entries of the residual beyond m stay zero
    HIP_CHECK(hipMemsetAsync(d_.r64, 0, sizeof(double) * f.mp, st_));
    // the next group's pivots, panels and strips run on a second stream
    // (default priority) alongside the current group's pass; created after
    // the allocations, so that a failed allocation does not leave them behind
    HIP_CHECK(hipStreamCreateWithFlags(&st2_, hipStreamNonBlocking));
    HIP_CHECK(hipEventCreateWithFlags(&fork_, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&join_, hipEventDisableTiming));
  }

  // M = A_s A_s^T of the current scaling and its inverse
  void factorize() {
    timed(KC_COND, [&] { launch_fac_copy(d_, f_, st_); });
    timed(KC_FAC_SYRK, [&] { launch_fac_syrk(f_, st_); });
    // Steps in groups of kFacGroup: one pass over S per group (each strip
    // brings the next block of the group up to date before its pivot).  The
    // pass first updates the next group's block rows and columns; the next
    // group's chain of pivots, panels and strips (latency-bound, a few
    // workgroups) then runs on the second stream while the rest of the pass
    // runs here.  They touch disjoint tiles and W slots; the next pass waits
    // for the chain.  The chain's launches are not part of the pass's timing.
    const int nb = f_.nb;
    auto chain = [&](int K0, hipStream_t s) {
      const int cnt = std::min(kFacGroup, nb - K0);
      for (int g = 0; g < cnt; ++g) {
        launch_fac_pivot_panel(f_, K0 + g, K0, s);
        if (g + 1 < cnt) launch_fac_strip(f_, K0, g + 1, s);
      }
    };
    timed(KC_FAC_PANEL, [&] { chain(0, st_); });
    for (int K0 = 0; K0 < nb; K0 += kFacGroup) {
      const int cnt = std::min(kFacGroup, nb - K0), nxt = K0 + kFacGroup;
      if (nxt >= nb) {
        timed(KC_FAC_UPDATE, [&] { launch_fac_pass(f_, K0, cnt, st_); });
        continue;
      }
      const int cntn = std::min(kFacGroup, nb - nxt);
      timed(KC_FAC_UPDATE, [&] {
        launch_fac_pass_next(f_, K0, cnt, nxt, cntn, st_);
        HIP_CHECK(hipEventRecord(fork_, st_));
        HIP_CHECK(hipStreamWaitEvent(st2_, fork_, 0));
        {
          LaunchEvents* timing = launch_events();
          launch_events() = nullptr;
          chain(nxt, st2_);
          launch_events() = timing;
        }
        HIP_CHECK(hipEventRecord(join_, st2_));
        launch_fac_pass_rest(f_, K0, cnt, nxt, cntn, st_);
      });
      HIP_CHECK(hipStreamWaitEvent(st_, join_, 0));
    }
    timed(KC_FAC_PANEL, [&] { launch_fac_mirror(f_, st_); });
    factored_ = true;
  }

  void setup_device() {
    const Problem& p = *P_;
    Dev<VT>& d = d_;
    std::memset(&d, 0, sizeof(d));
    d.m = p.m;
    d.n = p.n;
    d.n_orth = p.n_orth;
    d.n_soc = int(p.soc_size.size());
    d.mu = S.mu;
    auto up = [&](auto* dst, const auto& vec) {
      HIP_CHECK(hipMemcpyAsync(dst, vec.data(), vec.size() * sizeof(vec[0]), hipMemcpyHostToDevice, st_));
    };
    int32_t* soc_off = arena_.alloc<int32_t>(p.soc_off.size());
    double* b = arena_.alloc<double>(p.m);
    double* c = arena_.alloc<double>(p.n);
    up(soc_off, p.soc_off);
    up(b, p.b);
    up(c, p.c);
    {
      int32_t* rperm = arena_.alloc<int32_t>(p.m);
      up(rperm, p.row_perm);
      d.row_perm = rperm;
      d.mtmp = arena_.alloc<VT>(p.m);
    }
    if (p.dense)
      setup_dense(up);
    else
      setup_sparse(up);
    if (S.projection == ACS_PROJ_FACTOR) setup_factor();
    d.soc_off = soc_off;
    d.b = b;
    d.c = c;
    d.O = arena_.alloc<double>(p.n);
    d.chat = arena_.alloc<double>(p.n);
    d.dsq = arena_.alloc<double>(p.m);
    d.dinv = arena_.alloc<double>(p.m);
    d.bs = arena_.alloc<double>(p.m);
    d.p = arena_.alloc<VT>(p.n);
    d.v = arena_.alloc<VT>(p.n);
    d.zt = arena_.alloc<double>(p.n);
    d.w = arena_.alloc<double>(p.m);
    d.r = arena_.alloc<VT>(p.m);
    d.q = arena_.alloc<VT>(p.m);
    d.t = arena_.alloc<VT>(p.n);
    d.xout = arena_.alloc<double>(p.n);
    d.zout = arena_.alloc<double>(p.n);
    d.yout = arena_.alloc<double>(p.m);
    d.xhat = arena_.alloc<double>(p.n);
    d.xc = arena_.alloc<double>(p.n);
    d.zc = arena_.alloc<double>(p.n);
    d.ounit = arena_.alloc<double>(size_t(p.n_orth) + p.soc_size.size());
    d.ctl = arena_.alloc<Ctl>(1);
    const size_t units = size_t(p.n_orth) + p.soc_size.size();
    nparts_ = std::max<size_t>({p.a_blocks.size(), size_t(d.st.wg_max), size_t(d.st_cg.wg_max), size_t(d.sa.wg_max), units / kBlock + 1,
                                 p.soc_size.size() / 4 + 1, size_t(p.m) / kBlock + 1, size_t(p.n) / kBlock + 1,
                                 size_t(p.m) / 16 + 1, 1});
    d.partials = arena_.alloc<double>(nparts_ * kMaxSums);
    if (S.equilibrate) {
      d.eq = arena_.alloc<double>(p.n);
      d.eq_u = arena_.alloc<double>(p.m);
      d.eq_c = arena_.alloc<double>(p.n);
    }
    s_buf_[0] = arena_.alloc<VT>(p.n);
    s_buf_[1] = arena_.alloc<VT>(p.n);
    if (res_.status) {
      hs_ = res_.status->take();
      if (!hs_) throw AcsError(ACS_ERR_NOMEM, "no free status record");
    } else {
      HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&hs_), sizeof(HostStatus),
                              hipHostMallocMapped | hipHostMallocCoherent));
    }
    std::memset(hs_, 0, sizeof(HostStatus));
    hs_->cg_done_iter = -1;
    hs_->check_iter = -1;
    HostStatus* hs_dev = nullptr;
    HIP_CHECK(hipHostGetDevicePointer(reinterpret_cast<void**>(&hs_dev), hs_, 0));
    d.hs = hs_dev;
    // cone groups: lanes per Lorentz cone, ~ the mean size, power of two in [4, 64]
    if (!p.soc_size.empty()) {
      double mean = double(p.n - p.n_orth) / double(p.soc_size.size());
      cone_group_ = 4;
      while (cone_group_ < 64 && cone_group_ < mean) cone_group_ <<= 1;
    }
    // zero the vectors that may be read before their first write
    std::vector<VT> zv(std::max(p.m, p.n), VT(0));
    std::vector<double> zd(std::max(p.m, p.n), 0.0);
    HIP_CHECK(hipMemcpyAsync(d.zt, zd.data(), sizeof(double) * p.n, hipMemcpyHostToDevice, st_));
    HIP_CHECK(hipMemcpyAsync(d.t, zv.data(), sizeof(VT) * p.n, hipMemcpyHostToDevice, st_));
    HIP_CHECK(hipMemcpyAsync(d.q, zv.data(), sizeof(VT) * p.m, hipMemcpyHostToDevice, st_));
    HIP_CHECK(hipMemcpyAsync(d.xout, zd.data(), sizeof(double) * p.n, hipMemcpyHostToDevice, st_));
    HIP_CHECK(hipMemcpyAsync(d.zout, zd.data(), sizeof(double) * p.n, hipMemcpyHostToDevice, st_));
    HIP_CHECK(hipMemcpyAsync(d.yout, zd.data(), sizeof(double) * p.m, hipMemcpyHostToDevice, st_));
    launch_ctl_reset(d, S.cg_max, st_);
    check_launch();
    HIP_CHECK(hipStreamSynchronize(st_));
  }

  // Sinkhorn-Knopp equilibration: E from eq_sweeps sweeps, kept on the device
  // (the conditioning reads it) and on the host (the initial O)
  void equilibrate() {
    const Problem& p = *P_;
    std::vector<double> ones(p.n, 1.0);
    HIP_CHECK(hipMemcpyAsync(d_.eq, ones.data(), sizeof(double) * p.n, hipMemcpyHostToDevice, st_));
    launch_equilibrate(d_, S.eq_sweeps, st_);
    check_launch();
    eq_.resize(p.n);
    HIP_CHECK(hipMemcpyAsync(eq_.data(), d_.eq, sizeof(double) * p.n, hipMemcpyDeviceToHost, st_));
    HIP_CHECK(hipStreamSynchronize(st_));
  }

  // x = z = e_K in the scaled variables, O = E (1 without equilibration), w = 0 (l = 0)
  void set_initial() {
    const Problem& p = *P_;
    std::vector<double> e(p.n, 0.0);
    for (int j = 0; j < p.n_orth; ++j) e[j] = 1.0;
    for (size_t i = 0; i < p.soc_size.size(); ++i) e[p.soc_off[i]] = 1.0;
    std::vector<double> sp(p.n), sc(p.n), O(eq_.empty() ? std::vector<double>(p.n, 1.0) : eq_), w(p.m, 0.0);
    for (int j = 0; j < p.n; ++j) {
      sp[j] = (1.0 + S.mu) * e[j];
      sc[j] = (1.0 - S.mu) * e[j];
    }
    set_state(0, sp.data(), sc.data(), O.data(), w.data());
  }

  template <typename T>
  void upload_vt(VT* dst, const T* src, size_t n) {
    std::vector<VT> tmp(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = VT(src[i]);
    HIP_CHECK(hipMemcpyAsync(dst, tmp.data(), n * sizeof(VT), hipMemcpyHostToDevice, st_));
    HIP_CHECK(hipStreamSynchronize(st_));
  }

  void set_state(int l, const double* s_prev, const double* s, const double* O, const double* w) override {
    const Problem& p = *P_;
    if (l < 0) throw AcsError(ACS_ERR_ARG, "l must be >= 0");
    for (int j = 0; j < p.n; ++j)
      if (!(O[j] > 0) || !std::isfinite(O[j])) throw AcsError(ACS_ERR_ARG, "O must be positive and finite");
    for (size_t i = 0; i < p.soc_size.size(); ++i)
      for (int e = p.soc_off[i] + 1; e < p.soc_off[i + 1]; ++e)
        if (O[e] != O[p.soc_off[i]]) throw AcsError(ACS_ERR_ARG, "O must be constant on every cone");
    HIP_CHECK(hipStreamSynchronize(st_));
    // progress records compare against iteration numbers: start them afresh,
    // since l may be earlier than the iterations already run
    __atomic_store_n(&hs_->cg_done_iter, -1, __ATOMIC_RELEASE);
    __atomic_store_n(&hs_->check_iter, -1, __ATOMIC_RELEASE);
    checked_iter_ = -1;
    cur_ = 0;
    upload_vt(s_buf_[0], s, p.n);
    upload_vt(s_buf_[1], s_prev, p.n);
    HIP_CHECK(hipMemcpyAsync(d_.O, O, sizeof(double) * p.n, hipMemcpyHostToDevice, st_));
    {
      std::vector<double> wi(p.m);  // internal row order
      for (int i = 0; i < p.m; ++i) wi[i] = w[p.row_perm[i]];
      HIP_CHECK(hipMemcpyAsync(d_.w, wi.data(), sizeof(double) * p.m, hipMemcpyHostToDevice, st_));
      HIP_CHECK(hipStreamSynchronize(st_));
    }
    launch_ctl_reset(d_, S.cg_max, st_);
    launch_rescale(d_, 2, st_);  // A_s, b_s, chat for O; w -> scaled
    check_launch();
    l_ = l;
    factored_ = false;
    if (sched_.contains(l + 1)) {
      // the conditioning of iteration l+1 reads abs_K(s_prev) on the cones
      launch_cone(d_, s_prev_dev(), false, true, cone_group_, st_);
    } else {
      prologue();
      if (fac_) factorize();
    }
    check_launch();
    HIP_CHECK(hipStreamSynchronize(st_));
    have_xyz_ = false;
    info = acs_info{};
    info.iterations = l;
  }

  VT* s_cur_dev() { return s_buf_[cur_]; }
  VT* s_prev_dev() { return s_buf_[cur_ ^ 1]; }

  // p = abs_K(s), v = p - chat - A_s^T w for the current s
  void prologue() {
    timed(KC_UPDATE, [&] { launch_update(d_, s_cur_dev(), s_prev_dev(), UPD_PROLOGUE, false, st_); });
    if (d_.n_soc) timed(KC_CONE, [&] { launch_cone(d_, s_cur_dev(), false, true, cone_group_, st_); });
  }

  // Alg. 2 steps 5-14 at the start of iteration l, then the prologue
  void condition() {
    timed(KC_COND, [&] {
      launch_cond_ratio(d_, s_prev_dev(), s_cur_dev(), S.t, st_);
      launch_cond_scale(d_, s_cur_dev(), st_);
      launch_rescale(d_, 1, st_);
    });
    info.conditionings += 1;
    prologue();
    if (fac_) factorize();
  }

  // ----------------------------------------------------------- profiling
  struct ProfEv {
    int cls;
    hipEvent_t a, b;
  };
  template <class F>
  void timed(int cls, F&& f) {
    if (!(prof_mask_ >> cls & 1u)) {
      f();
      check_launch();
      return;
    }
    ProfEv e{cls, nullptr, nullptr};
    if (prof_free_.empty()) {
      HIP_CHECK(hipEventCreate(&e.a));
      HIP_CHECK(hipEventCreate(&e.b));
    } else {
      e = prof_free_.back();
      prof_free_.pop_back();
      e.cls = cls;
    }
    LaunchEvents le{e.a, e.b, 0};
    struct Slot {
      explicit Slot(LaunchEvents* p) { launch_events() = p; }
      ~Slot() { launch_events() = nullptr; }
    };
    {
      Slot slot(&le);
      f();
    }
    check_launch();
    if (le.launches == 0) {  // nothing launched (e.g. no cones): not counted
      prof_free_.push_back(e);
      return;
    }
    prof_pending_.push_back(e);
  }
  void collect_profile() {
    if (prof_pending_.empty()) return;
    HIP_CHECK(hipStreamSynchronize(st_));
    for (auto& e : prof_pending_) {
      float ms = 0;
      HIP_CHECK(hipEventElapsedTime(&ms, e.a, e.b));
      prof_count_[e.cls] += 1;
      prof_ms_[e.cls] += ms;
      prof_free_.push_back(e);
    }
    prof_pending_.clear();
  }
  void profile(uint32_t mask) override {
    collect_profile();
    if (mask) {
      for (int i = 0; i < KC_N; ++i) {
        prof_count_[i] = 0;
        prof_ms_[i] = 0;
      }
    }
    prof_mask_ = mask & ((1u << KC_N) - 1);
  }
  void timing(int cls, int64_t* count, double* total_ms) override {
    if (cls < 0 || cls >= KC_N) throw AcsError(ACS_ERR_ARG, "timing class out of range");
    collect_profile();
    if (count) *count = prof_count_[cls];
    if (total_ms) *total_ms = prof_ms_[cls];
  }

  // --------------------------------------------------------- host waits
  // Spins on the pinned progress record; the stream is queried (a runtime
  // call, which takes the runtime's locks that concurrent solves on other
  // threads need to launch) only every 200 us, to catch a stream that went
  // idle without posting or failed.
  template <class Pred>
  void wait_for(Pred pred) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    auto next_query = t0 + std::chrono::microseconds(200);
    int spins = 0;
    while (!pred()) {
      std::atomic_thread_fence(std::memory_order_acquire);
      if (++spins < 256) continue;
      spins = 0;
      const auto now = clk::now();
      if (now < next_query) continue;
      next_query = now + std::chrono::microseconds(200);
      hipError_t q = hipStreamQuery(st_);
      if (q == hipSuccess) {
        // stream idle: every record has landed; re-test once
        std::atomic_thread_fence(std::memory_order_seq_cst);
        if (pred()) return;
        throw AcsError(ACS_ERR_DEVICE, "stream idle but progress record missing");
      }
      if (q != hipErrorNotReady) throw AcsError(ACS_ERR_DEVICE, std::string("stream error: ") + hipGetErrorString(q));
      if (now - t0 > std::chrono::seconds(120)) throw AcsError(ACS_ERR_DEVICE, "timed out waiting for the GPU");
      std::this_thread::yield();
    }
  }
  long long hs_launch_seq() { return __atomic_load_n(&hs_->launch_seq, __ATOMIC_ACQUIRE); }
  int hs_cg_done() { return __atomic_load_n(&hs_->cg_done_iter, __ATOMIC_ACQUIRE); }
  int hs_check() { return __atomic_load_n(&hs_->check_iter, __ATOMIC_ACQUIRE); }

  // CG for outer iteration `it`: chunks of launches, at most one chunk ahead.
  // Each step's id reaches the host's record from k_fin_cg_a, or (one-slice
  // layout, whose k_cg_t finalizes the step before it) from k_cg_a_one; there
  // the last step of a capped CG gets a k_fin_cg_a of its own.
  void run_cg(int it, int cg_max) {
    // steps of n >= 2^20 take longer than the host's turnaround: one step in
    // flight ahead keeps the GPU busy and launches about one step fewer after
    // convergence (each a set of exit-at-once dispatches); smaller steps need
    // two, and the few-microsecond steps of n < 2^14 five (measured: 7% less
    // time per CG step on small LPs than with two, 8% more at n = 50000)
    const int chunk = d_.n >= (1 << 20) ? 1 : d_.n >= (1 << 14) ? 2 : 5;
    const bool folded = cg_fin_folded(d_);
    int launched = 0;
    while (launched < cg_max) {
      const int c = std::min(chunk, cg_max - launched);
      for (int i = 0; i < c; ++i) {
        const int j = launched + i;
        const long long id = ++launch_id_;
        timed(KC_CG_T, [&] { launch_cg_t(d_, j, st_); });
        timed(KC_CG_A, [&] { launch_cg_a(d_, id, st_); });
        timed(KC_CG_COMB, [&] { launch_cg_comb(d_, st_); });
        if (!folded) timed(KC_FIN, [&] { launch_fin_cg_a(d_, id, st_); });
      }
      launched += c;
      if (launched >= cg_max) {
        if (folded) timed(KC_FIN, [&] { launch_fin_cg_a(d_, launch_id_, st_); });
        break;
      }
      const long long target = launch_id_ - c;
      wait_for([&] { return hs_cg_done() >= it || hs_launch_seq() >= target; });
      if (hs_cg_done() >= it) return;
    }
  }

  // consume a finished check; returns true when the KKT tolerance is met
  bool read_check(int l) {
    std::atomic_thread_fence(std::memory_order_acquire);
    const HostStatus& h = *hs_;
    info.eps_p = h.kkt[0];
    info.eps_d = h.kkt[1];
    info.eps_gap = h.kkt[2];
    info.eps_cone = h.kkt[3];
    info.kkt = h.kkt[4];
    info.pobj = h.kkt[5];
    info.dobj = h.kkt[6];
    info.eps_obj = h.kkt[8];
    info.cg_steps = h.cg_total;
    checked_iter_ = l;
    if (S.verbose)
        std::fprintf(stderr, "acs l=%d kkt=%.3e p=%.2e d=%.2e g=%.2e k=%.2e o=%.2e obj=%.10e cg=%lld\n", l, info.kkt,
                   info.eps_p, info.eps_d, info.eps_gap, info.eps_cone, info.eps_obj, info.pobj,
                   (long long)h.cg_total);
    if (__atomic_load_n(&hs_->numeric, __ATOMIC_ACQUIRE)) {
      info.status = ACS_NUMERIC;
      return true;
    }
    return info.kkt <= S.eps_kkt && info.eps_obj * S.obj_stop <= S.eps_kkt;
  }

  // ------------------------------------------------------------ iterate
  void run(int iters, bool stop_on_converge) override {
    const Problem& p = *P_;
    const auto t0 = std::chrono::steady_clock::now();
    const double red2 = S.cg_reduce * S.cg_reduce, abs2 = S.cg_abs * S.cg_abs;
    int pending = -1;  // iteration of a launched, unread check
    bool converged = false, stop_now = false;
    info.status = ACS_MAX_ITER;
    for (int it = 0; it < iters && !stop_now; ++it) {
      if (pending >= 0 && hs_check() >= pending) {  // a check finished meanwhile
        const bool ok = read_check(pending);
        pending = -1;
        if (ok && stop_on_converge) {
          converged = true;
          break;
        }
      }
      const int l = l_ + 1;
      if (sched_.contains(l)) condition();
      const bool next_event = sched_.contains(l + 1);
      // x, z of this iteration set O at l + 1: project accurately
      const double r2 = next_event ? std::min(red2, kEventCgReduce * kEventCgReduce) : red2;
      const int cg_max = next_event ? S.cg_max * kEventCgMaxFactor : S.cg_max;
      timed(KC_RESID, [&] { launch_resid(d_, st_); });
      if (fac_) {  // w += M^{-1} r
        timed(KC_FIN, [&] { launch_fin_resid(d_, l, r2, abs2, 0, st_); });
        timed(KC_FAC_APPLY, [&] { launch_fac_apply(d_, f_, st_); });
      } else {
        timed(KC_FIN, [&] { launch_fin_resid(d_, l, r2, abs2, cg_max, st_); });
        run_cg(l, cg_max);
      }
      bool check = (l % S.check_every == 0) || it == iters - 1;
      if (check && pending >= 0) {  // one check in flight at a time
        wait_for([&] { return hs_check() >= pending; });
        const bool ok = read_check(pending);
        pending = -1;
        if (ok && stop_on_converge) {  // finish this iteration, keep the converged x, y, z
          converged = true;
          check = false;
          stop_now = true;
        }
      }
      timed(KC_UPDATE, [&] {
        launch_update(d_, s_cur_dev(), s_prev_dev(), next_event ? UPD_UPDATE_ONLY : UPD_UPDATE, check, st_);
      });
      if (d_.n_soc) timed(KC_CONE, [&] { launch_cone(d_, s_prev_dev(), check, !next_event, cone_group_, st_); });
      cur_ ^= 1;
      l_ = l;
      if (check) {
        timed(KC_CHECK, [&] { launch_pres(d_, l, p.bnorm, p.cnorm, st_); });
        pending = l;
      }
    }
    if (pending >= 0) {
      wait_for([&] { return hs_check() >= pending; });
      if (read_check(pending)) converged = true;
    }
    HIP_CHECK(hipStreamSynchronize(st_));
    if (info.status != ACS_NUMERIC) info.status = converged ? ACS_SOLVED : ACS_MAX_ITER;
    info.iterations = checked_iter_ >= 0 ? checked_iter_ : l_;
    have_xyz_ = checked_iter_ >= 0;
    Ctl ctl;
    HIP_CHECK(hipMemcpy(&ctl, d_.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    info.cg_steps = ctl.cg_total;
    info.alpha = ctl.cond[3];
    info.o_range = -ctl.cond[1] - ctl.cond[0];
    if (info.o_range > S.t) info.o_range = info.alpha * info.o_range;
    info.solve_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }

  int current_l() const override { return l_; }

  // (A O^2 A^T)^{-1} of the last factorization, m x m in the caller's row
  // order: M^{-1} = diag(d)^{-1} (A O^2 A^T)^{-1} diag(d)^{-1}
  void normal_inverse(double* out) override {
    const Problem& p = *P_;
    if (!fac_) throw AcsError(ACS_ERR_STATE, "the state does not use the direct projection");
    if (!factored_) throw AcsError(ACS_ERR_STATE, "no factorization since the state was set");
    HIP_CHECK(hipStreamSynchronize(st_));
    std::vector<double> di(p.m), row(p.m);
    HIP_CHECK(hipMemcpy(di.data(), d_.dinv, sizeof(double) * p.m, hipMemcpyDeviceToHost));
    for (int i = 0; i < p.m; ++i) {
      HIP_CHECK(hipMemcpy(row.data(), f_.S + size_t(i) * f_.mp, sizeof(double) * p.m, hipMemcpyDeviceToHost));
      double* o = out + size_t(p.row_perm[i]) * p.m;
      for (int j = 0; j < p.m; ++j) o[p.row_perm[j]] = (di[i] * di[j]) * row[j];  // symmetric rounding
    }
  }

  void check_now() override {
    if (!have_xyz_) throw AcsError(ACS_ERR_STATE, "no iteration has been run since the state was set");
  }

  void get(int* l, double* s_prev, double* s, double* O, double* w, double* x, double* y, double* z) override {
    const Problem& p = *P_;
    HIP_CHECK(hipStreamSynchronize(st_));
    if (l) *l = l_;
    auto down_vt = [&](double* dst, const VT* src, size_t n) {
      std::vector<VT> tmp(n);
      HIP_CHECK(hipMemcpy(tmp.data(), src, n * sizeof(VT), hipMemcpyDeviceToHost));
      for (size_t i = 0; i < n; ++i) dst[i] = double(tmp[i]);
    };
    if (s_prev) down_vt(s_prev, s_prev_dev(), p.n);
    if (s) down_vt(s, s_cur_dev(), p.n);
    if (O) HIP_CHECK(hipMemcpy(O, d_.O, sizeof(double) * p.n, hipMemcpyDeviceToHost));
    if (w) {
      std::vector<double> ws(p.m), di(p.m);
      HIP_CHECK(hipMemcpy(ws.data(), d_.w, sizeof(double) * p.m, hipMemcpyDeviceToHost));
      HIP_CHECK(hipMemcpy(di.data(), d_.dinv, sizeof(double) * p.m, hipMemcpyDeviceToHost));
      for (int i = 0; i < p.m; ++i) w[p.row_perm[i]] = ws[i] * di[i];
    }
    if (x || y || z) {
      if (!have_xyz_) throw AcsError(ACS_ERR_STATE, "x, y, z need at least one iteration after the state was set");
      if (x) HIP_CHECK(hipMemcpy(x, d_.xout, sizeof(double) * p.n, hipMemcpyDeviceToHost));
      if (z) HIP_CHECK(hipMemcpy(z, d_.zout, sizeof(double) * p.n, hipMemcpyDeviceToHost));
      if (y) {
        std::vector<double> yi(p.m);
        HIP_CHECK(hipMemcpy(yi.data(), d_.yout, sizeof(double) * p.m, hipMemcpyDeviceToHost));
        for (int i = 0; i < p.m; ++i) y[p.row_perm[i]] = yi[i];
      }
    }
  }

  // x, y, z of the last check into caller-owned device buffers, ordered on
  // the instance's stream and complete on return
  void get_device(double* x, double* y, double* z) override {
    if (!have_xyz_) throw AcsError(ACS_ERR_STATE, "x, y, z need at least one iteration after the state was set");
    launch_out_device(d_, x, y, z, st_);
    check_launch();
    HIP_CHECK(hipStreamSynchronize(st_));
  }

  void spmv(int which, const void* x, void* y, int reps, double* avg_ms) override {
    if (which != 0 && which != 1) throw AcsError(ACS_ERR_ARG, "which must be 0 or 1");
    if (!x || !y) throw AcsError(ACS_ERR_ARG, "null vector");
    reps = std::max(reps, 1);
    hipEvent_t a, b;
    HIP_CHECK(hipEventCreate(&a));
    HIP_CHECK(hipEventCreate(&b));
    HIP_CHECK(hipEventRecord(a, st_));
    for (int i = 0; i < reps; ++i) launch_spmv(d_, which, static_cast<const VT*>(x), static_cast<VT*>(y), st_);
    check_launch();
    HIP_CHECK(hipEventRecord(b, st_));
    HIP_CHECK(hipEventSynchronize(b));
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (avg_ms) *avg_ms = double(ms) / reps;
  }

 private:
  std::shared_ptr<const Problem> P_;
  InstanceResources res_;
  Schedule sched_;
  hipStream_t st_ = nullptr;
  bool own_stream_ = false;
  DeviceArena arena_;
  Dev<VT> d_{};
  VT* s_buf_[2] = {nullptr, nullptr};
  int cur_ = 0;
  int l_ = 0;
  long long launch_id_ = 0;
  int checked_iter_ = -1;
  bool have_xyz_ = false;
  int cone_group_ = 4;
  size_t nparts_ = 1;
  bool fac_ = false;       // direct projection
  std::vector<double> eq_;  // E of the equilibration (empty without it)
  bool factored_ = false;  // M^{-1} matches the current scaling
  FacDev f_{};
  hipStream_t st2_ = nullptr;                     // the next sweep group's chain
  hipEvent_t fork_ = nullptr, join_ = nullptr;    // pass -> chain, chain -> next pass
  HostStatus* hs_ = nullptr;
  uint32_t prof_mask_ = 0;  // kernel classes timed with events
  std::vector<ProfEv> prof_pending_, prof_free_;
  int64_t prof_count_[KC_N] = {0};
  double prof_ms_[KC_N] = {0};
};

static std::unique_ptr<InstanceBase> make_instance(std::shared_ptr<const Problem> p, const acs_settings& s,
                                                   hipStream_t st,
                                                   const InstanceResources& res = InstanceResources()) {
  if (s.precision == ACS_PREC_FP64) return std::make_unique<Instance<double>>(std::move(p), s, st, res);
  return std::make_unique<Instance<float>>(std::move(p), s, st, res);
}

SolveOut solve_one_instance(std::shared_ptr<const Problem> p, const acs_settings& s, void* stream,
                            const InstanceResources& res) {
  auto inst = make_instance(p, s, static_cast<hipStream_t>(stream), res);
  inst->run(inst->S.max_iter, true);
  SolveOut o;
  o.x.resize(p->n);
  o.z.resize(p->n);
  o.y.resize(p->m);
  inst->get(nullptr, nullptr, nullptr, nullptr, nullptr, o.x.data(), o.y.data(), o.z.data());
  o.info = inst->info;
  return o;
}

int64_t instance_device_bytes(const Problem& p, int precision, int projection, int equilibrate, int a_slices) {
  return estimate_bytes(p, precision, a_slices) + (projection == ACS_PROJ_FACTOR ? factor_bytes(p) : 0) +
         (equilibrate ? 8 * (2 * int64_t(p.n) + p.m) + 3 * 256 : 0);
}

static int g_device = -1;
static std::mutex g_init_mu;

void ensure_device() {
  std::lock_guard<std::mutex> lk(g_init_mu);
  if (g_device >= 0) {
    HIP_CHECK(hipSetDevice(g_device));
    return;
  }
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count < 1) {
    (void)hipGetLastError();
    throw AcsError(ACS_ERR_DEVICE, "no HIP device available");
  }
  hipDeviceProp_t prop;
  HIP_CHECK(hipGetDeviceProperties(&prop, 0));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    throw AcsError(ACS_ERR_DEVICE, std::string("device 0 is ") + prop.gcnArchName + ", this library is built for gfx950");
  HIP_CHECK(hipSetDevice(0));
  g_device = 0;
}

// ----------------------------------------------------------------------------
// solves that allocate nothing (acs_solve_device_noalloc)
// ----------------------------------------------------------------------------
// The instance's device arrays come from this file-scope array.  In host code
// `scratch` is only a stand-in for the symbol: its device address, one per
// GPU, comes from hipGetSymbolAddress at set-up and is the only form handed
// to kernels and copies.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct NoAllocDevice {
  std::mutex mu;                                  // calls on the device share the array: one at a time
  void* ptr = nullptr;                            // device address of `scratch` on this device
  std::unique_ptr<SubAllocator> mem;              // first-fit over ptr (no allocation)
  std::unique_ptr<StatusPool> status;             // one pinned progress record
  hipStream_t stream = nullptr;                   // used when the caller passes no stream
};
// device 0 (the only device this library drives); never destroyed, so that
// nothing of it is released after the HIP runtime at process exit
static NoAllocDevice* const g_noalloc = new NoAllocDevice;
static std::mutex g_noalloc_setup_mu;

// Once per device, with the device current: the array's address, the status
// record and the fallback stream.  Called by acs_init and by the entry point.
static NoAllocDevice& noalloc_device() {
  std::lock_guard<std::mutex> lk(g_noalloc_setup_mu);
  NoAllocDevice& na = *g_noalloc;
  if (na.ptr) return na;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    throw AcsError(ACS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  auto status = std::make_unique<StatusPool>(1);
  hipStream_t st = nullptr;
  HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  na.mem = std::make_unique<SubAllocator>(ptr, kNoAllocBytes);
  na.status = std::move(status);
  na.stream = st;
  na.ptr = ptr;
  return na;
}

}  // namespace acs

// ============================================================================
// C ABI
// ============================================================================
using namespace acs;

struct acs_state {
  std::unique_ptr<InstanceBase> inst;
};

extern "C" {

const char* acs_version(void) { return "acs 0.1 (gfx950)"; }

const char* acs_last_error(void) { return g_last_error.c_str(); }

int acs_init(int32_t device) {
  return guarded([&] {
    if (device != 0) throw AcsError(ACS_ERR_ARG, "only device 0 is supported");
    ensure_device();
    noalloc_device();
  });
}

void acs_settings_default(acs_settings* s) {
  if (!s) return;
  std::memset(s, 0, sizeof(*s));
  s->mu = 1.0;
  s->t = 9.2;
  s->l_first = 300;
  s->l_every = 100;
  s->l_last = -1;
  s->auto_params = 1;
  s->max_iter = 20000;
  s->check_every = 10;
  s->eps_kkt = 1e-4;
  s->precision = ACS_PREC_MIXED;
  s->cg_max = 500;
  s->cg_reduce = 0.0;  // per class: kCgReduceLp, kCgReduceSocp
  s->cg_abs = 0.0;
  s->verbose = 0;
  s->obj_stop = 1;
  s->equilibrate = 0;
  s->eq_sweeps = 25;
}

int acs_problem_create(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                       const double* val, const double* b, const double* c, int32_t n_orth, int32_t n_soc,
                       const int32_t* soc_sizes, acs_problem** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out) throw AcsError(ACS_ERR_ARG, "out is null");
    auto p = std::make_shared<Problem>();
    std::string err;
    if (!build_problem(m, n, nnz, row_ptr, col_idx, val, b, c, n_orth, n_soc, soc_sizes, p.get(), &err))
      throw AcsError(ACS_ERR_ARG, err);
    *out = new acs_problem{std::move(p)};
  });
}

int acs_problem_create_dense(int32_t m, int32_t n, const double* a, const double* b, const double* c, int32_t n_orth,
                             int32_t n_soc, const int32_t* soc_sizes, acs_problem** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out) throw AcsError(ACS_ERR_ARG, "out is null");
    auto p = std::make_shared<Problem>();
    std::string err;
    if (!build_problem_dense(m, n, a, b, c, n_orth, n_soc, soc_sizes, p.get(), &err)) throw AcsError(ACS_ERR_ARG, err);
    *out = new acs_problem{std::move(p)};
  });
}

void acs_problem_destroy(acs_problem* p) { delete p; }

int64_t acs_problem_device_bytes(const acs_problem* p, int32_t precision) {
  if (!p) return -1;
  return estimate_bytes(*p->p, precision, 0);
}

int acs_state_create(const acs_problem* p, const acs_settings* s, void* stream, acs_state** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!p || !s || !out) throw AcsError(ACS_ERR_ARG, "null argument");
    ensure_device();
    auto st = std::make_unique<acs_state>();
    st->inst = make_instance(p->p, *s, static_cast<hipStream_t>(stream));
    *out = st.release();
  });
}

void acs_state_destroy(acs_state* st) { delete st; }

int acs_state_set(acs_state* st, int32_t l, const double* s_prev, const double* s, const double* O,
                  const double* w) {
  return guarded([&] {
    if (!st || !s_prev || !s || !O || !w) throw AcsError(ACS_ERR_ARG, "null argument");
    st->inst->set_state(l, s_prev, s, O, w);
  });
}

int acs_state_step(acs_state* st, int32_t iters) {
  return guarded([&] {
    if (!st || iters < 0) throw AcsError(ACS_ERR_ARG, "bad argument");
    if (iters > 0) st->inst->run(iters, false);
  });
}

int acs_state_solve(acs_state* st, acs_info* info) {
  return guarded([&] {
    if (!st) throw AcsError(ACS_ERR_ARG, "null state");
    InstanceBase& in = *st->inst;
    const int left = in.S.max_iter - in.current_l();
    if (left > 0) in.run(left, true);
    if (info) *info = in.info;
  });
}

int acs_state_get(acs_state* st, int32_t* l, double* s_prev, double* s, double* O, double* w, double* x, double* y,
                  double* z) {
  return guarded([&] {
    if (!st) throw AcsError(ACS_ERR_ARG, "null state");
    int li = 0;
    st->inst->get(&li, s_prev, s, O, w, x, y, z);
    if (l) *l = li;
  });
}

int acs_state_info(acs_state* st, acs_info* info) {
  return guarded([&] {
    if (!st || !info) throw AcsError(ACS_ERR_ARG, "null argument");
    *info = st->inst->info;
  });
}

int acs_state_check(acs_state* st, acs_info* info) {
  return guarded([&] {
    if (!st) throw AcsError(ACS_ERR_ARG, "null state");
    st->inst->check_now();
    if (info) *info = st->inst->info;
  });
}

int acs_state_spmv(acs_state* st, int32_t which, const void* x, void* y, int32_t reps, double* avg_ms) {
  return guarded([&] {
    if (!st) throw AcsError(ACS_ERR_ARG, "null state");
    st->inst->spmv(which, x, y, reps, avg_ms);
  });
}

int acs_state_profile(acs_state* st, int32_t enable) {
  return guarded([&] {
    if (!st) throw AcsError(ACS_ERR_ARG, "null state");
    st->inst->profile(uint32_t(enable));
  });
}

int acs_state_normal_inverse(acs_state* st, double* out) {
  return guarded([&] {
    if (!st || !out) throw AcsError(ACS_ERR_ARG, "null argument");
    st->inst->normal_inverse(out);
  });
}

int64_t acs_problem_factor_bytes(const acs_problem* p) {
  if (!p) return -1;
  return factor_bytes(*p->p);
}

int acs_state_timing(acs_state* st, int32_t cls, int64_t* count, double* total_ms) {
  return guarded([&] {
    if (!st) throw AcsError(ACS_ERR_ARG, "null state");
    st->inst->timing(cls, count, total_ms);
  });
}

int acs_solve_device(const acs_problem* p, const acs_settings* s, double* x, double* y, double* z,
                     acs_info* info, void* stream) {
  return guarded([&] {
    if (!p || !s) throw AcsError(ACS_ERR_ARG, "null argument");
    ensure_device();
    for (const void* ptr : {static_cast<const void*>(x), static_cast<const void*>(y), static_cast<const void*>(z)}) {
      if (!ptr) continue;
      hipPointerAttribute_t attr;
      if (hipPointerGetAttributes(&attr, ptr) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        throw AcsError(ACS_ERR_ARG, "acs_solve_device: x, y and z must be device allocations");
      }
    }
    auto inst = make_instance(p->p, *s, static_cast<hipStream_t>(stream));
    inst->run(inst->S.max_iter, true);
    if (x || y || z) inst->get_device(x, y, z);
    if (info) *info = inst->info;
  });
}

int acs_solve_device_noalloc(const acs_problem* p, const acs_settings* s, double* x, double* y, double* z,
                             acs_info* info, void* stream) {
  return guarded([&] {
    if (!p || !s) throw AcsError(ACS_ERR_ARG, "null argument");
    ensure_device();
    NoAllocDevice& na = noalloc_device();
    for (const void* ptr : {static_cast<const void*>(x), static_cast<const void*>(y), static_cast<const void*>(z)}) {
      if (!ptr) continue;
      hipPointerAttribute_t attr;
      if (hipPointerGetAttributes(&attr, ptr) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        throw AcsError(ACS_ERR_ARG, "acs_solve_device_noalloc: x, y and z must be device allocations");
      }
    }
    if (s->projection != ACS_PROJ_CG)
      throw AcsError(ACS_ERR_ARG, "acs_solve_device_noalloc: only the CG projection (ACS_PROJ_CG)");
    const int64_t need = instance_device_bytes(*p->p, s->precision, ACS_PROJ_CG, s->equilibrate, s->a_slices);
    if (need > int64_t(kNoAllocBytes))
      throw AcsError(ACS_ERR_NOMEM, "acs_solve_device_noalloc: the problem needs " + std::to_string(need) +
                                        " device bytes, the fixed scratch holds " + std::to_string(kNoAllocBytes));
    std::lock_guard<std::mutex> lk(na.mu);
    const InstanceResources res{na.mem.get(), na.status.get()};
    auto inst = make_instance(p->p, *s, stream ? static_cast<hipStream_t>(stream) : na.stream, res);
    inst->run(inst->S.max_iter, true);
    if (x || y || z) inst->get_device(x, y, z);
    if (info) *info = inst->info;
  });
}

int acs_solve(const acs_problem* p, const acs_settings* s, double* x, double* y, double* z, acs_info* info,
              void* stream) {
  return guarded([&] {
    if (!p || !s) throw AcsError(ACS_ERR_ARG, "null argument");
    ensure_device();
    auto inst = make_instance(p->p, *s, static_cast<hipStream_t>(stream));
    inst->run(inst->S.max_iter, true);
    if (x || y || z) inst->get(nullptr, nullptr, nullptr, nullptr, nullptr, x, y, z);
    if (info) *info = inst->info;
  });
}

}  // extern "C"
