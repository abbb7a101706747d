// Internal types shared by the host code and the HIP kernels of libacs.
#pragma once

#include <cstdint>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/acs.h"

namespace acs {

// Row range [r0, r1) of a CSR matrix processed by one workgroup.  A range
// holds at most kStageNnz nonzeros, unless it is a single longer row.
struct RowBlock {
  int32_t r0;
  int32_t r1;
};

constexpr int kBlock = 256;       // threads per workgroup (4 wave64)
constexpr int kStageNnz = 2048;   // products staged in LDS per multi-row block
constexpr int kSlices = 8;        // column slices of A, one per XCD
constexpr int32_t kOneSliceMaxN = 262144;  // settings.a_slices = 0: one slice up to this n
constexpr int32_t kAutoFactorMaxM = 2048;  // ACS_PROJ_AUTO: the direct projection up to this m
// The iteration whose x, z feed a conditioning event (Alg. 2 steps 5-10 read
// the x, z of the previous iteration) projects accurately: its CG runs to a
// relative residual reduction of kEventCgReduce, with up to kEventCgMaxFactor
// times the usual step cap.  The ratios o = x/z of complementary pairs are
// taken between numbers that go to zero, so a loose projection there sets O
// from noise; the paper's projection is exact.
constexpr double kEventCgReduce = 1e-6;
constexpr int kEventCgMaxFactor = 8;
// CG residual reduction of the other iterations when settings.cg_reduce = 0
constexpr double kCgReduceLp = 0.1;
constexpr double kCgReduceSocp = 0.2;
constexpr int kSellChunk = 64;    // rows per SELL chunk (one per lane of a wave64)
constexpr int kSellMaxLen = 64;   // longest row packed into a chunk
constexpr int kWaveRowMax = 2048; // longest row given to one wave; longer rows get a workgroup
constexpr int kSellWindow = 16384; // rows sorted by length within windows of this many rows
constexpr int kHostThreads = 16;  // host threads that build the layouts of one large problem

// SELL-64 layout of the products of the CG (each output row is a dot product
// of a sparse row with a gathered vector).  The rows are split into slices
// (column ranges of A for A t, one per XCD; a single slice for A^T r).  Per
// slice, a row longer than kWaveRowMax is a "long task" run by a whole
// workgroup; every other row belongs to a "wave task": a row longer than
// kSellMaxLen gets a wave of its own (lanes stride the row), shorter rows are
// packed 64 to a chunk (one row per lane, entries stored column-major so a
// wave's loads are contiguous, padded to the chunk's longest row).  Within a
// window of kSellWindow rows the chunk rows are sorted by length, which keeps
// padding small while the rows written by neighbouring chunks stay close.
// Every row of every slice is covered exactly once (empty rows too, so that
// each output is written).
struct Sell {
  int32_t slices = 0;
  std::vector<int32_t> long_off;            // slices+1 offsets into long_*
  std::vector<int32_t> long_row, long_beg;  // row and first entry of each long task
  std::vector<int32_t> long_end;
  std::vector<int32_t> wt_off;  // slices+1 offsets into wt_*
  std::vector<int32_t> wt_ptr;  // first entry of the task
  std::vector<int32_t> wt_len;  // entries of the row (wave row) or per lane (chunk)
  std::vector<int32_t> wt_row;  // >= 0: row of a wave-row task; -1: a chunk
  std::vector<int32_t> chunk_row;  // kSellChunk per wave task (indexed by task): row of each
                                   // lane of a chunk, -1 = unused lane (all -1 for wave rows)
  std::vector<int32_t> col;        // column of each entry
  std::vector<int32_t> src;        // position of the entry in A's CSR, -1 = padding
  std::vector<int32_t> wg;         // workgroups of each slice: long tasks + ceil(wave tasks / 4)
  int32_t wg_max = 0;
};

struct SellPair {
  Sell a;  // A t, 1 or kSlices column slices of A (residual sweeps, plain products)
  Sell t;  // A^T r, one slice (update sweeps)
  // With kSlices column slices the CG's products run with the columns of A
  // renumbered within each slice in the order `a` first reads them (its
  // entries in storage order), so the CG vector t lives in that order: a
  // gather that comes first in a wave's reads lands next to its neighbours'.
  // a_cg_col is `a`'s column array in the new numbering (tasks, entries and
  // values are `a`'s); t_cg is the A^T layout with its rows (columns of A) in
  // the new order; cg_col[j'] is the column of A that new index j' stands
  // for.  With one slice (t small enough for the caches) the CG uses `a` and
  // `t` and these stay empty (cg_own false).
  bool cg_own = false;
  std::vector<int32_t> a_cg_col;
  Sell t_cg;
  std::vector<int32_t> cg_col;
};

// Host copy of a validated problem (Sec. II): CSR of A, b, c, cone list.
// Rows are renumbered by decreasing length (ties in the caller's order): the
// vector gathered by the A^T products then has its most used entries packed
// together.  Internal row i is the caller's row row_perm[i]; every m-vector
// crossing the C ABI (y, w) is mapped with it.
struct Problem {
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  // Dense A (acs_problem_create_dense): row-major, leading dimension ld (n
  // rounded up to 64, padding zero), FP32 values; dlo holds the FP32 rounding
  // error of each value when some value is not an FP32 number (empty
  // otherwise), so hi + lo is the value for the FP64 sweeps.  The sparse
  // fields below are then empty and row_perm is the identity.
  bool dense = false;
  int32_t ld = 0;
  std::vector<float> dhi, dlo;
  std::vector<int32_t> row_perm;  // m
  std::vector<int32_t> row_ptr;  // m+1
  std::vector<int32_t> col;      // nnz
  std::vector<double> val;       // nnz
  std::vector<double> b, c;
  int32_t n_orth = 0;
  std::vector<int32_t> soc_size;  // sizes of the Lorentz cones after the orthant block
  std::vector<int32_t> soc_off;   // n_soc+1 absolute offsets, soc_off[0] = n_orth
  // pattern of A^T (CSR over columns of A): t_row_ptr (n+1), t_col (row of A), t_perm (index into val)
  std::vector<int32_t> t_row_ptr, t_col, t_perm;
  std::vector<RowBlock> a_blocks, t_blocks;
  double bnorm = 0, cnorm = 0;
  int32_t max_soc = 0;
  bool is_socp() const { return !soc_size.empty(); }
  // SELL layouts of the CG products with A split into `slices` (1 or
  // kSlices) column slices, built on first use by the one-instance path (the
  // batched kernel does not use them).
  const SellPair& sell(int slices) const;
  // the column slices settings.a_slices asks for (0: by size)
  int a_slices(int requested) const { return requested ? requested : (n <= kOneSliceMaxN ? 1 : kSlices); }

 private:
  mutable std::once_flag sell_once_[2];
  mutable std::unique_ptr<SellPair> sell_[2];
};

// Validates and copies a dense problem (A row-major m x n).
bool build_problem_dense(int32_t m, int32_t n, const double* a, const double* b, const double* c, int32_t n_orth,
                         int32_t n_soc, const int32_t* soc_sizes, Problem* out, std::string* err);

// Validates and copies a problem; on failure returns false and sets err.
bool build_problem(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                   const double* val, const double* b, const double* c, int32_t n_orth, int32_t n_soc,
                   const int32_t* soc_sizes, Problem* out, std::string* err);

// Partition rows of a CSR into RowBlocks (LDS-staged multi-row blocks of at
// most `stage` nonzeros; a longer row gets a block of its own).  Long-row
// blocks are placed first so they start early.
std::vector<RowBlock> make_row_blocks(const int32_t* row_ptr, int32_t rows, int32_t stage);

// SELL layout of rp.size() slices: slice x has rows 0..rows-1 with entries
// [rp[x][i], rp[x][i+1]) of (col, src); pad[x] is the column that padding
// entries point at.  Throws AcsError if the layout would exceed 2^31-1 entries.
void build_sell(const std::vector<const int32_t*>& rp, int32_t rows, const int32_t* col, const int32_t* src,
                const std::vector<int32_t>& pad, Sell* out, int32_t window = kSellWindow,
                int32_t max_len = kSellMaxLen);
// Checks that every row of every slice is covered once and every entry once.
bool check_sell(const Sell& s, int32_t rows, int64_t entries, std::string* err);

// Error reporting (thread-local message).
void set_error(const std::string& msg);

// Error carried inside the library; converted to a return code at the ABI.
struct AcsError : std::runtime_error {
  int code;
  AcsError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Settings with the per-class defaults resolved and validated.
acs_settings resolve_settings(const acs_settings& in, const Problem& p);

// Select device 0 (gfx950) once per process.
void ensure_device();

// First-fit sub-allocator over one device allocation (256-B granularity).
// Serving uses it so that no hipMalloc/hipFree (hipFree waits for the whole
// device) happens while requests run.  Thread-safe.
class SubAllocator {
 public:
  explicit SubAllocator(size_t bytes);
  // first-fit over caller-provided device memory [base, base + bytes)
  // (256-B aligned); allocates nothing and frees nothing
  SubAllocator(void* base, size_t bytes);
  ~SubAllocator();
  void* alloc(size_t bytes);  // nullptr when no free range fits
  void release(void* p);
  size_t capacity() const { return size_; }

 private:
  struct Impl;
  Impl* impl_;
  char* base_ = nullptr;
  size_t size_ = 0;
  bool own_ = true;
};

struct HostStatus;
// Pinned, device-mapped host records for the kernels' progress reports.
class StatusPool {
 public:
  explicit StatusPool(int count);
  ~StatusPool();
  HostStatus* take();  // nullptr when exhausted
  void give(HostStatus* h);

 private:
  struct Impl;
  Impl* impl_;
};

// Optional resources an instance draws on instead of allocating its own.
struct InstanceResources {
  SubAllocator* mem = nullptr;
  StatusPool* status = nullptr;
};

// One-instance solve (the acs_solve path) on a given stream.
struct SolveOut {
  std::vector<double> x, y, z;
  acs_info info;
};
SolveOut solve_one_instance(std::shared_ptr<const Problem> p, const acs_settings& s, void* stream,
                            const InstanceResources& res = InstanceResources());
int64_t instance_device_bytes(const Problem& p, int precision, int projection, int equilibrate = 0,
                              int a_slices = 0);

template <class F>
int guarded(F&& f) {
  try {
    f();
    return ACS_OK;
  } catch (const AcsError& e) {
    set_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return ACS_ERR_NOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return ACS_ERR_DEVICE;
  }
}

}  // namespace acs

// Library-side body of the opaque problem handle.
struct acs_problem {
  std::shared_ptr<const acs::Problem> p;
};
