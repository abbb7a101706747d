// Internal types shared by the host code and the HIP kernels of libacs.
#pragma once

#include <cstdint>
#include <memory>
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

// Host copy of a validated problem (Sec. II): CSR of A, b, c, cone list.
struct Problem {
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
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
  // A split by column ranges [x*w, (x+1)*w), w = ceil(n/kSlices): the nonzeros
  // of slice x in row order; s_row_ptr holds kSlices row pointers of m+1
  // absolute offsets; s_perm maps to the position in A's CSR.
  std::vector<int32_t> s_row_ptr, s_col, s_perm;
  std::vector<RowBlock> s_blocks;     // row blocks of every slice, slice after slice
  std::vector<int32_t> s_blk_off;     // kSlices + 1 offsets into s_blocks
  double bnorm = 0, cnorm = 0;
  int32_t max_soc = 0;
  bool is_socp() const { return !soc_size.empty(); }
};

// Validates and copies a problem; on failure returns false and sets err.
bool build_problem(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                   const double* val, const double* b, const double* c, int32_t n_orth, int32_t n_soc,
                   const int32_t* soc_sizes, Problem* out, std::string* err);

// Partition rows of a CSR into RowBlocks (LDS-staged multi-row blocks of at
// most `stage` nonzeros; a longer row gets a block of its own).  Long-row
// blocks are placed first so they start early.
std::vector<RowBlock> make_row_blocks(const int32_t* row_ptr, int32_t rows, int32_t stage);

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
  ~SubAllocator();
  void* alloc(size_t bytes);  // nullptr when no free range fits
  void release(void* p);
  size_t capacity() const { return size_; }

 private:
  struct Impl;
  Impl* impl_;
  char* base_ = nullptr;
  size_t size_ = 0;
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
int64_t instance_device_bytes(const Problem& p, int precision);

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
