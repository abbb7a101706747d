// Problem validation, CSR transpose and row-block partitioning (host only).
#include <algorithm>
#include <cmath>
#include <sstream>

#include "acs_internal.h"

namespace acs {

static bool fail(std::string* err, const std::string& msg) {
  if (err) *err = msg;
  return false;
}

bool build_problem(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                   const double* val, const double* b, const double* c, int32_t n_orth, int32_t n_soc,
                   const int32_t* soc_sizes, Problem* out, std::string* err) {
  if (m < 1 || n < 1) return fail(err, "m and n must be >= 1");
  if (nnz < 0 || nnz >= (int64_t(1) << 31) - 1) return fail(err, "nnz must be in [0, 2^31-1)");
  if (!row_ptr || (nnz > 0 && (!col_idx || !val)) || !b || !c) return fail(err, "null array argument");
  if (n_orth < 0 || n_soc < 0) return fail(err, "n_orth and n_soc must be >= 0");
  if (n_soc > 0 && !soc_sizes) return fail(err, "soc_sizes is null");
  if (row_ptr[0] != 0) return fail(err, "row_ptr[0] must be 0");
  if (row_ptr[m] != nnz) return fail(err, "row_ptr[m] must equal nnz");
  Problem& p = *out;
  p.m = m;
  p.n = n;
  p.nnz = nnz;
  p.row_ptr.resize(size_t(m) + 1);
  for (int32_t i = 0; i <= m; ++i) {
    if (i > 0 && row_ptr[i] < row_ptr[i - 1]) {
      std::ostringstream os;
      os << "row_ptr decreases at row " << i - 1;
      return fail(err, os.str());
    }
    p.row_ptr[i] = int32_t(row_ptr[i]);
  }
  p.col.assign(col_idx, col_idx + nnz);
  p.val.assign(val, val + nnz);
  for (int32_t i = 0; i < m; ++i) {
    for (int32_t k = p.row_ptr[i]; k < p.row_ptr[i + 1]; ++k) {
      int32_t j = p.col[k];
      if (j < 0 || j >= n) {
        std::ostringstream os;
        os << "column index " << j << " out of range in row " << i;
        return fail(err, os.str());
      }
      if (k > p.row_ptr[i] && j <= p.col[k - 1]) {
        std::ostringstream os;
        os << "column indices not strictly ascending in row " << i;
        return fail(err, os.str());
      }
      if (!std::isfinite(p.val[k])) return fail(err, "non-finite matrix value");
    }
  }
  p.b.assign(b, b + m);
  p.c.assign(c, c + n);
  for (double v : p.b)
    if (!std::isfinite(v)) return fail(err, "non-finite entry in b");
  for (double v : p.c)
    if (!std::isfinite(v)) return fail(err, "non-finite entry in c");
  int64_t total = n_orth;
  p.n_orth = n_orth;
  p.soc_size.assign(soc_sizes, soc_sizes + n_soc);
  p.soc_off.resize(size_t(n_soc) + 1);
  p.soc_off[0] = n_orth;
  p.max_soc = 0;
  for (int32_t i = 0; i < n_soc; ++i) {
    if (p.soc_size[i] < 1) return fail(err, "second-order cone sizes must be >= 1");
    total += p.soc_size[i];
    if (total > n) return fail(err, "cone sizes exceed n");
    p.soc_off[i + 1] = int32_t(total);
    p.max_soc = std::max(p.max_soc, p.soc_size[i]);
  }
  if (total != n) return fail(err, "n_orth + sum(soc_sizes) must equal n");

  // transpose pattern by counting sort over columns (columns ascending in A^T rows = rows of A)
  p.t_row_ptr.assign(size_t(n) + 1, 0);
  for (int64_t k = 0; k < nnz; ++k) p.t_row_ptr[p.col[k] + 1]++;
  for (int32_t j = 0; j < n; ++j) p.t_row_ptr[j + 1] += p.t_row_ptr[j];
  p.t_col.resize(nnz);
  p.t_perm.resize(nnz);
  std::vector<int32_t> fill(p.t_row_ptr.begin(), p.t_row_ptr.end() - 1);
  for (int32_t i = 0; i < m; ++i) {
    for (int32_t k = p.row_ptr[i]; k < p.row_ptr[i + 1]; ++k) {
      int32_t pos = fill[p.col[k]]++;
      p.t_col[pos] = i;
      p.t_perm[pos] = k;
    }
  }
  // column slices of A (one per XCD): gathers of an n-vector stay within 1/kSlices of it
  {
    const int64_t w = (int64_t(n) + kSlices - 1) / kSlices;
    p.s_row_ptr.assign(size_t(kSlices) * (m + 1), 0);
    for (int32_t i = 0; i < m; ++i)
      for (int32_t k = p.row_ptr[i]; k < p.row_ptr[i + 1]; ++k) {
        const int x = int(p.col[k] / w);
        p.s_row_ptr[size_t(x) * (m + 1) + i + 1]++;
      }
    int32_t base = 0;
    for (int x = 0; x < kSlices; ++x) {
      int32_t* rp = &p.s_row_ptr[size_t(x) * (m + 1)];
      rp[0] = base;
      for (int32_t i = 0; i < m; ++i) rp[i + 1] += rp[i];
      base = rp[m];
    }
    p.s_col.resize(nnz);
    p.s_perm.resize(nnz);
    std::vector<int32_t> fill(size_t(kSlices) * m);
    for (int x = 0; x < kSlices; ++x)
      for (int32_t i = 0; i < m; ++i) fill[size_t(x) * m + i] = p.s_row_ptr[size_t(x) * (m + 1) + i];
    for (int32_t i = 0; i < m; ++i)
      for (int32_t k = p.row_ptr[i]; k < p.row_ptr[i + 1]; ++k) {
        const int x = int(p.col[k] / w);
        const int32_t pos = fill[size_t(x) * m + i]++;
        p.s_col[pos] = p.col[k];
        p.s_perm[pos] = k;
      }
    p.s_blk_off.assign(kSlices + 1, 0);
    for (int x = 0; x < kSlices; ++x) {
      std::vector<RowBlock> b = make_row_blocks(&p.s_row_ptr[size_t(x) * (m + 1)], m, kStageNnz);
      p.s_blocks.insert(p.s_blocks.end(), b.begin(), b.end());
      p.s_blk_off[x + 1] = int32_t(p.s_blocks.size());
    }
  }
  p.a_blocks = make_row_blocks(p.row_ptr.data(), m, kStageNnz);
  p.t_blocks = make_row_blocks(p.t_row_ptr.data(), n, kStageNnz);
  double bb = 0, cc = 0;
  for (double v : p.b) bb += v * v;
  for (double v : p.c) cc += v * v;
  p.bnorm = std::sqrt(bb);
  p.cnorm = std::sqrt(cc);
  return true;
}

std::vector<RowBlock> make_row_blocks(const int32_t* row_ptr, int32_t rows, int32_t stage) {
  std::vector<RowBlock> longs, shorts;
  int32_t r = 0;
  while (r < rows) {
    int32_t len = row_ptr[r + 1] - row_ptr[r];
    if (len > stage) {
      longs.push_back({r, r + 1});
      ++r;
      continue;
    }
    int32_t r0 = r;
    int32_t base = row_ptr[r0];
    // extend while the staged products fit; cap rows so each row group is at
    // least one lane (more rows than threads are looped over)
    while (r < rows && row_ptr[r + 1] - base <= stage && (r - r0) < 8 * kBlock) ++r;
    shorts.push_back({r0, r});
  }
  // longest rows first
  std::sort(longs.begin(), longs.end(), [&](const RowBlock& a, const RowBlock& b) {
    return (row_ptr[a.r1] - row_ptr[a.r0]) > (row_ptr[b.r1] - row_ptr[b.r0]);
  });
  longs.insert(longs.end(), shorts.begin(), shorts.end());
  return longs;
}

}  // namespace acs
