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

// b, c and the cone list (shared by the sparse and the dense builder)
static bool set_vectors_and_cones(int32_t m, int32_t n, const double* b, const double* c, int32_t n_orth,
                                  int32_t n_soc, const int32_t* soc_sizes, Problem* out, std::string* err) {
  for (int32_t i = 0; i < m; ++i)
    if (!std::isfinite(b[i])) return fail(err, "non-finite entry in b");
  for (int32_t j = 0; j < n; ++j)
    if (!std::isfinite(c[j])) return fail(err, "non-finite entry in c");
  Problem& p = *out;
  p.m = m;
  p.n = n;
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
  double bb = 0, cc = 0;
  for (int32_t i = 0; i < m; ++i) bb += b[i] * b[i];
  for (int32_t j = 0; j < n; ++j) cc += c[j] * c[j];
  p.bnorm = std::sqrt(bb);
  p.cnorm = std::sqrt(cc);
  return true;
}

bool build_problem_dense(int32_t m, int32_t n, const double* a, const double* b, const double* c, int32_t n_orth,
                         int32_t n_soc, const int32_t* soc_sizes, Problem* out, std::string* err) {
  if (m < 1 || n < 1) return fail(err, "m and n must be >= 1");
  if (!a || !b || !c) return fail(err, "null array argument");
  if (n_orth < 0 || n_soc < 0) return fail(err, "n_orth and n_soc must be >= 0");
  if (n_soc > 0 && !soc_sizes) return fail(err, "soc_sizes is null");
  const int64_t ld = (int64_t(n) + 63) / 64 * 64;
  if (ld * m >= (int64_t(1) << 31) - 1) return fail(err, "dense matrix too large (m * n must stay below 2^31)");
  Problem& p = *out;
  if (!set_vectors_and_cones(m, n, b, c, n_orth, n_soc, soc_sizes, &p, err)) return false;
  p.dense = true;
  p.ld = int32_t(ld);
  p.nnz = int64_t(m) * n;
  p.dhi.assign(size_t(ld) * m, 0.0f);
  bool exact = true;
  for (int32_t i = 0; i < m; ++i)
    for (int32_t j = 0; j < n; ++j) {
      const double v = a[int64_t(i) * n + j];
      if (!std::isfinite(v)) return fail(err, "non-finite matrix value");
      const float h = float(v);
      p.dhi[size_t(i) * ld + j] = h;
      exact = exact && double(h) == v;
    }
  if (!exact) {
    p.dlo.assign(size_t(ld) * m, 0.0f);
    for (int32_t i = 0; i < m; ++i)
      for (int32_t j = 0; j < n; ++j) {
        const double v = a[int64_t(i) * n + j];
        p.dlo[size_t(i) * ld + j] = float(v - double(p.dhi[size_t(i) * ld + j]));
      }
  }
  p.row_perm.resize(m);
  for (int32_t i = 0; i < m; ++i) p.row_perm[i] = i;
  p.b.assign(b, b + m);
  p.c.assign(c, c + n);
  return true;
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
  for (int32_t i = 0; i < m; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) {
      std::ostringstream os;
      os << "row_ptr decreases at row " << i;
      return fail(err, os.str());
    }
  }
  for (int32_t i = 0; i < m; ++i) {
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t j = col_idx[k];
      if (j < 0 || j >= n) {
        std::ostringstream os;
        os << "column index " << j << " out of range in row " << i;
        return fail(err, os.str());
      }
      if (k > row_ptr[i] && j <= col_idx[k - 1]) {
        std::ostringstream os;
        os << "column indices not strictly ascending in row " << i;
        return fail(err, os.str());
      }
      if (!std::isfinite(val[k])) return fail(err, "non-finite matrix value");
    }
  }
  Problem& p = *out;
  if (!set_vectors_and_cones(m, n, b, c, n_orth, n_soc, soc_sizes, &p, err)) return false;
  p.nnz = nnz;

  // rows by decreasing length, ties in the caller's order
  p.row_perm.resize(m);
  for (int32_t i = 0; i < m; ++i) p.row_perm[i] = i;
  std::stable_sort(p.row_perm.begin(), p.row_perm.end(), [&](int32_t a, int32_t b2) {
    return row_ptr[a + 1] - row_ptr[a] > row_ptr[b2 + 1] - row_ptr[b2];
  });
  p.row_ptr.resize(size_t(m) + 1);
  p.col.resize(nnz);
  p.val.resize(nnz);
  p.b.resize(m);
  p.row_ptr[0] = 0;
  for (int32_t i = 0; i < m; ++i) {
    const int32_t o = p.row_perm[i];
    const int64_t k0 = row_ptr[o], len = row_ptr[o + 1] - k0;
    std::copy(col_idx + k0, col_idx + k0 + len, p.col.begin() + p.row_ptr[i]);
    std::copy(val + k0, val + k0 + len, p.val.begin() + p.row_ptr[i]);
    p.row_ptr[i + 1] = p.row_ptr[i] + int32_t(len);
    p.b[i] = b[o];
  }
  p.c.assign(c, c + n);

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
  p.a_blocks = make_row_blocks(p.row_ptr.data(), m, kStageNnz);
  p.t_blocks = make_row_blocks(p.t_row_ptr.data(), n, kStageNnz);
  return true;
}

const SellPair& Problem::sell(int slices) const {
  if (dense) throw AcsError(ACS_ERR_STATE, "a dense problem has no sparse layout");
  if (slices != 1 && slices != kSlices) throw AcsError(ACS_ERR_ARG, "column slices of A must be 1 or 8");
  const int which = slices == 1 ? 0 : 1;
  std::call_once(sell_once_[which], [this, slices, which] {
    auto sp = std::make_unique<SellPair>();
    // A t by column slices [x*w, (x+1)*w), w = ceil(n/slices): slice x holds
    // the nonzeros of its columns, in row order
    const int64_t w = (int64_t(n) + slices - 1) / slices;
    std::vector<int32_t> srp(size_t(slices) * (m + 1), 0), scol(nnz), ssrc(nnz);
    for (int32_t i = 0; i < m; ++i)
      for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) srp[size_t(col[k] / w) * (m + 1) + i + 1]++;
    int32_t base = 0;
    for (int x = 0; x < slices; ++x) {
      int32_t* rp = &srp[size_t(x) * (m + 1)];
      rp[0] = base;
      for (int32_t i = 0; i < m; ++i) rp[i + 1] += rp[i];
      base = rp[m];
    }
    std::vector<int32_t> fill(size_t(slices) * m);
    for (int x = 0; x < slices; ++x)
      for (int32_t i = 0; i < m; ++i) fill[size_t(x) * m + i] = srp[size_t(x) * (m + 1) + i];
    for (int32_t i = 0; i < m; ++i)
      for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        const int32_t pos = fill[size_t(col[k] / w) * m + i]++;
        scol[pos] = col[k];
        ssrc[pos] = k;
      }
    std::vector<const int32_t*> rps;
    std::vector<int32_t> pads;
    for (int x = 0; x < slices; ++x) {
      rps.push_back(&srp[size_t(x) * (m + 1)]);
      pads.push_back(int32_t(std::min<int64_t>(x * w, n - 1)));
    }
    build_sell(rps, m, scol.data(), ssrc.data(), pads, &sp->a);
    build_sell({t_row_ptr.data()}, n, t_col.data(), t_perm.data(), {0}, &sp->t);
    std::string err;
    if (!check_sell(sp->a, m, nnz, &err) || !check_sell(sp->t, n, nnz, &err))
      throw AcsError(ACS_ERR_DEVICE, "internal error in the SELL layout: " + err);
    if (slices == 1) {
      sell_[which] = std::move(sp);
      return;
    }
    // the CG's column order: within each slice, columns in the order the A
    // layout first reads them (padding entries aside), then the columns no
    // entry reads; slice x keeps its columns and its index range [x*w, ...)
    sp->cg_own = true;
    std::vector<int32_t> cinv(size_t(n), -1);
    std::vector<int64_t> cursor(static_cast<size_t>(slices));
    for (int x = 0; x < slices; ++x) cursor[size_t(x)] = int64_t(x) * w;
    const Sell& A = sp->a;
    for (size_t e = 0; e < A.col.size(); ++e) {
      const int32_t c = A.col[e];
      if (A.src[e] >= 0 && cinv[size_t(c)] < 0) cinv[size_t(c)] = int32_t(cursor[size_t(c / w)]++);
    }
    for (int32_t c = 0; c < n; ++c)
      if (cinv[size_t(c)] < 0) cinv[size_t(c)] = int32_t(cursor[size_t(c / w)]++);
    sp->cg_col.assign(size_t(n), 0);
    for (int32_t c = 0; c < n; ++c) sp->cg_col[size_t(cinv[size_t(c)])] = c;
    sp->a_cg_col.resize(A.col.size());
    for (size_t e = 0; e < A.col.size(); ++e) sp->a_cg_col[e] = cinv[size_t(A.col[e])];
    // A^T with its rows in the new order
    std::vector<int32_t> nrp(size_t(n) + 1, 0), ncol(static_cast<size_t>(nnz)), nsrc(static_cast<size_t>(nnz));
    for (int32_t j = 0; j < n; ++j) {
      const int32_t c = sp->cg_col[size_t(j)];
      const int32_t b = t_row_ptr[size_t(c)], len = t_row_ptr[size_t(c) + 1] - b;
      nrp[size_t(j) + 1] = nrp[size_t(j)] + len;
      std::copy(t_col.begin() + b, t_col.begin() + b + len, ncol.begin() + nrp[size_t(j)]);
      std::copy(t_perm.begin() + b, t_perm.begin() + b + len, nsrc.begin() + nrp[size_t(j)]);
    }
    build_sell({nrp.data()}, n, ncol.data(), nsrc.data(), {0}, &sp->t_cg);
    if (!check_sell(sp->t_cg, n, nnz, &err))
      throw AcsError(ACS_ERR_DEVICE, "internal error in the SELL layout: " + err);
    sell_[which] = std::move(sp);
  });
  return *sell_[which];
}

void build_sell(const std::vector<const int32_t*>& rps, int32_t rows, const int32_t* col, const int32_t* src,
                const std::vector<int32_t>& pad, Sell* out, int32_t window, int32_t max_len) {
  Sell& S = *out;
  S = Sell();
  S.slices = int32_t(rps.size());
  S.long_off.push_back(0);
  S.wt_off.push_back(0);
  int64_t used = 0;
  auto append = [&](int32_t c, int32_t s) {
    S.col.push_back(c);
    S.src.push_back(s);
    if (++used >= (int64_t(1) << 31) - 1) throw AcsError(ACS_ERR_ARG, "matrix too large for the SELL layout");
  };
  for (int x = 0; x < S.slices; ++x) {
    const int32_t* rp = rps[x];
    auto len = [&](int32_t i) { return rp[i + 1] - rp[i]; };
    std::vector<int32_t> longs, waves;
    for (int32_t i = 0; i < rows; ++i) {
      if (len(i) > kWaveRowMax)
        longs.push_back(i);
      else if (len(i) > max_len)
        waves.push_back(i);
    }
    auto by_len = [&](int32_t a, int32_t b) { return len(a) > len(b); };
    std::stable_sort(longs.begin(), longs.end(), by_len);
    std::stable_sort(waves.begin(), waves.end(), by_len);
    for (int32_t i : longs) {
      S.long_row.push_back(i);
      S.long_beg.push_back(int32_t(used));
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) append(col[k], src[k]);
      S.long_end.push_back(int32_t(used));
    }
    for (int32_t i : waves) {
      S.wt_ptr.push_back(int32_t(used));
      S.wt_len.push_back(len(i));
      S.wt_row.push_back(i);
      for (int l = 0; l < kSellChunk; ++l) S.chunk_row.push_back(-1);
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) append(col[k], src[k]);
    }
    std::vector<int32_t> win;
    for (int32_t w0 = 0; w0 < rows; w0 += window) {
      win.clear();
      const int32_t w1 = std::min<int32_t>(rows, w0 + window);
      for (int32_t i = w0; i < w1; ++i)
        if (len(i) <= max_len) win.push_back(i);
      std::stable_sort(win.begin(), win.end(), by_len);
      for (size_t c0 = 0; c0 < win.size(); c0 += kSellChunk) {
        const size_t c1 = std::min(win.size(), c0 + kSellChunk);
        int32_t clen = 0;
        for (size_t q = c0; q < c1; ++q) clen = std::max(clen, len(win[q]));
        S.wt_ptr.push_back(int32_t(used));
        S.wt_len.push_back(clen);
        S.wt_row.push_back(-1);
        for (int l = 0; l < kSellChunk; ++l) S.chunk_row.push_back(c0 + l < c1 ? win[c0 + l] : -1);
        for (int32_t k = 0; k < clen; ++k)
          for (int l = 0; l < kSellChunk; ++l) {
            const int32_t i = c0 + l < c1 ? win[c0 + l] : -1;
            if (i >= 0 && k < len(i))
              append(col[rp[i] + k], src[rp[i] + k]);
            else
              append(pad[x], -1);
          }
      }
    }
    S.long_off.push_back(int32_t(S.long_row.size()));
    S.wt_off.push_back(int32_t(S.wt_ptr.size()));
    const int32_t nl = S.long_off[x + 1] - S.long_off[x], nw = S.wt_off[x + 1] - S.wt_off[x];
    S.wg.push_back(nl + (nw + 3) / 4);
    S.wg_max = std::max(S.wg_max, S.wg.back());
  }
}

bool check_sell(const Sell& S, int32_t rows, int64_t entries, std::string* err) {
  if (S.chunk_row.size() != S.wt_ptr.size() * kSellChunk) return fail(err, "chunk rows not one block per task");
  int64_t real = 0;
  std::vector<uint8_t> seen;
  for (int x = 0; x < S.slices; ++x) {
    seen.assign(rows, 0);
    auto mark = [&](int32_t i) {
      if (i < 0 || i >= rows || seen[i]) return false;
      seen[i] = 1;
      return true;
    };
    for (int32_t t = S.long_off[x]; t < S.long_off[x + 1]; ++t) {
      if (!mark(S.long_row[t])) return fail(err, "long row repeated or out of range");
      real += S.long_end[t] - S.long_beg[t];
    }
    for (int32_t t = S.wt_off[x]; t < S.wt_off[x + 1]; ++t) {
      if (S.wt_row[t] >= 0) {
        if (!mark(S.wt_row[t])) return fail(err, "wave row repeated or out of range");
        real += S.wt_len[t];
      } else {
        for (int l = 0; l < kSellChunk; ++l) {
          const int32_t i = S.chunk_row[size_t(t) * kSellChunk + l];
          if (i >= 0 && !mark(i)) return fail(err, "chunk row repeated or out of range");
          for (int32_t k = 0; k < S.wt_len[t]; ++k)
            if (S.src[size_t(S.wt_ptr[t]) + size_t(k) * kSellChunk + l] >= 0) ++real;
        }
      }
    }
    for (int32_t i = 0; i < rows; ++i)
      if (!seen[i]) return fail(err, "row not covered");
  }
  if (real != entries) return fail(err, "entry count mismatch");
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
