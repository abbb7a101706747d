// Problem validation, CSR transpose and row-block partitioning (host only).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <exception>
#include <mutex>
#include <sstream>
#include <system_error>
#include <thread>

#include "acs_internal.h"

namespace acs {

// fn(i) for i in [0, count), on up to host_threads() threads when `big`
// (else inline); each i must write only what it owns.  Fewer threads when the
// system refuses more; the first exception is rethrown after the join.
static int64_t host_threads() {  // kHostThreads, the machine's, or ACS_HOST_THREADS if smaller
  static const int64_t n = [] {
    int64_t t = std::min<int64_t>(kHostThreads, std::max<int64_t>(1, int64_t(std::thread::hardware_concurrency())));
    if (const char* e = std::getenv("ACS_HOST_THREADS")) {
      const long v = std::strtol(e, nullptr, 10);
      if (v >= 1) t = std::min<int64_t>(t, v);
    }
    return t;
  }();
  return n;
}

template <class F>
static void parallel_for(int64_t count, bool big, F&& fn) {
  const int64_t want = big ? std::min<int64_t>(host_threads(), count) : 1;
  if (want <= 1) {
    for (int64_t i = 0; i < count; ++i) fn(i);
    return;
  }
  std::atomic<int64_t> next{0};
  std::exception_ptr first;
  std::mutex mu;
  auto body = [&] {
    try {
      for (int64_t i; (i = next.fetch_add(1)) < count;) fn(i);
    } catch (...) {
      std::lock_guard<std::mutex> lk(mu);
      if (!first) first = std::current_exception();
      next = count;
    }
  };
  std::vector<std::thread> pool;
  for (int64_t t = 1; t < want; ++t) {
    try {
      pool.emplace_back(body);
    } catch (const std::system_error&) {
      break;
    }
  }
  body();
  for (auto& th : pool) th.join();
  if (first) std::rethrow_exception(first);
}

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
  const bool big = int64_t(m) + nnz >= (int64_t(1) << 18);
  p.row_ptr.resize(size_t(m) + 1);
  p.col.resize(nnz);
  p.val.resize(nnz);
  p.b.resize(m);
  p.row_ptr[0] = 0;
  for (int32_t i = 0; i < m; ++i) {
    const int32_t o = p.row_perm[i];
    p.row_ptr[i + 1] = p.row_ptr[i] + int32_t(row_ptr[o + 1] - row_ptr[o]);
    p.b[i] = b[o];
  }
  const int64_t rb = 8192;
  parallel_for((int64_t(m) + rb - 1) / rb, big, [&](int64_t r) {
    const int32_t i1 = int32_t(std::min<int64_t>(m, (r + 1) * rb));
    for (int32_t i = int32_t(r * rb); i < i1; ++i) {
      const int32_t o = p.row_perm[i];
      const int64_t k0 = row_ptr[o], len = row_ptr[o + 1] - k0;
      std::copy(col_idx + k0, col_idx + k0 + len, p.col.begin() + p.row_ptr[i]);
      std::copy(val + k0, val + k0 + len, p.val.begin() + p.row_ptr[i]);
    }
  });
  p.c.assign(c, c + n);

  // transpose pattern by counting sort over columns (columns ascending in A^T rows = rows of A);
  // each host thread owns a range of columns and scans every entry, so each A^T row is filled
  // by one thread in row order
  const int64_t ranges = big ? std::min<int64_t>(host_threads(), int64_t(n)) : 1;
  const int64_t cw = (int64_t(n) + ranges - 1) / ranges;
  p.t_row_ptr.assign(size_t(n) + 1, 0);
  parallel_for(ranges, big, [&](int64_t r) {
    const int32_t c0 = int32_t(r * cw), c1 = int32_t(std::min<int64_t>(n, (r + 1) * cw));
    for (int64_t k = 0; k < nnz; ++k) {
      const int32_t j = p.col[k];
      if (j >= c0 && j < c1) p.t_row_ptr[j + 1]++;
    }
  });
  for (int32_t j = 0; j < n; ++j) p.t_row_ptr[j + 1] += p.t_row_ptr[j];
  p.t_col.resize(nnz);
  p.t_perm.resize(nnz);
  std::vector<int32_t> fill(p.t_row_ptr.begin(), p.t_row_ptr.end() - 1);
  parallel_for(ranges, big, [&](int64_t r) {
    const int32_t c0 = int32_t(r * cw), c1 = int32_t(std::min<int64_t>(n, (r + 1) * cw));
    for (int32_t i = 0; i < m; ++i) {
      for (int32_t k = p.row_ptr[i]; k < p.row_ptr[i + 1]; ++k) {
        const int32_t j = p.col[k];
        if (j < c0 || j >= c1) continue;
        const int32_t pos = fill[j]++;
        p.t_col[pos] = i;
        p.t_perm[pos] = k;
      }
    }
  });
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
    const bool big = int64_t(m) + nnz >= (int64_t(1) << 18);
    // blocks of rows (or columns, entries) for the host threads
    const int64_t rb = 8192;
    const int64_t nrb = (int64_t(m) + rb - 1) / rb;
    std::vector<int32_t> srp(size_t(slices) * (m + 1), 0), scol(nnz), ssrc(nnz);
    parallel_for(nrb, big, [&](int64_t r) {
      const int32_t i1 = int32_t(std::min<int64_t>(m, (r + 1) * rb));
      for (int32_t i = int32_t(r * rb); i < i1; ++i)
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) srp[size_t(col[k] / w) * (m + 1) + i + 1]++;
    });
    int32_t base = 0;
    for (int x = 0; x < slices; ++x) {
      int32_t* rp = &srp[size_t(x) * (m + 1)];
      rp[0] = base;
      for (int32_t i = 0; i < m; ++i) rp[i + 1] += rp[i];
      base = rp[m];
    }
    parallel_for(nrb, big, [&](int64_t r) {  // each row's entries go to its own positions
      const int32_t i1 = int32_t(std::min<int64_t>(m, (r + 1) * rb));
      int32_t at[kSlices];
      for (int32_t i = int32_t(r * rb); i < i1; ++i) {
        for (int x = 0; x < slices; ++x) at[x] = srp[size_t(x) * (m + 1) + i];
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
          const int32_t pos = at[col[k] / w]++;
          scol[pos] = col[k];
          ssrc[pos] = k;
        }
      }
    });
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
    const Sell& A = sp->a;
    // entries of slice x: [sbeg[x], sbeg[x+1]) (longs, wave rows, then chunks)
    std::vector<int64_t> sbeg(size_t(slices) + 1, int64_t(A.col.size()));
    for (int x = slices - 1; x >= 0; --x) {
      if (A.long_off[x + 1] > A.long_off[x])
        sbeg[x] = A.long_beg[A.long_off[x]];
      else if (A.wt_off[x + 1] > A.wt_off[x])
        sbeg[x] = A.wt_ptr[A.wt_off[x]];
      else
        sbeg[x] = sbeg[x + 1];
    }
    std::vector<int32_t> cinv(size_t(n), -1);
    parallel_for(slices, big, [&](int64_t xi) {  // a slice's entries read only its own columns
      const int x = int(xi);
      int64_t next = int64_t(x) * w;
      for (int64_t e = sbeg[x]; e < sbeg[x + 1]; ++e) {
        const int32_t c = A.col[size_t(e)];
        if (A.src[size_t(e)] >= 0 && cinv[size_t(c)] < 0) cinv[size_t(c)] = int32_t(next++);
      }
      const int64_t c1 = std::min<int64_t>(n, (int64_t(x) + 1) * w);
      for (int64_t c = int64_t(x) * w; c < c1; ++c)
        if (cinv[size_t(c)] < 0) cinv[size_t(c)] = int32_t(next++);
    });
    sp->cg_col.assign(size_t(n), 0);
    for (int32_t c = 0; c < n; ++c) sp->cg_col[size_t(cinv[size_t(c)])] = c;
    sp->a_cg_col.resize(A.col.size());
    const int64_t eb = int64_t(1) << 16;
    parallel_for((int64_t(A.col.size()) + eb - 1) / eb, big, [&](int64_t r) {
      const int64_t e1 = std::min<int64_t>(int64_t(A.col.size()), (r + 1) * eb);
      for (int64_t e = r * eb; e < e1; ++e) sp->a_cg_col[size_t(e)] = cinv[size_t(A.col[size_t(e)])];
    });
    // A^T with its rows in the new order
    std::vector<int32_t> nrp(size_t(n) + 1, 0), ncol(static_cast<size_t>(nnz)), nsrc(static_cast<size_t>(nnz));
    for (int32_t j = 0; j < n; ++j) {
      const int32_t c = sp->cg_col[size_t(j)];
      nrp[size_t(j) + 1] = nrp[size_t(j)] + (t_row_ptr[size_t(c) + 1] - t_row_ptr[size_t(c)]);
    }
    parallel_for((int64_t(n) + rb - 1) / rb, big, [&](int64_t r) {
      const int32_t j1 = int32_t(std::min<int64_t>(n, (r + 1) * rb));
      for (int32_t j = int32_t(r * rb); j < j1; ++j) {
        const int32_t c = sp->cg_col[size_t(j)];
        const int32_t b0 = t_row_ptr[size_t(c)], len = t_row_ptr[size_t(c) + 1] - b0;
        std::copy(t_col.begin() + b0, t_col.begin() + b0 + len, ncol.begin() + nrp[size_t(j)]);
        std::copy(t_perm.begin() + b0, t_perm.begin() + b0 + len, nsrc.begin() + nrp[size_t(j)]);
      }
    });
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
  const int slices = int(rps.size());
  S.slices = slices;
  int64_t in_entries = 0;
  for (int x = 0; x < slices; ++x) in_entries += int64_t(rps[x][rows]) - rps[x][0];
  const bool big = int64_t(rows) * slices + in_entries >= (int64_t(1) << 18);
  const int nwin = int((int64_t(rows) + window - 1) / window);
  // per slice: long rows and wave rows, longest first (ties in row order)
  struct Head {
    std::vector<int32_t> longs, waves;
    int64_t long_entries = 0, wave_entries = 0;
  };
  std::vector<Head> head(slices);
  parallel_for(slices, big, [&](int64_t xi) {
    const int x = int(xi);
    const int32_t* rp = rps[x];
    auto len = [&](int32_t i) { return rp[i + 1] - rp[i]; };
    Head& h = head[x];
    for (int32_t i = 0; i < rows; ++i) {
      if (len(i) > kWaveRowMax) {
        h.longs.push_back(i);
        h.long_entries += len(i);
      } else if (len(i) > max_len) {
        h.waves.push_back(i);
        h.wave_entries += len(i);
      }
    }
    auto by_len = [&](int32_t a, int32_t b) { return len(a) > len(b); };
    std::stable_sort(h.longs.begin(), h.longs.end(), by_len);
    std::stable_sort(h.waves.begin(), h.waves.end(), by_len);
  });
  // per (slice, window): its short rows, longest first, and the chunks' lengths
  struct Win {
    std::vector<int32_t> rows;
    std::vector<int32_t> clen;
    int64_t entries = 0;
  };
  std::vector<Win> win(size_t(slices) * nwin);
  parallel_for(int64_t(slices) * nwin, big, [&](int64_t u) {
    const int x = int(u / nwin);
    const int32_t w0 = int32_t((u % nwin) * window), w1 = std::min<int32_t>(rows, w0 + window);
    const int32_t* rp = rps[x];
    auto len = [&](int32_t i) { return rp[i + 1] - rp[i]; };
    Win& wv = win[size_t(u)];
    for (int32_t i = w0; i < w1; ++i)
      if (len(i) <= max_len) wv.rows.push_back(i);
    std::stable_sort(wv.rows.begin(), wv.rows.end(), [&](int32_t a, int32_t b) { return len(a) > len(b); });
    for (size_t c0 = 0; c0 < wv.rows.size(); c0 += kSellChunk) {
      int32_t cl = 0;
      for (size_t q = c0; q < std::min(wv.rows.size(), c0 + kSellChunk); ++q) cl = std::max(cl, len(wv.rows[q]));
      wv.clen.push_back(cl);
      wv.entries += int64_t(cl) * kSellChunk;
    }
  });
  // offsets: per slice its long tasks, its wave rows, then its windows' chunks, in that order
  std::vector<int64_t> head_entry(slices), win_entry(win.size());
  std::vector<int32_t> head_task(slices), win_task(win.size());
  int64_t entries = 0;
  int64_t tasks = 0, longs = 0;
  S.long_off.push_back(0);
  S.wt_off.push_back(0);
  for (int x = 0; x < slices; ++x) {
    head_entry[x] = entries;
    head_task[x] = int32_t(tasks);
    entries += head[x].long_entries + head[x].wave_entries;
    tasks += int64_t(head[x].waves.size());
    for (int w = 0; w < nwin; ++w) {
      const size_t u = size_t(x) * nwin + w;
      win_entry[u] = entries;
      win_task[u] = int32_t(tasks);
      entries += win[u].entries;
      tasks += int64_t(win[u].clen.size());
    }
    longs += int64_t(head[x].longs.size());
    if (entries >= (int64_t(1) << 31) - 1) throw AcsError(ACS_ERR_ARG, "matrix too large for the SELL layout");
    S.long_off.push_back(int32_t(longs));
    S.wt_off.push_back(int32_t(tasks));
    const int32_t nl = S.long_off[x + 1] - S.long_off[x], nw = S.wt_off[x + 1] - S.wt_off[x];
    S.wg.push_back(nl + (nw + 3) / 4);
    S.wg_max = std::max(S.wg_max, S.wg.back());
  }
  S.col.resize(size_t(entries));
  S.src.resize(size_t(entries));
  S.long_row.resize(size_t(longs));
  S.long_beg.resize(size_t(longs));
  S.long_end.resize(size_t(longs));
  S.wt_ptr.resize(size_t(tasks));
  S.wt_len.resize(size_t(tasks));
  S.wt_row.resize(size_t(tasks));
  S.chunk_row.assign(size_t(tasks) * kSellChunk, -1);
  // fill: slice heads, then windows, each at its own offsets
  parallel_for(slices, big, [&](int64_t xi) {
    const int x = int(xi);
    const int32_t* rp = rps[x];
    const Head& h = head[x];
    int64_t e = head_entry[x];
    for (size_t q = 0; q < h.longs.size(); ++q) {
      const int32_t i = h.longs[q], t = S.long_off[x] + int32_t(q);
      S.long_row[t] = i;
      S.long_beg[t] = int32_t(e);
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k, ++e) {
        S.col[size_t(e)] = col[k];
        S.src[size_t(e)] = src[k];
      }
      S.long_end[t] = int32_t(e);
    }
    for (size_t q = 0; q < h.waves.size(); ++q) {
      const int32_t i = h.waves[q], t = head_task[x] + int32_t(q);
      S.wt_ptr[t] = int32_t(e);
      S.wt_len[t] = rp[i + 1] - rp[i];
      S.wt_row[t] = i;
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k, ++e) {
        S.col[size_t(e)] = col[k];
        S.src[size_t(e)] = src[k];
      }
    }
  });
  parallel_for(int64_t(slices) * nwin, big, [&](int64_t u) {
    const int x = int(u / nwin);
    const int32_t* rp = rps[x];
    const Win& wv = win[size_t(u)];
    int64_t e = win_entry[size_t(u)];
    for (size_t c = 0; c < wv.clen.size(); ++c) {
      const int32_t t = win_task[size_t(u)] + int32_t(c), cl = wv.clen[c];
      const size_t c0 = c * kSellChunk, c1 = std::min(wv.rows.size(), c0 + kSellChunk);
      S.wt_ptr[t] = int32_t(e);
      S.wt_len[t] = cl;
      S.wt_row[t] = -1;
      for (size_t q = c0; q < c1; ++q) S.chunk_row[size_t(t) * kSellChunk + (q - c0)] = wv.rows[q];
      for (int32_t k = 0; k < cl; ++k)
        for (int l = 0; l < kSellChunk; ++l, ++e) {
          const int32_t i = c0 + l < c1 ? wv.rows[c0 + l] : -1;
          if (i >= 0 && k < rp[i + 1] - rp[i]) {
            S.col[size_t(e)] = col[rp[i] + k];
            S.src[size_t(e)] = src[rp[i] + k];
          } else {
            S.col[size_t(e)] = pad[x];
            S.src[size_t(e)] = -1;
          }
        }
    }
  });
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
