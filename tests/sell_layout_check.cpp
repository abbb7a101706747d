// Host check of the row renumbering and of the SELL layouts of the CG
// products (built with g++ against acs_problem.cpp; no GPU).  For each matrix
// it builds the problem, replays the GPU task decomposition on the CPU
// (long rows by workgroup, wave rows, 64-row chunks, every slice and task
// index the kernels visit) and compares the two products with plain CSR sums
// of the caller's matrix.  Prints one line per case and "ok" at the end;
// exits non-zero on the first mismatch.  A "hash" line per case digests
// every array the build produced (to compare builds on different numbers of
// host threads).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "../paper_2103_00736_amd/csrc/acs_internal.h"

namespace acs {
void set_error(const std::string&) {}
}

using namespace acs;

struct Csr {
  int m = 0, n = 0;
  std::vector<int64_t> rp{0};
  std::vector<int32_t> col;
  std::vector<double> val;
};

// sum over the slices/tasks of a Sell layout, emulating the kernels' indexing
static std::vector<double> sell_product(const Sell& S, int rows, const std::vector<double>& vals,
                                        const std::vector<double>& vec, std::vector<int>* writes) {
  std::vector<double> out(size_t(S.slices) * rows, NAN);
  writes->assign(size_t(S.slices) * rows, 0);
  auto emit = [&](int x, int r, double s) {
    out[size_t(x) * rows + r] = s;
    (*writes)[size_t(x) * rows + r]++;
  };
  for (int x = 0; x < S.slices; ++x) {
    const int nl = S.long_off[x + 1] - S.long_off[x];
    for (int lb = 0; lb < S.wg_max; ++lb) {
      if (lb >= S.wg[x]) continue;
      if (lb < nl) {
        const int li = S.long_off[x] + lb;
        double s = 0;
        for (int k = S.long_beg[li]; k < S.long_end[li]; ++k) s += vals[k] * vec[S.col[k]];
        emit(x, S.long_row[li], s);
        continue;
      }
      for (int wv = 0; wv < 4; ++wv) {
        const int t = S.wt_off[x] + (lb - nl) * 4 + wv;
        if (t >= S.wt_off[x + 1]) continue;
        const int ptr = S.wt_ptr[t], len = S.wt_len[t], row = S.wt_row[t];
        if (row >= 0) {
          double s = 0;
          for (int k = ptr; k < ptr + len; ++k) s += vals[k] * vec[S.col[k]];
          emit(x, row, s);
          continue;
        }
        for (int lane = 0; lane < kSellChunk; ++lane) {
          double s = 0;
          for (int k = 0; k < len; ++k) {
            const size_t e = size_t(ptr) + size_t(k) * kSellChunk + lane;
            s += vals[e] * vec[S.col[e]];
          }
          const int r = S.chunk_row[size_t(t) * kSellChunk + lane];
          if (r >= 0) emit(x, r, s);
        }
      }
    }
  }
  return out;
}

static int check_case(const char* name, const Csr& A) {
  Problem p;
  std::string err;
  std::vector<double> b(A.m, 1.0), c(A.n, 1.0);
  if (!build_problem(A.m, A.n, int64_t(A.col.size()), A.rp.data(), A.col.data(), A.val.data(), b.data(), c.data(),
                     A.n, 0, nullptr, &p, &err)) {
    std::printf("%s: build failed: %s\n", name, err.c_str());
    return 1;
  }
  // renumbering: a permutation, lengths non-increasing, rows copied intact
  std::vector<int> seen(A.m, 0);
  for (int i = 0; i < A.m; ++i) {
    const int o = p.row_perm[i];
    if (o < 0 || o >= A.m || seen[o]++) return std::printf("%s: row_perm not a permutation\n", name), 1;
    if (i > 0 && p.row_ptr[i + 1] - p.row_ptr[i] > p.row_ptr[i] - p.row_ptr[i - 1])
      return std::printf("%s: rows not by decreasing length\n", name), 1;
    if (p.row_ptr[i + 1] - p.row_ptr[i] != A.rp[o + 1] - A.rp[o]) return std::printf("%s: row length\n", name), 1;
    for (int k = 0; k < p.row_ptr[i + 1] - p.row_ptr[i]; ++k)
      if (p.col[p.row_ptr[i] + k] != A.col[A.rp[o] + k] || p.val[p.row_ptr[i] + k] != A.val[A.rp[o] + k])
        return std::printf("%s: row contents\n", name), 1;
  }
  std::mt19937_64 rng(3);
  std::normal_distribution<double> N(0, 1);
  std::vector<double> xn(A.n), xm(A.m);
  for (auto& v : xn) v = N(rng);
  for (auto& v : xm) v = N(rng);
  // values of each layout from A's (renumbered) CSR, as the value kernel does
  auto vals_of = [&](const Sell& S) {
    std::vector<double> v(S.col.size());
    for (size_t e = 0; e < v.size(); ++e) v[e] = S.src[e] >= 0 ? p.val[S.src[e]] : 0.0;
    return v;
  };
  // reference products in the caller's order
  std::vector<double> ax(A.m, 0), atx(A.n, 0), ax_abs(A.m, 0), atx_abs(A.n, 0);
  for (int i = 0; i < A.m; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      ax[i] += A.val[k] * xn[A.col[k]];
      ax_abs[i] += std::fabs(A.val[k] * xn[A.col[k]]);
      atx[A.col[k]] += A.val[k] * xm[i];
      atx_abs[A.col[k]] += std::fabs(A.val[k] * xm[i]);
    }
  // A x with 1 and with kSlices column slices: slices summed in order,
  // written back through row_perm
  std::vector<int> writes;
  for (const int slices : {1, kSlices}) {
    const SellPair& sa = p.sell(slices);
    if (sa.a.slices != slices) return std::printf("%s: %d slices asked, %d built\n", name, slices, sa.a.slices), 1;
    std::vector<double> part = sell_product(sa.a, A.m, vals_of(sa.a), xn, &writes);
    for (int w : writes)
      if (w != 1) return std::printf("%s: A side output written %d times (%d slices)\n", name, w, slices), 1;
    const int64_t w = (int64_t(A.n) + slices - 1) / slices;
    for (int i = 0; i < A.m; ++i) {
      double s = 0;
      for (int x = 0; x < slices; ++x) s += part[size_t(x) * A.m + i];
      const int o = p.row_perm[i];
      if (std::fabs(s - ax[o]) > 1e-12 * (ax_abs[o] + 1e-300))
        return std::printf("%s: A x row %d (%d slices)\n", name, o, slices), 1;
    }
    // every A-side entry lies in its slice's column range
    for (int x = 0; x < slices; ++x) {
      for (int t = sa.a.wt_off[x]; t < sa.a.wt_off[x + 1]; ++t) {
        const int64_t span = sa.a.wt_row[t] >= 0 ? sa.a.wt_len[t] : int64_t(sa.a.wt_len[t]) * kSellChunk;
        for (int64_t e = sa.a.wt_ptr[t]; e < sa.a.wt_ptr[t] + span; ++e)
          if (sa.a.col[e] / w != x) return std::printf("%s: entry outside slice %d\n", name, x), 1;
      }
    }
    // one slice: the CG runs on these layouts themselves
    if (slices == 1) {
      if (sa.cg_own || !sa.cg_col.empty() || !sa.a_cg_col.empty() || !sa.t_cg.col.empty())
        return std::printf("%s: one slice has its own CG layouts\n", name), 1;
      continue;
    }
    // the CG's column numbering: a permutation that keeps every column in its
    // slice, numbered in the order of first reading by the A layout
    if (!sa.cg_own || int(sa.cg_col.size()) != A.n || sa.a_cg_col.size() != sa.a.col.size())
      return std::printf("%s: CG numbering sizes (%d slices)\n", name, slices), 1;
    std::vector<int> cinv(A.n, -1);
    for (int j = 0; j < A.n; ++j) {
      const int c = sa.cg_col[j];
      if (c < 0 || c >= A.n || cinv[c] >= 0) return std::printf("%s: cg_col not a permutation\n", name), 1;
      if (c / w != j / w) return std::printf("%s: cg_col leaves its slice\n", name), 1;
      cinv[c] = j;
    }
    std::vector<int64_t> next(slices);
    for (int x = 0; x < slices; ++x) next[x] = int64_t(x) * w;
    std::vector<char> met(A.n, 0);
    for (size_t e = 0; e < sa.a.col.size(); ++e) {
      if (sa.a_cg_col[e] != cinv[sa.a.col[e]]) return std::printf("%s: a_cg_col entry %zu\n", name, e), 1;
      const int c = sa.a.col[e];
      if (sa.a.src[e] < 0 || met[c]) continue;
      met[c] = 1;
      if (cinv[c] != next[c / w]++) return std::printf("%s: column %d out of first-reading order\n", name, c), 1;
    }
    // the CG's products: A t with t in the new order, A^T r into the new order
    Sell acg = sa.a;
    acg.col = sa.a_cg_col;
    std::vector<double> xn_cg(A.n);
    for (int j = 0; j < A.n; ++j) xn_cg[j] = xn[sa.cg_col[j]];
    part = sell_product(acg, A.m, vals_of(sa.a), xn_cg, &writes);
    for (int i = 0; i < A.m; ++i) {
      double s = 0;
      for (int x = 0; x < slices; ++x) s += part[size_t(x) * A.m + i];
      const int o = p.row_perm[i];
      if (std::fabs(s - ax[o]) > 1e-12 * (ax_abs[o] + 1e-300))
        return std::printf("%s: CG A t row %d (%d slices)\n", name, o, slices), 1;
    }
    std::vector<double> xm_i(A.m);
    for (int i = 0; i < A.m; ++i) xm_i[i] = xm[p.row_perm[i]];
    std::vector<double> tc = sell_product(sa.t_cg, A.n, vals_of(sa.t_cg), xm_i, &writes);
    for (int wv : writes)
      if (wv != 1) return std::printf("%s: CG A^T side output written %d times\n", name, wv), 1;
    for (int j = 0; j < A.n; ++j) {
      const int c = sa.cg_col[j];
      if (std::fabs(tc[j] - atx[c]) > 1e-12 * (atx_abs[c] + 1e-300))
        return std::printf("%s: CG A^T r col %d (%d slices)\n", name, c, slices), 1;
    }
  }
  const SellPair& sp = p.sell(kSlices);
  // A^T x: input in internal order
  std::vector<double> xm_int(A.m);
  for (int i = 0; i < A.m; ++i) xm_int[i] = xm[p.row_perm[i]];
  std::vector<double> t = sell_product(sp.t, A.n, vals_of(sp.t), xm_int, &writes);
  for (int wv : writes)
    if (wv != 1) return std::printf("%s: A^T side output written %d times\n", name, wv), 1;
  for (int j = 0; j < A.n; ++j)
    if (std::fabs(t[j] - atx[j]) > 1e-12 * (atx_abs[j] + 1e-300)) return std::printf("%s: A^T x col %d\n", name, j), 1;
  const double pad_a = double(sp.a.col.size()) / std::max<double>(1, A.col.size());
  const double pad_t = double(sp.t.col.size()) / std::max<double>(1, A.col.size());
  std::printf("%s: m=%d n=%d nnz=%zu stored A %.3fx A^T %.3fx long %zu/%zu wave tasks %zu/%zu\n", name, A.m, A.n,
              A.col.size(), pad_a, pad_t, sp.a.long_row.size(), sp.t.long_row.size(), sp.a.wt_ptr.size(),
              sp.t.wt_ptr.size());
  // FNV-1a over everything the problem build and both layouts produced, so
  // that builds on different numbers of host threads can be compared
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const std::vector<int32_t>& v) {
    for (int32_t x : v) {
      h ^= uint32_t(x);
      h *= 1099511628211ull;
    }
    h ^= v.size();
    h *= 1099511628211ull;
  };
  auto mix_sell = [&](const Sell& S) {
    for (const auto* v : {&S.long_off, &S.long_row, &S.long_beg, &S.long_end, &S.wt_off, &S.wt_ptr, &S.wt_len,
                          &S.wt_row, &S.chunk_row, &S.col, &S.src, &S.wg})
      mix(*v);
  };
  mix(p.row_perm);
  mix(p.row_ptr);
  mix(p.col);
  mix(p.t_row_ptr);
  mix(p.t_col);
  mix(p.t_perm);
  for (const int slices : {1, kSlices}) {
    const SellPair& q = p.sell(slices);
    mix_sell(q.a);
    mix_sell(q.t);
    mix_sell(q.t_cg);
    mix(q.a_cg_col);
    mix(q.cg_col);
  }
  std::printf("hash %s %016llx\n", name, (unsigned long long)h);
  return 0;
}

// rows drawn with Chung-Lu weights (power law), `per` distinct rows per column
static Csr powerlaw(int m, int n, int per, uint64_t seed) {
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(0, 1);
  std::vector<double> cw(m);
  double acc = 0;
  for (int i = 0; i < m; ++i) cw[i] = (acc += std::pow(1 - U(rng), -1.0 / 1.5));
  std::vector<std::vector<int>> rows(m);
  for (int j = 0; j < n; ++j) {
    std::set<int> got;
    while (int(got.size()) < std::min(per, m)) {
      int r = int(std::upper_bound(cw.begin(), cw.end(), U(rng) * acc) - cw.begin());
      got.insert(std::min(r, m - 1));
    }
    for (int r : got) rows[r].push_back(j);
  }
  Csr A;
  A.m = m;
  A.n = n;
  std::normal_distribution<double> N(0, 1);
  for (int i = 0; i < m; ++i) {
    for (int j : rows[i]) {
      A.col.push_back(j);
      A.val.push_back(N(rng));
    }
    A.rp.push_back(int64_t(A.col.size()));
  }
  return A;
}

// explicit rows: lengths chosen to hit every task kind and boundary
static Csr edges(uint64_t seed) {
  std::mt19937_64 rng(seed);
  const int n = 40000;
  std::vector<int> lens = {0, 1, 31, 32, 33, 64, 65, 2047, 2048, 2049, 5000, 0, 0, 7, 3};
  for (int i = 0; i < 5000; ++i) lens.push_back(int(rng() % 12));
  for (int i = 0; i < 300; ++i) lens.push_back(20 + int(rng() % 200));
  Csr A;
  A.m = int(lens.size());
  A.n = n;
  std::normal_distribution<double> N(0, 1);
  for (int L : lens) {
    std::set<int> cols;
    while (int(cols.size()) < L) cols.insert(int(rng() % n));
    for (int j : cols) {
      A.col.push_back(j);
      A.val.push_back(N(rng));
    }
    A.rp.push_back(int64_t(A.col.size()));
  }
  // one dense column (a long row of A^T) and a band of wave-length columns
  std::vector<std::vector<int>> rows(A.m);
  for (int i = 0; i < A.m; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) rows[i].push_back(A.col[k]);
  for (int i = 0; i < A.m; i += 2) rows[i].push_back(17);
  for (int i = 0; i < A.m; i += 50) rows[i].push_back(23);
  Csr B;
  B.m = A.m;
  B.n = n;
  for (int i = 0; i < A.m; ++i) {
    std::sort(rows[i].begin(), rows[i].end());
    rows[i].erase(std::unique(rows[i].begin(), rows[i].end()), rows[i].end());
    for (int j : rows[i]) {
      B.col.push_back(j);
      B.val.push_back(N(rng));
    }
    B.rp.push_back(int64_t(B.col.size()));
  }
  return B;
}

int main() {
  int bad = 0;
  bad |= check_case("powerlaw 20000x80000", powerlaw(20000, 80000, 5, 1));
  bad |= check_case("powerlaw 3000x6000 per 8", powerlaw(3000, 6000, 8, 2));
  bad |= check_case("edges", edges(4));
  Csr tiny;
  tiny.m = 1;
  tiny.n = 3;
  tiny.rp = {0, 2};
  tiny.col = {0, 2};
  tiny.val = {1.5, -2.0};
  bad |= check_case("one row", tiny);
  Csr empty;
  empty.m = 3;
  empty.n = 5;
  empty.rp = {0, 0, 0, 0};
  bad |= check_case("no nonzeros", empty);
  if (bad) return 1;
  std::printf("ok\n");
  return 0;
}
