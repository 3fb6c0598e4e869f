#include "host_csr.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <stdexcept>
#include <thread>

namespace fsi {

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& f, int64_t min_n) {
  if (n <= 0) return;
  unsigned hw = std::thread::hardware_concurrency();
  int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 1, 32));
  if (n < min_n || nt == 1) {
    f(0, n);
    return;
  }
  nt = std::min<int64_t>(nt, n);
  std::vector<std::thread> th;
  th.reserve(nt);
  for (int64_t t = 0; t < nt; ++t) {
    int64_t b = n * t / nt, e = n * (t + 1) / nt;
    th.emplace_back([=, &f] { f(b, e); });
  }
  for (auto& t : th) t.join();
}

std::string csr_check(int64_t nrows, int64_t ncols, int64_t nnz, const int64_t* rp, const int32_t* ci,
                      const double* v) {
  char buf[256];
  if (nrows < 0 || ncols < 0 || nnz < 0) return "negative size";
  if (ncols >= (int64_t(1) << 31)) return "ncols does not fit int32 columns";
  if (!rp) return "NULL row pointer";
  if (nnz > 0 && (!ci || !v)) return "NULL column or value array";
  if (rp[0] != 0) return "rowptr[0] != 0";
  if (rp[nrows] != nnz) {
    std::snprintf(buf, sizeof buf, "rowptr[nrows] = %lld != nnz = %lld", (long long)rp[nrows], (long long)nnz);
    return buf;
  }
  for (int64_t i = 0; i < nrows; ++i)
    if (rp[i + 1] < rp[i]) {
      std::snprintf(buf, sizeof buf, "rowptr decreases at row %lld", (long long)i);
      return buf;
    }
  // rows checked on the host threads; the first failing row (in row order)
  // is reported, whatever the thread count
  std::atomic<int64_t> bad{nrows};
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e && i < bad.load(); ++i) {
      bool ok = true;
      for (int64_t k = rp[i]; k < rp[i + 1] && ok; ++k)
        ok = ci[k] >= 0 && ci[k] < ncols && (k == rp[i] || ci[k] > ci[k - 1]) && std::isfinite(v[k]);
      if (!ok) {
        int64_t cur = bad.load();
        while (i < cur && !bad.compare_exchange_weak(cur, i)) {
        }
        return;
      }
    }
  }, int64_t(1) << 14);
  const int64_t i = bad.load();
  if (i == nrows) return "";
  for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
    if (ci[k] < 0 || ci[k] >= ncols) {
      std::snprintf(buf, sizeof buf, "column %d out of range in row %lld", ci[k], (long long)i);
      return buf;
    }
    if (k > rp[i] && ci[k] <= ci[k - 1]) {
      std::snprintf(buf, sizeof buf, "columns not strictly increasing in row %lld", (long long)i);
      return buf;
    }
    if (!std::isfinite(v[k])) {
      std::snprintf(buf, sizeof buf, "non-finite value in row %lld", (long long)i);
      return buf;
    }
  }
  return "invalid row";
}

HCsr csr_copy(int64_t nrows, int64_t ncols, const int64_t* rp, const int32_t* ci, const double* v) {
  HCsr A;
  A.nrows = nrows;
  A.ncols = ncols;
  A.rp.assign(rp, rp + nrows + 1);
  A.ci.assign(ci, ci + rp[nrows]);
  A.v.assign(v, v + rp[nrows]);
  return A;
}

HCsr transpose(const HCsr& A) {
  HCsr T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.rp.assign(T.nrows + 1, 0);
  T.ci.resize(A.nnz());
  T.v.resize(A.nnz());
  // row ranges of A on nt host threads, each with its own column counts (so
  // at most 256 MiB of counts); a thread's entries of column c go after those
  // of the threads before it, so every row of T stays in ascending order
  unsigned hw = std::thread::hardware_concurrency();
  int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 1, 32));
  nt = std::min<int64_t>(nt, std::max<int64_t>(1, (int64_t(1) << 25) / std::max<int64_t>(A.ncols, 1)));
  if (A.nnz() < (int64_t(1) << 20)) nt = 1;
  std::vector<std::vector<int64_t>> pos(nt, std::vector<int64_t>(A.ncols, 0));
  auto range = [&](int64_t t, int64_t& b, int64_t& e) {
    b = A.nrows * t / nt;
    e = A.nrows * (t + 1) / nt;
  };
  parallel_for(nt, [&](int64_t t0, int64_t t1) {
    for (int64_t t = t0; t < t1; ++t) {
      int64_t b, e;
      range(t, b, e);
      for (int64_t k = A.rp[b]; k < A.rp[e]; ++k) pos[t][A.ci[k]]++;
    }
  }, 2);
  int64_t off = 0;
  for (int64_t c = 0; c < A.ncols; ++c) {
    T.rp[c] = off;
    for (int64_t t = 0; t < nt; ++t) {
      const int64_t n = pos[t][c];
      pos[t][c] = off;
      off += n;
    }
  }
  T.rp[A.ncols] = off;
  parallel_for(nt, [&](int64_t t0, int64_t t1) {
    for (int64_t t = t0; t < t1; ++t) {
      int64_t b, e;
      range(t, b, e);
      std::vector<int64_t>& p = pos[t];
      for (int64_t i = b; i < e; ++i)
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
          const int64_t q = p[A.ci[k]]++;
          T.ci[q] = int32_t(i);
          T.v[q] = A.v[k];
        }
    }
  }, 2);
  return T;
}

void spgemm_row(const HCsr& A, const HCsr& B, int64_t i, SpgemmWork& w, std::vector<int32_t>& oc,
                std::vector<double>& ov) {
  if (w.acc.size() != size_t(B.ncols)) {
    w.acc.assign(B.ncols, 0.0);
    w.mark.assign(B.ncols, -1);
  }
  w.cols.clear();
  for (int64_t ka = A.rp[i]; ka < A.rp[i + 1]; ++ka) {
    const int32_t k = A.ci[ka];
    const double a = A.v[ka];
    for (int64_t kb = B.rp[k]; kb < B.rp[k + 1]; ++kb) {
      const int32_t j = B.ci[kb];
      if (w.mark[j] != i) {
        w.mark[j] = i;
        w.acc[j] = 0.0;
        w.cols.push_back(j);
      }
      w.acc[j] += a * B.v[kb];
    }
  }
  std::sort(w.cols.begin(), w.cols.end());
  for (int32_t j : w.cols) {
    if (w.acc[j] != 0.0) {
      oc.push_back(j);
      ov.push_back(w.acc[j]);
    }
  }
}

HCsr spgemm(const HCsr& A, const HCsr& B) {
  HCsr C;
  C.nrows = A.nrows;
  C.ncols = B.ncols;
  const int64_t n = A.nrows;
  // chunked rows: each chunk builds its own arrays, then they are concatenated;
  // the chunks (at least 256 rows each) run on the host threads, and every
  // row is formed the same way on any thread
  const int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>(256, n / 256));
  std::vector<std::vector<int32_t>> cc(nchunk);
  std::vector<std::vector<double>> cv(nchunk);
  std::vector<int64_t> rowlen(n, 0);
  parallel_for(nchunk, [&](int64_t cb, int64_t ce) {
    SpgemmWork w;
    for (int64_t ch = cb; ch < ce; ++ch) {
      int64_t r0 = n * ch / nchunk, r1 = n * (ch + 1) / nchunk;
      for (int64_t i = r0; i < r1; ++i) {
        const size_t before = cc[ch].size();
        spgemm_row(A, B, i, w, cc[ch], cv[ch]);
        rowlen[i] = int64_t(cc[ch].size() - before);
      }
    }
  }, 2);
  C.rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) C.rp[i + 1] = C.rp[i] + rowlen[i];
  C.ci.reserve(C.rp[n]);
  C.v.reserve(C.rp[n]);
  for (int64_t ch = 0; ch < nchunk; ++ch) {
    C.ci.insert(C.ci.end(), cc[ch].begin(), cc[ch].end());
    C.v.insert(C.v.end(), cv[ch].begin(), cv[ch].end());
  }
  return C;
}

HCsr add(const HCsr& A, const HCsr& B, double alpha) {
  // merge of row i of A and alpha * row i of B: out == nullptr only counts
  auto merge = [&](int64_t i, int32_t* oc, double* ov) {
    int64_t ka = A.rp[i], kb = B.rp[i], n = 0;
    while (ka < A.rp[i + 1] || kb < B.rp[i + 1]) {
      const int32_t ja = ka < A.rp[i + 1] ? A.ci[ka] : INT32_MAX;
      const int32_t jb = kb < B.rp[i + 1] ? B.ci[kb] : INT32_MAX;
      double val;
      int32_t j;
      if (ja == jb) { j = ja; val = A.v[ka++] + alpha * B.v[kb++]; }
      else if (ja < jb) { j = ja; val = A.v[ka++]; }
      else { j = jb; val = alpha * B.v[kb++]; }
      if (val != 0.0) {
        if (oc) { oc[n] = j; ov[n] = val; }
        ++n;
      }
    }
    return n;
  };
  return build_rows(A.nrows, A.ncols, [&](int64_t i) { return merge(i, nullptr, nullptr); },
                    [&](int64_t i, int32_t* oc, double* ov) { merge(i, oc, ov); });
}

HCsr sub_block(const HCsr& A, int64_t r0, int64_t r1, int64_t c0, int64_t c1) {
  // the columns of a row are sorted: the block's part is one contiguous run
  auto run = [&](int64_t i, int64_t& k0, int64_t& k1) {
    const int32_t* b = A.ci.data() + A.rp[i];
    const int32_t* e = A.ci.data() + A.rp[i + 1];
    k0 = std::lower_bound(b, e, int64_t(c0), [](int32_t c, int64_t x) { return c < x; }) - A.ci.data();
    k1 = std::lower_bound(b, e, int64_t(c1), [](int32_t c, int64_t x) { return c < x; }) - A.ci.data();
  };
  return build_rows(r1 - r0, c1 - c0,
                    [&](int64_t q) {
                      int64_t k0, k1;
                      run(r0 + q, k0, k1);
                      return k1 - k0;
                    },
                    [&](int64_t q, int32_t* oc, double* ov) {
                      int64_t k0, k1;
                      run(r0 + q, k0, k1);
                      for (int64_t k = k0; k < k1; ++k) {
                        *oc++ = int32_t(A.ci[k] - c0);
                        *ov++ = A.v[k];
                      }
                    });
}

void drop_zeros(HCsr& A) {
  HCsr C = build_rows(A.nrows, A.ncols,
                      [&](int64_t i) {
                        int64_t n = 0;
                        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) n += A.v[k] != 0.0;
                        return n;
                      },
                      [&](int64_t i, int32_t* oc, double* ov) {
                        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
                          if (A.v[k] != 0.0) {
                            *oc++ = A.ci[k];
                            *ov++ = A.v[k];
                          }
                      });
  A = std::move(C);
}

void scale_rows(HCsr& A, const std::vector<double>& s) {
  parallel_for(A.nrows, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i)
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) A.v[k] = s[i] * A.v[k];
  });
}

void scale_cols(HCsr& A, const std::vector<double>& s) {
  parallel_for(A.nrows, [&](int64_t b, int64_t e) {
    for (int64_t k = A.rp[b]; k < A.rp[e]; ++k) A.v[k] = A.v[k] * s[A.ci[k]];
  });
}

std::vector<double> diagonal(const HCsr& A) {
  std::vector<double> d(A.nrows, 0.0);
  parallel_for(A.nrows, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i)
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
        if (A.ci[k] == i) d[i] = A.v[k];
  });
  return d;
}

void matvec(const HCsr& A, const double* x, double* y) {
  // rows on the host threads; each row summed in storage order on any thread
  parallel_for(A.nrows, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      double s = 0.0;
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) s += A.v[k] * x[A.ci[k]];
      y[i] = s;
    }
  }, int64_t(1) << 15);
}

HCsr group_rows(const HCsr& A, int64_t r0, int64_t r1, int g, std::vector<double>& val) {
  // merge of the g sorted column lists of group q: cols == nullptr only counts
  auto merge = [&](int64_t q, int32_t* cols, double* vals) {
    const int64_t row = r0 + q * g;
    int64_t k[8];
    for (int r = 0; r < g; ++r) k[r] = A.rp[row + r];
    int64_t n = 0;
    while (true) {
      int32_t c = INT32_MAX;
      for (int r = 0; r < g; ++r)
        if (k[r] < A.rp[row + r + 1]) c = std::min(c, A.ci[k[r]]);
      if (c == INT32_MAX) break;
      if (cols) cols[n] = c;
      for (int r = 0; r < g; ++r) {
        const bool has = k[r] < A.rp[row + r + 1] && A.ci[k[r]] == c;
        if (cols) vals[n * g + r] = has ? A.v[k[r]] : 0.0;
        if (has) ++k[r];
      }
      ++n;
    }
    return n;
  };
  if (g < 1 || g > 8) throw std::invalid_argument("group_rows: group size must be in 1..8");
  HCsr G;
  G.nrows = (r1 - r0) / g;
  G.ncols = A.ncols;
  G.rp.assign(G.nrows + 1, 0);
  parallel_for(G.nrows, [&](int64_t b, int64_t e) {
    for (int64_t q = b; q < e; ++q) G.rp[q + 1] = merge(q, nullptr, nullptr);
  });
  for (int64_t q = 0; q < G.nrows; ++q) G.rp[q + 1] += G.rp[q];
  G.ci.resize(G.rp[G.nrows]);
  val.assign(size_t(G.rp[G.nrows]) * g, 0.0);
  parallel_for(G.nrows, [&](int64_t b, int64_t e) {
    for (int64_t q = b; q < e; ++q) merge(q, G.ci.data() + G.rp[q], val.data() + size_t(G.rp[q]) * g);
  });
  return G;
}

int64_t group_entries(const HCsr& A, int64_t r0, int64_t r1, int g) {
  std::atomic<int64_t> total{0};
  parallel_for((r1 - r0) / g, [&](int64_t q0, int64_t q1) {
    int64_t cnt = 0;
    std::vector<int64_t> k(g);
    for (int64_t q = q0; q < q1; ++q) {
      const int64_t row = r0 + q * g;
      for (int r = 0; r < g; ++r) k[r] = A.rp[row + r];
      while (true) {
        int32_t c = INT32_MAX;
        for (int r = 0; r < g; ++r)
          if (k[r] < A.rp[row + r + 1]) c = std::min(c, A.ci[k[r]]);
        if (c == INT32_MAX) break;
        ++cnt;
        for (int r = 0; r < g; ++r)
          if (k[r] < A.rp[row + r + 1] && A.ci[k[r]] == c) ++k[r];
      }
    }
    total += cnt;
  });
  return total.load();
}

}  // namespace fsi
