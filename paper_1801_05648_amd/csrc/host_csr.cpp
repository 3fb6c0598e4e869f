#include "host_csr.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
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
  for (int64_t i = 0; i < nrows; ++i) {
    if (rp[i + 1] < rp[i]) {
      std::snprintf(buf, sizeof buf, "rowptr decreases at row %lld", (long long)i);
      return buf;
    }
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
  }
  return "";
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
  for (int64_t k = 0; k < A.nnz(); ++k) T.rp[A.ci[k] + 1]++;
  for (int64_t i = 0; i < T.nrows; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(A.nnz());
  T.v.resize(A.nnz());
  std::vector<int64_t> pos(T.rp.begin(), T.rp.end() - 1);
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      int64_t p = pos[A.ci[k]]++;
      T.ci[p] = int32_t(i);
      T.v[p] = A.v[k];
    }
  return T;
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
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<int64_t> mark(B.ncols, -1);
    std::vector<int32_t> cols;
    for (int64_t ch = cb; ch < ce; ++ch) {
      int64_t r0 = n * ch / nchunk, r1 = n * (ch + 1) / nchunk;
      for (int64_t i = r0; i < r1; ++i) {
        cols.clear();
        for (int64_t ka = A.rp[i]; ka < A.rp[i + 1]; ++ka) {
          const int32_t k = A.ci[ka];
          const double a = A.v[ka];
          for (int64_t kb = B.rp[k]; kb < B.rp[k + 1]; ++kb) {
            const int32_t j = B.ci[kb];
            if (mark[j] != i) {
              mark[j] = i;
              acc[j] = 0.0;
              cols.push_back(j);
            }
            acc[j] += a * B.v[kb];
          }
        }
        std::sort(cols.begin(), cols.end());
        int64_t len = 0;
        for (int32_t j : cols) {
          if (acc[j] != 0.0) {
            cc[ch].push_back(j);
            cv[ch].push_back(acc[j]);
            ++len;
          }
        }
        rowlen[i] = len;
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
  HCsr C;
  C.nrows = A.nrows;
  C.ncols = A.ncols;
  C.rp.assign(A.nrows + 1, 0);
  for (int64_t i = 0; i < A.nrows; ++i) {
    int64_t ka = A.rp[i], kb = B.rp[i];
    while (ka < A.rp[i + 1] || kb < B.rp[i + 1]) {
      int32_t ja = ka < A.rp[i + 1] ? A.ci[ka] : INT32_MAX;
      int32_t jb = kb < B.rp[i + 1] ? B.ci[kb] : INT32_MAX;
      double val;
      int32_t j;
      if (ja == jb) { j = ja; val = A.v[ka++] + alpha * B.v[kb++]; }
      else if (ja < jb) { j = ja; val = A.v[ka++]; }
      else { j = jb; val = alpha * B.v[kb++]; }
      if (val != 0.0) {
        C.ci.push_back(j);
        C.v.push_back(val);
      }
    }
    C.rp[i + 1] = int64_t(C.ci.size());
  }
  return C;
}

HCsr sub_block(const HCsr& A, int64_t r0, int64_t r1, int64_t c0, int64_t c1) {
  HCsr C;
  C.nrows = r1 - r0;
  C.ncols = c1 - c0;
  C.rp.assign(C.nrows + 1, 0);
  for (int64_t i = r0; i < r1; ++i) {
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] >= c0 && A.ci[k] < c1) {
        C.ci.push_back(int32_t(A.ci[k] - c0));
        C.v.push_back(A.v[k]);
      }
    C.rp[i - r0 + 1] = int64_t(C.ci.size());
  }
  return C;
}

void drop_zeros(HCsr& A) {
  int64_t w = 0;
  std::vector<int64_t> rp(A.nrows + 1, 0);
  for (int64_t i = 0; i < A.nrows; ++i) {
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.v[k] != 0.0) {
        A.ci[w] = A.ci[k];
        A.v[w] = A.v[k];
        ++w;
      }
    rp[i + 1] = w;
  }
  A.rp.swap(rp);
  A.ci.resize(w);
  A.v.resize(w);
}

void scale_rows(HCsr& A, const std::vector<double>& s) {
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) A.v[k] = s[i] * A.v[k];
}

void scale_cols(HCsr& A, const std::vector<double>& s) {
  for (int64_t k = 0; k < A.nnz(); ++k) A.v[k] = A.v[k] * s[A.ci[k]];
}

std::vector<double> diagonal(const HCsr& A) {
  std::vector<double> d(A.nrows, 0.0);
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] == i) d[i] = A.v[k];
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
  HCsr G;
  G.nrows = (r1 - r0) / g;
  G.ncols = A.ncols;
  G.rp.assign(G.nrows + 1, 0);
  val.clear();
  std::vector<int64_t> k(g);
  for (int64_t q = 0; q < G.nrows; ++q) {
    const int64_t row = r0 + q * g;
    for (int r = 0; r < g; ++r) k[r] = A.rp[row + r];
    while (true) {  // merge the g sorted column lists
      int32_t c = INT32_MAX;
      for (int r = 0; r < g; ++r)
        if (k[r] < A.rp[row + r + 1]) c = std::min(c, A.ci[k[r]]);
      if (c == INT32_MAX) break;
      G.ci.push_back(c);
      for (int r = 0; r < g; ++r) {
        if (k[r] < A.rp[row + r + 1] && A.ci[k[r]] == c) val.push_back(A.v[k[r]++]);
        else val.push_back(0.0);
      }
    }
    G.rp[q + 1] = int64_t(G.ci.size());
  }
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
