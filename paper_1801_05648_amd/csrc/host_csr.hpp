// Host-side CSR containers and the sparse kernels the preconditioner setup
// needs (transpose, sparse products, sums, sub-blocks).  Setup only: nothing
// here runs inside the solve.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace fsi {

struct HCsr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rp{0};
  std::vector<int32_t> ci;
  std::vector<double> v;
  int64_t nnz() const { return int64_t(ci.size()); }
};

// Run f(begin, end) over [0, n) on the host's hardware threads (on the
// calling thread alone when n < min_n: items too small to pay for threads).
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& f, int64_t min_n = 4096);

// Rows [0, nrows) of a CSR matrix built on the host threads in two passes:
// count(i) gives the length of row i, fill(i, ci, v) writes the row at ci, v.
// Every row is formed the same way on any thread, so the result does not
// depend on the thread count.
template <class Count, class Fill>
HCsr build_rows(int64_t nrows, int64_t ncols, Count&& count, Fill&& fill, int64_t min_n = 4096) {
  HCsr C;
  C.nrows = nrows;
  C.ncols = ncols;
  C.rp.assign(nrows + 1, 0);
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) C.rp[i + 1] = count(i);
  }, min_n);
  for (int64_t i = 0; i < nrows; ++i) C.rp[i + 1] += C.rp[i];
  C.ci.resize(C.rp[nrows]);
  C.v.resize(C.rp[nrows]);
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) fill(i, C.ci.data() + C.rp[i], C.v.data() + C.rp[i]);
  }, min_n);
  return C;
}

// Well-formedness: row pointers, column range, strictly increasing columns,
// finite values.  Returns an empty string when valid.
std::string csr_check(int64_t nrows, int64_t ncols, int64_t nnz, const int64_t* rp, const int32_t* ci,
                      const double* v);

HCsr csr_copy(int64_t nrows, int64_t ncols, const int64_t* rp, const int32_t* ci, const double* v);
HCsr transpose(const HCsr& A);
// C = A B; entry (i, j) summed over the stored entries of row i of A in
// storage order, each contributing A_ik * B_kj in the storage order of row k.
HCsr spgemm(const HCsr& A, const HCsr& B);
// Work arrays of one host thread for spgemm_row (sized on first use).
struct SpgemmWork {
  std::vector<double> acc;
  std::vector<int64_t> mark;
  std::vector<int32_t> cols;
};
// Row i of A B exactly as spgemm forms it (columns ascending, exact zeros
// dropped), appended to oc, ov.
void spgemm_row(const HCsr& A, const HCsr& B, int64_t i, SpgemmWork& w, std::vector<int32_t>& oc,
                std::vector<double>& ov);
// C = A + alpha B (union pattern, exact zeros dropped).
HCsr add(const HCsr& A, const HCsr& B, double alpha);
HCsr sub_block(const HCsr& A, int64_t r0, int64_t r1, int64_t c0, int64_t c1);
void drop_zeros(HCsr& A);
void scale_rows(HCsr& A, const std::vector<double>& s);
void scale_cols(HCsr& A, const std::vector<double>& s);

// Rows [r0, r1) of A in groups of g consecutive rows sharing one column list
// (the union of the group's columns): the result has (r1 - r0) / g rows with
// that list, and val holds, per listed entry, the g values of the group's
// rows (0 where a row has no entry in that column).
HCsr group_rows(const HCsr& A, int64_t r0, int64_t r1, int g, std::vector<double>& val);

// Column-list entries of rows [r0, r1) stored in groups of g rows, i.e. the
// number of distinct columns of each group summed over the groups (the
// grouped form holds g times as many values).
int64_t group_entries(const HCsr& A, int64_t r0, int64_t r1, int g);
std::vector<double> diagonal(const HCsr& A);
void matvec(const HCsr& A, const double* x, double* y);

}  // namespace fsi
