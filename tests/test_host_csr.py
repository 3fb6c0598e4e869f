"""Host-side CSR helpers of the library on the CPU (no GPU): the row grouping
behind the grouped storage of A_h's fluid-velocity rows, of the large vector
AMG levels and of the C_fm | C_fs product.

`host_csr.cpp` is plain C++; a small driver compiled here with g++ calls
`group_rows` and `group_entries` and the results are checked against the
definition written out with numpy: group q of rows [r0, r1) in groups of g is
the sorted union of the column lists of rows r0 + q g ... r0 + q g + g - 1, and
each listed column carries the g rows' values (0 where a row has no entry)."""
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1801_05648_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "host_csr.hpp"
template <typename T> static void rd(FILE* f, std::vector<T>& v, size_t n) {
  v.resize(n);
  if (n && fread(v.data(), sizeof(T), n, f) != n) throw 1;
}
template <typename T> static void wr(FILE* f, const std::vector<T>& v) {
  if (!v.empty()) fwrite(v.data(), sizeof(T), v.size(), f);
}
int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  int64_t hdr[6];  // nrows, ncols, nnz, r0, r1, g
  if (fread(hdr, 8, 6, f) != 6) return 2;
  fsi::HCsr A;
  A.nrows = hdr[0];
  A.ncols = hdr[1];
  rd(f, A.rp, size_t(hdr[0] + 1));
  rd(f, A.ci, size_t(hdr[2]));
  rd(f, A.v, size_t(hdr[2]));
  fclose(f);
  std::vector<double> val;
  fsi::HCsr G = fsi::group_rows(A, hdr[3], hdr[4], int(hdr[5]), val);
  const int64_t entries = fsi::group_entries(A, hdr[3], hdr[4], int(hdr[5]));
  FILE* o = fopen(argv[2], "wb");
  int64_t out[3] = {G.nrows, G.nnz(), entries};
  fwrite(out, 8, 3, o);
  wr(o, G.rp);
  wr(o, G.ci);
  wr(o, val);
  fclose(o);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("hostcsr")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run(["g++", "-std=c++17", "-O1", "-pthread", "-I", CSRC, str(src),
                    os.path.join(CSRC, "host_csr.cpp"), "-o", str(exe)], check=True)
    return d, exe


def _run(driver, A, r0, r1, g):
    d, exe = driver
    A = A.tocsr()
    A.sort_indices()
    inp, out = d / "in.bin", d / "out.bin"
    with open(inp, "wb") as f:
        np.array([A.shape[0], A.shape[1], A.nnz, r0, r1, g], np.int64).tofile(f)
        A.indptr.astype(np.int64).tofile(f)
        A.indices.astype(np.int32).tofile(f)
        A.data.astype(np.float64).tofile(f)
    subprocess.run([str(exe), str(inp), str(out)], check=True)
    raw = open(out, "rb").read()
    nrows, nnz, entries = np.frombuffer(raw, np.int64, 3)
    o = 24
    rp = np.frombuffer(raw, np.int64, nrows + 1, o); o += 8 * (nrows + 1)
    ci = np.frombuffer(raw, np.int32, nnz, o); o += 4 * nnz
    val = np.frombuffer(raw, np.float64, nnz * g, o)
    return int(nrows), rp, ci, val.reshape(nnz, g), int(entries)


def _reference(A, r0, r1, g):
    """Group q: the sorted union of its rows' columns; per column the g values."""
    A = A.tocsr()
    A.sort_indices()
    rp, cols, vals = [0], [], []
    for q in range((r1 - r0) // g):
        rows = range(r0 + q * g, r0 + q * g + g)
        union = sorted(set(np.concatenate([A.indices[A.indptr[r]:A.indptr[r + 1]] for r in rows]).tolist()))
        for c in union:
            cols.append(c)
            vals.append([A[r, c] for r in rows])
        rp.append(len(cols))
    return np.array(rp), np.array(cols, dtype=np.int64), np.array(vals, dtype=np.float64).reshape(-1, g)


@pytest.mark.parametrize("n,g,r0,r1,density,seed", [
    (30, 2, 0, 30, 0.2, 1),      # whole matrix, pairs
    (31, 3, 4, 31, 0.15, 2),     # sub-range, triples
    (40, 3, 1, 39, 0.0, 3),      # no entries at all
    (24, 2, 6, 18, 0.9, 4),      # nearly dense rows
])
def test_group_rows_matches_definition(driver, n, g, r0, r1, density, seed):
    rng = np.random.default_rng(seed)
    A = sp.random(n, n + 7, density=density, random_state=rng, format="csr")
    A.data = rng.standard_normal(A.nnz)
    A.data[A.indptr[5]:A.indptr[6]] = 0.0  # an empty row (its zeros removed below)
    A.eliminate_zeros()
    nrows, rp, ci, val, entries = _run(driver, A, r0, r1, g)
    erp, eci, evals = _reference(A, r0, r1, g)
    assert nrows == (r1 - r0) // g
    assert np.array_equal(rp, erp)
    assert np.array_equal(ci, eci)
    assert np.array_equal(val, evals)  # values copied, zeros where a row has no entry
    assert entries == len(eci)


def test_group_entries_threaded_count(driver):
    """Enough groups (> 4096) that the count runs on several host threads;
    it must equal the single-pass union count."""
    rng = np.random.default_rng(7)
    n, g = 3 * 6000, 3
    # block-structured rows (a node's three rows share columns) plus noise
    base = sp.random(n // g, n // g, density=5.0 / (n // g), random_state=rng, format="csr")
    A = sp.kron(base, np.ones((g, g))).tocsr() + sp.random(n, n, density=1e-4, random_state=rng, format="csr")
    A.sort_indices()
    nrows, rp, ci, val, entries = _run(driver, A, 0, n, g)
    union = 0
    for q in range(n // g):
        union += np.unique(A.indices[A.indptr[q * g]:A.indptr[q * g + g]]).size
    assert nrows == n // g and entries == union == ci.size


OPS_DRIVER = r"""
#include <cstdio>
#include <vector>
#include "host_csr.hpp"
template <typename T> static void rd(FILE* f, std::vector<T>& v, size_t n) {
  v.resize(n);
  if (n && fread(v.data(), sizeof(T), n, f) != n) throw 1;
}
static fsi::HCsr rcsr(FILE* f) {
  int64_t h[3];
  if (fread(h, 8, 3, f) != 3) throw 1;
  fsi::HCsr A;
  A.nrows = h[0];
  A.ncols = h[1];
  rd(f, A.rp, size_t(h[0] + 1));
  rd(f, A.ci, size_t(h[2]));
  rd(f, A.v, size_t(h[2]));
  return A;
}
static void wcsr(FILE* o, const fsi::HCsr& A) {
  int64_t h[3] = {A.nrows, A.ncols, A.nnz()};
  fwrite(h, 8, 3, o);
  fwrite(A.rp.data(), 8, A.rp.size(), o);
  if (A.nnz()) {
    fwrite(A.ci.data(), 4, A.ci.size(), o);
    fwrite(A.v.data(), 8, A.v.size(), o);
  }
}
int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  fsi::HCsr A = rcsr(f), B = rcsr(f), C = rcsr(f);
  int64_t blk[4];
  double alpha;
  if (fread(blk, 8, 4, f) != 4 || fread(&alpha, 8, 1, f) != 1) return 2;
  fclose(f);
  FILE* o = fopen(argv[2], "wb");
  wcsr(o, fsi::transpose(A));
  wcsr(o, fsi::add(A, B, alpha));
  wcsr(o, fsi::sub_block(A, blk[0], blk[1], blk[2], blk[3]));
  wcsr(o, fsi::spgemm(A, C));
  fsi::HCsr Z = A;
  for (int64_t k = 0; k < Z.nnz(); k += 3) Z.v[k] = 0.0;
  fsi::drop_zeros(Z);
  wcsr(o, Z);
  fclose(o);
  return 0;
}
"""


@pytest.fixture(scope="module")
def ops_driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("hostops")
    src = d / "ops.cpp"
    src.write_text(OPS_DRIVER)
    exe = d / "ops"
    subprocess.run(["g++", "-std=c++17", "-O2", "-pthread", "-I", CSRC, str(src),
                    os.path.join(CSRC, "host_csr.cpp"), "-o", str(exe)], check=True)
    return d, exe


def _wcsr(f, A):
    A = A.tocsr()
    A.sort_indices()
    np.array([A.shape[0], A.shape[1], A.nnz], np.int64).tofile(f)
    A.indptr.astype(np.int64).tofile(f)
    A.indices.astype(np.int32).tofile(f)
    A.data.astype(np.float64).tofile(f)


def _rcsr(raw, o):
    nr, nc, nnz = (int(v) for v in np.frombuffer(raw, np.int64, 3, o))
    o += 24
    rp = np.frombuffer(raw, np.int64, nr + 1, o); o += 8 * (nr + 1)
    ci = np.frombuffer(raw, np.int32, nnz, o); o += 4 * nnz
    v = np.frombuffer(raw, np.float64, nnz, o); o += 8 * nnz
    return (nr, nc, rp, ci, v), o


def _same_bits(got, ref):
    ref = ref.tocsr()
    ref.sort_indices()
    nr, nc, rp, ci, v = got
    return ((nr, nc) == ref.shape and np.array_equal(rp, ref.indptr) and np.array_equal(ci, ref.indices)
            and np.array_equal(v, ref.data))


@pytest.mark.parametrize("n,density,seed", [(3000, 0.004, 11), (60000, 3e-4, 12)])
def test_threaded_csr_operations_match_scipy_bitwise(ops_driver, n, density, seed):
    """transpose, A + alpha B, sub-blocks, the product and the zero drop on
    the host threads (the larger case: 1.08e6 entries, 60,000 rows, above
    every threading threshold) give scipy's arrays bit for bit: scipy adds,
    multiplies and sums in the same order and also drops exact zeros."""
    d, exe = ops_driver
    rng = np.random.default_rng(seed)
    A = sp.random(n, n + 5, density=density, random_state=rng, format="csr")
    A.data = rng.standard_normal(A.nnz)
    B = sp.random(n, n + 5, density=density, random_state=rng, format="csr")
    B.data = rng.standard_normal(B.nnz)
    B = (B + A.multiply(0.5)).tocsr()  # shared entries, some cancelling exactly below
    C = sp.random(n + 5, 700, density=6.0 / 700, random_state=rng, format="csr")
    C.data = rng.standard_normal(C.nnz)
    alpha = -2.0
    blk = (n // 7, n // 2, n // 5, n // 5 + n // 3)
    inp, out = d / "in.bin", d / "out.bin"
    with open(inp, "wb") as f:
        for M in (A, B, C):
            _wcsr(f, M)
        np.array(blk, np.int64).tofile(f)
        np.array([alpha], np.float64).tofile(f)
    subprocess.run([str(exe), str(inp), str(out)], check=True)
    raw = open(out, "rb").read()
    T, o = _rcsr(raw, 0)
    S, o = _rcsr(raw, o)
    Sb, o = _rcsr(raw, o)
    Pr, o = _rcsr(raw, o)
    Z, o = _rcsr(raw, o)
    A.sort_indices()
    assert _same_bits(T, A.T.tocsr())
    ref_sum = (A + alpha * B).tocsr()
    ref_sum.eliminate_zeros()
    assert _same_bits(S, ref_sum)
    assert _same_bits(Sb, A[blk[0]:blk[1], blk[2]:blk[3]])
    ref_prod = (A @ C).tocsr()
    ref_prod.eliminate_zeros()
    assert _same_bits(Pr, ref_prod)
    Az = A.copy()
    Az.data[::3] = 0.0
    Az.eliminate_zeros()
    assert _same_bits(Z, Az)
