"""The library's smoothed-aggregation setup (`sa_setup.cpp`, host C++) against
the oracle's (`oracle/amg.py`) on identical inputs, on the CPU (no GPU).

A small driver compiled here with g++ calls `fsi::sa_setup` on the matrix,
node block size and near-nullspace the oracle uses for each of the five
hierarchies of the C1 system (40-row coarse grids, so that every hierarchy has
several levels).  Both implement the same written rules (strength on squared
block Frobenius norms, three-phase aggregation in node order, aggregate QR of
the near-nullspace, filtered Jacobi prolongator smoothing, Galerkin product):

* the level sizes and every aggregate are identical (integer decisions on
  values that agree to rounding; ties are broken by the same rule);
* omega = (4/3) / rho from the same power iteration within 1e-10;
* P, R = P^T and the Galerkin products A_c have the same sparsity pattern and
  values within 1e-11 relative (different summation order).

A second driver pins the coarsest-level inverse `fsi::dense_inverse` (LU with
partial pivoting, threaded from 256 rows) against A X = I and numpy's inverse,
and checks that a singular matrix is reported.
"""
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from conftest import system

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1801_05648_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "sa_setup.hpp"
template <typename T> static void rd(FILE* f, std::vector<T>& v, size_t n) {
  v.resize(n);
  if (n && fread(v.data(), sizeof(T), n, f) != n) throw 1;
}
template <typename T> static void wr(FILE* f, const std::vector<T>& v) {
  if (!v.empty()) fwrite(v.data(), sizeof(T), v.size(), f);
}
static void wcsr(FILE* o, const fsi::HCsr& A) {
  int64_t h[3] = {A.nrows, A.ncols, A.nnz()};
  fwrite(h, 8, 3, o);
  wr(o, A.rp);
  wr(o, A.ci);
  wr(o, A.v);
}
int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  int64_t hdr[6];  // nrows, ncols, nnz, block, k, max_coarse
  double eps0;
  if (fread(hdr, 8, 6, f) != 6 || fread(&eps0, 8, 1, f) != 1) return 2;
  fsi::HCsr A;
  A.nrows = hdr[0];
  A.ncols = hdr[1];
  rd(f, A.rp, size_t(hdr[0] + 1));
  rd(f, A.ci, size_t(hdr[2]));
  rd(f, A.v, size_t(hdr[2]));
  std::vector<double> B;
  rd(f, B, size_t(hdr[0] * hdr[4]));
  fclose(f);
  fsi::SaParams prm;
  prm.eps0 = eps0;
  prm.max_coarse = int(hdr[5]);
  fsi::SaHierarchy H;
  std::string err = fsi::sa_setup(A, int(hdr[3]), B, int(hdr[4]), prm, H);
  if (!err.empty()) {
    fprintf(stderr, "%s\n", err.c_str());
    return 3;
  }
  FILE* o = fopen(argv[2], "wb");
  int64_t nl = int64_t(H.levels.size());
  fwrite(&nl, 8, 1, o);
  for (int64_t l = 0; l < nl; ++l) {
    const fsi::SaLevel& L = H.levels[size_t(l)];
    int64_t meta[2] = {L.block, int64_t(L.agg.size())};
    fwrite(meta, 8, 2, o);
    fwrite(&L.omega, 8, 1, o);
    wcsr(o, L.A);
    wr(o, L.agg);
    if (l + 1 < nl) {
      wcsr(o, L.P);
      wcsr(o, L.R);
    }
  }
  fclose(o);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("sasetup")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run(["g++", "-std=c++17", "-O2", "-pthread", "-I", CSRC, str(src),
                    os.path.join(CSRC, "sa_setup.cpp"), os.path.join(CSRC, "host_csr.cpp"), "-o", str(exe)],
                   check=True)
    return d, exe


class _Reader:
    def __init__(self, raw):
        self.raw, self.o = raw, 0

    def take(self, dtype, n):
        a = np.frombuffer(self.raw, dtype, n, self.o)
        self.o += a.nbytes
        return a

    def csr(self):
        nr, nc, nnz = self.take(np.int64, 3)
        rp = self.take(np.int64, nr + 1)
        ci = self.take(np.int32, nnz)
        v = self.take(np.float64, nnz)
        return sp.csr_matrix((v, ci, rp), shape=(int(nr), int(nc)))


def _run(driver, A, block, B, eps0, max_coarse):
    d, exe = driver
    A = A.tocsr().copy()
    A.sort_indices()
    B = np.ascontiguousarray(B, dtype=np.float64)
    inp, out = d / "in.bin", d / "out.bin"
    with open(inp, "wb") as f:
        np.array([A.shape[0], A.shape[1], A.nnz, block, B.shape[1], max_coarse], np.int64).tofile(f)
        np.array([eps0], np.float64).tofile(f)
        A.indptr.astype(np.int64).tofile(f)
        A.indices.astype(np.int32).tofile(f)
        A.data.astype(np.float64).tofile(f)
        B.tofile(f)
    subprocess.run([str(exe), str(inp), str(out)], check=True)
    rd = _Reader(open(out, "rb").read())
    nl = int(rd.take(np.int64, 1)[0])
    levels = []
    for l in range(nl):
        block_l, nagg = rd.take(np.int64, 2)
        omega = float(rd.take(np.float64, 1)[0])
        Al = rd.csr()
        agg = rd.take(np.int32, nagg)
        P = R = None
        if l + 1 < nl:
            P, R = rd.csr(), rd.csr()
        levels.append(dict(block=int(block_l), omega=omega, A=Al, agg=agg, P=P, R=R))
    return levels


def _same(a, b, tol):
    """Same sparsity pattern, values within tol relative to the largest."""
    a, b = a.tocsr(), b.tocsr()
    a.sort_indices()
    b.sort_indices()
    assert a.shape == b.shape
    assert np.array_equal(a.indptr, b.indptr) and np.array_equal(a.indices, b.indices)
    return np.abs(a.data - b.data).max(initial=0.0) <= tol * np.abs(b.data).max(initial=1.0)


def _inputs(bs):
    from oracle import amg
    d = bs.dim
    o = bs.sys.offsets
    vs_nodes = bs.sys.dof_node[o[1]:o[1] + bs.n_vs:d]
    xyz = bs.sys.coords[vs_nodes]
    L = bs.mesh_scalar()
    return {
        "H_M": (L, 1, amg.constant_modes(L.shape[0])),
        "H_SIG": (bs.solid_schur(), d, amg.rigid_body_modes(xyz)),
        "H_MS": (bs.S_uu, 1, amg.constant_modes(bs.n_vs)),
        "H_A": (bs.A_f, d, amg.translation_modes(bs.n_vf // d, d)),
        "H_P": (bs.fluid_schur(), 1, amg.constant_modes(bs.n_p)),
    }


@pytest.mark.parametrize("name", ["c1", "tiny3d"])
def test_library_sa_setup_matches_oracle(driver, name):
    from oracle import amg, blocks
    bs = blocks.BlockSystem(system(name, seed=2))
    mc = 40
    for hname, (A, block, B) in _inputs(bs).items():
        ho = amg.setup(A, block, B, eps0=amg.EPS0, max_coarse=mc)
        lib = _run(driver, A, block, B, amg.EPS0, mc)
        assert len(lib) == ho.nlevels, hname
        for l, (g, o) in enumerate(zip(lib, ho.levels)):
            assert g["A"].shape == o.A.shape, (hname, l)
            assert _same(g["A"], o.A, 1e-11), (hname, l, "A")
            if l + 1 == ho.nlevels:
                break
            assert g["block"] == o.block, (hname, l)
            assert np.array_equal(g["agg"].astype(np.int64), np.asarray(o.aggregates, np.int64)), (hname, l)
            assert abs(g["omega"] - o.omega) <= 1e-10 * o.omega, (hname, l, g["omega"], o.omega)
            assert _same(g["P"], o.P, 1e-11), (hname, l, "P")
            assert _same(g["R"], o.R, 1e-11), (hname, l, "R")


INV_DRIVER = r"""
#include <cstdio>
#include <vector>
#include "sa_setup.hpp"
int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  int64_t n;
  if (fread(&n, 8, 1, f) != 1) return 2;
  std::vector<double> a(size_t(n) * n), inv;
  if (n && fread(a.data(), 8, a.size(), f) != a.size()) return 2;
  fclose(f);
  const int64_t ok = fsi::dense_inverse(a, n, inv) ? 1 : 0;
  FILE* o = fopen(argv[2], "wb");
  fwrite(&ok, 8, 1, o);
  if (ok) fwrite(inv.data(), 8, inv.size(), o);
  fclose(o);
  return 0;
}
"""


@pytest.fixture(scope="module")
def inv_driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("denseinv")
    src = d / "inv.cpp"
    src.write_text(INV_DRIVER)
    exe = d / "inv"
    subprocess.run(["g++", "-std=c++17", "-O2", "-pthread", "-I", CSRC, str(src),
                    os.path.join(CSRC, "sa_setup.cpp"), os.path.join(CSRC, "host_csr.cpp"), "-o", str(exe)],
                   check=True)
    return d, exe


def _inverse(inv_driver, a):
    d, exe = inv_driver
    a = np.ascontiguousarray(a, dtype=np.float64)
    n = a.shape[0]
    with open(d / "a.bin", "wb") as f:
        np.array([n], np.int64).tofile(f)
        a.tofile(f)
    subprocess.run([str(exe), str(d / "a.bin"), str(d / "x.bin")], check=True)
    raw = open(d / "x.bin", "rb").read()
    ok = int(np.frombuffer(raw, np.int64, 1)[0])
    return (np.frombuffer(raw, np.float64, n * n, 8).reshape(n, n) if ok else None)


@pytest.mark.parametrize("n", [1, 3, 50, 300])
def test_dense_inverse_of_the_coarsest_level(inv_driver, n):
    """The coarsest-level inverse (LU with partial pivoting on the host, the
    row updates and column solves shared among threads from 256 rows on):
    A X = I and X = numpy's inverse within rounding, on nonsymmetric systems
    that need row exchanges (a small diagonal)."""
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, n)) + n ** 0.5 * np.eye(n)
    a[np.arange(n), np.arange(n)] *= 1e-3  # pivoting needed
    a += 0.1 * n ** 0.5 * np.eye(n, k=1)
    x = _inverse(inv_driver, a)
    assert x is not None
    cond = np.linalg.cond(a)
    assert np.abs(a @ x - np.eye(n)).max() <= 1e-13 * cond
    ref = np.linalg.inv(a)
    assert np.abs(x - ref).max() <= 1e-13 * cond * np.abs(ref).max()


def test_dense_inverse_refuses_a_singular_matrix(inv_driver):
    """A zero pivot column (here a zero column, in the threaded size range
    too) is reported, not divided by."""
    for n in (4, 260):
        a = np.random.default_rng(5).standard_normal((n, n))
        a[:, n // 2] = 0.0
        assert _inverse(inv_driver, a) is None, n
    # a permutation matrix needs a row exchange at every step and is its own transpose's inverse
    p = np.eye(6)[[3, 0, 5, 1, 4, 2]]
    assert np.array_equal(_inverse(inv_driver, p), p.T)
