"""Host code under the compiler's sanitizers, on the CPU.

The preconditioner's host setup (`sa_setup.cpp`, `host_csr.cpp`: sparse
products, aggregation and the power iteration on a hand-rolled thread pool
with atomic work counters, the threaded dense inverse) and the input
generator (`fsigen.cpp`) are built with g++ and run on workloads large
enough to engage the threads:

* AddressSanitizer + UndefinedBehaviorSanitizer: no report, and the SA
  setup's output is byte-identical to the plain build's;
* ThreadSanitizer (SA setup and dense inverse): no data race reported.

The generator's OpenMP loops run under ASan/UBSan only: ThreadSanitizer needs
an instrumented OpenMP runtime, which this toolchain does not provide.
"""
import os
import subprocess

import numpy as np
import scipy.sparse as sp
import pytest

from conftest import system

import test_sa_setup_cpu as sa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1801_05648_amd", "csrc")
GEN = os.path.join(ROOT, "fsigen", "csrc")

ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
TSAN = ["-fsanitize=thread", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24",
           TSAN_OPTIONS="halt_on_error=1:exitcode=25")


def _build(tmp, name, src_text, flags, extra_sources, extra=()):
    src = tmp / f"{name}.cpp"
    src.write_text(src_text)
    exe = tmp / name
    subprocess.run(["g++", "-std=c++17", "-pthread", *flags, "-I", CSRC, str(src), *extra_sources, *extra,
                    "-o", str(exe)], check=True)
    return exe


def _sa_inputs(name="c2"):
    from oracle import blocks
    bs = blocks.BlockSystem(system(name, seed=2))
    return sa._inputs(bs)


def _write_input(path, A, block, B, eps0, max_coarse):
    A = A.tocsr().copy()
    A.sort_indices()
    B = np.ascontiguousarray(B, dtype=np.float64)
    with open(path, "wb") as f:
        np.array([A.shape[0], A.shape[1], A.nnz, block, B.shape[1], max_coarse], np.int64).tofile(f)
        np.array([eps0], np.float64).tofile(f)
        A.indptr.astype(np.int64).tofile(f)
        A.indices.astype(np.int32).tofile(f)
        A.data.astype(np.float64).tofile(f)
        B.tofile(f)


@pytest.fixture(scope="module")
def sa_builds(tmp_path_factory):
    d = tmp_path_factory.mktemp("sasan")
    srcs = [os.path.join(CSRC, "sa_setup.cpp"), os.path.join(CSRC, "host_csr.cpp")]
    return d, {"plain": _build(d, "plain", sa.DRIVER, ["-O2"], srcs),
               "asan": _build(d, "asan", sa.DRIVER, ASAN, srcs),
               "tsan": _build(d, "tsan", sa.DRIVER, TSAN, srcs)}


@pytest.mark.parametrize("hname", ["H_A", "H_SIG", "H_M"])
def test_sa_setup_under_address_and_undefined_sanitizers(sa_builds, hname):
    """256x64 operators (A_f: 121,792 rows, above the thread pool's 4096-row
    threshold): clean under ASan/UBSan and byte-identical to the plain build."""
    d, exe = sa_builds
    A, block, B = _sa_inputs()[hname]
    inp = d / f"in_{hname}.bin"
    _write_input(inp, A, block, B, 0.08, 500)
    outs = {}
    for kind in ("plain", "asan"):
        out = d / f"out_{hname}_{kind}.bin"
        r = subprocess.run([str(exe[kind]), str(inp), str(out)], capture_output=True, text=True, env=ENV)
        assert r.returncode == 0, (kind, r.returncode, r.stderr[-3000:])
        assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
        outs[kind] = out.read_bytes()
    assert outs["plain"] == outs["asan"]


def test_sa_setup_under_thread_sanitizer(sa_builds):
    """The threaded sparse products, filtered matrix and power iteration of
    the 256x64 A_f hierarchy: no data race reported."""
    d, exe = sa_builds
    A, block, B = _sa_inputs()["H_A"]
    inp = d / "in_tsan.bin"
    _write_input(inp, A, block, B, 0.08, 500)
    r = subprocess.run([str(exe["tsan"]), str(inp), str(d / "out_tsan.bin")], capture_output=True, text=True,
                       env=ENV)
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-3000:]


def test_dense_inverse_under_sanitizers(tmp_path):
    """The threaded coarsest-level inverse (from 256 rows) on 300 rows under
    ASan/UBSan and under TSan: clean, and A X = I."""
    srcs = [os.path.join(CSRC, "sa_setup.cpp"), os.path.join(CSRC, "host_csr.cpp")]
    n = 300
    rng = np.random.default_rng(3)
    a = rng.standard_normal((n, n)) + 20.0 * np.eye(n)
    with open(tmp_path / "a.bin", "wb") as f:
        np.array([n], np.int64).tofile(f)
        a.tofile(f)
    for kind, flags in (("asan", ASAN), ("tsan", TSAN)):
        exe = _build(tmp_path, f"inv_{kind}", sa.INV_DRIVER, flags, srcs)
        r = subprocess.run([str(exe), str(tmp_path / "a.bin"), str(tmp_path / f"x_{kind}.bin")],
                           capture_output=True, text=True, env=ENV)
        assert r.returncode == 0, (kind, r.stderr[-3000:])
        assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
        raw = open(tmp_path / f"x_{kind}.bin", "rb").read()
        assert int(np.frombuffer(raw, np.int64, 1)[0]) == 1
        x = np.frombuffer(raw, np.float64, n * n, 8).reshape(n, n)
        assert np.abs(a @ x - np.eye(n)).max() <= 1e-12


def test_threaded_csr_operations_under_sanitizers(tmp_path):
    """The host-thread CSR operations (transpose with per-thread column
    counts, the two-pass row builder behind sums, sub-blocks and zero drops,
    the chunked product) on 60,000 rows and 1.08e6 entries: clean under
    ASan/UBSan and under TSan, with the plain build's bytes."""
    import test_host_csr as hc
    rng = np.random.default_rng(12)
    n = 60000
    A = sp.random(n, n + 5, density=3e-4, random_state=rng, format="csr")
    A.data = rng.standard_normal(A.nnz)
    B = sp.random(n, n + 5, density=3e-4, random_state=rng, format="csr")
    B.data = rng.standard_normal(B.nnz)
    B = (B + A.multiply(0.5)).tocsr()
    C = sp.random(n + 5, 700, density=6.0 / 700, random_state=rng, format="csr")
    C.data = rng.standard_normal(C.nnz)
    inp = tmp_path / "in.bin"
    with open(inp, "wb") as f:
        for M in (A, B, C):
            hc._wcsr(f, M)
        np.array((n // 7, n // 2, n // 5, n // 5 + n // 3), np.int64).tofile(f)
        np.array([-2.0], np.float64).tofile(f)
    srcs = [os.path.join(CSRC, "host_csr.cpp")]
    outs = {}
    for kind, flags in (("plain", ["-O2"]), ("asan", ASAN), ("tsan", TSAN)):
        exe = _build(tmp_path, f"ops_{kind}", hc.OPS_DRIVER, flags, srcs)
        out = tmp_path / f"out_{kind}.bin"
        r = subprocess.run([str(exe), str(inp), str(out)], capture_output=True, text=True, env=ENV)
        assert r.returncode == 0, (kind, r.returncode, r.stderr[-3000:])
        assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
        outs[kind] = out.read_bytes()
    assert outs["plain"] == outs["asan"] == outs["tsan"]


GEN_DRIVER = r"""
#include "fsigen.cpp"
#include <cstdio>
#include <vector>
// Assemble one configuration through the library's C entry points and read
// every array back (sizes from the same calls).
int main(int argc, char** argv) {
  fsigen_cfg c{};
  c.dim = std::atoi(argv[1]);
  for (int a = 0; a < 3; ++a) { c.nc[a] = std::atoi(argv[2 + a]); c.L[a] = a == 0 ? 2.0 : 0.5; }
  for (int a = 0; a < 3; ++a) { c.solid_lo[a] = std::atoi(argv[5 + a]); c.solid_hi[a] = std::atoi(argv[8 + a]); }
  c.rho_f = 1e3; c.nu_f = 1e-3; c.rho_s = 1e4; c.mu_s = 5e5; c.lambda_s = 2e6; c.dt = 1e-2; c.theta = 1.0;
  c.v_peak = 1.0; c.u_peak = 6.25e-3; c.p_amp = 10.0; c.seed = 1; c.t_phase = 0.3;
  fsigen_handle* h = nullptr;
  char err[512];
  if (fsigen_build(&c, &h, err, 512) != 0) { std::fprintf(stderr, "%s\n", err); return 3; }
  int64_t s[9];
  fsigen_sizes(h, s);
  double sum = 0.0;
  for (int b = 0; b < 8; ++b) {
    int64_t bs[3];
    fsigen_block_sizes(h, b, bs);
    std::vector<int64_t> rp(bs[0] + 1);
    std::vector<int32_t> ci(bs[2]);
    std::vector<double> v(bs[2]);
    fsigen_block_copy(h, b, rp.data(), ci.data(), v.data());
    for (double x : v) sum += x;
  }
  std::vector<double> rhs(s[2]), coords(s[1] * s[0]);
  std::vector<int32_t> ijk(s[1] * s[0]), dn(s[2]);
  std::vector<uint8_t> flags(s[1]);
  std::vector<int8_t> comp(s[2]);
  fsigen_rhs(h, rhs.data());
  fsigen_nodes(h, coords.data(), ijk.data(), flags.data(), dn.data(), comp.data());
  double jr[2];
  fsigen_jrange(h, jr);
  std::vector<double> dU(s[2], 1e-3), R(s[2]);
  if (fsigen_residual(&c, dU.data(), 1e-6, R.data(), s[2], err, 512) != 0) { std::fprintf(stderr, "%s\n", err); return 4; }
  fsigen_free(h);
  std::printf("N=%lld sum=%.6e J=[%.4f,%.4f]\n", (long long)s[2], sum, jr[0], jr[1]);
  return 0;
}
"""


@pytest.mark.parametrize("args", [["2", "32", "8", "1", "12", "0", "0", "20", "2", "1"],
                                  ["3", "8", "4", "4", "2", "0", "1", "4", "1", "3"]])
def test_generator_under_address_and_undefined_sanitizers(tmp_path, args):
    """The assembler's OpenMP loops, block extraction, node arrays and the
    residual for finite differences, on a 2D 32x8 and a 3D 8x4x4 grid: no
    ASan/UBSan report."""
    src = tmp_path / "gen.cpp"
    src.write_text(GEN_DRIVER)
    exe = tmp_path / "gen"
    subprocess.run(["g++", "-std=c++17", "-fopenmp", *ASAN, "-I", GEN, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe), *args], capture_output=True, text=True, env=dict(ENV, OMP_NUM_THREADS="4"))
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    assert r.stdout.startswith("N=")
