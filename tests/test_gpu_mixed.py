"""Mixed precision: FP32 preconditioner (V-cycles, coupling products) inside
the FP64 FGMRES loop (Arnoldi, Givens, A_h products, true residual and the
coarsest solves stay FP64).  The error against the FP64 oracle is stated for
every result."""
import numpy as np
import pytest

from conftest import system

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _solver(name, precision):
    from paper_1801_05648_amd import FsiSolver
    s = FsiSolver.from_system(system(name), device=0)
    s.build_precond(precision)
    return s


@pytest.mark.parametrize("hname", ["H_M", "H_SIG", "H_MS", "H_A", "H_P"])
def test_fp32_vcycle_error_vs_fp64_oracle(hname):
    """An FP32 V-cycle differs from the FP64 oracle cycle on the same
    hierarchy by FP32 rounding amplified by the level operators: the bound
    here, 1e-4 relative, is ~1e3 unit roundoffs (2^-24)."""
    from oracle import amg, blocks, precond
    bs = blocks.BlockSystem(system("c1"))
    H = precond.build_hierarchies(bs)
    s = _solver("c1", "f32")
    import test_gpu_parity as tp
    tp._import_oracle_hierarchies(s, H)
    h = H[hname]
    rng = np.random.default_rng(7)
    if hname == "H_M":
        b = rng.standard_normal(bs.n_m)
        ref = precond.mesh_solve(bs, lambda v: amg.vcycle(h, v), b)
    else:
        b = rng.standard_normal(h.levels[0].A.shape[0])
        ref = amg.vcycle(h, b)
    x = s.vcycle(hname, _dev(b)).cpu().numpy()
    err = _rel(x, ref)
    print(f"{hname}: FP32 V-cycle rel. error vs FP64 oracle {err:.2e}")
    assert err <= 1e-4
    s.close()


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_fp32_preconditioner_reaches_fp64_accuracy(name):
    """The FP64 outer loop keeps a 1e-8 true residual attainable; the solution
    matches the FP64 GPU solve within the conditioning of the system."""
    from oracle import blocks
    sysm = system(name)
    bs = blocks.BlockSystem(sysm)
    b = _dev(sysm.b)
    s64 = _solver(name, "f64")
    x64, i64 = s64.solve(b)
    s64.close()
    s32 = _solver(name, "f32")
    x32, i32 = s32.solve(b)
    s32.close()
    assert i64.converged and i32.converged
    xr = x32.cpu().numpy()
    r = np.linalg.norm(sysm.b - bs.matvec(xr)) / np.linalg.norm(sysm.b)
    assert r <= 1e-8 * 1.001
    err = _rel(xr, x64.cpu().numpy())
    print(f"{name}: f64 {i64.iters} it {i64.t_total_ms:.1f} ms | f32-precond {i32.iters} it "
          f"{i32.t_total_ms:.1f} ms | rel. diff {err:.2e}")
    assert err <= 1e-6
    assert i32.iters <= 1.2 * i64.iters + 2


BENCH_PRECOND = dict(max_coarse=2000, cheb_degree=4, cheb=("H_SIG", "H_P"), poly=("H_MS",), poly_degree=3)


@pytest.mark.parametrize("name", ["c2", "m3"])
def test_fp32_preconditioner_in_the_benchmark_configuration(name):
    """The benchmarked preconditioner (Chebyshev V-cycles on H_SIG and H_P,
    Chebyshev steps alone for M_s, 2000-row coarse grids) in FP32: the 1e-8
    FP64 true residual is reached, the solution is within 1e-6 of the FP64
    solve with the same options, and the iteration count barely moves."""
    from oracle import blocks
    from paper_1801_05648_amd import FsiSolver
    sysm = system(name)
    bs = blocks.BlockSystem(sysm)
    b = _dev(sysm.b)
    res = {}
    for prec in ("f64", "f32"):
        s = FsiSolver.from_system(sysm, device=0)
        s.build_precond(prec, **BENCH_PRECOND)
        x, info = s.solve(b)
        s.close()
        assert info.converged
        res[prec] = (x.cpu().numpy(), info)
    xr = res["f32"][0]
    r = np.linalg.norm(sysm.b - bs.matvec(xr)) / np.linalg.norm(sysm.b)
    err = _rel(xr, res["f64"][0])
    print(f"{name}: f64 {res['f64'][1].iters} it {res['f64'][1].t_total_ms:.1f} ms | f32-precond "
          f"{res['f32'][1].iters} it {res['f32'][1].t_total_ms:.1f} ms | rel. diff {err:.2e}")
    assert r <= 1e-8 * 1.001
    assert err <= 1e-6 if name == "c2" else err <= 1e-5
    assert res["f32"][1].iters <= 1.2 * res["f64"][1].iters + 2


@pytest.mark.parametrize("hname,deg", [("H_SIG", 4), ("H_P", 4)])
def test_fp32_chebyshev_vcycle_error_vs_fp64_oracle(hname, deg):
    """FP32 Chebyshev V-cycle against the FP64 oracle cycle on the same
    (imported) hierarchy: ~1e3 unit roundoffs."""
    from oracle import amg, blocks, precond
    from paper_1801_05648_amd import FsiSolver
    bs = blocks.BlockSystem(system("c1"))
    H = precond.build_hierarchies(bs, max_coarse=40)
    s = FsiSolver.from_system(system("c1"), device=0)
    s.build_precond("f32", max_coarse=40, cheb_degree=deg, cheb=(hname,))
    import test_gpu_parity as tp
    tp._import_oracle_hierarchies(s, {hname: H[hname]})
    h = H[hname]
    b = np.random.default_rng(11).standard_normal(h.levels[0].A.shape[0])
    ref = amg.vcycle_cheb(h, b, deg)
    x = s.vcycle(hname, _dev(b)).cpu().numpy()
    err = _rel(x, ref)
    print(f"{hname}: FP32 Chebyshev({deg}) V-cycle rel. error vs FP64 oracle {err:.2e}")
    assert err <= 1e-4
    s.close()
