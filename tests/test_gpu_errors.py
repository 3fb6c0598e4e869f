"""Failure handling through the C ABI: every error is a status code with a
message, the context keeps its previous state, and the solver stays usable."""
import copy

import numpy as np
import pytest

from conftest import system

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _solver(name="c1"):
    from paper_1801_05648_amd import FsiSolver
    s = FsiSolver.from_system(system(name), device=0)
    s.build_precond("f64")
    return s


def test_iteration_bound_returns_the_best_iterate():
    from oracle import blocks
    sysm = system("c1")
    bs = blocks.BlockSystem(sysm)
    s = _solver()
    x, info = s.solve(_dev(sysm.b), maxit=3)
    assert info.status == "FSI_NOT_CONVERGED" and not info.converged and info.iters == 3
    xh = x.cpu().numpy()
    r = np.linalg.norm(sysm.b - bs.matvec(xh)) / np.linalg.norm(sysm.b)
    assert np.all(np.isfinite(xh)) and r < 1.0
    assert abs(info.true_rel_resid - r) <= 1e-6 * r
    x2, info2 = s.solve(_dev(sysm.b))  # still usable
    assert info2.converged
    s.close()


def test_zero_rhs_gives_zero_solution_without_iterations():
    s = _solver()
    b = torch.zeros(s.N, dtype=torch.float64, device="cuda:0")
    x, info = s.solve(b)
    assert info.converged and info.iters == 0
    assert torch.count_nonzero(x).item() == 0
    s.close()


def test_non_finite_rhs_is_rejected():
    from paper_1801_05648_amd import FsiError
    sysm = system("c1")
    s = _solver()
    b = sysm.b.copy()
    b[17] = np.nan
    with pytest.raises(FsiError) as e:
        s.solve(_dev(b))
    assert e.value.name == "FSI_ERR_NUMERIC"
    _, info = s.solve(_dev(sysm.b))
    assert info.converged
    s.close()


def test_out_of_range_column_is_rejected_and_the_system_kept():
    from paper_1801_05648_amd import FsiError, FsiSolver
    sysm = system("c1")
    s = _solver()
    _, info0 = s.solve(_dev(sysm.b))
    bad = copy.deepcopy(sysm.blocks)
    blk = bad["F"]
    blk.col = blk.col.copy()
    blk.col[5] = blk.ncols  # one past the last column
    with pytest.raises(FsiError) as e:
        s.set_system(bad, FsiSolver.layout_of(sysm))
    assert e.value.name == "FSI_ERR_CSR"
    _, info1 = s.solve(_dev(sysm.b))  # the previous system and preconditioner are intact
    assert info1.converged and info1.iters == info0.iters
    s.close()


def test_zero_diagonal_is_rejected_at_preconditioner_build():
    from paper_1801_05648_amd import FsiError, FsiSolver
    sysm = system("c1")
    bad = copy.deepcopy(sysm.blocks)
    M = bad["M"]
    M.val = M.val.copy()
    d = sysm.dim
    for row in range(d):  # node 0 of the mesh: both components, keeping M = L (x) I_d
        for k in range(M.rowptr[row], M.rowptr[row + 1]):
            if M.col[k] == row:
                M.val[k] = 0.0
    s = FsiSolver(bad, FsiSolver.layout_of(sysm), device=0)
    with pytest.raises(FsiError) as e:
        s.build_precond("f64")
    assert e.value.name == "FSI_ERR_NUMERIC"
    s.close()


def test_call_order_and_argument_checks():
    from paper_1801_05648_amd import FsiError, FsiSolver
    sysm = system("c1")
    s = FsiSolver.from_system(sysm, device=0)
    with pytest.raises(FsiError) as e:
        s.solve(_dev(sysm.b))
    assert e.value.name == "FSI_ERR_STATE"
    s.build_precond("f64")
    with pytest.raises(TypeError):
        s.solve(torch.from_numpy(sysm.b))  # host tensor
    with pytest.raises(FsiError) as e:
        s.solve(_dev(sysm.b), tol=-1.0)
    assert e.value.name == "FSI_ERR_ARG"
    b = _dev(sysm.b)
    with pytest.raises(FsiError) as e:
        s.solve(b, b)  # x aliases b
    assert e.value.name == "FSI_ERR_ARG"
    with pytest.raises(FsiError) as e:
        s.build_precond("f64", cheb_degree=3, cheb=("H_A",))
    assert e.value.name == "FSI_ERR_ARG"
    # an unknown precision code is refused (the three known: FP64, FP32, FP32 + BF16 diagonals)
    import ctypes
    from paper_1801_05648_amd import fsi as F
    o = F.CPrecondOpts()
    s.lib.fsi_default_precond_opts(ctypes.byref(o))
    o.precision = 7
    assert F.STATUS[s.lib.fsi_build_precond(s.ctx, ctypes.byref(o))] == "FSI_ERR_ARG"
    for k in (-1, 17):  # inner GMRES steps of the fluid inverse: 0..16
        with pytest.raises(FsiError) as e:
            s.build_precond("f64", fluid_inner=k)
        assert e.value.name == "FSI_ERR_ARG"
    o.precision = 0
    o.fluid_inner, o.fluid_inner_pc = 2, 5  # an unknown inner preconditioner
    assert F.STATUS[s.lib.fsi_build_precond(s.ctx, ctypes.byref(o))] == "FSI_ERR_ARG"
    o.fluid_inner, o.fluid_inner_pc, o.order = 0, 0, 6  # an unknown block order
    assert F.STATUS[s.lib.fsi_build_precond(s.ctx, ctypes.byref(o))] == "FSI_ERR_ARG"
    _, info = s.solve(_dev(sysm.b))  # the failed calls left the preconditioner in place
    assert info.converged
    assert s.spmv_bytes() > 0
    s.close()
    # queries before the system is set up
    ctx = ctypes.c_void_p()
    assert F.STATUS[F.load().fsi_create(ctypes.byref(ctx), 0, None)] == "FSI_OK"
    b = ctypes.c_double()
    assert F.STATUS[F.load().fsi_spmv_bytes(ctx, ctypes.byref(b))] == "FSI_ERR_STATE"
    assert F.STATUS[F.load().fsi_spmv_bytes(ctx, None)] == "FSI_ERR_STATE"
    F.load().fsi_destroy(ctx)


@pytest.mark.parametrize("name", ["c1", "m3"])
def test_hierarchy_reuse_rules(name):
    """reuse=True needs a previous build of the same system with the same AMG
    parameters and Schur option (else FSI_ERR_STATE, context unchanged); a
    new system drops the right to reuse; a reused build solves like a fresh
    one (bit-identical: the same host hierarchies, with the A P products and
    R A counts they keep, are uploaded; on the 3D system the products and
    the row grouping run on the device)."""
    from paper_1801_05648_amd import FsiError, FsiSolver
    sysm = system(name)
    s = FsiSolver.from_system(sysm, device=0)
    with pytest.raises(FsiError) as e:
        s.build_precond("f32", reuse=True)
    assert e.value.name == "FSI_ERR_STATE"
    s.build_precond("f64", max_coarse=40)
    b = _dev(sysm.b)
    x64, i64 = s.solve(b)
    for bad in (dict(max_coarse=500), dict(max_coarse=40, strength0=0.04), dict(max_coarse=40, schur="simplec")):
        with pytest.raises(FsiError) as e:
            s.build_precond("f32", reuse=True, **bad)
        assert e.value.name == "FSI_ERR_STATE", bad
    x, i = s.solve(b)  # the failed calls left the FP64 preconditioner in place
    assert torch.equal(x, x64) and i.iters == i64.iters
    s.build_precond("f32", reuse=True, max_coarse=40, cheb_degree=3, cheb=("H_SIG",))
    xr, ir = s.solve(b)
    s.set_from_system(sysm)
    with pytest.raises(FsiError) as e:
        s.build_precond("f32", reuse=True, max_coarse=40)
    assert e.value.name == "FSI_ERR_STATE"
    s.build_precond("f32", max_coarse=40, cheb_degree=3, cheb=("H_SIG",))
    xf, i_f = s.solve(b)
    s.close()
    assert ir.converged and torch.equal(xr, xf) and ir.iters == i_f.iters
