"""Chebyshev-smoothed V-cycles on the GPU against the FP64 oracle.

With cheb_degree k the hierarchies in the mask use k Chebyshev steps for
D^{-1} A before and after the coarse correction instead of one Jacobi sweep.
Parity is at FP64 rounding on the oracle's own hierarchies (imported), and
the whole solve matches the oracle's Chebyshev-preconditioned FGMRES."""
import numpy as np
import pytest

from conftest import system

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

_cache = {}


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _oracle(name, mc):
    from oracle import blocks, precond
    if (name, mc) not in _cache:
        bs = blocks.BlockSystem(system(name))
        _cache[(name, mc)] = (bs, precond.build_hierarchies(bs, max_coarse=mc))
    return _cache[(name, mc)]


def _solver(name, mc, deg, cheb):
    from paper_1801_05648_amd import FsiSolver
    s = FsiSolver.from_system(system(name), device=0)
    s.build_precond("f64", max_coarse=mc, cheb_degree=deg, cheb=cheb)
    return s


def _import(s, H, names):
    import test_gpu_parity as tp
    tp._import_oracle_hierarchies(s, {k: H[k] for k in names})


@pytest.mark.parametrize("deg", [1, 2, 3])
@pytest.mark.parametrize("hname", ["H_M", "H_SIG", "H_MS", "H_P"])
@pytest.mark.parametrize("name,mc", [("c1", 40), ("tiny3d", 10)])
def test_chebyshev_vcycle_parity(name, mc, hname, deg):
    from oracle import amg, precond
    bs, H = _oracle(name, mc)
    h = H[hname]
    s = _solver(name, mc, deg, (hname,))
    _import(s, H, [hname])
    rng = np.random.default_rng(4)
    if hname == "H_M":
        b = rng.standard_normal(bs.n_m)
        ref = precond.mesh_solve(bs, lambda v: amg.vcycle_cheb(h, v, deg), b)
    else:
        b = rng.standard_normal(h.levels[0].A.shape[0])
        ref = amg.vcycle_cheb(h, b, deg)
    x = s.vcycle(hname, _dev(b)).cpu().numpy()
    err = _rel(x, ref)
    print(f"{name} {hname} deg {deg} ({h.nlevels} levels): rel. err {err:.2e}")
    assert err <= 1e-12
    s.close()


def test_chebyshev_solve_matches_oracle_and_graphs(monkeypatch):
    """C1 with 40-row coarse grids, Chebyshev(3) on H_MS, H_SIG, H_P: the
    solution at 1e-8 is within 1e-6 of the oracle's 1e-12 solution with the
    same hierarchies; graph replays and plain launches agree bit for bit."""
    from oracle import krylov, precond
    bs, H = _oracle("c1", 40)
    names = ("H_MS", "H_SIG", "H_P")
    P = precond.amg_preconditioner(bs, H, cheb={k: 3 for k in names})
    xo, io = krylov.fgmres(bs.matvec, P, bs.sys.b, tol=1e-12, restart=50, maxit=2000)
    b = _dev(bs.sys.b)
    s = _solver("c1", 40, 3, names)
    _import(s, H, list(H.keys()))
    x1, i1 = s.solve(b, tol=1e-8)
    x2, i2 = s.solve(b, tol=1e-8)
    s.close()
    monkeypatch.setenv("FSI_GRAPHS", "0")
    e = _solver("c1", 40, 3, names)
    _import(e, H, list(H.keys()))
    x3, i3 = e.solve(b, tol=1e-8)
    e.close()
    err = _rel(x1.cpu().numpy(), xo)
    print(f"c1 Chebyshev(3): GPU {i1.iters} it, oracle {io.iters} it to 1e-12, rel. diff {err:.2e}")
    assert i1.converged and err <= 1e-6
    assert i1.iters == i2.iters == i3.iters
    assert torch.equal(x1, x2) and torch.equal(x1, x3)


def test_chebyshev_cuts_3d_iterations():
    """32x8x8-cell 3D Jacobian: Chebyshev(3) sweeps on the solid and pressure
    hierarchies need far fewer FGMRES iterations than Jacobi sweeps, and both
    solutions agree."""
    sysm = system("m3")
    b = _dev(sysm.b)
    from paper_1801_05648_amd import FsiSolver
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64")
    xj, ij = s.solve(b, tol=1e-8)
    s.build_precond("f64", cheb_degree=3)
    xc, ic = s.solve(b, tol=1e-8)
    s.close()
    diff = _rel(xc.cpu().numpy(), xj.cpu().numpy())
    print(f"m3: Jacobi {ij.iters} it {ij.t_total_ms:.1f} ms, Chebyshev(3) {ic.iters} it {ic.t_total_ms:.1f} ms, "
          f"rel. diff {diff:.2e}")
    assert ij.converged and ic.converged
    assert ic.iters < 0.5 * ij.iters
    assert diff <= 1e-5


def test_chebyshev_on_the_fluid_velocity_hierarchy_is_rejected():
    from paper_1801_05648_amd import FsiError, FsiSolver
    s = FsiSolver.from_system(system("c1"), device=0)
    with pytest.raises(FsiError):
        s.build_precond("f64", cheb_degree=2, cheb=("H_A",))
    s.close()


@pytest.mark.parametrize("deg,ratio", [(2, 8.0), (3, 8.0), (5, 4.0)])
@pytest.mark.parametrize("hname", ["H_MS", "H_SIG", "H_M"])
@pytest.mark.parametrize("name,mc", [("c1", 40), ("tiny3d", 10)])
def test_chebyshev_only_inverse_parity(name, mc, hname, deg, ratio):
    """k Chebyshev steps alone on the finest matrix (no coarse grid), the
    option meant for the solid mass matrix."""
    from oracle import amg, precond
    from paper_1801_05648_amd import FsiSolver
    bs, H = _oracle(name, mc)
    h = H[hname]
    assert h.nlevels >= 2
    s = FsiSolver.from_system(system(name), device=0)
    s.build_precond("f64", max_coarse=mc, poly=(hname,), poly_degree=deg, poly_ratio=ratio)
    _import(s, H, [hname])
    L0 = h.levels[0]
    inv = lambda v: amg.chebyshev(L0.A, L0.dinv, v, np.zeros_like(v), deg, amg.CHEB_BOOST * L0.rho, ratio)
    rng = np.random.default_rng(6)
    if hname == "H_M":
        b = rng.standard_normal(bs.n_m)
        ref = precond.mesh_solve(bs, inv, b)
    else:
        b = rng.standard_normal(L0.A.shape[0])
        ref = inv(b)
    x = s.vcycle(hname, _dev(b)).cpu().numpy()
    err = _rel(x, ref)
    print(f"{name} {hname} Chebyshev-only k={deg} ratio {ratio}: rel. err {err:.2e}")
    assert err <= 1e-12
    s.close()


def test_chebyshev_only_mass_inverse_solve_matches_oracle():
    """C1, 40-row coarse grids: M_s by 3 Chebyshev steps alone, Chebyshev(4)
    V-cycles on H_SIG and H_P; the GPU solution at 1e-8 against the oracle's
    1e-12 solution with the same hierarchies and inverses."""
    from oracle import krylov, precond
    from paper_1801_05648_amd import FsiSolver
    bs, H = _oracle("c1", 40)
    P = precond.amg_preconditioner(bs, H, cheb={"H_SIG": 4, "H_P": 4}, poly={"H_MS": (3, 8.0)})
    xo, io = krylov.fgmres(bs.matvec, P, bs.sys.b, tol=1e-12, restart=50, maxit=2000)
    s = FsiSolver.from_system(system("c1"), device=0)
    s.build_precond("f64", max_coarse=40, cheb_degree=4, cheb=("H_SIG", "H_P"), poly=("H_MS",), poly_degree=3)
    _import(s, H, list(H.keys()))
    x, info = s.solve(_dev(bs.sys.b), tol=1e-8)
    err = _rel(x.cpu().numpy(), xo)
    print(f"c1 M_s Chebyshev-only: GPU {info.iters} it, oracle {io.iters} it to 1e-12, rel. diff {err:.2e}")
    assert info.converged and err <= 1e-6
    s.close()


def _cheb_cycle_bytes(h, deg, fuse_below=2 ** 18):
    """Bytes of one FP64 Chebyshev(deg) V-cycle as the library counts them:
    per smoothing level 2 deg - 1 products with A, the restriction (R alone,
    or R and R A on their union pattern, 4 + 16 bytes per entry, where R A
    has fewer than 2^18 entries and the restriction joins the last
    pre-smoothing launch; finest level only), P and A P, six vectors per
    step, two diagonal reads, the coarse vectors; the dense coarsest
    inverse."""
    total = 0.0
    for l, lev in enumerate(h.levels[:-1]):
        A, P, R = lev.A.tocsr(), lev.P.tocsr(), lev.R.tocsr()
        n, nc = A.shape[0], P.shape[1]
        csr = lambda M: 12.0 * M.nnz + 8.0 * (M.shape[0] + 1)
        RA = (abs(R) @ abs(A)).tocsr()
        if l == 0 and RA.nnz < fuse_below:
            U = (abs(R) + RA).tocsr()
            rbytes = 20.0 * U.nnz + 8.0 * (nc + 1)
        else:
            rbytes = csr(R)
        AP = (abs(A) @ abs(P)).tocsr()
        total += csr(A) * (2 * deg - 1) + rbytes + csr(P) + csr(AP) + n * (6.0 * deg * 8 + 2 * 8) + nc * 2 * 8
    nL = h.levels[-1].A.shape[0]
    return total + 8.0 * nL * nL


@pytest.mark.parametrize("hname", ["H_SIG", "H_P"])
def test_fused_restriction_at_full_size(hname):
    """2D 256x64-cell system, 2000-row coarse grids, Chebyshev(4): the small
    finest levels of H_SIG and H_P restrict inside the last pre-smoothing
    launch (b_c = R r_{k-1} - (R A) d_k).  The cycle on the oracle's imported
    hierarchy matches the oracle's, and the bytes the library reports are the
    fused layout's (so the fused kernel ran)."""
    from oracle import amg
    bs, H = _oracle("c2", 2000)
    h = H[hname]
    s = _solver("c2", 2000, 4, (hname,))
    _import(s, H, [hname])
    b = np.random.default_rng(23).standard_normal(h.levels[0].A.shape[0])
    x = s.vcycle(hname, _dev(b)).cpu().numpy()
    got = s.vcycle_bytes(hname)
    s.close()
    ref = amg.vcycle_cheb(h, b, 4)
    assert _rel(x, ref) <= 1e-12, _rel(x, ref)
    expect = _cheb_cycle_bytes(h, 4)
    plain = _cheb_cycle_bytes(h, 4, fuse_below=0)
    print(f"{hname}: cycle bytes {got:.0f}, fused layout {expect:.0f}, separate restriction {plain:.0f}")
    assert abs(got - expect) <= 2e-3 * expect
    assert abs(plain - expect) >= 2e-2 * expect  # the two layouts are told apart
