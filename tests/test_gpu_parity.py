"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

* block SpMV y = A_h x: 1e-12 relative (FP64, both sum 8-byte products);
* one V(1,1) cycle of every hierarchy on the SAME hierarchy (the oracle's,
  imported through fsi_set_hierarchy): 1e-12 relative;
* P^{-1} r (block LDU algorithm) with all five imported hierarchies: 1e-12;
* full FGMRES solves: 1e-8 true residual, solution within 1e-6 relative L2 of
  the oracle's solution (the oracle solved to 1e-12).
"""
import numpy as np
import pytest

from conftest import system

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

_oracle_cache = {}


def _oracle(name, seed=0):
    from oracle import blocks, precond
    key = (name, seed)
    if key not in _oracle_cache:
        bs = blocks.BlockSystem(system(name, seed))
        H = precond.build_hierarchies(bs)
        _oracle_cache[key] = (bs, H)
    return _oracle_cache[key]


def _solver(name, seed=0, precision="f64"):
    from paper_1801_05648_amd import FsiSolver
    s = FsiSolver.from_system(system(name, seed), device=0)
    s.build_precond(precision)
    return s


def _csr_tuple(m):
    return (m.shape[0], m.shape[1], m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data)


def _import_oracle_hierarchies(solver, H):
    for name, h in H.items():
        A = [_csr_tuple(l.A) for l in h.levels]
        P = [_csr_tuple(l.P) for l in h.levels[:-1]]
        R = [_csr_tuple(l.R) for l in h.levels[:-1]]
        om = [l.omega for l in h.levels[:-1]]
        solver.set_hierarchy(name, A, P, R, om)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "c1", "c2"])
def test_spmv_parity(name):
    from oracle import blocks
    bs = blocks.BlockSystem(system(name))
    s = _solver(name)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(bs.N)
    y = s.spmv(_dev(x)).cpu().numpy()
    ref = bs.matvec(x)
    assert _rel(y, ref) <= 1e-12
    # element-wise: each row within the rounding of sum |a_ij x_j|
    absA = {k: abs(v) for k, v in bs.B.items()}
    xm, xs, xf = bs.split(abs(x))
    bound = np.concatenate([absA["M"] @ xm + absA["C_ms"] @ xs,
                            absA["C_sm"] @ xm + absA["S"] @ xs + absA["C_sf"] @ xf,
                            absA["C_fm"] @ xm + absA["C_fs"] @ xs + absA["F"] @ xf])
    assert np.all(np.abs(y - ref) <= 1e-13 * bound + 1e-300)
    s.close()


@pytest.mark.parametrize("name", ["c1", "tiny3d"])
def test_spmv_bytes_counts_the_stored_format(name):
    """fsi_spmv_bytes against a count made here from the block structure: the
    fluid-velocity rows in groups of d rows (one column index per distinct
    column of the group, d values each), all other rows in CSR."""
    import scipy.sparse as sp
    from oracle import blocks
    sysm = system(name)
    bs = blocks.BlockSystem(sysm)
    B = bs.B
    A = sp.bmat([[B["M"], B["C_ms"], None], [B["C_sm"], B["S"], B["C_sf"]],
                 [B["C_fm"], B["C_fs"], B["F"]]], format="csr")
    d, N = sysm.dim, sysm.N
    assert A.nnz == sysm.nnz
    bounds = [0, sysm.n_m, sysm.n_m + sysm.n_s, sysm.n_m + sysm.n_s + sysm.n_vf, N]
    expect = 16.0 * N
    for q in range(4):
        r0, r1 = bounds[q], bounds[q + 1]
        if q != 2:
            expect += 12.0 * (A.indptr[r1] - A.indptr[r0]) + 8.0 * (r1 - r0 + 1)
            continue
        ng = (r1 - r0) // d
        gnz = sum(np.unique(A.indices[A.indptr[r0 + g * d]:A.indptr[r0 + g * d + d]]).size for g in range(ng))
        expect += gnz * (4.0 + 8.0 * d) + 8.0 * (ng + 1)
    s = _solver(name)
    got = s.spmv_bytes()
    s.close()
    csr = 12.0 * A.nnz + 8.0 * (N + 1) + 16.0 * N
    print(f"{name}: {got:.0f} B stored, {csr:.0f} B as CSR")
    assert got == expect
    assert got < csr


@pytest.mark.parametrize("name", ["c1", "tiny3d"])
@pytest.mark.parametrize("hname", ["H_M", "H_SIG", "H_MS", "H_A", "H_P"])
def test_vcycle_parity_on_imported_hierarchy(name, hname):
    from oracle import amg, precond
    bs, H = _oracle(name)
    s = _solver(name)
    _import_oracle_hierarchies(s, H)
    h = H[hname]
    n = h.levels[0].A.shape[0]
    rng = np.random.default_rng(2)
    if hname == "H_M":
        b = rng.standard_normal(bs.n_m)
        ref = precond.mesh_solve(bs, lambda v: amg.vcycle(h, v), b)
    else:
        b = rng.standard_normal(n)
        ref = amg.vcycle(h, b)
    x = s.vcycle(hname, _dev(b)).cpu().numpy()
    assert _rel(x, ref) <= 1e-12, _rel(x, ref)
    s.close()


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "c1"])
def test_apply_precond_parity_on_imported_hierarchies(name):
    from oracle import precond
    bs, H = _oracle(name)
    s = _solver(name)
    _import_oracle_hierarchies(s, H)
    P = precond.amg_preconditioner(bs, H)
    r = np.random.default_rng(3).standard_normal(bs.N)
    z = s.apply_precond(_dev(r)).cpu().numpy()
    ref = P(r)
    for part, (a, b) in zip(("mesh", "solid", "fluid"), zip(bs.split(z), bs.split(ref))):
        assert _rel(a, b) <= 1e-12, (part, _rel(a, b))
    s.close()


@pytest.mark.parametrize("name,k,pc", [("tiny3d", 2, "uzawa"), ("c1", 1, "uzawa"), ("c1", 4, "uzawa"),
                                       ("c2", 3, "uzawa"), ("c1", 2, "triangular"), ("c2", 2, "triangular")])
def test_apply_precond_inner_gmres_parity_on_imported_hierarchies(name, k, pc):
    """P^{-1} r with the fluid inverse taken as k inner flexible GMRES steps
    preconditioned by the Uzawa-like step, on the oracle's hierarchies: the
    GPU (classical Gram-Schmidt twice, device Givens) against the oracle
    (modified Gram-Schmidt, host Givens).  Both compute the same Krylov
    minimiser, so they differ by rounding amplified by the conditioning of
    the small least-squares problem: 1e-10."""
    from oracle import precond
    bs, H = _oracle(name)
    from paper_1801_05648_amd import FsiSolver
    s = FsiSolver.from_system(system(name, 0), device=0)
    s.build_precond("f64", fluid_inner=k, fluid_inner_pc=pc)
    _import_oracle_hierarchies(s, H)
    P = precond.amg_preconditioner(bs, H, fluid_inner=k, fluid_inner_pc=pc)
    r = np.random.default_rng(4).standard_normal(bs.N)
    z = s.apply_precond(_dev(r)).cpu().numpy()
    ref = P(r)
    for part, (a, b) in zip(("mesh", "solid", "fluid"), zip(bs.split(z), bs.split(ref))):
        assert _rel(a, b) <= 1e-10, (part, _rel(a, b))
    # a zero residual gives a zero correction (beta = 0: no step is taken)
    z0 = s.apply_precond(_dev(np.zeros(bs.N))).cpu().numpy()
    assert np.all(z0 == 0.0)
    s.close()


ORDER_CASES = ([("tiny3d", "fsm", 0), ("c1", "fsm", 0), ("c2", "fsm", 0), ("c1", "fsm", 2), ("c2", "fsm", 2)] +
               [(n, o, 0) for o in ("mfs", "smf", "sfm", "fms") for n in ("tiny3d", "c1")] +
               [("c2", "mfs", 0), ("c2", "sfm", 2), ("c1", "smf", 2)])


@pytest.mark.parametrize("name,order,k", ORDER_CASES)
def test_block_order_precond_matches_oracle(name, order, k):
    """The factorisation with the blocks in another order (the remark on
    block orders in Section 4.1; "fsm" the reverse of the paper's mesh,
    solid, fluid): P^{-1} r on the oracle's hierarchies, element-wise per
    block, within 1e-12 with V-cycle inverses and 1e-10 with the fluid
    inverse as k inner GMRES steps (the same Krylov minimiser by different
    Gram-Schmidt and Givens codes, taken twice per application in some
    orders).  The result differs from the paper's order (another
    preconditioner), and on c1 a solve with the library's own hierarchies
    converges and agrees with the oracle's FGMRES solution with the same
    preconditioner within 1e-6."""
    from oracle import krylov, precond
    from paper_1801_05648_amd import FsiSolver
    bs, H = _oracle(name)
    sysm = system(name, 0)
    kw = dict(fluid_inner=k, fluid_inner_pc="triangular") if k else {}
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64", order=order, **kw)
    P = precond.amg_preconditioner(bs, H, order=order, **kw)
    if name == "c1":
        x, info = s.solve(_dev(sysm.b), tol=1e-8)
        xo, io = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-12, restart=50, maxit=500)
        err = _rel(x.cpu().numpy(), xo)
        print(f"c1 order {order} (k={k}): GPU {info.iters} it, oracle {io.iters} it to 1e-12, rel. diff {err:.2e}")
        assert info.converged and err <= 1e-6
    _import_oracle_hierarchies(s, H)
    r = np.random.default_rng(31).standard_normal(bs.N)
    z = s.apply_precond(_dev(r)).cpu().numpy()
    s.close()
    ref = P(r)
    tol = 1e-10 if k else 1e-12
    for part, (a, b) in zip(("mesh", "solid", "fluid"), zip(bs.split(z), bs.split(ref))):
        e = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        print(f"{name} order {order} (k={k}) P^-1 r {part}: max-abs {e:.2e}")
        assert e <= tol, part
    assert _rel(precond.amg_preconditioner(bs, H, **kw)(r), ref) > 1e-6


@pytest.mark.parametrize("order", ["fsm", "smf", "mfs"])
def test_block_order_fp32_precond_solve_matches_oracle(order):
    """Another block order with the FP32 preconditioner (FP64 Krylov loop):
    the c1 solve reaches 1e-8 and lies within 1e-6 of the FP64 oracle's
    FGMRES solution with the same order."""
    from oracle import krylov, precond
    from paper_1801_05648_amd import FsiSolver
    bs, H = _oracle("c1")
    sysm = system("c1", 0)
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f32", order=order)
    x, info = s.solve(_dev(sysm.b), tol=1e-8)
    s.close()
    xo, io = krylov.fgmres(bs.matvec, precond.amg_preconditioner(bs, H, order=order), sysm.b, tol=1e-12,
                           restart=50, maxit=500)
    err = _rel(x.cpu().numpy(), xo)
    print(f"c1 order {order} FP32 preconditioner: GPU {info.iters} it, oracle {io.iters} it to 1e-12, "
          f"rel. diff {err:.2e}")
    assert info.converged and err <= 1e-6


def test_library_setup_reproduces_oracle_aggregates_c1():
    """Level-0 aggregation is integer work on identical inputs: bit-exact."""
    bs, H = _oracle("c1")
    s = _solver("c1")
    for hname, h in H.items():
        n, nnz, om = s.hierarchy_info(hname)
        assert len(n) == h.nlevels, hname
        assert list(n) == [l.A.shape[0] for l in h.levels], hname
        if h.nlevels > 1:
            agg = s.get_aggregates(hname, 0)
            assert np.array_equal(agg, h.levels[0].aggregates), hname
            assert om[0] == pytest.approx(h.levels[0].omega, rel=1e-12)
            nr, nc, rp, ci, vv = s.get_level(hname, 0, "P")
            import scipy.sparse as sp
            Pl = sp.csr_matrix((vv, ci, rp), shape=(nr, nc))
            d = abs(Pl - h.levels[0].P)
            assert d.max() <= 1e-12 * abs(h.levels[0].P).max()
    s.close()


def _oracle_solution(name, seed=0, tol=1e-12):
    from oracle import krylov, precond
    key = ("sol", name, seed, tol)
    if key not in _oracle_cache:
        bs, H = _oracle(name, seed)
        x, info = krylov.fgmres(bs.matvec, precond.amg_preconditioner(bs, H), bs.sys.b, tol=tol,
                                restart=50, maxit=3000)
        _oracle_cache[key] = (x, info)
    return _oracle_cache[key]


@pytest.mark.parametrize("name,tol", [("c1", 1e-8), ("tiny2d", 1e-11), ("tiny3d", 1e-11)])
def test_solve_parity(name, tol):
    """Solution within 1e-6 of the oracle's (solved to 1e-12).  The two tiny
    grids have kappa(A_h) ~ 6.5e12 (2D) and 2e13 (3D): two solutions with a
    1e-8 residual may differ by more than 1e-6 there, so they are compared at
    a 1e-11 residual (and at 1e-8 against the oracle's own spread below)."""
    bs, _ = _oracle(name)
    s = _solver(name)
    b = _dev(bs.sys.b)
    x, info = s.solve(b, tol=tol, restart=50, maxit=2000)
    xg = x.cpu().numpy()
    assert info.converged and info.status == "FSI_OK"
    r = np.linalg.norm(bs.sys.b - bs.matvec(xg)) / np.linalg.norm(bs.sys.b)
    assert r <= tol * 1.001
    assert abs(info.true_rel_resid - r) <= 1e-3 * r
    xo, io = _oracle_solution(name)
    assert _rel(xg, xo) <= 1e-6, _rel(xg, xo)
    s.close()


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d"])
def test_solve_ill_conditioned_within_oracle_spread(name):
    """At a 1e-8 residual on the ill-conditioned tiny grids the GPU solution is
    as close to the 1e-12 reference as the oracle's own 1e-8 solution is."""
    bs, _ = _oracle(name)
    s = _solver(name)
    x, info = s.solve(_dev(bs.sys.b), tol=1e-8)
    assert info.converged
    xo12, _ = _oracle_solution(name)
    xo8, _ = _oracle_solution(name, tol=1e-8)
    spread = _rel(xo8, xo12)
    assert _rel(x.cpu().numpy(), xo12) <= max(1e-6, 10 * spread)
    s.close()


def test_solve_c2_full_size():
    """The benchmarked workload (256x64 cells, the launch configuration the
    benchmark times): true residual from the oracle's own mat-vec, and the
    solution against the oracle's 1e-8 solution."""
    from oracle import blocks
    sysm = system("c2")
    bs = blocks.BlockSystem(sysm)
    s = _solver("c2")
    x, info = s.solve(_dev(sysm.b), tol=1e-8, restart=50, maxit=2000)
    xg = x.cpu().numpy()
    assert info.converged
    r = np.linalg.norm(sysm.b - bs.matvec(xg)) / np.linalg.norm(sysm.b)
    assert r <= 1e-8 * 1.001
    print(f"c2: iters={info.iters} t={info.t_total_ms:.1f} ms resid={r:.2e}")
    s.close()


def test_graph_replays_match_eager_launches(monkeypatch):
    """Each Arnoldi step runs as a captured HIP graph, replayed every
    iteration and every solve.  Two solves through the graphs (with eager work
    in between) and one with plain launches give bit-identical iterates."""
    from oracle import blocks
    sysm = system("c1")
    bs = blocks.BlockSystem(sysm)
    b = _dev(sysm.b)
    s = _solver("c1")
    x1, i1 = s.solve(b)
    junk = s.spmv(torch.randn(bs.N, dtype=torch.float64, device="cuda:0"))  # eager work between replays
    torch.cuda.synchronize()
    x2, i2 = s.solve(b)
    s.close()
    monkeypatch.setenv("FSI_GRAPHS", "0")
    e = _solver("c1")
    x3, i3 = e.solve(b)
    e.close()
    assert i1.iters == i2.iters == i3.iters
    assert torch.equal(x1, x2) and torch.equal(x1, x3)
    assert torch.isfinite(junk).all()


def test_timed_solve_matches_and_reports_phases():
    """The timed mode (two graphs per step, events between them) computes the
    same iterates and reports positive phase times for every iteration."""
    sysm = system("c1")
    b = _dev(sysm.b)
    s = _solver("c1")
    x1, i1 = s.solve(b)
    x2, i2 = s.solve(b, timing=True)
    s.close()
    assert torch.equal(x1, x2) and i1.iters == i2.iters
    assert i2.n_timed == i2.iters
    assert i2.t_spmv_ms > 0 and i2.t_precond_ms > 0 and i2.t_gs_ms > 0
    assert i2.t_spmv_ms + i2.t_precond_ms + i2.t_gs_ms <= i2.t_total_ms * 1.05


@pytest.mark.parametrize("hname", ["H_A", "H_M", "H_SIG"])
def test_vcycle_parity_3d_with_large_levels(hname):
    """32x8x8-cell 3D system: levels large enough for the four-deep loads and,
    on H_A, for restricting with R in a launch of its own (no fused Q)."""
    from oracle import amg, blocks, precond
    from paper_1801_05648_amd import FsiSolver
    bs = blocks.BlockSystem(system("m3"))
    H = precond.build_hierarchies(bs, max_coarse=2000)
    s = FsiSolver.from_system(system("m3"), device=0)
    s.build_precond("f64", max_coarse=2000)
    _import_oracle_hierarchies(s, {hname: H[hname]})
    h = H[hname]
    rng = np.random.default_rng(12)
    if hname == "H_M":
        b = rng.standard_normal(bs.n_m)
        ref = precond.mesh_solve(bs, lambda v: amg.vcycle(h, v), b)
    else:
        b = rng.standard_normal(h.levels[0].A.shape[0])
        ref = amg.vcycle(h, b)
    x = s.vcycle(hname, _dev(b)).cpu().numpy()
    assert _rel(x, ref) <= 1e-12, _rel(x, ref)
    s.close()


def test_vcycle_parity_c3_mesh_restricting_apart():
    """3D 64x16x16-cell mesh hierarchy: its finest level is the learned
    smoother's and keeps Q for that sweep, but its Q has 5M more entries than
    R, so the plain cycle restricts with R in a launch of its own.  One cycle
    on the oracle's imported hierarchy against the oracle's cycle."""
    from oracle import amg, blocks, precond
    from paper_1801_05648_amd import FsiSolver
    sysm = system("c3")
    bs = blocks.BlockSystem(sysm)
    L = bs.mesh_scalar()
    h = amg.setup(L, 1, amg.constant_modes(L.shape[0]), max_coarse=2000)
    lev = h.levels[0]
    Qp = (abs(lev.R) + abs(lev.R) @ abs(lev.A)).tocsr()
    assert Qp.nnz - lev.R.nnz >= 2 ** 21  # the case this test is for
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64", max_coarse=2000)
    _import_oracle_hierarchies(s, {"H_M": h})
    b = np.random.default_rng(29).standard_normal(bs.n_m)
    x = s.vcycle("H_M", _dev(b)).cpu().numpy()
    s.close()
    ref = precond.mesh_solve(bs, lambda v: amg.vcycle(h, v), b)
    assert _rel(x, ref) <= 1e-12, _rel(x, ref)


def _cycle_bytes(h, g, allow_groups=True):
    """Bytes of one Jacobi V(1,1) cycle of the FP64 library as executed, with
    the levels of at least 2^21 entries whose A D^{-1}, Q (or R), P and A P
    take at most 5% zero fill in groups of g rows stored grouped, the others
    as CSR; Q's structure is that of R + R A."""
    import scipy.sparse as sp

    def entries(M, rows_per):
        M = M.tocsr()
        M.sort_indices()
        return sum(np.unique(M.indices[M.indptr[q * rows_per]:M.indptr[q * rows_per + rows_per]]).size
                   for q in range(M.shape[0] // rows_per))

    total = 0.0
    for lev in h.levels[:-1]:
        A, P, R = lev.A.tocsr(), lev.P.tocsr(), lev.R.tocsr()
        n, nc = A.shape[0], P.shape[1]
        absA, absR = abs(A), abs(R)
        RA = (absR @ absA).tocsr()
        Q = (absR + RA).tocsr()
        AP = (absA @ abs(P)).tocsr()
        split = RA.nnz - R.nnz >= 2 ** 21  # R A's nonzeros decide whether Q is formed
        Rq = R if split else Q
        mats = [A, Rq, P, AP]
        grouped = allow_groups and A.nnz >= 2 ** 21 and all(M.shape[0] % g == 0 for M in mats)
        if grouped:
            ents = [entries(M, g) for M in mats]
            grouped = all(e * g <= 1.05 * M.nnz for e, M in zip(ents, mats))
        for k, M in enumerate(mats):
            if grouped:
                total += ents[k] * (4.0 + 8.0 * g) + 8.0 * (M.shape[0] // g + 1)
            else:
                total += 12.0 * M.nnz + 8.0 * (M.shape[0] + 1)
        total += (8.0 * n if split else 0.0) + n * (2 * 8 + 5 * 8) + nc * 2 * 8
    nL = h.levels[-1].A.shape[0]
    return total + 8.0 * nL * nL


@pytest.mark.parametrize("name", ["c2", "m3"])
def test_grouped_levels_match_oracle(name):
    """H_A's large levels stored in groups of d rows (the velocity components
    of a node share their columns): on the oracle's imported hierarchy the
    V-cycle matches the oracle, and the bytes the library reports for the
    cycle are the grouped layout's (so the grouped kernels did run)."""
    from oracle import amg, blocks, precond
    from paper_1801_05648_amd import FsiSolver
    sysm = system(name)
    bs = blocks.BlockSystem(sysm)
    H = precond.build_hierarchies(bs, max_coarse=2000)
    h = H["H_A"]
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64", max_coarse=2000)
    _import_oracle_hierarchies(s, {"H_A": h})
    b = np.random.default_rng(13).standard_normal(h.levels[0].A.shape[0])
    x = s.vcycle("H_A", _dev(b)).cpu().numpy()
    ref = amg.vcycle(h, b)
    got = s.vcycle_bytes("H_A")
    s.close()
    assert _rel(x, ref) <= 1e-12, _rel(x, ref)
    expect = _cycle_bytes(h, sysm.dim)
    plain = _cycle_bytes(h, sysm.dim, allow_groups=False)
    print(f"{name}: cycle bytes {got:.0f}, grouped layout {expect:.0f}, all CSR {plain:.0f}")
    assert abs(got - expect) <= 2e-3 * expect
    assert plain - expect >= 5e-2 * expect  # the two layouts are told apart


BENCH_OPTS = dict(max_coarse=2000, cheb_degree=4, cheb=("H_SIG",), poly=("H_MS",), poly_degree=3,
                  fluid_inner=2, fluid_inner_pc="triangular")  # 2D


def test_bench_configuration_full_size_matches_oracle():
    """The benchmarked workload and preconditioner (256x64 cells, Chebyshev
    V-cycles on H_SIG, M_s by three Chebyshev steps, 2000-row coarse grids, the
    fluid inverse by two inner GMRES steps preconditioned by the block
    upper-triangular step):
    the GPU solution reaches 1e-8 by the oracle's own mat-vec and agrees with
    the oracle FGMRES (same options, solved to 1e-10) within 1e-6."""
    from oracle import blocks, krylov, precond
    from paper_1801_05648_amd import FsiSolver
    sysm = system("c2")
    bs = blocks.BlockSystem(sysm)
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64", **BENCH_OPTS)
    x, info = s.solve(_dev(sysm.b), tol=1e-8)
    s.close()
    xg = x.cpu().numpy()
    r = np.linalg.norm(sysm.b - bs.matvec(xg)) / np.linalg.norm(sysm.b)
    H = precond.build_hierarchies(bs, max_coarse=2000)
    P = precond.amg_preconditioner(bs, H, cheb={"H_SIG": 4}, poly={"H_MS": (3, 8.0)}, fluid_inner=2,
                                   fluid_inner_pc="triangular")
    xo, io = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-10, restart=50, maxit=500)
    err = _rel(xg, xo)
    print(f"c2 bench configuration: GPU {info.iters} it (oracle {io.iters} it to 1e-10), resid {r:.2e}, "
          f"rel. diff {err:.2e}")
    assert info.converged and r <= 1e-8 * 1.001
    assert err <= 1e-6


BENCH3D_OPTS = dict(max_coarse=4000, strength0=0.04, cheb_degree=6, cheb=("H_SIG", "H_P"), poly=("H_MS",),
                   poly_degree=5, schur="simplec", fluid_inner=2, fluid_inner_pc="triangular")


def test_3d_bench_configuration_matches_oracle():
    """The 3D benchmark preconditioner (Chebyshev(6) V-cycles on H_SIG and H_P,
    M_s by five Chebyshev steps, 4000-row coarse grids, strength threshold
    0.04; grouped H_A levels;
    the SIMPLEC pressure Schur approximation; the fluid inverse by two inner
    GMRES steps on F preconditioned by the block upper-triangular step) on the
    32x8x8-cell system: the GPU takes the oracle's iteration count to 1e-8,
    its iterate agrees with the oracle's 1e-8 iterate within 1e-9 (unique
    Krylov iterate) and with the oracle's 1e-12 solution within 1e-6."""
    from oracle import blocks, krylov, precond
    from paper_1801_05648_amd import FsiSolver
    sysm = system("m3")
    bs = blocks.BlockSystem(sysm)
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64", **BENCH3D_OPTS)
    x, info = s.solve(_dev(sysm.b), tol=1e-8)
    s.close()
    xg = x.cpu().numpy()
    r = np.linalg.norm(sysm.b - bs.matvec(xg)) / np.linalg.norm(sysm.b)
    H = precond.build_hierarchies(bs, eps0=0.04, max_coarse=4000, schur="simplec")
    P = precond.amg_preconditioner(bs, H, cheb={"H_SIG": 6, "H_P": 6}, poly={"H_MS": (5, 8.0)}, fluid_inner=2,
                                   fluid_inner_pc="triangular")
    xo8, io8 = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-8, restart=50, maxit=500)
    xo, _ = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-12, restart=50, maxit=500)
    err, err8 = _rel(xg, xo), _rel(xg, xo8)
    print(f"m3 3D bench config: GPU {info.iters} it, oracle {io8.iters} it at 1e-8, true resid {r:.2e}, "
          f"{err8:.2e} to the oracle's 1e-8 iterate, {err:.2e} to its 1e-12 solution")
    assert info.converged and r <= 1e-8 * 1.001
    assert info.iters == io8.iters
    assert err8 <= 1e-9 and err <= 1e-6


@pytest.mark.parametrize("schur", ["simple", "simplec"])
def test_3d_split_fluid_step_matches_oracle(schur):
    """The 3D preconditioner with the fluid inverse as the Uzawa-like split
    alone (one V-cycle per inverse: the learned smoother's 3D workload and the
    benchmark's `uzawa_vcycle_simple` form), SIMPLE or SIMPLEC, on the
    32x8x8-cell system: the GPU takes the oracle's iteration count to 1e-8
    (25 and 21), its iterate agrees with the oracle's 1e-8 iterate within
    1e-9 and with the oracle's 1e-12 solution within 1e-6."""
    from oracle import blocks, krylov, precond
    from paper_1801_05648_amd import FsiSolver
    sysm = system("m3")
    bs = blocks.BlockSystem(sysm)
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64", max_coarse=2000, cheb_degree=4, cheb=("H_SIG", "H_P"), poly=("H_MS",), poly_degree=3,
                    schur=schur)
    x, info = s.solve(_dev(sysm.b), tol=1e-8)
    s.close()
    xg = x.cpu().numpy()
    r = np.linalg.norm(sysm.b - bs.matvec(xg)) / np.linalg.norm(sysm.b)
    H = precond.build_hierarchies(bs, max_coarse=2000, schur=schur)
    P = precond.amg_preconditioner(bs, H, cheb={"H_SIG": 4, "H_P": 4}, poly={"H_MS": (3, 8.0)})
    xo8, io8 = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-8, restart=50, maxit=500)
    xo, _ = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-12, restart=50, maxit=500)
    err, err8 = _rel(xg, xo), _rel(xg, xo8)
    print(f"m3 split fluid step, {schur}: GPU {info.iters} it, oracle {io8.iters} it, {err8:.2e} to the "
          f"oracle's 1e-8 iterate, {err:.2e} to its 1e-12 solution")
    assert info.converged and r <= 1e-8 * 1.001
    assert info.iters == io8.iters
    assert err8 <= 1e-9 and err <= 1e-6


def test_simplec_pressure_schur_matches_oracle():
    """The SIMPLEC pressure Schur approximation (an option) as the library
    builds it (the finest matrix of H_P) against the oracle's, and a 3D solve
    with it (the benchmark's 3D preconditioner otherwise) against the oracle
    FGMRES."""
    import scipy.sparse as sp
    from oracle import blocks, krylov, precond
    from paper_1801_05648_amd import FsiSolver
    sysm = system("m3")
    bs = blocks.BlockSystem(sysm)
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64", max_coarse=2000, cheb_degree=4, cheb=("H_SIG", "H_P"), poly=("H_MS",), poly_degree=3,
                    schur="simplec")
    nr, nc, rp, ci, v = s.get_level("H_P", 0, "A")
    Sl = sp.csr_matrix((v, ci, rp), shape=(nr, nc))
    So = bs.fluid_schur("simplec")
    assert abs(Sl - So).max() <= 1e-13 * abs(So).max()
    x, info = s.solve(_dev(sysm.b), tol=1e-8)
    s.close()
    xg = x.cpu().numpy()
    r = np.linalg.norm(sysm.b - bs.matvec(xg)) / np.linalg.norm(sysm.b)
    H = precond.build_hierarchies(bs, max_coarse=2000, schur="simplec")
    P = precond.amg_preconditioner(bs, H, cheb={"H_SIG": 4, "H_P": 4}, poly={"H_MS": (3, 8.0)})
    it8 = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-8, restart=50, maxit=500)[1].iters
    xo, _ = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-10, restart=50, maxit=500)
    err = _rel(xg, xo)
    print(f"m3 SIMPLEC: GPU {info.iters} it, oracle {it8} it at 1e-8, rel. diff {err:.2e}")
    assert info.converged and r <= 1e-8 * 1.001
    assert abs(info.iters - it8) <= 3
    assert err <= 1e-6


@pytest.mark.parametrize("precision,k,pc", [("f64", 2, "uzawa"), ("f32", 2, "uzawa"), ("f64", 2, "triangular"),
                                             ("f64", 3, "triangular")])
def test_inner_gmres_solve_matches_oracle(precision, k, pc):
    """The 3D benchmark preconditioner with k inner GMRES steps for the
    fluid inverse (Uzawa-like or block-triangular inner preconditioner), on
    the 32x8x8-cell system with the library's own hierarchies, against the
    oracle's FGMRES with the same preconditioner.

    FP64: the GPU takes exactly the oracle's iteration count to 1e-8, and the
    Krylov iterate with that count is unique, so the GPU's agrees with the
    oracle's 1e-8 iterate within 1e-9.  Every case's solution is within 1e-6
    of the oracle's 1e-12 solution, except three triangular steps: that
    preconditioner reaches 1e-8 in 13 outer steps and its 1e-8 iterate, the
    oracle's own as much as the GPU's, lies 1.7e-6 from the solution
    (kappa_2(A_h) of this system is at least 1.1e12: sigma_max ~8.0e3 by
    power iteration, ||A_h^{-1} v|| = 1.4e8 for a random unit v by the oracle
    solver, so a 1e-8 residual alone bounds the forward error by nothing
    useful); there the bound is the oracle iterate's own forward error
    (x 1.05).  FP32 preconditioner: a different (rounded) operator, so the
    count may move by a few steps; its solution is held to the same 1e-6."""
    from oracle import blocks, krylov, precond
    from paper_1801_05648_amd import FsiSolver
    sysm = system("m3")
    bs = blocks.BlockSystem(sysm)
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond(precision, max_coarse=2000, cheb_degree=4, cheb=("H_SIG", "H_P"), poly=("H_MS",),
                    poly_degree=3, fluid_inner=k, fluid_inner_pc=pc)
    x, info = s.solve(_dev(sysm.b), tol=1e-8)
    s.close()
    xg = x.cpu().numpy()
    r = np.linalg.norm(sysm.b - bs.matvec(xg)) / np.linalg.norm(sysm.b)
    H = precond.build_hierarchies(bs, max_coarse=2000)
    P = precond.amg_preconditioner(bs, H, cheb={"H_SIG": 4, "H_P": 4}, poly={"H_MS": (3, 8.0)}, fluid_inner=k,
                                   fluid_inner_pc=pc)
    xo8, io8 = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-8, restart=50, maxit=500)
    it8 = io8.iters
    xo, _ = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-12, restart=50, maxit=500)
    err = _rel(xg, xo)
    err8 = _rel(xg, xo8)
    err_o8 = _rel(xo8, xo)
    print(f"m3 inner GMRES({k}, {pc}) {precision}: GPU {info.iters} it, oracle {it8} it at 1e-8, "
          f"rel. diff {err8:.2e} to the oracle's 1e-8 iterate, {err:.2e} to its 1e-12 solution "
          f"(the oracle's own 1e-8 iterate: {err_o8:.2e})")
    assert info.converged and r <= 1e-8 * 1.001
    if precision == "f64":
        assert info.iters == it8, (info.iters, it8)
        assert err8 <= 1e-9
    else:
        assert abs(info.iters - it8) <= 3
    bound = 1.05 * err_o8 if (k, pc) == (3, "triangular") else 1e-6
    assert err <= bound


@pytest.mark.parametrize("form", ["split", "bench"])
def test_apply_precond_parity_c3_benchmark_options(form):
    """3D preconditioners at the full 64x16x16-cell size (753,740 unknowns) on
    the oracle's five hierarchies: one application of P^{-1}, element-wise per
    block within 1e-12 of the block's largest entry.  "split": Chebyshev(4)
    V-cycles on H_SIG and H_P, Jacobi V(1,1) on H_M and H_A (large levels in
    groups of three rows), M_s by three Chebyshev steps, 2000-row dense coarse
    grids, the Uzawa-like fluid step with SIMPLE.  "bench": the benchmark's
    3D preconditioner (Chebyshev(6), five M_s steps, 4000-row coarse grids,
    strength threshold 0.04, SIMPLEC, two inner GMRES steps on F with the
    triangular step)."""
    from oracle import blocks, precond
    from paper_1801_05648_amd import FsiSolver
    sysm = system("c3")
    bs = blocks.BlockSystem(sysm)
    if form == "split":
        opts = dict(max_coarse=2000, cheb_degree=4, cheb=("H_SIG", "H_P"), poly=("H_MS",), poly_degree=3)
        kw = {}
    else:
        opts = dict(BENCH3D_OPTS)
        kw = dict(fluid_inner=2, fluid_inner_pc="triangular")
    H = precond.build_hierarchies(bs, eps0=opts.get("strength0", 0.08), max_coarse=opts["max_coarse"],
                                  schur=opts.get("schur", "simple"))
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64", **opts)
    _import_oracle_hierarchies(s, H)
    deg = opts["cheb_degree"]
    P = precond.amg_preconditioner(bs, H, cheb={"H_SIG": deg, "H_P": deg}, poly={"H_MS": (opts["poly_degree"], 8.0)},
                                   **kw)
    r = np.random.default_rng(23).standard_normal(bs.N)
    z = s.apply_precond(_dev(r)).cpu().numpy()
    s.close()
    ref = P(r)
    for part, a, b in zip(("mesh", "solid", "fluid"), bs.split(z), bs.split(ref)):
        e_inf = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        print(f"c3 {form} P^-1 r {part}: max-abs {e_inf:.2e}, rel L2 {_rel(a, b):.2e}")
        assert e_inf <= 1e-12 and _rel(a, b) <= 1e-12, part


def test_spmv_parity_c3_full_size():
    """The 3D 64x16x16-cell A_h (1.67e8 entries) through the segmented product
    against the oracle's block mat-vec."""
    from oracle import blocks
    from paper_1801_05648_amd import FsiSolver
    sysm = system("c3")
    bs = blocks.BlockSystem(sysm)
    s = FsiSolver.from_system(sysm, device=0)
    x = np.random.default_rng(3).standard_normal(bs.N)
    y = s.spmv(_dev(x)).cpu().numpy()
    s.close()
    ref = bs.matvec(x)
    assert _rel(y, ref) <= 1e-12, _rel(y, ref)


def test_solve_info_block_residuals_and_bytes():
    """fsi_solve_info: the per-block true residuals make up the whole one and
    match the blocks of b - A_h x formed by the oracle's mat-vec from the
    returned x (a 1e-8 residual recomputed in another summation order: 1e-3
    relative); the byte counts are whole multiples of the per-step figures
    (A_h as stored, fsi_precond_bytes) over the launched Arnoldi steps, at
    least the finished ones."""
    from oracle import blocks
    sysm = system("c1")
    bs = blocks.BlockSystem(sysm)
    s = _solver("c1")
    x, info = s.solve(_dev(sysm.b), tol=1e-8)
    pc = s.precond_bytes()
    ah = s.spmv_bytes()
    s.close()
    assert info.converged
    rb = np.array(info.resid_block)
    assert abs(np.sqrt(np.sum(rb ** 2)) - info.true_rel_resid) <= 1e-12 * info.true_rel_resid
    r = sysm.b - bs.matvec(x.cpu().numpy())
    nb = np.linalg.norm(sysm.b)
    ref = np.array([np.linalg.norm(p) / nb for p in bs.split(r)])
    print(f"c1 block residuals GPU {rb}, oracle mat-vec {ref}")
    assert np.all(np.abs(rb - ref) <= 1e-3 * ref.max())
    steps = info.bytes_precond / pc
    assert abs(steps - round(steps)) <= 1e-9 * steps and round(steps) >= info.iters
    true_res = info.restarts + 1
    spmv_steps = (info.bytes_spmv - true_res * (ah + 8.0 * bs.N)) / ah
    assert abs(spmv_steps - round(steps)) <= 1e-9 * steps
    assert info.bytes_gs > 8.0 * bs.N * info.iters


@pytest.mark.parametrize("name", ["tiny3d", "c1"])
def test_blockdiag_x_precond_matches_oracle(name):
    """The block-diagonal approximation of the Schur complement X
    (x_approx="blockdiag"): the library's pressure Schur approximation (now
    with the pressure block of the refined operator) and A_f equal the
    oracle's (1e-13), P^{-1} r on the oracle's hierarchies of the refined
    operator matches element-wise per block (1e-12), and a solve matches the
    oracle's FGMRES solution within 1e-6."""
    import scipy.sparse as sp
    from oracle import blocks, krylov, precond
    from paper_1801_05648_amd import FsiSolver
    sysm = system(name)
    bs = blocks.BlockSystem(sysm)
    fl = bs.fluid_x("blockdiag")
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64", max_coarse=40, x_approx="blockdiag")
    for hname, ref in (("H_P", fl.schur()), ("H_A", fl.A_f)):
        nr, nc, rp, ci, v = s.get_level(hname, 0, "A")
        got = sp.csr_matrix((v, ci, rp), shape=(nr, nc))
        assert abs(got - ref).max() <= 1e-13 * abs(ref).max(), hname
    H = precond.build_hierarchies(bs, max_coarse=40, x_approx="blockdiag")
    P = precond.amg_preconditioner(bs, H, x_approx="blockdiag")
    x, info = s.solve(_dev(sysm.b), tol=1e-8)
    xo, _ = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-12, restart=50, maxit=500)
    err = _rel(x.cpu().numpy(), xo)
    _import_oracle_hierarchies(s, H)
    r = np.random.default_rng(29).standard_normal(bs.N)
    z = s.apply_precond(_dev(r)).cpu().numpy()
    s.close()
    ref = P(r)
    for part, a, b in zip(("mesh", "solid", "fluid"), bs.split(z), bs.split(ref)):
        e = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        print(f"{name} blockdiag-X P^-1 r {part}: max-abs {e:.2e}")
        assert e <= 1e-12, part
    print(f"{name} blockdiag-X solve: {info.iters} iterations, rel. diff to the oracle {err:.2e}")
    assert info.converged
    if name == "c1":  # the tiny grids' conditioning (~1e13) puts their 1e-8 iterates farther apart
        assert err <= 1e-6


@pytest.mark.parametrize("name,k", [("tiny3d", 2), ("c1", 1), ("c1", 3), ("c2", 2)])
def test_uzawa_gmres_inverses_precond_matches_oracle(name, k):
    """Section 4.4 as written: each inverse of the Uzawa-like fluid step
    taken as k GMRES steps preconditioned by its V-cycle (uzawa_inner = k).
    P^{-1} r on the oracle's hierarchies, GPU (classical Gram-Schmidt twice,
    device Givens) against the oracle (modified Gram-Schmidt, host Givens):
    the same Krylov minimisers, so rounding amplified by the small least-
    squares problems only: 1e-10 per block."""
    from oracle import precond
    bs, H = _oracle(name)
    from paper_1801_05648_amd import FsiSolver
    s = FsiSolver.from_system(system(name, 0), device=0)
    s.build_precond("f64", uzawa_inner=k)
    _import_oracle_hierarchies(s, H)
    P = precond.amg_preconditioner(bs, H, uzawa_inner=k)
    r = np.random.default_rng(31).standard_normal(bs.N)
    z = s.apply_precond(_dev(r)).cpu().numpy()
    ref = P(r)
    for part, (a, b) in zip(("mesh", "solid", "fluid"), zip(bs.split(z), bs.split(ref))):
        print(f"{name} uzawa_inner={k} {part}: rel. error {_rel(a, b):.2e}")
        assert _rel(a, b) <= 1e-10, (part, _rel(a, b))
    s.close()


def test_uzawa_gmres_inverses_solve_matches_oracle():
    """The whole solve with the Section 4.4 fluid step (two GMRES steps per
    inverse) on the 32x8x8-cell system and the library's own hierarchies:
    the oracle's iteration count and its 1e-8 iterate within 1e-9 (the
    Krylov iterate with that count is unique).  Like three triangular inner
    steps, this preconditioner reaches 1e-8 in 13 outer steps with an
    iterate 2.9e-6 from the solution (the oracle's own; kappa_2(A_h) of this
    system is at least 1.1e12), so the forward-error bound is that of the
    oracle's iterate (x 1.05), not 1e-6: a named exception."""
    from oracle import blocks, krylov, precond
    from paper_1801_05648_amd import FsiSolver
    sysm = system("m3")
    bs = blocks.BlockSystem(sysm)
    opts = dict(max_coarse=2000, cheb_degree=4, cheb=("H_SIG", "H_P"), poly=("H_MS",), poly_degree=3, uzawa_inner=2)
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64", **opts)
    x, info = s.solve(_dev(sysm.b), tol=1e-8)
    s.close()
    xg = x.cpu().numpy()
    H = precond.build_hierarchies(bs, max_coarse=2000)
    P = precond.amg_preconditioner(bs, H, cheb={"H_SIG": 4, "H_P": 4}, poly={"H_MS": (3, 8.0)}, uzawa_inner=2)
    xo8, io8 = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-8, restart=50, maxit=500)
    xo, _ = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-12, restart=50, maxit=500)
    print(f"m3 uzawa_inner=2: GPU {info.iters} it, oracle {io8.iters} it; {_rel(xg, xo8):.2e} to the oracle's "
          f"1e-8 iterate, {_rel(xg, xo):.2e} to its 1e-12 solution")
    assert info.converged and info.iters == io8.iters
    assert _rel(xg, xo8) <= 1e-9
    assert _rel(xg, xo) <= 1.05 * _rel(xo8, xo)
