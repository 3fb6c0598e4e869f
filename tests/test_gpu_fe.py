"""GPU finite-element assembly and quasi-Newton loop against the oracle.

The library assembles the discrete ALE-FSI residual R(U) of Section 3 and its
Jacobian A'(U) on the device (fsi_fe_residual, fsi_fe_jacobian) and runs the
quasi-Newton loop of Section 6 (fsi_newton).  The oracle (oracle/fe.py)
evaluates the same residual with numpy and the Jacobian by complex steps.

* residual: element by element within 1e-12 of the largest residual entry
  (sums of cell contributions in another order), at the given fields and at
  a state off them, on 2D and 3D grids of several cells per chunk of 32 local
  rows and both cell parities (tiny2d, tiny3d, c1, m3);
* Jacobian: the assembled A_h times a random vector against the oracle's
  A'(U) times it, per row within 1e-12 of sum_j |a_ij x_j| -- the product
  every Krylov step uses, so every stored value (plain rows and the d-row
  groups of the fluid velocity) is exercised; on m3 the rows whose cells lie
  in a sample of slabs (the solid's upstream face and the outflow);
* Newton: the converged iterate's oracle residual meets the stopping test,
  the residual norms the library reports equal the oracle's at its final
  iterate, the reassembly decisions follow the rule on the reported norms, and
  the iterate is near the oracle's exact-Newton root.
"""
import ctypes

import numpy as np
import pytest
import torch

import fsigen
from oracle import fe

pytestmark = pytest.mark.gpu

_cache = {}


def _sys(name, **over):
    key = (name, tuple(sorted(over.items())))
    if key not in _cache:
        s = fsigen.generate(fsigen.config(name, **over), fe=True)
        _cache[key] = (s, fe.FeProblem(s.cfg, s.fe, s.N))
    return _cache[key]


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _state(s, seed):
    """A state off the given fields: small smooth-ish offsets on the free dofs."""
    return np.random.default_rng(seed).standard_normal(s.N) * 1e-3


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "c1", "m3"])
def test_residual_matches_oracle(name):
    from paper_1801_05648_amd import FsiSolver
    s, P = _sys(name)
    g = FsiSolver.from_system(s, device=0)
    for dU in (None, _state(s, 1)):
        Rg = g.fe_residual(None if dU is None else _dev(dU)).cpu().numpy()
        Ro = P.residual(dU)
        err = np.max(np.abs(Rg - Ro))
        print(f"{name} residual ({'fields' if dU is None else 'offset'}): max diff {err:.2e} of {np.max(np.abs(Ro)):.2e}")
        assert err <= 1e-12 * np.max(np.abs(Ro)), err
    g.close()


def _sample_cells(s):
    """m3: three slabs of cells across the solid's upstream face and the
    outflow slab (the oracle's complex steps over all 2048 cells take minutes)."""
    C = np.stack(np.meshgrid(*[np.arange(n) for n in s.cfg.cells], indexing="ij"), -1).reshape(-1, s.dim)
    return np.nonzero(((C[:, 0] >= 7) & (C[:, 0] < 10)) | (C[:, 0] == s.cfg.cells[0] - 1))[0]


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "c1", "m3"])
def test_jacobian_matches_oracle(name):
    from paper_1801_05648_amd import FsiSolver
    s, P = _sys(name)
    g = FsiSolver.from_system(s, device=0)
    dU = _state(s, 2)
    g.fe_jacobian(_dev(dU), host_blocks=False)
    if name == "m3":
        cells = _sample_cells(s)
        A = P.jacobian(dU, cells)
        rows = fe.rows_covered(P, cells)
    else:
        A = P.jacobian(dU)
        rows = np.arange(s.N)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(s.N)
    y = g.spmv(_dev(x)).cpu().numpy()[rows]
    ref = (A @ x)[rows]
    bound = (abs(A) @ np.abs(x))[rows]
    rel = np.max(np.abs(y - ref) / (bound + 1e-300))
    print(f"{name} Jacobian product on {len(rows)} of {s.N} rows: max |diff| / sum|a x| = {rel:.2e}")
    assert np.all(np.abs(y - ref) <= 1e-12 * bound + 1e-300), rel
    g.close()


def test_jacobian_at_the_given_fields_is_the_generators_matrix():
    """At dU = 0 the device assembly reproduces the matrix the context was
    set up with (the generator's, a third implementation)."""
    from paper_1801_05648_amd import FsiSolver
    s, _ = _sys("tiny3d")
    g = FsiSolver.from_system(s, device=0)
    x = _dev(np.random.default_rng(4).standard_normal(s.N))
    y0 = g.spmv(x).cpu().numpy()
    g.fe_jacobian(None, host_blocks=True)
    y1 = g.spmv(x).cpu().numpy()
    assert np.max(np.abs(y1 - y0)) <= 1e-12 * np.max(np.abs(y0))
    g.close()


@pytest.mark.parametrize("name,precond,root", [("tiny2d", "rebuild", True), ("c1", "rebuild", True),
                                               ("c1", "keep", True), ("tiny3d", "reuse", True),
                                               ("m3", "rebuild", False)])
def test_newton_matches_oracle(name, precond, root):
    from paper_1801_05648_amd import FsiSolver
    s, P = _sys(name)
    g = FsiSolver.from_system(s, device=0)
    g.build_precond("f64")
    dU, info = g.newton(precond=precond)
    torch.cuda.synchronize()
    r = info.residuals
    print(f"{name} ({precond}): {info.status} {info.steps} steps, {info.reassemblies} assemblies, "
          f"GMRES {info.lin_iters}, ||r||_inf {['%.2e' % v for v in r]}, {info.t_total_ms:.1f} ms")
    assert info.converged and info.status == "FSI_OK"
    # Section 6's rule on the reported norms
    for k, a in enumerate(info.reassembled):
        assert a == (k == 0 or r[k] > 0.1 * r[k - 1]), (k, r)
    assert r[-1] < 1e-6 * r[0] and all(r[k] >= 1e-6 * r[0] for k in range(len(r) - 1))
    dUg = dU.cpu().numpy()
    Ro = P.residual(dUg)
    r0 = np.max(np.abs(P.residual()))
    assert abs(r[0] - r0) <= 1e-12 * r0
    # the library's last norm is the oracle's residual at that iterate
    assert abs(np.max(np.abs(Ro)) - r[-1]) <= 1e-11 * r0, (np.max(np.abs(Ro)), r[-1])
    assert np.max(np.abs(Ro)) < 1e-6 * r0
    if root:
        dUo, io = fe.quasi_newton(P.residual, P.jacobian, s.N, rtol=1e-12, ratio=0.0)
        dist = np.max(np.abs(dUg - dUo)) / np.max(np.abs(dUo))
        print(f"  oracle exact Newton: {io.steps} steps; iterate distance {dist:.2e} (max-norm, relative)")
        assert dist <= 1e-4, dist
    g.close()


def test_fe_errors_are_reported():
    from paper_1801_05648_amd import FsiSolver
    from paper_1801_05648_amd.fsi import FsiError
    s, P = _sys("tiny2d")
    plain = fsigen.generate("tiny2d")
    g = FsiSolver.from_system(plain, device=0)
    with pytest.raises(FsiError) as e:
        g.fe_residual(None)
    assert e.value.name == "FSI_ERR_STATE"
    bad = dict(s.fe)
    bad["vdof"] = s.fe["vdof"].copy()
    k = int(np.nonzero(bad["vdof"] >= 0)[0][0])
    bad["vdof"][k] = s.N + 5  # out of range
    with pytest.raises(FsiError) as e:
        g.fe_setup(s.cfg, bad)
    assert e.value.name == "FSI_ERR_ARG"
    with pytest.raises(FsiError) as e:
        g.fe_setup(s.cfg.with_(dt=2e-2), s.fe)
    assert e.value.name == "FSI_ERR_ARG"
    # a grid whose parity classes do not fit one launch each is refused before
    # any node array is read (the arrays are NULL here)
    from paper_1801_05648_amd.fsi import CFeMesh
    m = CFeMesh()
    m.dim = 2
    for a in range(3):
        m.cells[a] = 65535 if a < 2 else 1
        m.extent[a] = 1.0
        m.solid_hi[a] = 1
    for k in ("rho_f", "nu_f", "rho_s", "mu_s", "lambda_s", "dt", "theta"):
        setattr(m, k, float(getattr(s.cfg, k)))
    m.n_nodes = 131071 ** 2
    with pytest.raises(FsiError) as e:
        g._check(g.lib.fsi_fe_setup(g.ctx, ctypes.byref(m)))
    assert e.value.name == "FSI_ERR_ARG" and "2^31" in str(e.value)
    g.fe_setup(s.cfg, s.fe)
    # a displacement offset that folds a fluid cell: J <= 0 is reported, not assembled
    dU = np.zeros(s.N)
    dU[:s.n_m] = 10.0 * np.random.default_rng(5).standard_normal(s.n_m)
    with pytest.raises(FsiError) as e:
        g.fe_residual(_dev(dU))
    assert e.value.name == "FSI_ERR_NUMERIC"
    # a failed Jacobian assembly leaves A_h as it was
    x = _dev(np.random.default_rng(6).standard_normal(s.N))
    y0 = g.spmv(x).cpu().numpy()
    with pytest.raises(FsiError) as e:
        g.fe_jacobian(_dev(dU), host_blocks=True)
    assert e.value.name == "FSI_ERR_NUMERIC"
    assert np.array_equal(g.spmv(x).cpu().numpy(), y0)
    R = g.fe_residual(None).cpu().numpy()  # the context still works
    assert np.max(np.abs(R - P.residual())) <= 1e-12 * np.max(np.abs(R))
    g.close()


# ---------------------------------------------------------------- theta scheme
def _theta_case(name, theta, seed=21):
    """A theta step on a workload: the generator's pattern and layout at dt theta
    (so that the layout's dt theta is the step's), the workload's fields with a
    previous level off the given one."""
    base = fsigen.config(name)
    s = fsigen.generate(base.with_(dt=base.dt * theta), fe=True)
    f = {k: np.array(v, copy=True) for k, v in s.fe.items()}
    rng = np.random.default_rng(seed)
    f["v_old"] = 0.8 * f["v"] + 0.05 * rng.standard_normal(f["v"].shape)
    f["u_old"] = 0.7 * f["u"]
    return s, base.with_(theta=theta), f


@pytest.mark.parametrize("name,theta", [("tiny2d", 0.5), ("tiny3d", 0.51), ("c1", 0.51)])
def test_theta_residual_and_jacobian_match_oracle(name, theta):
    from paper_1801_05648_amd import FsiSolver
    s, cfg, f = _theta_case(name, theta)
    P = fe.FeProblem(cfg, f, s.N)
    g = FsiSolver.from_system(s, device=0)
    g.fe_setup(cfg, f)
    dU = _state(s, 3)
    Rg = g.fe_residual(_dev(dU)).cpu().numpy()
    Ro = P.residual(dU)
    err = np.max(np.abs(Rg - Ro))
    assert err <= 1e-12 * np.max(np.abs(Ro)), err
    g.fe_jacobian(_dev(dU), host_blocks=True)
    A = P.jacobian(dU)
    x = np.random.default_rng(4).standard_normal(s.N)
    y = g.spmv(_dev(x)).cpu().numpy()
    bound = abs(A) @ np.abs(x)
    rel = np.max(np.abs(y - A @ x) / (bound + 1e-300))
    print(f"{name} theta={theta}: residual {err:.2e} of {np.max(np.abs(Ro)):.2e}, Jacobian product {rel:.2e}")
    assert rel <= 1e-12, rel
    g.close()


@pytest.mark.parametrize("name,theta", [("tiny2d", 0.5 + 1e-2), ("c1", 0.5)])
def test_theta_time_steps_match_oracle(name, theta):
    """Three steps of the shifted Crank-Nicolson (tiny2d) and Crank-Nicolson
    (c1) schemes: quasi-Newton on the GPU, exact Newton in the oracle, the
    fields after every step compared."""
    from paper_1801_05648_amd import FsiSolver
    s, cfg, f = _theta_case(name, theta)
    g = FsiSolver.from_system(s, device=0)
    g.fe_setup(cfg, f)
    g.build_precond("f64")
    fo = f
    n_nodes = f["vdof"].shape[0]
    for step in range(3):
        info = g.time_step(rtol=1e-11, precond="reuse")
        assert info.converged, info
        P = fe.FeProblem(cfg, fo, s.N)
        dUo, io = fe.quasi_newton(P.residual, P.jacobian, s.N, rtol=1e-13, ratio=0.0)
        assert io.converged
        fo = fe.advance(P, dUo)
        v, u, p = g.fe_fields(n_nodes, s.dim)
        dv = np.max(np.abs(v - fo["v"])) / np.max(np.abs(fo["v"]))
        du = np.max(np.abs(u - fo["u"])) / np.max(np.abs(fo["u"]))
        dp = np.max(np.abs(p - fo["p"])) / np.max(np.abs(fo["p"]))
        print(f"{name} theta={theta} step {step}: {info.steps} Newton steps ({info.reassemblies} assemblies), "
              f"oracle {io.steps}; fields v {dv:.1e} u {du:.1e} p {dp:.1e}")
        assert max(dv, du, dp) <= 1e-7, (dv, du, dp)
    g.close()
