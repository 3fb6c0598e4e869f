"""Pins of the oracle's finite-element residual, Jacobian and quasi-Newton loop.

The oracle (oracle/fe.py) evaluates the discrete ALE-FSI residual of Section
3 and forms its Jacobian by complex steps.  It is pinned to things other than
itself:

* the input generator's residual and assembled blocks -- a separate
  implementation (C++, forward-mode dual numbers, its own element loop) of
  the same equations;
* central finite differences of the oracle's own residual at a state away
  from the given fields (a derivative check that needs no second
  implementation);
* closed forms: a constant velocity field (mass terms only: each nodal
  residual is rho v0 times the integral of its basis function, known in
  closed form for the Q2 basis), and a constant pressure (only the pressure
  term: the integral of a basis function's derivative is a difference of
  its end values);
* the quasi-Newton rule of Section 6 on a scalar equation worked by hand,
  and quadratic convergence of the exact Newton iteration;
* the one-step-theta scheme (Section 3.2): theta = 1 is the pinned residual
  bit for bit and the residual is affine in theta; closed forms for the
  kinematics rows, the previous level's solid stress, the new and previous
  viscous shares adding to dt (outflow face included) and the fluid mass term
  with theta J + (1 - theta) J_old; central differences of the Jacobian.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import fsigen
from oracle import fe

_cache = {}


def _sys(name, **over):
    key = (name, tuple(sorted(over.items())))
    if key not in _cache:
        cfg = fsigen.config(name, **over)
        s = fsigen.generate(cfg, fe=True)
        _cache[key] = (s, fe.FeProblem(s.cfg, s.fe, s.N))
    return _cache[key]


def _ah(s):
    B = {k: sp.csr_matrix((b.val, b.col, b.rowptr), shape=(b.nrows, b.ncols)) for k, b in s.blocks.items()}
    return sp.bmat([[B["M"], B["C_ms"], None], [B["C_sm"], B["S"], B["C_sf"]],
                    [B["C_fm"], B["C_fs"], B["F"]]]).tocsr()


CASES = [("tiny2d", {}), ("tiny3d", {}), ("c1", {}), ("tiny3d", {"newton_mesh": 1}), ("tiny2d_unit", {})]


@pytest.mark.parametrize("name,over", CASES)
def test_residual_matches_the_generator(name, over):
    s, P = _sys(name, **over)
    R0 = P.residual()
    assert np.max(np.abs(R0 + s.b)) <= 1e-13 * np.max(np.abs(s.b))
    d = np.random.default_rng(7).standard_normal(s.N) * 1e-3
    Rg = fsigen.residual(s.cfg, 0, d, 1.0)
    Ro = P.residual(d)
    assert np.max(np.abs(Ro - Rg)) <= 1e-13 * np.max(np.abs(Rg))


@pytest.mark.parametrize("name,over", CASES)
def test_jacobian_matches_the_generator(name, over):
    s, P = _sys(name, **over)
    A = P.jacobian()
    G = _ah(s)
    scale = abs(G).max()
    assert abs(A - G).max() <= 1e-13 * scale
    # the generator stores nonzeros only; every one of them is an oracle entry
    Gc, Ac = G.tocoo(), A.tocsr()
    assert np.all(Ac[Gc.row, Gc.col].A1 != 0.0)


@pytest.mark.parametrize("name,over", [("tiny2d", {}), ("tiny3d", {"newton_mesh": 1}), ("c1", {})])
def test_jacobian_is_the_derivative_of_the_residual(name, over):
    s, P = _sys(name, **over)
    rng = np.random.default_rng(11)
    U = rng.standard_normal(s.N) * 1e-2  # a state off the given fields
    A = P.jacobian(U)
    for trial in range(2):
        d = rng.standard_normal(s.N)
        Ad = A @ d
        err = []
        for eps in (1e-5, 1e-6):
            fd = (P.residual(U + eps * d) - P.residual(U - eps * d)) / (2 * eps)
            err.append(np.linalg.norm(fd - Ad) / np.linalg.norm(Ad))
        # the difference is the central difference's own O(eps^2) error
        assert err[1] <= 1e-5 and 30.0 <= err[0] / err[1] <= 300.0, (trial, err)


def _basis_integrals():
    """Integrals over [0, 1] of the Q2 Lagrange basis (nodes 0, 1/2, 1) and end-value differences."""
    return np.array([1.0, 4.0, 1.0]) / 6.0, np.array([-1.0, 0.0, 1.0])


def _cells_of_node(s, I):
    D = s.dim
    ranges = []
    for a in range(D):
        if I[a] % 2:
            ranges.append([(I[a] - 1) // 2])
        else:
            ranges.append([c for c in (I[a] // 2 - 1, I[a] // 2) if 0 <= c < s.cfg.cells[a]])
    return list(itertools.product(*ranges))


def _solid(s, C):
    return all(s.cfg.solid_lo[a] <= C[a] < s.cfg.solid_hi[a] for a in range(s.dim))


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d"])
def test_constant_velocity_gives_the_mass_terms_in_closed_form(name):
    s, P0 = _sys(name)
    D = s.dim
    v0 = np.array([0.7, -0.3, 0.2][:D])
    f = {k: np.array(v, copy=True) for k, v in s.fe.items()}
    for k in ("u", "v_old", "u_old", "w", "u_fz"):
        f[k][:] = 0.0
    f["p"][:] = 0.0
    f["v"][:] = v0
    P = fe.FeProblem(s.cfg, f, s.N)
    R = P.residual()
    ints, _ = _basis_integrals()
    h = np.array(s.cfg.extent[:D]) / np.array(s.cfg.cells[:D])
    NN = 2 * np.array(s.cfg.cells[:D]) + 1
    checked = 0
    for n in range(int(np.prod(NN))):
        I = np.unravel_index(n, tuple(NN))
        mass_v = mass_u = 0.0
        for C in _cells_of_node(s, I):
            w = np.prod([h[a] * ints[I[a] - 2 * C[a]] for a in range(D)])
            mass_v += (s.cfg.rho_s if _solid(s, C) else s.cfg.rho_f) * w
            if _solid(s, C):
                mass_u += w
        if f["vdof"][n] >= 0:
            np.testing.assert_allclose(R[f["vdof"][n]:f["vdof"][n] + D], mass_v * v0, rtol=1e-13, atol=0)
            checked += 1
        if f["udof"][n] >= 0 and mass_u > 0:  # solid kinematics: -dt theta v
            np.testing.assert_allclose(R[f["udof"][n]:f["udof"][n] + D], -s.cfg.dt * mass_u * v0,
                                       rtol=1e-13, atol=0)
    pd = f["pdof"][f["pdof"] >= 0]  # tr(grad v) of a constant field: zero up to rounding
    assert np.max(np.abs(R[pd])) <= 1e-13 * np.max(np.abs(R)) and checked > 0


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d"])
def test_constant_pressure_gives_the_pressure_term_in_closed_form(name):
    s, _ = _sys(name)
    D = s.dim
    p0 = 3.5
    f = {k: np.array(v, copy=True) for k, v in s.fe.items()}
    for k in ("v", "u", "v_old", "u_old", "w", "u_fz"):
        f[k][:] = 0.0
    f["p"][:] = p0
    P = fe.FeProblem(s.cfg, f, s.N)
    R = P.residual()
    ints, ends = _basis_integrals()
    h = np.array(s.cfg.extent[:D]) / np.array(s.cfg.cells[:D])
    NN = 2 * np.array(s.cfg.cells[:D]) + 1
    for n in range(int(np.prod(NN))):
        if f["vdof"][n] < 0:
            continue
        I = np.unravel_index(n, tuple(NN))
        ref = np.zeros(D)
        for C in _cells_of_node(s, I):
            if _solid(s, C):
                continue
            loc = [I[a] - 2 * C[a] for a in range(D)]
            for c in range(D):  # -p0 * integral over the cell of d_c phi
                ref[c] -= p0 * ends[loc[c]] * np.prod([h[a] * ints[loc[a]] for a in range(D) if a != c])
        np.testing.assert_allclose(R[f["vdof"][n]:f["vdof"][n] + D], ref, rtol=1e-12, atol=1e-13 * p0)
    pd = f["pdof"][f["pdof"] >= 0]
    assert np.all(np.abs(R[pd]) == 0.0)


def test_quasi_newton_rule_on_a_scalar_equation():
    # r(x) = x^2 - 4 from x = 1 (dU is the offset from 1); worked by hand:
    # k=0 assemble J=2 -> x1 = 2.5, r1 = 2.25 > 0.3 -> assemble J=5 -> x2 = 2.05,
    # r2 = 0.2025 <= 0.225 -> keep J=5 -> x3 = 2.0095, r3 = 0.03809025 > 0.02025
    # -> assemble J=4.019 -> x4 = 2.0095 - 0.03809025/4.019
    res = lambda d: np.array([(1.0 + d[0]) ** 2 - 4.0])
    jac = lambda d: sp.csr_matrix([[2.0 * (1.0 + d[0])]])
    solve = lambda A, b: np.array([b[0] / A[0, 0]])
    dU, info = fe.quasi_newton(res, jac, 1, rtol=1e-9, linear_solve=solve)
    assert info.reassembled[:4] == [True, True, False, True]
    np.testing.assert_allclose(info.residuals[:4], [3.0, 2.25, 0.2025, 0.03809025], rtol=1e-13)
    x4 = 2.0095 - 0.03809025 / 4.019
    assert info.converged and abs(1.0 + dU[0] - 2.0) <= 3e-9 / 4.0  # |r| < 3e-9, r'(2) = 4
    # the fourth iterate of the loop, recomputed by hand
    _, info4 = fe.quasi_newton(res, jac, 1, rtol=1e-9, linear_solve=solve, max_steps=4)
    assert abs(info4.residuals[4] - abs(x4 * x4 - 4.0)) <= 1e-9 * abs(x4 * x4 - 4.0)
    assert info.reassemblies == sum(info.reassembled)


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d_unit"])
def test_exact_newton_converges_quadratically(name):
    s, P = _sys(name)
    dU, info = fe.quasi_newton(P.residual, P.jacobian, s.N, rtol=1e-12, ratio=0.0)
    r = info.residuals
    assert info.converged and all(info.reassembled)
    # in the asymptotic range (r_k < 1e-3 r_0) the scaled ratio (r_{k+1}/r_0) / (r_k/r_0)^2
    # stays bounded (it grows without bound under linear convergence)
    tail = [(r[k] / r[0], r[k + 1] / r[0]) for k in range(1, len(r) - 1)
            if r[k] < 1e-3 * r[0] and r[k + 1] > 1e-14 * r[0]]
    assert tail, r
    for a, b in tail:
        assert b <= 50.0 * a * a, r
    R = P.residual(dU)
    assert np.max(np.abs(R)) < 1e-12 * r[0]


# ---------------------------------------------------------------- theta scheme
def _fields(s, **vals):
    f = {k: np.array(v, copy=True) for k, v in s.fe.items()}
    for k in ("v", "u", "v_old", "u_old", "w", "u_fz"):
        f[k][:] = 0.0
    f["p"][:] = 0.0
    for k, v in vals.items():
        f[k] = v
    return f


def _coords(s):
    D = s.dim
    h = np.array(s.cfg.extent[:D]) / np.array(s.cfg.cells[:D])
    NN = 2 * np.array(s.cfg.cells[:D]) + 1
    I = np.stack(np.unravel_index(np.arange(int(np.prod(NN))), tuple(NN)), -1)
    return 0.5 * h * I, h, NN


@pytest.mark.parametrize("name,theta", [("tiny2d", 0.5), ("tiny3d", 0.5 + 1e-2)])
def test_theta_scheme_is_affine_in_theta_and_reduces_at_one(name, theta):
    s, P1 = _sys(name)
    U = np.random.default_rng(12).standard_normal(s.N) * 1e-3
    R = {t: fe.FeProblem(s.cfg.with_(theta=t), s.fe, s.N).residual(U) for t in (0.5, 0.75, 1.0)}
    assert np.array_equal(R[1.0], P1.residual(U))
    np.testing.assert_allclose(R[0.75], 0.5 * (R[0.5] + R[1.0]), rtol=0, atol=1e-12 * np.max(np.abs(R[1.0])))


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d"])
def test_theta_scheme_kinematics_in_closed_form(name):
    # constant fields: the solid kinematics rows are
    # int phi [(u - u_old) - dt (theta v + (1 - theta) v_old)]
    s, _ = _sys(name)
    D, theta = s.dim, 0.5
    v0, v1 = np.array([0.3, -0.2, 0.1][:D]), np.array([-0.4, 0.5, 0.2][:D])
    u0, u1 = np.array([1e-3, 2e-3, -1e-3][:D]), np.array([-2e-3, 1e-3, 3e-3][:D])
    f = _fields(s)
    f["v"][:], f["v_old"][:], f["u"][:], f["u_old"][:] = v0, v1, u0, u1
    R = fe.FeProblem(s.cfg.with_(theta=theta), f, s.N).residual()
    ints, _ = _basis_integrals()
    _, h, NN = _coords(s)
    dt = s.cfg.dt
    checked = 0
    for n in range(int(np.prod(NN))):
        I = np.unravel_index(n, tuple(NN))
        mass_u = 0.0
        for C in _cells_of_node(s, I):
            if _solid(s, C):
                mass_u += np.prod([h[a] * ints[I[a] - 2 * C[a]] for a in range(D)])
        if f["udof"][n] >= 0 and mass_u > 0:
            ref = mass_u * ((u0 - u1) - dt * (theta * v0 + (1 - theta) * v1))
            np.testing.assert_allclose(R[f["udof"][n]:f["udof"][n] + D], ref, rtol=1e-12, atol=1e-18)
            checked += 1
    assert checked > 0


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d"])
def test_theta_scheme_previous_solid_stress_in_closed_form(name):
    # the previous level strained uniformly (u_old = A x), everything else zero:
    # only (1 - theta) dt (F_old S_old, grad phi) remains on the velocity rows
    s, _ = _sys(name)
    D, theta = s.dim, 0.5
    X, h, NN = _coords(s)
    A = np.array([[0.02, -0.01, 0.005], [0.01, -0.015, 0.0], [0.0, 0.004, 0.01]])[:D, :D]
    f = _fields(s, u_old=X @ A.T)
    R = fe.FeProblem(s.cfg.with_(theta=theta), f, s.N).residual()
    F = np.eye(D) + A
    E = 0.5 * (F.T @ F - np.eye(D))
    Pk = F @ (2 * s.cfg.mu_s * E + s.cfg.lambda_s * np.trace(E) * np.eye(D))
    ints, ends = _basis_integrals()
    dto = (1 - theta) * s.cfg.dt
    checked = 0
    for n in range(int(np.prod(NN))):
        if f["vdof"][n] < 0:
            continue
        I = np.unravel_index(n, tuple(NN))
        ref = np.zeros(D)
        for C in _cells_of_node(s, I):
            if not _solid(s, C):
                continue
            loc = [I[a] - 2 * C[a] for a in range(D)]
            for c in range(D):
                for k in range(D):
                    ref[c] += dto * Pk[c, k] * ends[loc[k]] * np.prod([h[a] * ints[loc[a]] for a in range(D) if a != k])
        np.testing.assert_allclose(R[f["vdof"][n]:f["vdof"][n] + D], ref, rtol=1e-10, atol=1e-12 * np.max(np.abs(Pk)))
        checked += int(np.any(ref != 0))
    assert checked > 0


@pytest.mark.parametrize("name,theta", [("tiny2d", 0.5), ("tiny2d", 0.6), ("tiny3d", 0.5)])
def test_theta_scheme_viscous_shares_add_to_dt(name, theta):
    # v = v_old = B x with B nilpotent (no convection, no divergence): the new
    # and previous viscous stresses and outflow corrections together carry dt
    s, _ = _sys(name)
    D = s.dim
    X, h, NN = _coords(s)
    B = np.zeros((D, D))
    B[0, 1] = 0.7  # B @ B = 0, tr B = 0
    f = _fields(s, v=X @ B.T, v_old=X @ B.T)
    R = fe.FeProblem(s.cfg.with_(theta=theta), f, s.N).residual()
    mu_dt = s.cfg.dt * s.cfg.rho_f * s.cfg.nu_f
    sig = mu_dt * (B + B.T)
    ints, ends = _basis_integrals()
    nc = s.cfg.cells
    for n in range(int(np.prod(NN))):
        if f["vdof"][n] < 0:
            continue
        I = np.unravel_index(n, tuple(NN))
        ref = np.zeros(D)
        for C in _cells_of_node(s, I):
            if _solid(s, C):
                continue
            loc = [I[a] - 2 * C[a] for a in range(D)]
            for c in range(D):
                for k in range(D):
                    ref[c] += sig[c, k] * ends[loc[k]] * np.prod([h[a] * ints[loc[a]] for a in range(D) if a != k])
            if C[0] == nc[0] - 1 and loc[0] == 2:  # outflow face x = L: -dt rho nu grad v^T e_0
                face = np.prod([h[a] * ints[loc[a]] for a in range(1, D)])
                ref -= mu_dt * B[0, :] * face
        np.testing.assert_allclose(R[f["vdof"][n]:f["vdof"][n] + D], ref, rtol=1e-10, atol=1e-12 * mu_dt)


def test_theta_scheme_fluid_mass_uses_the_weighted_jacobian():
    # constant velocities, uniformly stretched new and previous displacements:
    # fluid velocity rows are rho (theta J + (1 - theta) J_old)(v - v_old) int phi
    s, _ = _sys("tiny2d")
    D, theta = s.dim, 0.7  # not 0.5, where swapping J and J_old would go unseen
    X, h, NN = _coords(s)
    al, be = 0.01, -0.02
    v0, v1 = np.array([0.3, -0.2]), np.array([-0.1, 0.4])
    f = _fields(s, u=al * X, u_old=be * X)
    f["v"][:], f["v_old"][:] = v0, v1
    R = fe.FeProblem(s.cfg.with_(theta=theta), f, s.N).residual()
    Jth = theta * (1 + al) ** D + (1 - theta) * (1 + be) ** D
    ints, _ = _basis_integrals()
    checked = 0
    for n in range(int(np.prod(NN))):
        if f["vdof"][n] < 0:
            continue
        I = np.unravel_index(n, tuple(NN))
        cells = _cells_of_node(s, I)
        if any(_solid(s, C) for C in cells):
            continue
        mass = sum(np.prod([h[a] * ints[I[a] - 2 * C[a]] for a in range(D)]) for C in cells)
        np.testing.assert_allclose(R[f["vdof"][n]:f["vdof"][n] + D], s.cfg.rho_f * Jth * mass * (v0 - v1),
                                   rtol=1e-12)
        checked += 1
    assert checked > 0


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d"])
def test_theta_scheme_jacobian_is_the_derivative(name):
    s, _ = _sys(name)
    rng = np.random.default_rng(13)
    f = {k: np.array(v, copy=True) for k, v in s.fe.items()}
    f["v_old"] = f["v_old"] * 1.1 + 0.01 * rng.standard_normal(f["v_old"].shape)
    f["u_old"] = f["u_old"] * 0.8
    P = fe.FeProblem(s.cfg.with_(theta=0.5 + s.cfg.dt), f, s.N)
    U = rng.standard_normal(s.N) * 1e-2
    A = P.jacobian(U)
    d = rng.standard_normal(s.N)
    Ad = A @ d
    err = []
    for eps in (1e-5, 1e-6):
        fd = (P.residual(U + eps * d) - P.residual(U - eps * d)) / (2 * eps)
        err.append(np.linalg.norm(fd - Ad) / np.linalg.norm(Ad))
    assert err[1] <= 1e-5 and 30.0 <= err[0] / err[1] <= 300.0, err
