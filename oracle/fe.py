"""Residual and Jacobian of the discrete ALE-FSI equations (oracle; test infrastructure only).

What is computed.  The nonlinear residual of the monolithic ALE-FSI problem
of Section 3: the semi-linear form A(U)(Phi) minus the linear form F(Phi),
i.e. the sum of the variational equations (equation fsi:all), for one time
step of the one-step-theta scheme (Section 3.2), and its Jacobian A'(U) --
the matrix of the Newton step (Algorithm newton, Section 3.3).  The terms
below are those of theta = 1; for theta < 1 the convection, viscous stress,
outflow correction and solid stress carry dt theta at the new level and
dt (1 - theta) at the previous one (its velocity advecting itself), the fluid
mass term J^theta = theta J + (1 - theta) J_old, the kinematics
dt (theta v + (1 - theta) v_old); pressure, mesh velocity, incompressibility
and mesh motion stay implicit (the paper treats the pressure implicitly for
every theta).  Unknowns and test functions (Section 3.1):

* fluid cells -- momentum in ALE form
    ( rho J (v - v_old), phi ) + dt theta ( rho J (grad v F^{-1}) w, phi )
      - ( rho J (grad v F^{-1}) (u - u_old), phi )
      + ( dt theta rho nu J (grad v F^{-1} + F^{-T} grad v^T) F^{-T} - J p F^{-T}, grad phi )
      - dt theta < rho nu J F^{-T} grad v^T F^{-T} n, phi >  on the outflow face x = L,
  incompressibility ( J tr(grad v F^{-1}), psi ), and the harmonic mesh
  motion ( (1/J_m) grad u, grad phi^u ) with Jacobian-scaled stiffness;
* solid cells -- St. Venant-Kirchhoff elastodynamics
    ( rho_s (v - v_old), phi ) + dt theta ( F S, grad phi ),
    S = 2 mu E + lambda tr(E) I,  E = (F^T F - I) / 2,
  and the kinematics ( (u - u_old) - dt theta v, phi^u );

with F = I + grad u and J = det F.  Discretisation (Section 3.5): Q2
velocity and displacement, Q1 pressure on the structured channel, every
integral by the tensor 3-point Gauss rule (the outflow face by the same rule
on the face).

Readings of the paper (it is silent on these points; the workload fixes them):
* the advecting velocity w of the convective term is a given field (an
  Oseen-type linearisation of the ALE convection), as are v_old and u_old;
* J_m in the mesh equation is det(I + grad u_fz) of a given displacement
  u_fz, or, with ``newton_mesh``, the current J (then differentiated);
* the displacement test functions of the mesh equation vanish on the
  interface (Section 3.1), those of the solid kinematics do not; velocity
  test functions vanish on Dirichlet nodes; a constrained dof holds the
  state's value (the given field).

The Jacobian is formed cell by cell by complex-step differentiation of the
cell residual, d R / d U_s = Im R(U + i h e_s) / h with h = 1e-30, which is
exact to rounding for these analytic integrands and shares nothing with the
dual-number evaluation of the library; the cell matrices are summed into a
scipy CSR matrix over the free dofs.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

GAUSS_X = 0.5 + np.array([-np.sqrt(0.15), 0.0, np.sqrt(0.15)])  # 3-point Gauss on [0, 1]
GAUSS_W = np.array([5.0, 8.0, 5.0]) / 18.0
CS_STEP = 1e-30


def _lagrange(nodes, x):
    """Values and derivatives of the 1D Lagrange basis on `nodes` at points x."""
    n = len(nodes)
    val = np.ones((len(x), n))
    der = np.zeros((len(x), n))
    for i in range(n):
        for j in range(n):
            if j == i:
                continue
            f = (x - nodes[j]) / (nodes[i] - nodes[j])
            # product rule: d/dx of prod_j f_j
            der[:, i] = der[:, i] * f + val[:, i] / (nodes[i] - nodes[j])
            val[:, i] = val[:, i] * f
    return val, der


def _det(F):
    d = F.shape[-1]
    if d == 2:
        return F[..., 0, 0] * F[..., 1, 1] - F[..., 0, 1] * F[..., 1, 0]
    return (F[..., 0, 0] * (F[..., 1, 1] * F[..., 2, 2] - F[..., 1, 2] * F[..., 2, 1])
            - F[..., 0, 1] * (F[..., 1, 0] * F[..., 2, 2] - F[..., 1, 2] * F[..., 2, 0])
            + F[..., 0, 2] * (F[..., 1, 0] * F[..., 2, 1] - F[..., 1, 1] * F[..., 2, 0]))


def _inv(F, J):
    """Inverse by cofactors (analytic, so complex steps pass through)."""
    d = F.shape[-1]
    G = np.empty_like(F)
    if d == 2:
        G[..., 0, 0] = F[..., 1, 1]
        G[..., 0, 1] = -F[..., 0, 1]
        G[..., 1, 0] = -F[..., 1, 0]
        G[..., 1, 1] = F[..., 0, 0]
    else:
        for i in range(3):
            for j in range(3):
                r = [a for a in range(3) if a != j]
                c = [b for b in range(3) if b != i]
                m = F[..., r[0], c[0]] * F[..., r[1], c[1]] - F[..., r[0], c[1]] * F[..., r[1], c[0]]
                G[..., i, j] = m if (i + j) % 2 == 0 else -m
    return G / J[..., None, None]


def _mm(A, B):
    return np.einsum("...ij,...jk->...ik", A, B)


def _T(A):
    return np.swapaxes(A, -1, -2)


@dataclasses.dataclass
class Material:
    rho_f: float
    nu_f: float
    rho_s: float
    mu_s: float
    lambda_s: float
    dt_theta: float
    newton_mesh: bool
    theta: float = 1.0
    dt: float = 0.0


class FeProblem:
    """The discrete residual R(U) and Jacobian A'(U) of one workload.

    cfg: the workload's grid and material data (dim, cells, extent, solid box
    [solid_lo, solid_hi) in cells, rho_f, nu_f, rho_s, mu_s, lambda_s, dt,
    theta, newton_mesh); fe: its node arrays (vdof, udof, pdof, v, u, p,
    v_old, u_old, w, u_fz) on the Q2 lattice, nodes numbered row-major with
    axis 0 slowest; N: the number of free dofs.  A state is the given fields
    plus an offset dU on the free dofs.
    """

    def __init__(self, cfg, fe: dict, N: int):
        if not (0.0 < cfg.theta <= 1.0):
            raise ValueError("theta must lie in (0, 1]")
        D = self.D = int(cfg.dim)
        nc = np.array(cfg.cells[:D])
        h = np.array(cfg.extent[:D], float) / nc
        NN = 2 * nc + 1
        self.N, self.h, self.nc = int(N), h, nc
        self.mat = Material(cfg.rho_f, cfg.nu_f, cfg.rho_s, cfg.mu_s, cfg.lambda_s, cfg.dt * cfg.theta,
                            bool(cfg.newton_mesh), float(cfg.theta), float(cfg.dt))
        self.fe = fe
        # cells, row-major over (C_0, ..., C_{D-1})
        C = np.stack(np.meshgrid(*[np.arange(n) for n in nc], indexing="ij"), -1).reshape(-1, D)
        lo, hi = np.array(cfg.solid_lo[:D]), np.array(cfg.solid_hi[:D])
        self.solid = np.all((C >= lo) & (C < hi), axis=1)
        self.outflow = (~self.solid) & (C[:, 0] == nc[0] - 1)
        nq2, nq1 = 3 ** D, 2 ** D
        self.nq2, self.nq1 = nq2, nq1
        off2 = np.array([[(l // 3 ** a) % 3 for a in range(D)] for l in range(nq2)])
        off1 = np.array([[2 * ((l // 2 ** a) % 2) for a in range(D)] for l in range(nq1)])
        self.nodes = np.ravel_multi_index(tuple(np.moveaxis(2 * C[:, None, :] + off2[None], -1, 0)), tuple(NN))
        self.verts = np.ravel_multi_index(tuple(np.moveaxis(2 * C[:, None, :] + off1[None], -1, 0)), tuple(NN))
        # quadrature: volume points, then the outflow face x_0 = 1 (reference)
        qi = np.array([[(q // 3 ** a) % 3 for a in range(D)] for q in range(3 ** D)])
        xq = GAUSS_X[qi]
        wq = np.prod(GAUSS_W[qi], axis=1) * np.prod(h)
        fi = np.array([[(q // 3 ** (a - 1)) % 3 for a in range(1, D)] for q in range(3 ** (D - 1))])
        xf = np.concatenate([np.ones((len(fi), 1)), GAUSS_X[fi]], axis=1)
        wf = np.prod(GAUSS_W[fi], axis=1) * np.prod(h[1:])
        self.vol = self._shapes(xq, off2, off1, wq)
        self.face = self._shapes(xf, off2, off1, wf)
        # local dofs: v (node-major, component), u (same), p (vertices)
        NV = nq2 * D
        self.NV, self.nloc = NV, 2 * NV + nq1
        vd, ud, pd = fe["vdof"][self.nodes], fe["udof"][self.nodes], fe["pdof"][self.verts]
        comp = np.arange(D)
        gv = np.where(vd[..., None] >= 0, vd[..., None] + comp, -1).reshape(len(C), NV)
        gu = np.where(ud[..., None] >= 0, ud[..., None] + comp, -1).reshape(len(C), NV)
        gp = np.where(self.solid[:, None], -1, pd)
        self.gd = np.concatenate([gv, gu, gp], axis=1)
        # test functions: v where free; u where free and (solid cell, or a node
        # of no solid cell: the mesh equation is not tested on the interface); p where free
        node_in_solid = np.zeros(len(fe["vdof"]), bool)
        node_in_solid[self.nodes[self.solid].ravel()] = True
        ut = (ud[..., None] >= 0) & (self.solid[:, None, None] | ~node_in_solid[self.nodes][..., None])
        ut = np.broadcast_to(ut, (len(C), nq2, D)).reshape(len(C), NV)
        self.test = np.concatenate([gv >= 0, ut, gp >= 0], axis=1)
        self.ncells = len(C)

    def _shapes(self, x, off2, off1, w):
        D, h = self.D, self.h
        v2, d2, v1 = [], [], []
        for a in range(D):
            val, der = _lagrange(np.array([0.0, 0.5, 1.0]), x[:, a])
            v2.append(val)
            d2.append(der / h[a])
            v1.append(_lagrange(np.array([0.0, 1.0]), x[:, a])[0])
        nq = x.shape[0]
        N = np.ones((nq, len(off2)))
        dN = np.ones((nq, len(off2), D))
        M = np.ones((nq, len(off1)))
        for a in range(D):
            N *= v2[a][:, off2[:, a]]
            M *= v1[a][:, off1[:, a] // 2]
            for k in range(D):
                dN[:, :, k] *= (d2[a] if a == k else v2[a])[:, off2[:, a]]
        return dict(N=N, dN=dN, M=M, w=w)

    # ------------------------------------------------------------- states
    def local_state(self, dU):
        """Cell arrays (v, u: (cells, 3^D, D); p: (cells, 2^D)) of the state fields + dU."""
        fe, D = self.fe, self.D
        dU = np.zeros(self.N) if dU is None else np.asarray(dU)
        ext = np.concatenate([dU, np.zeros(1, dU.dtype)])  # index -1 -> 0
        nv = self.nodes.shape[1] * D
        v = fe["v"][self.nodes] + ext[self.gd[:, :nv]].reshape(-1, self.nq2, D)
        u = fe["u"][self.nodes] + ext[self.gd[:, nv:2 * nv]].reshape(-1, self.nq2, D)
        p = fe["p"][self.verts] + ext[self.gd[:, 2 * nv:]]
        return v, u, p

    # ------------------------------------------------------------ cell forms
    def cell_residual(self, v, u, p, sel=slice(None)):
        """Local residual of every cell (or of cells[sel]), (cells, nloc), all
        local test functions."""
        m, D = self.mat, self.D
        fe = self.fe
        nodes, solid, outflow = self.nodes[sel], self.solid[sel], self.outflow[sel]
        S = self.vol
        N, dN, M, w = S["N"], S["dN"], S["M"], S["w"]
        I = np.eye(D)
        vq = np.einsum("ql,cld->cqd", N, v)
        uq = np.einsum("ql,cld->cqd", N, u)
        Gv = np.einsum("qlk,cld->cqdk", dN, v)
        Gu = np.einsum("qlk,cld->cqdk", dN, u)
        pq = np.einsum("ql,cl->cq", M, p)
        wq = np.einsum("ql,cld->cqd", N, fe["w"][nodes])
        vo = np.einsum("ql,cld->cqd", N, fe["v_old"][nodes])
        uo = np.einsum("ql,cld->cqd", N, fe["u_old"][nodes])
        Gz = np.einsum("qlk,cld->cqdk", dN, fe["u_fz"][nodes])
        F = I + Gu
        J = _det(F)
        Fi = _inv(F, J)
        FiT = _T(Fi)
        # fluid
        GF = _mm(Gv, Fi)  # grad v F^{-1}
        fV_f = (m.rho_f * J[..., None] * (vq - vo)
                + m.dt_theta * m.rho_f * J[..., None] * np.einsum("cqdk,cqk->cqd", GF, wq)
                - m.rho_f * J[..., None] * np.einsum("cqdk,cqk->cqd", GF, uq - uo))
        sig = m.dt_theta * m.rho_f * m.nu_f * (GF + _T(GF))
        gV_f = J[..., None, None] * (_mm(sig, FiT) - pq[..., None, None] * FiT)
        fP_f = J * np.trace(GF, axis1=-2, axis2=-1)
        Jm = J if m.newton_mesh else _det(I + Gz)
        gU_f = Gu / Jm[..., None, None]
        # solid
        E = 0.5 * (_mm(_T(F), F) - I)
        Ss = 2.0 * m.mu_s * E + m.lambda_s * np.trace(E, axis1=-2, axis2=-1)[..., None, None] * I
        gV_s = m.dt_theta * _mm(F, Ss)
        fV_s = m.rho_s * (vq - vo)
        fU_s = (uq - uo) - m.dt_theta * vq
        if m.theta < 1.0:
            # the one-step-theta scheme (Section 3.2): the explicit share (1 - theta) dt of the
            # convection, viscous stress and solid stress at the previous level (the previous
            # velocity advecting itself), J^theta = theta J + (1 - theta) J_old in the fluid mass
            # term, and (1 - theta) dt v_old in the kinematics; pressure, mesh velocity,
            # incompressibility and mesh motion stay implicit
            dto = (1.0 - m.theta) * m.dt
            Gvo = np.einsum("qlk,cld->cqdk", dN, fe["v_old"][nodes])
            Guo = np.einsum("qlk,cld->cqdk", dN, fe["u_old"][nodes])
            Fo = I + Guo
            Jo = _det(Fo)
            Fio = _inv(Fo, Jo)
            GFo = _mm(Gvo, Fio)
            Jth = m.theta * J + (1.0 - m.theta) * Jo
            fV_f = (m.rho_f * Jth[..., None] * (vq - vo)
                    + m.dt_theta * m.rho_f * J[..., None] * np.einsum("cqdk,cqk->cqd", GF, wq)
                    - m.rho_f * J[..., None] * np.einsum("cqdk,cqk->cqd", GF, uq - uo)
                    + dto * m.rho_f * Jo[..., None] * np.einsum("cqdk,cqk->cqd", GFo, vo))
            sigo = dto * m.rho_f * m.nu_f * (GFo + _T(GFo))
            gV_f = gV_f + Jo[..., None, None] * _mm(sigo, _T(Fio))
            Eo = 0.5 * (_mm(_T(Fo), Fo) - I)
            So = 2.0 * m.mu_s * Eo + m.lambda_s * np.trace(Eo, axis1=-2, axis2=-1)[..., None, None] * I
            gV_s = gV_s + dto * _mm(Fo, So)
            fU_s = fU_s - dto * vo
        sol = solid[:, None]
        fV = np.where(sol[..., None], fV_s, fV_f)
        gV = np.where(sol[..., None, None], gV_s, gV_f)
        fU = np.where(sol[..., None], fU_s, 0.0)
        gU = np.where(sol[..., None, None], 0.0, gU_f)
        fP = np.where(sol, 0.0, fP_f)
        Rv = np.einsum("q,cqd,ql->cld", w, fV, N) + np.einsum("q,cqdk,qlk->cld", w, gV, dN)
        Ru = np.einsum("q,cqd,ql->cld", w, fU, N) + np.einsum("q,cqdk,qlk->cld", w, gU, dN)
        Rp = np.einsum("q,cq,ql->cl", w, fP, M)
        # outflow face (normal e_0) of the fluid cells at x = L
        out = np.nonzero(outflow)[0]
        if len(out):
            Sf = self.face
            Nf, dNf, wf = Sf["N"], Sf["dN"], Sf["w"]
            Gvf = np.einsum("qlk,cld->cqdk", dNf, v[out])
            Ff = I + np.einsum("qlk,cld->cqdk", dNf, u[out])
            Jf = _det(Ff)
            Fif = _inv(Ff, Jf)
            n = np.zeros(D)
            n[0] = 1.0
            a = np.einsum("cqkm,m->cqk", _T(Fif), n)        # F^{-T} n
            b = np.einsum("cqmk,cqm->cqk", Gvf, a)          # grad v^T F^{-T} n
            t = np.einsum("cqdk,cqk->cqd", _T(Fif), b)      # F^{-T} grad v^T F^{-T} n
            fO = -m.dt_theta * m.rho_f * m.nu_f * Jf[..., None] * t
            if m.theta < 1.0:  # the previous level's share of the outflow correction
                no = nodes[out]
                Gvfo = np.einsum("qlk,cld->cqdk", dNf, fe["v_old"][no])
                Ffo = I + np.einsum("qlk,cld->cqdk", dNf, fe["u_old"][no])
                Jfo = _det(Ffo)
                Fifo = _inv(Ffo, Jfo)
                ao = np.einsum("cqkm,m->cqk", _T(Fifo), n)
                bo = np.einsum("cqmk,cqm->cqk", Gvfo, ao)
                to = np.einsum("cqdk,cqk->cqd", _T(Fifo), bo)
                fO = fO - (1.0 - m.theta) * m.dt * m.rho_f * m.nu_f * Jfo[..., None] * to
            Rv[out] = Rv[out] + np.einsum("q,cqd,ql->cld", wf, fO, Nf)
        nc = v.shape[0]
        return np.concatenate([Rv.reshape(nc, -1), Ru.reshape(nc, -1), Rp], axis=1)

    # --------------------------------------------------------------- global
    def residual(self, dU=None) -> np.ndarray:
        """R(U) on the free dofs (tested equations summed over cells)."""
        Rl = self.cell_residual(*self.local_state(dU))
        R = np.zeros(self.N)
        np.add.at(R, self.gd[self.test], Rl[self.test])
        return R

    def cell_jacobians(self, dU=None, cells=None) -> np.ndarray:
        """d R_cell / d U_cell of every cell (or of the listed cells), (cells,
        nloc, nloc), by complex steps."""
        sel = slice(None) if cells is None else np.asarray(cells)
        v, u, p = (a[sel] for a in self.local_state(dU))
        NV, D = self.NV, self.D
        K = np.zeros((v.shape[0], self.nloc, self.nloc))
        for s in range(self.nloc):
            vc, uc, pc = v.astype(complex), u.astype(complex), p.astype(complex)
            if s < NV:
                vc[:, s // D, s % D] += 1j * CS_STEP
            elif s < 2 * NV:
                uc[:, (s - NV) // D, (s - NV) % D] += 1j * CS_STEP
            else:
                pc[:, s - 2 * NV] += 1j * CS_STEP
            K[:, :, s] = self.cell_residual(vc, uc, pc, sel).imag / CS_STEP
        return K

    def jacobian(self, dU=None, cells=None) -> sp.csr_matrix:
        """A'(U) over the free dofs, rows = tested equations, columns = free
        dofs; with `cells` only their contributions (complete in the rows
        that rows_covered(cells) lists)."""
        K = self.cell_jacobians(dU, cells)
        sel = slice(None) if cells is None else np.asarray(cells)
        gd, test = self.gd[sel], self.test[sel]
        rows = np.broadcast_to(gd[:, :, None], K.shape)
        cols = np.broadcast_to(gd[:, None, :], K.shape)
        keep = test[:, :, None] & (gd[:, None, :] >= 0)
        A = sp.coo_matrix((K[keep], (rows[keep], cols[keep])), shape=(self.N, self.N)).tocsr()
        A.sum_duplicates()
        return A


def rows_covered(prob: FeProblem, cells) -> np.ndarray:
    """Rows (tested equations) all of whose cell contributions come from `cells`."""
    total = np.zeros(prob.N, np.int64)
    np.add.at(total, prob.gd[prob.test], 1)
    part = np.zeros(prob.N, np.int64)
    sel = np.asarray(cells)
    np.add.at(part, prob.gd[sel][prob.test[sel]], 1)
    return np.nonzero((total > 0) & (part == total))[0]


def advance(prob: FeProblem, dU) -> dict:
    """The node fields of the next time step after a converged step: the state
    becomes the previous level and the linearisation fields (v_old, u_old, w,
    u_fz and the state v, u, p all take the new values; constrained dofs keep
    theirs)."""
    fe, D = prob.fe, prob.D
    new = {k: np.array(fe[k], copy=True) for k in fe}
    for key, dof in (("v", "vdof"), ("u", "udof")):
        idx = fe[dof] >= 0
        new[key][idx] = fe[key][idx] + np.asarray(dU)[fe[dof][idx][:, None] + np.arange(D)]
    idx = fe["pdof"] >= 0
    new["p"][idx] = fe["p"][idx] + np.asarray(dU)[fe["pdof"][idx]]
    new["v_old"], new["u_old"] = new["v"].copy(), new["u"].copy()
    new["w"], new["u_fz"] = new["v"].copy(), new["u"].copy()
    return new


def max_norm(r) -> float:
    return float(np.max(np.abs(r))) if len(r) else 0.0


@dataclasses.dataclass
class NewtonInfo:
    converged: bool = False
    steps: int = 0
    reassemblies: int = 0
    residuals: list = dataclasses.field(default_factory=list)   # ||r_k||_inf, k = 0, 1, ...
    reassembled: list = dataclasses.field(default_factory=list)  # per step: Jacobian assembled at U_k


def reassemble_now(k: int, residuals, ratio: float) -> bool:
    """Section 6's quasi-Newton rule: assemble at k = 0, and afterwards only
    when the last step reduced the max-norm residual by less than 1/ratio,
    i.e. ||r_k|| > ratio ||r_{k-1}||."""
    return k == 0 or residuals[k] > ratio * residuals[k - 1]


def quasi_newton(residual, jacobian, N: int, rtol: float = 1e-6, ratio: float = 0.1, max_steps: int = 25,
                 linear_solve=None, dU0=None):
    """Algorithm newton (Section 3.3) with Section 6's quasi-Newton rule and
    stopping test ||r_k||_inf < rtol ||r_0||_inf; r_0 is the initial residual.

    residual(dU) -> R, jacobian(dU) -> sparse A'; linear_solve(A, rhs) -> x
    (default: a sparse direct solve, i.e. the exact Newton step).
    Returns (dU, NewtonInfo).
    """
    solve = linear_solve or (lambda A, b: spla.spsolve(A.tocsc(), b))
    dU = np.zeros(N) if dU0 is None else np.array(dU0, float)
    info = NewtonInfo()
    r = residual(dU)
    info.residuals.append(max_norm(r))
    A = None
    for k in range(max_steps + 1):
        rk = info.residuals[k]
        if rk == 0.0 or rk < rtol * info.residuals[0]:
            info.converged = True
            break
        if k == max_steps:
            break
        if reassemble_now(k, info.residuals, ratio):
            A = jacobian(dU)
            info.reassemblies += 1
            info.reassembled.append(True)
        else:
            info.reassembled.append(False)
        dU = dU + solve(A, -r)
        r = residual(dU)
        info.residuals.append(max_norm(r))
        info.steps += 1
    return dU, info
