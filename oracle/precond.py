"""Approximate block-LDU preconditioner (oracle; test infrastructure only).

Algorithm "Evaluation of P^{-1} r" of the paper's Section 4.1, obtained from
the block LDU factorisation of A_h after dropping C_sm and approximating the
fluid Schur complement X by F:

  1. x_m = M^{-1} r_m
  2. x_s = S^{-1} r_s
  3. x_f = F^{-1} (r_f - C_fm x_m - C_fs x_s)
  4. x_s = x_s - S^{-1} C_sf x_f
  5. x_m = x_m - M^{-1} C_ms x_s

with the approximate inverses

* M^{-1}: one AMG V-cycle on the scalar Laplacian L (M = L (x) I_d), applied
  to each displacement component (Section 4.2);
* S^{-1}: the solid Schur-complement algorithm of Section 4.3 with AMG on
  Sigma_s = S_vv + dt theta S_vu and on the mass block S_uu:
      y = V_Ms(r_u);  x_v = V_Sigma(r_v - S_vu y);  x_u = V_Ms(r_u - S_uv x_v);
* F^{-1}: the same Schur-complement (Uzawa-like) elimination on
  F = [[A_f, G], [D, 0]] with the pressure Schur approximation
  S_p = -D diag(A_f)^{-1} G (Section 4.4, reading in the design notes):
      y = V_A(r_v);  x_p = V_p(r_p - D y);  x_v = V_A(r_v - G x_p).
  Optionally (the paper's choice for the fluid sub-problem, Section 4.4) F^{-1}
  is k steps of flexible GMRES on F from zero, right-preconditioned by that
  Uzawa-like step or by the cheaper block upper-triangular step
      x_p = V_p(r_p);  x_v = V_A(r_v - G x_p)
  (fluid_gmres_solve, fluid_triangular_solve).  Or, as Section 4.4 reads,
  the Uzawa-like step itself with each occurring inverse approximated by k
  GMRES steps preconditioned by its V-cycle (fluid_schur_gmres_solve).
"""
from __future__ import annotations

import numpy as np

from . import amg, krylov
from .blocks import BlockSystem

# Inner GMRES of the fluid step: it stops before k steps only when its
# residual estimate falls to this fraction of ||r_f|| (an exact solve).
INNER_TOL = 1e-14

H_NAMES = ("H_M", "H_SIG", "H_MS", "H_A", "H_P")


def build_hierarchies(bs: BlockSystem, eps0=amg.EPS0, max_coarse=amg.MAX_COARSE,
                      max_levels=amg.MAX_LEVELS, schur: str = "simple", x_approx: str = "F") -> dict:
    """The five SA hierarchies of the preconditioner (`schur`: the pressure
    Schur approximation, see FluidBlock.schur; `x_approx`: the fluid operator
    standing for the Schur complement X, see BlockSystem.fluid_x)."""
    d = bs.dim
    sysm = bs.sys
    o = sysm.offsets
    # coordinates of the solid velocity nodes (rigid-body modes of Sigma_s)
    vs_nodes = sysm.dof_node[o[1]:o[1] + bs.n_vs:d]
    xyz = sysm.coords[vs_nodes]
    kw = dict(eps0=eps0, max_coarse=max_coarse, max_levels=max_levels)
    L = bs.mesh_scalar()
    fl = bs.fluid_x(x_approx)
    H = {
        "H_M": amg.setup(L, 1, amg.constant_modes(L.shape[0]), **kw),
        "H_SIG": amg.setup(bs.solid_schur(), d, amg.rigid_body_modes(xyz), **kw),
        "H_MS": amg.setup(bs.S_uu, 1, amg.constant_modes(bs.n_vs), **kw),
        "H_A": amg.setup(fl.A_f, d, amg.translation_modes(bs.n_vf // d, d), **kw),
        "H_P": amg.setup(fl.schur(schur), 1, amg.constant_modes(bs.n_p), **kw),
    }
    return H


class BlockLDU:
    """P^{-1} r by the paper's algorithm, with pluggable sub-inverses.

    ``mesh_inv``, ``solid_inv`` and ``fluid_inv`` map a residual of the
    corresponding block to an approximate solution.  ``cfs`` is the coupling
    used in step 3 (C_fs in the paper's algorithm; the exact factorisation
    uses C_fs - C_fm M^{-1} C_ms there) and ``fluid_inv`` may be replaced by
    an exact inverse of the Schur complement X for identity tests.

    ``order``: the block order of the factorisation, a permutation of
    "msf" (m mesh, s solid, f fluid).  "msf" (default) is the paper's order
    and its algorithm "Evaluation of P^{-1} r" (Section 4.1), written out in
    ``apply``.  The remark after the factorisation in Section 4.1 notes that
    another order gives another preconditioner.  Factorising A' (C_sm
    dropped, as in the paper) in the order (a, b, c) and dropping every
    perturbation of the pivots and multipliers, as the paper does for its own
    order (X by F, C~_fs by C_fs), leaves a block symmetric Gauss-Seidel
    sweep in that order,

        forward:   x_i = A_ii^{-1} (r_i - sum_{j before i} A_ij x_j),
        backward:  x_i -= A_ii^{-1} sum_{j after i} A_ij x_j  (i = b, then a),

    with A_mm = M, A_ss = S, A_ff = F and the couplings C_fm, C_fs, C_sf,
    C_ms (C_sm and C_mf are zero).  For "msf" these are exactly the paper's
    five steps.  E.g. the reverse order "fsm":
    x_f = F^{-1} r_f;  x_s = S^{-1} (r_s - C_sf x_f);
    x_m = M^{-1} (r_m - C_ms x_s);  x_f -= F^{-1} (C_fm x_m + C_fs x_s).

    ``csm`` (orders other than "msf") stands for the solid-mesh coupling,
    which the preconditioner drops; identity tests with the exact pivots of
    an elimination set it to the entry that elimination leaves there.
    """

    ORDERS = ("msf", "fsm", "mfs", "smf", "sfm", "fms")

    def __init__(self, bs: BlockSystem, mesh_inv, solid_inv, fluid_inv, cfs=None, order: str = "msf", csm=None):
        if order not in self.ORDERS:
            raise ValueError(f"unknown block order {order!r}")
        self.bs = bs
        self.mesh_inv, self.solid_inv, self.fluid_inv = mesh_inv, solid_inv, fluid_inv
        self.cfs = cfs
        self.order = order
        self.csm = csm

    def _coupling(self, i: str, j: str):
        """x_j -> A_ij x_j for the off-diagonal block (i, j) of A', or None."""
        B = self.bs.B
        if (i, j) == ("f", "m"):
            return lambda x: B["C_fm"] @ x
        if (i, j) == ("f", "s"):
            return self.cfs if self.cfs is not None else (lambda x: B["C_fs"] @ x)
        if (i, j) == ("s", "f"):
            return lambda x: B["C_sf"] @ x
        if (i, j) == ("m", "s"):
            return lambda x: B["C_ms"] @ x
        if (i, j) == ("s", "m"):
            return self.csm
        return None  # (m, f): no mesh-fluid coupling

    def _apply_ordered(self, r: np.ndarray) -> np.ndarray:
        bs = self.bs
        inv = {"m": self.mesh_inv, "s": self.solid_inv, "f": self.fluid_inv}
        rb = dict(zip("msf", bs.split(r)))
        o = self.order
        x = {}

        def coupled(i, js):
            terms = [(self._coupling(i, j), j) for j in js]
            terms = [(A, j) for A, j in terms if A is not None]
            if not terms:
                return None
            return sum(A(x[j]) for A, j in terms)

        for k, i in enumerate(o):
            c = coupled(i, o[:k])
            x[i] = inv[i](rb[i] if c is None else rb[i] - c)
        for k in (1, 0):
            i = o[k]
            c = coupled(i, o[k + 1:])
            if c is not None:
                x[i] = x[i] - inv[i](c)
        return bs.join(x["m"], x["s"], x["f"])

    def apply(self, r: np.ndarray) -> np.ndarray:
        if self.order != "msf":
            return self._apply_ordered(r)
        bs = self.bs
        B = bs.B
        r_m, r_s, r_f = bs.split(r)
        x_m = self.mesh_inv(r_m)
        x_s = self.solid_inv(r_s)
        cfs_xs = self.cfs(x_s) if self.cfs is not None else B["C_fs"] @ x_s
        x_f = self.fluid_inv(r_f - B["C_fm"] @ x_m - cfs_xs)
        x_s = x_s - self.solid_inv(B["C_sf"] @ x_f)
        x_m = x_m - self.mesh_inv(B["C_ms"] @ x_s)
        return bs.join(x_m, x_s, x_f)

    __call__ = apply


def solid_schur_solve(bs: BlockSystem, ms_inv, sig_inv, r_s: np.ndarray) -> np.ndarray:
    """Solid algorithm of Section 4.3 (u_s eliminated, then recovered)."""
    nvs = bs.n_vs
    r_v, r_u = r_s[:nvs], r_s[nvs:]
    y = ms_inv(r_u)
    x_v = sig_inv(r_v - bs.S_vu @ y)
    x_u = ms_inv(r_u - bs.S_uv @ x_v)
    return np.concatenate([x_v, x_u])


def fluid_schur_solve(bs: BlockSystem, a_inv, p_inv, r_f: np.ndarray) -> np.ndarray:
    """Uzawa-like Schur elimination of the fluid saddle point (Section 4.4)."""
    nvf = bs.n_vf
    r_v, r_p = r_f[:nvf], r_f[nvf:]
    y = a_inv(r_v)
    x_p = p_inv(r_p - bs.D @ y)
    x_v = a_inv(r_v - bs.G @ x_p)
    return np.concatenate([x_v, x_p])


def fluid_triangular_solve(bs: BlockSystem, a_inv, p_inv, r_f: np.ndarray) -> np.ndarray:
    """Block upper-triangular step for F = [[A_f, G], [D, 0]]: the inverse of
    U = [[A_f, G], [0, S]] (S = -D A_f^{-1} G, the Schur complement) with the
    approximate inverses a_inv ~ A_f^{-1}, p_inv ~ S^{-1}.  F U^{-1} is then
    unit lower block-triangular: with exact inverses two GMRES steps solve."""
    nvf = bs.n_vf
    r_v, r_p = r_f[:nvf], r_f[nvf:]
    x_p = p_inv(r_p)
    x_v = a_inv(r_v - bs.G @ x_p)
    return np.concatenate([x_v, x_p])


def fluid_gmres_solve(bs: BlockSystem, uzawa, r_f: np.ndarray, k: int) -> np.ndarray:
    """F^{-1} r_f as k steps of flexible GMRES on F = [[A_f, G], [D, 0]] from
    x = 0, right-preconditioned by `uzawa` (the Uzawa-like step): the fluid
    sub-problem solved by AMG-preconditioned GMRES (Section 4.4; the step
    count k is a parameter, the paper does not state one).  The result
    minimises ||r_f - F x|| over x in span{uzawa(v_1), ..., uzawa(v_k)} of the
    Arnoldi vectors v_j."""
    if k < 1:
        raise ValueError("inner GMRES needs k >= 1 steps")
    F = bs.F
    x, _ = krylov.fgmres(lambda v: F @ v, uzawa, r_f, tol=INNER_TOL, restart=k, maxit=k)
    return x


def gmres_steps(A, pc, b: np.ndarray, k: int) -> np.ndarray:
    """k steps of right-preconditioned GMRES on A x = b from x = 0 with the
    preconditioner pc (stopping before k steps only at an exact solve)."""
    if k < 1:
        raise ValueError("GMRES needs k >= 1 steps")
    x, _ = krylov.fgmres(lambda v: A @ v, pc, b, tol=INNER_TOL, restart=k, maxit=k)
    return x


def fluid_schur_gmres_solve(fl, S_p, a_pc, p_pc, r_f: np.ndarray, k: int) -> np.ndarray:
    """Section 4.4 as written: the Uzawa-like elimination of the fluid saddle
    point with every occurring inverse approximated by AMG-preconditioned
    GMRES, here k steps from zero each: A_f^{-1} (twice) by GMRES on A_f
    preconditioned by the A_f V-cycle a_pc, S_p^{-1} by GMRES on the explicit
    pressure Schur approximation S_p preconditioned by its V-cycle p_pc."""
    a_inv = lambda b: gmres_steps(fl.A_f, a_pc, b, k)
    p_inv = lambda b: gmres_steps(S_p, p_pc, b, k)
    return fluid_schur_solve(fl, a_inv, p_inv, r_f)


def mesh_solve(bs: BlockSystem, l_inv, r_m: np.ndarray) -> np.ndarray:
    """M^{-1} r_m with M = L (x) I_d: the scalar inverse per component."""
    d = bs.dim
    x = np.empty_like(r_m)
    for c in range(d):
        x[c::d] = l_inv(np.ascontiguousarray(r_m[c::d]))
    return x


def amg_preconditioner(bs: BlockSystem, H: dict, cheb: dict | None = None, poly: dict | None = None,
                       fluid_inner: int = 0, fluid_inner_pc: str = "uzawa", x_approx: str = "F",
                       uzawa_inner: int = 0, order: str = "msf") -> BlockLDU:
    """The preconditioner of the hot path: every inverse one V(1,1) cycle
    (Jacobi sweeps; Chebyshev sweeps of degree cheb[name] for the hierarchies
    named in `cheb`).  For the names in `poly`, {name: (k, ratio)}, the
    inverse is instead k Chebyshev steps alone on the finest matrix (no coarse
    grid), on [lam/ratio, lam] with lam = 1.1 rho of that level.  With
    fluid_inner = k > 0 the fluid inverse is k inner GMRES steps
    preconditioned by the Uzawa-like step (fluid_inner_pc = "uzawa") or by
    the block upper-triangular step ("triangular").  x_approx: the fluid
    operator those steps invert in place of the Schur complement X (F, or
    its block-diagonal approximation; the hierarchies H must be built with
    the same choice).  uzawa_inner = k > 0: the Uzawa-like step with every
    occurring inverse taken as k GMRES steps preconditioned by its V-cycle
    (fluid_schur_gmres_solve; not combined with fluid_inner).  order: the
    block order of the factorisation (BlockLDU)."""
    cheb = cheb or {}
    fl = bs.fluid_x(x_approx)
    poly = poly or {}

    def inv(name, h):
        if name in poly and h.nlevels > 1:
            k, ratio = poly[name]
            L0 = h.levels[0]
            lam = amg.CHEB_BOOST * L0.rho
            return lambda b: amg.chebyshev(L0.A, L0.dinv, b, np.zeros_like(b), k, lam, ratio)
        if name in cheb:
            k = cheb[name]
            return lambda b: amg.vcycle_cheb(h, b, k)
        return lambda b: amg.vcycle(h, b)
    V = {k: inv(k, h) for k, h in H.items()}
    mesh = lambda r: mesh_solve(bs, V["H_M"], r)
    solid = lambda r: solid_schur_solve(bs, V["H_MS"], V["H_SIG"], r)
    uzawa = lambda r: fluid_schur_solve(fl, V["H_A"], V["H_P"], r)
    fluid = uzawa
    if uzawa_inner > 0:
        if fluid_inner > 0:
            raise ValueError("inner GMRES on F and on the Uzawa step's inverses do not combine")
        S_p = H["H_P"].levels[0].A
        fluid = lambda r: fluid_schur_gmres_solve(fl, S_p, V["H_A"], V["H_P"], r, uzawa_inner)
    if fluid_inner > 0:
        if fluid_inner_pc == "uzawa":
            inner = uzawa
        elif fluid_inner_pc == "triangular":
            inner = lambda r: fluid_triangular_solve(fl, V["H_A"], V["H_P"], r)
        else:
            raise ValueError(f"unknown inner fluid preconditioner {fluid_inner_pc!r}")
        fluid = lambda r: fluid_gmres_solve(fl, inner, r, fluid_inner)
    return BlockLDU(bs, mesh, solid, fluid, order=order)
