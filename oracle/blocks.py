"""The 3x3 block Jacobian and its sub-blocks (oracle; test infrastructure only).

A_h = [[M, C_ms, 0], [C_sm, S, C_sf], [C_fm, C_fs, F]] with the unknowns
ordered (mesh, solid, fluid), paper Section 3.4 (the block matrix A_h).
The solid block is split as S = [[S_vv, S_vu], [S_uv, S_uu]] over
(v_s, u_s) (Section 4.3) and the fluid block as F = [[A_f, G], [D, 0]] over
(v_f, p) (Section 4.4).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

NAMES = ("M", "C_ms", "C_sm", "S", "C_sf", "C_fm", "C_fs", "F")


def to_scipy(b) -> sp.csr_matrix:
    """fsigen.Csr -> scipy CSR (same arrays, canonical order)."""
    m = sp.csr_matrix((b.val, b.col.astype(np.int64), b.rowptr), shape=(b.nrows, b.ncols))
    m.sort_indices()
    return m


def spmv(A: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """y_i = sum_k val[k] * x[col[k]] over row i, summed in storage order.

    Pinned against dense mat-vec and unit columns (tests/test_oracle_blocks).
    """
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    return np.bincount(rows, weights=A.data * x[A.indices], minlength=A.shape[0])


class FluidBlock:
    """A fluid operator in saddle form [[A_f, G], [D, Z]] over (v_f | p): the
    fluid block F of A_h (Z empty) or an approximation of the Schur
    complement X of Section 4.1 (BlockSystem.fluid_x)."""

    def __init__(self, F: sp.csr_matrix, n_vf: int):
        self.F = F.tocsr()
        self.F.sort_indices()
        self.n_vf = n_vf
        self.A_f = self.F[:n_vf, :n_vf].tocsr()
        self.G = self.F[:n_vf, n_vf:].tocsr()
        self.D = self.F[n_vf:, :n_vf].tocsr()
        self.F_pp = self.F[n_vf:, n_vf:].tocsr()
        for m in (self.A_f, self.G, self.D, self.F_pp):
            m.sort_indices()

    def schur(self, variant: str = "simple") -> sp.csr_matrix:
        """S_p = Z - D W^{-1} G, a pressure Schur approximation.

        The paper applies to the fluid block the same Schur-complement
        elimination as for the solid (Section 4.4) without stating the
        approximation; this is the reading recorded in the design notes.
        variant "simple": W = diag(A_f) (SIMPLE); "simplec": W = the diagonal
        of the absolute row sums sum_j |a_ij| of A_f (SIMPLEC, one of the
        alternatives the paper lists as open).
        Pinned: both equal the exact Schur complement Z - D A_f^{-1} G when A_f
        is diagonal with a positive diagonal (test), and are symmetric because
        G = -D^T (F itself, Z = 0).
        """
        if variant == "simple":
            dinv = 1.0 / self.A_f.diagonal()
        elif variant == "simplec":
            dinv = 1.0 / np.asarray(abs(self.A_f).sum(axis=1)).ravel()
        else:
            raise ValueError(f"unknown Schur variant {variant!r}")
        m = (-(self.D @ sp.diags(dinv) @ self.G)).tocsr()
        if self.F_pp.nnz:
            m = (m + self.F_pp).tocsr()
        m.eliminate_zeros()
        m.sort_indices()
        return m


def node_block_inverse(A: sp.csr_matrix, b: int) -> sp.csr_matrix:
    """Inverse of the node-block diagonal of A: the entries (i, j) with
    i // b == j // b, inverted b x b block by block (dense numpy inverses)."""
    n = A.shape[0]
    Ad = A.tocoo()
    keep = (Ad.row // b) == (Ad.col // b)
    blocks = np.zeros((n // b, b, b))
    blocks[Ad.row[keep] // b, Ad.row[keep] % b, Ad.col[keep] % b] = Ad.data[keep]
    inv = np.linalg.inv(blocks)
    rows = (np.arange(n // b)[:, None, None] * b + np.arange(b)[None, :, None]) + np.zeros((1, 1, b), dtype=int)
    cols = (np.arange(n // b)[:, None, None] * b + np.arange(b)[None, None, :]) + np.zeros((1, b, 1), dtype=int)
    m = sp.csr_matrix((inv.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n))
    m.sort_indices()
    return m


class BlockSystem:
    """A_h with its block views, built from one fsigen.FsiSystem."""

    def __init__(self, sysm):
        self.sys = sysm
        self.dim = sysm.dim
        self.n_m, self.n_s, self.n_f = sysm.n_m, sysm.n_s, sysm.n_f
        self.n_vs, self.n_vf, self.n_p = sysm.n_vs, sysm.n_vf, sysm.n_p
        self.N = sysm.N
        self.dt_theta = sysm.dt_theta
        self.B = {k: to_scipy(v) for k, v in sysm.blocks.items()}
        nvs, nvf = self.n_vs, self.n_vf
        S, F = self.B["S"], self.B["F"]
        # solid sub-blocks over (v_s | u_s)
        self.S_vv = S[:nvs, :nvs].tocsr()
        self.S_vu = S[:nvs, nvs:].tocsr()
        self.S_uv = S[nvs:, :nvs].tocsr()
        self.S_uu = S[nvs:, nvs:].tocsr()
        # fluid sub-blocks over (v_f | p)
        self.fluid = FluidBlock(F, nvf)
        self.A_f, self.G, self.D, self.F_pp = self.fluid.A_f, self.fluid.G, self.fluid.D, self.fluid.F_pp
        for m in (self.S_vv, self.S_vu, self.S_uv, self.S_uu):
            m.sort_indices()

    @property
    def F(self) -> sp.csr_matrix:
        return self.B["F"]

    # -- splitting ---------------------------------------------------------
    def split(self, x):
        a, b = self.n_m, self.n_m + self.n_s
        return x[:a], x[a:b], x[b:]

    def join(self, xm, xs, xf):
        return np.concatenate([xm, xs, xf])

    # -- block mat-vec, Section 3.4 ------------------------------------------
    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = A_h x over the eight stored blocks (C_sm included)."""
        B = self.B
        xm, xs, xf = self.split(x)
        ym = spmv(B["M"], xm) + spmv(B["C_ms"], xs)
        ys = spmv(B["C_sm"], xm) + spmv(B["S"], xs) + spmv(B["C_sf"], xf)
        yf = spmv(B["C_fm"], xm) + spmv(B["C_fs"], xs) + spmv(B["F"], xf)
        return self.join(ym, ys, yf)

    def dense(self, drop_csm: bool = False) -> np.ndarray:
        """Dense A_h (tiny systems only), optionally with C_sm := 0."""
        N = self.N
        A = np.zeros((N, N))
        o = (0, self.n_m, self.n_m + self.n_s, N)
        place = {"M": (0, 0), "C_ms": (0, 1), "C_sm": (1, 0), "S": (1, 1), "C_sf": (1, 2),
                 "C_fm": (2, 0), "C_fs": (2, 1), "F": (2, 2)}
        for name, (i, j) in place.items():
            if drop_csm and name == "C_sm":
                continue
            A[o[i]:o[i + 1], o[j]:o[j + 1]] = self.B[name].toarray()
        return A

    # -- derived operators ---------------------------------------------------
    def solid_schur(self) -> sp.csr_matrix:
        """Sigma_s = S_vv + dt*theta*S_vu.

        Eliminating u_s with S_uu = M and S_uv = -dt*theta*M (equal-order
        mass matrices, Section 4.3) gives x_u = M^{-1} r_u + dt*theta*x_v and
        hence (S_vv + dt*theta*S_vu) x_v = r_v - S_vu M^{-1} r_u.  On rows of
        pure solid nodes this is rho_s M + dt^2 theta^2 K of Section 4.3.
        Pinned by the dense solid-equivalence test.
        """
        m = (self.S_vv + self.dt_theta * self.S_vu).tocsr()
        m.sort_indices()
        return m

    def fluid_schur(self, variant: str = "simple") -> sp.csr_matrix:
        """The pressure Schur approximation of F (FluidBlock.schur)."""
        return self.fluid.schur(variant)

    def fluid_x(self, approx: str = "F") -> FluidBlock:
        """The fluid operator that the preconditioner inverts in place of the
        Schur complement X = F - C~_fs S^{-1} C_sf, C~_fs = C_fs - C_fm M^{-1}
        C_ms, of the factorisation in Section 4.1 (garbled there; the reading
        in the design notes).

        approx "F": X ~ F, the perturbation dropped (the paper's choice, and
        the algorithm "Evaluation of P^{-1} r").  approx "blockdiag": S and M
        replaced by their node-block diagonals (d x d blocks of each field,
        per node), which are inverted exactly: X ~ F - C~ D_S^{-1} C_sf with
        C~ = C_fs - C_fm D_M^{-1} C_ms (the block-diagonal approximation the
        paper cites from Langer and Yang, 2016).  Here the C_fm D_M^{-1} C_ms
        part adds nothing: C_ms reads only u_s, while D_S^{-1} C_sf has only
        v_s rows (the u_s rows of C_sf, the solid kinematics, hold no fluid
        entries, and D_S does not mix the fields).  Pinned: with S and M block
        diagonal themselves it is the exact X (dense test)."""
        if approx == "F":
            return self.fluid
        if approx != "blockdiag":
            raise ValueError(f"unknown approximation of X {approx!r}")
        B = self.B
        d = self.dim
        DSi = node_block_inverse(B["S"], d)
        DMi = node_block_inverse(B["M"], d)
        Ct = (B["C_fs"] - B["C_fm"] @ DMi @ B["C_ms"]).tocsr()
        X = (B["F"] - Ct @ DSi @ B["C_sf"]).tocsr()
        X.eliminate_zeros()
        return FluidBlock(X, self.n_vf)

    def mesh_scalar(self) -> sp.csr_matrix:
        """Scalar Laplacian L with M = L (x) I_d (frozen Jacobian-scaled mesh).

        Raises if M does not have that structure.
        """
        d = self.dim
        M = self.B["M"]
        L = M[0::d, 0::d].tocsr()
        L.sort_indices()
        K = sp.kron(L, sp.identity(d), format="csr")
        diff = abs(K - M)
        if diff.nnz and diff.max() > 0.0:
            raise ValueError("mesh block is not L (x) I_d")
        return L
