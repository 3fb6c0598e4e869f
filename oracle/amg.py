"""Smoothed-aggregation AMG and dense LU (oracle; test infrastructure only).

The paper approximates every inverse of its block preconditioner by AMG
(Trilinos ML, smoothed aggregation; Sections 4.2-4.4) without giving any
parameter.  The concrete, deterministic algorithm below is the reading the
design notes record; both this oracle and the GPU library implement it
independently.

Setup of level l (matrix A_l, node block size b_l, near-nullspace B_l, n_l x k):

1. omega_l = (4/3) / rho_l, rho_l = ||D^{-1} A x_30||_2 after 30 normalised
   power steps x_{j+1} = D^{-1} A x_j / ||D^{-1} A x_j||_2 from
   x_0 = (1 + (i mod 7)/7)_i / norm, D = diag(A_l).
2. Strength between nodes I != J: s_IJ = sum of A_ij^2 over the stored
   entries of the b x b node block (rows of I ascending, columns in storage
   order); strong iff s_IJ^2 >= eps_l^4 * (s_II * s_JJ) (i.e. Frobenius norm
   a_IJ >= eps_l sqrt(a_II a_JJ)), eps_0 = 0.08, eps_{l+1} = eps_l / 2.
   N(I) = strong neighbours from row I.
3. Aggregation, nodes in increasing id:
   (1) I unaggregated with N(I) non-empty and every J in N(I) unaggregated
       seeds a new aggregate {I} + N(I);
   (2) every node still unaggregated joins the aggregate of the phase-1 node
       J in N(I) with the largest s_IJ (values within a relative 1e-8 of the
       largest count as ties; ties go to the smallest aggregate id);
   (3) every node still unaggregated seeds a new aggregate with its
       unaggregated strong neighbours (an isolated node is a singleton).
4. Tentative prolongator: per aggregate (nodes ascending, dofs node*b + c)
   thin QR of the aggregate's rows of B_l by modified Gram-Schmidt in the
   column order of B_l; a column with r_jj <= 1e-10 ||B_agg||_F is rank
   deficient and set to zero.  Q gives the k columns of the aggregate in
   P_tent, R gives the aggregate's k rows of B_{l+1}; b_{l+1} = k.
5. Filtered matrix A^F: entries of weak node pairs are dropped and their sum
   (storage order) is added to the diagonal entry of the row.
   P_l = P_tent - (omega_l / diag(A^F)) * (A^F P_tent).
6. R_l = P_l^T, A_{l+1} = R_l A_l P_l, exact zeros dropped; a coarse dof with
   an empty row gets diagonal 1.
7. Stop when n_l <= max_coarse (500), when l = max_levels - 1 (10 levels),
   or when n_{l+1} > 0.8 n_l: level L is then solved by dense LU with partial
   pivoting.

V(1,1) cycle: vcycle(l, b) = LU^{-1} b at l = L, otherwise
  x = omega_l D_l^{-1} b;  r = b - A_l x;  x += P_l vcycle(l+1, R_l r);
  x += omega_l D_l^{-1} (b - A_l x).

Chebyshev variant (vcycle_cheb): both sweeps are k steps of the Chebyshev
iteration for D_l^{-1} A_l on [lam/30, lam], lam = 1.1 rho_l (the power
estimate underestimates the spectral radius), instead of one Jacobi sweep.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

EPS0 = 0.08
MAX_COARSE = 500
MAX_LEVELS = 10
POWER_ITERS = 30
RANK_TOL = 1e-10
TIE_REL = 1e-8
MAX_DENSE_COARSE = 6000
CHEB_RATIO = 30.0
CHEB_BOOST = 1.1


# ----------------------------------------------------------------- dense LU
def lu_factor(A: np.ndarray):
    """Doolittle LU with partial pivoting (ties: smallest row index).

    Returns (LU, piv) with the unit lower factor below the diagonal and piv[k]
    the row swapped with k at step k.  Pinned: 3x3 against Cramer's rule and
    random well-conditioned systems against a known solution.
    """
    LU = np.array(A, dtype=np.float64, copy=True)
    n = LU.shape[0]
    piv = np.arange(n)
    for k in range(n):
        p = k + int(np.argmax(np.abs(LU[k:, k])))  # argmax returns the first maximum
        if LU[p, k] == 0.0:
            raise ZeroDivisionError("singular matrix in dense LU")
        piv[k] = p
        if p != k:
            LU[[k, p], :] = LU[[p, k], :]
        LU[k + 1:, k] /= LU[k, k]
        LU[k + 1:, k + 1:] -= np.outer(LU[k + 1:, k], LU[k, k + 1:])
    return LU, piv


def lu_solve(fac, b: np.ndarray) -> np.ndarray:
    LU, piv = fac
    x = np.array(b, dtype=np.float64, copy=True)
    n = LU.shape[0]
    for k in range(n):
        p = piv[k]
        if p != k:
            x[k], x[p] = x[p], x[k]
    for i in range(n):  # forward, unit lower
        x[i] -= LU[i, :i] @ x[:i]
    for i in range(n - 1, -1, -1):
        x[i] = (x[i] - LU[i, i + 1:] @ x[i + 1:]) / LU[i, i]
    return x


# ---------------------------------------------------------------- structures
@dataclasses.dataclass
class Level:
    A: sp.csr_matrix
    P: sp.csr_matrix | None = None
    R: sp.csr_matrix | None = None
    dinv: np.ndarray | None = None
    omega: float = 0.0
    rho: float = 0.0
    block: int = 1
    aggregates: np.ndarray | None = None
    B: np.ndarray | None = None


@dataclasses.dataclass
class Hierarchy:
    levels: list
    coarse_lu: tuple

    @property
    def nlevels(self) -> int:
        return len(self.levels)

    def operator_complexity(self) -> float:
        return sum(l.A.nnz for l in self.levels) / self.levels[0].A.nnz


# --------------------------------------------------------------------- setup
def spectral_radius(A: sp.csr_matrix, dinv: np.ndarray) -> float:
    n = A.shape[0]
    x = 1.0 + (np.arange(n) % 7) / 7.0
    x = x / np.linalg.norm(x)
    for _ in range(POWER_ITERS):
        y = dinv * (A @ x)
        x = y / np.linalg.norm(y)
    return float(np.linalg.norm(dinv * (A @ x)))


def strength(A: sp.csr_matrix, b: int, eps: float):
    """Node-block squared Frobenius norms and the strong-neighbour lists."""
    n = A.shape[0]
    nn = n // b
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    I = rows // b
    J = A.indices // b
    # node-pair ids in storage order; accumulate sequentially with np.add.at
    key = I.astype(np.int64) * nn + J
    uniq, inv = np.unique(key, return_inverse=True)
    s = np.zeros(uniq.shape[0])
    np.add.at(s, inv, A.data * A.data)
    pI = uniq // nn
    pJ = uniq % nn
    sdiag = np.zeros(nn)
    on = pI == pJ
    sdiag[pI[on]] = s[on]
    e2 = eps * eps
    e4 = e2 * e2
    off = ~on
    strong = np.zeros(uniq.shape[0], dtype=bool)
    strong[off] = s[off] * s[off] >= e4 * (sdiag[pI[off]] * sdiag[pJ[off]])
    strong &= s > 0.0
    # neighbour lists per node (ascending J), with their s values
    sel = np.nonzero(strong)[0]
    ptr = np.zeros(nn + 1, dtype=np.int64)
    np.add.at(ptr, pI[sel] + 1, 1)
    ptr = np.cumsum(ptr)
    return ptr, pJ[sel].copy(), s[sel].copy(), (pI, pJ, strong)


def aggregate(nn: int, ptr, nbr, sval):
    agg = -np.ones(nn, dtype=np.int64)
    nagg = 0
    ptr = ptr.tolist()
    nbr_l = nbr.tolist()
    sval_l = sval.tolist()
    # phase 1
    for I in range(nn):
        if agg[I] >= 0:
            continue
        lo, hi = ptr[I], ptr[I + 1]
        if hi == lo:
            continue
        if all(agg[J] < 0 for J in nbr_l[lo:hi]):
            agg[I] = nagg
            for J in nbr_l[lo:hi]:
                agg[J] = nagg
            nagg += 1
    phase1 = agg >= 0
    # phase 2
    new = agg.copy()
    for I in range(nn):
        if agg[I] >= 0:
            continue
        lo, hi = ptr[I], ptr[I + 1]
        cand = [(sval_l[k], int(agg[nbr_l[k]])) for k in range(lo, hi) if phase1[nbr_l[k]]]
        if not cand:
            continue
        smax = max(c[0] for c in cand)
        thr = smax * (1.0 - TIE_REL)
        new[I] = min(a for sv, a in cand if sv >= thr)
    agg = new
    # phase 3
    for I in range(nn):
        if agg[I] >= 0:
            continue
        agg[I] = nagg
        for J in nbr_l[ptr[I]:ptr[I + 1]]:
            if agg[J] < 0:
                agg[J] = nagg
        nagg += 1
    return agg, nagg


def tentative(agg: np.ndarray, nagg: int, b: int, B: np.ndarray):
    """Aggregate-wise thin QR (modified Gram-Schmidt) of the near-nullspace."""
    k = B.shape[1]
    order = np.argsort(agg, kind="stable")
    starts = np.searchsorted(agg[order], np.arange(nagg + 1))
    rows, cols, vals = [], [], []
    Bc = np.zeros((nagg * k, k))
    for a in range(nagg):
        nodes = order[starts[a]:starts[a + 1]]  # ascending node ids
        dofs = (nodes[:, None] * b + np.arange(b)[None, :]).reshape(-1)
        Ba = B[dofs, :]
        fro = float(np.sqrt(np.sum(Ba * Ba)))
        Q = np.zeros_like(Ba)
        Rm = np.zeros((k, k))
        for j in range(k):
            w = Ba[:, j].copy()
            for i in range(j):
                r = float(Q[:, i] @ w)
                Rm[i, j] = r
                w = w - r * Q[:, i]
            rjj = float(np.sqrt(w @ w))
            if rjj <= RANK_TOL * fro:
                continue  # rank deficient: zero column, zero R entry
            Rm[j, j] = rjj
            Q[:, j] = w / rjj
            rows.append(dofs)
            cols.append(np.full(dofs.shape[0], a * k + j))
            vals.append(Q[:, j])
        Bc[a * k:(a + 1) * k, :] = Rm
    n = B.shape[0]
    if rows:
        Pt = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                           shape=(n, nagg * k))
    else:
        Pt = sp.csr_matrix((n, nagg * k))
    Pt.sort_indices()
    return Pt, Bc


def filtered(A: sp.csr_matrix, b: int, strong_pairs) -> sp.csr_matrix:
    """A^F: weak off-node entries dropped and lumped into the row diagonal."""
    pI, pJ, strong = strong_pairs
    n = A.shape[0]
    nn = n // b
    strong_set = set((pI[strong] * nn + pJ[strong]).tolist())
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    I = rows // b
    J = A.indices // b
    key = I.astype(np.int64) * nn + J
    keep = (I == J) | np.isin(key, np.fromiter(strong_set, dtype=np.int64, count=len(strong_set)))
    data = A.data.copy()
    lump = np.zeros(n)
    np.add.at(lump, rows[~keep], data[~keep])
    diag_pos = np.nonzero(rows == A.indices)[0]
    AF = sp.csr_matrix((np.where(keep, data, 0.0), A.indices.copy(), A.indptr.copy()), shape=A.shape)
    AF.data[diag_pos] = AF.data[diag_pos] + lump[rows[diag_pos]]
    AF.eliminate_zeros()
    AF.sort_indices()
    return AF


def setup(A: sp.csr_matrix, block: int, B: np.ndarray, eps0: float = EPS0,
          max_coarse: int = MAX_COARSE, max_levels: int = MAX_LEVELS) -> Hierarchy:
    """Smoothed-aggregation hierarchy of A (see the module docstring)."""
    A = A.tocsr().copy()
    A.sort_indices()
    levels = []
    eps = eps0
    b = block
    Bl = np.array(B, dtype=np.float64)
    while True:
        n = A.shape[0]
        d = A.diagonal()
        if np.any(d == 0.0):
            raise ZeroDivisionError("zero diagonal in AMG level matrix")
        lev = Level(A=A, dinv=1.0 / d, block=b, B=Bl)
        levels.append(lev)
        if n <= max_coarse or len(levels) == max_levels:
            break
        lev.rho = spectral_radius(A, lev.dinv)
        lev.omega = (4.0 / 3.0) / lev.rho
        ptr, nbr, sval, pairs = strength(A, b, eps)
        agg, nagg = aggregate(n // b, ptr, nbr, sval)
        Pt, Bc = tentative(agg, nagg, b, Bl)
        AF = filtered(A, b, pairs)
        dF = AF.diagonal()
        if np.any(dF == 0.0):
            raise ZeroDivisionError("zero diagonal in the filtered AMG matrix")
        scale = lev.omega / dF
        P = (Pt - sp.diags(scale) @ (AF @ Pt)).tocsr()
        P.eliminate_zeros()
        P.sort_indices()
        nc = P.shape[1]
        if nc > 0.8 * n or nc == 0:
            lev.rho = lev.omega = 0.0
            break
        R = P.T.tocsr()
        R.sort_indices()
        Ac = (R @ (A @ P)).tocsr()
        Ac.eliminate_zeros()
        empty = np.nonzero(np.diff(Ac.indptr) == 0)[0]
        if empty.size:
            Ac = (Ac + sp.csr_matrix((np.ones(empty.size), (empty, empty)), shape=Ac.shape)).tocsr()
        Ac.sort_indices()
        lev.P, lev.R, lev.aggregates = P, R, agg
        A, Bl, b, eps = Ac, Bc, Bc.shape[1], eps / 2.0
    last = levels[-1]
    if last.A.shape[0] > MAX_DENSE_COARSE:
        raise RuntimeError("AMG coarsening stalled: coarse level too large for dense LU")
    return Hierarchy(levels, lu_factor(last.A.toarray()))


def vcycle(H: Hierarchy, b: np.ndarray, l: int = 0) -> np.ndarray:
    """One V(1,1) cycle with damped Jacobi, zero initial guess."""
    if l == H.nlevels - 1:
        return lu_solve(H.coarse_lu, b)
    L = H.levels[l]
    x = L.omega * (L.dinv * b)
    r = b - L.A @ x
    x = x + L.P @ vcycle(H, L.R @ r, l + 1)
    x = x + L.omega * (L.dinv * (b - L.A @ x))
    return x


def chebyshev(A, dinv: np.ndarray, b: np.ndarray, x: np.ndarray, degree: int, lam_max: float,
              ratio: float = CHEB_RATIO) -> np.ndarray:
    """`degree` steps of the Chebyshev iteration for A x = b preconditioned by
    D^{-1}, tuned to the interval [lam_max/ratio, lam_max] of D^{-1} A
    (three-term recurrence of the scaled Chebyshev polynomials), from x.
    The error after the k steps is T_k((theta - D^{-1}A)/delta) /
    T_k(theta/delta) applied to the initial error, theta and delta the
    centre and half-width of the interval."""
    lam_min = lam_max / ratio
    theta = 0.5 * (lam_max + lam_min)
    delta = 0.5 * (lam_max - lam_min)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = b - A @ x
    d = (dinv * r) / theta
    x = x + d
    for _ in range(degree - 1):
        r = r - A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = (rho_new * rho) * d + (2.0 * rho_new / delta) * (dinv * r)
        x = x + d
        rho = rho_new
    return x


def vcycle_cheb(H: Hierarchy, b: np.ndarray, degree: int, l: int = 0) -> np.ndarray:
    """V-cycle with `degree` Chebyshev steps as pre- and post-smoother."""
    if l == H.nlevels - 1:
        return lu_solve(H.coarse_lu, b)
    L = H.levels[l]
    lam = CHEB_BOOST * L.rho
    x = chebyshev(L.A, L.dinv, b, np.zeros_like(b), degree, lam)
    x = x + L.P @ vcycle_cheb(H, L.R @ (b - L.A @ x), degree, l + 1)
    return chebyshev(L.A, L.dinv, b, x, degree, lam)


# ------------------------------------------------------- near-nullspaces
def constant_modes(n: int) -> np.ndarray:
    return np.ones((n, 1))


def translation_modes(n_nodes: int, d: int) -> np.ndarray:
    B = np.zeros((n_nodes * d, d))
    for c in range(d):
        B[c::d, c] = 1.0
    return B


def rigid_body_modes(xyz: np.ndarray) -> np.ndarray:
    """Rigid-body modes of a d-vector field at the given node coordinates.

    Columns: d translations, then rotations (2D: (-y, x); 3D: about x
    (0, -z, y), about y (z, 0, -x), about z (-y, x, 0)); coordinates are
    taken relative to the centroid of the nodes.
    """
    n, d = xyz.shape
    c = xyz - xyz.mean(axis=0)
    if d == 2:
        B = np.zeros((n * 2, 3))
        B[0::2, 0] = 1.0
        B[1::2, 1] = 1.0
        B[0::2, 2] = -c[:, 1]
        B[1::2, 2] = c[:, 0]
        return B
    B = np.zeros((n * 3, 6))
    for t in range(3):
        B[t::3, t] = 1.0
    x, y, z = c[:, 0], c[:, 1], c[:, 2]
    B[1::3, 3], B[2::3, 3] = -z, y
    B[0::3, 4], B[2::3, 4] = z, -x
    B[0::3, 5], B[1::3, 5] = -y, x
    return B
