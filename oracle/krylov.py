"""Flexible GMRES(m), right preconditioned (oracle; test infrastructure only).

The paper solves every Newton system with GMRES preconditioned by its block
LDU factorisation (Sections 1, 4 and the solver settings of Section 6).  The
variant here is Saad's flexible GMRES (right preconditioning, the
preconditioned vectors z_j are stored), restarted every m steps, with
modified Gram-Schmidt Arnoldi, Givens rotations for the least-squares
problem, and acceptance only on the recomputed true residual
||b - A x||_2 <= tol ||b||_2.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Info:
    iters: int = 0
    restarts: int = 0
    converged: bool = False
    true_rel_resid: float = float("nan")
    history: list = dataclasses.field(default_factory=list)  # |g_{j+1}| / ||b|| per iteration
    arnoldi: list = dataclasses.field(default_factory=list)  # (V, Z, Hbar) of each cycle, if kept


def givens(a: float, b: float):
    """Rotation (c, s) with -s a + c b = 0 (overflow-safe form)."""
    if b == 0.0:
        return 1.0, 0.0
    if abs(b) > abs(a):
        t = a / b
        s = 1.0 / math.sqrt(1.0 + t * t)
        return s * t, s
    t = b / a
    c = 1.0 / math.sqrt(1.0 + t * t)
    return c, c * t


def fgmres(A, P, b: np.ndarray, x0=None, tol: float = 1e-8, restart: int = 50,
           maxit: int = 2000, keep_arnoldi: bool = False):
    """Solve A x = b; A and P are callables (mat-vec and P^{-1} application)."""
    info = Info()
    bnorm = float(np.linalg.norm(b))
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    if bnorm == 0.0:
        info.converged, info.true_rel_resid = True, 0.0
        return np.zeros(n), info
    m = restart
    while True:
        r = b - A(x)
        beta = float(np.linalg.norm(r))
        info.true_rel_resid = beta / bnorm
        if beta / bnorm <= tol:
            info.converged = True
            return x, info
        if info.iters >= maxit:
            return x, info
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        j_end = 0
        for j in range(m):
            Z[j] = P(V[j])
            w = A(Z[j])
            w_before = float(np.linalg.norm(w))
            for i in range(j + 1):
                H[i, j] = float(w @ V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            breakdown = H[j + 1, j] <= 1e-14 * w_before
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            Hbar_col = H[:j + 2, j].copy()
            for i in range(j):
                hi, hi1 = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * hi + sn[i] * hi1
                H[i + 1, j] = -sn[i] * hi + cs[i] * hi1
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info.iters += 1
            info.history.append(abs(g[j + 1]) / bnorm)
            if keep_arnoldi:
                info.arnoldi.append(Hbar_col)
            j_end = j + 1
            if abs(g[j + 1]) / bnorm <= tol or breakdown or info.iters >= maxit:
                break
        k = j_end
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        if keep_arnoldi:
            info.arnoldi.append(("cycle", V[:k + 1].copy(), Z[:k].copy()))
        info.restarts += 1
