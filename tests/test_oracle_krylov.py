"""Oracle pins: flexible GMRES against brute force and textbook properties."""
import numpy as np
import pytest

from oracle import krylov


def _problem(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 3 * np.sqrt(n) * np.eye(n)
    b = rng.standard_normal(n)
    return A, b


def test_n_steps_reach_the_exact_solution():
    A, b = _problem(24, 0)
    x, info = krylov.fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-15, restart=24, maxit=24)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-10 * np.linalg.norm(x)


@pytest.mark.parametrize("k", [1, 3, 6])
def test_k_steps_minimise_the_residual_over_the_krylov_space(k):
    """x_k = argmin ||b - A x|| over K_k(A, b), computed by brute-force least squares."""
    A, b = _problem(40, 1)
    x, info = krylov.fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-30, restart=k, maxit=k)
    K = np.column_stack([np.linalg.matrix_power(A, i) @ b for i in range(k)])
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
    assert np.allclose(x, Q @ y, rtol=1e-9, atol=1e-12)


def test_right_preconditioned_minimises_over_preconditioned_space():
    A, b = _problem(30, 2)
    Pm = np.diag(1.0 / np.diag(A)) + 0.01 * np.random.default_rng(3).standard_normal((30, 30))
    k = 4
    x, _ = krylov.fgmres(lambda v: A @ v, lambda v: Pm @ v, b, tol=1e-30, restart=k, maxit=k)
    AP = A @ Pm
    K = np.column_stack([np.linalg.matrix_power(AP, i) @ b for i in range(k)])
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(AP @ Q, b, rcond=None)
    assert np.allclose(x, Pm @ Q @ y, rtol=1e-9, atol=1e-12)


def test_arnoldi_relation_orthonormality_and_residual_estimate():
    A, b = _problem(50, 4)
    Pm = np.diag(1.0 / np.diag(A))
    m = 12
    x, info = krylov.fgmres(lambda v: A @ v, lambda v: Pm @ v, b, tol=1e-30, restart=m, maxit=m,
                            keep_arnoldi=True)
    cols = [c for c in info.arnoldi if not isinstance(c, tuple)]
    _, V, Z = info.arnoldi[-1]
    Hbar = np.zeros((m + 1, m))
    for j, c in enumerate(cols):
        Hbar[:j + 2, j] = c
    assert np.allclose(A @ Z.T, V.T @ Hbar, atol=1e-11 * np.abs(A).max())
    # modified Gram-Schmidt loses orthogonality ~ eps * cond([r0, A Z]) (Bjorck);
    # the residual falls by ~1e-6 here, so ~1e-10 is the expected level
    assert np.allclose(V @ V.T, np.eye(m + 1), atol=1e-8)
    # |g_{j+1}| equals the true residual of the least-squares iterate (fixed P)
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert np.isclose(info.history[-1], true, rtol=1e-8)
    assert all(h2 <= h1 * (1 + 1e-14) for h1, h2 in zip(info.history, info.history[1:]))


def test_restarts_stop_on_true_residual_and_maxit():
    A, b = _problem(60, 5)
    x, info = krylov.fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-10, restart=5, maxit=500)
    assert info.converged and np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    assert info.restarts >= 2
    x2, info2 = krylov.fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-14, restart=5, maxit=3)
    assert not info2.converged and info2.iters == 3


def test_zero_rhs_and_breakdown():
    A, b = _problem(10, 6)
    x, info = krylov.fgmres(lambda v: A @ v, lambda v: v, np.zeros(10))
    assert info.converged and not x.any() and info.iters == 0
    # b an eigenvector: happy breakdown after one step, exact solution
    D = np.diag(np.arange(1.0, 11.0))
    e = np.zeros(10)
    e[3] = 2.0
    x, info = krylov.fgmres(lambda v: D @ v, lambda v: v, e, tol=1e-14)
    assert info.iters == 1 and np.allclose(x, e / 4.0)


def test_givens_zeroes_second_component():
    for a, b in [(3.0, 4.0), (-1e-3, 2.0), (5.0, -1e-8), (0.0, 1.0), (2.0, 0.0)]:
        c, s = krylov.givens(a, b)
        assert np.isclose(c * c + s * s, 1.0)
        assert abs(-s * a + c * b) <= 1e-15 * max(abs(a), abs(b))
        assert np.isclose(abs(c * a + s * b), np.hypot(a, b))
