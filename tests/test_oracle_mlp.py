"""Oracle pins for the per-node MLP smoother: hand-written gradients against
central differences, positive homogeneity, closed forms, Adam's first step."""
import numpy as np
import pytest

from oracle import mlp


def _case(seed, n=40, k=18, h=16, d=2):
    rng = np.random.default_rng(seed)
    W = mlp.init_weights(k, h, d, seed)
    z = rng.standard_normal((n, k))
    e = rng.standard_normal((n, d))
    w = rng.random(n) + 0.5
    return W, z, e, w


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradients_match_central_differences(seed):
    W, z, e, w = _case(seed)
    L, G = mlp.loss_and_grad(W, z, e, w)
    rng = np.random.default_rng(seed + 10)
    h = 1e-6
    for li in range(3):
        for _ in range(6):
            i = rng.integers(W[li].shape[0])
            j = rng.integers(W[li].shape[1])
            Wp = [x.copy() for x in W]
            Wm = [x.copy() for x in W]
            Wp[li][i, j] += h
            Wm[li][i, j] -= h
            fd = (mlp.loss_and_grad(Wp, z, e, w)[0] - mlp.loss_and_grad(Wm, z, e, w)[0]) / (2 * h)
            assert abs(fd - G[li][i, j]) <= 1e-6 * max(1.0, abs(fd))


def test_positive_homogeneity_and_zero_input():
    W, z, e, w = _case(3)
    y, _ = mlp.forward(W, z)
    for a in (0.5, 3.0, 1e-3):
        ya, _ = mlp.forward(W, a * z)
        assert np.allclose(ya, a * y, rtol=1e-13, atol=1e-15)
    y0, _ = mlp.forward(W, np.zeros_like(z))
    assert not y0.any()


def test_linear_regime_closed_form():
    """All pre-activations positive: the network is the product W1 W2 W3."""
    rng = np.random.default_rng(4)
    W = [np.abs(rng.standard_normal((5, 4))), np.abs(rng.standard_normal((4, 4))), rng.standard_normal((4, 2))]
    z = np.abs(rng.standard_normal((7, 5)))
    y, _ = mlp.forward(W, z)
    assert np.allclose(y, z @ W[0] @ W[1] @ W[2], rtol=1e-14)


def test_adam_first_step_moves_by_lr_times_sign():
    """At t = 1 the bias-corrected step is lr * g / (|g| + eps)."""
    W = [np.ones((2, 3))]
    G = [np.array([[1.0, -2.0, 0.5], [-1e-3, 3.0, -4.0]])]
    m = [np.zeros((2, 3))]
    v = [np.zeros((2, 3))]
    W1, m1, v1 = mlp.adam_step(W, G, m, v, 1, lr=0.01)
    assert np.allclose(W1[0], 1.0 - 0.01 * G[0] / (np.abs(G[0]) + 1e-8), rtol=1e-12)


def test_stencil_inputs_layout():
    v = np.arange(12.0).reshape(6, 2)
    nbr = np.array([[0, 1, -1], [5, -1, 2]])
    z = mlp.stencil_inputs(v, nbr)
    assert z.tolist() == [[0, 1, 2, 3, 0, 0], [10, 11, 0, 0, 4, 5]]


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.14159265, 0.0])
    r = mlp.round_bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0  # ties to even
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == -2.5 and r[5] == 0.0
    assert abs(r[4] - 3.140625) < 1e-12


def test_training_reduces_the_loss():
    """A few Adam steps on a learnable target (the target is itself an MLP)."""
    W_true, z, _, w = _case(5, n=200)
    e, _ = mlp.forward(W_true, z)
    W = mlp.init_weights(18, 16, 2, 99)
    m = [np.zeros_like(x) for x in W]
    v = [np.zeros_like(x) for x in W]
    L0 = mlp.loss_and_grad(W, z, e, w)[0]
    for t in range(1, 301):
        L, G = mlp.loss_and_grad(W, z, e, w)
        W, m, v = mlp.adam_step(W, G, m, v, t, lr=3e-3)
    assert L < 0.2 * L0


def _small_hierarchy():
    from oracle import amg
    import scipy.sparse as sp
    n = 60
    A = sp.diags([-np.ones(n - 1), 2.0 + 0.1 * np.arange(n) / n, -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    return amg.setup(A, 1, amg.constant_modes(n), max_coarse=8)


def test_learned_vcycle_with_jacobi_correction_is_the_plain_cycle():
    """Feeding the damped-Jacobi sweep omega D^{-1} b as the network's output
    must reproduce the standard V(1,1) cycle: the learned branch changes only
    where the first sweep comes from."""
    from oracle import amg
    H = _small_hierarchy()
    assert H.nlevels >= 2
    rng = np.random.default_rng(0)
    B = rng.standard_normal((60, 2))
    L = H.levels[0]
    X0 = L.omega * L.dinv[:, None] * B
    out = mlp.learned_vcycle(H, B, X0)
    ref = np.column_stack([amg.vcycle(H, B[:, c]) for c in range(2)])
    assert np.allclose(out, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_learned_vcycle_falls_back_on_bad_corrections():
    from oracle import amg
    H = _small_hierarchy()
    rng = np.random.default_rng(1)
    b = rng.standard_normal((60, 1))
    ref = amg.vcycle(H, b[:, 0])[:, None]
    for X0 in (np.full((60, 1), np.nan), 1e3 * rng.standard_normal((60, 1))):
        assert np.array_equal(mlp.learned_vcycle(H, b, X0), ref)
    # a zero correction keeps the residual norm: the learned branch is taken
    # and gives the V(0,1) cycle, which differs from V(1,1)
    z = mlp.learned_vcycle(H, b, np.zeros((60, 1)))
    L = H.levels[0]
    e = amg.vcycle(H, L.R @ b[:, 0], 1)
    x = L.P @ e
    x = x + L.omega * L.dinv * (b[:, 0] - L.A @ x)
    assert np.allclose(z[:, 0], x, rtol=0, atol=1e-14 * np.abs(x).max())
    assert not np.allclose(z, ref)


def _spd_case(seed=0, n=30, nc=7):
    rng = np.random.default_rng(seed)
    A = np.diag(2.0 + rng.random(n)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    P = np.zeros((n, nc))
    for i in range(n):  # piecewise-linear interpolation from nc coarse points
        t = i * (nc - 1) / (n - 1)
        k = min(int(t), nc - 2)
        P[i, k] += 1 - (t - k)
        P[i, k + 1] += t - k
    return A, P, P.T @ A @ P, rng


def test_energy_gradient_matches_central_differences():
    A, P, Ac, rng = _spd_case()
    b = rng.standard_normal((30, 2))
    delta = rng.standard_normal((30, 2))
    L, g = mlp.two_grid_energy(delta, b, A, P, Ac)
    h = 1e-6
    for _ in range(10):
        i, c = rng.integers(30), rng.integers(2)
        dp, dm = delta.copy(), delta.copy()
        dp[i, c] += h
        dm[i, c] -= h
        fd = (mlp.two_grid_energy(dp, b, A, P, Ac)[0] - mlp.two_grid_energy(dm, b, A, P, Ac)[0]) / (2 * h)
        assert abs(fd - g[i, c]) <= 1e-6 * max(1.0, abs(fd))


def test_energy_minimum_is_the_coarse_complement_of_the_error():
    """L + e.b >= 0 everywhere, = 0 with zero gradient at delta = e - P Ac^{-1} P^T b
    (the part of the error the coarse grid cannot represent), and with
    P = I the coarse correction is exact for every delta."""
    A, P, Ac, rng = _spd_case(1)
    b = rng.standard_normal((30, 1))
    e = np.linalg.solve(A, b)
    eb = float(np.sum(e * b))
    for _ in range(5):
        L, _ = mlp.two_grid_energy(rng.standard_normal((30, 1)), b, A, P, Ac)
        assert L + eb >= -1e-12 * eb
    dstar = e - P @ np.linalg.solve(Ac, P.T @ b)
    L, g = mlp.two_grid_energy(dstar, b, A, P, Ac)
    assert abs(L + eb) <= 1e-12 * eb
    assert np.abs(g).max() <= 1e-12 * np.abs(b).max()
    I = np.eye(30)
    for _ in range(3):
        L, _ = mlp.two_grid_energy(rng.standard_normal((30, 1)), b, A, I, A)
        assert abs(L + eb) <= 1e-10 * eb
    # a zero correction leaves exactly the coarse-grid complement of e
    L0, _ = mlp.two_grid_energy(np.zeros((30, 1)), b, A, P, Ac)
    w = e - P @ np.linalg.solve(Ac, P.T @ b)
    assert abs(L0 + eb - float(np.sum(w * (A @ w)))) <= 1e-12 * eb


def test_energy_residual_form_identity():
    """For symmetric A the loss equals -delta.b - delta.r - rc.c with
    r = b - A delta, rc = P^T r, c = Ac^{-1} rc, and the gradient is
    -2 (r - A P c): the form a device evaluates without solving on level 0."""
    A, P, Ac, rng = _spd_case(2)
    b = rng.standard_normal((30, 1))
    delta = rng.standard_normal((30, 1))
    L, g = mlp.two_grid_energy(delta, b, A, P, Ac)
    r = b - A @ delta
    rc = P.T @ r
    c = np.linalg.solve(Ac, rc)
    L2 = -float(np.sum(delta * b)) - float(np.sum(delta * r)) - float(np.sum(rc * c))
    assert abs(L - L2) <= 1e-10 * max(1.0, abs(L))
    assert np.allclose(g, -2.0 * (r - A @ P @ c), rtol=0, atol=1e-10 * np.abs(g).max())


def test_network_energy_gradient_matches_central_differences():
    A, P, Ac, rng = _spd_case(3, n=24)
    d = 2
    W = mlp.init_weights(18, 8, d, 4)
    z = rng.standard_normal((12, 18))
    b = rng.standard_normal(24)
    L, G = mlp.energy_loss_and_grad(W, z, b, A, P, Ac)
    h = 1e-6
    for li in range(3):
        for _ in range(4):
            i, j = rng.integers(W[li].shape[0]), rng.integers(W[li].shape[1])
            Wp = [x.copy() for x in W]
            Wm = [x.copy() for x in W]
            Wp[li][i, j] += h
            Wm[li][i, j] -= h
            fd = (mlp.energy_loss_and_grad(Wp, z, b, A, P, Ac)[0] - mlp.energy_loss_and_grad(Wm, z, b, A, P, Ac)[0]) / (2 * h)
            assert abs(fd - G[li][i, j]) <= 1e-6 * max(1.0, abs(fd))
