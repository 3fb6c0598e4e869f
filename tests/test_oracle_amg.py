"""Oracle pins: smoothed-aggregation setup and V-cycle."""
import numpy as np
import pytest
import scipy.sparse as sp

from conftest import system

from oracle import amg, blocks


def lap1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")


def test_aggregation_of_a_chain_by_hand():
    """Tridiagonal chain: every link strong; phase 1 seeds at 0, 3, 6."""
    A = lap1d(7)
    ptr, nbr, sval, _ = amg.strength(A, 1, 0.08)
    agg, nagg = amg.aggregate(7, ptr, nbr, sval)
    assert agg.tolist() == [0, 0, 1, 1, 1, 2, 2] and nagg == 3


def test_aggregation_phase2_and_singletons():
    # chain 0-1-2-3 plus isolated node 4; weak link between 2 and 3
    D = np.array([[2, -1, 0, 0, 0], [-1, 2, -1, 0, 0], [0, -1, 2, -1e-3, 0],
                  [0, 0, -1e-3, 2, 0], [0, 0, 0, 0, 1.0]])
    A = sp.csr_matrix(D)
    ptr, nbr, sval, _ = amg.strength(A, 1, 0.08)
    agg, nagg = amg.aggregate(5, ptr, nbr, sval)
    # phase 1: {0,1}; phase 2: 2 joins via its strongest phase-1 link (1);
    # phase 3: 3 and 4 have no strong links -> singletons
    assert agg.tolist() == [0, 0, 0, 1, 2] and nagg == 3


@pytest.mark.parametrize("n,lo", [(8, 0.999), (50, 0.95)])
def test_spectral_radius_closed_form(n, lo):
    # D^{-1} A of the chain Laplacian has eigenvalues 1 - cos(k pi / (n+1));
    # the power estimate approaches the largest one from below
    A = lap1d(n)
    rho = amg.spectral_radius(A, 1.0 / A.diagonal())
    exact = 1.0 + np.cos(np.pi / (n + 1))
    assert exact * lo <= rho <= exact * (1 + 1e-12)


def test_strength_block_frobenius():
    rng = np.random.default_rng(2)
    D = rng.standard_normal((6, 6))
    A = sp.csr_matrix(D)
    ptr, nbr, sval, (pI, pJ, strong) = amg.strength(A, 2, 0.5)
    for I in range(3):
        for k in range(ptr[I], ptr[I + 1]):
            J = nbr[k]
            blk = D[2 * I:2 * I + 2, 2 * J:2 * J + 2]
            assert np.isclose(sval[k], np.sum(blk ** 2), rtol=1e-14)
            aII = np.sqrt(np.sum(D[2 * I:2 * I + 2, 2 * I:2 * I + 2] ** 2))
            aJJ = np.sqrt(np.sum(D[2 * J:2 * J + 2, 2 * J:2 * J + 2] ** 2))
            assert np.sqrt(sval[k]) >= 0.5 * np.sqrt(aII * aJJ) * (1 - 1e-12)


def _hierarchies(name, max_coarse):
    s = system(name)
    bs = blocks.BlockSystem(s)
    from oracle import precond
    return bs, precond.build_hierarchies(bs, max_coarse=max_coarse)


@pytest.mark.parametrize("hname", ["H_M", "H_SIG", "H_MS", "H_A", "H_P"])
def test_tentative_reproduces_nullspace_and_galerkin(hname):
    bs, H = _hierarchies("c1", 40)
    h = H[hname]
    assert h.nlevels >= 2
    for l, lev in enumerate(h.levels[:-1]):
        # aggregates partition the nodes
        nn = lev.A.shape[0] // lev.block
        assert lev.aggregates.shape == (nn,) and lev.aggregates.min() >= 0
        Pt, Bc = amg.tentative(lev.aggregates, lev.aggregates.max() + 1, lev.block, lev.B)
        # P_tent has orthonormal columns (or zero ones) and P_tent B_{l+1} = B_l
        G = (Pt.T @ Pt).toarray()
        nz = np.diag(G) > 0
        assert np.allclose(G[np.ix_(nz, nz)], np.eye(nz.sum()), atol=1e-12)
        full_rank = np.all(np.abs(np.diag(Bc.reshape(-1, Bc.shape[1], Bc.shape[1])[0])) > 0)
        recon = Pt @ Bc
        if full_rank and nz.all():
            assert np.allclose(recon, lev.B, atol=1e-12 * np.abs(lev.B).max())
        # Galerkin product against dense
        Ad, Pd = lev.A.toarray(), lev.P.toarray()
        Ac = Pd.T @ Ad @ Pd
        nxt = h.levels[l + 1].A.toarray()
        empty = ~np.any(Ac != 0, axis=1)
        Ac[empty, empty] = 1.0
        assert np.allclose(nxt, Ac, rtol=0, atol=1e-12 * np.abs(Ac).max())
        assert np.array_equal(lev.R.toarray(), Pd.T)


@pytest.mark.parametrize("hname", ["H_M", "H_MS", "H_P"])
def test_vcycle_symmetric_and_contracting(hname):
    """Symmetric A: V(1,1) Jacobi with R = P^T is a symmetric operator and
    ||I - V A||_A < 1."""
    bs, H = _hierarchies("c1", 40)
    h = H[hname]
    A = h.levels[0].A.toarray()
    assert np.abs(A - A.T).max() <= 1e-10 * np.abs(A).max()
    n = A.shape[0]
    V = np.column_stack([amg.vcycle(h, e) for e in np.eye(n)])
    assert np.abs(V - V.T).max() <= 1e-10 * np.abs(V).max()
    E = np.eye(n) - V @ A
    Lc = np.linalg.cholesky(A)
    Ea = Lc.T @ E @ np.linalg.inv(Lc.T)
    assert np.linalg.norm(Ea, 2) < 1.0


def test_vcycle_coarsest_is_exact():
    A = lap1d(30)
    h = amg.setup(A, 1, amg.constant_modes(30), max_coarse=500)
    assert h.nlevels == 1
    b = np.arange(30.0)
    assert np.allclose(A @ amg.vcycle(h, b), b, rtol=1e-12)


@pytest.mark.parametrize("degree", [1, 2, 3, 5])
def test_chebyshev_error_is_the_scaled_chebyshev_polynomial(degree):
    """With A = diag(lambda), D = I and b = 0 the iterate is the error, and
    after k steps it equals T_k((theta - lambda)/delta) / T_k(theta/delta)
    times the initial error (T_k evaluated by numpy's Chebyshev series)."""
    from numpy.polynomial import chebyshev as C
    lam = np.linspace(0.01, 2.0, 40)
    A = sp.diags(lam).tocsr()
    x0 = 1.0 + np.arange(40) / 40.0
    lmax, ratio = 2.2, 30.0
    x = amg.chebyshev(A, np.ones(40), np.zeros(40), x0, degree, lmax, ratio)
    lmin = lmax / ratio
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    Tk = np.zeros(degree + 1)
    Tk[degree] = 1.0
    ref = C.chebval((theta - lam) / delta, Tk) / C.chebval(theta / delta, Tk) * x0
    assert np.allclose(x, ref, rtol=0, atol=1e-13 * np.abs(x0).max())
    # inside the interval the error is bounded by 1 / T_k(theta / delta)
    inside = lam >= lmin
    assert np.all(np.abs(x[inside] / x0[inside]) <= 1.0 / C.chebval(theta / delta, Tk) * (1 + 1e-12))


def test_chebyshev_degree_one_is_damped_jacobi():
    A = lap1d(20)
    dinv = 1.0 / A.diagonal()
    b = np.sin(np.arange(20.0))
    lmax = 2.2
    theta = 0.5 * (lmax + lmax / amg.CHEB_RATIO)
    assert np.allclose(amg.chebyshev(A, dinv, b, np.zeros(20), 1, lmax), dinv * b / theta, rtol=1e-15)


@pytest.mark.parametrize("hname", ["H_M", "H_MS", "H_P"])
def test_chebyshev_vcycle_symmetric_and_contracting(hname):
    """The same polynomial before and after the coarse correction keeps the
    cycle symmetric for symmetric A; it contracts in the A-norm."""
    bs, H = _hierarchies("c1", 40)
    h = H[hname]
    A = h.levels[0].A.toarray()
    n = A.shape[0]
    V = np.column_stack([amg.vcycle_cheb(h, e, 3) for e in np.eye(n)])
    assert np.abs(V - V.T).max() <= 1e-10 * np.abs(V).max()
    E = np.eye(n) - V @ A
    Lc = np.linalg.cholesky(A)
    Ea = Lc.T @ E @ np.linalg.inv(Lc.T)
    assert np.linalg.norm(Ea, 2) < 1.0
