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


# ------------------------------------------------------------------------
# Filtered matrix and prolongator smoothing (the SA setup's steps 5-6).  The
# references below are written from the definitions, by explicit loops over
# dense node blocks, and the checks are invariants that a dropped term, a
# lump into the wrong diagonal or the wrong scaling would break.

def _strong_pairs_by_blocks(Ad, b, eps):
    """Strong node pairs from the definition: Frobenius norm of the (I, J)
    node block at least eps * sqrt(norm(I, I) * norm(J, J)), I != J."""
    nn = Ad.shape[0] // b
    F = np.array([[np.sqrt(np.sum(Ad[I * b:(I + 1) * b, J * b:(J + 1) * b] ** 2)) for J in range(nn)]
                  for I in range(nn)])
    return {(I, J) for I in range(nn) for J in range(nn)
            if I != J and F[I, J] > 0 and F[I, J] >= eps * np.sqrt(F[I, I] * F[J, J])}


def _filtered_by_loops(A, b, strong):
    """A^F by loops over the stored entries: keep same-node and strong-pair
    entries, add every other entry of the row to the row's diagonal."""
    n = A.shape[0]
    AF = np.zeros((n, n))
    for i in range(n):
        lump = 0.0
        for k in range(A.indptr[i], A.indptr[i + 1]):
            j = int(A.indices[k])
            if i // b == j // b or (i // b, j // b) in strong:
                AF[i, j] += A.data[k]
            else:
                lump += A.data[k]
        AF[i, i] += lump
    return AF


def _integer_test_matrix(nn=8, b=2, seed=3):
    """Nonsymmetric integer-valued matrix in node blocks of b: dominant
    diagonal blocks, strong (|entries| ~ 20) and weak (|entries| <= 2)
    off-node blocks, so every row sum is exact in FP64."""
    rng = np.random.default_rng(seed)
    n = nn * b
    Ad = np.zeros((n, n))
    for I in range(nn):
        Ad[I * b:(I + 1) * b, I * b:(I + 1) * b] = rng.integers(-5, 6, (b, b))
        for a in range(b):
            Ad[I * b + a, I * b + a] = 200 + rng.integers(0, 20)
        for J in range(nn):
            if J == I:
                continue
            kind = rng.integers(0, 3)  # 0 none, 1 weak, 2 strong
            if kind == 1:
                Ad[I * b:(I + 1) * b, J * b:(J + 1) * b] = rng.integers(-2, 1, (b, b))
            elif kind == 2:
                Ad[I * b:(I + 1) * b, J * b:(J + 1) * b] = rng.integers(-25, -15, (b, b))
    return Ad


def test_filtered_matrix_keeps_row_sums_and_drops_weak_pairs():
    b, eps = 2, 0.08
    Ad = _integer_test_matrix(b=b)
    A = sp.csr_matrix(Ad)
    A.sort_indices()
    _, _, _, pairs = amg.strength(A, b, eps)
    strong = _strong_pairs_by_blocks(Ad, b, eps)
    assert strong and len(strong) < np.count_nonzero(
        [np.any(Ad[I * b:(I + 1) * b, J * b:(J + 1) * b]) for I in range(8) for J in range(8) if I != J])
    AF = amg.filtered(A, b, pairs).toarray()
    ref = _filtered_by_loops(A, b, strong)
    assert np.array_equal(AF, ref)
    # integer entries: lumping keeps every row sum exactly
    assert np.array_equal(AF.sum(axis=1), Ad.sum(axis=1))
    # weak off-node blocks are gone, strong and same-node ones untouched
    # except the diagonal
    nn = 8
    for I in range(nn):
        for J in range(nn):
            blkF = AF[I * b:(I + 1) * b, J * b:(J + 1) * b]
            blkA = Ad[I * b:(I + 1) * b, J * b:(J + 1) * b]
            if I == J:
                off = ~np.eye(b, dtype=bool)
                assert np.array_equal(blkF[off], blkA[off])
            elif (I, J) in strong:
                assert np.array_equal(blkF, blkA)
            else:
                assert not np.any(blkF)


def _weighted_graph_laplacian(n=24, seed=5):
    """Zero-row-sum nonsymmetric M-matrix: a chain with integer weights, a few
    long-range strong links and many weak (weight 1e-3 x) ones."""
    rng = np.random.default_rng(seed)
    W = np.zeros((n, n))
    for i in range(n - 1):
        W[i, i + 1] = rng.integers(5, 10)
        W[i + 1, i] = rng.integers(5, 10)
    for _ in range(2 * n):
        i, j = rng.integers(0, n, 2)
        if abs(i - j) > 1:
            W[i, j] = 2.0 ** -10 * rng.integers(1, 4)  # weak, exact binary fraction
    for _ in range(3):
        i, j = rng.integers(0, n, 2)
        if abs(i - j) > 1:
            W[i, j] = rng.integers(5, 10)
    return np.diag(W.sum(axis=1)) - W


def test_smoothed_prolongator_reproduces_constants_for_zero_row_sums():
    """With zero row sums and the constant near-nullspace, A^F (lumped) also
    has zero row sums, so (I - omega D_F^{-1} A^F) leaves B unchanged and the
    smoothed P still reproduces it: P B_c = B.  Dropping weak entries without
    lumping breaks this."""
    Ad = _weighted_graph_laplacian()
    n = Ad.shape[0]
    A = sp.csr_matrix(Ad)
    h = amg.setup(A, 1, amg.constant_modes(n), max_coarse=4)
    assert h.nlevels >= 2
    lev = h.levels[0]
    _, Bc = amg.tentative(lev.aggregates, lev.aggregates.max() + 1, 1, lev.B)
    assert np.allclose(lev.P @ Bc, np.ones((n, 1)), rtol=0, atol=1e-14)
    # the weak links were really filtered (not every entry is strong)
    strong = _strong_pairs_by_blocks(Ad, 1, amg.EPS0)
    assert len(strong) < np.count_nonzero(Ad - np.diag(np.diag(Ad)))


@pytest.mark.parametrize("b,seed", [(1, 5), (2, 3)])
def test_smoothed_prolongator_is_the_damped_filtered_jacobi_step(b, seed):
    """P = P_tent - omega diag(A^F)^{-1} A^F P_tent with A^F by explicit loops
    and P_tent from the (separately pinned) aggregate QR; omega from the
    (separately pinned) power estimate of rho(D^{-1} A)."""
    Ad = _weighted_graph_laplacian(seed=seed) if b == 1 else _integer_test_matrix(b=b, seed=seed)
    n = Ad.shape[0]
    A = sp.csr_matrix(Ad)
    B = amg.constant_modes(n) if b == 1 else amg.translation_modes(n // b, b)
    h = amg.setup(A, b, B, max_coarse=2)
    assert h.nlevels >= 2
    lev = h.levels[0]
    assert np.isclose(lev.omega, (4.0 / 3.0) / amg.spectral_radius(A, 1.0 / np.diag(Ad)), rtol=1e-15)
    Pt, _ = amg.tentative(lev.aggregates, lev.aggregates.max() + 1, b, B)
    AF = _filtered_by_loops(A, b, _strong_pairs_by_blocks(Ad, b, amg.EPS0))
    dF = np.diag(AF)
    # the lumped diagonal differs from A's somewhere: diag(A) would be wrong
    assert np.any(dF != np.diag(Ad))
    ref = Pt.toarray() - (lev.omega / dF)[:, None] * (AF @ Pt.toarray())
    assert np.allclose(lev.P.toarray(), ref, rtol=0, atol=1e-14 * np.abs(ref).max())


def test_smoothed_prolongator_of_the_chain_closed_form():
    """Chain Laplacian, all links strong, aggregates {0,1}, {2,3,4}, {5,6}:
    the middle column of the smoothed prolongator is the textbook
    (omega/2, 1 - omega/2, 1, 1 - omega/2, omega/2) / sqrt(3) pattern."""
    A = lap1d(7)
    h = amg.setup(A, 1, amg.constant_modes(7), max_coarse=2)
    lev = h.levels[0]
    assert lev.aggregates.tolist() == [0, 0, 1, 1, 1, 2, 2]
    w = lev.omega
    col = lev.P.toarray()[:, 1]
    ref = np.array([0.0, w / 2, 1 - w / 2, 1.0, 1 - w / 2, w / 2, 0.0]) / np.sqrt(3.0)
    assert np.allclose(col, ref, rtol=0, atol=1e-15)


def test_tentative_rank_deficient_aggregate():
    """Rigid-body modes on single-node aggregates in 2D: translations span the
    node's two dofs, so the rotation column is dependent (r_33 = 0).  Its P_tent
    column is zero, its coarse row of B_c is zero, P_tent B_c = B still holds
    and the Galerkin coarse matrix gets the unit diagonal there."""
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.5]])
    B = amg.rigid_body_modes(xy)
    agg = np.array([0, 1, 2])
    Pt, Bc = amg.tentative(agg, 3, 2, B)
    P = Pt.toarray()
    assert P.shape == (6, 9)
    for a in range(3):
        assert not np.any(P[:, 3 * a + 2])                   # rotation column zeroed
        assert not np.any(Bc[3 * a + 2, :])                  # and its coarse row
        Q = P[:, 3 * a:3 * a + 2]
        assert np.allclose(Q.T @ Q, np.eye(2), atol=1e-15)  # the rest orthonormal
    assert np.allclose(P @ Bc, B, rtol=0, atol=1e-14)
    # a two-node aggregate in 2D spans the rotation: full rank there
    Pt2, Bc2 = amg.tentative(np.array([0, 0, 1]), 2, 2, B)
    assert np.all(np.abs(np.diag(Bc2[:3, :])) > 0)
    assert not np.any(Pt2.toarray()[:, 5])
    assert np.allclose(Pt2 @ Bc2, B, rtol=0, atol=1e-14)


def test_setup_with_rank_deficient_aggregates_gets_unit_coarse_diagonal():
    """An elasticity-like vector operator whose coarse aggregates are single
    nodes in places: the empty coarse rows of the zeroed columns get 1."""
    # 2D, nodes on a line: rotation is independent on 2+-node aggregates only
    nn, b = 13, 2
    L1 = lap1d(nn).toarray()
    # the last node only weakly coupled: it ends up a singleton aggregate
    L1[nn - 2, nn - 1] = L1[nn - 1, nn - 2] = -1e-3
    L1[nn - 1, nn - 1] = 1.0
    Ad = np.kron(L1, np.eye(b))
    xy = np.column_stack([np.arange(nn, dtype=float), np.zeros(nn)])
    A = sp.csr_matrix(Ad)
    h = amg.setup(A, b, amg.rigid_body_modes(xy), max_coarse=2)
    assert h.nlevels >= 2
    lev = h.levels[0]
    assert lev.aggregates[-1] not in lev.aggregates[:-1]
    Pt, Bc = amg.tentative(lev.aggregates, lev.aggregates.max() + 1, b, lev.B)
    zero_cols = np.nonzero(~np.any(Pt.toarray() != 0, axis=0))[0]
    assert zero_cols.size >= 1
    Ac = h.levels[1].A.toarray()
    for c in zero_cols:
        assert Ac[c, c] == 1.0 and np.count_nonzero(Ac[c]) == 1 and np.count_nonzero(Ac[:, c]) == 1


def test_zero_filtered_diagonal_is_an_error():
    """A row whose weak entries cancel its diagonal under lumping leaves the
    smoothing step undefined: the setup raises instead of producing Inf."""
    Ad = lap1d(6).toarray() * 10.0
    # node 5: diagonal 1, weak link -1 to node 0 (lumped: 1 - 1 = 0)
    Ad[5, :] = 0.0
    Ad[5, 5] = 1.0
    Ad[5, 0] = -1.0 * 0.05  # weak: 0.05 < 0.08 * sqrt(20 * 1)
    Ad[5, 5] = 0.05
    Ad[4, 5] = -1e-3
    A = sp.csr_matrix(Ad)
    with pytest.raises(ZeroDivisionError, match="filtered"):
        amg.setup(A, 1, amg.constant_modes(6), max_coarse=2)
