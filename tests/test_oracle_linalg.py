"""Oracle pins: dense LU, CSR and block mat-vec, near-nullspaces."""
import itertools

import numpy as np
import pytest

from conftest import system

from oracle import amg, blocks


def _cramer3(A, b):
    det = lambda m: (m[0, 0] * (m[1, 1] * m[2, 2] - m[1, 2] * m[2, 1])
                     - m[0, 1] * (m[1, 0] * m[2, 2] - m[1, 2] * m[2, 0])
                     + m[0, 2] * (m[1, 0] * m[2, 1] - m[1, 1] * m[2, 0]))
    d = det(A)
    x = np.empty(3)
    for i in range(3):
        Ai = A.copy()
        Ai[:, i] = b
        x[i] = det(Ai) / d
    return x


def test_lu_3x3_cramer():
    A = np.array([[1e-3, 2.0, 3.0], [4.0, 5.0, 6.0], [7.0, 8.0, 10.0]])
    b = np.array([1.0, -2.0, 0.5])
    x = amg.lu_solve(amg.lu_factor(A), b)
    assert np.allclose(x, _cramer3(A, b), rtol=1e-13, atol=0)


def test_lu_pivot_ties_take_smallest_row():
    A = np.array([[1.0, 1.0], [-1.0, 2.0]])
    LU, piv = amg.lu_factor(A)
    assert piv[0] == 0  # |1| == |-1|: keep the smaller row index


@pytest.mark.parametrize("n", [1, 7, 60])
def test_lu_known_solution(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    x = rng.standard_normal(n)
    y = amg.lu_solve(amg.lu_factor(A), A @ x)
    assert np.linalg.norm(y - x) <= 1e-13 * np.linalg.norm(x) * n


def test_lu_singular_raises():
    with pytest.raises(ZeroDivisionError):
        amg.lu_factor(np.array([[1.0, 2.0], [2.0, 4.0]]))


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d"])
def test_spmv_unit_columns_and_dense(name):
    s = system(name)
    bs = blocks.BlockSystem(s)
    # dense A_h from the raw CSR arrays with explicit loops
    o = s.offsets
    A = np.zeros((s.N, s.N))
    place = {"M": (0, 0), "C_ms": (0, 1), "C_sm": (1, 0), "S": (1, 1), "C_sf": (1, 2),
             "C_fm": (2, 0), "C_fs": (2, 1), "F": (2, 2)}
    for nm, (bi, bj) in place.items():
        b = s.blocks[nm]
        for r in range(b.nrows):
            for k in range(b.rowptr[r], b.rowptr[r + 1]):
                A[o[bi] + r, o[bj] + b.col[k]] = b.val[k]
    for j in range(0, s.N, 7):
        e = np.zeros(s.N)
        e[j] = 1.0
        assert np.array_equal(bs.matvec(e), A[:, j])
    x = np.random.default_rng(0).standard_normal(s.N)
    assert np.allclose(bs.matvec(x), A @ x, rtol=1e-14, atol=1e-14 * np.abs(A).max() * np.abs(x).max())
    assert np.array_equal(bs.dense(), A)
    Ad = bs.dense(drop_csm=True)
    assert not Ad[o[1]:o[2], o[0]:o[1]].any()


def test_spmv_definition_on_csr():
    rng = np.random.default_rng(5)
    D = rng.standard_normal((9, 6)) * (rng.random((9, 6)) < 0.4)
    D[3] = 0.0  # empty row
    import scipy.sparse as sp
    A = sp.csr_matrix(D)
    x = rng.standard_normal(6)
    y = blocks.spmv(A, x)
    for i in range(9):
        acc = 0.0
        for k in range(A.indptr[i], A.indptr[i + 1]):
            acc += A.data[k] * x[A.indices[k]]
        assert y[i] == acc


def test_rigid_body_modes_are_kernel_of_linear_strain():
    """Rigid motions have zero symmetric gradient: check on a 3D point cloud."""
    rng = np.random.default_rng(1)
    xyz = rng.random((20, 3))
    B = amg.rigid_body_modes(xyz)
    c = xyz - xyz.mean(axis=0)
    for j in range(6):
        u = B[:, j].reshape(-1, 3)
        # fit u = a + W c with W skew: residual must vanish
        X = np.hstack([np.ones((20, 1)), c])
        coef, *_ = np.linalg.lstsq(X, u, rcond=None)
        W = coef[1:].T
        assert np.allclose(u, X @ coef, atol=1e-12)
        assert np.allclose(W + W.T, 0.0, atol=1e-12)
    assert np.linalg.matrix_rank(B) == 6
    B2 = amg.rigid_body_modes(rng.random((5, 2)))
    assert B2.shape == (10, 3) and np.linalg.matrix_rank(B2) == 3
