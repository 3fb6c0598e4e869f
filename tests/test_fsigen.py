"""Synthetic input generator: Jacobian consistency and block structure.

These pin the inputs both sides read: the assembled blocks are the exact
derivative of the generator's residual (frozen fields held fixed; the
FSI-related derivative theorem of Section 3.3 enters through it), and the
block structure is the one Section 3.4 and Section 4.3 rely on.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from conftest import system

import fsigen


def _csr(b):
    return sp.csr_matrix((b.val, b.col, b.rowptr), shape=(b.nrows, b.ncols))


def _dense_ah(s):
    """A_h placed block by block with explicit loops (independent of the oracle)."""
    o = s.offsets
    A = np.zeros((s.N, s.N))
    place = {"M": (0, 0), "C_ms": (0, 1), "C_sm": (1, 0), "S": (1, 1), "C_sf": (1, 2),
             "C_fm": (2, 0), "C_fs": (2, 1), "F": (2, 2)}
    for name, (bi, bj) in place.items():
        b = s.blocks[name]
        for r in range(b.nrows):
            for k in range(b.rowptr[r], b.rowptr[r + 1]):
                A[o[bi] + r, o[bj] + b.col[k]] += b.val[k]
    return A


@pytest.mark.parametrize("name,N,nnz", [("tiny2d", 104, None), ("tiny3d", 449, None),
                                        ("c1", 4093, 170470)])
def test_sizes(name, N, nnz):
    s = system(name)
    assert s.N == N
    assert s.n_s == 2 * s.n_vs and s.n_f == s.n_vf + s.n_p
    if nnz is not None:
        assert s.nnz == nnz
    for b in s.blocks.values():
        assert b.rowptr[0] == 0 and b.rowptr[-1] == b.nnz
        assert np.all(np.diff(b.rowptr) >= 0)
        for r in range(b.nrows):
            cols = b.col[b.rowptr[r]:b.rowptr[r + 1]]
            assert np.all(np.diff(cols) > 0)
        assert b.nnz == 0 or (b.col.min() >= 0 and b.col.max() < b.ncols)


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "c1", "tiny2d_unit"])
def test_jacobian_matches_central_differences(name):
    s = system(name, seed=3)
    A = _dense_ah(s) if s.N < 1000 else None
    rng = np.random.default_rng(11)
    d = rng.standard_normal(s.N)
    eps = 1e-6
    fd = (fsigen.residual(name, 3, d, eps) - fsigen.residual(name, 3, d, -eps)) / (2 * eps)
    if A is not None:
        Jd = A @ d
    else:
        o = s.offsets
        B = {k: _csr(v) for k, v in s.blocks.items()}
        xm, xs, xf = d[:o[1]], d[o[1]:o[2]], d[o[2]:]
        Jd = np.concatenate([B["M"] @ xm + B["C_ms"] @ xs,
                             B["C_sm"] @ xm + B["S"] @ xs + B["C_sf"] @ xf,
                             B["C_fm"] @ xm + B["C_fs"] @ xs + B["F"] @ xf])
    assert np.linalg.norm(fd - Jd) <= 1e-6 * np.linalg.norm(Jd)


def test_rhs_is_negative_residual():
    s = system("tiny3d")
    R0 = fsigen.residual("tiny3d", 0, np.zeros(s.N), 0.0)
    assert np.array_equal(s.b, -R0)


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "c1"])
def test_block_structure(name):
    s = system(name)
    nvs, nvf = s.n_vs, s.n_vf
    S = _csr(s.blocks["S"]).toarray() if s.n_s < 3000 else None
    Sm = _csr(s.blocks["S"])
    S_uv = Sm[nvs:, :nvs].toarray()
    S_uu = Sm[nvs:, nvs:].toarray()
    # equal-order mass matrices: S_uv = -dt theta S_uu (Section 4.3)
    assert np.abs(S_uv + s.dt_theta * S_uu).max() <= 1e-12 * np.abs(S_uu).max()
    # S_uu is a mass matrix (SPD), component-diagonal
    np.linalg.cholesky(S_uu)
    assert np.allclose(S_uu, S_uu.T, rtol=0, atol=1e-15 * np.abs(S_uu).max())
    # frozen mesh block: symmetric positive definite and L (x) I_d
    M = _csr(s.blocks["M"]).toarray()
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    np.linalg.cholesky(M)
    d = s.dim
    L = M[0::d, 0::d]
    assert np.array_equal(M, np.kron(L, np.eye(d)))
    # G = -D^T (both J F^{-T} : grad forms with the same quadrature)
    F = _csr(s.blocks["F"]).toarray()
    G, D, Fpp = F[:nvf, nvf:], F[nvf:, :nvf], F[nvf:, nvf:]
    assert np.abs(G + D.T).max() <= 1e-13 * np.abs(G).max()
    assert not Fpp.any()
    del S


@pytest.mark.parametrize("name", ["tiny3d", "c1"])
def test_solid_only_schur_block_spd(name):
    """On pure-solid nodes Sigma_s = rho_s M + dt^2 theta^2 K (STVK tangent): SPD."""
    s = system(name)
    nvs, d = s.n_vs, s.dim
    Sm = _csr(s.blocks["S"])
    Sig = (Sm[:nvs, :nvs] + s.dt_theta * Sm[:nvs, nvs:]).toarray()
    o = s.offsets
    nodes = s.dof_node[o[1]:o[1] + nvs]
    interface = (s.node_flags[nodes] & 3) == 3
    keep = ~interface
    Sub = Sig[np.ix_(keep, keep)]
    assert np.abs(Sub - Sub.T).max() <= 1e-10 * np.abs(Sub).max()
    np.linalg.cholesky(Sub)


def test_laplacian_rows_sum_to_zero_away_from_boundaries():
    s = system("c1")
    M = _csr(s.blocks["M"])
    Cms = _csr(s.blocks["C_ms"])
    d = s.dim
    L = M[0::d, 0::d]
    rs = np.asarray(L.sum(axis=1)).ravel()
    # rows whose node has no Dirichlet or interface neighbour: partition of unity
    coupled = np.asarray(abs(Cms[0::d]).sum(axis=1)).ravel() > 0
    ijk = s.node_ijk[s.dof_node[0:s.n_m:d]]
    nx, ny = 2 * s.cfg.cells[0], 2 * s.cfg.cells[1]
    inner = (ijk[:, 0] > 2) & (ijk[:, 0] < nx - 2) & (ijk[:, 1] > 2) & (ijk[:, 1] < ny - 2) & ~coupled
    assert inner.sum() > 100
    assert np.abs(rs[inner]).max() <= 1e-12 * np.abs(L.diagonal()).max()


def test_seed_and_phase_change_values_not_structure():
    a, b = system("c1", seed=0), system("c1", seed=1)
    c = system("c1", seed=0, t_phase=0.7)
    for k in a.blocks:
        assert np.array_equal(a.blocks[k].rowptr, b.blocks[k].rowptr)
    assert not np.array_equal(a.blocks["C_fm"].val, b.blocks["C_fm"].val)
    assert not np.array_equal(a.b, c.b)
    assert 0.8 < a.j_range[0] <= a.j_range[1] < 1.2
