"""The AMG setup's sparse products on the device.

The library forms the setup products C = A B on the GPU: one wavefront per
row, the row's distinct columns in an LDS hash set (1024 or 4096 of them,
longer rows on the host), then the values added in the host's order of k.
The result must be the host product bit for bit, so that the hierarchy does
not depend on where it was built.  Checked two ways:

* the hierarchies the library builds (device products) equal, array for
  array, the ones the host-only setup (a g++ build of the same setup code
  with host products) builds from the library's own level-0 operator: level
  matrices, prolongators, aggregates and Jacobi weights;
* an imported hierarchy with one aggregate of 5,000 nodes and one of 1,500,
  whose rows of R A exceed the 4096- and the 1024-column tables, cycles as
  the oracle's V-cycle on the same hierarchy does (the level sweeps' products
  A P and R A then take all three paths).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from conftest import system

import test_sa_setup_cpu as sa

pytestmark = pytest.mark.gpu

driver = sa.driver  # the host-only setup build (module fixture)


def _csr(t):
    nr, nc, rp, ci, vv = t
    return sp.csr_matrix((vv, ci, rp), shape=(nr, nc))


def _modes(hname, n, d):
    from oracle import amg
    if hname == "H_A":
        return d, amg.translation_modes(n // d, d)
    return 1, amg.constant_modes(n)


@pytest.mark.parametrize("name", ["c2", "m3"])
def test_device_products_build_the_host_hierarchy_bitwise(driver, name):
    from paper_1801_05648_amd import FsiSolver
    sysm = system(name)
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64", max_coarse=40, strength0=0.08)
    for hname in ("H_M", "H_MS", "H_A", "H_P"):
        n, nnz, om = s.hierarchy_info(hname)
        nl = len(n)
        A0 = _csr(s.get_level(hname, 0, "A"))
        block, B = _modes(hname, A0.shape[0], sysm.dim)
        host = sa._run(driver, A0, block, B, 0.08, 40)
        assert len(host) == nl, (hname, len(host), nl)
        for l in range(nl):
            _, _, rp, ci, vv = s.get_level(hname, l, "A")
            H = host[l]["A"]
            assert np.array_equal(rp, H.indptr) and np.array_equal(ci, H.indices), (hname, l, "A pattern")
            assert np.array_equal(vv, H.data), (hname, l, "A values")
            if l + 1 == nl:
                break
            _, _, rp, ci, vv = s.get_level(hname, l, "P")
            H = host[l]["P"]
            assert np.array_equal(rp, H.indptr) and np.array_equal(ci, H.indices), (hname, l, "P pattern")
            assert np.array_equal(vv, H.data), (hname, l, "P values")
            assert np.array_equal(s.get_aggregates(hname, l), host[l]["agg"]), (hname, l, "aggregates")
            assert om[l] == host[l]["omega"], (hname, l, om[l], host[l]["omega"])
        print(f"{name} {hname}: {nl} levels, nnz {list(nnz)} bitwise equal")
    s.close()


def test_long_product_rows_cycle_as_the_oracle():
    from oracle import amg, blocks, precond
    from paper_1801_05648_amd import FsiSolver
    sysm = system("c2")
    bs = blocks.BlockSystem(sysm)
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond("f64")
    L = _csr(s.get_level("H_M", 0, "A"))
    n = L.shape[0]
    # aggregates: nodes [0, 5000), [5000, 6500), then runs of 32 nodes
    agg = np.empty(n, np.int64)
    agg[:5000] = 0
    agg[5000:6500] = 1
    agg[6500:] = 2 + (np.arange(n - 6500) // 32)
    nc = int(agg.max()) + 1
    size = np.bincount(agg, minlength=nc).astype(np.float64)
    P = sp.csr_matrix((1.0 / np.sqrt(size[agg]), (np.arange(n), agg)), shape=(n, nc))
    R = P.T.tocsr()
    R.sort_indices()
    Ac = (R @ L @ P).tocsr()
    Ac.sort_indices()
    dinv = 1.0 / L.diagonal()
    omega = (4.0 / 3.0) / amg.spectral_radius(L, dinv)
    # distinct columns of the rows of R A (structural: no cancellation) exceed
    # the tables for aggregates 0 and 1
    RA = (abs(R) @ abs(L)).tocsr()
    lens = np.diff(RA.indptr)
    assert lens[0] > 4096 and 1024 < lens[1] <= 4096 and lens[2:].max() <= 1024, lens[:3]
    tup = lambda m: (m.shape[0], m.shape[1], m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data)
    s.set_hierarchy("H_M", [tup(L), tup(Ac)], [tup(P)], [tup(R)], [omega])
    h = amg.Hierarchy([amg.Level(A=L, P=P, R=R, dinv=dinv, omega=omega), amg.Level(A=Ac)],
                      amg.lu_factor(Ac.toarray()))
    rng = np.random.default_rng(5)
    b = rng.standard_normal(bs.n_m)
    ref = precond.mesh_solve(bs, lambda v: amg.vcycle(h, v), b)
    x = s.vcycle("H_M", torch.from_numpy(b).to("cuda:0")).cpu().numpy()
    rel = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    print(f"c2 H_M, aggregates of 5000 and 1500 nodes: V-cycle {rel:.2e} to the oracle")
    assert rel <= 1e-12, rel
    s.close()
