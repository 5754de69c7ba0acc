"""Pins of the oracle's multigrid: the LU-correction postcondition, transfer
invariants, agreement with direct solves, polynomial reproduction and
fourth-order convergence (CPU only)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.fields import Field
from oracle.multigrid import Hierarchy, MGParams
from paper_2410_05865_amd import inputs


@pytest.fixture(scope="module")
def sphere16_two_level():
    dom, phi = inputs.sphere_workload(16)
    dom.n_min = 8
    return Hierarchy(dom), Field(phi)


def test_lu_correction_zeroes_phi2_residual(sphere32):
    """After SMO-2 the phi_2 rows hold exactly (Sec. 5.3, the residual identity)."""
    H, F = sphere32
    op = H.ops[0]
    rng = np.random.default_rng(0)
    s = rng.standard_normal(op.L.shape[0])
    e = op.smo1(rng.standard_normal(op.L.shape[0]), s, 0.8)
    e = op.smo2(e, s)
    res = s - op.L @ e
    assert np.max(np.abs(res[op.i2])) < 1e-10 * np.max(np.abs(s))
    assert np.max(np.abs(res[op.i1])) > 1e-3


def test_smo1_is_weighted_jacobi_on_phi1(sphere32):
    H, F = sphere32
    op = H.ops[0]
    rng = np.random.default_rng(1)
    s = rng.standard_normal(op.L.shape[0])
    e = rng.standard_normal(op.L.shape[0])
    out = op.smo1(e, s, 0.5)
    # phi_2 untouched, and a phi_1 entry moves by omega * residual / diagonal
    assert np.array_equal(out[op.i2], e[op.i2])
    i = op.i1[len(op.i1) // 2]
    row = op.L[i].toarray().ravel()
    assert out[i] == pytest.approx(e[i] + 0.5 * (s[i] - row @ e) / row[i], rel=1e-13)


def test_transfers_preserve_constants(sphere32):
    H, F = sphere32
    fl, cl = H.levels[0], H.levels[1]
    ones = np.ones(fl.N)
    c = H.restrict(0, ones)
    # coarse cells whose 8 children are all phi_1 receive exactly the constant
    nf, nc = fl.n, cl.n
    g = np.zeros(nf ** 3)
    g[fl.unknowns[fl.phi1_mask()]] = 1.0
    full = (g.reshape(nc, 2, nc, 2, nc, 2).sum(axis=(1, 3, 5)).reshape(-1) == 8)[cl.unknowns]
    assert np.all(c[full] == 1.0)
    assert np.all(c[~full] < 1.0)
    e = H.prolong_add(0, np.zeros(fl.N), np.full(cl.N, 2.5))
    assert np.all(e[fl.phi1_mask()] == 2.5) and np.all(e[~fl.phi1_mask()] == 0.0)


def test_multigrid_matches_sparse_direct_solve(sphere32):
    H, F = sphere32
    lv = H.fine
    r = lv.rhs(F.laplacian_desc(), F)
    x, hist = H.solve(r, MGParams(tol=1e-13))
    xd = spla.splu(lv.L.tocsc()).solve(r)
    assert hist[-1] < 1e-13
    assert np.max(np.abs(x - xd)) < 1e-10 * np.max(np.abs(xd))


def test_multigrid_matches_dense_direct_solve(sphere16_two_level):
    """Brute force on a tiny grid: numpy dense LU of the assembled operator."""
    H, F = sphere16_two_level
    lv = H.fine
    r = lv.rhs(F.laplacian_desc(), F)
    x, hist = H.solve(r, MGParams(tol=1e-13))
    xd = np.linalg.solve(lv.L.toarray(), r)
    assert np.max(np.abs(x - xd)) < 1e-10 * np.max(np.abs(xd))


def test_vcycle_reduction_factor(sphere32):
    H, F = sphere32
    lv = H.fine
    r = lv.rhs(F.laplacian_desc(), F)
    x, hist = H.solve(r, MGParams(tol=1e-10))
    rates = [hist[i + 1] / hist[i] for i in range(2, len(hist) - 1)]
    assert len(hist) < 25
    assert max(rates) < 0.4


def test_polynomial_reproduction():
    """Every row is exact on quartics, so their exact cell averages are the
    discrete solution."""
    dom = inputs.ellipsoid_domain(n=32, seed=7, count=2, axes_range=(0.08, 0.14), h_coarse=1 / 16)
    dom.n_min = 16
    H = Hierarchy(dom)
    P = Field(inputs.poly_field([(4, 0, 0, 1.0), (0, 2, 2, -2.0), (1, 1, 1, 1.0), (0, 0, 0, 1.0),
                                 (2, 0, 1, 0.4)]))
    lv = H.fine
    r = lv.rhs(P.laplacian_desc(), P)
    x, hist = H.solve(r, MGParams(tol=1e-13))
    ex = lv.region_average(P)
    assert np.max(np.abs(x - ex)) < 1e-10 * np.max(np.abs(ex))


def test_fourth_order_convergence(sphere32, sphere16_two_level):
    errs = []
    for H, F in (sphere16_two_level, sphere32):
        lv = H.fine
        r = lv.rhs(F.laplacian_desc(), F)
        x, _ = H.solve(r, MGParams(tol=1e-12))
        errs.append(np.max(np.abs(x - lv.region_average(F))))
    ratio = errs[0] / errs[1]
    assert ratio > 11.0, errs      # fourth order: 16 asymptotically


def _ell32_robin(bc, robin):
    dom = inputs.ellipsoid_domain(n=32, seed=7, count=2, axes_range=(0.08, 0.14), h_coarse=1 / 16)
    dom.n_min = 16
    for ob in dom.obstacles:
        ob.bc = bc
        ob.robin = robin
    return dom


def test_robin_rows_reduce_to_dirichlet_and_neumann():
    """A Robin condition alpha phi + beta dphi/dn with (1, 0) gives the
    Dirichlet rows and with (0, 1) the Neumann rows (same data scaling)."""
    from oracle.discretize import Level
    for robin, plain in (((1.0, 0.0), inputs.DIRICHLET), ((0.0, 1.0), inputs.NEUMANN)):
        a = Level(_ell32_robin(inputs.ROBIN, robin), 32)
        b = Level(_ell32_robin(plain, (1.0, 0.0)), 32)
        assert a.plg.keys() == b.plg.keys()
        for k in a.plg:
            assert list(a.plg[k][0]) == list(b.plg[k][0])
            assert np.max(np.abs(np.asarray(a.plg[k][1]) - np.asarray(b.plg[k][1]))) <= 1e-12 * np.max(
                np.abs(b.plg[k][1]))


def test_polynomial_reproduction_robin():
    """With Robin data on the obstacles every row is still exact on quartics."""
    H = Hierarchy(_ell32_robin(inputs.ROBIN, (1.0, 0.3)))
    P = Field(inputs.poly_field([(4, 0, 0, 1.0), (0, 2, 2, -2.0), (1, 1, 1, 1.0), (0, 0, 0, 1.0),
                                 (2, 0, 1, 0.4)]))
    lv = H.fine
    r = lv.rhs(P.laplacian_desc(), P)
    x, hist = H.solve(r, MGParams(tol=1e-13, max_iter=300))
    ex = lv.region_average(P)
    assert np.max(np.abs(x - ex)) < 1e-10 * np.max(np.abs(ex))


def _sphere_robin_walls(n, robin, bcs):
    dom, phi = inputs.sphere_workload(n)
    dom.n_min = 8 if n == 16 else 16
    dom.wall_bc = bcs
    dom.wall_robin = robin
    return dom, phi


def test_robin_walls_reduce_to_dirichlet_and_neumann():
    """Robin walls with (1, 0) give the Dirichlet walls' operator and
    right-hand side, with (0, 1) the Neumann walls' (same data)."""
    from oracle.discretize import Level
    F = Field(inputs.expcos_field())
    for robin, plain in (((1.0, 0.0), inputs.DIRICHLET), ((0.0, 1.0), inputs.NEUMANN)):
        a = Level(_sphere_robin_walls(16, (robin,) * 6, (inputs.ROBIN,) * 6)[0], 16)
        b = Level(_sphere_robin_walls(16, ((1.0, 0.0),) * 6, (plain,) * 6)[0], 16)
        assert np.array_equal(a.unknowns, b.unknowns) and np.array_equal(a.phi2, b.phi2)
        d = abs(a.L - b.L)
        assert d.max() <= 1e-12 * abs(b.L).max()
        ra, rb = a.rhs(F.laplacian_desc(), F), b.rhs(F.laplacian_desc(), F)
        assert np.max(np.abs(ra - rb)) <= 1e-12 * np.max(np.abs(rb))


def test_polynomial_reproduction_robin_walls():
    """With Robin conditions on four walls every row is exact on quartics, so
    the solve returns their exact cell averages.  (The sphere workload: the
    two-ellipsoid 32^3 domain above has a 16^3 coarse level on which its
    ellipsoids span 1-2 cells, and the plain iteration stalls there already
    with Neumann walls.)"""
    mixed = (inputs.ROBIN, inputs.ROBIN, inputs.DIRICHLET, inputs.ROBIN, inputs.NEUMANN, inputs.ROBIN)
    robin = ((1.0, 0.5), (0.3, 1.0), (1.0, 0.0), (2.0, 0.05), (1.0, 0.0), (0.7, 0.7))
    H = Hierarchy(_sphere_robin_walls(16, robin, mixed)[0])
    P = Field(inputs.poly_field([(4, 0, 0, 1.0), (0, 2, 2, -2.0), (1, 1, 1, 1.0), (0, 0, 0, 1.0),
                                 (2, 0, 1, 0.4)]))
    lv = H.fine
    r = lv.rhs(P.laplacian_desc(), P)
    x, hist = H.solve(r, MGParams(tol=1e-13, max_iter=300))
    ex = lv.region_average(P)
    assert np.max(np.abs(x - ex)) < 1e-10 * np.max(np.abs(ex))
