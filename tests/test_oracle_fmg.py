"""Pins of the oracle's full multigrid (Sec. 5, algorithm FMG): its two
transfers against closed forms, the limit of many V-cycles against a sparse
direct solve, and the theorem's claim that a few V-cycles per level reach the
discretization error (CPU only)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.fields import Field
from oracle.multigrid import Hierarchy, MGParams
from paper_2410_05865_amd import inputs


def _centres(lv, cells):
    n = lv.n
    i, j, k = cells % n, (cells // n) % n, cells // (n * n)
    return (i + 0.5) / n, (j + 0.5) / n, (k + 0.5) / n


def test_fmg_restrict_constant(sphere32):
    """2^-3 of the sum over 8 children: a constant right-hand side gives the
    constant on every coarse cell whose 8 children all carry an unknown, and
    a value in [0, c] elsewhere."""
    H, _ = sphere32
    fl, cl = H.levels[0], H.levels[1]
    sc = H.fmg_restrict(0, np.full(fl.N, 2.5))
    has = np.zeros(fl.n ** 3, dtype=bool)
    has[fl.unknowns] = True
    nc = cl.n
    full = has.reshape(nc, 2, nc, 2, nc, 2).all(axis=(1, 3, 5)).reshape(-1)[cl.unknowns]
    assert full.sum() > 0.5 * cl.N
    assert np.all(sc[full] == 2.5)
    assert np.all((sc >= 0) & (sc <= 2.5))


def test_fmg_prolong_constants_and_linears(sphere32):
    """Renormalised trilinear weights: constants are reproduced at every fine
    unknown; a linear function of the cell centres is reproduced exactly where
    all 8 surrounding coarse cells lie in the box and carry an unknown."""
    H, _ = sphere32
    fl, cl = H.levels[0], H.levels[1]
    assert np.allclose(H.fmg_prolong(0, np.full(cl.N, -1.25)), -1.25, rtol=0, atol=1e-15)
    lin = lambda x, y, z: 0.3 + 1.7 * x - 0.9 * y + 2.2 * z
    xc, yc, zc = _centres(cl, cl.unknowns)
    out = H.fmg_prolong(0, lin(xc, yc, zc))
    xf, yf, zf = _centres(fl, fl.unknowns)
    has = np.zeros(cl.n ** 3, dtype=bool)
    has[cl.unknowns] = True
    nf, nc = fl.n, cl.n
    inner = []
    for p in fl.unknowns:
        ok = True
        for i in (p % nf, (p // nf) % nf, p // (nf * nf)):
            lo = i // 2 - 1 if i % 2 == 0 else i // 2
            ok &= 0 <= lo and lo + 1 < nc
        if ok:
            i, j, k = p % nf, (p // nf) % nf, p // (nf * nf)
            los = [(x // 2 - 1 if x % 2 == 0 else x // 2) for x in (i, j, k)]
            ok = all(has[(los[0] + a) + nc * ((los[1] + b) + nc * (los[2] + c))]
                     for a in (0, 1) for b in (0, 1) for c in (0, 1))
        inner.append(ok)
    inner = np.array(inner)
    assert inner.sum() > 0.5 * fl.N
    ref = lin(xf, yf, zf)
    assert np.max(np.abs(out[inner] - ref[inner])) < 1e-13


def test_fmg_many_cycles_is_the_direct_solve(sphere32):
    H, F = sphere32
    lv = H.fine
    r = lv.rhs(F.laplacian_desc(), F)
    x = H.fmg(r, cycles=30)
    xd = spla.splu(H.ops[0].L.tocsc()).solve(r)
    assert np.max(np.abs(x - xd)) < 1e-10 * np.max(np.abs(xd))


def test_fmg_reaches_discretization_error(sphere32):
    """The FMG theorem: a fixed number of V-cycles per level brings the
    algebraic error to the discretization error.  With the trilinear
    interpolation (second order, where the theorem assumes order p = 4) each
    extra cycle per level cuts the algebraic error by more than 5x, and six
    cycles leave the error against the exact cell averages within 10% of the
    converged discrete solution's."""
    H, F = sphere32
    lv = H.fine
    r = lv.rhs(F.laplacian_desc(), F)
    ex = lv.region_average(F)
    x_conv, _ = H.solve(r, MGParams(tol=1e-12))
    e_conv = np.max(np.abs(x_conv - ex))
    alg = [np.max(np.abs(H.fmg(r, cycles=c) - x_conv)) for c in (1, 2, 3)]
    assert alg[1] < 0.2 * alg[0] and alg[2] < 0.2 * alg[1], alg
    e6 = np.max(np.abs(H.fmg(r, cycles=6) - ex))
    print(f"FMG algebraic errors {alg}, FMG(6) error {e6:.3e}, converged error {e_conv:.3e}")
    assert e6 < 1.1 * e_conv


def test_fmg_with_level_rhs_on_boundary_data():
    """With non-zero boundary data (ellipsoids, Neumann on two walls) the
    restricted right-hand side is not a discretisation of the same problem on
    the coarse level (its boundary terms carry the fine h), and FMG from it
    stays far from the solution; from each level's own right-hand side FMG(2)
    is 50x closer and leaves a residual below 1e-4."""
    ell = inputs.ellipsoid_domain(n=32, seed=7, count=2, axes_range=(0.08, 0.14), h_coarse=1 / 16)
    ell.wall_bc = (0, 1, 0, 0, 1, 0)
    ell.n_min = 16
    H = Hierarchy(ell)
    F = Field(inputs.expcos_field())
    lv = H.fine
    r = lv.rhs(F.laplacian_desc(), F)
    ex = lv.region_average(F)
    cr = [lm.rhs(F.laplacian_desc(), F) for lm in H.levels[1:]]
    x_r = H.fmg(r, 2)
    x_l = H.fmg(r, 2, coarse_rhs=cr)
    e_r, e_l = np.max(np.abs(x_r - ex)), np.max(np.abs(x_l - ex))
    res_l = np.max(np.abs(r - H.ops[0].L @ x_l)) / np.max(np.abs(r))
    print(f"FMG(2) error: restricted rhs {e_r:.3e}, per-level rhs {e_l:.3e}; residual {res_l:.2e}")
    assert e_l < e_r / 50 and res_l < 1e-4
