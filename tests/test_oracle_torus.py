"""Pins of the oracle's polynomial level sets (the torus of the paper's
Problem 2, Sec. 6) against what geometry and algebra fix independently of it:

  * the torus quartic equals the product form ((rho-R)^2 + z^2 - r^2)
    ((rho+R)^2 + z^2 - r^2) evaluated from coordinates;
  * a quadric written as a polynomial evaluates, differentiates and restricts
    like the quadric, and its Taylor box bound is the quadric's closed-form
    bound;
  * the Taylor bound contains the range of the polynomial on the box;
  * univariate roots against numpy's companion-matrix roots;
  * the torus volume 2 pi^2 R r^2, area 4 pi^2 R r, the flux of x through the
    surface (divergence theorem) and two second moments in closed form, over the
    unit box cut into cells (also for a rotated, shifted torus);
  * a cell whose face is tangent to the torus along a circle (h = 1/20) gets a
    bounded rule and its full volume.
(CPU only.)"""
import math

import numpy as np
import pytest

import oracle.quadrature as qd
from paper_2410_05865_amd import inputs

R0, r0 = 0.2, 0.1


def _rot(seed):
    return inputs._quat_rotation(np.random.default_rng(seed).uniform(0.0, 1.0, 3))


def _product_form(X, c, R, r, rot):
    u = (np.atleast_2d(X) - np.asarray(c)[None, :]) @ rot     # coordinates in the torus frame
    rho = np.hypot(u[:, 0], u[:, 1])
    z2 = u[:, 2] ** 2
    return ((rho - R) ** 2 + z2 - r * r) * ((rho + R) ** 2 + z2 - r * r)


@pytest.mark.parametrize("seed", [0, 1])
def test_torus_quartic_is_the_product_form(seed):
    rng = np.random.default_rng(seed)
    rot = np.eye(3) if seed == 0 else _rot(seed)
    c = rng.uniform(0.3, 0.7, 3)
    p = qd.torus_poly(c, R0, r0, rot)
    X = rng.uniform(0.0, 1.0, (500, 3))
    ref = _product_form(X, c, R0, r0, rot)
    assert np.max(np.abs(p(X) - ref)) < 1e-14
    # inside the tube negative, outside positive
    assert np.all((p(X) < 0) == (ref < 0))


def test_quadric_as_polynomial():
    rng = np.random.default_rng(3)
    qf = qd.ellipsoid_quadric(rng.uniform(0.3, 0.7, 3), rng.uniform(0.1, 0.3, 3), _rot(3))
    pf = qd.poly_from_quadric(qf)
    X = rng.uniform(0.0, 1.0, (200, 3))
    assert np.max(np.abs(pf(X) - qf(X))) < 1e-12
    assert np.max(np.abs(pf.grad(X) - qf.grad(X))) < 1e-11
    for k in range(3):
        Y = X[:, [i for i in range(3) if i != k]]
        assert np.max(np.abs(pf.restrict(k, 0.37)(Y) - qf.restrict(k, 0.37)(Y))) < 1e-12
    for _ in range(20):
        lo = rng.uniform(0.0, 0.9, 3)
        hi = lo + rng.uniform(0.01, 0.1, 3)
        v, spread = pf.bounds(lo, hi)
        m, w = 0.5 * (lo + hi), 0.5 * (hi - lo)
        # the quadric's bound: |grad f(m)| . w + w^T |Q| w
        g = qf.grad(m)[0]
        assert v == pytest.approx(float(qf(m)[0]), abs=1e-13)
        assert spread == pytest.approx(float(np.abs(g) @ w + w @ np.abs(qf.Q) @ w), rel=1e-12)
        assert qd.box_sign(pf, lo, hi) == qd.box_sign(qf, lo, hi)


def test_taylor_bound_contains_the_range():
    rng = np.random.default_rng(4)
    p = qd.torus_poly([0.5, 0.5, 0.5], R0, r0, _rot(4))
    for size in (0.01, 0.05, 0.2):
        for _ in range(10):
            lo = rng.uniform(0.2, 0.8 - size, 3)
            hi = lo + size
            v, spread = p.bounds(lo, hi)
            X = lo + (hi - lo) * rng.uniform(0.0, 1.0, (2000, 3))
            X[:8] = [[(hi if (b >> i) & 1 else lo)[i] for i in range(3)] for b in range(8)]   # the corners
            dev = np.abs(p(X) - v)
            assert np.all(dev <= spread * (1 + 1e-12) + 1e-18)
            assert v == pytest.approx(float(p(0.5 * (lo + hi))[0]), abs=1e-15)


def test_univariate_roots_against_numpy():
    rng = np.random.default_rng(5)
    for _ in range(200):
        deg = int(rng.integers(1, 5))
        roots = rng.uniform(-1.0, 2.0, deg)
        a = np.poly(roots)[::-1] * rng.uniform(0.5, 2.0)       # lowest power first
        if rng.uniform() < 0.3 and deg >= 2:                  # a complex pair instead of two real roots
            a = np.polymul(np.atleast_1d(np.poly(roots[:deg - 2]))[::-1], [1.0, 0.0, 1.0])
        a = np.concatenate([a, np.zeros(5 - len(a))])
        got = np.array(qd._poly1_roots(a, 0.0, 1.0))
        ref = np.roots(a[::-1][np.argmax(a[::-1] != 0):])
        ref = np.sort(ref[(np.abs(ref.imag) < 1e-12)].real)
        ref = ref[(ref > 1e-9) & (ref < 1 - 1e-9)]
        # double roots do not change sign: drop those numpy reports twice
        uniq = [x for x in ref if np.sum(np.abs(ref - x) < 1e-6) % 2 == 1]
        assert len(got) == len(uniq), (a, got, ref)
        assert np.allclose(np.sort(got), uniq, atol=1e-10)


def _box_integrals(psi, n, q):
    h = 1.0 / n
    V = A = F = M = Z = 0.0
    for i in range(n):
        for j in range(n):
            for k in range(n):
                lo = np.array([i, j, k]) * h
                (Xv, Wv), (Xs, Ws, Ns) = qd.region_rules(lo, lo + h, psi, q)
                V += Wv.sum()
                A += Ws.sum()
                F += np.sum(Ws * np.sum(Xs * Ns, axis=1))
                M += np.sum(Wv * ((Xv[:, 0] - 0.5) ** 2 + (Xv[:, 1] - 0.5) ** 2))
                Z += np.sum(Wv * (Xv[:, 2] - 0.5) ** 2)
    return V, A, F, M, Z


def test_torus_volume_area_flux_moments():
    psi = qd.torus_poly([0.5, 0.5, 0.5], R0, r0, np.eye(3))
    V, A, F, M, Z = _box_integrals(psi, 8, 8)
    vt = 2 * math.pi ** 2 * R0 * r0 ** 2
    assert V == pytest.approx(1.0 - vt, abs=1e-13)
    assert A == pytest.approx(4 * math.pi ** 2 * R0 * r0, abs=1e-10)
    # div x = 3: the integral of x.n over the box walls is 3, so over the torus
    # surface (n out of Omega) it is 3 V - 3
    assert F == pytest.approx(-3.0 * vt, abs=1e-10)
    # second moments of the solid torus: int rho^2 = vt (R^2 + 3 r^2 / 4),
    # int z^2 = vt r^2 / 4; of the box about its centre: 1/6 and 1/12
    assert M == pytest.approx(1.0 / 6.0 - vt * (R0 ** 2 + 0.75 * r0 ** 2), abs=1e-13)
    assert Z == pytest.approx(1.0 / 12.0 - vt * r0 ** 2 / 4.0, abs=1e-13)


def test_rotated_torus_volume_and_area():
    psi = qd.torus_poly([0.52, 0.47, 0.5], 0.25, 0.08, _rot(9))
    V, A, F, _, _ = _box_integrals(psi, 8, 6)
    vt = 2 * math.pi ** 2 * 0.25 * 0.08 ** 2
    # six points per piece on cells of 1/8, the tube radius 0.64 h: quadrature
    # errors of ~1e-10 (volume) and ~1e-7 (area)
    assert V == pytest.approx(1.0 - vt, abs=1e-9)
    assert A == pytest.approx(4 * math.pi ** 2 * 0.25 * 0.08, rel=1e-6)
    assert F == pytest.approx(-3.0 * vt, abs=1e-7)


def test_face_tangent_along_a_circle():
    """At h = 1/20 the plane z = 0.4 touches the torus (centre z 0.5, r 0.1)
    along the circle rho = R: cell (6, 7, 7) lies below it, wholly in Omega."""
    psi = qd.torus_poly([0.5, 0.5, 0.5], R0, r0, np.eye(3))
    h = 1.0 / 20
    lo = np.array([6, 7, 7]) * h
    (Xv, Wv), (Xs, Ws, Ns) = qd.region_rules(lo, lo + h, psi, 12)
    assert len(Wv) < 200_000
    assert Wv.sum() == pytest.approx(h ** 3, rel=1e-13)
    assert Ws.sum() < 1e-12 * h * h


def test_inside_any_obstacle_torus():
    dom, _ = inputs.torus_problem(32)
    assert inputs.inside_any_obstacle(dom, np.array([0.7, 0.5, 0.5]))       # on the tube's core circle
    assert not inputs.inside_any_obstacle(dom, np.array([0.5, 0.5, 0.5]))   # the hole
    assert not inputs.inside_any_obstacle(dom, np.array([0.7, 0.5, 0.61]))  # above the tube
    assert inputs.inside_any_obstacle(dom, np.array([0.5, 0.31, 0.55]))
