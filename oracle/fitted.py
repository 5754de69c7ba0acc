"""The paper's geometry front end (Sec. 3.1 boundary fitting, Sec. 3.2
numerical cubature) on one cut cell, as a check of the exact geometry the
solver uses, and the accuracy test of the paper's Table 1 (Sec. 6.1).

Test infrastructure: imported only by tests/ (see oracle/__init__.py).

Per cut cell C = box ∩ Omega with boundary patch S = box ∩ dOmega:

  * points of dOmega inside the box: the nodes of a FIT_Q-point height-function
    surface rule on the exact level set (at least 6 of them);
  * the height axis w is the axis of the largest component of the patch's mean
    normal (components within a relative 1e-12 of the largest tie, and ties go
    to the lowest axis), u < v the other two;
  * in the cell-centred scaled coordinates (U, V, W) = (x - centre) / h the
    quadratic W = p(U, V) = a U^2 + b U V + c V^2 + d U + e V + g is fitted by
    least squares to the points (singular values below FIT_RCOND times the
    largest are dropped: the minimum-norm solution);
  * the fitted region is {s (W - p(U, V)) > 0} in the box, s the sign that
    puts Omega's side (the side the exact level set's gradient points to) on
    the positive side: a quadric, so its volume and patch integrals use the
    same height-function rule as the exact geometry.

The paper evaluates integrals over the fitted region by the divergence theorem
and Green's formula; here the fitted quadric is integrated directly with the
height-function Gauss rule (12 points per piece), which integrates the same
region to rounding for smooth integrands.

Table 1 errors per cut cell: the average of u over the exact region minus its
average over the fitted region, and the same for the boundary patches; norms
(1/N sum |e_i|^p)^(1/p) for p = 1, 2 and the max, over the N cut cells.
"""
from __future__ import annotations

import numpy as np

from . import quadrature as qd
from .geometry import CUT, Q_ORDER, LevelGeometry

FIT_Q = 4             # points: the surface nodes of a 4-point-per-piece rule on the exact patch
FIT_RCOND = 1e-12     # relative singular-value cutoff of the least-squares fit


def _basis(U, V):
    return np.stack([U * U, U * V, V * V, U, V, np.ones_like(U)], axis=1)


def fit_patch(psi, lo, hi):
    """(axis w, coefficients (a, b, c, d, e, g), fitted level set as a Quadric)
    for the cell [lo, hi], or None if the exact patch yields fewer than 6
    points."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    _, (Xs, Ws, Ns) = qd.region_rules(lo, hi, psi, FIT_Q)
    if len(Xs) < 6:
        return None
    nbar = (Ws[:, None] * Ns).sum(axis=0)
    a = np.abs(nbar)
    w = int(next(i for i in range(3) if a[i] >= a.max() * (1.0 - qd.TIE)))
    u, v = [i for i in range(3) if i != w]
    c = 0.5 * (lo + hi)
    h = float(hi[0] - lo[0])
    P = (Xs - c[None, :]) / h
    coef, *_ = np.linalg.lstsq(_basis(P[:, u], P[:, v]), P[:, w], rcond=FIT_RCOND)
    # Ns points out of Omega, so Omega lies toward -Ns: s (W - p) grows toward
    # Omega when s has the sign of -nbar_w
    s = 1.0 if -nbar[w] > 0 else -1.0
    # s (W - p(U, V)) as a quadric in x, with U = (x_u - c_u)/h etc.; scaled by h
    # (positive) to keep the level set in length units
    Q = np.zeros((3, 3))
    b = np.zeros(3)
    A2, B2, C2, D1, E1, G0 = coef
    # -s h p: quadratic part -s (A2 (x_u - c_u)^2 + B2 (x_u - c_u)(x_v - c_v) + C2 (x_v - c_v)^2) / h
    Q[u, u] = -s * A2 / h
    Q[v, v] = -s * C2 / h
    Q[u, v] = Q[v, u] = -s * B2 / (2.0 * h)
    cu, cv, cw = c[u], c[v], c[w]
    b[u] = -s * (-2.0 * A2 * cu / h - B2 * cv / h + D1)
    b[v] = -s * (-2.0 * C2 * cv / h - B2 * cu / h + E1)
    b[w] = s
    const = -s * (A2 * cu * cu / h + B2 * cu * cv / h + C2 * cv * cv / h - D1 * cu - E1 * cv + G0 * h) - s * cw
    return w, coef, qd.Quadric(Q, b, const)


def patch_averages(psi, lo, hi, field):
    """(volume, area, average of field over the region, over the patch) of
    {psi > 0} in the box, from the Q_ORDER height-function rule."""
    (Xv, Wv), (Xs, Ws, _) = qd.region_rules(np.asarray(lo, float), np.asarray(hi, float), psi, Q_ORDER)
    V, A = float(Wv.sum()), float(Ws.sum())
    cav = float(Wv @ field.value(Xv)) / V if V > 0 else np.nan
    fav = float(Ws @ field.value(Xs)) / A if A > 0 else np.nan
    return V, A, cav, fav


def cut_cell_fits(domain, n, field):
    """Per cut cell of the n^3 grid (ascending index): cell index, height axis,
    coefficients, and (V, A, cell average, patch average) for the exact and the
    fitted region.  Cells whose exact patch gives fewer than 6 points carry
    axis -1 and NaN."""
    geo = LevelGeometry(domain, n)
    out = []
    for p in sorted(k for k in geo.cut):
        if geo.cls[p] != CUT:
            continue
        lo, hi = geo.cell_box(p)
        psi = geo.quadrics[geo.owner[p]]
        exact = patch_averages(psi, lo, hi, field)
        f = fit_patch(psi, lo, hi)
        if f is None:
            out.append((p, -1, np.full(6, np.nan), exact, (np.nan,) * 4))
            continue
        w, coef, qf = f
        out.append((p, w, coef, exact, patch_averages(qf, lo, hi, field)))
    return out


def table1_errors(rows):
    """Cell-average and face-average error norms (Linf, L1, L2) over the rows
    of cut_cell_fits with a fit and nonempty fitted region and patch."""
    ec, ef = [], []
    for p, w, coef, ex, fi in rows:
        if w < 0 or not (fi[0] > 0 and fi[1] > 0):
            continue
        ec.append(ex[2] - fi[2])
        ef.append(ex[3] - fi[3])
    ec, ef = np.abs(np.array(ec)), np.abs(np.array(ef))
    norms = lambda e: (float(e.max()), float(e.mean()), float(np.sqrt(np.mean(e * e))))
    return norms(ec), norms(ef), len(ec)
