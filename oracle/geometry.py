"""Cut-cell geometry of one grid level (Sec. 2.2).

Cells C_i = (x_O + i h, x_O + (i+1) h) of the box R; cut cells
C_i ∩ Ω, their volumes, the boundary patches S_i = C_i ∩ ∂Ω, and the
interior / exterior / cut classification.  Ω is the box minus obstacles
(ellipsoids, quadric level sets; a torus, the quartic level set of the
paper's Problem 2), or (domain.inside) the interior of one ellipsoid: its
quadric is negated so that Ω = {psi > 0} either way, and cells away from it
are exterior.

Per cut cell the oracle keeps the quadrature nodes (for right-hand sides)
and the normalised moments used by the polynomial fits (Sec. 2.3):
  m_b  = <xi^b>            over the cut cell,         |b| <= 4
  sm_b = <<xi^b>>          over the patch,            |b| <= 4
  sn_{d,b} = <<n_d xi^b>>  over the patch,            |b| <= 3
with xi = (x - x_i)/h the cell-centred scaled coordinate and n the unit
normal pointing out of Ω.  Linear cell index: i + n (j + n k), x fastest.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List

import numpy as np

from . import quadrature as qd

EXTERIOR, INTERIOR, CUT = 0, 1, 2
TORUS = 1               # obstacle kind code of a torus (0: an ellipsoid)
Q_ORDER = 12
VOL_EPS = 1e-12


class GeometryError(RuntimeError):
    pass


def monomials(deg: int):
    out = []
    for d in range(deg + 1):
        for a in range(d, -1, -1):
            for b in range(d - a, -1, -1):
                out.append((a, b, d - a - b))
    return out


MONO4 = monomials(4)
MONO3 = monomials(3)
MONO4_INDEX = {e: i for i, e in enumerate(MONO4)}


def mono_eval(xi: np.ndarray, exps) -> np.ndarray:
    xi = np.atleast_2d(xi)
    out = np.empty((len(xi), len(exps)))
    for j, (a, b, c) in enumerate(exps):
        out[:, j] = xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c
    return out


def _full_cell_moments() -> np.ndarray:
    """<xi^b> over the unit cube [-1/2, 1/2]^3 (closed form)."""
    def mu(k):
        return 0.0 if k % 2 else 1.0 / ((k + 1) * 2 ** k)
    return np.array([mu(a) * mu(b) * mu(c) for a, b, c in MONO4])


_FULL = _full_cell_moments()


def full_cell_moments() -> np.ndarray:
    return _FULL


@dataclasses.dataclass
class CutCell:
    idx: int
    obst: int
    vol: float              # absolute volume
    m: np.ndarray           # (35,)
    area: float             # absolute patch area
    sm: np.ndarray          # (35,)
    sn: np.ndarray          # (3, 20)
    Xv: np.ndarray
    Wv: np.ndarray
    Xs: np.ndarray
    Ws: np.ndarray
    Ns: np.ndarray


class LevelGeometry:
    def __init__(self, domain, n: int):
        self.domain = domain
        self.n = n
        self.h = 1.0 / n
        self.origin = np.asarray(domain.origin, float)
        self.inside = bool(getattr(domain, "inside", False))
        self.quadrics = [qd.torus_poly(o.center, o.radii[0], o.radii[1], o.rot)
                         if getattr(o, "kind", 0) == TORUS else qd.ellipsoid_quadric(o.center, o.axes, o.rot)
                         for o in domain.obstacles]
        if self.inside:
            if len(self.quadrics) != 1 or not isinstance(self.quadrics[0], qd.Quadric):
                raise GeometryError("an interior domain is bounded by exactly one ellipsoid")
            q = self.quadrics[0]
            self.quadrics = [qd.Quadric(-q.Q, -q.b, -q.c)]
        N = n ** 3
        self.owner = np.full(N, -1, dtype=np.int64)
        self.cls = np.full(N, EXTERIOR if self.inside else INTERIOR, dtype=np.int8)
        self.vol = np.full(N, 0.0 if self.inside else self.h ** 3)
        self.cut: Dict[int, CutCell] = {}
        self._claim()
        self._classify()

    # ---------------------------------------------------------- indexing
    def idx(self, i, j, k):
        return i + self.n * (j + self.n * k)

    def ijk(self, p):
        n = self.n
        return p % n, (p // n) % n, p // (n * n)

    def cell_box(self, p):
        i, j, k = self.ijk(p)
        lo = self.origin + self.h * np.array([i, j, k], float)
        return lo, lo + self.h

    def center(self, p):
        i, j, k = self.ijk(p)
        return self.origin + self.h * (np.array([i, j, k], float) + 0.5)

    # ---------------------------------------------------------- building
    def _claim(self):
        """Each obstacle claims the cells that meet its bounding sphere; a
        cell claimed twice, or a claimed cell on a wall layer, is rejected."""
        n, h = self.n, self.h
        for t, o in enumerate(self.domain.obstacles):
            R = o.bounding_radius()
            c = np.asarray(o.center, float)
            lo_i = np.floor((c - R - self.origin) / h).astype(int) - 1
            hi_i = np.floor((c + R - self.origin) / h).astype(int) + 1
            lo_i = np.maximum(lo_i, 0)
            hi_i = np.minimum(hi_i, n - 1)
            ii = [np.arange(lo_i[d], hi_i[d] + 1) for d in range(3)]
            I, J, K = np.meshgrid(*ii, indexing="ij")
            I, J, K = I.ravel(), J.ravel(), K.ravel()
            lo = self.origin[None, :] + h * np.stack([I, J, K], 1)
            hi = lo + h
            dist = np.maximum(np.maximum(lo - c[None, :], 0.0), c[None, :] - hi)
            hit = np.sum(dist * dist, axis=1) < R * R
            I, J, K = I[hit], J[hit], K[hit]
            p = I + n * (J + n * K)
            if np.any(self.owner[p] >= 0):
                raise GeometryError("a cell meets two obstacles")
            wall = (I == 0) | (I == n - 1) | (J == 0) | (J == n - 1) | (K == 0) | (K == n - 1)
            if np.any(wall):
                raise GeometryError("an obstacle reaches the wall layer")
            self.owner[p] = t

    def _classify(self):
        h = self.h
        h3 = h ** 3
        for p in np.nonzero(self.owner >= 0)[0]:
            p = int(p)
            psi = self.quadrics[self.owner[p]]
            lo, hi = self.cell_box(p)
            (Xv, Wv), (Xs, Ws, Ns) = qd.region_rules(lo, hi, psi, Q_ORDER)
            V = float(Wv.sum())
            if V < VOL_EPS * h3:
                self.cls[p] = EXTERIOR
                self.vol[p] = 0.0
                continue
            if V > (1.0 - VOL_EPS) * h3:
                self.cls[p] = INTERIOR
                self.vol[p] = h3
                continue
            self.cls[p] = CUT
            self.vol[p] = V
            xc = self.center(p)
            xi = (Xv - xc[None, :]) / h
            m = mono_eval(xi, MONO4).T @ Wv / V
            A = float(Ws.sum())
            xs = (Xs - xc[None, :]) / h
            Ms = mono_eval(xs, MONO4)
            sm = Ms.T @ Ws / A
            M3 = mono_eval(xs, MONO3)
            sn = np.stack([M3.T @ (Ws * Ns[:, d]) / A for d in range(3)])
            self.cut[p] = CutCell(p, int(self.owner[p]), V, m, A, sm, sn, Xv, Wv, Xs, Ws, Ns)

    # ---------------------------------------------------------- queries
    def moments(self, p) -> np.ndarray:
        if p in self.cut:
            return self.cut[p].m
        return full_cell_moments()

    def face_area(self, p: int, d: int, side: int) -> float:
        """Area of the face of cell p on side (+1/-1) of axis d, intersected with Ω."""
        i, j, k = self.ijk(p)
        ijk = [i, j, k]
        q_ijk = list(ijk)
        q_ijk[d] += side
        if not (0 <= q_ijk[d] < self.n):
            return 0.0
        q = self.idx(*q_ijk)
        if self.cls[p] == EXTERIOR or self.cls[q] == EXTERIOR:
            return 0.0
        t = self.owner[p] if self.owner[p] >= 0 else self.owner[q]
        if t < 0:
            return self.h ** 2
        xf = self.origin[d] + self.h * (ijk[d] + (1 if side > 0 else 0))
        psi2 = self.quadrics[t].restrict(d, xf)
        lo, hi = self.cell_box(p)
        keep = [a for a in range(3) if a != d]
        (Xv, Wv), _ = qd.region_rules(lo[keep], hi[keep], psi2, Q_ORDER)
        return float(Wv.sum())
