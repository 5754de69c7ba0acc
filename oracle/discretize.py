"""Discretisation of one grid level: L phi = r := f - N g (Sec. 2.4).

Rows
  * regular cells (phi_1): the cell-averaged fourth-order Laplacian
    (Sec. 2.3, eq. regularLaplaceDiscretization), with ghost cells beyond
    the walls filled from the boundary data (Sec. 2.3, Dirichlet and
    Neumann ghost formulas);
  * every other unknown (phi_2): FV-PLG (Secs. 2.3 and 4.1): a poised
    triangular lattice T of 35 cells around the cell, the boundary patches
    of the cut cells in T, a weighted least-squares fit of a degree-4
    polynomial, and the cell average of its Laplacian.

Readings of the paper (the unit tests pin each against mathematics):
  * the second Dirichlet ghost formula's face coefficient is 300/12 (the
    printed 75 does not reproduce constants);
  * phi_1 iff the cell is a plain interior cell (not merged) and each of
    its 12 axis neighbours at distance 1 and 2 is a plain interior cell or
    lies beyond a wall whose ghost fill reads only plain interior cells;
  * PLG search: windows of 5 cells per axis, per-axis coordinate numberings
    that grow contiguously, the cell as shallow in the lattice as possible,
    preferring steps away from the nearest obstacle; first lattice in a
    fixed enumeration order (see `plg_select`);
  * sites: the 35 lattice cells, the boundary patches of cut cells among
    them and the wall faces of those on the box boundary; weights
    w = max(1, |j - i|^2)^-4 in grid units (steep enough that L_22 has no
    eigenvalues of the wrong sign and the V-cycle factor matches the
    obstacle-free one);
  * Neumann patch data enter as h <<dphi/dn>> with the scaled functional
    <<n . grad_xi xi^a>>.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from math import comb

from . import quadrature as qd
from .geometry import (CUT, EXTERIOR, INTERIOR, LevelGeometry, MONO3, MONO4,
                       GeometryError)
from .merging import THETA, groups, merge_cells
from .fields import Field

DIRICHLET, NEUMANN, ROBIN = 0, 1, 2

# Ghost-cell formulas: value of ghost 1 and ghost 2 beyond a wall as
# combinations of the 4 nearest interior cells (nearest last) and the face
# datum.  Dirichlet datum: <phi> on the face; Neumann: 12 h <dphi/dn>.
GHOST_DIRICHLET = {1: ((3, -17, 43, -77), 60, 12.0),
                   2: ((27, -145, 335, -505), 300, 12.0)}
GHOST_NEUMANN = {1: ((1, -5, 9, 5), 12, 10.0),
                 2: ((3, -15, 29, -15), 12, 2.0)}
STENCIL5 = {-2: -1.0, -1: 16.0, 0: -30.0, 1: 16.0, 2: -1.0}


def robin_ghost_rule(alpha: float, beta: float, h: float):
    """Ghost-cell formulas beyond a wall with the condition alpha phi + beta
    dphi/dn = g (n out of the box), derived as the Dirichlet and Neumann ones
    are: in units of h along the wall normal (the wall at 0, interior cells
    [j-1, j], j = 1..4, ghost g = [-g, 1-g]), the quartic P whose averages over
    the 4 interior cells are A_1..A_4 and with alpha P(0) - (beta/h) P'(0) = D,
    D the face average of g; each ghost average of P is a combination of the
    A_j and D.  Returns {g: (coefficients of A_4, A_3, A_2, A_1, coefficient of
    D)}."""
    def avg(k, a, b):
        return (b ** (k + 1) - a ** (k + 1)) / ((k + 1) * (b - a))
    M = np.zeros((5, 5))
    for j in range(1, 5):
        M[j - 1] = [avg(k, j - 1, j) for k in range(5)]
    M[4] = [alpha, -beta / h, 0.0, 0.0, 0.0]
    out = {}
    for g in (1, 2):
        m = np.array([avg(k, -g, 1 - g) for k in range(5)])
        r = np.linalg.solve(M.T, m)          # ghost = r . (A_1, .., A_4, D)
        out[g] = (tuple(r[3::-1]), float(r[4]))
    return out


def ghost_rule(bc: int, robin, h: float):
    """{g: (coefficients of the 4 interior cells farthest first, datum
    coefficient)} for a Dirichlet (datum <g>), Neumann (datum <dphi/dn>) or
    Robin (datum <alpha g + beta dg/dn>) wall."""
    if bc == DIRICHLET:
        return {g: (tuple(c / den for c in cs), dat / den) for g, (cs, dat, den) in GHOST_DIRICHLET.items()}
    if bc == NEUMANN:
        return {g: (tuple(c / den for c in cs), dat * h / den) for g, (cs, dat, den) in GHOST_NEUMANN.items()}
    return robin_ghost_rule(robin[0], robin[1], h)


class PLGError(RuntimeError):
    pass


def lattice_exponents():
    return [e for e in MONO4]   # the 35 (k0, k1, k2) with k0 + k1 + k2 <= 4


LATTICE = lattice_exponents()
MONO3_INDEX = {e: j for j, e in enumerate(MONO3)}


def _sequences(n_fwd: int, n_bwd: int):
    """All orderings of n_fwd 'F' and n_bwd 'B' moves, lexicographic, F < B."""
    out = []
    for pos in itertools.combinations(range(n_fwd + n_bwd), n_bwd):
        s = ["F"] * (n_fwd + n_bwd)
        for p in pos:
            s[p] = "B"
        out.append("".join(s))
    return sorted(set(out))


def _shift_order():
    vs = list(itertools.product(range(3), repeat=3))
    return sorted(vs, key=lambda v: (sum(v), -v[0], -v[1], -v[2]))


SHIFTS = _shift_order()


class Level:
    """Geometry, merging, unknowns, rows and right-hand side of one level."""

    def __init__(self, domain, n: int, theta: float = THETA):
        self.domain = domain
        self.n = n
        self.h = 1.0 / n
        self.geo = LevelGeometry(domain, n)
        self.host = merge_cells(self.geo, theta)
        self.groups = groups(self.host)
        self.unknowns = np.array(sorted(self.groups), dtype=np.int64)
        self.N = len(self.unknowns)
        self.uidx = np.full(n ** 3, -1, dtype=np.int64)
        self.uidx[self.unknowns] = np.arange(self.N)
        self.wall_bc = list(domain.wall_bc)
        self.wall_robin = [tuple(map(float, ab)) for ab in getattr(domain, "wall_robin", ((1.0, 0.0),) * 6)]
        n3 = n ** 3
        self.plain = np.zeros(n3, dtype=bool)
        for p, mem in self.groups.items():
            if len(mem) == 1 and self.geo.cls[p] == INTERIOR:
                self.plain[p] = True
        self.is_phi1 = np.zeros(n3, dtype=bool)
        for p in self.unknowns:
            self.is_phi1[p] = self._regular_ok(int(p))
        self.phi2 = np.array([p for p in self.unknowns if not self.is_phi1[p]], dtype=np.int64)
        self._build_rows()

    # ------------------------------------------------------------ helpers
    def ijk(self, p):
        return self.geo.ijk(p)

    def idx(self, i, j, k):
        return self.geo.idx(i, j, k)

    def _regular_ok(self, p: int) -> bool:
        if not self.plain[p]:
            return False
        n = self.n
        ijk = list(self.ijk(p))
        for d in range(3):
            for o in (-2, -1, 1, 2):
                c = ijk[d] + o
                q = list(ijk)
                if 0 <= c < n:
                    q[d] = c
                    if not self.plain[self.idx(*q)]:
                        return False
                else:
                    # ghost fill reads the 4 cells nearest the wall on this line
                    rng = range(n - 4, n) if c >= n else range(0, 4)
                    for t in rng:
                        q[d] = t
                        if not self.plain[self.idx(*q)]:
                            return False
        return True

    # -------------------------------------------------------- regular rows
    def regular_row(self, p: int):
        """Returns ({cell: coeff}, [(axis, side, coeff)]) for the row of a
        phi_1 cell; coefficients include 1/(12 h^2).  Each wall term
        multiplies the wall datum (Dirichlet <g>, Neumann <dphi/dn>)."""
        n, h = self.n, self.h
        s = 1.0 / (12.0 * h * h)
        ijk = list(self.ijk(p))
        cols = {}
        walls = []
        for d in range(3):
            i = ijk[d]
            for o, c5 in STENCIL5.items():
                t = i + o
                if 0 <= t < n:
                    q = list(ijk)
                    q[d] = t
                    key = self.idx(*q)
                    cols[key] = cols.get(key, 0.0) + c5 * s
                    continue
                side = 1 if t >= n else -1
                g = t - (n - 1) if side > 0 else -t     # ghost number 1 or 2
                wall = 2 * d + (1 if side > 0 else 0)
                coefs, datum = ghost_rule(self.wall_bc[wall], self.wall_robin[wall], h)[g]
                # interior cells, farthest first: for the upper wall n-4..n-1
                line = list(range(n - 4, n)) if side > 0 else [3, 2, 1, 0]
                for cc, tt in zip(coefs, line):
                    q = list(ijk)
                    q[d] = tt
                    key = self.idx(*q)
                    cols[key] = cols.get(key, 0.0) + c5 * s * cc
                walls.append((d, side, c5 * s * datum))
        return cols, walls

    # ------------------------------------------------------- PLG selection
    def _inward_signs(self, p: int):
        xc = self.geo.center(p)
        best, bt = None, -1
        for t, o in enumerate(self.domain.obstacles):
            dist = float(np.linalg.norm(xc - o.center)) - o.bounding_radius()
            if best is None or dist < best:
                best, bt = dist, t
        if bt < 0:
            return np.ones(3, dtype=int)
        psi = self.geo.quadrics[bt]
        if isinstance(psi, qd.Quadric):
            g = psi.Q @ (xc - np.asarray(self.domain.obstacles[bt].center))
        else:
            g = psi.grad(xc)[0]
        gn = float(np.linalg.norm(g))
        return np.where(g < -1e-9 * gn, -1, 1)

    def _axis_numberings(self, i: int, lo: int, sgn: int):
        """Contiguous-growth numberings (p_0..p_4) of the window coordinates
        lo..lo+4: start anywhere, then extend the covered interval by one at
        either end.  Sorted by the position k of i in the numbering, then by
        the signed offsets s (p_j - i) in decreasing order (inward first).
        Returns [(k, coords - lo)]."""
        out = []
        for start in range(lo, lo + 5):
            below = start - lo
            above = 4 - below
            for moves in _sequences(above, below):       # 'F' = up here
                a = b = start
                pts = [start]
                for mv in moves:
                    if mv == "F":
                        b += 1
                        pts.append(b)
                    else:
                        a -= 1
                        pts.append(a)
                k = pts.index(i)
                key = (k, tuple(-sgn * (t - i) for t in pts))
                out.append((key, np.array(pts) - lo))
        out.sort(key=lambda t: t[0])
        return [(key[0], pts) for key, pts in out]

    def plg_select(self, p: int):
        """A poised triangular lattice T (35 cells, in LATTICE order) of
        unknown cells with p in T (Def. of the PLG problem, Sec. 4.1).

        Search order: depth of p in T (k_0 + k_1 + k_2 of its lattice
        position) ascending; then windows of 5 cells per axis, the centred
        one first and then shifted away from the nearest obstacle by
        (o_0, o_1, o_2) in {0,1,2}^3 ordered by total shift and x-shifts
        first; then the per-axis numberings in `_axis_numberings` order."""
        n = self.n
        ijk = np.array(self.ijk(p))
        sgn = self._inward_signs(p)
        known = (self.host >= 0) & (self.host == np.arange(n ** 3))
        lat = np.array(LATTICE)
        cache = {}
        for depth in range(5):
            for o in SHIFTS:
                lo = np.clip(ijk - 2 + sgn * np.array(o), 0, n - 5)
                key = tuple(lo)
                if key not in cache:
                    win = np.zeros((5, 5, 5), dtype=bool)
                    for a in range(5):
                        for b in range(5):
                            for c in range(5):
                                win[a, b, c] = known[self.idx(lo[0] + a, lo[1] + b, lo[2] + c)]
                    nums = [self._axis_numberings(int(ijk[d]), int(lo[d]), int(sgn[d]))
                            for d in range(3)]
                    cache[key] = (win, nums)
                win, nums = cache[key]
                K = [np.array([k for k, _ in nums[d]]) for d in range(3)]
                C = [np.array([c for _, c in nums[d]]) for d in range(3)]
                ix, iy, iz = np.meshgrid(np.arange(len(K[0])), np.arange(len(K[1])),
                                         np.arange(len(K[2])), indexing="ij")
                ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
                sel = (K[0][ix] + K[1][iy] + K[2][iz]) == depth
                ix, iy, iz = ix[sel], iy[sel], iz[sel]
                if len(ix) == 0:
                    continue
                a = C[0][ix][:, lat[:, 0]]
                b = C[1][iy][:, lat[:, 1]]
                c = C[2][iz][:, lat[:, 2]]
                ok = np.all(win[a, b, c], axis=1)
                if np.any(ok):
                    t0 = int(np.argmax(ok))
                    return [self.idx(lo[0] + a[t0, t], lo[1] + b[t0, t], lo[2] + c[t0, t])
                            for t in range(len(lat))]
        raise PLGError(f"no poised lattice for cell {p}")

    # -------------------------------------------------------- PLG fitting
    def _target_frame_cell_avg(self, p_target: int, group):
        """<xi^a> over the union of `group` cells, xi centred at the target:
        each member's own-frame moments moved to the target frame by the
        binomial theorem, then volume-weighted."""
        tot = np.zeros(len(MONO4))
        vol = 0.0
        it = np.array(self.ijk(p_target))
        for m in group:
            dl = tuple(int(v) for v in np.array(self.ijk(m)) - it)
            mom = self.geo.moments(m)
            v = self.geo.vol[m]
            tot += v * (shift_matrix(dl, MONO4) @ mom)
            vol += v
        return tot / vol

    def _target_frame_laplacian(self, p_target: int):
        """ell_a = <Delta phi_a> over the target's region, phi_a = xi^a."""
        h = self.h
        mom = self._target_frame_cell_avg(p_target, self.groups[p_target])
        idx = {e: j for j, e in enumerate(MONO4)}
        ell = np.zeros(len(MONO4))
        for j, e in enumerate(MONO4):
            for d in range(3):
                if e[d] >= 2:
                    f = list(e)
                    f[d] -= 2
                    ell[j] += e[d] * (e[d] - 1) * mom[idx[tuple(f)]]
        return ell / (h * h)

    def _robin_scale(self, m: int):
        """(alpha, beta, s) of the Robin condition on cut cell m's patch, with
        s = h / (|alpha| h + |beta|) scaling its site row to unit size."""
        alpha, beta = self.domain.obstacles[self.geo.cut[m].obst].robin
        return alpha, beta, self.h / (abs(alpha) * self.h + abs(beta))

    def _patch_functional(self, p_target: int, m: int, bc: int):
        """Dirichlet: <<xi^a>> over the patch of cell m; Neumann:
        <<n . grad_xi xi^a>> (xi centred at the target); Robin (alpha phi +
        beta dphi/dn): s (alpha <<xi^a>> + (beta / h) <<n . grad_xi xi^a>>)
        with s = h / (|alpha| h + |beta|), which is the Dirichlet row for
        beta = 0 and the Neumann row for alpha = 0."""
        cc = self.geo.cut[m]
        dl = tuple(int(v) for v in np.array(self.ijk(m)) - np.array(self.ijk(p_target)))
        if bc == ROBIN:
            alpha, beta, s = self._robin_scale(m)
            return s * (alpha * self._patch_functional(p_target, m, DIRICHLET)
                        + (beta / self.h) * self._patch_functional(p_target, m, NEUMANN))
        if bc == DIRICHLET:
            return shift_matrix(dl, MONO4) @ cc.sm
        S3 = shift_matrix(dl, MONO3)
        sn = [S3 @ cc.sn[d] for d in range(3)]
        out = np.zeros(len(MONO4))
        for j, e in enumerate(MONO4):
            for d in range(3):
                if e[d]:
                    f = list(e)
                    f[d] -= 1
                    out[j] += e[d] * sn[d][MONO3_INDEX[tuple(f)]]
        return out

    # weights w_k = max(1, |j_k - i|^2)^(-WEIGHT_POW) in grid units
    WEIGHT_POW = 4.0

    def plg_sites(self, p: int):
        """(cells, sites): stencil cells, then boundary sites.  A boundary
        site is ('S', m, bc, None) for the irregular patch of cut cell m, or
        ('W', m, bc, (axis, side)) for the wall face of a stencil cell m on
        the box boundary.  Patches are listed per stencil cell (group members
        in index order), wall faces per stencil cell in axis order."""
        cells = self.plg_select(p)
        sites = []
        for c in cells:
            for m in self.groups[c]:
                if m in self.geo.cut and self.geo.cut[m].area > 0:
                    bc = self.domain.obstacles[self.geo.cut[m].obst].bc
                    sites.append(("S", m, bc, None))
        for c in cells:
            ijk = self.ijk(c)
            for d in range(3):
                for side in (-1, 1):
                    if (side < 0 and ijk[d] == 0) or (side > 0 and ijk[d] == self.n - 1):
                        bc = self.wall_bc[2 * d + (1 if side > 0 else 0)]
                        sites.append(("W", c, bc, (d, side)))
        return cells, sites

    def _wall_robin_scale(self, d: int, side: int):
        """(alpha, beta, s) of a Robin wall, s = h / (|alpha| h + |beta|)."""
        alpha, beta = self.wall_robin[2 * d + (1 if side > 0 else 0)]
        return alpha, beta, self.h / (abs(alpha) * self.h + abs(beta))

    def _wall_functional(self, p_target: int, c: int, bc: int, d: int, side: int):
        """Dirichlet: <xi^a> over the wall face of cell c; Neumann:
        <n . grad_xi xi^a> there (n = side e_d); Robin: s (alpha <xi^a> +
        (beta / h) <n . grad_xi xi^a>), scaled as on obstacle patches; xi
        centred at the target."""
        if bc == ROBIN:
            alpha, beta, sc = self._wall_robin_scale(d, side)
            return sc * (alpha * self._wall_functional(p_target, c, DIRICHLET, d, side)
                         + (beta / self.h) * self._wall_functional(p_target, c, NEUMANN, d, side))
        dl = np.array(self.ijk(c)) - np.array(self.ijk(p_target))
        xf = dl[d] + 0.5 * side                    # face position in xi_d
        def avg(k, delta):                         # mean of (t + delta)^k on [-1/2, 1/2]
            return ((delta + 0.5) ** (k + 1) - (delta - 0.5) ** (k + 1)) / (k + 1)
        out = np.zeros(len(MONO4))
        for j, e in enumerate(MONO4):
            inplane = 1.0
            for a in range(3):
                if a != d:
                    inplane *= avg(e[a], dl[a])
            if bc == DIRICHLET:
                out[j] = inplane * xf ** e[d]
            elif e[d] > 0:
                out[j] = side * e[d] * xf ** (e[d] - 1) * inplane
        return out

    def plg_row(self, p: int):
        """Returns (cells, cell_coeffs, patches, patch_coeffs)."""
        h = self.h
        cells, patches = self.plg_sites(p)
        xt = self.geo.center(p)
        it = np.array(self.ijk(p))
        rows, wts = [], []
        for c in cells:
            rows.append(self._target_frame_cell_avg(p, self.groups[c]))
            dl = np.array(self.ijk(c)) - it
            wts.append(max(1.0, float(dl @ dl)) ** (-self.WEIGHT_POW))
        for kind, m, bc, extra in patches:
            if kind == "S":
                rows.append(self._patch_functional(p, m, bc))
            else:
                rows.append(self._wall_functional(p, m, bc, *extra))
            dl = np.array(self.ijk(m)) - it
            wts.append(max(1.0, float(dl @ dl)) ** (-self.WEIGHT_POW))
        A = np.array(rows)
        sw = np.sqrt(np.array(wts))
        M = sw[:, None] * A
        ell = self._target_frame_laplacian(p)
        y = np.linalg.lstsq(M.T, ell, rcond=None)[0]
        c = sw * y
        return cells, c[:len(cells)], patches, c[len(cells):]

    # ------------------------------------------------------------ assembly
    def _build_rows(self):
        rows, cols, vals = [], [], []
        self.wall_terms = {}      # compact row -> [(p_cell, axis, side, coeff)]
        self.patch_terms = {}     # compact row -> [(site, coeff)]
        self.plg = {}             # compact row -> (cells, coeffs)
        for r, p in enumerate(self.unknowns):
            p = int(p)
            if self.is_phi1[p]:
                cc, walls = self.regular_row(p)
                for q, v in cc.items():
                    rows.append(r)
                    cols.append(self.uidx[q])
                    vals.append(v)
                if walls:
                    self.wall_terms[r] = [(p, d, s, v) for d, s, v in walls]
            else:
                cells, cv, patches, pv = self.plg_row(p)
                for q, v in zip(cells, cv):
                    rows.append(r)
                    cols.append(self.uidx[q])
                    vals.append(v)
                self.plg[r] = (cells, cv)
                self.patch_terms[r] = [(site, v) for site, v in zip(patches, pv)]
        if np.any(np.array(cols) < 0):
            raise GeometryError("a row references a cell without an unknown")
        self.L = sp.csr_matrix((vals, (rows, cols)), shape=(self.N, self.N))
        self.L.sum_duplicates()

    # --------------------------------------------------- right-hand sides
    def region_average(self, field: Field) -> np.ndarray:
        """Exact (to quadrature accuracy on cut cells) average of a field over
        each unknown's region (a merged group counts as one region)."""
        h = self.h
        out = np.zeros(self.N)
        full = [p for p in self.unknowns if len(self.groups[p]) == 1 and p not in self.geo.cut]
        full = np.array(full, dtype=np.int64)
        if len(full):
            i, j, k = self.ijk(full)
            lo = np.stack([i, j, k], 1) * h + np.asarray(self.domain.origin)[None, :]
            out[self.uidx[full]] = field.box_average(lo, lo + h)
        for p in self.unknowns:
            mem = self.groups[p]
            if len(mem) == 1 and p not in self.geo.cut:
                continue
            tot, vol = 0.0, 0.0
            for m in mem:
                if m in self.geo.cut:
                    cc = self.geo.cut[m]
                    tot += float(field.value(cc.Xv) @ cc.Wv)
                    vol += cc.vol
                else:
                    lo, hi = self.geo.cell_box(m)
                    tot += float(field.box_average(lo[None], hi[None])[0]) * h ** 3
                    vol += h ** 3
            out[self.uidx[p]] = tot / vol
        return out

    def wall_datum(self, field: Field, p: int, d: int, side: int, bc: int) -> float:
        lo, hi = self.geo.cell_box(p)
        lo = lo.copy()
        hi = hi.copy()
        # the wall face on this grid line (not the row cell's own face)
        xw = self.domain.origin[d] + (self.n * self.h if side > 0 else 0.0)
        lo[d] = hi[d] = xw
        if bc == DIRICHLET:
            return float(field.box_average(lo[None], hi[None])[0])
        dn = side * float(field.box_average_grad(lo[None], hi[None], d)[0])
        if bc == NEUMANN:
            return dn
        alpha, beta = self.wall_robin[2 * d + (1 if side > 0 else 0)]
        return alpha * float(field.box_average(lo[None], hi[None])[0]) + beta * dn

    def rhs(self, f: Field, g: Field) -> np.ndarray:
        """r = f_avg - N g: cell averages of f minus the boundary-data terms."""
        h = self.h
        r = self.region_average(f)
        for row, terms in self.wall_terms.items():
            for p, d, s, v in terms:
                bc = self.wall_bc[2 * d + (1 if s > 0 else 0)]
                r[row] -= v * self.wall_datum(g, p, d, s, bc)
        for row, terms in self.patch_terms.items():
            for (kind, m, bc, extra), v in terms:
                if kind == "W":
                    d, side = extra
                    dat = self.wall_datum(g, m, d, side, bc)
                    if bc == NEUMANN:
                        dat *= h
                    elif bc == ROBIN:
                        dat *= self._wall_robin_scale(d, side)[2]
                    r[row] -= v * dat
                    continue
                cc = self.geo.cut[m]
                if bc == DIRICHLET:
                    dat = float(g.value(cc.Xs) @ cc.Ws) / cc.area
                elif bc == NEUMANN:
                    dn = np.sum(g.grad(cc.Xs) * cc.Ns, axis=1)
                    dat = h * float(dn @ cc.Ws) / cc.area
                else:
                    # Robin datum <<alpha g + beta dg/dn>> with the row's scale
                    alpha, beta, sc = self._robin_scale(m)
                    dn = np.sum(g.grad(cc.Xs) * cc.Ns, axis=1)
                    dat = sc * float((alpha * g.value(cc.Xs) + beta * dn) @ cc.Ws) / cc.area
                r[row] -= v * dat
        return r

    # -------------------------------------------------------- conversions
    def to_grid(self, x: np.ndarray) -> np.ndarray:
        """Compact unknown vector -> n^3 array (absorbed cells hold their
        host's value, exterior cells 0)."""
        out = np.zeros(self.n ** 3)
        valid = self.host >= 0
        out[valid] = x[self.uidx[self.host[valid]]]
        return out

    def from_grid(self, g: np.ndarray) -> np.ndarray:
        return np.asarray(g)[self.unknowns].copy()

    def phi1_mask(self) -> np.ndarray:
        return self.is_phi1[self.unknowns]


_SHIFT_CACHE = {}


def shift_matrix(delta, exps):
    """S with (S m)_a = <(xi + delta)^a> given m_b = <xi^b> (binomial theorem)."""
    key = (tuple(delta), len(exps))
    if key in _SHIFT_CACHE:
        return _SHIFT_CACHE[key]
    index = {e: j for j, e in enumerate(exps)}
    S = np.zeros((len(exps), len(exps)))
    for j, a in enumerate(exps):
        for b0 in range(a[0] + 1):
            for b1 in range(a[1] + 1):
                for b2 in range(a[2] + 1):
                    c = (comb(a[0], b0) * comb(a[1], b1) * comb(a[2], b2)
                         * delta[0] ** (a[0] - b0) * delta[1] ** (a[1] - b1) * delta[2] ** (a[2] - b2))
                    S[j, index[(b0, b1, b2)]] += c
    _SHIFT_CACHE[key] = S
    return S


def _mono(xi):
    xi = np.atleast_2d(xi)
    out = np.empty((len(xi), len(MONO4)))
    for j, (a, b, c) in enumerate(MONO4):
        out[:, j] = xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c
    return out


def _mono_grad(xi):
    xi = np.atleast_2d(xi)
    out = np.zeros((len(xi), len(MONO4), 3))
    for j, e in enumerate(MONO4):
        for d in range(3):
            if e[d] == 0:
                continue
            f = list(e)
            f[d] -= 1
            out[:, j, d] = e[d] * xi[:, 0] ** f[0] * xi[:, 1] ** f[1] * xi[:, 2] ** f[2]
    return out
