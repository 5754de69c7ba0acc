"""The modified geometric multigrid of Sec. 5.3.

  SMO-1  omega-weighted Jacobi on the phi_1 unknowns, D = diag(L_11);
  SMO-2  LU-correction: phi_2 <- L_22^{-1} (r_2 - L_21 phi_1), from a
         precomputed sparse LU (SuperLU here; the ordering P does not
         change the result);
  Restrict  coarse <- 2^-3 sum of the 8 children, phi_2 residuals set to 0;
  Prolong   piecewise constant, added to phi_1 unknowns only;
  VCycle / Multigrid as in the two algorithms of Sec. 5.3, with the
  bottom level solved by a precomputed LU of the whole L^(M);
  FMG       the full-multigrid algorithm of Sec. 5 (right-hand side
            restricted level by level, coarsest level solved, then per level
            upward: interpolate and apply a fixed number of V-cycles).

Readings: each "smoother and LU-correction" application is one SMO-1
followed by one SMO-2, on every level m < M; the stopping test uses the
max norm; every level is re-discretised on the same domain; levels are
n, n/2, ... down to the first size below 2 * n_min.  FMG readings: its
Restrict acts on a right-hand side, so phi_2 children count (see
fmg_restrict); its Prolong is trilinear (fmg_prolong), since the error bound
of the FMG theorem needs an interpolation accurate to h^p, which the V-cycle's
piecewise-constant prolongation (O(h)) is not.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.sparse.linalg as spla

from .discretize import Level



@dataclasses.dataclass
class MGParams:
    omega: float = 0.8
    nu1: int = 3
    nu2: int = 3
    tol: float = 1e-10
    max_iter: int = 200


def level_sizes(n: int, n_min: int) -> List[int]:
    sizes = [n]
    while sizes[-1] % 2 == 0 and sizes[-1] // 2 >= n_min:
        sizes.append(sizes[-1] // 2)
    return sizes


class LevelOps:
    """Per-level operators used by the V-cycle."""

    def __init__(self, lev: Level, bottom: bool):
        self.lev = lev
        L = lev.L.tocsr()
        self.L = L
        m1 = lev.phi1_mask()
        self.m1 = m1
        self.i1 = np.nonzero(m1)[0]
        self.i2 = np.nonzero(~m1)[0]
        self.D = L.diagonal()
        self.bottom = bottom
        if bottom:
            self.lu_all = spla.splu(L.tocsc())
        if len(self.i2):
            self.L22 = L[self.i2][:, self.i2].tocsc()
            self.L21 = L[self.i2][:, self.i1].tocsr()
            self.lu22 = spla.splu(self.L22)

    def smo1(self, e, s, omega):
        """SMO-1: e1 <- e1 + omega D^-1 (s - L e)_1 (all phi_1 at once)."""
        res = s - self.L @ e
        out = e.copy()
        out[self.i1] += omega * res[self.i1] / self.D[self.i1]
        return out

    def smo2(self, e, s):
        """SMO-2: e2 <- L22^-1 (s2 - L21 e1)."""
        out = e.copy()
        if len(self.i2):
            b = s[self.i2] - self.L21 @ e[self.i1]
            out[self.i2] = self.lu22.solve(b)
        return out


class Hierarchy:
    def __init__(self, domain, n: int | None = None, n_min: int | None = None, theta: float = 0.1):
        n = domain.n if n is None else n
        n_min = domain.n_min if n_min is None else n_min
        self.sizes = level_sizes(n, n_min)
        self.levels = [Level(domain, m, theta) for m in self.sizes]
        self.ops = [LevelOps(lv, i == len(self.levels) - 1) for i, lv in enumerate(self.levels)]

    @property
    def fine(self) -> Level:
        return self.levels[0]

    # ------------------------------------------------------------ transfers
    def restrict(self, m: int, s_fine: np.ndarray) -> np.ndarray:
        """2^-3 sum over the 8 children; only phi_1 residuals contribute."""
        fl, cl = self.levels[m], self.levels[m + 1]
        g = np.zeros(fl.n ** 3)
        keep = fl.unknowns[fl.phi1_mask()]
        g[keep] = s_fine[fl.uidx[keep]]
        nf, nc = fl.n, cl.n
        G = g.reshape(nf, nf, nf)          # [k, j, i]
        C = 0.125 * G.reshape(nc, 2, nc, 2, nc, 2).sum(axis=(1, 3, 5))
        return C.reshape(-1)[cl.unknowns]

    def prolong_add(self, m: int, e_fine: np.ndarray, e_coarse: np.ndarray) -> np.ndarray:
        """Add the parent's value to every phi_1 unknown of the fine level."""
        fl, cl = self.levels[m], self.levels[m + 1]
        cg = cl.to_grid(e_coarse)
        nf, nc = fl.n, cl.n
        p = fl.unknowns[fl.phi1_mask()]
        i, j, k = p % nf, (p // nf) % nf, p // (nf * nf)
        parent = (i // 2) + nc * ((j // 2) + nc * (k // 2))
        out = e_fine.copy()
        out[fl.uidx[p]] += cg[parent]
        return out

    # ------------------------------------------------------------- V-cycle
    def vcycle(self, m: int, s: np.ndarray, prm: MGParams) -> np.ndarray:
        op = self.ops[m]
        if m == len(self.levels) - 1:
            return op.lu_all.solve(s)
        e = np.zeros_like(s)
        for _ in range(prm.nu1):
            e = op.smo1(e, s, prm.omega)
            e = op.smo2(e, s)
        res = s - op.L @ e
        sc = self.restrict(m, res)
        ec = self.vcycle(m + 1, sc, prm)
        e = self.prolong_add(m, e, ec)
        for _ in range(prm.nu2):
            e = op.smo1(e, s, prm.omega)
            e = op.smo2(e, s)
        return e

    # ------------------------------------------------------------- FMG
    def fmg_restrict(self, m: int, s_fine: np.ndarray) -> np.ndarray:
        """Right-hand side transfer of the FMG algorithm (Sec. 5, algorithm
        FMG): 2^-3 times the sum of s over the 8 children; children that carry
        no unknown (exterior, or absorbed into a host) count 0, and phi_2
        children count like phi_1 ones (the V-cycle's restriction drops phi_2
        children because their residual is zero after SMO-2; a right-hand side
        has no such zero)."""
        fl, cl = self.levels[m], self.levels[m + 1]
        g = np.zeros(fl.n ** 3)
        g[fl.unknowns] = s_fine
        nf, nc = fl.n, cl.n
        C = 0.125 * g.reshape(nc, 2, nc, 2, nc, 2).sum(axis=(1, 3, 5))
        return C.reshape(-1)[cl.unknowns]

    def fmg_prolong(self, m: int, x_coarse: np.ndarray) -> np.ndarray:
        """Interpolation of the FMG algorithm: trilinear in the coarse cell
        centres, over the 8 coarse cells around each fine centre that lie in
        the box and carry an unknown, with their weights renormalised (a fine
        cell whose 8 coarse cells carry none gets 0).  Exact for linear
        functions where all 8 cells are present, for constants wherever one
        is."""
        fl, cl = self.levels[m], self.levels[m + 1]
        nf, nc = fl.n, cl.n
        has = np.zeros(nc ** 3, dtype=bool)
        has[cl.unknowns] = True
        val = np.zeros(nc ** 3)
        val[cl.unknowns] = x_coarse
        out = np.zeros(fl.N)
        for q, p in enumerate(fl.unknowns):
            idx = (p % nf, (p // nf) % nf, p // (nf * nf))
            # fine centre (i + 1/2) h in coarse index units: i/2 - 1/4
            axes = []
            for i in idx:
                lo = i // 2 - 1 if i % 2 == 0 else i // 2
                t = 0.75 if i % 2 == 0 else 0.25
                axes.append(((lo, 1.0 - t), (lo + 1, t)))
            num = den = 0.0
            for kz, wz in axes[2]:
                for jy, wy in axes[1]:
                    for ix, wx in axes[0]:
                        if not (0 <= ix < nc and 0 <= jy < nc and 0 <= kz < nc):
                            continue
                        c = ix + nc * (jy + nc * kz)
                        if not has[c]:
                            continue
                        w = wx * wy * wz
                        num += w * val[c]
                        den += w
            out[q] = num / den if den > 0 else 0.0
        return out

    def fmg(self, r: np.ndarray, cycles: int, prm: MGParams = MGParams(), coarse_rhs=None) -> np.ndarray:
        """Full multigrid (Sec. 5, algorithm FMG), written as its recursion
        unrolled: each coarser level's right-hand side is coarse_rhs[m - 1]
        (the same problem discretised on that level) or, if None, the
        restriction of the finer one; the coarsest level is solved directly,
        and from the coarsest level up each level's solution is the
        interpolated coarser one improved by `cycles` V-cycles (residual on
        that level, V-cycle correction, update).  The theorem behind FMG
        assumes every level solves a discretisation of the same problem; a
        restricted right-hand side is one only when the boundary data vanish,
        since its boundary terms carry the fine level's h."""
        M = len(self.levels) - 1
        rhs = [r]
        for m in range(M):
            rhs.append(self.fmg_restrict(m, rhs[m]) if coarse_rhs is None else coarse_rhs[m])
        x = self.ops[M].lu_all.solve(rhs[M])
        for m in range(M - 1, -1, -1):
            x = self.fmg_prolong(m, x)
            for _ in range(cycles):
                x = x + self.vcycle(m, rhs[m] - self.ops[m].L @ x, prm)
        return x

    def solve(self, r: np.ndarray, prm: MGParams = MGParams(), guess=None):
        """Multigrid driver; returns (phi, history of max-norm relative residuals)."""
        L = self.ops[0].L
        phi = np.zeros_like(r) if guess is None else guess.copy()
        rn = float(np.max(np.abs(r)))
        hist = []
        for _ in range(prm.max_iter):
            s = r - L @ phi
            rel = float(np.max(np.abs(s))) / rn
            hist.append(rel)
            if rel < prm.tol:
                break
            phi = phi + self.vcycle(0, s, prm)
        return phi, hist
