"""Local Fourier analysis (LFA) of the obstacle-free V-cycle.

A test helper, independent of the oracle: it never imports `oracle`.  On an
infinite (periodic) grid with no obstacles every unknown is a regular cell, the
LU-correction is empty and the V-cycle of Sec. 5.3 is built from four
translation-invariant pieces whose Fourier symbols are written out here from
the paper's formulas:

  * the cell-averaged fourth-order Laplacian (Sec. 2.3, the regular
    discretisation): per axis (-1, 16, -30, 16, -1) / (12 h^2), so for the
    mode exp(i theta . j) the symbol is
        sum_d (-2 cos 2 theta_d + 32 cos theta_d - 30) / (12 h^2);
  * SMO-1, omega-weighted Jacobi with the row diagonal -90 / (12 h^2):
        S(theta) = 1 - omega L(theta) / D;
  * restriction, 2^-3 times the sum of the 8 children: the fine mode theta
    lands on the coarse frequency 2 theta with the factor
        r(theta) = 2^-3 prod_d (1 + exp(i theta_d));
  * prolongation, piecewise constant (each child receives its parent's
    value): the coarse mode Theta excites the 8 fine harmonics
    theta = Theta / 2 + pi alpha, alpha in {0, 1}^3, with the factors
    conj(r(theta)).

Each level is re-discretised (coarse symbol with spacing 2h) and the coarsest
level is solved exactly.  For one frequency Theta_M of the coarsest level the
8^(M) fine harmonics that alias to it form an invariant subspace; on it the
V-cycle error propagation is the matrix

    E_l = S_l^nu2 (I - P_l (I - E_{l+1}) L_{l+1}^{-1} R_l L_l) S_l^nu1,
    E_M = 0,

and the asymptotic convergence factor is the largest spectral radius of E_0
over the sampled Theta_M.
"""
from __future__ import annotations

import itertools

import numpy as np

ALPHAS = np.array(list(itertools.product((0, 1), repeat=3)), dtype=float)   # (8, 3)


def laplacian_symbol(theta: np.ndarray, h: float) -> np.ndarray:
    """Symbol of the regular fourth-order cell-average Laplacian."""
    t = np.asarray(theta, dtype=float)
    return np.sum(-2.0 * np.cos(2.0 * t) + 32.0 * np.cos(t) - 30.0, axis=-1) / (12.0 * h * h)


def restriction_symbol(theta: np.ndarray) -> np.ndarray:
    """Factor of the 2^-3 children sum on the fine mode theta."""
    return np.prod(1.0 + np.exp(1j * np.asarray(theta, dtype=float)), axis=-1) / 8.0


def _alias_classes(theta_coarsest: np.ndarray, levels: int):
    """Frequencies of each level (finest first) that alias to theta_coarsest;
    entry i of level l has its parent at index i // 8 on level l + 1."""
    sets = [np.asarray(theta_coarsest, dtype=float)[None, :]]
    for _ in range(levels - 1):
        coarse = sets[0]
        fine = (coarse[:, None, :] / 2.0 + np.pi * ALPHAS[None, :, :]).reshape(-1, 3)
        sets.insert(0, fine)
    return sets


def vcycle_block(theta_coarsest, levels: int, h: float, omega: float, nu1: int, nu2: int) -> np.ndarray:
    """Error propagation matrix of the `levels`-level V-cycle on the alias class
    of theta_coarsest (finest-level harmonics, 8^(levels-1) of them)."""
    sets = _alias_classes(theta_coarsest, levels)
    M = levels - 1
    E = np.zeros((1, 1), dtype=complex)
    for lv in range(M - 1, -1, -1):
        f = sets[lv]
        c = sets[lv + 1]
        hl = h * 2.0 ** lv
        K, Kc = len(f), len(c)
        Lf = laplacian_symbol(f, hl)
        Lc = laplacian_symbol(c, 2.0 * hl)
        D = -90.0 / (12.0 * hl * hl)
        S = 1.0 - omega * Lf / D
        r = restriction_symbol(f)
        parent = np.arange(K) // 8
        R = np.zeros((Kc, K), dtype=complex)
        R[parent, np.arange(K)] = r
        P = np.zeros((K, Kc), dtype=complex)
        P[np.arange(K), parent] = np.conj(r)
        coarse_solve = (np.eye(Kc) - E) / Lc[:, None]
        cgc = np.eye(K) - P @ coarse_solve @ R * Lf[None, :]
        E = (S ** nu2)[:, None] * cgc * (S ** nu1)[None, :]
    return E


def vcycle_factor(levels: int, omega: float, nu1: int = 3, nu2: int = 3, samples: int = 5,
                  h: float = 1.0) -> float:
    """Largest spectral radius of the V-cycle block over coarsest-level
    frequencies Theta in [0, pi]^3 on a grid of `samples` points per axis.

    Symmetries reduce the search: reflecting an axis about a cell face
    (j -> -1 - j) maps every 2-cell coarsening pair onto another one, so the
    cycle commutes with it and theta_d -> -theta_d leaves the spectrum alone;
    permuting the axes does too, so only Theta_x <= Theta_y <= Theta_z is
    sampled.  Theta = 0 (the constant, singular on the periodic grid) is
    replaced by its limit (1e-3, 0, 0).  The factor does not depend on h
    (every symbol scales with 1/h^2)."""
    g = np.linspace(0.0, np.pi, samples)
    worst = 0.0
    for a, b, c in itertools.combinations_with_replacement(range(samples), 3):
        t = np.array([g[a], g[b], g[c]])
        if not np.any(t):
            t[0] = 1e-3
        E = vcycle_block(t, levels, h, omega, nu1, nu2)
        worst = max(worst, float(np.max(np.abs(np.linalg.eigvals(E)))))
    return worst


def smoothing_factor(omega: float, samples: int = 16) -> float:
    """max |S(theta)| over the high frequencies (max_d |theta_d| >= pi / 2) on a
    grid of 4 samples + 1 points per axis in [-pi, pi] (pi / 2 and pi included)."""
    g = np.linspace(-np.pi, np.pi, 4 * samples + 1)
    T = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    high = np.max(np.abs(T), axis=1) >= np.pi / 2 - 1e-12
    S = 1.0 - omega * laplacian_symbol(T[high], 1.0) / (-90.0 / 12.0)
    return float(np.max(np.abs(S)))
