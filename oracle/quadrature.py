"""High-order quadrature on boxes cut by a polynomial level set (a quadric,
or a quartic such as the torus).

The paper integrates over cut cells with surface/line-integral cubature on
its fitted boundary (Sec. 3.2).  The domains here are exact quadrics, so
the cut-cell integrals are computed with the dimension-recursive
height-function scheme of R. Saye, "High-order quadrature methods for
implicitly defined surfaces and volumes in hyperrectangles", SIAM J. Sci.
Comput. 37 (2015) A993-A1019, restated in our own terms:

  * a quadratic phi(x) = x^T Q x + b^T x + c, or a polynomial of degree <= 4,
    is given on a box;
  * if bounds prove phi has one sign on the box, the box is all-in or all-out;
  * otherwise pick the height axis k maximising |d phi/dx_k| at the centre;
    if d phi/dx_k may vanish on the box, bisect the box (depth-limited);
  * the box is then the graph domain of the single root of phi along k; the
    integral over the (e-1)-dimensional base is itself computed by the same
    scheme, with the restrictions of phi to the two k-faces as the functions
    across whose zero sets the base integrand has kinks;
  * along each base line the interval is cut at the roots and each piece
    gets a q-point Gauss-Legendre rule.

Bounds of a polynomial p on a box come from its Taylor expansion at the box
centre in the scaled variables t (x = m + w t, |t_i| <= 1):
p = sum_a d_a t^a, so |p - d_0| <= sum_{a != 0} |d_a|; for a quadric this is
exactly the bound written out below for Quadric.  Roots along a line: a
quadric's in closed form; a general polynomial's are bracketed between the
roots of its derivative (recursively) and found by bisection.

Every decision (height axis, bisection, inclusion) is fixed by rules stated
in this file so that an independent implementation makes the same ones.
"""
from __future__ import annotations

import numpy as np

MAX_DEPTH = 12          # bisection limit per recursion dimension
POLY_SPLIT_DEPTH = 4    # the same limit in split_rule when a live function is a
                        # polynomial: a face plane tangent to a torus along a
                        # whole circle leaves a double zero there that no box
                        # bound can separate, and bisecting along it to depth
                        # 12 costs ~2^12 boxes; transversal zero sets of the
                        # torus resolve by depth 1
TIE = 1e-12             # relative tie tolerance in axis selection
_GL = {}


def gauss(q: int):
    if q not in _GL:
        _GL[q] = np.polynomial.legendre.leggauss(q)
    return _GL[q]


class Quadric:
    """phi(x) = x^T Q x + b^T x + c in e variables."""
    __slots__ = ("Q", "b", "c")

    def __init__(self, Q, b, c):
        self.Q = np.asarray(Q, float)
        self.b = np.asarray(b, float)
        self.c = float(c)

    @property
    def dim(self):
        return len(self.b)

    def __call__(self, X):
        X = np.atleast_2d(X)
        return np.einsum("pi,ij,pj->p", X, self.Q, X) + X @ self.b + self.c

    def grad(self, X):
        X = np.atleast_2d(X)
        return 2.0 * X @ self.Q + self.b[None, :]

    def restrict(self, k: int, val: float) -> "Quadric":
        keep = [i for i in range(self.dim) if i != k]
        Q = self.Q[np.ix_(keep, keep)]
        b = self.b[keep] + 2.0 * self.Q[k, keep] * val
        c = self.c + self.b[k] * val + self.Q[k, k] * val * val
        return Quadric(Q, b, c)


def ellipsoid_quadric(center, axes, rot) -> Quadric:
    """(x-c)^T A (x-c) - 1 with A = R diag(1/a^2) R^T; positive outside."""
    R = np.asarray(rot, float)
    A = R @ np.diag(1.0 / np.asarray(axes, float) ** 2) @ R.T
    c = np.asarray(center, float)
    return Quadric(A, -2.0 * A @ c, float(c @ A @ c) - 1.0)


DEG = 4                  # polynomial level sets: total degree at most 4


def _binom(n, k):
    from math import comb
    return comb(n, k)


class Poly:
    """p(x) = sum_a C[a] x^a over exponents a with |a| <= 4 in e variables;
    C is a dense array of shape (5,) * e (entries of degree > 4 are 0)."""
    __slots__ = ("C",)

    def __init__(self, C):
        self.C = np.asarray(C, float)

    @property
    def dim(self):
        return self.C.ndim

    @staticmethod
    def const(v, e):
        C = np.zeros((DEG + 1,) * e)
        C[(0,) * e] = v
        return Poly(C)

    @staticmethod
    def coord(i, e, shift=0.0):
        """x_i - shift."""
        C = np.zeros((DEG + 1,) * e)
        C[(0,) * e] = -shift
        idx = [0] * e
        idx[i] = 1
        C[tuple(idx)] = 1.0
        return Poly(C)

    def __add__(self, o):
        return Poly(self.C + (o.C if isinstance(o, Poly) else Poly.const(o, self.dim).C))

    def __sub__(self, o):
        return Poly(self.C - (o.C if isinstance(o, Poly) else Poly.const(o, self.dim).C))

    def __rmul__(self, a):
        return Poly(a * self.C)

    def __mul__(self, o):
        if not isinstance(o, Poly):
            return Poly(o * self.C)
        out = np.zeros_like(self.C)
        for a in zip(*np.nonzero(self.C)):
            for b in zip(*np.nonzero(o.C)):
                c = tuple(x + y for x, y in zip(a, b))
                if sum(c) > DEG:
                    raise ValueError("degree above 4")
                out[c] += self.C[a] * o.C[b]
        return Poly(out)

    def _powers(self, X):
        X = np.atleast_2d(np.asarray(X, float))
        return [X[:, i][:, None] ** np.arange(DEG + 1)[None, :] for i in range(self.dim)]

    def __call__(self, X):
        P = self._powers(X)
        e = self.dim
        if e == 0:
            return np.full(len(np.atleast_2d(X)), float(self.C))
        letters = "abc"[:e]
        spec = letters + "," + ",".join("p" + l for l in letters) + "->p"
        return np.einsum(spec, self.C, *P)

    def deriv(self, k):
        e = self.dim
        D = np.zeros_like(self.C)
        for a in range(1, DEG + 1):
            src = [slice(None)] * e
            dst = [slice(None)] * e
            src[k] = a
            dst[k] = a - 1
            D[tuple(dst)] = a * self.C[tuple(src)]
        return Poly(D)

    def grad(self, X):
        return np.stack([self.deriv(k)(X) for k in range(self.dim)], axis=1)

    def restrict(self, k, val):
        w = float(val) ** np.arange(DEG + 1)
        return Poly(np.tensordot(self.C, w, axes=([k], [0])))

    def taylor(self, m, w):
        """Coefficients d of p(m + w t) in t (same layout as C)."""
        D = self.C
        for i in range(self.dim):
            T = np.zeros((DEG + 1, DEG + 1))     # T[a, b]: x^a -> t^b
            for a_ in range(DEG + 1):
                for b_ in range(a_ + 1):
                    T[a_, b_] = _binom(a_, b_) * float(m[i]) ** (a_ - b_) * float(w[i]) ** b_
            D = np.moveaxis(np.tensordot(D, T, axes=([i], [0])), -1, i)
        return D

    def bounds(self, lo, hi):
        """(value at the centre, bound of |p - value| on the box)."""
        m = 0.5 * (np.asarray(lo, float) + np.asarray(hi, float))
        w = 0.5 * (np.asarray(hi, float) - np.asarray(lo, float))
        d = self.taylor(m, w)
        c0 = float(d[(0,) * self.dim])
        return c0, float(np.sum(np.abs(d))) - abs(c0)

    def line(self, k, Xo):
        """Coefficients (P, 5) of p along x_k at base points Xo (P, e-1):
        p = sum_j a_j x_k^j."""
        e = self.dim
        keep = [i for i in range(e) if i != k]
        Ck = np.moveaxis(self.C, k, -1)                  # (..., 5) with x_k last
        Xo = np.atleast_2d(Xo)
        out = np.empty((len(Xo), DEG + 1))
        for j in range(DEG + 1):
            out[:, j] = Poly(Ck[..., j])(Xo) if e > 1 else float(Ck[j])
        return out


def poly_from_quadric(q: "Quadric") -> Poly:
    e = q.dim
    p = Poly.const(q.c, e)
    for i in range(e):
        p = p + q.b[i] * Poly.coord(i, e)
        for j in range(e):
            p = p + q.Q[i, j] * (Poly.coord(i, e) * Poly.coord(j, e))
    return p


def torus_poly(center, R: float, r: float, rot) -> Poly:
    """(|x-c|^2 + R^2 - r^2)^2 - 4 R^2 rho^2 with rho the distance of x from the
    torus axis, the line through c along the third column of rot: negative
    inside the tube of radius r around the circle of radius R, positive
    outside.  (It factors as ((rho - R)^2 + z^2 - r^2) ((rho + R)^2 + z^2 - r^2),
    z the coordinate along the axis, and the second factor is positive when
    r < R.)"""
    rot = np.asarray(rot, float)
    d = [Poly.coord(j, 3, center[j]) for j in range(3)]
    u = []
    for i in range(3):
        ui = Poly.const(0.0, 3)
        for j in range(3):
            ui = ui + rot[j, i] * d[j]
        u.append(ui)
    rho2 = u[0] * u[0] + u[1] * u[1]
    T = rho2 + u[2] * u[2] + (R * R - r * r)
    return T * T - (4.0 * R * R) * rho2


def _eval1(a, t):
    """sum_j a_j t^j by Horner's rule."""
    v = 0.0
    for c in a[::-1]:
        v = v * t + c
    return v


def _poly1_roots(a, lo, hi):
    """Roots strictly inside (lo, hi) at which the univariate polynomial
    sum_j a_j t^j changes sign: the roots of its derivative cut the interval
    into pieces on which it is monotone; a piece whose ends differ in sign
    holds one root, found by bisection."""
    a = np.asarray(a, float)
    nz = np.nonzero(a)[0]
    deg = int(nz[-1]) if len(nz) else 0
    if deg == 0:
        return []
    if deg == 1:
        t = -a[0] / a[1]
        return [t] if lo < t < hi else []
    da = np.array([j * a[j] for j in range(1, deg + 1)])
    cuts = [lo] + _poly1_roots(da, lo, hi) + [hi]
    out = []
    for x0, x1 in zip(cuts[:-1], cuts[1:]):
        f0, f1 = _eval1(a, x0), _eval1(a, x1)
        if f0 != 0.0 and f1 != 0.0 and (f0 < 0) != (f1 < 0):
            out.append(float(_monotone_root(a[None, :deg + 1], x0, x1)[0]))
    return out


def _monotone_root(coef, lo, hi):
    """The root in (lo, hi) of univariate polynomials (rows of coef, lowest
    power first) that are monotone on the interval, by bisection to the last
    bit; NaN where the two ends do not differ in sign."""
    P, D = coef.shape

    def ev(t):
        v = coef[:, D - 1].copy()
        for j in range(D - 2, -1, -1):
            v = v * t + coef[:, j]
        return v
    a = np.full(P, float(lo))
    b = np.full(P, float(hi))
    fa, fb = ev(a), ev(b)
    ok = (fa < 0) != (fb < 0)
    ok &= (fa != 0) & (fb != 0)
    for _ in range(1100):       # halving a double interval ends in far fewer steps
        m = 0.5 * (a + b)
        done = (m <= a) | (m >= b)
        if np.all(done | ~ok):
            break
        fm = ev(m)
        same = (fm < 0) == (fa < 0)
        a = np.where(same & ~done, m, a)
        fa = np.where(same & ~done, fm, fa)
        b = np.where(~same & ~done, m, b)
    r = 0.5 * (a + b)
    return np.where(ok, r, np.nan)


def box_sign(f, lo, hi) -> int:
    """+1 / -1 if f provably has that sign on the box, else 0."""
    if isinstance(f, Poly):
        v, spread = f.bounds(lo, hi)
        return 1 if v - spread > 0 else (-1 if v + spread < 0 else 0)
    m = 0.5 * (lo + hi)
    w = 0.5 * (hi - lo)
    v = float(f(m)[0])
    g = f.grad(m)[0]
    spread = float(np.sum(np.abs(g) * w) + w @ np.abs(f.Q) @ w)
    if v - spread > 0:
        return 1
    if v + spread < 0:
        return -1
    return 0


def monotone(f, k: int, lo, hi) -> bool:
    """True if d f / d x_k cannot vanish on the box (for a quadric it is
    affine in x; for a polynomial its Taylor bound decides)."""
    if isinstance(f, Poly):
        v, spread = f.deriv(k).bounds(lo, hi)
        return abs(v) > spread
    m = 0.5 * (lo + hi)
    w = 0.5 * (hi - lo)
    dk = float(f.grad(m)[0][k])
    return abs(dk) > float(np.sum(np.abs(2.0 * f.Q[k, :]) * w))


SLOPE = 4.0             # height-function slope bound for the top level


def graph_ok(f, k: int, lo, hi) -> bool:
    """Top-level test: |d f/dx_k| >= |grad f| / SLOPE everywhere on the box,
    from bounds of each derivative (affine for a quadric, Taylor for a
    polynomial), so the zero set is a graph over the k-face with bounded
    slope."""
    if isinstance(f, Poly):
        b = [f.deriv(i).bounds(lo, hi) for i in range(f.dim)]
        low_k = abs(b[k][0]) - b[k][1]
        up_g = float(np.sqrt(sum((abs(v) + s_) ** 2 for v, s_ in b)))
        return low_k > 0 and SLOPE * low_k >= up_g
    m = 0.5 * (lo + hi)
    w = 0.5 * (hi - lo)
    g = f.grad(m)[0]
    spread = np.abs(2.0 * f.Q) @ w
    low_k = abs(float(g[k])) - float(spread[k])
    up_g = float(np.sqrt(np.sum((np.abs(g) + spread) ** 2)))
    return low_k > 0 and SLOPE * low_k >= up_g


def choose_axis(funcs, lo, hi) -> int:
    m = 0.5 * (lo + hi)
    score = np.zeros(len(lo))
    for f in funcs:
        g = f.grad(m)[0]
        nrm = float(np.sqrt(g @ g))
        if nrm > 0:
            score += np.abs(g) / nrm
    best = float(np.max(score))
    for k in range(len(lo)):
        if score[k] >= best * (1.0 - TIE):
            return k
    return 0


def tensor_gauss(lo, hi, q):
    x, w = gauss(q)
    e = len(lo)
    pts = [0.5 * (lo[i] + hi[i]) + 0.5 * (hi[i] - lo[i]) * x for i in range(e)]
    wts = [0.5 * (hi[i] - lo[i]) * w for i in range(e)]
    grids = np.meshgrid(*pts, indexing="ij")
    wgrid = np.ones_like(grids[0])
    for i, wi in enumerate(wts):
        shape = [1] * e
        shape[i] = q
        wgrid = wgrid * wi.reshape(shape)
    return np.stack([g.ravel() for g in grids], axis=1), wgrid.ravel()


def _line_coeffs(f: Quadric, k: int, Xo: np.ndarray):
    """f along x_k at base points Xo (P, e-1): alpha t^2 + beta t + gamma."""
    keep = [i for i in range(f.dim) if i != k]
    Qr = f.Q[np.ix_(keep, keep)]
    alpha = np.full(len(Xo), f.Q[k, k])
    beta = 2.0 * Xo @ f.Q[keep, k] + f.b[k]
    gamma = np.einsum("pi,ij,pj->p", Xo, Qr, Xo) + Xo @ f.b[keep] + f.c
    return alpha, beta, gamma


def quad_roots(alpha, beta, gamma, lo, hi):
    """Real roots of alpha t^2 + beta t + gamma strictly inside (lo, hi);
    returns (P, 2) with NaN where absent."""
    P = len(beta)
    r = np.full((P, 2), np.nan)
    lin = np.abs(alpha) <= 1e-300
    with np.errstate(invalid="ignore", divide="ignore"):
        # linear case
        rl = -gamma / beta
        r[:, 0] = np.where(lin & (beta != 0), rl, np.nan)
        disc = beta * beta - 4.0 * alpha * gamma
        sq = np.sqrt(np.where(disc >= 0, disc, 0.0))
        qq = -0.5 * (beta + np.where(beta >= 0, sq, -sq))
        r1 = qq / alpha
        r2 = gamma / qq
        quad_ok = (~lin) & (disc >= 0)
        r[:, 0] = np.where(quad_ok, r1, r[:, 0])
        r[:, 1] = np.where(quad_ok & (qq != 0), r2, np.nan)
        lo_a = np.broadcast_to(lo, (P,))
        hi_a = np.broadcast_to(hi, (P,))
        inside = (r > lo_a[:, None]) & (r < hi_a[:, None])
    r[~inside] = np.nan
    return r


def line_roots(f, k: int, Xo: np.ndarray, lo_k, hi_k):
    """Roots of f along x_k inside (lo_k, hi_k) at base points Xo, where f is
    known to be monotone along x_k: (P, 2) for a quadric (closed form), (P, 1)
    for a polynomial (bisection); NaN where absent."""
    if isinstance(f, Poly):
        return _monotone_root(f.line(k, Xo), lo_k, hi_k)[:, None]
    al, be, ga = _line_coeffs(f, k, Xo)
    return quad_roots(al, be, ga, lo_k, hi_k)


def interval_roots(f, lo, hi):
    """All sign-changing roots inside (lo, hi) of a function of one variable."""
    if isinstance(f, Poly):
        return np.array(_poly1_roots(f.C, lo, hi) or [np.nan])
    return quad_roots(np.array([f.Q[0, 0]]), np.array([f.b[0]]), np.array([f.c]), lo, hi)[0]


def _segments(Wo, Xo, k, lo_k, hi_k, roots, q, e):
    """Cut [lo_k, hi_k] at the given roots for every base point; q-point rule
    on each piece.  Returns X (M, e), W (M,), and the piece index of each node."""
    P = len(Xo)
    br = np.concatenate([np.full((P, 1), lo_k), np.where(np.isnan(roots), hi_k, roots),
                         np.full((P, 1), hi_k)], axis=1)
    br = np.sort(br, axis=1)
    a, b = br[:, :-1], br[:, 1:]
    x, w = gauss(q)
    mid = 0.5 * (a + b)
    half = 0.5 * (b - a)
    t = mid[:, :, None] + half[:, :, None] * x[None, None, :]          # (P, S, q)
    wt = Wo[:, None, None] * half[:, :, None] * w[None, None, :]
    S = a.shape[1]
    Xb = np.repeat(Xo[:, None, None, :], S, axis=1)
    Xb = np.repeat(Xb, q, axis=2)
    X = np.empty((P, S, q, e))
    keep = [i for i in range(e) if i != k]
    X[..., keep] = Xb
    X[..., k] = t
    return X.reshape(-1, e), wt.reshape(-1), mid, half


def split_rule(lo, hi, funcs, q, depth=0):
    """Nodes/weights on a box for integrands smooth away from the zero sets
    of `funcs` (every piece is included)."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    e = len(lo)
    live = [f for f in funcs if box_sign(f, lo, hi) == 0]
    if not live:
        return tensor_gauss(lo, hi, q)
    if e == 1:
        roots = np.concatenate([interval_roots(f, lo[0], hi[0]) for f in live])[None, :]
        X, W, _, half = _segments(np.ones(1), np.zeros((1, 0)), 0, lo[0], hi[0], roots, q, 1)
        keep = W != 0
        return X[keep], W[keep]
    k = choose_axis(live, lo, hi)
    if not all(monotone(f, k, lo, hi) for f in live):
        limit = POLY_SPLIT_DEPTH if any(isinstance(f, Poly) for f in live) else MAX_DEPTH
        if depth < limit:
            return _bisect(lo, hi, lambda a, b: split_rule(a, b, funcs, q, depth + 1))
        live = [f for f in live if monotone(f, k, lo, hi)]
        if not live:
            return tensor_gauss(lo, hi, q)
    keep = [i for i in range(e) if i != k]
    faces = []
    for f in live:
        faces.append(f.restrict(k, lo[k]))
        faces.append(f.restrict(k, hi[k]))
    Xo, Wo = split_rule(lo[keep], hi[keep], faces, q, 0)
    roots = np.concatenate([line_roots(f, k, Xo, lo[k], hi[k]) for f in live], axis=1)
    X, W, _, _ = _segments(Wo, Xo, k, lo[k], hi[k], roots, q, e)
    nz = W != 0
    return X[nz], W[nz]


def _bisect(lo, hi, fn):
    e = len(lo)
    mid = 0.5 * (lo + hi)
    Xs, Ws = [], []
    for code in range(1 << e):
        a = lo.copy()
        b = hi.copy()
        for i in range(e):
            if (code >> i) & 1:
                a[i] = mid[i]
            else:
                b[i] = mid[i]
        X, W = fn(a, b)
        Xs.append(X)
        Ws.append(W)
    return np.concatenate(Xs), np.concatenate(Ws)


def _empty(e):
    return np.zeros((0, e)), np.zeros(0)


def region_rules(lo, hi, psi, q: int, depth: int = 0):
    """Quadrature for {psi > 0} inside the box and for the surface {psi = 0}.

    Returns ((Xv, Wv), (Xs, Ws, Ns)): volume nodes/weights; surface nodes,
    weights (area element) and unit normals pointing out of {psi > 0}."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    e = len(lo)
    es = (np.zeros((0, e)), np.zeros(0), np.zeros((0, e)))
    s = box_sign(psi, lo, hi)
    if s > 0:
        return tensor_gauss(lo, hi, q), es
    if s < 0:
        return _empty(e), es
    m = 0.5 * (lo + hi)
    g = np.abs(psi.grad(m)[0])
    best = float(np.max(g))
    k = next(i for i in range(e) if g[i] >= best * (1.0 - TIE))
    if not graph_ok(psi, k, lo, hi):
        if depth < MAX_DEPTH:
            parts = []
            mid = 0.5 * (lo + hi)
            for code in range(1 << e):
                a = lo.copy()
                b = hi.copy()
                for i in range(e):
                    if (code >> i) & 1:
                        a[i] = mid[i]
                    else:
                        b[i] = mid[i]
                parts.append(region_rules(a, b, psi, q, depth + 1))
            vol = (np.concatenate([p[0][0] for p in parts]), np.concatenate([p[0][1] for p in parts]))
            sur = tuple(np.concatenate([p[1][j] for p in parts]) for j in range(3))
            return vol, sur
        if float(psi(m)[0]) > 0:
            return tensor_gauss(lo, hi, q), es
        return _empty(e), es
    keep = [i for i in range(e) if i != k]
    faces = [psi.restrict(k, lo[k]), psi.restrict(k, hi[k])]
    Xo, Wo = split_rule(lo[keep], hi[keep], faces, q, 0)
    roots = line_roots(psi, k, Xo, lo[k], hi[k])
    # psi is monotone along x_k here: at most one root on the interval
    root = roots[:, 0] if roots.shape[1] == 1 else np.where(np.isnan(roots[:, 0]), roots[:, 1], roots[:, 0])
    X, W, mid, half = _segments(Wo, Xo, k, lo[k], hi[k], root[:, None], q, e)
    P, S = mid.shape
    Xm = np.empty((P, S, e))
    Xm[..., keep] = Xo[:, None, :]
    Xm[..., k] = mid
    inside = (psi(Xm.reshape(-1, e)) > 0).reshape(P, S)
    incl = np.repeat(inside[:, :, None], q, axis=2).reshape(-1)
    sel = incl & (W != 0)
    Xv, Wv = X[sel], W[sel]
    has = ~np.isnan(root)
    Xs = np.empty((int(has.sum()), e))
    Xs[:, keep] = Xo[has]
    Xs[:, k] = root[has]
    G = psi.grad(Xs)
    gn = np.sqrt(np.sum(G * G, axis=1))
    Ws = Wo[has] * gn / np.abs(G[:, k])
    Ns = -G / gn[:, None]
    return (Xv, Wv), (Xs, Ws, Ns)
