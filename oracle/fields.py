"""Analytic fields: pointwise value, gradient, Laplacian and exact averages.

Averages over axis-aligned boxes and faces use closed-form primitives of
the separable factors (the definition of a cell average, Sec. 2.3), written
in cancellation-free forms.  Polynomials use a 3-point Gauss-Legendre
product rule, which is exact for degree <= 5.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf, erfc

_GL3 = np.polynomial.legendre.leggauss(3)


class Field:
    def __init__(self, desc: dict):
        self.desc = desc
        self.kind = desc["kind"]

    # ------------------------------------------------------------ points
    def value(self, X: np.ndarray) -> np.ndarray:
        X = np.atleast_2d(X)
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        d = self.desc
        k = self.kind
        if k == "zero":
            return np.zeros(len(X))
        if k == "poly":
            out = np.zeros(len(X))
            for a, b, c, v in d["terms"]:
                out += v * x ** a * y ** b * z ** c
            return out
        if k == "sinprod":
            kk, p = d["k"], d["p"]
            return d["amp"] * np.sin(kk[0] * x + p[0]) * np.sin(kk[1] * y + p[1]) * np.sin(kk[2] * z + p[2])
        if k == "expcos":
            return d["amp"] * np.exp(d["a"] * x + d["b"] * y) * np.cos(d["c"] * z + d["p"])
        if k == "gauss":
            out = np.zeros(len(X))
            for A, mu, s in zip(d["amp"], d["mu"], d["sigma"]):
                r2 = (x - mu[0]) ** 2 + (y - mu[1]) ** 2 + (z - mu[2]) ** 2
                out += A * np.exp(-r2 / (2 * s * s))
            return out
        if k == "xsinexp":
            return d["amp"] * x * np.sin(y) * np.exp(z)
        raise ValueError(k)

    def grad(self, X: np.ndarray) -> np.ndarray:
        X = np.atleast_2d(X)
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        d = self.desc
        k = self.kind
        G = np.zeros((len(X), 3))
        if k == "zero":
            return G
        if k == "poly":
            for a, b, c, v in d["terms"]:
                if a:
                    G[:, 0] += v * a * x ** (a - 1) * y ** b * z ** c
                if b:
                    G[:, 1] += v * b * x ** a * y ** (b - 1) * z ** c
                if c:
                    G[:, 2] += v * c * x ** a * y ** b * z ** (c - 1)
            return G
        if k == "sinprod":
            kk, p, A = d["k"], d["p"], d["amp"]
            s = [np.sin(kk[i] * X[:, i] + p[i]) for i in range(3)]
            co = [np.cos(kk[i] * X[:, i] + p[i]) for i in range(3)]
            G[:, 0] = A * kk[0] * co[0] * s[1] * s[2]
            G[:, 1] = A * kk[1] * s[0] * co[1] * s[2]
            G[:, 2] = A * kk[2] * s[0] * s[1] * co[2]
            return G
        if k == "expcos":
            e = d["amp"] * np.exp(d["a"] * x + d["b"] * y)
            G[:, 0] = d["a"] * e * np.cos(d["c"] * z + d["p"])
            G[:, 1] = d["b"] * e * np.cos(d["c"] * z + d["p"])
            G[:, 2] = -d["c"] * e * np.sin(d["c"] * z + d["p"])
            return G
        if k == "gauss":
            for A, mu, s in zip(d["amp"], d["mu"], d["sigma"]):
                dx = X - np.asarray(mu)[None, :]
                g = A * np.exp(-np.sum(dx * dx, axis=1) / (2 * s * s))
                G += (-dx / (s * s)) * g[:, None]
            return G
        if k == "xsinexp":
            A = d["amp"]
            G[:, 0] = A * np.sin(y) * np.exp(z)
            G[:, 1] = A * x * np.cos(y) * np.exp(z)
            G[:, 2] = A * x * np.sin(y) * np.exp(z)
            return G
        raise ValueError(k)

    def laplacian_desc(self) -> "Field":
        """The Laplacian as a field, where it stays in a closed family."""
        d = self.desc
        k = self.kind
        if k == "zero":
            return Field(d)
        if k == "sinprod":
            s = sum(v * v for v in d["k"])
            return Field(dict(d, amp=-s * d["amp"]))
        if k == "expcos":
            s = d["a"] ** 2 + d["b"] ** 2 - d["c"] ** 2
            return Field(dict(d, amp=s * d["amp"]))
        if k == "poly":
            acc = {}
            for a, b, c, v in d["terms"]:
                for e, (da, db, dc) in ((a, (2, 0, 0)), (b, (0, 2, 0)), (c, (0, 0, 2))):
                    if e >= 2:
                        key = (a - da, b - db, c - dc)
                        acc[key] = acc.get(key, 0.0) + v * e * (e - 1)
            return Field({"kind": "poly", "terms": [(*kk, v) for kk, v in acc.items()]})
        if k == "gauss":
            return _GaussLaplacian(d)
        if k == "xsinexp":                     # x sin(y) e^z is harmonic
            return Field({"kind": "zero"})
        raise ValueError(k)

    def laplacian(self, X):
        return self.laplacian_desc().value(X)

    # --------------------------------------------------------- averages
    def box_average(self, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
        """Exact average over boxes [lo, hi] (arrays (P,3)); degenerate axes
        (lo == hi) are treated as point evaluations along that axis, which
        gives face averages."""
        lo = np.atleast_2d(lo).astype(float)
        hi = np.atleast_2d(hi).astype(float)
        d = self.desc
        k = self.kind
        if k == "zero":
            return np.zeros(len(lo))
        if k == "poly":
            return _poly_box_average(d["terms"], lo, hi)
        if k == "sinprod":
            out = np.full(len(lo), d["amp"])
            for i in range(3):
                out *= _avg_sin(d["k"][i], d["p"][i], lo[:, i], hi[:, i])
            return out
        if k == "expcos":
            return (d["amp"] * _avg_exp(d["a"], lo[:, 0], hi[:, 0]) * _avg_exp(d["b"], lo[:, 1], hi[:, 1])
                    * _avg_cos(d["c"], d["p"], lo[:, 2], hi[:, 2]))
        if k == "gauss":
            out = np.zeros(len(lo))
            for A, mu, s in zip(d["amp"], d["mu"], d["sigma"]):
                t = np.full(len(lo), A)
                for i in range(3):
                    t *= _avg_gauss(mu[i], s, lo[:, i], hi[:, i])
                out += t
            return out
        if k == "xsinexp":
            return (d["amp"] * 0.5 * (lo[:, 0] + hi[:, 0]) * _avg_sin(1.0, 0.0, lo[:, 1], hi[:, 1])
                    * _avg_exp(1.0, lo[:, 2], hi[:, 2]))
        raise ValueError(k)

    def box_average_grad(self, lo, hi, axis: int) -> np.ndarray:
        """Exact average of d(phi)/dx_axis over boxes/faces."""
        lo = np.atleast_2d(lo).astype(float)
        hi = np.atleast_2d(hi).astype(float)
        d = self.desc
        k = self.kind
        if k == "zero":
            return np.zeros(len(lo))
        if k == "poly":
            terms = []
            for a, b, c, v in d["terms"]:
                e = (a, b, c)
                if e[axis] == 0:
                    continue
                ee = list(e)
                ee[axis] -= 1
                terms.append((*ee, v * e[axis]))
            return _poly_box_average(terms, lo, hi)
        if k == "sinprod":
            out = np.full(len(lo), d["amp"] * d["k"][axis])
            for i in range(3):
                if i == axis:
                    out *= _avg_cos(d["k"][i], d["p"][i], lo[:, i], hi[:, i])
                else:
                    out *= _avg_sin(d["k"][i], d["p"][i], lo[:, i], hi[:, i])
            return out
        if k == "expcos":
            fx = _avg_exp(d["a"], lo[:, 0], hi[:, 0])
            fy = _avg_exp(d["b"], lo[:, 1], hi[:, 1])
            if axis == 2:
                fz = -d["c"] * _avg_sin(d["c"], d["p"], lo[:, 2], hi[:, 2])
            else:
                fz = _avg_cos(d["c"], d["p"], lo[:, 2], hi[:, 2])
            if axis == 0:
                fx = d["a"] * fx
            if axis == 1:
                fy = d["b"] * fy
            return d["amp"] * fx * fy * fz
        if k == "gauss":
            out = np.zeros(len(lo))
            for A, mu, s in zip(d["amp"], d["mu"], d["sigma"]):
                t = np.full(len(lo), A)
                for i in range(3):
                    if i == axis:
                        t *= _avg_gauss_d1(mu[i], s, lo[:, i], hi[:, i])
                    else:
                        t *= _avg_gauss(mu[i], s, lo[:, i], hi[:, i])
                out += t
            return out
        if k == "xsinexp":
            fx = 0.5 * (lo[:, 0] + hi[:, 0]) if axis != 0 else np.ones(len(lo))
            fy = _avg_cos(1.0, 0.0, lo[:, 1], hi[:, 1]) if axis == 1 else _avg_sin(1.0, 0.0, lo[:, 1], hi[:, 1])
            return d["amp"] * fx * fy * _avg_exp(1.0, lo[:, 2], hi[:, 2])
        raise ValueError(k)


class _GaussLaplacian(Field):
    """Laplacian of a Gaussian sum: sum over axes of (g'' along that axis) x g x g."""

    def __init__(self, d):
        super().__init__(dict(d, kind="gausslap"))
        self.g = d

    def value(self, X):
        X = np.atleast_2d(X)
        out = np.zeros(len(X))
        for A, mu, s in zip(self.g["amp"], self.g["mu"], self.g["sigma"]):
            dx = X - np.asarray(mu)[None, :]
            r2 = np.sum(dx * dx, axis=1)
            out += A * (r2 / s ** 4 - 3.0 / s ** 2) * np.exp(-r2 / (2 * s * s))
        return out

    def box_average(self, lo, hi):
        lo = np.atleast_2d(lo).astype(float)
        hi = np.atleast_2d(hi).astype(float)
        out = np.zeros(len(lo))
        for A, mu, s in zip(self.g["amp"], self.g["mu"], self.g["sigma"]):
            f0 = [_avg_gauss(mu[i], s, lo[:, i], hi[:, i]) for i in range(3)]
            f2 = [_avg_gauss_d2(mu[i], s, lo[:, i], hi[:, i]) for i in range(3)]
            out += A * (f2[0] * f0[1] * f0[2] + f0[0] * f2[1] * f0[2] + f0[0] * f0[1] * f2[2])
        return out


# ------------------------------------------------------- 1D averages
def _avg_sin(k, p, a, b):
    """mean of sin(k t + p) over [a, b]  (= value at a when a == b)."""
    w = b - a
    mid = 0.5 * (a + b)
    half = 0.5 * k * w
    sinc = np.where(np.abs(half) > 0, np.sin(half) / np.where(half == 0, 1.0, half), 1.0)
    return np.sin(k * mid + p) * sinc


def _avg_cos(k, p, a, b):
    w = b - a
    mid = 0.5 * (a + b)
    half = 0.5 * k * w
    sinc = np.where(np.abs(half) > 0, np.sin(half) / np.where(half == 0, 1.0, half), 1.0)
    return np.cos(k * mid + p) * sinc


def _avg_exp(c, a, b):
    w = b - a
    t = c * w
    rel = np.where(np.abs(t) > 0, np.expm1(t) / np.where(t == 0, 1.0, t), 1.0)
    return np.exp(c * a) * rel


def _avg_gauss(mu, s, a, b):
    """mean of exp(-(t-mu)^2 / (2 s^2)) over [a, b]."""
    w = b - a
    r = np.sqrt(2.0) * s
    A = (a - mu) / r
    B = (b - mu) / r
    pos = A > 0
    neg = B < 0
    diff = np.where(pos, erfc(A) - erfc(B), np.where(neg, erfc(-B) - erfc(-A), erf(B) - erf(A)))
    with np.errstate(invalid="ignore", divide="ignore"):
        avg = s * np.sqrt(np.pi / 2.0) * diff / np.where(w > 0, w, 1.0)
    point = np.exp(-((a - mu) ** 2) / (2 * s * s))
    return np.where(w > 0, avg, point)


def _gauss_d1(mu, s, t):
    return -(t - mu) / (s * s) * np.exp(-((t - mu) ** 2) / (2 * s * s))


def _avg_gauss_d1(mu, s, a, b):
    w = b - a
    g = lambda t: np.exp(-((t - mu) ** 2) / (2 * s * s))
    with np.errstate(invalid="ignore", divide="ignore"):
        avg = (g(b) - g(a)) / np.where(w > 0, w, 1.0)
    return np.where(w > 0, avg, _gauss_d1(mu, s, a))


def _avg_gauss_d2(mu, s, a, b):
    w = b - a
    with np.errstate(invalid="ignore", divide="ignore"):
        avg = (_gauss_d1(mu, s, b) - _gauss_d1(mu, s, a)) / np.where(w > 0, w, 1.0)
    point = ((a - mu) ** 2 / s ** 4 - 1.0 / s ** 2) * np.exp(-((a - mu) ** 2) / (2 * s * s))
    return np.where(w > 0, avg, point)


def _poly_box_average(terms, lo, hi):
    x0, w0 = _GL3
    out = np.zeros(len(lo))
    # product Gauss rule: exact for every monomial of degree <= 5 per axis
    pts = []
    for i in range(3):
        mid = 0.5 * (lo[:, i] + hi[:, i])
        half = 0.5 * (hi[:, i] - lo[:, i])
        pts.append(mid[:, None] + half[:, None] * x0[None, :])
    for a, b, c, v in terms:
        fa = (pts[0] ** a) @ w0 * 0.5
        fb = (pts[1] ** b) @ w0 * 0.5
        fc = (pts[2] ** c) @ w0 * 0.5
        out += v * fa * fb * fc
    return out
