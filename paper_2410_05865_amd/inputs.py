"""Seeded synthetic workloads: domain and field descriptors.

This module only draws and packages problem data (obstacle lists, field
parameters).  It contains none of the method's arithmetic, so both the
CPU oracle and the HIP library may consume its output.

Domains are the unit box R = [0,1]^3 with obstacles removed (the cut-cell
setting of Sec. 2.2): ellipsoids, or a torus (the paper's Problem 2); the
Cartesian grid has n cells per axis and h = 1/n.  Wall order everywhere is (-x, +x, -y, +y, -z, +z).

Field descriptors are plain dicts; the meaning of each kind is:
  zero     : 0
  poly     : sum_c coef * x^a0 y^a1 z^a2 over terms [(a0, a1, a2, coef)], degree <= 4
  sinprod  : amp * sin(k0 x + p0) sin(k1 y + p1) sin(k2 z + p2)
  expcos   : amp * exp(a x + b y) * cos(c z + p)
  gauss    : sum_j amp_j * exp(-|x - mu_j|^2 / (2 sigma_j^2))
  xsinexp  : amp * x * sin(y) * exp(z)
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

DIRICHLET = 0
NEUMANN = 1
ROBIN = 2                       # alpha phi + beta dphi/dn = g (obstacle surfaces and box walls)

ELLIPSOID = 0                   # obstacle kinds
TORUS = 1


@dataclasses.dataclass
class Obstacle:
    center: np.ndarray          # (3,)
    axes: np.ndarray            # (3,) semi-axes
    rot: np.ndarray             # (3,3); column j is the direction of semi-axis j
    bc: int = DIRICHLET         # boundary condition on this obstacle's surface
    robin: Tuple[float, float] = (1.0, 0.0)   # (alpha, beta) of a ROBIN condition
    kind: int = ELLIPSOID
    radii: Tuple[float, float] = (0.0, 0.0)   # TORUS: (major R, minor r), R > r; the
                                              # torus axis is rot[:, 2] through center

    def bounding_radius(self) -> float:
        if self.kind == TORUS:
            return float(self.radii[0] + self.radii[1])
        return float(np.max(self.axes))


@dataclasses.dataclass
class Domain:
    n: int
    obstacles: List[Obstacle]
    wall_bc: Sequence[int] = (DIRICHLET,) * 6
    origin: Sequence[float] = (0.0, 0.0, 0.0)
    n_min: int = 16             # coarsest grid size of the multigrid hierarchy
    inside: bool = False        # Omega = the interior of obstacles[0] instead of the box minus the obstacles
    wall_robin: Sequence[Tuple[float, float]] = ((1.0, 0.0),) * 6   # (alpha, beta) of ROBIN walls

    @property
    def h(self) -> float:
        return 1.0 / self.n

    def with_n(self, n: int) -> "Domain":
        return dataclasses.replace(self, n=n)


def _quat_rotation(u: np.ndarray) -> np.ndarray:
    """Uniformly distributed rotation from three U[0,1) numbers (Shoemake 1992)."""
    u1, u2, u3 = u
    a = math.sqrt(1.0 - u1)
    b = math.sqrt(u1)
    qx, qy = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    qz, qw = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw)],
        [2 * (qx * qy + qz * qw), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw)],
        [2 * (qx * qz - qy * qw), 2 * (qy * qz + qx * qw), 1 - 2 * (qx * qx + qy * qy)],
    ])


def sphere_domain(n: int = 32, radius: float = 0.25, center=(0.5, 0.5, 0.5),
                  bc: int = DIRICHLET, n_min: int = 16) -> Domain:
    """Unit box minus one sphere, Dirichlet walls (the small sphere workload)."""
    ob = Obstacle(np.array(center, float), np.full(3, float(radius)), np.eye(3), bc)
    return Domain(n=n, obstacles=[ob], wall_bc=(DIRICHLET,) * 6, n_min=n_min)


def ellipsoid_domain(n: int, seed: int = 1, count: int = 8,
                     axes_range=(0.05, 0.15), h_coarse: float = 1.0 / 32,
                     obstacle_bc: int = NEUMANN, n_min: int = 32,
                     max_tries: int = 200000) -> Domain:
    """Unit box minus `count` seeded, non-overlapping random ellipsoids.

    Semi-axes ~ U[axes_range], orientation uniform, centre ~ U[m + 2H, 1 - m - 2H]^3
    with m the largest semi-axis and H = h_coarse; bounding spheres are kept at
    least 2H apart (rejection), so no cell of any level with spacing <= H meets
    two obstacles and every obstacle stays 2H clear of the walls.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    obs: List[Obstacle] = []
    tries = 0
    while len(obs) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("ellipsoid generator: rejection sampling did not converge")
        axes = rng.uniform(axes_range[0], axes_range[1], size=3)
        rot = _quat_rotation(rng.uniform(0.0, 1.0, size=3))
        m = float(np.max(axes))
        lo, hi = m + 2 * h_coarse, 1.0 - m - 2 * h_coarse
        if lo >= hi:
            continue
        c = rng.uniform(lo, hi, size=3)
        ok = all(np.linalg.norm(c - o.center) >= m + o.bounding_radius() + 2 * h_coarse
                 for o in obs)
        if ok:
            obs.append(Obstacle(c, axes, rot, obstacle_bc))
    return Domain(n=n, obstacles=obs, wall_bc=(DIRICHLET,) * 6, n_min=n_min)


def torus_domain(n: int, R: float = 0.2, r: float = 0.1, center=(0.5, 0.5, 0.5), rot=None,
                 bc: int = NEUMANN, n_min: int = 32) -> Domain:
    """Unit box minus a solid torus: the points within r of the circle of
    radius R around `center` in the plane normal to rot[:, 2] (default the
    z axis); Dirichlet walls."""
    rot = np.eye(3) if rot is None else np.asarray(rot, float)
    ob = Obstacle(np.array(center, float), np.array([R + r, R + r, r]), rot, bc, kind=TORUS,
                  radii=(float(R), float(r)))
    return Domain(n=n, obstacles=[ob], wall_bc=(DIRICHLET,) * 6, n_min=n_min)


def inside_any_obstacle(domain: Domain, x: np.ndarray) -> bool:
    for o in domain.obstacles:
        d = o.rot.T @ (x - o.center)
        if o.kind == TORUS:
            R, r = o.radii
            if (math.hypot(d[0], d[1]) - R) ** 2 + d[2] ** 2 < r * r:
                return True
        elif float(np.sum((d / o.axes) ** 2)) < 1.0:
            return True
    return False


# ---------------------------------------------------------------- fields
def zero_field() -> dict:
    return {"kind": "zero"}


def poly_field(terms) -> dict:
    """terms: iterable of (a0, a1, a2, coef) with a0 + a1 + a2 <= 4."""
    terms = [(int(a), int(b), int(c), float(v)) for a, b, c, v in terms]
    assert all(a + b + c <= 4 for a, b, c, _ in terms)
    return {"kind": "poly", "terms": terms}


def sinprod_field(amp=1.0, k=(2 * math.pi,) * 3, p=(0.0,) * 3) -> dict:
    return {"kind": "sinprod", "amp": float(amp), "k": [float(v) for v in k],
            "p": [float(v) for v in p]}


def expcos_field(amp=1.0, a=1.0, b=0.5, c=3.0, p=0.0) -> dict:
    return {"kind": "expcos", "amp": float(amp), "a": float(a), "b": float(b),
            "c": float(c), "p": float(p)}


def gauss_field(amps, mus, sigmas) -> dict:
    return {"kind": "gauss", "amp": [float(v) for v in amps],
            "mu": [[float(t) for t in m] for m in mus],
            "sigma": [float(v) for v in sigmas]}


def xsinexp_field(amp=10.0) -> dict:
    """amp x sin(y) e^z: the function of the paper's geometry accuracy test
    (Sec. 6.1, Table 1) with amp = 10."""
    return {"kind": "xsinexp", "amp": float(amp)}


def table1_domain(n: int) -> Domain:
    """The geometry accuracy test of the paper's Table 1: the sphere of radius
    0.2 centred at (0.5, 0.5, 0.5) on an n^3 grid of the unit box."""
    return sphere_domain(n=n, radius=0.2, n_min=min(n, 16))


def gaussian_rhs(domain: Domain, seed: int, count: int = 16,
                 sigma_range=(0.02, 0.1)) -> dict:
    """Sum of `count` seeded Gaussians with centres in the domain (not inside obstacles)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    amps, mus, sigmas = [], [], []
    while len(amps) < count:
        mu = rng.uniform(0.0, 1.0, size=3)
        if inside_any_obstacle(domain, mu):
            continue
        mus.append(mu)
        sigmas.append(rng.uniform(*sigma_range))
        amps.append(rng.uniform(-1.0, 1.0))
    return gauss_field(amps, mus, sigmas)


# ------------------------------------------------------- named workloads
def sphere_workload(n: int = 32):
    """Box minus sphere r=0.25 at the centre; Dirichlet everywhere;
    manufactured phi = sin(2 pi x) sin(2 pi y) sin(2 pi z)."""
    return sphere_domain(n=n), sinprod_field()


def sphere_interior_problem(n: int = 50, n_min: int = 25):
    """The paper's Problem 1: Poisson's equation inside the sphere of radius 0.3
    centred at (0.5, 0.5, 0.5), Dirichlet data, exact solution
    exp(-x^2 - y^2 - z^2) (a Gaussian with sigma^2 = 1/2 at the origin)."""
    ob = Obstacle(np.array([0.5, 0.5, 0.5]), np.full(3, 0.3), np.eye(3), DIRICHLET)
    dom = Domain(n=n, obstacles=[ob], wall_bc=(DIRICHLET,) * 6, n_min=n_min, inside=True)
    return dom, gauss_field([1.0], [[0.0, 0.0, 0.0]], [math.sqrt(0.5)])


def sphere03_workload(n: int = 256):
    """The solving-time workload of the paper's Table 4: the unit cube minus the
    sphere of radius 0.3 at its centre.  The table states no solution or
    boundary conditions; here Dirichlet on walls and sphere with the
    manufactured phi = exp(x + y/2) cos(3 z)."""
    return sphere_domain(n=n, radius=0.3, n_min=32), expcos_field()


def torus_problem(n: int = 64, n_min: int = 32):
    """The paper's Problem 2: the unit cube minus the torus of major radius 0.2
    and minor radius 0.1 centred at (0.5, 0.5, 0.5) (axis z); Dirichlet on the
    cube, Neumann on the torus, data from u = cos(pi x) cos(pi y) sin(pi z).
    The same domain is the torus workload of the paper's Table 4."""
    return (torus_domain(n=n, n_min=n_min),
            sinprod_field(1.0, (math.pi, math.pi, math.pi), (0.5 * math.pi, 0.5 * math.pi, 0.0)))


def ellipsoid_workload(n: int = 128, seed: int = 1):
    """Box minus 8 seeded ellipsoids; Dirichlet walls, Neumann obstacles;
    manufactured phi = exp(x + y/2) cos(3 z)."""
    return ellipsoid_domain(n=n, seed=seed), expcos_field()
