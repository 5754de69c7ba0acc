"""Writes tests/golden/torus32.npz: oracle results on the paper's Problem 2 at
32^3 (unit box minus the torus R = 0.2, r = 0.1 about the z axis through the
centre, Dirichlet walls, Neumann torus, u = cos(pi x) cos(pi y) sin(pi z);
levels 32 and 16) at sampled cells.

Calls only the oracle and the seeded input generators.  The oracle needs about
a minute to build this hierarchy (its quartic level set is the slow part), so
the results it computes in full are stored at a seeded sample of cells:

  * hashes of the level-0 integer decisions (cell types 0/1/2, hosts) and of
    the FV-PLG stencils (target cells, 35 column cells per row);
  * the cells that carry no unknown (exterior or absorbed), so a test can
    build the same grid inputs;
  * for seeded grid inputs x, r (standard normal at every cell, zero where no
    unknown): L x, r - L x, one SMO-1 sweep (omega 0.8), one V-cycle of r
    (nu 3/3), at the sampled cells;
  * the manufactured right-hand side, the converged solution (1e-10), its
    V-cycle count and residual history, at the sampled cells.

    python tests/golden/make_torus32.py      # ~2 min of CPU
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.fields import Field                       # noqa: E402
from oracle.multigrid import Hierarchy, MGParams      # noqa: E402
from paper_2410_05865_amd import inputs               # noqa: E402

N = 32
N_MIN = 16
INPUT_SEED = 2025
SAMPLE_SEED = 8
SAMPLE_CELLS = 6000       # unknown cells drawn uniformly
SAMPLE_PHI2 = 4000        # phi_2 cells drawn uniformly (FV-PLG rows, near the torus)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "torus32.npz")


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def grid_inputs(n, absent):
    """The seeded grid inputs x, r: standard normal per cell, 0 where no unknown."""
    rng = np.random.default_rng(INPUT_SEED)
    x = rng.standard_normal(n ** 3)
    r = rng.standard_normal(n ** 3)
    x[absent] = 0.0
    r[absent] = 0.0
    return x, r


def main():
    t0 = time.time()
    dom, phi = inputs.torus_problem(N, n_min=N_MIN)
    H = Hierarchy(dom)
    lv, op = H.fine, H.ops[0]
    print(f"oracle hierarchy {H.sizes}: {time.time() - t0:.0f} s", flush=True)
    n3 = N ** 3
    typ = np.zeros(n3, np.uint8)
    typ[lv.unknowns] = np.where(lv.is_phi1[lv.unknowns], 1, 2)
    host = np.asarray(lv.host, dtype=np.int32)
    cols = np.array([lv.plg[lv.uidx[p]][0] for p in lv.phi2], dtype=np.int32).reshape(-1, 35)
    absent = np.setdiff1d(np.arange(n3), lv.unknowns).astype(np.int32)

    rng = np.random.default_rng(SAMPLE_SEED)
    cells = np.union1d(rng.choice(lv.unknowns, SAMPLE_CELLS, replace=False),
                       rng.choice(lv.phi2, min(SAMPLE_PHI2, len(lv.phi2)), replace=False)).astype(np.int64)
    ui = lv.uidx[cells]

    xg, rg = grid_inputs(N, absent)
    x, r = xg[lv.unknowns], rg[lv.unknowns]
    Lx = lv.L @ x
    smo1 = op.smo1(x, r, 0.8)
    vc = H.vcycle(0, r, MGParams(omega=0.8, nu1=3, nu2=3))
    print(f"steps: {time.time() - t0:.0f} s", flush=True)

    F = Field(phi)
    rhs = lv.rhs(F.laplacian_desc(), F)
    sol, hist = H.solve(rhs, MGParams(tol=1e-10))
    print(f"solve ({len(hist) - 1} V-cycles): {time.time() - t0:.0f} s", flush=True)

    np.savez_compressed(
        OUT, n=N, n_min=N_MIN, input_seed=INPUT_SEED,
        type_sha=sha(typ), host_sha=sha(host), plg_cells_sha=sha(np.asarray(lv.phi2, dtype=np.int32)),
        plg_cols_sha=sha(cols), n_unknowns=lv.N, n_phi2=len(lv.phi2),
        absent=absent, cells=cells.astype(np.int32),
        apply=Lx[ui], residual=(r - Lx)[ui], smo1=smo1[ui], vcycle=vc[ui],
        rhs=rhs[ui], solution=sol[ui], history=np.array(hist),
        plg_vals_rows=np.asarray(lv.phi2[:64], dtype=np.int32),
        plg_vals=np.array([lv.plg[lv.uidx[p]][1] for p in lv.phi2[:64]]),
        norms=np.array([np.max(np.abs(Lx)), np.max(np.abs(r - Lx)), np.max(np.abs(smo1)), np.max(np.abs(vc)),
                        np.max(np.abs(rhs)), np.max(np.abs(sol))]))
    print(f"wrote {OUT}: {os.path.getsize(OUT) / 1e6:.2f} MB, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
