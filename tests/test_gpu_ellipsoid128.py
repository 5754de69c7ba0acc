"""The 128^3 ellipsoid workload (unit box minus 8 seeded ellipsoids, seed 1)
against the oracle, in the launch configuration the build picks for it (the
regular-row schedule its autotuner keeps) and with the z-marching kernels at 8
and 16 planes per workgroup.

The oracle needs minutes to build this size, so its results were written by
tests/golden/make_ellipsoid128.py (oracle only) into
tests/golden/ellipsoid128_seed1.npz: hashes of the integer decisions, the
cells without an unknown, and L x, r - L x, SMO-1, one V-cycle, the assembled
right-hand side and the converged solution at a seeded sample of ~16k cells
(12000 unknown cells and 4000 FV-PLG cells, drawn uniformly), with the full
vectors' max norms.
Tolerances as for the smaller workloads (relative to the full max norm):
apply and residual 1e-12, SMO-1 1e-13, V-cycle 1e-12, right-hand side 1e-12,
converged solution 1e-11 with the same V-cycle count."""
import hashlib
import os

import numpy as np
import pytest

from paper_2410_05865_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ellipsoid128_seed1.npz")


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_05865_amd import _lib
    _lib.load()
    g = dict(np.load(GOLD, allow_pickle=False))
    n = int(g["n"])
    dom, phi = inputs.ellipsoid_workload(n, seed=int(g["seed"]))
    print(f"[ellipsoid128] building the library problem", flush=True)
    P = _lib.Problem(dom, use_graph=0)
    rng = np.random.default_rng(int(g["input_seed"]))
    x = rng.standard_normal(n ** 3)
    r = rng.standard_normal(n ** 3)
    x[g["absent"]] = 0.0
    r[g["absent"]] = 0.0
    yield _lib, P, g, phi, x, r
    P.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _at(t, cells):
    return t.detach().cpu().numpy()[cells]


def test_integer_decisions_identical(case):
    L, P, g, phi, x, r = case
    typ, host, vf = P.export_cells(0)
    assert _sha(typ) == str(g["type_sha"])
    assert _sha(host.astype(np.int32)) == str(g["host_sha"])
    cell, cols, vals = P.export_plg(0)
    assert _sha(cell.astype(np.int32)) == str(g["plg_cells_sha"])
    assert _sha(cols.astype(np.int32).reshape(-1, 35)) == str(g["plg_cols_sha"])
    info = P.level_info(0)
    assert info["n_unknowns"] == int(g["n_unknowns"]) and info["n_phi2"] == int(g["n_phi2"])
    # FV-PLG coefficients of the first rows: QR (library) against SVD (oracle)
    k = len(g["plg_vals_rows"])
    assert np.array_equal(cell[:k], g["plg_vals_rows"])
    gap = np.max(np.abs(vals[:k] - g["plg_vals"]), axis=1) / np.max(np.abs(g["plg_vals"]), axis=1)
    print(f"[ellipsoid128] FV-PLG rows, QR vs SVD: max relative gap {gap.max():.2e}", flush=True)
    assert gap.max() < 1e-11


@pytest.mark.parametrize("sched", [(-1, 0), (1, 8), (1, 16), (2, 16)])
def test_steps_match_oracle(case, sched):
    """(-1, 0): the build's autotuned schedule; (1, 8) and (1, 16): the
    z-marching kernels with one and two unrolled chunks of 8 planes; (2, 16):
    the same in the XCD-aware tile order."""
    L, P, g, phi, x, r = case
    P.set_stencil_schedule(0, *sched)
    try:
        c = g["cells"]
        nrm = g["norms"]
        y = _dev(np.zeros_like(x))
        P.apply(0, _dev(x), y)
        assert np.max(np.abs(_at(y, c) - g["apply"])) < 1e-12 * nrm[0]
        s = _dev(np.zeros_like(x))
        P.residual(0, _dev(r), _dev(x), s)
        assert np.max(np.abs(_at(s, c) - g["residual"])) < 1e-12 * nrm[1]
        e = _dev(x)
        P.smo1(0, _dev(r), e)
        assert np.max(np.abs(_at(e, c) - g["smo1"])) < 1e-13 * nrm[2]
        e = _dev(np.zeros_like(x))
        P.vcycle(0, _dev(r), e)
        assert np.max(np.abs(_at(e, c) - g["vcycle"])) < 1e-12 * nrm[3]
    finally:
        P.set_stencil_schedule(-1, -1, 0)


def test_converged_solve_matches_oracle(case):
    L, P, g, phi, x, r = case
    c = g["cells"]
    nrm = g["norms"]
    n3 = x.size
    rhs = torch.zeros(n3, dtype=torch.float64, device="cuda")
    P.assemble_rhs(phi, phi, rhs, f_mode=L.CC_LAPLACIAN)
    assert np.max(np.abs(_at(rhs, c) - g["rhs"])) < 1e-12 * nrm[4]
    sol = torch.zeros_like(rhs)
    info = P.solve(rhs, sol)
    hist = g["history"]
    assert info["converged"] and info["iterations"] == len(hist) - 1
    assert np.max(np.abs(_at(sol, c) - g["solution"])) < 1e-11 * nrm[5]
    for a, b in zip(info["history"], hist):
        assert a == pytest.approx(b, rel=1e-5, abs=1e-14)
