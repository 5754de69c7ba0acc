"""The allocation-free full-multigrid entry point (cc_fmg_noalloc) against
cc_fmg, through the C ABI: two calls in a row on one GPU, the second on a
smaller problem (so the fixed scratch keeps the first call's larger contents),
with per-level right-hand sides and with restricted ones.  Same kernels in the
same order, so the two agree to the FP64 parity bar (1e-11 relative; the
LU-correction's atomic additions may change the last bits)."""
import numpy as np
import pytest

from paper_2410_05865_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _problem(L, dom, phi):
    P = L.Problem(dom)
    n3 = P.n() ** 3
    r = torch.zeros(n3, dtype=torch.float64, device="cuda")
    P.assemble_rhs(phi, phi, r, f_mode=L.CC_LAPLACIAN)
    coarse = []
    for m in range(1, P.num_levels):
        rm = torch.zeros(P.n(m) ** 3, dtype=torch.float64, device="cuda")
        P.assemble_rhs(phi, phi, rm, f_mode=L.CC_LAPLACIAN, level=m)
        coarse.append(rm)
    return P, r, coarse


def _rel(a, b):
    return float((a - b).abs().max()) / float(b.abs().max())


def test_fmg_noalloc_matches_fmg_on_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_05865_amd import _lib as L
    L.load()
    big_dom, big_phi = inputs.sphere_domain(n=96, radius=0.1, n_min=24), inputs.sinprod_field()
    small_dom, small_phi = inputs.sphere_workload(32)
    for dom, phi, cycles in ((big_dom, big_phi, 2), (small_dom, small_phi, 1)):
        print(f"[no-alloc] n = {dom.n}, cycles = {cycles}", flush=True)
        P, r, coarse = _problem(L, dom, phi)
        for crhs in (coarse, None):
            ref = torch.zeros_like(r)
            P.fmg(r, ref, cycles, coarse_rhs=crhs)
            got = torch.full_like(r, 7.0)        # every cell is written
            P.fmg_noalloc(r, got, cycles, coarse_rhs=crhs)
            torch.cuda.synchronize()
            assert bool(torch.isfinite(got).all())
            assert _rel(got, ref) < 1e-11, (dom.n, crhs is None)
            # the result starts a solve like cc_fmg's does
            info = P.solve(r, got)
            assert info["converged"]
        P.close()
