"""Degenerate inputs of the solve (32^3 sphere workload): a zero right-hand
side (alone and inside a batch), a non-finite one, the iteration limit, and a
restart from a converged iterate."""
import numpy as np
import pytest

from paper_2410_05865_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prob():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_05865_amd import _lib
    _lib.load()
    dom, phi = inputs.sphere_workload(32)
    P = _lib.Problem(dom)
    r = torch.zeros(32 ** 3, dtype=torch.float64, device="cuda")
    P.assemble_rhs(phi, phi, r, f_mode=_lib.CC_LAPLACIAN)
    yield _lib, P, r
    P.close()


@pytest.mark.parametrize("mode", ["fp64", "mixed", "krylov"])
def test_zero_rhs_converges_at_once(prob, mode):
    L, P, r = prob
    P.set_precision(L.CC_MIXED if mode == "mixed" else L.CC_FP64)
    P.set_krylov(20 if mode == "krylov" else 0)
    x = torch.zeros_like(r)
    info = P.solve(torch.zeros_like(r), x)
    P.set_precision(L.CC_FP64)
    P.set_krylov(0)
    assert info["converged"] and info["iterations"] == 0
    assert float(x.abs().max()) == 0.0


@pytest.mark.parametrize("mode", ["fp64", "mixed", "krylov"])
def test_zero_rhs_from_a_nonzero_guess_returns_zero(prob, mode):
    """L phi = 0 has the solution 0 (L is nonsingular); the relative stopping
    test is undefined there, so the guess must not be returned unchanged."""
    L, P, r = prob
    P.set_precision(L.CC_MIXED if mode == "mixed" else L.CC_FP64)
    P.set_krylov(20 if mode == "krylov" else 0)
    x = torch.randn(r.shape, dtype=torch.float64, device="cuda")
    info = P.solve(torch.zeros_like(r), x)
    P.set_precision(L.CC_FP64)
    P.set_krylov(0)
    assert info["converged"] and info["iterations"] == 0
    assert float(x.abs().max()) == 0.0


def test_zero_member_of_a_batch(prob):
    L, P, r = prob
    rb = torch.stack([r, torch.zeros_like(r), 2.0 * r]).contiguous()
    xb = torch.randn(rb.shape, dtype=torch.float64, device="cuda")
    infos = P.solve_batched(rb, xb)
    assert all(i["converged"] for i in infos)
    assert float(xb[1].abs().max()) == 0.0
    # linearity: the third member is twice the first
    assert float((xb[2] - 2.0 * xb[0]).abs().max()) <= 1e-9 * float(xb[2].abs().max())


def test_non_finite_rhs_is_an_error_and_the_problem_stays_usable(prob):
    L, P, r = prob
    bad = r.clone()
    bad[12345] = float("nan")
    x = torch.zeros_like(r)
    with pytest.raises(L.CutCellError) as e:
        P.solve(bad, x)
    assert e.value.code == L.CC_EINVAL
    info = P.solve(r, x)
    assert info["converged"] and info["rel_residual"] < 1e-10


def test_iteration_limit_reports_no_convergence(prob):
    L, P, r = prob
    dom, _ = inputs.sphere_workload(32)
    Q = L.Problem(dom, max_iter=2)
    x = torch.zeros_like(r)
    info = Q.solve(r, x)
    Q.close()
    assert not info["converged"]
    assert info["iterations"] == 2 and info["rel_residual"] > 1e-10
    assert len(info["history"]) == 3 and info["history"][2] < info["history"][0]
    assert bool(torch.isfinite(x).all())


def test_restart_from_a_converged_iterate(prob):
    L, P, r = prob
    x = torch.zeros_like(r)
    first = P.solve(r, x)
    kept = x.clone()
    again = P.solve(r, x)
    assert first["converged"] and again["converged"] and again["iterations"] == 0
    assert torch.equal(x, kept)


def test_repeated_solves_agree_within_a_bound(prob):
    """The forward LU sweeps add contributions with FP64 atomics, so the order
    of those additions, and the last bits, may change between runs: repeated
    solves must take the same V-cycle count and agree to 1e-12 relative."""
    L, P, r = prob
    xs, its = [], []
    for _ in range(4):
        x = torch.zeros_like(r)
        info = P.solve(r, x)
        xs.append(x)
        its.append(info["iterations"])
    assert len(set(its)) == 1
    ref = float(xs[0].abs().max())
    for x in xs[1:]:
        assert float((x - xs[0]).abs().max()) <= 1e-12 * ref
