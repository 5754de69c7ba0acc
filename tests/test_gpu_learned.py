"""GPU parity of the learned-guess network (BF16-MFMA kernels) against the numpy
reference, training, and the guess inside the multigrid solve."""
import numpy as np
import pytest

from oracle import learned as ol

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_05865_amd import _lib
    _lib.load()
    return _lib


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


def _inputs(n, nb, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((nb, n, n, n, 2)).astype(np.float32)
    x[..., 1] = rng.random((nb, n, n, n))
    t = (rng.standard_normal((nb, n, n, n)) * 0.3).astype(np.float32)
    mask = (rng.random((nb, n, n, n)) < 0.85).astype(np.uint8)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a.reshape(nb, -1, *a.shape[4:]))).cuda()
    return x, t, mask, dev(x), dev(t), dev(mask)


@pytest.mark.parametrize("C,depth,n,nb", [(16, 3, 16, 2), (32, 3, 16, 2), (32, 4, 32, 1)])
def test_forward_and_gradients_match_reference(C, depth, n, nb):
    """The device network equals the reference with the same BF16 rounding
    points to a few BF16 ulps (FP32 versus FP64 accumulation can move a rounding
    by one ulp), and the exact-arithmetic reference to BF16 accuracy; layers
    whose input channels come in groups of 32 run on the double-K MFMA."""
    L = _lib()
    net = L.Net(C, seed=3, depth=depth)
    params = net.get_params().astype(np.float64)
    assert params.size == ol.num_params(C, depth)
    x, t, mask, xd, td, md = _inputs(n, nb, 5)
    print(f"[learned] C={C} depth={depth} forward", flush=True)
    y = torch.zeros(nb, n ** 3, dtype=torch.float32, device="cuda")
    net.forward(xd, y, n, nb)
    yg = y.cpu().numpy().reshape(nb, n, n, n)
    y_bf, _ = ol.forward(params, x.astype(np.float64), C, bf16=True, depth=depth)
    y_ex, _ = ol.forward(params, x.astype(np.float64), C, bf16=False, depth=depth)
    assert _rel(yg, y_bf) < 2e-2
    assert _rel(yg, y_ex) < 5e-2
    print(f"  forward rel err vs bf16 ref {_rel(yg, y_bf):.2e}, vs exact {_rel(yg, y_ex):.2e}", flush=True)
    loss, g = net.loss_grad(xd, td, md, n, nb, want_grad=True)
    loss_bf, g_bf = ol.loss_and_grad(params, x.astype(np.float64), t.astype(np.float64), mask, C, bf16=True,
                                     depth=depth)
    assert loss == pytest.approx(loss_bf, rel=1e-2)
    off = 0
    for li, (ci, co) in enumerate(ol.layer_shapes(C, depth)):
        for name, size in (("W", 27 * ci * co), ("b", co)):
            a, b = g[off:off + size].astype(np.float64), g_bf[off:off + size]
            off += size
            if np.max(np.abs(b)) == 0:
                assert np.max(np.abs(a)) == 0
                continue
            cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
            print(f"  layer {li} {name}: rel max err {_rel(a, b):.2e}, cosine {cos:.6f}", flush=True)
            assert cos > 0.999, (li, name, cos)
            assert _rel(a, b) < 5e-2, (li, name)
    net.close()


def test_training_reduces_loss():
    L = _lib()
    n, nb = 16, 2
    net = L.Net(16, seed=4)
    _, _, _, xd, td, md = _inputs(n, nb, 6)
    l0 = net.loss_grad(xd, td, md, n, nb)
    for _ in range(80):
        net.loss_grad(xd, td, md, n, nb)
        net.adam_step(3e-3)
    l1 = net.loss_grad(xd, td, md, n, nb)
    print(f"[learned] overfit loss {l0:.3e} -> {l1:.3e}", flush=True)
    assert l1 < 0.3 * l0
    net.close()


def test_training_is_reproducible():
    """Gradients are reduced in a fixed order (no atomics), so two runs from the
    same seed on the same data give bit-identical parameters and losses."""
    L = _lib()
    n, nb = 16, 4
    _, _, _, xd, td, md = _inputs(n, nb, 8)
    runs = []
    for _ in range(2):
        net = L.Net(16, seed=6)
        losses = []
        for _ in range(30):
            losses.append(net.loss_grad(xd, td, md, n, nb))
            net.adam_step(3e-3)
        runs.append((np.array(losses), net.get_params()))
        net.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])


def test_learned_guess_in_solve():
    """Train on solver-generated pairs (64^3 problems, network on their 32^3
    level; pairs built by the library from batched assembly and solves), then
    solve held-out problems from the network's guess.  The guessed solves reach
    the same tolerance and the same solution, and on average they take fewer
    V-cycles than from the zero guess."""
    L = _lib()
    from paper_2410_05865_amd import inputs, learned
    log = lambda s: print(s, flush=True)
    net, info = learned.fit(n_fine=64, level=1, geometries=6, rhs_per_geometry=64, steps=1500, seed=2, log=log)
    log(f"[learned] {info}")
    assert info["pairs"] >= 128
    assert info["final_loss"] < 0.1 * info["first_loss"]
    gains = []
    for s in range(4):
        dom = inputs.ellipsoid_domain(n=64, seed=777 + s)
        P = L.Problem(dom)
        r = torch.zeros(64 ** 3, dtype=torch.float64, device="cuda")
        P.assemble_rhs(inputs.gaussian_rhs(dom, seed=4242 + s), None, r)
        phi0 = torch.zeros_like(r)
        i0 = P.solve(r, phi0)
        phi1 = torch.zeros_like(r)
        P.learned_guess(net, 1, learned.PHI_SCALE, r, phi1)
        g_rel = float((phi1 - phi0).abs().max() / phi0.abs().max())
        i1 = P.solve(r, phi1)
        assert i0["converged"] and i1["converged"]
        assert float((phi1 - phi0).abs().max() / phi0.abs().max()) < 1e-8
        log(f"[learned] held-out {s}: guess rel error {g_rel:.3f}, initial rel residual "
            f"{i1['history'][0]:.3e}; V-cycles zero guess {i0['iterations']}, learned guess {i1['iterations']}")
        gains.append(i0["iterations"] - i1["iterations"])
        P.close()
    log(f"[learned] V-cycles saved per solve: {gains}")
    assert np.mean(gains) > 0
    net.close()


def test_learned_fmg_start_saves_vcycles():
    """The network's output fed in at a coarse level (cc_learned_fmg): trained
    on pairs at the 64^3 level of 128^3 problems, its prediction there is the
    iterate the full multigrid ascent starts from (2 V-cycles per level).  On
    held-out problems the solve from that iterate takes fewer V-cycles than
    from the zero guess, every time; FMG(2) from the exact coarsest solve is
    reported beside it."""
    L = _lib()
    from paper_2410_05865_amd import inputs, learned
    log = lambda s: print(s, flush=True)
    net, info = learned.fit(n_fine=128, level=1, geometries=3, rhs_per_geometry=32, steps=600, batch=4, seed=5,
                            log=log)
    log(f"[learned-fmg] {info}")
    rows = []
    for s in range(3):
        dom = inputs.ellipsoid_domain(n=128, seed=888 + s)
        P = L.Problem(dom)
        f = inputs.gaussian_rhs(dom, seed=5151 + s)
        r = torch.zeros(128 ** 3, dtype=torch.float64, device="cuda")
        P.assemble_rhs(f, None, r)
        coarse = []
        for m in range(1, P.num_levels):
            rm = torch.zeros(P.n(m) ** 3, dtype=torch.float64, device="cuda")
            P.assemble_rhs(f, None, rm, level=m)
            coarse.append(rm)
        x0 = torch.zeros_like(r)
        i0 = P.solve(r, x0)
        x1 = torch.zeros_like(r)
        P.learned_fmg(net, 1, learned.PHI_SCALE, r, x1, cycles=2, coarse_rhs=coarse)
        i1 = P.solve(r, x1)
        x2 = torch.zeros_like(r)
        P.fmg(r, x2, 2, coarse_rhs=coarse)
        i2 = P.solve(r, x2)
        assert i0["converged"] and i1["converged"] and i2["converged"]
        assert float((x1 - x0).abs().max() / x0.abs().max()) < 1e-8
        rows.append((i0["iterations"], i1["iterations"], i2["iterations"]))
        log(f"[learned-fmg] held-out {s}: V-cycles zero guess {i0['iterations']}, learned FMG start "
            f"{i1['iterations']}, FMG(2) {i2['iterations']}")
        P.close()
    assert all(a > b for a, b, _ in rows), rows
    net.close()
