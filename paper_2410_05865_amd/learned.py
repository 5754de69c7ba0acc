"""Training data and training loop of the learned initial guess.

Pairs come from the solver itself: for each seeded geometry of the ellipsoid
family, independent right-hand sides f = sums of 16 seeded Gaussians (g = 0)
are assembled in one batched call, solved to 1e-10 with the batched multigrid
solve, and reduced by the library (cc_net_pairs) to the level the network
works on (m cells per axis):
  features  x[V] = (mean of r over V) / max|r|,  volume fraction of V
  target    t[V] = PHI_SCALE * (mean of phi over the unknown cells of V) / max|r|
  mask      V holds at least one unknown cell.
The network (cc_net_*, the library's BF16-MFMA kernels) is trained with Adam
on the masked mean-square loss; at solve time `Problem.learned_fmg` builds the
same features on the device and starts the full multigrid ascent from the
network's output on that level (`Problem.learned_guess` instead interpolates
the output to the fine grid).
PyTorch only holds the device arrays and picks the mini-batches.
"""
from __future__ import annotations

import time

import numpy as np

from . import _lib, inputs

PHI_SCALE = 100.0


def make_pairs(n_fine: int = 128, level: int = 2, geometries: int = 8, rhs_per_geometry: int = 64,
               seed: int = 0, log=None, max_attempts: int = None):
    """Solver-generated (features, target, mask) at level `level` of n_fine
    problems (geometry seeds 10000 + 100 seed + g, right-hand-side seeds drawn
    from `seed`); returns float32/uint8 CUDA tensors (S, m^3, 2), (S, m^3),
    (S, m^3) and the number of geometries used.  Geometries on which the
    plain iteration does not converge give no pairs; up to max_attempts
    geometries (default: `geometries`, at most 100) are drawn to collect
    `geometries` that do."""
    import torch
    xs, ts, ms = [], [], []
    rng = np.random.default_rng(seed)
    used = 0
    attempts = min(100, geometries if max_attempts is None else max_attempts)
    for g in range(attempts):
        if used == geometries:
            break
        t0 = time.perf_counter()
        dom = inputs.ellipsoid_domain(n=n_fine, seed=10_000 + seed * 100 + g)
        P = _lib.Problem(dom)
        n3 = n_fine ** 3
        fields = [inputs.gaussian_rhs(dom, seed=int(rng.integers(1 << 30))) for _ in range(rhs_per_geometry)]
        r = torch.zeros(rhs_per_geometry, n3, dtype=torch.float64, device="cuda")
        P.assemble_rhs_batched(fields, None, r)
        phi = torch.zeros_like(r)
        infos = P.solve_batched(r, phi)
        if not all(i["converged"] for i in infos):
            # the multigrid iteration does not converge on every geometry of the
            # family; such geometries give no pairs
            if log:
                log(f"[learned] geometry {g}: solve did not converge, skipped")
            P.close()
            continue
        x, t, mask = P.net_pairs(level, r, phi, PHI_SCALE)
        xs.append(x)
        ts.append(t)
        ms.append(mask)
        used += 1
        del r, phi
        P.close()
        if log:
            log(f"[learned] geometry {g}: {rhs_per_geometry} pairs in {time.perf_counter() - t0:.1f} s")
    return torch.cat(xs), torch.cat(ts), torch.cat(ms), used


def train(net, x, t, mask, m: int, steps: int = 400, batch: int = 4, lr: float = 1e-3, seed: int = 0,
          log=None, log_every: int = 100):
    """Adam on random mini-batches; returns the loss history."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    S = x.shape[0]
    hist = []
    for step in range(steps):
        idx = torch.randint(0, S, (batch,), generator=g).cuda()
        xb = x.index_select(0, idx).contiguous()
        tb = t.index_select(0, idx).contiguous()
        mb = mask.index_select(0, idx).contiguous()
        loss = net.loss_grad(xb, tb, mb, m, batch)
        net.adam_step(lr)
        hist.append(loss)
        if log and (step % log_every == 0 or step == steps - 1):
            log(f"[learned] step {step}: loss {loss:.4e}")
    return hist


def relative_error(net, x, t, mask, m: int):
    """Masked max-norm relative error of the network on the pairs (on the host)."""
    import torch
    y = torch.zeros(x.shape[0], m ** 3, dtype=torch.float32, device="cuda")
    for s in range(x.shape[0]):
        net.forward(x[s:s + 1].contiguous(), y[s:s + 1], m, 1)
    yh, th, mk = y.cpu().numpy(), t.cpu().numpy(), mask.cpu().numpy().astype(bool)
    err = np.max(np.abs(yh - th) * mk, axis=1) / np.maximum(np.max(np.abs(th) * mk, axis=1), 1e-30)
    return err


def fit(n_fine: int = 128, level: int = 2, geometries: int = 8, rhs_per_geometry: int = 64, steps: int = 2000,
        batch: int = 8, lr: float = 1e-3, base_channels: int = 16, depth: int = 3, seed: int = 0, log=None,
        max_attempts: int = None):
    """Generate pairs (make_pairs) and train a network (Adam, learning rate lr
    for half of the steps, lr/3 and lr/10 for a quarter each).  Returns
    (net, info)."""
    t0 = time.perf_counter()
    x, t, mask, used = make_pairs(n_fine, level, geometries, rhs_per_geometry, seed=seed, log=log,
                                  max_attempts=max_attempts)
    t_data = time.perf_counter() - t0
    m = round(x.shape[1] ** (1.0 / 3.0))
    net = _lib.Net(base_channels, seed=seed + 1, depth=depth)
    t1 = time.perf_counter()
    hist = []
    for phase, (st, l) in enumerate(((steps // 2, lr), (steps // 4, lr / 3), (steps - steps // 2 - steps // 4, lr / 10))):
        hist += train(net, x, t, mask, m, steps=st, batch=batch, lr=l, seed=seed * 10 + phase, log=log,
                      log_every=max(1, steps // 4))
    t_train = time.perf_counter() - t1
    err = relative_error(net, x[: min(32, x.shape[0])], t[: min(32, x.shape[0])], mask[: min(32, x.shape[0])], m)
    info = {"pairs": int(x.shape[0]), "geometries": used, "fine_grid": n_fine, "grid": m, "depth": depth,
            "base_channels": base_channels, "data_s": t_data, "train_s": t_train, "steps": steps,
            "first_loss": hist[0], "final_loss": hist[-1], "train_median_rel_err": float(np.median(err)),
            "params": net.num_params}
    return net, info
