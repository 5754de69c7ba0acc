"""Pins of the learned-guess reference network (oracle/learned.py): the
convolution against a direct loop and scipy, pooling/upsampling against their
definitions, BF16 rounding against known values, and the loss gradient against
central finite differences."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import learned as ol


def test_conv_matches_direct_loop_and_scipy():
    rng = np.random.default_rng(0)
    n, ci, co = 5, 3, 2
    x = rng.standard_normal((1, n, n, n, ci))
    W = rng.standard_normal((27, co, ci))
    b = rng.standard_normal(co)
    got = ol.conv(x, W, b)
    ref = np.zeros((1, n, n, n, co))
    for z in range(n):
        for y in range(n):
            for xx in range(n):
                for t in range(27):
                    dx, dy, dz = t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1
                    zz, yy, x2 = z + dz, y + dy, xx + dx
                    if 0 <= zz < n and 0 <= yy < n and 0 <= x2 < n:
                        ref[0, z, y, xx] += W[t] @ x[0, zz, yy, x2]
    ref += b
    assert np.max(np.abs(got - ref)) < 1e-12
    # one channel: scipy correlation with kernel K[dz+1, dy+1, dx+1] = W[tap]
    K = W[:, 0, 0].reshape(3, 3, 3)
    sc = ndi.correlate(x[0, ..., 0], K, mode="constant", cval=0.0)
    assert np.max(np.abs(ol.conv(x[..., :1], W[:, :1, :1], None)[0, ..., 0] - sc)) < 1e-12


def test_pool_and_up_definitions():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 4, 4, 3))
    p = ol.pool(x)
    assert p.shape == (2, 2, 2, 2, 3)
    assert np.allclose(p[1, 1, 0, 1], x[1, 2:4, 0:2, 2:4].mean(axis=(0, 1, 2)))
    u = ol.up(p)
    assert u.shape == x.shape
    assert np.array_equal(u[0, 3, 1, 2], p[0, 1, 0, 1])


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.14159265])
    got = ol.round_bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa (1.0) wins;
    # 1 + 3*2^-9 lies above the midpoint and rounds up
    assert list(got[:4]) == [1.0, 1.0, 1.0 + 2 ** -7, -2.5]
    assert abs(got[4] - 3.140625) < 1e-12


# central-difference steps: a step crosses ReLU kinks of the activations it
# moves (the first layer's biases move a whole channel), which the 4-level net
# has more of, so its step is smaller; the loss is O(0.05), rounding stays far
# below the tolerance
@pytest.mark.parametrize("C,depth,per_layer,eps", [(16, 3, 12, 1e-6), (16, 4, 8, 1e-7)])
def test_gradient_matches_finite_differences(C, depth, per_layer, eps):
    rng = np.random.default_rng(2)
    n, nb = 16, 1
    npar = ol.num_params(C, depth)
    last = 2 * depth - 1
    params = rng.standard_normal(npar) * 0.2
    # zero the padded slots, as in the library; the 4-level weights scaled by
    # their fan-in so that activations stay of order one through 8 layers
    off = 0
    for li, (ci, co) in enumerate(ol.layer_shapes(C, depth)):
        if depth > 3:
            params[off:off + 27 * co * ci] *= 5.0 / np.sqrt(27.0 * ci)
        W = params[off:off + 27 * co * ci].reshape(27, co, ci)
        if li == 0:
            W[:, :, 2:] = 0.0
        if li == last:
            W[:, 1:, :] = 0.0
        off += 27 * co * ci + co
    x = rng.standard_normal((nb, n, n, n, 2))
    t = rng.standard_normal((nb, n, n, n)) * 0.1
    mask = rng.random((nb, n, n, n)) < 0.8
    loss, g = ol.loss_and_grad(params, x, t, mask, C, depth=depth)
    # a sample of parameters from every layer (weights and biases)
    idx, off = [], 0
    for li, (ci, co) in enumerate(ol.layer_shapes(C, depth)):
        nW = 27 * co * ci
        k_ = per_layer
        cand = [off + k for k in rng.integers(0, nW, k_)]
        if li == 0:
            cand = [off + (k // 16) * 16 + k % 2 for k in rng.integers(0, nW, k_)]   # real input slots
        if li == last:
            cand = [off + (tap * co + 0) * ci + c for tap, c in zip(rng.integers(0, 27, k_), rng.integers(0, ci, k_))]
        idx += cand + [off + nW + int(rng.integers(0, co if li < last else 1))]
        off += nW + co
    for k in idx:
        p1 = params.copy()
        p1[k] += eps
        p2 = params.copy()
        p2[k] -= eps
        fd = (ol.forward_loss(p1, x, t, mask, C, depth=depth) - ol.forward_loss(p2, x, t, mask, C, depth=depth)) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 + 1e-5 * abs(fd), (k, fd, g[k])
