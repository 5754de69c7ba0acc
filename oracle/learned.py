"""Reference of the learned-guess network (test infrastructure; not from the
paper: the learned initial guess is an addition on top of its method).

Plain numpy, FP64: a 3-level 3D U-Net written from its definition, with
the gradient of the masked mean-square loss by the chain rule.  Optionally the
BF16 rounding of the device path is applied at the same points (inputs,
weights, stored activations and activation gradients) so that the device can
be compared closely.

Tensors are (batch, z, y, x, channel); the flat voxel index x + n (y + n z)
matches the library's i + n (j + n k).  Parameters are one flat array in layer
order, each layer W[27][Cout][Cin] (tap = (dz+1) 9 + (dy+1) 3 + (dx+1)) then
bias[Cout].

Pins (tests/test_oracle_learned.py): the convolution against a direct loop and
against scipy.ndimage.correlate, pooling/upsampling against their definitions,
and the gradient against central finite differences of the loss.
"""
from __future__ import annotations

import numpy as np


def layer_shapes(C: int):
    return [(16, C), (C, 2 * C), (2 * C, 2 * C), (4 * C, 2 * C), (3 * C, C), (C, 16)]


def num_params(C: int) -> int:
    return sum(27 * ci * co + co for ci, co in layer_shapes(C))


def unpack(params: np.ndarray, C: int):
    out, off = [], 0
    for ci, co in layer_shapes(C):
        W = params[off:off + 27 * co * ci].reshape(27, co, ci)
        off += 27 * co * ci
        b = params[off:off + co]
        off += co
        out.append((W, b))
    return out


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


TAPS = [(t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1) for t in range(27)]   # (dx, dy, dz)


def _shift(x: np.ndarray, dx: int, dy: int, dz: int) -> np.ndarray:
    """s[..., z, y, x, :] = x[..., z + dz, y + dy, x + dx, :], zero outside."""
    n = x.shape[1]
    p = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    return p[:, 1 + dz:1 + dz + n, 1 + dy:1 + dy + n, 1 + dx:1 + dx + n, :]


def conv(x: np.ndarray, W: np.ndarray, b) -> np.ndarray:
    """out[v, co] = b[co] + sum_tap sum_ci x[v + off(tap), ci] W[tap, co, ci]."""
    out = np.zeros(x.shape[:4] + (W.shape[1],))
    for t, (dx, dy, dz) in enumerate(TAPS):
        out += np.einsum("bzyxc,oc->bzyxo", _shift(x, dx, dy, dz), W[t])
    if b is not None:
        out += b
    return out


def conv_grad(x, W, g):
    """Gradients of sum(g * conv(x, W, b)) with respect to x, W and b."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for t, (dx, dy, dz) in enumerate(TAPS):
        gW[t] = np.einsum("bzyxo,bzyxc->oc", g, _shift(x, dx, dy, dz))
        gx += np.einsum("bzyxo,oc->bzyxc", _shift(g, -dx, -dy, -dz), W[t])
    return gx, gW, g.sum(axis=(0, 1, 2, 3))


def pool(x):
    nb, n, _, _, c = x.shape
    return x.reshape(nb, n // 2, 2, n // 2, 2, n // 2, 2, c).mean(axis=(2, 4, 6))


def up(x):
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def forward(params, x2, C: int, bf16: bool = False):
    """x2: (nb, n, n, n, 2) -> y (nb, n, n, n) and the cache for the gradient."""
    rb = round_bf16 if bf16 else (lambda a: a)
    L = [(rb(W), b) for W, b in unpack(np.asarray(params, dtype=np.float64), C)]
    x = np.zeros(x2.shape[:4] + (16,))
    x[..., :2] = rb(x2)
    relu = lambda a: np.maximum(a, 0.0)
    e1 = rb(relu(conv(x, *L[0])))
    p1 = rb(pool(e1))
    e2 = rb(relu(conv(p1, *L[1])))
    p2 = rb(pool(e2))
    bt = rb(relu(conv(p2, *L[2])))
    cat2 = np.concatenate([up(bt), e2], axis=-1)
    d2 = rb(relu(conv(cat2, *L[3])))
    cat1 = np.concatenate([up(d2), e1], axis=-1)
    d1 = rb(relu(conv(cat1, *L[4])))
    y = conv(d1, *L[5])[..., 0]
    cache = dict(L=L, x=x, e1=e1, p1=p1, e2=e2, p2=p2, bt=bt, cat2=cat2, d2=d2, cat1=cat1, d1=d1)
    return y, cache


def loss_and_grad(params, x2, t, mask, C: int, bf16: bool = False):
    """Masked mean-square loss and its gradient with respect to params (flat)."""
    rb = round_bf16 if bf16 else (lambda a: a)
    y, c = forward(params, x2, C, bf16)
    L = c["L"]
    m = np.asarray(mask, dtype=bool)
    cnt = max(int(m.sum()), 1)
    d = np.where(m, y - t, 0.0)
    loss = float((d * d).sum() / cnt)
    gy = np.zeros(y.shape + (16,))
    gy[..., 0] = rb(2.0 * d / cnt)
    grads = [None] * 6
    gd1, gW, gb = conv_grad(c["d1"], L[5][0], gy)
    grads[5] = (gW, gb)
    gd1 = np.where(c["d1"] > 0, rb(gd1), 0.0)
    gcat1, gW, gb = conv_grad(c["cat1"], L[4][0], gd1)
    grads[4] = (gW, gb)
    gcat1 = rb(gcat1)
    C2 = 2 * C
    gu1, ge1_skip = gcat1[..., :C2], gcat1[..., C2:]
    nb, n = gu1.shape[0], gu1.shape[1]
    gd2 = rb(gu1.reshape(nb, n // 2, 2, n // 2, 2, n // 2, 2, C2).sum(axis=(2, 4, 6)))
    gd2 = np.where(c["d2"] > 0, gd2, 0.0)
    gcat2, gW, gb = conv_grad(c["cat2"], L[3][0], gd2)
    grads[3] = (gW, gb)
    gcat2 = rb(gcat2)
    gu2, ge2_skip = gcat2[..., :C2], gcat2[..., C2:]
    m2 = gu2.shape[1]
    gbt = rb(gu2.reshape(nb, m2 // 2, 2, m2 // 2, 2, m2 // 2, 2, C2).sum(axis=(2, 4, 6)))
    gbt = np.where(c["bt"] > 0, gbt, 0.0)
    gp2, gW, gb = conv_grad(c["p2"], L[2][0], gbt)
    grads[2] = (gW, gb)
    gp2 = rb(gp2)
    ge2 = rb(ge2_skip + up(gp2) / 8.0)
    ge2 = np.where(c["e2"] > 0, ge2, 0.0)
    gp1, gW, gb = conv_grad(c["p1"], L[1][0], ge2)
    grads[1] = (gW, gb)
    gp1 = rb(gp1)
    ge1 = rb(ge1_skip + up(gp1) / 8.0)
    ge1 = np.where(c["e1"] > 0, ge1, 0.0)
    _, gW, gb = conv_grad(c["x"], L[0][0], ge1)
    grads[0] = (gW, gb)
    flat = np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])
    return loss, flat


def forward_loss(params, x2, t, mask, C: int, bf16: bool = False) -> float:
    y, _ = forward(params, x2, C, bf16)
    m = np.asarray(mask, dtype=bool)
    d = np.where(m, y - t, 0.0)
    return float((d * d).sum() / max(int(m.sum()), 1))
