"""Reference of the learned-guess network (test infrastructure; not from the
paper: the learned initial guess is an addition on top of its method).

Plain numpy, FP64: a 3D U-Net of 3 or 4 levels written from its definition, with
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


def widths(C: int, depth: int = 3):
    """Channels of the encoder levels 0 .. depth-1 (the last is the bottleneck):
    C on the upper levels, 2C on the two coarsest."""
    return [C if l < depth - 2 else 2 * C for l in range(depth)]


def layer_shapes(C: int, depth: int = 3):
    """(Cin, Cout) of every layer in parameter order: the encoder convolutions
    of levels 0 .. depth-2, the bottleneck, the decoder convolutions of levels
    depth-2 .. 0 (input: the upsampled coarser result beside the skip), the
    output convolution."""
    w = widths(C, depth)
    shapes = [(16, w[0])]
    shapes += [(w[l - 1], w[l]) for l in range(1, depth - 1)]
    shapes.append((w[depth - 2], w[depth - 1]))
    shapes += [(w[l + 1] + w[l], w[l]) for l in range(depth - 2, -1, -1)]
    shapes.append((w[0], 16))
    return shapes


def num_params(C: int, depth: int = 3) -> int:
    return sum(27 * ci * co + co for ci, co in layer_shapes(C, depth))


def unpack(params: np.ndarray, C: int, depth: int = 3):
    out, off = [], 0
    for ci, co in layer_shapes(C, depth):
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


def forward(params, x2, C: int, bf16: bool = False, depth: int = 3):
    """x2: (nb, n, n, n, 2) -> y (nb, n, n, n) and the cache for the gradient."""
    rb = round_bf16 if bf16 else (lambda a: a)
    L = [(rb(W), b) for W, b in unpack(np.asarray(params, dtype=np.float64), C, depth)]
    x = np.zeros(x2.shape[:4] + (16,))
    x[..., :2] = rb(x2)
    relu = lambda a: np.maximum(a, 0.0)
    D = depth
    ins, e, p = [], [], []
    h = x
    for l in range(D - 1):                      # encoder: conv, then 2x2x2 average pooling
        ins.append(h)
        e.append(rb(relu(conv(h, *L[l]))))
        p.append(rb(pool(e[l])))
        h = p[l]
    bt = rb(relu(conv(h, *L[D - 1])))           # bottleneck
    d, cats = [None] * (D - 1), [None] * (D - 1)
    cur = bt
    for l in range(D - 2, -1, -1):              # decoder: nearest upsampling beside the skip
        cats[l] = np.concatenate([up(cur), e[l]], axis=-1)
        d[l] = rb(relu(conv(cats[l], *L[2 * D - 2 - l])))
        cur = d[l]
    y = conv(d[0], *L[2 * D - 1])[..., 0]
    cache = dict(L=L, ins=ins, e=e, p=p, bt=bt, d=d, cats=cats)
    return y, cache


def loss_and_grad(params, x2, t, mask, C: int, bf16: bool = False, depth: int = 3):
    """Masked mean-square loss and its gradient with respect to params (flat)."""
    rb = round_bf16 if bf16 else (lambda a: a)
    y, c = forward(params, x2, C, bf16, depth)
    L = c["L"]
    D = depth
    w = widths(C, D)
    m = np.asarray(mask, dtype=bool)
    cnt = max(int(m.sum()), 1)
    dd = np.where(m, y - t, 0.0)
    loss = float((dd * dd).sum() / cnt)
    gy = np.zeros(y.shape + (16,))
    gy[..., 0] = rb(2.0 * dd / cnt)
    grads = [None] * (2 * D)
    gd, gW, gb = conv_grad(c["d"][0], L[2 * D - 1][0], gy)
    grads[2 * D - 1] = (gW, gb)
    g = np.where(c["d"][0] > 0, rb(gd), 0.0)
    skips = [None] * (D - 1)
    for l in range(D - 1):                      # decoder, finest level first
        gcat, gW, gb = conv_grad(c["cats"][l], L[2 * D - 2 - l][0], g)
        grads[2 * D - 2 - l] = (gW, gb)
        gcat = rb(gcat)
        wu = w[l + 1]
        gu, skips[l] = gcat[..., :wu], gcat[..., wu:]
        nb, n = gu.shape[0], gu.shape[1]
        gnext = rb(gu.reshape(nb, n // 2, 2, n // 2, 2, n // 2, 2, wu).sum(axis=(2, 4, 6)))
        act = c["bt"] if l + 1 == D - 1 else c["d"][l + 1]
        g = np.where(act > 0, gnext, 0.0)
    gp, gW, gb = conv_grad(c["p"][D - 2], L[D - 1][0], g)   # bottleneck
    grads[D - 1] = (gW, gb)
    gp = rb(gp)
    for l in range(D - 2, -1, -1):              # encoder, coarsest level first
        ge = rb(skips[l] + up(gp) / 8.0)
        ge = np.where(c["e"][l] > 0, ge, 0.0)
        gin, gW, gb = conv_grad(c["ins"][l], L[l][0], ge)
        grads[l] = (gW, gb)
        gp = rb(gin)
    flat = np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])
    return loss, flat


def forward_loss(params, x2, t, mask, C: int, bf16: bool = False, depth: int = 3) -> float:
    y, _ = forward(params, x2, C, bf16, depth)
    m = np.asarray(mask, dtype=bool)
    d = np.where(m, y - t, 0.0)
    return float((d * d).sum() / max(int(m.sum()), 1))
