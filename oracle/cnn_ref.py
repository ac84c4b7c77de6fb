"""FP64 CPU reference of the warm-start network (test infrastructure only).

Plain NumPy forward and backward of the U-Net used by the learned warm start:
4 levels with channels b, 2b, 4b, 8b, two 3x3 convolutions + ReLU per level
(zero padding), 2x2 average pooling, nearest 2x upsampling, skip
concatenation (decoder input = [upsampled, encoder output]), a 1x1 head and a
residual connection out = head + scale * x; loss = mean((out - scale*t)^2).
Parameters use the library's flat layout: all weights [Cout][Cin][k][k] layer
by layer, then all biases layer by layer.

`bf16_storage=True` rounds what the GPU stores in BF16 (network input,
weights, activations, gradients between layers) the same way, so the
comparison isolates accumulation-order differences.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    a = np.asarray(x, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def layers(P, b):
    """(Cin, Cout, ksize, relu) of the 15 layers, in parameter order."""
    return [(P, b, 3, 1), (b, b, 3, 1), (b, 2 * b, 3, 1), (2 * b, 2 * b, 3, 1), (2 * b, 4 * b, 3, 1),
            (4 * b, 4 * b, 3, 1), (4 * b, 8 * b, 3, 1), (8 * b, 8 * b, 3, 1), (12 * b, 4 * b, 3, 1),
            (4 * b, 4 * b, 3, 1), (6 * b, 2 * b, 3, 1), (2 * b, 2 * b, 3, 1), (3 * b, b, 3, 1), (b, b, 3, 1),
            (b, P, 1, 0)]


def unpack(params, P, b):
    Ls = layers(P, b)
    ws, bs, off = [], [], 0
    for ci, co, k, _ in Ls:
        n = co * ci * k * k
        ws.append(params[off:off + n].reshape(co, ci, k, k))
        off += n
    for ci, co, k, _ in Ls:
        bs.append(params[off:off + co])
        off += co
    assert off == params.size
    return ws, bs


def im2col(x, k):
    """x [n][C][H][W] -> [n][C*k*k][H*W], zero padding k//2."""
    n, C, H, W = x.shape
    p = k // 2
    xp = np.pad(x, ((0, 0), (0, 0), (p, p), (p, p)))
    cols = np.empty((n, C, k, k, H, W))
    for ky in range(k):
        for kx in range(k):
            cols[:, :, ky, kx] = xp[:, :, ky:ky + H, kx:kx + W]
    return cols.reshape(n, C * k * k, H * W)


def col2im(cols, C, H, W, k):
    n = cols.shape[0]
    p = k // 2
    cols = cols.reshape(n, C, k, k, H, W)
    xp = np.zeros((n, C, H + 2 * p, W + 2 * p))
    for ky in range(k):
        for kx in range(k):
            xp[:, :, ky:ky + H, kx:kx + W] += cols[:, :, ky, kx]
    return xp[:, :, p:p + H, p:p + W]


def conv(x, w, bias):
    n, C, H, W = x.shape
    co, ci, k, _ = w.shape
    col = im2col(x, k)
    out = np.einsum("ok,nkp->nop", w.reshape(co, -1), col) + bias[None, :, None]
    return out.reshape(n, co, H, W), col


def conv_bwd(g, col, w, x_shape):
    """g: gradient of the pre-activation [n][Co][H][W]; returns (gW, gb, gx)."""
    n, Co, H, W = g.shape
    co, ci, k, _ = w.shape
    gf = g.reshape(n, Co, H * W)
    gW = np.einsum("nop,nkp->ok", gf, col).reshape(w.shape)
    gb = gf.sum(axis=(0, 2))
    gcol = np.einsum("ok,nop->nkp", w.reshape(co, -1), gf)
    gx = col2im(gcol, ci, H, W, k)
    return gW, gb, gx


def pool(x):
    n, C, H, W = x.shape
    return x.reshape(n, C, H // 2, 2, W // 2, 2).mean(axis=(3, 5))


def pool_bwd(g):
    return np.repeat(np.repeat(g, 2, axis=2), 2, axis=3) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def up_bwd(g):
    n, C, H, W = g.shape
    return g.reshape(n, C, H // 2, 2, W // 2, 2).sum(axis=(3, 5))


def loss_and_grad(params, x, t, P, b, scale, bf16_storage=False):
    """Returns (loss, flat gradient) in FP64."""
    R = bf16 if bf16_storage else (lambda a: np.asarray(a, dtype=np.float64))
    ws, bs = unpack(np.asarray(params, np.float64), P, b)
    ws = [R(w) for w in ws]
    Ls = layers(P, b)
    X = R(scale * np.asarray(x, np.float64))
    acts, cols = {}, {}

    def layer(i, inp):
        z, col = conv(inp, ws[i], bs[i])
        cols[i] = col
        o = np.maximum(z, 0.0) if Ls[i][3] else z
        return o

    a1 = R(layer(0, X))
    e1 = R(layer(1, a1))
    p1 = R(pool(e1))
    a2 = R(layer(2, p1))
    e2 = R(layer(3, a2))
    p2 = R(pool(e2))
    a3 = R(layer(4, p2))
    e3 = R(layer(5, a3))
    p3 = R(pool(e3))
    a4 = R(layer(6, p3))
    b4 = R(layer(7, a4))
    cat3 = np.concatenate([R(up(b4)), e3], axis=1)
    d3a = R(layer(8, cat3))
    d3 = R(layer(9, d3a))
    cat2 = np.concatenate([R(up(d3)), e2], axis=1)
    d2a = R(layer(10, cat2))
    d2 = R(layer(11, d2a))
    cat1 = np.concatenate([R(up(d2)), e1], axis=1)
    d1a = R(layer(12, cat1))
    d1 = R(layer(13, d1a))
    out = layer(14, d1) + scale * np.asarray(x, np.float64)
    diff = out - scale * np.asarray(t, np.float64)
    loss = float(np.mean(diff ** 2))
    g = R(2.0 * diff / diff.size)

    gW = [None] * 15
    gB = [None] * 15

    def back(i, gout, out_act, inp):
        gz = gout * (out_act > 0) if Ls[i][3] else gout
        gW[i], gB[i], gx = conv_bwd(gz, cols[i], ws[i], inp.shape)
        return R(gx)

    gd1 = back(14, g, None, d1)
    gd1a = back(13, gd1, d1, d1a)
    gcat1 = back(12, gd1a, d1a, cat1)
    c2 = 2 * b
    gd2 = R(up_bwd(gcat1[:, :c2]))
    ge1 = gcat1[:, c2:]
    gd2a = back(11, gd2, d2, d2a)
    gcat2 = back(10, gd2a, d2a, cat2)
    c3 = 4 * b
    gd3 = R(up_bwd(gcat2[:, :c3]))
    ge2 = gcat2[:, c3:]
    gd3a = back(9, gd3, d3, d3a)
    gcat3 = back(8, gd3a, d3a, cat3)
    c4 = 8 * b
    gb4 = R(up_bwd(gcat3[:, :c4]))
    ge3 = gcat3[:, c4:]
    ga4 = back(7, gb4, b4, a4)
    gp3 = back(6, ga4, a4, p3)
    ge3 = R(ge3 + pool_bwd(gp3))
    ga3 = back(5, ge3, e3, a3)
    gp2 = back(4, ga3, a3, p2)
    ge2 = R(ge2 + pool_bwd(gp2))
    ga2 = back(3, ge2, e2, a2)
    gp1 = back(2, ga2, a2, p1)
    ge1 = R(ge1 + pool_bwd(gp1))
    ga1 = back(1, ge1, e1, a1)
    back(0, ga1, a1, X)
    flat = np.concatenate([gw.ravel() for gw in gW] + [gb.ravel() for gb in gB])
    return loss, flat


def num_params(P, b):
    return sum(co * ci * k * k + co for ci, co, k, _ in layers(P, b))
