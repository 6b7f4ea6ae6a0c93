"""FP64 reference U-Net, its gradients and Adam (oracle; test infrastructure).

Not from the paper: the learned initial guess is an addition around the
paper's shifted solves (Sec. 2, eq. W_k_def).  This module is the plain
definition the GPU network is checked against: the same architecture and
flat parameter layout, written with NumPy in float64, with a hand-written
reverse pass.

Architecture (levels L, base channels C): level l has C 2^l channels.  Encoder
level l: two 3x3 convolutions (zero padding), each followed by ReLU; 2x2
average pooling to the next level.  Decoder level l (from L-2 down to 0):
nearest-neighbour 2x upsampling of the level below, concatenated as
[upsampled, skip], then two 3x3 convolutions with ReLU.  Output: a 1x1
convolution.  Loss: mean squared error.  Optimiser: Adam (Kingma & Ba 2015,
Algorithm 1).

Flat layout: enc_a[0], enc_b[0], ..., enc_a[L-1], enc_b[L-1], dec_a[0],
dec_b[0], ..., dec_a[L-2], dec_b[L-2], out; each as weights [cout][cin][k][k]
then bias [cout].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Conv:
    ci: int
    co: int
    k: int
    w: int      # offset of the weights
    b: int      # offset of the bias


def layout(levels: int, base: int, cin: int, cout: int):
    """Convolutions in flat order: (enc_a, enc_b, dec_a, dec_b, out, total size)."""
    off = 0
    ch = lambda l: base << l

    def conv(ci, co, k):
        nonlocal off
        c = Conv(ci, co, k, off, off + ci * co * k * k)
        off = c.b + co
        return c
    enc_a, enc_b, dec_a, dec_b = [], [], [], []
    for l in range(levels):
        enc_a.append(conv(cin if l == 0 else ch(l - 1), ch(l), 3))
        enc_b.append(conv(ch(l), ch(l), 3))
    for l in range(levels - 1):
        dec_a.append(conv(ch(l + 1) + ch(l), ch(l), 3))
        dec_b.append(conv(ch(l), ch(l), 3))
    out = conv(ch(0), cout, 1)
    return enc_a, enc_b, dec_a, dec_b, out, off


def _wb(p, c: Conv):
    w = p[c.w:c.b].reshape(c.co, c.ci, c.k, c.k)
    return w, p[c.b:c.b + c.co]


def _pad(x):
    return np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))


def conv3(x, w, b):
    """y[n, o, i, j] = sum_c sum_{dy,dx in -1..1} w[o, c, dy+1, dx+1] x[n, c, i+dy, j+dx] + b[o]."""
    n, _, H, W = x.shape
    xp = _pad(x)
    y = np.zeros((n, w.shape[0], H, W))
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("oc,nchw->nohw", w[:, :, ky, kx], xp[:, :, ky:ky + H, kx:kx + W])
    return y + b[None, :, None, None]


def conv3_backward(x, w, dy):
    """Gradients of conv3 with respect to x, w and b, given dL/dy."""
    _, _, H, W = x.shape
    xp = _pad(x)
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            dw[:, :, ky, kx] = np.einsum("nohw,nchw->oc", dy, xp[:, :, ky:ky + H, kx:kx + W])
            dxp[:, :, ky:ky + H, kx:kx + W] += np.einsum("oc,nohw->nchw", w[:, :, ky, kx], dy)
    return dxp[:, :, 1:-1, 1:-1], dw, dy.sum(axis=(0, 2, 3))


def pool(x):
    n, c, H, W = x.shape
    return x.reshape(n, c, H // 2, 2, W // 2, 2).mean(axis=(3, 5))


def pool_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=2), 2, axis=3) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def up_backward(dy):
    n, c, H, W = dy.shape
    return dy.reshape(n, c, H // 2, 2, W // 2, 2).sum(axis=(3, 5))


class UNet:
    """Parameters p (flat float64 vector) and the architecture sizes."""

    def __init__(self, levels: int, base: int, cin: int, cout: int, params: np.ndarray):
        self.L, self.base, self.cin, self.cout = levels, base, cin, cout
        self.enc_a, self.enc_b, self.dec_a, self.dec_b, self.out, n = layout(levels, base, cin, cout)
        params = np.asarray(params, dtype=np.float64)
        assert params.shape == (n,)
        self.p = params.copy()

    def forward(self, x):
        """Output and the cache of activations the reverse pass needs."""
        p, L = self.p, self.L
        cache = {"x": x, "enc1": [], "enc2": [], "pool": [], "up": {}, "dec1": {}, "dec2": {}}
        h = x
        for l in range(L):
            a = np.maximum(conv3(h, *_wb(p, self.enc_a[l])), 0.0)
            b = np.maximum(conv3(a, *_wb(p, self.enc_b[l])), 0.0)
            cache["enc1"].append(a)
            cache["enc2"].append(b)
            if l + 1 < L:
                h = pool(b)
                cache["pool"].append(h)
        cur = cache["enc2"][L - 1]
        for l in range(L - 2, -1, -1):
            u = np.concatenate([up(cur), cache["enc2"][l]], axis=1)
            a = np.maximum(conv3(u, *_wb(p, self.dec_a[l])), 0.0)
            b = np.maximum(conv3(a, *_wb(p, self.dec_b[l])), 0.0)
            cache["up"][l], cache["dec1"][l], cache["dec2"][l] = u, a, b
            cur = b
        w1, b1 = _wb(p, self.out)
        y = np.einsum("oc,nchw->nohw", w1[:, :, 0, 0], cur) + b1[None, :, None, None]
        cache["top"] = cur
        return y, cache

    def loss_and_grad(self, x, target):
        """MSE loss over all outputs and its gradient with respect to the flat parameters."""
        p, L = self.p, self.L
        y, c = self.forward(x)
        loss = float(np.mean((y - target) ** 2))
        g = np.zeros_like(p)
        dy = 2.0 * (y - target) / y.size

        def put(conv, dw, db):
            g[conv.w:conv.b] = dw.ravel()
            g[conv.b:conv.b + conv.co] = db

        w1, _ = _wb(p, self.out)
        put(self.out, np.einsum("nohw,nchw->oc", dy, c["top"])[:, :, None, None], dy.sum(axis=(0, 2, 3)))
        d = np.einsum("oc,nohw->nchw", w1[:, :, 0, 0], dy)
        dskip = {}
        for l in range(L - 1):                      # decoder, top level first
            d = d * (c["dec2"][l] > 0)
            da, dw, db = conv3_backward(c["dec1"][l], _wb(p, self.dec_b[l])[0], d)
            put(self.dec_b[l], dw, db)
            da = da * (c["dec1"][l] > 0)
            du, dw, db = conv3_backward(c["up"][l], _wb(p, self.dec_a[l])[0], da)
            put(self.dec_a[l], dw, db)
            cu = self.base << (l + 1)
            dskip[l] = du[:, cu:]
            d = up_backward(du[:, :cu])
        for l in range(L - 1, -1, -1):              # encoder, bottom level first
            if l < L - 1:
                d = pool_backward(d) + dskip[l]
            d = d * (c["enc2"][l] > 0)
            da, dw, db = conv3_backward(c["enc1"][l], _wb(p, self.enc_b[l])[0], d)
            put(self.enc_b[l], dw, db)
            da = da * (c["enc1"][l] > 0)
            inp = c["x"] if l == 0 else c["pool"][l - 1]
            d, dw, db = conv3_backward(inp, _wb(p, self.enc_a[l])[0], da)
            put(self.enc_a[l], dw, db)
        return loss, g


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns the new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
