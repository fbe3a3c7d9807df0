"""Element-wise error bounds of the GPU's CNN against the FP64 oracle (test
helper; no part of the method).

The GPU runs the oracle's network with its weights rounded to BF16 (the oracle
uses the same rounded weights), stores every activation and every
backpropagated gradient in BF16 and accumulates in FP32. Rounding to nearest
changes a value x by at most r |x| (r = 2^-8 for BF16, 2^-24 for FP32), spread
evenly over that interval: variance (r x)^2 / 3, independent between values.
A sum of n terms in FP32 adds at most n such errors of its partial sums.
Propagated to first order through the layers these give every output and
every gradient element a standard deviation sigma, and the test bound is
K sigma with K = 6. A ReLU passes its input's deviation on with a factor of
at most 1; where its input lies within its own bound of 0 the two sides may
take different branches, and the backward pass then differs by the whole
gradient there, which enters as a further independent term. A correct
kernel exceeds 6 sigma somewhere among 10^5 elements with probability about
10^-4; a local mistake (a wrong tap, channel or row in one tile) is off by
the size of the terms themselves.

Layout as in the oracle: activations [S][N][C], site v = x + L y + L^2 z,
conv tap d = (dz+1) 9 + (dy+1) 3 + (dx+1).
"""
from __future__ import annotations

import numpy as np

U = 2.0 ** -8     # BF16 rounding, relative
EPS = 2.0 ** -24  # FP32 rounding, relative
K = 6.0           # standard deviations of the bound


def _grid(a, L):
    return a.reshape(a.shape[0], L, L, L, a.shape[-1])  # [S][z][y][x][C]


def _offsets():
    for d in range(27):
        yield d, d % 3 - 1, (d // 3) % 3 - 1, d // 9 - 1


def conv(x, W, L, b=None):
    """y[v][co] = b[co] + sum_{d,ci} W[d][ci][co] x[v + off(d)][ci] (periodic)."""
    X = _grid(x, L)
    y = np.zeros(X.shape[:4] + (W.shape[2],))
    for d, dx, dy, dz in _offsets():
        y += np.roll(X, shift=(-dz, -dy, -dx), axis=(1, 2, 3)) @ W[d]
    y = y.reshape(x.shape[0], -1, W.shape[2])
    return y if b is None else y + b


def conv_t(g, W, L):
    """dx[u][ci] = sum_{d,co} W[d][ci][co] g[u - off(d)][co]."""
    G = _grid(g, L)
    out = np.zeros(G.shape[:4] + (W.shape[1],))
    for d, dx, dy, dz in _offsets():
        out += np.roll(G, shift=(dz, dy, dx), axis=(1, 2, 3)) @ W[d].T
    return out.reshape(g.shape[0], -1, W.shape[1])


def wgrad(x, g, L):
    """dW[d][ci][co] = sum_v x[v + off(d)][ci] g[v][co] over all shots."""
    X = _grid(x, L)
    G = g.reshape(-1, g.shape[-1])
    out = np.zeros((27, x.shape[-1], g.shape[-1]))
    for d, dx, dy, dz in _offsets():
        Xs = np.roll(X, shift=(-dz, -dy, -dx), axis=(1, 2, 3)).reshape(-1, x.shape[-1])
        out[d] = Xs.T @ G
    return out


def rounding_var(x, r=U):
    return (r * x) ** 2 / 3.0


def accumulation_var(n, mag):
    """FP32 sum of n terms whose magnitudes sum to mag."""
    return n * rounding_var(mag, EPS)


def forward_bounds(x0, layers, L):
    """Oracle-precision pre-activations y_l and activations a_l, and the
    variance V of the GPU's deviation of every pre-activation (the logits z
    last)."""
    a = [x0]
    ys, V = [], []
    var_in = np.zeros_like(x0)  # the input bits are exact
    for li, (W, b) in enumerate(layers):
        n = W.shape[0] * W.shape[1] + 1
        y = conv(a[-1], W, L, b)
        v = conv(var_in, W * W, L) + accumulation_var(n, conv(np.abs(a[-1]), np.abs(W), L) +
                                                      np.abs(b))
        ys.append(y)
        V.append(v)
        if li < len(layers) - 1:
            act = np.maximum(y, 0.0)
            a.append(act)
            near = np.abs(y) <= K * np.sqrt(v)  # the branch may differ
            m = np.where(near, 1.0, (y > 0).astype(np.float64))
            var_in = m * v + rounding_var(act)
    return ys, a, V


def forward_bound(x0, layers, L):
    """(z, bound) of the logits."""
    ys, _, V = forward_bounds(x0, layers, L)
    return ys[-1], K * np.sqrt(V[-1])


def gradient_bounds(x0, layers, L, target, count):
    """Gradients of the mean BCE of the logits against target [S][N][3]
    (`count` terms in the mean) and their bounds, per layer (dW, bound, db,
    bound), then the loss and its bound."""
    ys, a, V = forward_bounds(x0, layers, L)
    z = ys[-1]
    sig = 1.0 / (1.0 + np.exp(-z))
    dz = (sig - target) / count
    dsig = sig * (1.0 - sig)
    # the GPU's dz: the sigmoid of its own z, scaled, rounded to BF16
    Vg = (dsig / count) ** 2 * V[-1] + rounding_var(dz)
    g = dz
    R = x0.shape[0] * x0.shape[1]  # rows summed by a weight gradient
    out = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        x = a[li]
        Vx = np.zeros_like(x) if li == 0 else rounding_var(x) + V[li - 1]
        gw = wgrad(x, g, L)
        var_w = wgrad(Vx, g * g, L) + wgrad(x * x, Vg, L) + \
            accumulation_var(R, wgrad(np.abs(x), np.abs(g), L))
        gb = g.reshape(-1, g.shape[-1]).sum(axis=0)
        var_b = Vg.reshape(-1, g.shape[-1]).sum(axis=0) + \
            accumulation_var(R, np.abs(g).reshape(-1, g.shape[-1]).sum(axis=0))
        out[li] = (gw, K * np.sqrt(var_w), gb, K * np.sqrt(var_b))
        if li == 0:
            break
        n = W.shape[0] * W.shape[2]
        G = conv_t(g, W, L)
        VG = conv_t(Vg, W * W, L) + accumulation_var(n, conv_t(np.abs(g), np.abs(W), L))
        y = ys[li - 1]
        near = np.abs(y) <= K * np.sqrt(V[li - 1])
        mask = (y > 0).astype(np.float64)
        g = mask * G
        Vg = np.where(near, VG + G * G, mask * VG) + rounding_var(g)
    sp = np.maximum(z, 0) + np.log1p(np.exp(-np.abs(z)))
    terms = sp - target * z
    loss = float(terms.sum() / count)
    dl = sig - target  # d(term)/dz
    loss_bound = float(K * np.sqrt((dl * dl * V[-1]).sum() +
                                   accumulation_var(R * 3, np.abs(terms).sum())) / count)
    return out, loss, loss_bound
