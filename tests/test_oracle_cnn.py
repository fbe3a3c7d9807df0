"""Pins of the oracle's CNN prior (periodic 3x3x3 convolutions, ReLU, binary
cross-entropy): the gradient against central finite differences, the offset
convention, translation equivariance and the zero-parameter closed forms."""
import math

import numpy as np
import pytest

from inputs import random_bits, site
from oracle.oracle import CNN_CHANNELS, Oracle, cnn_layers, cnn_param_count


def random_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    p = np.zeros(cnn_param_count())
    for W, b in cnn_layers(p):
        fan_in = W.shape[0] * W.shape[1]
        W[...] = rng.normal(0, scale * math.sqrt(2.0 / fan_in), W.shape) * 3
        b[...] = rng.normal(0, 0.1, b.shape)
    return p


def test_param_count():
    n = sum(27 * a * b + b for a, b in zip(CNN_CHANNELS[:-1], CNN_CHANNELS[1:]))
    assert cnn_param_count() == n == 64899


def test_input_channels():
    L = 3
    o = Oracle(L)
    syn = random_bits(1, 2, o.n_faces, 0.5)
    prev = random_bits(2, 2, o.n_faces, 0.5)
    x0 = o.cnn_input(syn, prev)
    N = L ** 3
    for s in range(2):
        for v in (0, 5, 26):
            for n in range(3):
                assert x0[s, v, n] == syn[s, n * N + v]
                assert x0[s, v, 3 + n] == prev[s, n * N + v]
            assert x0[s, v, 6] == x0[s, v, 7] == 0


def test_gradient_matches_finite_differences():
    L, S = 3, 2
    o = Oracle(L)
    x0 = o.cnn_input(random_bits(3, S, o.n_faces, 0.3), random_bits(4, S, o.n_faces, 0.3))
    target = random_bits(5, S, o.n_edges, 0.2)
    params = random_params(6)
    loss, grad = o.cnn_loss_grad(x0, params, target)
    rng = np.random.default_rng(7)
    # a spread of weights and biases of every layer
    idx, off = [], 0
    for cin, cout in zip(CNN_CHANNELS[:-1], CNN_CHANNELS[1:]):
        nW = 27 * cin * cout
        idx += list(off + rng.choice(nW, size=12, replace=False))
        idx += list(off + nW + rng.choice(cout, size=min(3, cout), replace=False))
        off += nW + cout
    eps = 1e-6
    worst = 0.0
    for i in idx:
        p1, p2 = params.copy(), params.copy()
        p1[i] += eps
        p2[i] -= eps
        fd = (o.cnn_loss_grad(x0, p1, target)[0] - o.cnn_loss_grad(x0, p2, target)[0]) / (2 * eps)
        err = abs(fd - grad[i]) / max(abs(fd), 1e-7)
        worst = max(worst, err)
        assert abs(fd - grad[i]) <= 1e-6 * max(abs(fd), 1e-4), (i, fd, grad[i])
    assert worst < 1e-4


def test_offset_convention_and_wiring():
    """A network that copies input channel 0 from the +x neighbour in layer 1
    and passes it through the centre tap of the other layers outputs
    z[v][0] = x0[v + unit(x)][0]."""
    L = 4
    o = Oracle(L)
    params = np.zeros(cnn_param_count())
    layers = cnn_layers(params)
    d_plus_x = (0 + 1) * 9 + (0 + 1) * 3 + (1 + 1)  # dz=0, dy=0, dx=+1
    centre = 13
    layers[0][0][d_plus_x, 0, 0] = 1.0
    for W, _ in layers[1:]:
        W[centre, 0, 0] = 1.0
    syn = random_bits(8, 1, o.n_faces, 0.5)
    x0 = o.cnn_input(syn)
    z = o.cnn_forward(x0, params)
    for zz in range(L):
        for yy in range(L):
            for xx in range(L):
                assert z[0, site(L, xx, yy, zz), 0] == x0[0, site(L, xx + 1, yy, zz), 0]
    assert np.all(z[0, :, 1:] == 0)


def test_translation_equivariance():
    L = 4
    o = Oracle(L)
    N = L ** 3
    syn = random_bits(9, 1, o.n_faces, 0.4)
    prev = random_bits(10, 1, o.n_faces, 0.4)
    params = random_params(11)
    z = o.cnn_forward(o.cnn_input(syn, prev), params)

    def shift_faces(a, dx, dy, dz):
        out = np.empty_like(a)
        for n in range(3):
            for zz in range(L):
                for yy in range(L):
                    for xx in range(L):
                        out[0, n * N + site(L, xx + dx, yy + dy, zz + dz)] = \
                            a[0, n * N + site(L, xx, yy, zz)]
        return out

    z2 = o.cnn_forward(o.cnn_input(shift_faces(syn, 1, 2, 3), shift_faces(prev, 1, 2, 3)), params)
    for zz in range(L):
        for yy in range(L):
            for xx in range(L):
                np.testing.assert_allclose(z2[0, site(L, xx + 1, yy + 2, zz + 3)],
                                           z[0, site(L, xx, yy, zz)], rtol=1e-12, atol=1e-12)


def test_zero_parameters_closed_form():
    """All-zero parameters: every logit is 0, the loss is ln 2 and the last
    bias gradient of channel c is (S N / 2 - #errors on axis c) / (3 S N)."""
    L, S = 3, 3
    o = Oracle(L)
    N = L ** 3
    x0 = o.cnn_input(random_bits(12, S, o.n_faces, 0.5))
    target = random_bits(13, S, o.n_edges, 0.3)
    params = np.zeros(cnn_param_count())
    loss, grad = o.cnn_loss_grad(x0, params, target)
    assert abs(loss - math.log(2)) < 1e-12
    b4 = cnn_layers(grad)[3][1]
    for c in range(3):
        want = (S * N * 0.5 - target[:, c * N:(c + 1) * N].sum()) / (3 * S * N)
        assert abs(b4[c] - want) < 1e-12
    # with zero weights nothing reaches the earlier layers
    assert np.all(cnn_layers(grad)[0][0] == 0)
