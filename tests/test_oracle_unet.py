"""Pins of the FP64 reference of the steady-state surrogate network: the convolution against
scipy's 2-D correlation, pooling and upsampling against their adjoint identities, and the
hand-derived backward pass against central finite differences of the forward pass."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import unet_oracle as U


def random_layers(rng, scale=1.0):
    layers = []
    for ci, co in zip(U.CIN, U.COUT):
        layers.append((rng.standard_normal((co, 9 * ci)) * scale * np.sqrt(2.0 / (9 * ci)),
                       0.1 * rng.standard_normal(co)))
    return layers


def test_conv_is_zero_padded_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 11, 13, 1))
    k = rng.standard_normal((3, 3))
    W = k.reshape(1, 9)                      # tap 3 ky + kx reads (y + ky - 1, x + kx - 1)
    out = U.conv(x, W, np.array([0.5]))[0, :, :, 0]
    np.testing.assert_allclose(out, correlate2d(x[0, :, :, 0], k, mode="same") + 0.5, rtol=1e-13, atol=1e-13)


def test_conv_channels_add_up():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 6, 8, 3))
    W = rng.standard_normal((2, 27))
    out = U.conv(x, W, np.zeros(2))
    for co in range(2):
        ref = sum(correlate2d(x[n, :, :, ci], W[co].reshape(9, 3)[:, ci].reshape(3, 3), mode="same")
                  for ci in range(3) for n in [0])
        np.testing.assert_allclose(out[0, :, :, co], ref, rtol=1e-12, atol=1e-12)


def test_pool_and_up_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 8, 6, 3))
    y = rng.standard_normal((2, 4, 3, 3))
    assert np.isclose((U.pool(x) * y).sum(), (x * U.pool_backward(y)).sum(), rtol=1e-13)
    z = rng.standard_normal((2, 8, 6, 3))
    assert np.isclose((U.up(y) * z).sum(), (y * U.up_backward(z)).sum(), rtol=1e-13)


def test_packing_round_trip_and_count():
    rng = np.random.default_rng(3)
    layers = random_layers(rng)
    p = U.pack(layers)
    assert p.size == U.param_count()
    for (W, b), (W2, b2) in zip(layers, U.unpack(p)):
        np.testing.assert_array_equal(W, W2)
        np.testing.assert_array_equal(b, b2)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(4)
    layers = random_layers(rng)
    inputs = rng.random((1, 16, 16, 8))
    targets = rng.random((1, 16, 16))
    L0, g = U.loss_and_grad(layers, inputs, targets)
    assert np.isclose(L0, U.loss(layers, inputs, targets), rtol=1e-14)
    checked = 0
    for l in [0, 1, 3, 6, 7, 8, 10, 12, 13, 14]:
        W, b = layers[l]
        co = 0
        idx = [(int(rng.integers(W.shape[0]) if l != 14 else 0), int(rng.integers(W.shape[1]))) for _ in range(3)]
        if l == 0:
            idx = [(i, (j // 16) * 16 + j % 8) for i, j in idx]          # an input channel that is used
        for (i, j) in idx:
            h = 1e-7 * max(1.0, abs(W[i, j]))              # small: no ReLU kink in [-h, h]
            W[i, j] += h
            Lp = U.loss(layers, inputs, targets)
            W[i, j] -= 2 * h
            Lm = U.loss(layers, inputs, targets)
            W[i, j] += h
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[l][0][i, j]) <= 2e-5 * abs(fd) + 1e-10, (l, i, j, fd, g[l][0][i, j])
            checked += 1
        k = 0 if l == 14 else int(rng.integers(b.shape[0]))
        h = 1e-7
        b[k] += h
        Lp = U.loss(layers, inputs, targets)
        b[k] -= 2 * h
        Lm = U.loss(layers, inputs, targets)
        b[k] += h
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[l][1][k]) <= 2e-5 * abs(fd) + 1e-10, (l, "bias", fd, g[l][1][k])
    assert checked == 30
