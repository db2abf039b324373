"""FP64 reference of the steady-state surrogate network (test infrastructure only).

A plain numpy forward and hand-derived backward pass of the four-level U-Net described in the
library's header: 15 convolutions 3x3 (zero padding, stride 1), ReLU after all but the last,
2x2 average pooling, 2x nearest upsampling, additive skips after the decoder convolution's
ReLU.  Tensors are [B, H, W, C] (NHWC); parameters are packed per layer as W_l [Cout][9 Cin]
(index (3 ky + kx) Cin + ci, reading the input at (y + ky - 1, x + kx - 1)) then b_l [Cout].
The loss is the mean over nodes of (channel 0 of the output - target)^2.

This module shares no code with the HIP library; the tests pin it with finite differences and
with scipy's 2-D correlation.
"""
from __future__ import annotations

import numpy as np

CIN = [16, 32, 32, 64, 64, 128, 128, 256, 256, 128, 128, 64, 64, 32, 32]
COUT = [32, 32, 64, 64, 128, 128, 256, 256, 128, 128, 64, 64, 32, 32, 16]


def param_count() -> int:
    return sum(co * 9 * ci + co for ci, co in zip(CIN, COUT))


def unpack(params: np.ndarray):
    """[(W_l [Cout, 9 Cin], b_l [Cout]) for l in 0..14]."""
    out, o = [], 0
    for ci, co in zip(CIN, COUT):
        W = params[o:o + co * 9 * ci].reshape(co, 9 * ci)
        o += co * 9 * ci
        b = params[o:o + co]
        o += co
        out.append((W, b))
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in layers])


def conv(x, W, b):
    """out[n, y, x, co] = sum_{ky, kx, ci} x[n, y + ky - 1, x + kx - 1, ci] W[co, (3 ky + kx) Cin + ci] + b[co]."""
    B, H, Wd, C = x.shape
    xp = np.zeros((B, H + 2, Wd + 2, C))
    xp[:, 1:H + 1, 1:Wd + 1] = x
    out = np.zeros((B, H, Wd, W.shape[0])) + b
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        out += xp[:, ky:ky + H, kx:kx + Wd] @ W[:, tap * C:(tap + 1) * C].T
    return out


def conv_backward(x, W, dz):
    """Gradients of conv with respect to its weights, bias and input."""
    B, H, Wd, C = x.shape
    xp = np.zeros((B, H + 2, Wd + 2, C))
    xp[:, 1:H + 1, 1:Wd + 1] = x
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    dz2 = dz.reshape(-1, dz.shape[-1])
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        patch = xp[:, ky:ky + H, kx:kx + Wd].reshape(-1, C)
        dW[:, tap * C:(tap + 1) * C] = dz2.T @ patch
        dxp[:, ky:ky + H, kx:kx + Wd] += (dz2 @ W[:, tap * C:(tap + 1) * C]).reshape(B, H, Wd, C)
    return dW, dz2.sum(axis=0), dxp[:, 1:H + 1, 1:Wd + 1]


def pool(x):
    B, H, Wd, C = x.shape
    return x.reshape(B, H // 2, 2, Wd // 2, 2, C).mean(axis=(2, 4))


def pool_backward(d):
    return np.repeat(np.repeat(d, 2, axis=1), 2, axis=2) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_backward(d):
    B, H, Wd, C = d.shape
    return d.reshape(B, H // 2, 2, Wd // 2, 2, C).sum(axis=(2, 4))


def relu(z):
    return np.maximum(z, 0.0)


def pack_input(inputs):
    """[B, H, W, 8] -> [B, H, W, 16] with channels 8..15 zero."""
    x = np.zeros(inputs.shape[:3] + (16,))
    x[..., :8] = inputs
    return x


def forward(layers, inputs):
    """Output [B, H, W, 16] and the intermediates the backward pass needs."""
    c = {}
    L = layers
    c["x0"] = pack_input(inputs)
    c["a0"] = relu(conv(c["x0"], *L[0]))
    c["s0"] = relu(conv(c["a0"], *L[1]))
    c["p0"] = pool(c["s0"])
    c["a1"] = relu(conv(c["p0"], *L[2]))
    c["s1"] = relu(conv(c["a1"], *L[3]))
    c["p1"] = pool(c["s1"])
    c["a2"] = relu(conv(c["p1"], *L[4]))
    c["s2"] = relu(conv(c["a2"], *L[5]))
    c["p2"] = pool(c["s2"])
    c["a3"] = relu(conv(c["p2"], *L[6]))
    c["b3"] = relu(conv(c["a3"], *L[7]))
    c["u3"] = up(c["b3"])
    c["r8"] = relu(conv(c["u3"], *L[8]))
    c["u2"] = c["r8"] + c["s2"]
    c["v2"] = relu(conv(c["u2"], *L[9]))
    c["up2"] = up(c["v2"])
    c["r10"] = relu(conv(c["up2"], *L[10]))
    c["u1"] = c["r10"] + c["s1"]
    c["v1"] = relu(conv(c["u1"], *L[11]))
    c["up1"] = up(c["v1"])
    c["r12"] = relu(conv(c["up1"], *L[12]))
    c["u0"] = c["r12"] + c["s0"]
    c["v0"] = relu(conv(c["u0"], *L[13]))
    out = conv(c["v0"], *L[14])
    return out, c


def loss(layers, inputs, targets) -> float:
    out, _ = forward(layers, inputs)
    return float(np.mean((out[..., 0] - targets) ** 2))


def loss_and_grad(layers, inputs, targets):
    """Loss and [(dW_l, db_l)] by the chain rule, layer by layer."""
    out, c = forward(layers, inputs)
    npix = targets.size
    d = out[..., 0] - targets
    L = float(np.mean(d ** 2))
    g = [None] * 15
    dout = np.zeros_like(out)
    dout[..., 0] = 2.0 * d / npix

    def back(l, x, y, dy):
        """conv l with input x and ReLU output y (None: no ReLU), output gradient dy."""
        dz = dy if y is None else dy * (y > 0)
        dW, db, dx = conv_backward(x, layers[l][0], dz)
        g[l] = (dW, db)
        return dx

    dv0 = back(14, c["v0"], None, dout)
    du0 = back(13, c["u0"], c["v0"], dv0)
    dup1 = back(12, c["up1"], c["r12"], du0)
    dv1 = up_backward(dup1)
    du1 = back(11, c["u1"], c["v1"], dv1)
    dup2 = back(10, c["up2"], c["r10"], du1)
    dv2 = up_backward(dup2)
    du2 = back(9, c["u2"], c["v2"], dv2)
    du3 = back(8, c["u3"], c["r8"], du2)
    db3 = up_backward(du3)
    da3 = back(7, c["a3"], c["b3"], db3)
    dp2 = back(6, c["p2"], c["a3"], da3)
    ds2 = du2 + pool_backward(dp2)
    da2 = back(5, c["a2"], c["s2"], ds2)
    dp1 = back(4, c["p1"], c["a2"], da2)
    ds1 = du1 + pool_backward(dp1)
    da1 = back(3, c["a1"], c["s1"], ds1)
    dp0 = back(2, c["p0"], c["a1"], da1)
    ds0 = du0 + pool_backward(dp0)
    da0 = back(1, c["a0"], c["s0"], ds0)
    back(0, c["x0"], c["a0"], da0)
    return L, g
