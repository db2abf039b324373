"""The steady-state surrogate network's HIP kernels (forward, backward, Adam) against the FP64
numpy reference, through the C ABI.

Bars: BF16 activations and weights with FP32 accumulation against FP64.  The prediction and the
loss agree to 2e-2 (15 BF16 roundings at unit 2^-9 compound to about 3e-2 in the worst case;
measured 4e-3).  Gradients travel back through another 15 roundings, and a ReLU whose
pre-activation rounds across zero switches a path on or off, so every layer's weight and bias
gradient agrees to 1e-1 (rel-L2; measured 3.5e-2 at 32 x 32, 6.6e-2 for the 3 x 5-pixel bottom
level of the 24 x 40 case, where nothing averages out); a wrong tap, index or transpose gives
errors of order one.  The 256 x 256 case runs every level at a width the row-segment weight
gradients take."""
import sys

import numpy as np
import pytest
import torch

from oracle import unet_oracle as U
from paper_1503_06726_amd import lbib

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def bf16_round(x):
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def random_case(seed, B, H, W):
    rng = np.random.default_rng(seed)
    layers = []
    for l, (ci, co) in enumerate(zip(U.CIN, U.COUT)):
        Wl = rng.standard_normal((co, 9 * ci)) * np.sqrt(2.0 / (9 * ci))
        bl = 0.05 * rng.standard_normal(co)
        layers.append((Wl, bl))
    inputs = np.zeros((B, H, W, 8))
    inputs[..., 0] = rng.random((B, H, W)) < 0.3
    inputs[..., 1] = rng.random((B, H, W)) < 0.1
    inputs[..., 2] = rng.uniform(-1, 1, (B, 1, 1))
    inputs[..., 3] = rng.uniform(-1, 1, (B, 1, 1))
    inputs[..., 4] = rng.uniform(-1, 1, (B, 1, 1))
    targets = rng.random((B, H, W))
    return layers, inputs, targets


@pytest.mark.parametrize("B,H,W", [(2, 32, 32), (1, 24, 40), (1, 256, 256)])
def test_net_loss_and_gradients_match_reference(B, H, W):
    layers, inputs, targets = random_case(7, B, H, W)
    params = U.pack(layers).astype(np.float32)
    net = lbib.Net(H, W, B)
    net.set_params(params)
    xin = torch.tensor(inputs, dtype=torch.float32, device="cuda")
    tg = torch.tensor(targets, dtype=torch.float32, device="cuda")
    out = torch.zeros((B, H, W), dtype=torch.float32, device="cuda")
    net.predict(xin.data_ptr(), B, out.data_ptr())
    loss, grad = net.loss_grad(xin.data_ptr(), tg.data_ptr(), B)
    net.close()
    # reference with the same BF16-rounded weights and inputs (biases stay FP32 on the GPU)
    ref_layers = [(bf16_round(Wl), bl.astype(np.float32).astype(np.float64)) for Wl, bl in layers]
    ref_out, _ = U.forward(ref_layers, bf16_round(inputs))
    ref_loss, g = U.loss_and_grad(ref_layers, bf16_round(inputs), targets)
    r_out = rel(out.cpu().numpy(), ref_out[..., 0])
    say(f"  prediction rel-L2 {r_out:.2e}; loss GPU {loss:.6e} reference {ref_loss:.6e}")
    assert r_out <= 2e-2
    assert abs(loss - ref_loss) <= 2e-2 * ref_loss
    gl = U.unpack(grad.astype(np.float64))
    errs = [(rel(gl[l][0], g[l][0]), rel(gl[l][1], g[l][1])) for l in range(15)]
    say("  layer gradient rel-L2 (W, b): " + " ".join(f"{a:.1e}/{b:.1e}" for a, b in errs))
    for l, (rw, rb) in enumerate(errs):
        assert rw <= 1e-1 and rb <= 1e-1, (l, rw, rb)


def test_net_training_reduces_loss():
    # a small learnable map: the target is a fixed smoothing of the first input channel
    rng = np.random.default_rng(3)
    B, H, W = 4, 32, 32
    inputs = np.zeros((B, H, W, 8))
    inputs[..., 0] = rng.random((B, H, W)) < 0.2
    k = np.ones(5) / 5
    sm = inputs[..., 0]
    for ax in (1, 2):
        sm = np.apply_along_axis(lambda v: np.convolve(np.pad(v, 2, mode="wrap"), k, mode="valid"), ax, sm)
    layers, _, _ = random_case(9, B, H, W)
    layers[14] = (layers[14][0] * 0.1, np.zeros(16))
    net = lbib.Net(H, W, B)
    net.set_params(U.pack(layers).astype(np.float32))
    xin = torch.tensor(inputs, dtype=torch.float32, device="cuda")
    tg = torch.tensor(sm, dtype=torch.float32, device="cuda")
    first = net.train_step(xin.data_ptr(), tg.data_ptr(), B, 1e-3)
    for _ in range(300):
        last = net.train_step(xin.data_ptr(), tg.data_ptr(), B, 1e-3)
    net.close()
    say(f"  loss {first:.3e} -> {last:.3e}")
    assert last < 0.1 * first
