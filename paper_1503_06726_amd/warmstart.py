"""Learned warm start of the species' steady state.

The surrogate network (``lbib.Net``, a BF16 U-Net trained by the library's kernels) maps
per-node features of a static tissue sample to the dimensionless steady concentration
phi * decay / source:

  0  source mask        1 inside a source cell
  1  boundary mask      1 where a 4-neighbour carries another domain ID (the membranes)
  2  diffusivity        (D - 0.26) / 0.14
  3  decay              (log10(decay) + 4) / 0.6
  4  source fraction    (fraction of the domain inside source cells - 0.15) / 0.1
  5-7                   zero

The source fraction fixes the level of the slowest (uniform) mode, sigma * fraction / decay,
which a network of local convolutions could not see across the whole domain.

The prediction, scaled back by source / decay, seeds the D2Q5 populations (equilibrium
w_i phi); the ADE-only iteration then runs to the same tolerance as from zero, so the
prediction only changes how many iterations are needed.  Geometry, masks and features are
host-side preparation; every solve, prediction and training step runs in the library.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import time

import numpy as np

from . import lbib
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "data", "warmstart_unet.npz")

SOURCE = 1e-3          # source rate of the static-tissue samples


def init_params(seed: int, n_params: int | None = None) -> np.ndarray:
    """He-normal weights N(0, 2 / (9 Cin_used)), zero biases; the input channels of the first
    convolution beyond the five features and the unused output channels of the last are zero,
    and the last is scaled by 0.1 (packed in the library's layer order)."""
    cin = [16, 32, 32, 64, 64, 128, 128, 256, 256, 128, 128, 64, 64, 32, 32]
    cout = [32, 32, 64, 64, 128, 128, 256, 256, 128, 128, 64, 64, 32, 32, 16]
    rng = np.random.default_rng(np.random.SeedSequence([1503, 7, seed]))
    parts = []
    for l, (ci, co) in enumerate(zip(cin, cout)):
        used = 5 if l == 0 else ci
        w = rng.standard_normal((co, 9, ci)) * np.sqrt(2.0 / (9 * used))
        if l == 0:
            w[:, :, 5:] = 0.0
        if l == 14:
            w *= 0.1
            w[1:] = 0.0
        parts += [w.reshape(-1), np.zeros(co)]
    p = np.concatenate(parts).astype(np.float32)
    if n_params is not None and p.size != n_params:
        raise ValueError(f"parameter count {p.size} != network's {n_params}")
    return p


def id_map(w, stream=None) -> np.ndarray:
    """Domain-ID map of a workload's cells, rasterised by the library."""
    s = lbib.Simulation(w.params_dict(), stream=stream)
    s.set_cells(w.offsets, w.xy, w.rest_len, w.rest_area)
    m = s.get_fields(rho=False, u=False, phi=False, xy=False, mask=True)["mask"]
    s.close()
    return m


def masks(w, ids: np.ndarray):
    """(source mask, boundary mask) as uint8 [ny, nx]."""
    src_ids = np.flatnonzero(np.asarray(w.source_cells) != 0) + 1
    source = np.isin(ids, src_ids).astype(np.uint8)
    b = np.zeros(ids.shape, bool)
    b |= ids != np.roll(ids, 1, axis=1)
    b |= ids != np.roll(ids, -1, axis=1)
    b[1:] |= ids[1:] != ids[:-1]
    b[:-1] |= ids[:-1] != ids[1:]
    return source, b.astype(np.uint8)


IN_CH = 8


def features(w, source: np.ndarray, boundary: np.ndarray) -> np.ndarray:
    """[ny, nx, 8] float32 network input of one sample."""
    D, lam = w.species[0].D, w.species[0].c[1]
    f = np.zeros(source.shape + (IN_CH,), np.float32)
    f[..., 0] = source
    f[..., 1] = boundary
    f[..., 2] = (D - 0.26) / 0.14
    f[..., 3] = (np.log10(lam) + 4.0) / 0.6
    f[..., 4] = (float(source.mean()) - 0.15) / 0.1
    return f


def generate(indices, held_out: bool, workers: int = 8):
    """Static-tissue workloads for the given sample indices (host; a process pool when
    workers > 1, which must then run before the process touches the GPU)."""
    idx = list(indices)
    if workers <= 1:
        return [W.static_tissue(i, held_out) for i in idx]
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(W.static_tissue, idx, [held_out] * len(idx)))


def prepare(ws, stream=None):
    """Source masks, boundary masks and features of a list of workloads."""
    src, bnd, feat = [], [], []
    for w in ws:
        ids = id_map(w, stream)
        s, b = masks(w, ids)
        src.append(s)
        bnd.append(b)
        feat.append(features(w, s, b))
    return np.stack(src), np.stack(bnd), np.stack(feat)


def solve(ws, source: np.ndarray, phi0=None, tol: float = 1e-6, fp64: bool = True, batch: int = 64,
          max_iters: int = 1_000_000, stream=None):
    """Batched ADE-only steady states (one lattice size); samples are grouped by decay so a
    batch converges together.  Returns (iterations [N], phi [N, ny, nx])."""
    n = len(ws)
    ny, nx = ws[0].ny, ws[0].nx
    order = np.argsort([-w.species[0].c[1] for w in ws], kind="stable")
    its = np.zeros(n, np.int64)
    phi = np.zeros((n, ny, nx))
    for k in range(0, n, batch):
        idx = order[k:k + batch]
        D = [ws[i].species[0].D for i in idx]
        lam = [ws[i].species[0].c[1] for i in idx]
        p0 = None if phi0 is None else phi0[idx]
        it, ph = lbib.ade_batch(nx, ny, ws[0].bc_y, source[idx], D, [SOURCE] * len(idx), lam, phi0=p0, tol=tol,
                                max_iters=max_iters, fp64=fp64, stream=stream)
        its[idx] = it
        phi[idx] = ph
    return its, phi


def scale(w) -> float:
    """phi = prediction * scale(w)."""
    return SOURCE / w.species[0].c[1]


def save(params: np.ndarray, meta: dict, path: str = WEIGHTS):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez_compressed(path, params=np.asarray(params, np.float32), meta=np.array(json.dumps(meta)))


def load(path: str = WEIGHTS):
    """(params float32, meta dict); plain arrays only (no pickles)."""
    with np.load(path, allow_pickle=False) as z:
        return z["params"], json.loads(str(z["meta"]))


def predict(net: "lbib.Net", feats: np.ndarray, ws, batch: int = 16) -> np.ndarray:
    """phi-hat [N, ny, nx] (float64, clipped at 0) of a list of samples."""
    import torch
    n, ny, nx = feats.shape[0], feats.shape[1], feats.shape[2]
    out = np.zeros((n, ny, nx))
    o = torch.zeros((batch, ny, nx), dtype=torch.float32, device="cuda")
    for k in range(0, n, batch):
        x = torch.tensor(feats[k:k + batch], dtype=torch.float32, device="cuda").contiguous()
        b = x.shape[0]
        net.predict(x.data_ptr(), b, o.data_ptr())
        y = o[:b].cpu().numpy().astype(np.float64)
        for j in range(b):
            out[k + j] = np.maximum(y[j], 0.0) * scale(ws[k + j])
    return out


def train(net: "lbib.Net", feats, targets, epochs: int, batch: int = 16, lr: float = 1e-3, lr_min: float = 1e-5,
          seed: int = 0, log=print):
    """Adam over shuffled mini-batches with a cosine learning-rate decay; feats [N, ny, nx, 8]
    and targets [N, ny, nx] (dimensionless) are torch CUDA tensors.  Returns the mean loss of
    every epoch."""
    import torch
    n = feats.shape[0]
    rng = np.random.default_rng(seed)
    steps = epochs * (n // batch)
    hist, k = [], 0
    for e in range(epochs):
        perm = torch.tensor(rng.permutation(n), device="cuda")
        tot, cnt = 0.0, 0
        t0 = time.perf_counter()
        for s in range(n // batch):
            idx = perm[s * batch:(s + 1) * batch]
            x = feats.index_select(0, idx).contiguous()
            y = targets.index_select(0, idx).contiguous()
            a = lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * k / max(steps - 1, 1)))
            tot += net.train_step(x.data_ptr(), y.data_ptr(), batch, a)
            cnt += 1
            k += 1
        hist.append(tot / max(cnt, 1))
        log(f"epoch {e + 1}/{epochs}: mean loss {hist[-1]:.4e} ({time.perf_counter() - t0:.1f} s)")
    return hist
