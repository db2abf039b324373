"""Steady state of the ADE-only iteration by a sparse direct solve (test infrastructure only).

With u = 0 and the source/decay law R = sigma m(x) - lambda phi (or no reaction), one
iteration of a species lattice is linear in its populations g (D2Q5 equations of the
supplementary "Lattice Boltzmann Method" section):

    collision  g_i' = g_i - (g_i - w_i phi) / tau_D + w_i (sigma m - lambda phi),  phi = sum_j g_j
    streaming  g_i(x + v_i) = g_i'(x), or, across a wall (halfway bounce-back),
               g_opp(i)(x) = g_i'(x)

i.e. g <- P (A g + b) with A the per-node 5x5 collision matrix
(1 - 1/tau_D) I + (1/tau_D - lambda) w 1^T, b = sigma m w, and P the streaming
permutation.  The fixed point solves (I - P A) g = P b.  Populations are indexed
i * nx * ny + y * nx + x.  This module builds the matrix from those equations directly
(it shares nothing with the C oracle or the HIP library).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

VX = np.array([0, 1, 0, -1, 0])
VY = np.array([0, 0, 1, 0, -1])
OPP = np.array([0, 3, 4, 1, 2])
W = np.array([1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6])


def streaming_matrix(nx: int, ny: int, walls: bool) -> sp.csr_matrix:
    """P with (P g)[dest] = g[src] for the D2Q5 free flight (x periodic, y periodic or walls)."""
    nn = nx * ny
    y, x = np.divmod(np.arange(nn), nx)
    rows, cols = [], []
    for i in range(5):
        src = i * nn + y * nx + x
        yd = y + VY[i]
        xd = (x + VX[i]) % nx
        if walls:
            out = (yd < 0) | (yd >= ny)
            dest = np.where(out, OPP[i] * nn + y * nx + x, i * nn + np.clip(yd, 0, ny - 1) * nx + xd)
        else:
            dest = i * nn + (yd % ny) * nx + xd
        rows.append(dest)
        cols.append(src)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    return sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(5 * nn, 5 * nn))


def steady_state(nx: int, ny: int, walls: bool, D: float, source: float, decay: float,
                 m: np.ndarray) -> np.ndarray:
    """phi* [ny, nx] of the ADE-only iteration; m [ny, nx] is the source indicator (0/1)."""
    nn = nx * ny
    tau = 3.0 * D + 0.5
    blockA = (1.0 - 1.0 / tau) * np.eye(5) + (1.0 / tau - decay) * np.outer(W, np.ones(5))
    A = sp.kron(sp.csr_matrix(blockA), sp.identity(nn, format="csr"), format="csr")
    b = source * np.kron(W, (np.asarray(m, dtype=np.float64).reshape(-1) != 0).astype(np.float64))
    P = streaming_matrix(nx, ny, walls)
    M = (sp.identity(5 * nn, format="csr") - P @ A).tocsc()
    g = spla.spsolve(M, P @ b)
    return g.reshape(5, ny, nx).sum(axis=0)
