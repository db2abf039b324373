"""Parity at the workloads' own horizons, through the C ABI: the tissue workload (512^2, 100
Voronoi cells, two Schnakenberg species) over its 10,000 steps and the large workload (2048^2,
2000 cells, the bench's workload and launch configuration) over its 5,000, against the FP64
oracle's checkpoints.  The checkpoints (tests/golden/horizon_*.npz) were written by
make_horizon_goldens.py, which calls only the oracle and the seeded workload generator; they
hold the oracle's fields at seeded samples of lattice and membrane nodes (32,768 and 16,384),
its global sums, and its domain-ID map at the last checkpoint.

Bars at every checkpoint (tissue 100, 1,000, 10,000 steps; large 48, 100, 160, 1,000, 5,000),
over the sampled nodes: u, phi and X - X0 within 1e-5 relative L2; rho - rho0 within 1e-5 of
its size plus the FP32 rounding floor of the stored deviations (parity_bars); the lattice
sums of rho within 1e-9, of phi within 1e-5, of the momentum within 1e-4 relative (FP32
deviations); at the last checkpoint, domain IDs that differ only at lattice nodes within 1e-3
of a membrane edge.
"""
import os
import sys

import numpy as np
import pytest

import parity_bars as PB
from paper_1503_06726_amd import lbib
from paper_1503_06726_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def near_edge(offsets, xy, px, py, nx, ny):
    """Distance from lattice points (px, py) to the nearest membrane edge (periodic images);
    only the cells whose bounding box comes within 2 lattice units are measured."""
    d = np.full(px.shape, np.inf)
    for c in range(len(offsets) - 1):
        P = xy[offsets[c]:offsets[c + 1]]
        Q = np.roll(P, -1, 0)
        for sx in (-nx, 0, nx):
            for sy in (-ny, 0, ny):
                lo, hi = P.min(0) + (sx, sy) - 2.0, P.max(0) + (sx, sy) + 2.0
                sel = (px >= lo[0]) & (px <= hi[0]) & (py >= lo[1]) & (py <= hi[1])
                if not sel.any():
                    continue
                p = np.stack([px[sel] - sx, py[sel] - sy], -1)[:, None, :]
                ab = (Q - P)[None]
                t = np.clip(((p - P[None]) * ab).sum(-1) / (ab * ab).sum(-1), 0, 1)
                dist = np.sqrt(((p - (P[None] + t[..., None] * ab)) ** 2).sum(-1)).min(1)
                d[sel] = np.minimum(d[sel], dist)
    return d


@pytest.mark.parametrize("name", ["tissue", "large"])
def test_parity_at_the_workload_horizon(name):
    path = os.path.join(GOLD, f"horizon_{name}.npz")
    gold = np.load(path)
    w = W.WORKLOADS[name]()
    lat, nodes = gold["lat_idx"], gold["node_idx"]
    ks = [int(k) for k in gold["checkpoints"]]
    say(f"case {w.name}: checkpoints {ks}")
    g = lbib.from_workload(w)
    done = 0
    for k in ks:
        g.step(k - done)
        done = k
        last = k == ks[-1]
        F = g.get_fields(mask=last)
        G = {"rho": F["rho"].reshape(-1)[lat], "u": F["u"].reshape(2, -1)[:, lat],
             "phi": F["phi"].reshape(w.n_species, -1)[:, lat], "xy": F["xy"][nodes]}
        X0 = w.xy[nodes]
        R = {"rho": gold[f"drho_{k}"].astype(float) + w.rho0, "u": gold[f"u_{k}"].astype(float),
             "phi": gold[f"phi_{k}"].astype(float), "xy": gold[f"dX_{k}"].astype(float) + X0}
        errs = PB.field_errors(G, R, w.rho0, X0, k, w.n_species)
        red, inv = g.reduce(), gold[f"inv_{k}"]
        errs["sum rho"] = abs(red[0] - inv[0]) / abs(inv[0])
        errs["sum rho u"] = float(np.linalg.norm(red[1:3] - inv[1:3]) / max(np.linalg.norm(inv[1:3]), 1e-300))
        errs["sum phi"] = float(np.max(np.abs(red[3:] - inv[3:]) / np.abs(inv[3:])))
        say(f"  {k} steps:", PB.fmt(errs))
        PB.assert_fields(errs, what=f"{name} {k} steps")
        assert errs["sum rho"] <= 1e-9 and errs["sum phi"] <= 1e-5 and errs["sum rho u"] <= 1e-4
        if last:
            mo = gold[f"mask_{k}"].astype(np.int32)
            bad = np.argwhere(F["mask"] != mo)
            say(f"  domain IDs differing: {len(bad)} of {mo.size}")
            if len(bad):
                d = near_edge(w.offsets, F["xy"], bad[:, 1].astype(float), bad[:, 0].astype(float), w.nx, w.ny)
                say(f"  largest distance to an edge: {d.max():.2e}")
                assert d.max() < 1e-3
    g.close()
