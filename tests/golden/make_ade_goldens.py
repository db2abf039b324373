"""Steady states of held-out static-tissue samples by the sparse direct solve.

Writes tests/golden/ade_fixed_points.npz: for the first SAMPLES held-out samples of the
steady-state measurement (256 x 256, walls in y, a Voronoi tissue whose source cells hold a
source of 1e-3 per step, decay lambda, diffusivity D), the fixed point phi* [ny, nx] of the
ADE-only iteration, solved directly from the D2Q5 equations (oracle/ade_fixed_point.py), with
the source map rasterised by the oracle.  The benchmark compares the iterated solutions with
them (the true error of the stopping rule).  Calls only the oracle and the seeded workload
generator.  Usage: python tests/golden/make_ade_goldens.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ade_fixed_point as FP                 # noqa: E402
from oracle import oracle as O                           # noqa: E402
from paper_1503_06726_amd import workloads as W          # noqa: E402

SAMPLES = 8
SOURCE = 1e-3


def main():
    out = {}
    for i in range(SAMPLES):
        w = W.static_tissue(i, held_out=True)
        ids, _ = O.raster(w.params_dict(), w.offsets, w.xy)
        src_ids = np.flatnonzero(np.asarray(w.source_cells) != 0) + 1
        m = np.isin(ids, src_ids)
        D, lam = w.species[0].D, w.species[0].c[1]
        out[f"phi_{i}"] = FP.steady_state(w.nx, w.ny, w.bc_y == W.WALLS, D, SOURCE, lam, m).astype(np.float32)
        out[f"decay_{i}"] = np.float64(lam)
        print(f"sample {i}: D {D:.4f}, decay {lam:.3g}, max phi {out[f'phi_{i}'].max():.4g}", flush=True)
    np.savez_compressed(os.path.join(HERE, "ade_fixed_points.npz"), samples=np.int64(SAMPLES), **out)


if __name__ == "__main__":
    main()
