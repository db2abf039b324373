"""Membrane-leakage study on the library (Section "Validation", Case IV, and its figure of the
relative area error against lattice resolution and node spacing).

A circular cell under a constant membrane tension and no other force loses area only through
the immersed boundary's leakage: the cosine kernel spreads and interpolates over a band, so
fluid crosses the membrane and the tension squeezes the cell.  The paper measures the relative
area error after one unit of non-dimensional time at four resolutions (cell diameter 10, 20,
40, 80 lattice units) and three largest node spacings (0.1, 0.5, 2.5 lattice units), finds
spacings 0.1 and 0.5 indistinguishable, and fits a convergence order of about 1 between the
two finest lattices.

With the literal velocity u = sum f v / rho the membrane nodes also drift by half their
interpolated force density per step, outward for a contracting tension, and the cell grows;
with the half-force-shifted velocity u + f/2 (``--half-force``) the drift is gone and the cell
shrinks by leakage alone, as the paper's does.

Usage:  python -m paper_1503_06726_amd.leakage [--levels 0 1 2 3] [--maxlengths 0.1 0.5 2.5]
                                               [--samples 10] [--half-force] [--out results.json]
Prints one JSON line per case, then the observed orders log2(e_l / e_{l+1}).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

from . import lbib
from . import workloads as W


def run_case(level: int, maxlength: float, samples: int = 10, steps: int | None = None,
             stream: int | None = None, half_force: bool = False) -> dict:
    """Step one case for its full time (or ``steps``), sampling the cell's area ``samples``
    times; the error is relative to the initial polygon's area.  ``half_force``: the nodes
    move with the half-force-shifted velocity."""
    w = W.leakage_case(level, maxlength, steps)
    w.interp_half_force = half_force
    if w.steps % samples:
        raise ValueError("the step count must be a multiple of the samples")
    sim = lbib.from_workload(w, stream=stream)
    try:
        A0 = float(sim.get_forces()[1][0])
        traj = [(0, 0.0)]
        chunk = w.steps // samples
        t0 = time.perf_counter()
        for k in range(samples):
            sim.step(chunk)
            A = float(sim.get_forces()[1][0])
            traj.append(((k + 1) * chunk, (A - A0) / A0))
        seconds = time.perf_counter() - t0
    finally:
        sim.close()
    return {"level": level, "maxlength": maxlength, "half_force": half_force, "lattice": w.nx,
            "diameter": 10 * 2 ** level,
            "nodes": w.n_nodes, "steps": w.steps, "phi_m": w.phi_m, "area0": A0,
            "rel_area_error": traj[-1][1], "trajectory": traj, "seconds": round(seconds, 3)}


def orders(results: list[dict]) -> dict:
    """Observed convergence orders between consecutive levels, per node spacing."""
    out = {}
    for m in sorted({r["maxlength"] for r in results}):
        rs = sorted((r for r in results if r["maxlength"] == m), key=lambda r: r["level"])
        out[m] = [(a["level"], b["level"], math.log2(abs(a["rel_area_error"]) / abs(b["rel_area_error"])))
                  for a, b in zip(rs, rs[1:]) if b["level"] == a["level"] + 1
                  and a["rel_area_error"] != 0 and b["rel_area_error"] != 0]
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--levels", type=int, nargs="+", default=list(range(W.LEAKAGE_LEVELS)))
    ap.add_argument("--maxlengths", type=float, nargs="+", default=list(W.LEAKAGE_MAXLENGTHS))
    ap.add_argument("--samples", type=int, default=10)
    ap.add_argument("--half-force", action="store_true", help="nodes move with u + f/2")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    results = []
    for level in args.levels:
        for m in args.maxlengths:
            r = run_case(level, m, args.samples, half_force=args.half_force)
            results.append(r)
            print(json.dumps({k: v for k, v in r.items() if k != "trajectory"}), flush=True)
    od = orders(results)
    for m, v in od.items():
        print(json.dumps({"maxlength": m, "orders": [(a, b, round(o, 4)) for a, b, o in v]}), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"cases": results, "orders": {str(m): v for m, v in od.items()}}, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
