"""Growth validations on the library (Section "Validation", Cases I-III, their table of lattice
discretisations and their figures of the relative area and concentration errors against the
lattice resolution).

A circular cell with a no-flux species inside (initially 1) grows by a mass source for one unit
of non-dimensional time while the outer ring of the lattice holds the density (iso-pressure
outflow): a point source at the centre (Case I, A = A0 + T), a uniform source inside the cell
(Case II, the area doubles) or a uniform source proportional to the species' concentration
(Case III, A = A0 (1 + T) while the species is conserved).  Reported per case and resolution:
  * the relative area error at T = 1 against the analytical law, from the library's own cell
    area;
  * the relative error of the integrated concentration (the sum of phi over the lattice, which
    the no-flux membrane should conserve), as the mean of its magnitude over the samples (it
    jumps whenever the growing cell takes in a lattice node);
  * the observed orders log2(e_l / e_{l+1}) between consecutive resolutions.

The supplement's no-flux condition (equilibrium replacement with the wall at rest) loses the
species a moving membrane sweeps over; ``--bounce`` runs the membrane in the bounce-back form,
which conserves it.

Usage:  python -m paper_1503_06726_amd.growth [--cases 1 2 3] [--levels 0 1 2 3] [--samples 100]
                                              [--bounce] [--out results.json]
Prints one JSON line per case and level, then the observed orders per case.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import lbib
from . import workloads as W


def run_case(case: int, level: int, samples: int = 100, steps: int | None = None,
             maxlength: float = 0.5, stream: int | None = None, bounce: bool = False) -> dict:
    """Step one case for its full time (or ``steps``), sampling the cell's area and the
    integrated concentration ``samples`` times.  ``bounce``: the bounce-back no-flux form."""
    w = W.growth_case(case, level, maxlength, steps, bounce)
    if w.steps % samples:
        raise ValueError("the step count must be a multiple of the samples")
    sim = lbib.from_workload(w, stream=stream)
    try:
        A0 = float(sim.get_forces()[1][0])
        M0 = float(sim.get_fields()["phi"][0].sum())
        traj = [(0, 0.0, 0.0)]
        A = A0
        chunk = w.steps // samples
        t0 = time.perf_counter()
        for k in range(samples):
            sim.step(chunk)
            t = (k + 1) * chunk
            A = float(sim.get_forces()[1][0])
            M = float(sim.get_fields()["phi"][0].sum())
            law = W.growth_law(case, level, A0, t)
            traj.append((t, (A - law) / law, (M - M0) / M0))
        seconds = time.perf_counter() - t0
    finally:
        sim.close()
    return {"case": case, "level": level, "bounce": bounce, "lattice": w.nx, "diameter": 10 * 2 ** level, "nodes": w.n_nodes,
            "steps": w.steps, "area0": A0, "area_ratio": A / A0, "rel_area_error": traj[-1][1],
            "mean_abs_mass_error": float(np.mean([abs(m) for _, _, m in traj[1:]])),
            "trajectory": traj, "seconds": round(seconds, 3)}


def orders(results: list[dict], key: str) -> dict:
    """Observed convergence orders of ``key`` between consecutive levels, per case."""
    out = {}
    for c in sorted({r["case"] for r in results}):
        rs = sorted((r for r in results if r["case"] == c), key=lambda r: r["level"])
        out[c] = [(a["level"], b["level"], math.log2(abs(a[key]) / abs(b[key])))
                  for a, b in zip(rs, rs[1:]) if b["level"] == a["level"] + 1 and a[key] != 0 and b[key] != 0]
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--cases", type=int, nargs="+", default=list(W.GROWTH_CASES))
    ap.add_argument("--levels", type=int, nargs="+", default=list(range(W.LEAKAGE_LEVELS)))
    ap.add_argument("--samples", type=int, default=100)
    ap.add_argument("--bounce", action="store_true", help="the bounce-back no-flux form")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    results = []
    for case in args.cases:
        for level in args.levels:
            r = run_case(case, level, args.samples, bounce=args.bounce)
            results.append(r)
            print(json.dumps({k: v for k, v in r.items() if k != "trajectory"}), flush=True)
    oa, om = orders(results, "rel_area_error"), orders(results, "mean_abs_mass_error")
    for c in oa:
        print(json.dumps({"case": c, "area_orders": [(a, b, round(o, 4)) for a, b, o in oa[c]],
                          "mass_orders": [(a, b, round(o, 4)) for a, b, o in om[c]]}), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"cases": results, "area_orders": {str(c): v for c, v in oa.items()},
                       "mass_orders": {str(c): v for c, v in om.items()}}, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
