"""ADE-only iterations on the GPU (the steady-state measurement) against the FP64 oracle, the
source-cell subset in the coupled step, and the steady state against the sparse reference.

Bars: in FP64 the iteration count equals the oracle's (both decide the stopping rule in FP64)
and the concentration after a fixed number of iterations, read back through the context's
FP32 storage, agrees to 1e-7 (rel-L2); in FP32
the concentration agrees to 1e-5 and the count to 3 % (the change norm near the tolerance is
a difference of nearly equal FP32 values); at 256^2 the converged field is within twice the
asymptotic error tol / lambda of the sparse fixed point (the slowest mode decays at rate
lambda, so the remaining error is about the last change divided by lambda).
"""
import sys

import numpy as np
import pytest

from oracle import ade_fixed_point as F
import parity_bars as PB
from oracle import oracle as O
from paper_1503_06726_amd import lbib
from paper_1503_06726_amd import workloads as W

pytestmark = pytest.mark.gpu

H = 128          # ADE passes per captured batch in lbib_ade_steady


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b)


def small_static(nx, ny, n_cells, seed, D, decay, walls=True):
    off, xy = (W.voronoi_tissue(nx, ny, n_cells, W._rng(500 + seed, 0)) if walls else
               W.voronoi_tissue(nx, ny, n_cells, W._rng(500 + seed, 0), y_lo=2.0, y_hi=ny - 3.0))
    rng = np.random.default_rng(seed)
    src = (rng.random(n_cells) < 0.3).astype(np.uint8)
    src[0] = 1
    w = W.Workload(name=f"static {nx}x{ny} {n_cells} cells D={D} decay={decay}", nx=nx, ny=ny,
                   bc_y=W.WALLS if walls else W.PERIODIC, tau=1.0, rho0=1.0,
                   species=[W.Species(D=D, phi_ref=0.0, reaction=W.REACT_SOURCE_DECAY,
                                      c=(1e-3, decay, 0.0, 0.0))], steps=0)
    w = W._attach_geometry(w, off, xy)
    w.source_cells = src
    return w


CASES = {
    "walls": lambda: small_static(70, 45, 8, 0, 0.2, 2e-3),
    "periodic": lambda: small_static(64, 40, 6, 1, 0.05, 4e-3, walls=False),
    "slow": lambda: small_static(50, 37, 5, 2, 0.4, 3e-4),
}


@pytest.mark.parametrize("case", list(CASES))
def test_ade_fp64_iterations_equal_oracle(case):
    w = CASES[case]()
    say(f"case {w.name}: ADE to 1e-6 (GPU, FP64)")
    g = lbib.from_workload(w)
    k_gpu, ch = g.ade_steady(1e-6, 100000, fp64=True)
    g.close()
    say("  oracle")
    o = O.from_workload(w)
    k_orc, hist = o.ade_steady(1e-6, 100000, chunk=1024)
    say(f"  iterations GPU {k_gpu}, oracle {k_orc}; change at stop {ch:.3e}")
    assert k_orc > 0 and k_gpu == k_orc
    assert ch <= 1e-6


@pytest.mark.parametrize("case,fp64,tol", [("walls", True, 1e-7), ("periodic", True, 1e-7),
                                           ("walls", False, 1e-5), ("periodic", False, 1e-5)])
def test_ade_state_after_fixed_iterations(case, fp64, tol):
    # tol = 0 never stops early: one first pass plus whole batches of H passes.  The FP64
    # iteration hands its result back to the context's FP32 storage, so its bar is the FP32
    # rounding of each population (about 6e-8 relative), not FP64 round-off
    w = CASES[case]()
    n_iter = 200
    passes = 1 + H * ((n_iter + H - 1) // H)
    say(f"case {w.name}: {passes} ADE passes (GPU, {'FP64' if fp64 else 'FP32'})")
    g = lbib.from_workload(w)
    k, _ = g.ade_steady(0.0, n_iter, fp64=fp64)
    G = g.get_fields(rho=False, u=False, xy=False, mask=False)
    g.close()
    o = O.from_workload(w)
    o.ade_step(passes)
    R = o.get_fields()
    r = rel(G["phi"], R["phi"])
    say(f"  phi rel-L2 {r:.2e}")
    assert k == 0 and r <= tol


def test_ade_fp32_iterations_close_to_oracle():
    w = CASES["walls"]()
    g = lbib.from_workload(w)
    k32, _ = g.ade_steady(1e-6, 100000, fp64=False)
    g.close()
    o = O.from_workload(w)
    k_orc, _ = o.ade_steady(1e-6, 100000, chunk=1024)
    say(f"  iterations GPU FP32 {k32}, oracle {k_orc}")
    assert k32 > 0 and abs(k32 - k_orc) <= 0.03 * k_orc


def test_ade_warm_start_from_the_fixed_point_converges_sooner():
    # seeded with the steady concentration (equilibrium populations w_i phi*), only the
    # populations' non-equilibrium part is left to relax: far fewer iterations than from zero
    w = CASES["walls"]()
    o = O.from_workload(w)
    phi_star = F.steady_state(w.nx, w.ny, True, w.species[0].D, 1e-3, w.species[0].c[1], o.source_map() != 0)
    g = lbib.from_workload(w)
    k0, _ = g.ade_steady(1e-6, 100000, fp64=True)
    g.set_fields(phi=phi_star[None])
    kw, ch = g.ade_steady(1e-6, 100000, fp64=True)
    g.close()
    say(f"  from zero {k0} iterations, from phi* {kw} (change {ch:.2e})")
    assert 0 < kw < k0 / 5


def test_ade_full_size_sample_near_sparse_fixed_point():
    w = W.static_tissue(1)
    lam = w.species[0].c[1]
    say(f"case {w.name}: ADE to 1e-6 (GPU, FP64)")
    g = lbib.from_workload(w)
    k, ch = g.ade_steady(1e-6, 1_000_000, fp64=True)
    G = g.get_fields(rho=False, u=False, xy=False, mask=False)
    g.close()
    o = O.from_workload(w)
    phi_star = F.steady_state(w.nx, w.ny, True, w.species[0].D, 1e-3, lam, o.source_map() != 0)
    err = rel(G["phi"][0], phi_star)
    say(f"  {k} iterations; error against the sparse fixed point {err:.3e} (bound {1e-6 / lam:.3e})")
    assert k > 0 and err <= 2e-6 / lam


def test_source_subset_in_the_coupled_step():
    w = W.PARITY_CASES["walls"]()
    w.source_cells = (np.arange(w.n_cells) % 3 == 0).astype(np.uint8)
    g = lbib.from_workload(w)
    g.step(60)
    G = g.get_fields()
    g.close()
    o = O.from_workload(w)
    o.step(60)
    R = o.get_fields()
    r = PB.field_errors(G, R, w.rho0, w.xy, 60, w.n_species)
    say("  errors:", PB.fmt(r))
    PB.assert_fields(r)


def test_ade_and_source_errors():
    w = W.PARITY_CASES["walls"]()
    g = lbib.Simulation(w.params_dict())
    with pytest.raises(lbib.LbibError) as e:
        g.set_source_cells(np.ones(3, np.uint8))
    assert e.value.status == lbib.ESTATE
    with pytest.raises(lbib.LbibError) as e:
        g.ade_steady(-1.0, 10)
    assert e.value.status == lbib.EINVAL
    g.close()


# ------------------------------------------------------------------------------------------
# batched ADE-only solver: many problems of one lattice size per launch
# ------------------------------------------------------------------------------------------
def _source_mask(w):
    """Source indicator of a workload from the oracle's map (test side)."""
    o = O.from_workload(w)
    return (o.source_map() != 0).astype(np.uint8), o


def test_ade_batch_iterations_equal_oracle():
    ws = [small_static(60, 44, 6, s, D, lam) for s, D, lam in [(10, 0.2, 2e-3), (11, 0.08, 5e-3), (12, 0.3, 8e-4)]]
    masks, counts = [], []
    for w in ws:
        m, o = _source_mask(w)
        masks.append(m)
        k, _ = o.ade_steady(1e-6, 100000, chunk=1024)
        counts.append(k)
    its, phi = lbib.ade_batch(60, 44, W.WALLS, np.stack(masks), [w.species[0].D for w in ws], [1e-3] * 3,
                              [w.species[0].c[1] for w in ws], tol=1e-6, max_iters=100000, fp64=True)
    say(f"  batched {its.tolist()}, oracle {counts}")
    assert its.tolist() == counts


def test_ade_batch_equals_single_context_solver():
    ws = [W.static_tissue(i) for i in range(3)]
    masks = [_source_mask(w)[0] for w in ws]
    its, phi = lbib.ade_batch(256, 256, W.WALLS, np.stack(masks), [w.species[0].D for w in ws], [1e-3] * 3,
                              [w.species[0].c[1] for w in ws], tol=1e-6, max_iters=1_000_000, fp64=True)
    single = []
    for w in ws:
        g = lbib.from_workload(w)
        k, _ = g.ade_steady(1e-6, 1_000_000, fp64=True)
        g.close()
        single.append(k)
    say(f"  batched {its.tolist()}, one context each {single}")
    assert its.tolist() == single and min(single) > 0


def test_ade_batch_fixed_iterations_state():
    # tol = 0: one first pass plus whole batches of 64 passes
    w = small_static(48, 40, 5, 20, 0.15, 3e-3)
    m, o = _source_mask(w)
    phi0 = np.random.default_rng(0).random((48 * 40,)).reshape(1, 40, 48) * 0.5
    its, phi = lbib.ade_batch(48, 40, W.WALLS, m[None], [0.15], [1e-3], [3e-3], phi0=phi0, tol=0.0,
                              max_iters=100, fp64=True)
    o.set_fields(phi=phi0)
    o.ade_step(1 + 64 * 2)
    R = o.get_fields()["phi"][0]
    r = rel(phi[0], R)
    say(f"  phi rel-L2 {r:.2e}")
    assert its[0] == 0 and r <= 1e-12
