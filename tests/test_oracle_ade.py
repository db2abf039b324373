"""Pins of the oracle's ADE-only iteration (the steady-state measurement) and of the sparse
steady-state reference, against closed forms and conservation.

The iteration follows the D2Q5 equations of the supplementary "Lattice Boltzmann Method"
section with u = 0 and the source/decay law; the stopping rule is the relative change
||phi^k - phi^{k-1}||_2 / ||phi^k||_2.
"""
import numpy as np
import pytest

from oracle import ade_fixed_point as F
from oracle import oracle as O
from paper_1503_06726_amd import workloads as W


def _ade_params(nx, ny, walls, D, source, decay):
    return {"nx": nx, "ny": ny, "bc_y": W.WALLS if walls else W.PERIODIC, "tau": 1.0, "rho0": 1.0,
            "species": [{"D": D, "phi_ref": 0.0, "reaction": W.REACT_SOURCE_DECAY,
                         "c": (source, decay, 0.0, 0.0)}]}


@pytest.mark.parametrize("decay", [1e-3, 0.05])
def test_decay_only_uniform_field_changes_by_closed_form(decay):
    # no cells, uniform phi at equilibrium: collision keeps g = w phi (1 - lambda), streaming
    # keeps it uniform, so phi^k = (1 - lambda) phi^{k-1} and the relative change is
    # lambda / (1 - lambda) at every iteration
    s = O.Sim(_ade_params(20, 14, True, 0.1, 1e-3, decay))
    s.set_fields(phi=np.full((1, 14, 20), 2.5))
    ch = s.ade_step(7)[:, 0]
    np.testing.assert_allclose(ch, decay / (1.0 - decay), rtol=1e-12)
    phi = s.get_fields()["phi"][0]
    np.testing.assert_allclose(phi, 2.5 * (1.0 - decay) ** 7, rtol=1e-13)


def test_stopping_rule_counts_iterations():
    # the change is lambda / (1 - lambda) from the first iteration on: met at k = 1 when that
    # is within the tolerance, never otherwise
    lam = 1e-3
    s = O.Sim(_ade_params(16, 10, False, 0.1, 1e-3, lam))
    s.set_fields(phi=np.full((1, 10, 16), 1.0))
    k, _ = s.ade_steady(tol=1.01 * lam / (1 - lam), max_iters=50)
    assert k == 1
    s.set_fields(phi=np.full((1, 10, 16), 1.0))
    k, hist = s.ade_steady(tol=0.99 * lam / (1 - lam), max_iters=50)
    assert k == 0 and hist.shape == (50, 1)


def test_sparse_fixed_point_uniform_source():
    # a source at every node: the fixed point is the uniform balance phi = sigma / lambda
    phi = F.steady_state(15, 11, True, 0.3, 2e-3, 4e-4, np.ones((11, 15)))
    np.testing.assert_allclose(phi, 2e-3 / 4e-4, rtol=1e-11)


@pytest.mark.parametrize("walls", [True, False])
def test_sparse_fixed_point_mass_balance(walls):
    # streaming and collision conserve sum phi; at the fixed point the source must balance the
    # decay: sum (sigma m - lambda phi) = 0
    rng = np.random.default_rng(3)
    m = (rng.random((13, 17)) < 0.2).astype(float)
    phi = F.steady_state(17, 13, walls, 0.05, 1e-3, 3e-4, m)
    np.testing.assert_allclose(phi.sum(), 1e-3 * m.sum() / 3e-4, rtol=1e-10)
    assert phi.min() > 0.0


def _small_static(nx=40, ny=30, n_cells=6, seed=0):
    rng = np.random.default_rng(seed)
    off, xy = W.voronoi_tissue(nx, ny, n_cells, W._rng(400 + seed, 0))
    src = np.zeros(n_cells, np.uint8)
    src[rng.choice(n_cells, 2, replace=False)] = 1
    return off, xy, src


def test_source_map_is_the_raster_of_the_source_cells():
    # the source/decay law's map with a subset: nonzero exactly where the full domain-ID map
    # names a source cell (the Voronoi cells do not overlap)
    off, xy, src = _small_static()
    s = O.Sim(_ade_params(40, 30, True, 0.1, 1e-3, 1e-3))
    s.set_cells(off, xy)
    ids = s.get_fields()["mask"]
    assert (s.source_map() != 0).sum() == (ids != 0).sum()        # default: every cell
    s.set_source_cells(src)
    want = np.isin(ids, np.flatnonzero(src) + 1)
    np.testing.assert_array_equal(s.source_map() != 0, want)


@pytest.mark.parametrize("walls", [True, False])
def test_ade_iteration_reaches_the_sparse_fixed_point(walls):
    # iterate from zero until converged; the result is the fixed point of the same linear map
    # built independently as a sparse matrix
    off, xy, src = _small_static(seed=1 if walls else 2)
    prm = _ade_params(40, 30, walls, 0.2, 1e-3, 5e-3)
    s = O.Sim(prm)
    s.set_cells(off, xy)
    s.set_source_cells(src)
    k, hist = s.ade_steady(tol=1e-12, max_iters=20000)
    assert k > 0
    phi = s.get_fields()["phi"][0]
    want = F.steady_state(40, 30, walls, 0.2, 1e-3, 5e-3, s.source_map() != 0)
    np.testing.assert_allclose(phi, want, rtol=1e-8, atol=1e-12 * want.max())
    # the change decreases towards the end (no oscillation at convergence)
    assert hist[-1, 0] < hist[len(hist) // 2, 0]


def test_static_tissue_sample_is_seeded_and_valid():
    a, b = W.static_tissue(3), W.static_tissue(3)
    np.testing.assert_array_equal(a.xy, b.xy)
    np.testing.assert_array_equal(a.source_cells, b.source_cells)
    assert 50 <= a.n_cells <= 300 and a.source_cells.any()
    assert 0.02 <= a.species[0].D <= 0.5 and 1e-5 <= a.species[0].c[1] <= 1e-3
    t = W.static_tissue(3, held_out=False)
    assert t.n_cells != a.n_cells or not np.array_equal(t.xy, a.xy)
    from paper_1503_06726_amd import lbib
    lbib.validate_cells(a.params_dict(), a.offsets, a.xy)
