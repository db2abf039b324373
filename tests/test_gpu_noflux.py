"""No-flux cell membranes for a species (Section "Signalling"; Suppl. "No-flux Boundary
Condition for Reaction-Advection-Diffusion Equations": the first-order condition, and its
zeroth-order form as an option) through the C ABI.

Bars:
  * a moving tissue (springs, body acceleration) whose species sees the membranes as
    no-flux boundaries follows the FP64 oracle within the parity bar (1e-5 relative L2 for
    rho, u, phi and the node positions) over 60 steps, in FP32 storage, in both forms, and the
    first-order form still does after 160 steps (cuts deposited and cleared as cells move,
    ten list rebuilds and graph periods);
  * with static cells and a source inside them, the extracellular concentration stays
    exactly zero on the GPU too, while the cells fill;
  * the combinations the condition does not support are refused: a source subset, the
    ADE-only iteration, a batch.
"""
import sys

import numpy as np
import pytest

import parity_bars as PB
from oracle import oracle as O
from paper_1503_06726_amd import lbib
from paper_1503_06726_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


FORMS = pytest.mark.parametrize("form", ["first", "zeroth", "bounce"],
                                ids=["first-order", "zeroth-order", "bounce-back"])


def _form(w, form):
    w.no_flux_zeroth = form == "zeroth"
    w.no_flux_bounce = form == "bounce"
    return w


@FORMS
@pytest.mark.parametrize("static,steps", [(False, 60), (True, 60), (False, 160)])
def test_no_flux_matches_oracle(static, steps, form):
    if form == "zeroth" and steps > 60:
        pytest.skip("the long run covers the first-order and bounce-back forms")
    w = _form(W.no_flux_tissue(static=static), form)
    say(f"case {w.name}, {form} form: {steps} steps")
    g = lbib.from_workload(w)
    g.step(steps)
    G = g.get_fields()
    g.close()
    o = O.from_workload(w)
    o.step(steps)
    R = o.get_fields()
    errs = PB.field_errors(G, R, w.rho0, w.xy, steps, w.n_species)
    say("  errors:", PB.fmt(errs))
    PB.assert_fields(errs)
    assert np.array_equal(G["mask"], R["mask"])


@FORMS
def test_no_flux_confines_the_source_on_the_gpu(form):
    w = _form(W.no_flux_tissue(static=True), form)
    g = lbib.from_workload(w)
    g.step(100)
    F = g.get_fields()
    inside = F["mask"] != 0
    phi = F["phi"][0]
    assert np.all(phi[~inside] == 0.0)
    assert np.min(phi[inside]) > 0.0
    g.close()


def test_no_flux_refusals():
    w = W.no_flux_tissue(static=True)
    g = lbib.from_workload(w)
    with pytest.raises(lbib.LbibError) as e:
        g.set_source_cells(np.ones(w.n_cells, np.uint8))
    assert e.value.status == lbib.EINVAL
    with pytest.raises(lbib.LbibError) as e:
        g.ade_steady(1e-6, 10)
    assert e.value.status == lbib.EINVAL
    with pytest.raises(lbib.LbibError):
        lbib.Batch([g])
    g.set_source_cells(None)             # all cells: accepted
    g.step(3)
    g.close()


@pytest.mark.parametrize("form", ["first", "bounce"], ids=["first-order", "bounce-back"])
def test_no_flux_at_full_size(form):
    """The bench workload (2048 x 2048, 2000 cells, 726,782 nodes) with its species behind
    no-flux membranes: 36 steps cross two list rebuilds and replay one captured period (the
    bounce-back form's first step runs outside the graphs), and every field stays within the
    parity bar of the FP64 oracle."""
    w = _form(W.large(), form)
    w.species[0].no_flux = True
    steps = 36
    say(f"case {w.name}, {form} no-flux form: {steps} steps")
    g = lbib.from_workload(w)
    g.step(steps)
    G = g.get_fields(mask=False)
    g.close()
    o = O.from_workload(w)
    o.step(steps)
    R = o.get_fields()
    errs = PB.field_errors(G, R, w.rho0, w.xy, steps, w.n_species)
    say("  errors:", PB.fmt(errs))
    PB.assert_fields(errs)
