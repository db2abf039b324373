"""Saving and resuming a run (Section "Input and Output": solver states saved in a loadable
format), the FP64 monitor inside lbib_step, and the device watchdog, through the C ABI.

Bars:
  * resume is exact: a run of 2n steps and a run of n steps, saved, loaded into a new context
    and stepped n more, agree bit for bit in rho, u, phi, the node positions and the domain-ID
    map (n = 37: the save falls inside a list period and a graph period), for the plain path,
    both no-flux forms, mass sources with the pressure ring, node sources and pressure points
    (brought by the state into a context without them), FP16 storage and the monitor;
  * the monitor's sums, taken inside the captured step graphs every monitor_every steps, equal
    lbib_reduce's for the same state bit for bit, and the oracle's invariants within the
    reduction test's bars, on the tiny and tissue workloads;
  * a state that becomes non-finite (a body acceleration of 1e30) is caught: with the monitor,
    the next lbib_step returns LBIB_ENUMERIC and enqueues nothing, as do the reads; nodes that
    outrun their list margin are caught the same way.  Every kernel still ends normally (the
    values are IEEE infinities and NaNs).
"""
import ctypes as C
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


def resume_cases():
    walls = W.PARITY_CASES["walls"]
    return {
        "tiny": lambda: W.tiny_cell(),
        "walls": lambda: walls(),
        "no-flux first-order": lambda: W.no_flux_tissue(static=False),
        "no-flux zeroth-order": lambda: _set(W.no_flux_tissue(static=False), no_flux_zeroth=True),
        "mass sources and ring": lambda: _set(W.mass_source_tissue(no_flux=True), pressure_ring=True),
        "half-force": lambda: _set(walls(), interp_half_force=True),
        "node maps": lambda: _maps(W.growth_case(3, 0)),
        "bounce-back no-flux": lambda: _set(W.no_flux_tissue(static=False), no_flux_bounce=True),
    }


def _maps(w):
    """Case III's cell with a point source and interior pressure points as well: the loaded
    context has no maps of its own, so the state must bring them."""
    w.node_sources = np.zeros((w.ny, w.nx))
    w.node_sources[w.ny // 2, w.nx // 2] = 1e-2
    w.node_sources[20, 70] = -2e-3
    w.pressure_nodes = np.zeros((w.ny, w.nx), np.uint8)
    w.pressure_nodes[80, 30] = w.pressure_nodes[15, 15] = 1
    return w


def _set(w, **kw):
    for k, v in kw.items():
        setattr(w, k, v)
    return w


def _sim(w, storage=None, monitor=0):
    d = w.params_dict()
    if storage is not None:
        d["storage"] = storage
    d["monitor_every"] = monitor
    s = lbib.Simulation(d)
    if w.n_cells:
        s.set_cells(w.offsets, w.xy, w.rest_len, w.rest_area)
        if w.source_cells is not None:
            s.set_source_cells(w.source_cells)
    if w.node_sources is not None:
        s.set_node_sources(w.node_sources)
    if w.pressure_nodes is not None:
        s.set_pressure_nodes(w.pressure_nodes)
    if w.rho_init is not None or w.u_init is not None or w.phi_init is not None:
        s.set_fields(w.rho_init, w.u_init, w.phi_init)
    return s


@pytest.mark.parametrize("storage,monitor", [(None, 0), (lbib.STORAGE_FP16, 0), (None, 16)],
                         ids=["fp32", "fp16", "fp32+monitor"])
@pytest.mark.parametrize("case", list(resume_cases()))
def test_resume_is_exact(case, storage, monitor):
    if (storage is not None or monitor) and case not in ("walls", "mass sources and ring"):
        pytest.skip("storage and monitor variants on two cases")
    w = resume_cases()[case]()
    n = 37
    say(f"case {case}: 2 x {n} steps against {n}, save, load, {n}")
    a = _sim(w, storage, monitor)
    a.step(2 * n)
    A = a.get_fields()
    b = _sim(w, storage, monitor)
    b.step(n)
    state = b.save_state()
    b.step(3)                                  # the saved state is a copy
    c = lbib.Simulation(dict(w.params_dict(), storage=storage or lbib.STORAGE_FP32, monitor_every=monitor))
    c.load_state(state)
    c.step(n)
    Cf = c.get_fields()
    for k in ("rho", "u", "phi", "xy", "mask"):
        assert np.array_equal(A[k], Cf[k]), (case, k)
    if monitor:
        ma, na = a.monitor()
        mc, nc = c.monitor()
        say(f"  monitor: {na} sums taken in the whole run, {nc} after resuming")
        assert na >= 1 and nc >= 1
    for s in (a, b, c):
        s.close()


def test_resume_of_a_state_not_yet_stepped():
    """A state saved before its first step keeps that mark: under the bounce-back no-flux form
    the first step takes each node's own populations as the ones it sent, after loading too."""
    w = _set(W.growth_case(1, 0), no_flux_bounce=True)
    a = _sim(w)
    b = _sim(w)
    state = b.save_state()
    c = lbib.Simulation(w.params_dict())
    c.step(5)                                  # a stepped context: the load must reset the mark
    c.load_state(state)
    a.step(20)
    c.step(20)
    A, Cf = a.get_fields(), c.get_fields()
    for k in ("rho", "u", "phi", "xy", "mask"):
        assert np.array_equal(A[k], Cf[k]), k
    for s in (a, b, c):
        s.close()


def test_resume_refuses_other_parameters():
    w = W.PARITY_CASES["walls"]()
    a = _sim(w)
    a.step(5)
    state = a.save_state()
    other = lbib.Simulation(dict(w.params_dict(), tau=w.tau + 0.1))
    with pytest.raises(lbib.LbibError) as e:
        other.load_state(state)
    assert e.value.status == lbib.EINVAL
    with pytest.raises(lbib.LbibError) as e:
        a.load_state(state[:100])
    assert e.value.status == lbib.EINVAL
    # a node count beyond lbib_set_cells' limit is refused before anything is sized from it
    bad = bytearray(state)
    off = 16 + C.sizeof(lbib.Params) + 8
    bad[off:off + 8] = (10 ** 12).to_bytes(8, "little", signed=True)
    with pytest.raises(lbib.LbibError) as e:
        a.load_state(bytes(bad))
    assert e.value.status == lbib.EINVAL
    for s in (a, other):
        s.close()


@pytest.mark.parametrize("case,steps", [("tiny", 192), ("tissue", 64)])
def test_monitor_sums_equal_reduce_and_the_oracle(case, steps):
    w = W.tiny_cell() if case == "tiny" else W.tissue()
    g = _sim(w, monitor=16)
    assert g.monitor() == (None, 0)
    g.step(steps - 16)
    g.step(16)
    sums, taken = g.monitor()
    red = g.reduce()
    say(f"case {case}: {taken} monitor sums; latest {sums}; lbib_reduce {red}")
    assert taken == steps // 16
    assert np.array_equal(sums, red)
    o = O.from_workload(w)
    o.step(steps)
    inv = o.invariants()
    nn = w.nx * w.ny
    assert abs(sums[0] - inv[0]) <= 1e-9 * abs(inv[0])
    assert np.all(np.abs(sums[1:3] - inv[1:3]) <= 1e-4 * np.abs(inv[1:3]) + 1e-11 * nn)
    assert np.all(np.abs(sums[3:] - inv[3:]) <= 1e-5 * np.abs(inv[3:]))
    g.close()


def test_monitor_every_other_period():
    w = W.tiny_cell()
    g = _sim(w, monitor=32)
    g.step(40)                         # two periods (one graph each), then 8 direct steps
    assert g.monitor()[1] == 1
    g.step(24)                         # the fourth period ends
    assert g.monitor()[1] == 2
    g.close()


def test_watchdog_stops_a_blown_up_lattice():
    w = W.Workload(name="lattice blown up by a huge body force", nx=96, ny=64, bc_y=W.WALLS, tau=0.8,
                   body_accel=(1e30, 0.0))
    g = _sim(w, monitor=16)
    g.step(32)
    g.sync()
    with pytest.raises(lbib.LbibError) as e:
        g.step(16)
    assert e.value.status == lbib.ENUMERIC
    with pytest.raises(lbib.LbibError) as e:
        g.get_fields()
    assert e.value.status == lbib.ENUMERIC
    with pytest.raises(lbib.LbibError) as e:
        g.monitor()
    assert e.value.status == lbib.ENUMERIC
    g.close()


def test_watchdog_catches_nodes_outrunning_their_lists():
    w = W.tiny_cell()
    w.body_accel = (0.05, 0.0)         # the fluid and the cell accelerate by 0.05 per step
    g = _sim(w)
    g.step(16)
    g.sync()
    with pytest.raises(lbib.LbibError) as e:
        g.step(16)
        g.step(16)
        g.sync()
        g.step(16)
    assert e.value.status == lbib.ENUMERIC
    say(f"  {e.value}")
    g.close()
