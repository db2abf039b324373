"""Batched stepping (lbib_batch_*) through the C ABI.

Bars:
  * at the default tile height a batched simulation is bit-identical to the same simulation
    stepped alone (same kernels' arithmetic; list order is immaterial), across graph periods,
    odd step counts and the release of the batch;
  * another tile height changes only the grouping of the interpolation sums: every field
    within 1e-6 relative L2 of the simulation stepped alone;
  * the autotuner leaves every simulation's state bit-for-bit as it found it;
  * a batched simulation at a non-default tile height matches the FP64 oracle within the
    parity bar (1e-5 relative L2).
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


def close_fields(a, b, w, steps):
    """Round-off differences between two GPU runs of the same simulation: relative L2 of u,
    phi and X - X0, and the density deviation's difference over its FP32 rounding bar (scaled
    to 1e-6)."""
    out = {"u": rel(b["u"], a["u"]), "X-X0": rel(b["xy"] - w.xy, a["xy"] - w.xy)}
    if w.n_species:
        out["phi"] = rel(b["phi"], a["phi"])
    bar = PB.drho_bound(a["rho"] - w.rho0, a["u"], steps)
    out["drho/bar"] = 1e-6 * float(np.linalg.norm((b["rho"] - w.rho0) - (a["rho"] - w.rho0))) / bar
    return out


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def small_sweep(n=6, periodic_ny=98):
    """Uneven little lattices of the sweep recipe plus one periodic-y tissue (ny = 98 rules out
    tiles of 4 rows, ny = 96 admits them)."""
    ws = [W.sweep_member(i, side_lo=64.0, side_hi=190.0) for i in range(n - 1)]
    ws.append(W.small_tissue(nx=150, ny=periodic_ny, n_cells=10, bc_y=W.PERIODIC, n_species=1, seed=3))
    return ws


def make(ws):
    return [lbib.from_workload(w) for w in ws]


def fields(sims):
    return [s.get_fields() for s in sims]


def assert_bit_equal(FA, FB, what):
    for i, (a, b) in enumerate(zip(FA, FB)):
        for k in ("rho", "u", "phi", "xy", "mask"):
            assert np.array_equal(a[k], b[k]), f"{what}: simulation {i}, field {k} differs"


def close_all(*groups):
    for g in groups:
        for s in g:
            s.close()


def test_batched_bit_identical_to_alone():
    ws = small_sweep()
    say("sizes:", [(w.nx, w.ny, w.n_cells) for w in ws])
    A, B = make(ws), make(ws)
    batch = lbib.Batch(B)
    assert batch.tile == 8
    for n in (40, 13, 16):          # two graph periods + 8 direct steps, an odd count, one more period
        for s in A:
            s.step(n)
        batch.step(n)
        batch.sync()
        assert_bit_equal(fields(A), fields(B), f"after {n} more steps")
        say(f"  +{n} steps: bit-identical")
    batch.close()
    for s in A + B:
        s.step(7)
    assert_bit_equal(fields(A), fields(B), "after the release")
    close_all(A, B)


def test_two_groups_bit_identical_to_alone():
    """Two groups on two streams (one graph per period): still the same arithmetic per simulation."""
    ws = small_sweep()
    A, B = make(ws), make(ws)
    batch = lbib.Batch(B)
    batch.set_groups(2)
    assert batch.groups == 2
    for n in (37, 16):                 # two graph periods + 5 direct steps, then one more period
        for s in A:
            s.step(n)
        batch.step(n)
        batch.sync()
        assert_bit_equal(fields(A), fields(B), f"two groups, after {n} more steps")
    batch.step(11)                     # back to a period boundary (64 steps) before regrouping
    for s in A:
        s.step(11)
    batch.set_groups(1)
    batch.step(16)
    for s in A:
        s.step(16)
    batch.sync()
    assert_bit_equal(fields(A), fields(B), "after regrouping")
    batch.close()
    close_all(A, B)


@pytest.mark.parametrize("rows", [4, 16])
def test_other_tile_heights_round_off_only(rows):
    ws = small_sweep(periodic_ny=96)
    A, B = make(ws), make(ws)
    batch = lbib.Batch(B)
    batch.set_tile(rows)
    assert batch.tile == rows
    for s in A:
        s.step(48)
    batch.step(48)
    batch.sync()
    worst = 0.0
    for i, (a, b) in enumerate(zip(fields(A), fields(B))):
        for k, e in close_fields(a, b, ws[i], 48).items():
            worst = max(worst, e)
            assert e <= 1e-6, (rows, i, k, e)
    say(f"  tile height {rows}: worst rel-L2 {worst:.2e}")
    batch.close()
    # released contexts step on alone with their own lists
    for s in A + B:
        s.step(5)
    for a, b in zip(fields(A), fields(B)):
        assert rel(b["u"], a["u"]) <= 1e-6
    close_all(A, B)


def test_autotune_restores_state_and_keeps_parity():
    ws = small_sweep()
    A, B = make(ws), make(ws)
    batch = lbib.Batch(B)
    batch.step(16)
    for s in A:
        s.step(16)
    before = fields(B)
    rows, groups, ms = batch.autotune(periods=1)
    say(f"  autotune: {rows} rows, {groups} groups; ms per step {ms}")
    assert (groups, rows) in ms and batch.tile == rows and batch.groups == groups
    assert {(1, 8), (1, 16), (2, 8), (2, 16)} <= set(ms)
    assert (1, 4) not in ms and (2, 4) not in ms       # the periodic member has ny = 98
    assert_bit_equal(before, fields(B), "after autotuning")
    batch.step(32)
    for s in A:
        s.step(32)
    batch.sync()
    for i, (a, b) in enumerate(zip(fields(A), fields(B))):
        for k, e in close_fields(a, b, ws[i], 48).items():
            assert e <= 1e-6, (i, k, e)
    batch.close()
    close_all(A, B)


def test_batched_matches_oracle():
    w = W.sweep_member(3, steps=60, side_lo=64.0, side_hi=130.0)
    others = [W.sweep_member(i, side_lo=64.0, side_hi=130.0) for i in (5, 9)]
    say(f"case {w.name}: 60 steps batched at tile height 16, and the oracle")
    sims = make([w] + others)
    batch = lbib.Batch(sims)
    batch.set_tile(16)
    batch.step(60)
    batch.sync()
    G = sims[0].get_fields()
    o = O.from_workload(w)
    o.step(60)
    R = o.get_fields()
    out = PB.field_errors(G, R, w.rho0, w.xy, 60, w.n_species)
    say("  errors:", PB.fmt(out))
    PB.assert_fields(out)
    batch.close()
    close_all(sims)


def test_batch_errors():
    ws = small_sweep(3)
    A = make(ws)
    with pytest.raises(lbib.LbibError):
        lbib.Batch([A[0], A[0]])                      # repeated
    empty = lbib.Simulation(ws[0].params_dict())
    with pytest.raises(lbib.LbibError):
        lbib.Batch([A[0], empty])                     # no cells
    two = lbib.from_workload(W.small_tissue(nx=96, ny=70, n_cells=4, n_species=2, seed=1))
    with pytest.raises(lbib.LbibError):
        lbib.Batch([A[0], two])                       # species counts differ
    batch = lbib.Batch(A)
    with pytest.raises(lbib.LbibError):
        lbib.Batch([A[1]])                            # already adopted
    with pytest.raises(lbib.LbibError) as e:
        A[0].step(1)                                  # stepped by the batch
    assert e.value.status == lbib.ESTATE
    with pytest.raises(lbib.LbibError):
        batch.set_tile(5)
    batch.step(3)
    with pytest.raises(lbib.LbibError) as e:
        batch.set_tile(16)                            # between list periods
    assert e.value.status == lbib.ESTATE
    with pytest.raises(lbib.LbibError):
        batch.autotune(1)
    with pytest.raises(lbib.LbibError):
        batch.set_groups(2)                           # between list periods
    with pytest.raises(lbib.LbibError):
        batch.set_groups(3)
    A[2].close()                                      # the batch can no longer step
    with pytest.raises(lbib.LbibError) as e:
        batch.step(1)
    assert e.value.status == lbib.ESTATE
    batch.close()
    A[0].step(2)                                      # released
    close_all(A, [empty, two])


def test_full_sweep_sampled_members_bit_identical():
    """The 64-simulation sweep at its real sizes: three members stepped alone match their
    batched selves bit for bit over two list periods."""
    ws = [W.sweep_member(i) for i in range(W.SWEEP_SIMS)]
    say(f"sweep: {sum(w.nx * w.ny for w in ws)} lattice nodes, {sum(w.n_nodes for w in ws)} membrane nodes")
    B = make(ws)
    batch = lbib.Batch(B)
    batch.step(32)
    batch.sync()
    for i in (0, 31, 63):
        a = lbib.from_workload(ws[i])
        a.step(32)
        FA, FB = a.get_fields(), B[i].get_fields()
        for k in ("rho", "u", "phi", "xy", "mask"):
            assert np.array_equal(FA[k], FB[k]), (i, k)
        a.close()
        say(f"  member {i} ({ws[i].nx}x{ws[i].ny}, {ws[i].n_cells} cells): bit-identical")
    batch.close()
    close_all(B)
