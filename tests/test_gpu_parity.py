"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on seeded inputs.

Bar: relative L2 error <= 1e-5 on the velocity, the concentrations and the node displacement
X - X0 (FP32 populations against FP64), and on the density deviation rho - rho0 up to the
rounding floor of FP32 deviation storage (parity_bars); node order, cell IDs and the domain-ID
map of identical positions bit-exact; after several steps domain IDs may differ only at
lattice nodes whose distance to a membrane edge is below 1e-3 (positions then differ at
round-off level and the inside test is discontinuous there).
"""
import sys

import numpy as np
import pytest

import parity_bars as PB
from oracle import oracle as O
from paper_1503_06726_amd import lbib
from paper_1503_06726_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def edge_distance(offsets, xy, px, py, nx, ny):
    """Distance from lattice points (px, py) to the nearest membrane edge, over periodic images."""
    d = np.full(px.shape, np.inf)
    for c in range(len(offsets) - 1):
        P = xy[offsets[c]:offsets[c + 1]]
        Q = np.roll(P, -1, 0)
        ab = (Q - P)[None]
        for sx in (-nx, 0, nx):
            for sy in (-ny, 0, ny):
                p = np.stack([px + sx, py + sy], -1)[:, None, :]
                t = np.clip(((p - P[None]) * ab).sum(-1) / (ab * ab).sum(-1), 0, 1)
                proj = P[None] + t[..., None] * ab
                d = np.minimum(d, np.sqrt(((p - proj) ** 2).sum(-1)).min(1))
    return d


def compare(G, R, w, steps, tol=TOL, check_mask=True):
    """Gate u, phi and X - X0 at tol (relative L2) and rho - rho0 at its bar (FP32 rounding
    of the stored deviations; parity_bars); domain IDs may differ only next to an edge."""
    out = PB.field_errors(G, R, w.rho0, w.xy if w.n_cells else None, steps, w.n_species)
    say("  errors:", PB.fmt(out))
    PB.assert_fields(out, tol)
    if check_mask and w.n_cells:
        bad = np.argwhere(G["mask"] != R["mask"])
        if len(bad):
            d = edge_distance(w.offsets, R["xy"], bad[:, 1].astype(float), bad[:, 0].astype(float), w.nx, w.ny)
            say(f"  mask mismatches: {len(bad)}, max edge distance {d.max():.2e}")
            assert d.max() < 1e-3
    return out


def run_pair(w, steps):
    say(f"case {w.name}: {steps} steps (GPU)")
    g = lbib.from_workload(w)
    g.step(steps)
    G = g.get_fields()
    g.close()
    say("  oracle")
    o = O.from_workload(w)
    o.step(steps)
    R = o.get_fields()
    return G, R


# ------------------------------------------------------------------------------------------
# lattice alone (rows: D2Q9 collide/stream with body force, D2Q5 per species, walls)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("bc,S,nx,ny", [(0, 0, 200, 130), (1, 1, 200, 130), (1, 2, 67, 45), (0, 2, 64, 64),
                                        (0, 1, 4, 4), (1, 0, 131, 9),
                                        # tile orders: 8 or 16 tile columns with an odd or even
                                        # number of 8-row tile rows
                                        (0, 1, 512, 72), (1, 1, 1024, 40), (0, 0, 512, 64)])
def test_lattice_only(bc, S, nx, ny):
    w = W.Workload(name=f"lattice {nx}x{ny} bc={bc} S={S}", nx=nx, ny=ny, bc_y=bc, tau=0.8,
                   body_accel=(2e-5, -1e-5))
    if S == 1:
        w.species = [W.Species(D=0.1, phi_ref=0.1, reaction=W.REACT_SOURCE_DECAY, c=(1e-3, 1e-2, 0, 0))]
    if S == 2:
        sch = (0.1, 0.9, 0.01, 0.0)
        w.species = [W.Species(D=0.05, phi_ref=1.0, reaction=W.REACT_SCHNAKENBERG, c=sch),
                     W.Species(D=0.2, phi_ref=1.0, reaction=W.REACT_SCHNAKENBERG, c=sch)]
    W.random_fields(w, seed=nx + ny + S)
    G, R = run_pair(w, 40)
    compare(G, R, w, 40)


# ------------------------------------------------------------------------------------------
# membrane rows at identical positions: forces, spreading, domain IDs
# ------------------------------------------------------------------------------------------
CELL_CASES = W.PARITY_CASES


@pytest.mark.parametrize("case", list(CELL_CASES))
def test_forces_spread_raster_at_set_cells(case):
    w = CELL_CASES[case]()
    say(f"case {case}: forces / spread / raster")
    g = lbib.from_workload(w)
    F, A = g.get_forces()
    e = g.get_spread()
    m = g.get_fields()["mask"]
    xy = g.get_fields()["xy"]
    g.close()
    o = O.from_workload(w)
    Fo, Ao = o.forces()
    eo = np.stack(O.spread(w.params_dict(), w.xy, Fo))
    eo[0] += w.body_accel[0]
    eo[1] += w.body_accel[1]
    mo, ov = O.raster(w.params_dict(), w.offsets, w.xy)
    assert ov == 0
    assert np.array_equal(xy, w.xy)                      # positions round-trip exactly
    say(f"  F {rel(F, Fo):.2e}  A {rel(A, Ao):.2e}  e {rel(e, eo):.2e}")
    assert rel(F, Fo) < 1e-6
    assert rel(A, Ao) < 1e-12
    assert rel(e, eo) < 1e-6
    assert np.array_equal(m, mo)                          # bit-exact at identical positions


# ------------------------------------------------------------------------------------------
# coupled steps
# ------------------------------------------------------------------------------------------
def test_coupled_tiny_200_steps():
    w = W.tiny_cell(200)
    G, R = run_pair(w, 200)
    compare(G, R, w, 200)


@pytest.mark.parametrize("case", list(CELL_CASES))
def test_coupled_cases(case):
    w = CELL_CASES[case]()
    G, R = run_pair(w, 60)
    compare(G, R, w, 60)


@pytest.mark.parametrize("case", ["walls", "periodic", "peskin"])
def test_coupled_half_force_velocity(case):
    """The nodes move with the half-force-shifted velocity u + f/2 (the option of the
    forcing's velocity): the coupled step still follows the oracle, over 80 steps (five list
    rebuilds and graph periods)."""
    w = CELL_CASES[case]()
    w.interp_half_force = True
    G, R = run_pair(w, 80)
    compare(G, R, w, 80)


def test_coupled_tissue_full_size():
    w = W.tissue()
    G, R = run_pair(w, 100)
    compare(G, R, w, 100)


def test_coupled_large_full_size():
    """The bench's workload and launch configuration (2048^2, 2000 cells, whole 16-step
    periods replayed from captured graphs) for three list periods against the oracle."""
    w = W.large()
    G, R = run_pair(w, 48)
    compare(G, R, w, 48)


def test_large_mask_bit_exact_at_set_cells():
    w = W.large()
    g = lbib.from_workload(w)
    m = g.get_fields(rho=False, u=False, phi=False)["mask"]
    F, _ = g.get_forces()
    g.close()
    mo, ov = O.raster(w.params_dict(), w.offsets, w.xy)
    assert ov == 0
    assert np.array_equal(m, mo)
    Fo, _ = O.forces(w.params_dict(), w.offsets, w.xy, W.edge_lengths(w.offsets, w.xy), np.zeros(w.n_cells))
    assert rel(F, Fo) < 1e-5 or np.abs(F - Fo).max() < 1e-9     # springs at rest: F ~ 0


# ------------------------------------------------------------------------------------------
# determinism, invariants, edge cases
# ------------------------------------------------------------------------------------------
def test_rerun_bit_identical():
    w = W.small_tissue(stretch=0.9)
    outs = []
    for _ in range(2):
        g = lbib.from_workload(w)
        g.step(50)
        outs.append(g.get_fields())
        g.close()
    for k in ("rho", "u", "phi", "xy", "mask"):
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_reduce_matches_oracle_invariants():
    w = W.small_tissue(n_species=1, stretch=0.9)
    g = lbib.from_workload(w)
    o = O.from_workload(w)
    r0 = g.reduce()
    g.step(30)
    o.step(30)
    r1 = g.reduce()
    io = o.invariants()
    say("  gpu", r1, "oracle", io)
    assert abs(r1[0] - r0[0]) < 1e-6 * r0[0]                     # walls: mass conserved
    assert abs(r1[0] - io[0]) < 1e-6 * io[0]
    assert np.allclose(r1[1:3], io[1:3], rtol=1e-4, atol=1e-9)
    assert abs(r1[3] - io[3]) < 1e-5 * abs(io[3])
    g.close()


def test_step_zero_and_empty_cells():
    w = W.tiny_cell()
    g = lbib.from_workload(w)
    a = g.get_fields()
    g.step(0)
    b = g.get_fields()
    for k in ("rho", "u", "phi", "xy", "mask"):
        assert np.array_equal(a[k], b[k])
    g.set_cells(np.zeros(1, np.int32), np.zeros((0, 2)))       # remove all cells
    g.step(5)
    c = g.get_fields()
    assert (c["mask"] == 0).all()
    g.close()


def test_largest_cell():
    th = 2 * np.pi * np.arange(4096) / 4096
    xy = np.stack([128.3 + 90 * np.cos(th), 127.6 + 90 * np.sin(th)], 1)
    w = W.Workload(name="largest cell: 4096 nodes", nx=256, ny=256, bc_y=W.PERIODIC, tau=0.9, phi_m=1e-4,
                   species=[W.Species(D=0.1, reaction=W.REACT_SOURCE_DECAY, c=(1e-3, 1e-4, 0, 0))])
    W._attach_geometry(w, np.array([0, 4096], np.int32), xy)
    G, R = run_pair(w, 20)
    compare(G, R, w, 20)


def test_invalid_cells_leave_state_unchanged():
    w = W.tiny_cell()
    g = lbib.from_workload(w)
    bad = w.xy[::-1].copy()                                      # clockwise
    with pytest.raises(lbib.LbibError) as ei:
        g.set_cells(w.offsets, bad)
    assert ei.value.status == lbib.EINVAL and "counter-clockwise" in str(ei.value)
    g.step(3)
    assert g.get_fields()["xy"].shape == (64, 2)
    g.close()


# ------------------------------------------------------------------------------------------
# reduced-precision population storage (FP16 / BF16 deviations, FP32 collision): the error
# against the FP64 oracle is reported per field; the bound only catches gross mistakes
# (a wrong storage scale or a direction mix-up gives O(1) errors)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("storage,bound", [(lbib.STORAGE_FP16, 1e-2), (lbib.STORAGE_BF16, 1e-1)])
@pytest.mark.parametrize("case", ["tiny", "walls", "periodic"])
def test_reduced_precision_storage(storage, bound, case):
    w = CELL_CASES[case]()
    prm = dict(w.params_dict(), storage=storage)
    say(f"case {case} storage {storage}")
    g = lbib.Simulation(prm)
    if w.phi_init is not None:
        g.set_fields(phi=w.phi_init)
    g.set_cells(w.offsets, w.xy, w.rest_len, w.rest_area)
    g.step(60)
    G = g.get_fields()
    g.close()
    o = O.from_workload(w)
    o.step(60)
    R = o.get_fields()
    errs = PB.field_errors(G, R, w.rho0, w.xy, 60, w.n_species)
    say("  errors:", PB.fmt(errs))
    for k in ("u", "X-X0", "phi"):
        if k in errs:
            assert errs[k] < bound, (k, errs[k])


# per-field error of reduced-precision storage at the bench workload (2048^2, 2000 cells),
# against the FP64 oracle, next to the FP32 path on the same steps
@pytest.mark.parametrize("storage,bound", [(lbib.STORAGE_FP32, 1e-5), (lbib.STORAGE_FP16, 1e-2),
                                           (lbib.STORAGE_BF16, 1e-1)])
def test_precision_per_field_at_large(storage, bound, large_oracle_fields):
    w, R, steps = large_oracle_fields
    say(f"large workload, storage {storage}, {steps} steps")
    g = lbib.from_workload(w, storage=storage)
    g.step(steps)
    G = g.get_fields(mask=False)
    g.close()
    errs = PB.field_errors(G, R, w.rho0, w.xy, steps, w.n_species)
    say("  errors:", PB.fmt(errs))
    for k in ("u", "X-X0", "phi"):
        assert errs[k] < bound, (k, errs[k])
    if storage == lbib.STORAGE_FP32:
        PB.assert_fields(errs)


@pytest.fixture(scope="module")
def large_oracle_fields():
    w = W.large()
    steps = 4
    o = O.from_workload(w)
    o.step(steps)
    return w, o.get_fields(), steps


# ------------------------------------------------------------------------------------------
# captured step graphs: whole 16-step periods replay a graph; single steps launch directly.
# Every replay (with eager work and synchronisation in between) must match direct launches
# bit for bit.
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["walls", "periodic"])
def test_graph_replays_match_direct_launches(case):
    w = CELL_CASES[case]()
    a = lbib.from_workload(w)
    b = lbib.from_workload(w)
    for rep in range(4):
        a.step(16)                       # one graph replay
        for _ in range(16):
            b.step(1)                    # direct launches
        A, B = a.get_fields(), b.get_fields()
        for k in ("rho", "u", "phi", "xy", "mask"):
            assert np.array_equal(A[k], B[k]), (rep, k)
        a.reduce()                       # eager work between replays
    a.step(40)                           # 2 replays + 8 direct steps
    for _ in range(40):
        b.step(1)
    A, B = a.get_fields(), b.get_fields()
    for k in ("rho", "u", "phi", "xy", "mask"):
        assert np.array_equal(A[k], B[k]), k
    a.close()
    b.close()
