"""Seeded synthetic inputs shared by the HIP path, the oracle tests and the bench.

This module builds geometry and initial fields only: cell polygons (a jittered
circle, or a Voronoi tissue clipped between walls and periodic in x), their rest
lengths and rest areas, and initial concentration fields.  It holds none of the
method's arithmetic (no equilibria, collisions, delta kernels or forces), and it
imports nothing from the HIP binding or from the oracle.

Every random draw comes from ``numpy.random.SeedSequence(1503)`` spawned per
workload and per purpose, so both sides of a parity test see identical arrays.

The workloads follow the paper's setting of a fluid lattice with polygonal cells
(Section "Cell Representation": closed CCW polygons, domain ID on the left, zero
for the extracellular space) and its reaction laws (constant source and linear
decay; the Schnakenberg kinetics of the Turing example).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 1503

# reaction kinds (mirrors the C ABI enumerations by value)
REACT_NONE = 0
REACT_SOURCE_DECAY = 1
REACT_SCHNAKENBERG = 2

PERIODIC = 0
WALLS = 1

DELTA_COS4 = 0
DELTA_PESKIN4 = 1


def _rng(workload_id: int, purpose: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, workload_id, purpose]))


@dataclass
class Species:
    D: float
    phi_ref: float = 0.0
    reaction: int = REACT_NONE
    c: tuple = (0.0, 0.0, 0.0, 0.0)
    no_flux: bool = False       # the membranes are no-flux boundaries for the species


@dataclass
class Workload:
    """Everything one simulation needs.  Lattice units throughout (dx = dt = 1)."""
    name: str
    nx: int
    ny: int
    bc_y: int
    tau: float
    rho0: float = 1.0
    body_accel: tuple = (0.0, 0.0)
    delta_kernel: int = DELTA_COS4
    k_spring: float = 0.0
    phi_m: float = 0.0
    kappa_area: float = 0.0
    species: list = field(default_factory=list)
    mass_source: float = 0.0        # constant mass source per node inside a cell and step
    area_alpha: float = 0.0         # area controller: S_k = mass_source + area_alpha (A0_k - A_k)
    mass_phi_gamma: float = 0.0     # + mass_phi_gamma phi_0(x) inside cells (Case III's source)
    pressure_ring: bool = False     # the lattice's outer ring holds the density at rho0 (outflow)
    interp_half_force: bool = False  # membrane nodes move with the interpolated u + f/2
    no_flux_zeroth: bool = False    # no-flux membranes in the zeroth-order form
    no_flux_bounce: bool = False    # no-flux membranes in the bounce-back form (conserves the species)
    steps: int = 1
    # geometry (may be empty)
    offsets: np.ndarray = None      # int32 [n_cells+1]
    xy: np.ndarray = None           # float64 [N, 2], CCW per cell
    rest_len: np.ndarray = None     # float64 [N] or None (initial); edge k joins node k and its successor
    rest_area: np.ndarray = None    # float64 [n_cells] or None (initial)
    source_cells: np.ndarray = None  # uint8 [n_cells] source cells of the source/decay law, None: all
    node_sources: np.ndarray = None  # float64 [ny, nx] mass per node and step (point sources), None: none
    pressure_nodes: np.ndarray = None  # uint8 [ny, nx] pressure points held at rho0, None: none
    # initial fields (None = rho0, u = 0, phi = phi_ref)
    rho_init: np.ndarray = None     # float64 [ny, nx]
    u_init: np.ndarray = None       # float64 [2, ny, nx]
    phi_init: np.ndarray = None     # float64 [S, ny, nx]

    @property
    def n_cells(self) -> int:
        return 0 if self.offsets is None else len(self.offsets) - 1

    @property
    def n_nodes(self) -> int:
        return 0 if self.xy is None else int(self.xy.shape[0])

    @property
    def n_species(self) -> int:
        return len(self.species)

    def params_dict(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, bc_y=self.bc_y, tau=self.tau, rho0=self.rho0,
                    body_accel=tuple(self.body_accel), delta_kernel=self.delta_kernel,
                    k_spring=self.k_spring, phi_m=self.phi_m, kappa_area=self.kappa_area,
                    species=[dict(D=s.D, phi_ref=s.phi_ref, reaction=s.reaction, c=tuple(s.c),
                                  no_flux=bool(s.no_flux)) for s in self.species],
                    mass_source=self.mass_source, area_alpha=self.area_alpha,
                    mass_phi_gamma=self.mass_phi_gamma,
                    pressure_ring=self.pressure_ring, interp_half_force=self.interp_half_force,
                    no_flux_zeroth=self.no_flux_zeroth, no_flux_bounce=self.no_flux_bounce)

    def mask_needed(self) -> bool:
        return any(s.reaction == REACT_SOURCE_DECAY for s in self.species)


# --------------------------------------------------------------------------------------
# geometry helpers (input preparation only)
# --------------------------------------------------------------------------------------

def edge_lengths(offsets: np.ndarray, xy: np.ndarray) -> np.ndarray:
    """Length of the edge from node k to its cyclic successor within its cell."""
    out = np.empty(xy.shape[0])
    for c in range(len(offsets) - 1):
        a, b = int(offsets[c]), int(offsets[c + 1])
        p = xy[a:b]
        q = np.roll(p, -1, axis=0)
        out[a:b] = np.hypot(q[:, 0] - p[:, 0], q[:, 1] - p[:, 1])
    return out


def circle_cell(cx: float, cy: float, radius: float, n: int, jitter: float,
                rng: np.random.Generator | None):
    """One CCW polygon: node k at angle 2*pi*k/n, radius R + U(-jitter, jitter)."""
    th = 2.0 * np.pi * np.arange(n) / n
    r = np.full(n, float(radius))
    if rng is not None and jitter > 0:
        r = r + rng.uniform(-jitter, jitter, size=n)
    xy = np.stack([cx + r * np.cos(th), cy + r * np.sin(th)], axis=1)
    return np.array([0, n], dtype=np.int32), xy


def _resample(poly: np.ndarray, spacing: float) -> np.ndarray:
    """Split every edge of a closed polygon into ceil(L/spacing) equal segments."""
    out = []
    m = len(poly)
    for k in range(m):
        a = poly[k]
        b = poly[(k + 1) % m]
        L = float(np.hypot(*(b - a)))
        ns = max(1, int(math.ceil(L / spacing - 1e-9)))
        t = np.arange(ns) / ns
        out.append(a[None, :] + t[:, None] * (b - a)[None, :])
    return np.concatenate(out, axis=0)


def voronoi_tissue(nx: int, ny: int, n_cells: int, rng: np.random.Generator,
                   spacing: float = 0.5, inset: float = 0.5, y_lo: float = 2.0,
                   y_hi: float | None = None):
    """Voronoi tissue of ``n_cells`` uniform seeds, periodic in x, clipped to [y_lo, y_hi].

    Clipping uses mirror seeds across both clip lines (the bisector of a seed and
    its mirror image is the clip line), x-periodicity uses replicas at +-nx.  Each
    region's vertices are ordered by angle about its seed (CCW), pulled towards the
    polygon centroid by ``inset`` (capped at a quarter of the vertex-centroid
    distance), near-coincident vertices are merged, and every edge is split into
    segments no longer than ``spacing``.  Coordinates stay unwrapped in x.
    """
    from scipy.spatial import Voronoi

    if y_hi is None:
        y_hi = ny - 3.0
    seeds = np.stack([rng.uniform(0.0, nx, size=n_cells),
                      rng.uniform(y_lo + 1.0, y_hi - 1.0, size=n_cells)], axis=1)
    reps = []
    for dx in (0.0, -nx, nx):
        base = seeds + np.array([dx, 0.0])
        reps.append(base)
        lo = base.copy(); lo[:, 1] = 2 * y_lo - lo[:, 1]
        hi = base.copy(); hi[:, 1] = 2 * y_hi - hi[:, 1]
        reps.append(lo)
        reps.append(hi)
    pts = np.concatenate(reps, axis=0)
    vor = Voronoi(pts)
    polys = []
    for i in range(n_cells):
        reg = vor.regions[vor.point_region[i]]
        if len(reg) < 3 or -1 in reg:
            raise RuntimeError("unbounded Voronoi region for an interior seed")
        v = vor.vertices[reg]
        ang = np.arctan2(v[:, 1] - seeds[i, 1], v[:, 0] - seeds[i, 0])
        v = v[np.argsort(ang)]
        # area centroid
        q = np.roll(v, -1, axis=0)
        cr = v[:, 0] * q[:, 1] - q[:, 0] * v[:, 1]
        A = 0.5 * cr.sum()
        cxy = np.array([((v[:, 0] + q[:, 0]) * cr).sum(), ((v[:, 1] + q[:, 1]) * cr).sum()]) / (6 * A)
        d = cxy[None, :] - v
        dist = np.hypot(d[:, 0], d[:, 1])
        step = np.minimum(inset, 0.25 * dist)
        v = v + d * (step / dist)[:, None]
        # merge near-coincident consecutive vertices
        keep = [0]
        for k in range(1, len(v)):
            if np.hypot(*(v[k] - v[keep[-1]])) >= 0.25:
                keep.append(k)
        if len(keep) > 2 and np.hypot(*(v[keep[0]] - v[keep[-1]])) < 0.25:
            keep.pop()
        v = v[keep]
        if len(v) < 3:
            continue
        polys.append(_resample(v, spacing))
    offsets = np.zeros(len(polys) + 1, dtype=np.int32)
    offsets[1:] = np.cumsum([len(p) for p in polys])
    xy = np.concatenate(polys, axis=0).astype(np.float64)
    return offsets, xy


def _attach_geometry(w: Workload, offsets, xy, rest_len=None, rest_area=None):
    """Attach cells.  ``None`` rest lengths / areas mean "the initial ones", which each
    side (library and oracle) derives from the positions itself."""
    w.offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    w.xy = np.ascontiguousarray(xy, dtype=np.float64)
    w.rest_len = None if rest_len is None else np.ascontiguousarray(rest_len, dtype=np.float64)
    w.rest_area = None if rest_area is None else np.ascontiguousarray(rest_area, dtype=np.float64)
    return w


# --------------------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------------------

def tiny_cell(steps: int = 200) -> Workload:
    """64x64 periodic lattice, tau = 1, one jittered 64-node circle of radius 10 at (32, 32),
    springs k = 0.01 with rest length of the unjittered 64-gon edge, area pressure to
    rest area 100*pi, one species (D = 0.1) with a source of 1e-3 per step inside the
    cell and linear decay 1e-4, starting from zero concentration."""
    rng = _rng(1, 0)
    offsets, xy = circle_cell(32.0, 32.0, 10.0, 64, 0.5, rng)
    n = 64
    l0 = np.full(n, 2.0 * 10.0 * math.sin(math.pi / n))
    w = Workload(name="tiny: 64x64 periodic, 1 cell x 64 nodes, D2Q9 + 1 D2Q5",
                 nx=64, ny=64, bc_y=PERIODIC, tau=1.0, rho0=1.0,
                 k_spring=0.01, kappa_area=1e-3, delta_kernel=DELTA_COS4,
                 species=[Species(D=0.1, phi_ref=0.0, reaction=REACT_SOURCE_DECAY,
                                  c=(1e-3, 1e-4, 0.0, 0.0))],
                 steps=steps)
    return _attach_geometry(w, offsets, xy, rest_len=l0, rest_area=np.array([math.pi * 100.0]))


LEAKAGE_LEVELS = 4                     # lattice resolutions of the leakage study
LEAKAGE_MAXLENGTHS = (0.1, 0.5, 2.5)   # largest node spacing, in lattice units


def leakage_case(level: int, maxlength: float, steps: int | None = None) -> Workload:
    """The membrane-leakage validation (Section "Validation", Case IV): one circular cell under
    a constant membrane tension and nothing else (no springs, no area term, no mass source,
    no species), at resolution ``level`` = 0..3 of the paper's study:
      lattice 100 * 2^level squared, periodic in x and y, tau = 1 (nu = 1/6);
      cell diameter 10 * 2^level lattice units (the unit circle of area pi / 4 at dx =
      0.1 / 2^level), centred in the lattice;
      tension phi_m = 1e-3 / 2^level (the tabulated lattice force of each resolution);
      ceil(pi D / maxlength) equally spaced nodes, so no edge exceeds ``maxlength``;
      10^4 * 4^level steps (one unit of non-dimensional time, dt = 1e-4 / 4^level)."""
    if not 0 <= level < LEAKAGE_LEVELS:
        raise ValueError("level must be 0..3")
    L = 100 * 2 ** level
    D = 10.0 * 2 ** level
    n = int(math.ceil(math.pi * D / maxlength))
    offsets, xy = circle_cell(L / 2.0, L / 2.0, D / 2.0, n, 0.0, None)
    w = Workload(name=f"leakage level {level}: {L}x{L} periodic, one {n}-node circle of diameter {D:g}, "
                      f"max spacing {maxlength:g}",
                 nx=L, ny=L, bc_y=PERIODIC, tau=1.0, rho0=1.0, phi_m=1e-3 / 2 ** level,
                 delta_kernel=DELTA_COS4, steps=10000 * 4 ** level if steps is None else steps)
    return _attach_geometry(w, offsets, xy)


GROWTH_CASES = (1, 2, 3)        # the growth validations: point source, uniform source, phi-driven source


def growth_case(case: int, level: int, maxlength: float = 0.5, steps: int | None = None,
                bounce: bool = False) -> Workload:
    """The growth validations (Section "Validation", Cases I-III, and their table of lattice
    discretisations): a circular cell of diameter 10 * 2^level lattice units in the middle of a
    lattice 100 * 2^level squared (its centre 0.3 off the central node in x and y, so that no
    membrane node starts on a lattice line), tau = 1 for the fluid, one species with tau_D = 1
    (D = 1/6) that starts at 1 inside the polygon's inscribed circle and 0 elsewhere and sees
    the membrane as a no-flux boundary, no membrane forces, the outer ring held at rho0 (iso-pressure outflow), and
    10^4 * 4^level steps (one unit of non-dimensional time, dt = 1e-4 / 4^level).
    ceil(pi D / maxlength) equally spaced nodes.  The cell grows by
      case 1: a point source of 1e-2 lattice areas per step at the central node (the tabulated
              S^LB at every level), so A = A0 + 1e-2 t;
      case 2: a uniform source ln 2 * dt per inside node and step, so A = A0 2^(t dt), doubling
              in one unit of time;
      case 3: a uniform source dt * phi per inside node and step (strength 1 times the
              concentration), so A = A0 (1 + t dt) while the species is conserved.
    ``bounce``: the no-flux membrane in the bounce-back form, which conserves the species."""
    if case not in GROWTH_CASES:
        raise ValueError("case must be 1, 2 or 3")
    if not 0 <= level < LEAKAGE_LEVELS:
        raise ValueError("level must be 0..3")
    L = 100 * 2 ** level
    D = 10.0 * 2 ** level
    dt = 1e-4 / 4 ** level
    n = int(math.ceil(math.pi * D / maxlength))
    cx, cy = L / 2.0 + 0.3, L / 2.0 - 0.3
    offsets, xy = circle_cell(cx, cy, D / 2.0, n, 0.0, None)
    yy, xx = np.mgrid[0:L, 0:L]
    phi = (np.hypot(xx - cx, yy - cy) < D / 2.0 * math.cos(math.pi / n)).astype(np.float64)[None]
    w = Workload(name=f"growth case {case} level {level}: {L}x{L}, one {n}-node circle of diameter {D:g}",
                 nx=L, ny=L, bc_y=PERIODIC, tau=1.0, rho0=1.0, delta_kernel=DELTA_COS4,
                 species=[Species(D=1.0 / 6.0, phi_ref=0.0, reaction=REACT_NONE, no_flux=True)],
                 pressure_ring=True, steps=10000 * 4 ** level if steps is None else steps, phi_init=phi,
                 no_flux_bounce=bounce)
    if case == 1:
        w.node_sources = np.zeros((L, L))
        w.node_sources[L // 2, L // 2] = 1e-2
    elif case == 2:
        w.mass_source = math.log(2.0) * dt
    else:
        w.mass_phi_gamma = dt
    return _attach_geometry(w, offsets, xy)


def growth_law(case: int, level: int, area0: float, t: float) -> float:
    """The analytical area of ``growth_case(case, level)`` after t steps, from its initial area."""
    dt = 1e-4 / 4 ** level
    if case == 1:
        return area0 + 1e-2 * t
    if case == 2:
        return area0 * 2.0 ** (t * dt)
    return area0 * (1.0 + t * dt)


def tissue(steps: int = 10000) -> Workload:
    """512x512, no-slip walls in y, periodic in x, tau = 0.8, 100 Voronoi cells at 0.5 lu
    node spacing, springs k = 0.02 at their initial lengths, body acceleration 1e-6 along x,
    two Schnakenberg species (D = 0.05, 0.2; a = 0.1, b = 0.9, rate 0.01 per step)
    starting from 1 + N(0, 0.01)."""
    rng = _rng(2, 0)
    offsets, xy = voronoi_tissue(512, 512, 100, rng)
    frng = _rng(2, 1)
    phi = 1.0 + 0.01 * frng.standard_normal((2, 512, 512))
    sch = (0.1, 0.9, 0.01, 0.0)
    w = Workload(name="tissue: 512x512 walls-y, 100 Voronoi cells, D2Q9 + 2 D2Q5 (Schnakenberg)",
                 nx=512, ny=512, bc_y=WALLS, tau=0.8, rho0=1.0, body_accel=(1e-6, 0.0),
                 k_spring=0.02, delta_kernel=DELTA_COS4,
                 species=[Species(D=0.05, phi_ref=1.0, reaction=REACT_SCHNAKENBERG, c=sch),
                          Species(D=0.2, phi_ref=1.0, reaction=REACT_SCHNAKENBERG, c=sch)],
                 steps=steps, phi_init=phi)
    return _attach_geometry(w, offsets, xy)


def large(steps: int = 5000, n: int = 2048, n_cells: int = 2000) -> Workload:
    """2048x2048, walls in y, periodic in x, tau = 0.6, 2000 Voronoi cells (about 725k nodes),
    k = 0.02 at initial lengths, body acceleration 1e-6 along x, one species with the
    tiny workload's source/decay law (D = 0.1, source 1e-3 inside cells, decay 1e-4)."""
    rng = _rng(3, 0)
    offsets, xy = voronoi_tissue(n, n, n_cells, rng)
    w = Workload(name=f"large: {n}x{n} walls-y, {n_cells} Voronoi cells, D2Q9 + 1 D2Q5",
                 nx=n, ny=n, bc_y=WALLS, tau=0.6, rho0=1.0, body_accel=(1e-6, 0.0),
                 k_spring=0.02, delta_kernel=DELTA_COS4,
                 species=[Species(D=0.1, phi_ref=0.0, reaction=REACT_SOURCE_DECAY,
                                  c=(1e-3, 1e-4, 0.0, 0.0))],
                 steps=steps)
    return _attach_geometry(w, offsets, xy)


def small_tissue(nx: int = 200, ny: int = 130, n_cells: int = 12, bc_y: int = WALLS,
                 n_species: int = 1, tau: float = 0.7, seed: int = 0,
                 delta_kernel: int = DELTA_COS4, body=(2e-5, 0.0), k_spring: float = 0.02,
                 phi_m: float = 0.0, kappa_area: float = 0.0, stretch: float = 1.0,
                 steps: int = 50) -> Workload:
    """A parity-sized tissue with a ragged lattice (not a multiple of the tile sizes).

    ``stretch`` scales the rest lengths so the springs start loaded and drive flow."""
    rng = _rng(100 + seed, 0)
    if bc_y == WALLS:
        offsets, xy = voronoi_tissue(nx, ny, n_cells, rng)
    else:
        offsets, xy = voronoi_tissue(nx, ny, n_cells, rng, y_lo=2.0, y_hi=ny - 3.0)
    frng = _rng(100 + seed, 1)
    species = []
    phi = None
    if n_species >= 1:
        species.append(Species(D=0.1, phi_ref=0.0, reaction=REACT_SOURCE_DECAY, c=(1e-3, 1e-4, 0.0, 0.0)))
    if n_species == 2:
        sch = (0.1, 0.9, 0.01, 0.0)
        species = [Species(D=0.05, phi_ref=1.0, reaction=REACT_SCHNAKENBERG, c=sch),
                   Species(D=0.2, phi_ref=1.0, reaction=REACT_SCHNAKENBERG, c=sch)]
        phi = 1.0 + 0.01 * frng.standard_normal((2, ny, nx))
    w = Workload(name=f"small tissue {nx}x{ny}, {n_cells} cells, S={n_species}",
                 nx=nx, ny=ny, bc_y=bc_y, tau=tau, rho0=1.0, body_accel=tuple(body),
                 k_spring=k_spring, phi_m=phi_m, kappa_area=kappa_area,
                 delta_kernel=delta_kernel, species=species, steps=steps, phi_init=phi)
    rest = None if stretch == 1.0 else edge_lengths(offsets, xy) * stretch
    return _attach_geometry(w, offsets, xy, rest_len=rest)


def random_fields(w: Workload, seed: int, amp_rho: float = 1e-3, amp_u: float = 1e-3,
                  amp_phi: float = 0.05) -> Workload:
    """Smooth-ish random initial fields for lattice-only parity cases."""
    rng = _rng(200 + seed, 0)
    ny, nx = w.ny, w.nx
    w.rho_init = w.rho0 + amp_rho * rng.standard_normal((ny, nx))
    w.u_init = amp_u * rng.standard_normal((2, ny, nx))
    if w.n_species:
        base = np.array([s.phi_ref if s.phi_ref != 0 else 0.1 for s in w.species])[:, None, None]
        w.phi_init = base + amp_phi * rng.standard_normal((w.n_species, ny, nx))
    return w


def static_tissue(sample: int, held_out: bool = True, n: int = 256, source_p: float = 0.2) -> Workload:
    """One steady-state sample: an n x n lattice (walls in y, periodic in x) holding a static
    Voronoi tissue of 50..300 cells, of which each is a source with probability source_p
    (at least one), and one species with diffusivity D ~ U(0.02, 0.5), source 1e-3 inside
    the source cells and decay lambda ~ U(1e-5, 1e-3).  The fluid and the membranes stay at
    rest (no forces); the species starts from zero.  Held-out samples and training samples
    come from disjoint seed streams."""
    rng = _rng(5 if held_out else 6, sample)
    n_cells = int(rng.integers(50, 301))
    offsets, xy = voronoi_tissue(n, n, n_cells, rng)
    src = (rng.random(n_cells) < source_p).astype(np.uint8)
    if not src.any():
        src[int(rng.integers(n_cells))] = 1
    D = float(rng.uniform(0.02, 0.5))
    lam = float(rng.uniform(1e-5, 1e-3))
    w = Workload(name=f"static tissue {n}x{n} walls-y, {n_cells} cells ({int(src.sum())} sources), "
                      f"D = {D:.4g}, decay {lam:.3g}",
                 nx=n, ny=n, bc_y=WALLS, tau=1.0, rho0=1.0, species=[
                     Species(D=D, phi_ref=0.0, reaction=REACT_SOURCE_DECAY, c=(1e-3, lam, 0.0, 0.0))],
                 steps=0)
    w = _attach_geometry(w, offsets, xy)
    w.source_cells = src
    return w


def sweep_member(sim: int, steps: int = 2000, side_lo: float = 128.0, side_hi: float = 1024.0) -> Workload:
    """Simulation ``sim`` of the batched parameter sweep: nx and ny each drawn log-uniformly
    from [side_lo, side_hi] (rounded), walls in y and periodic in x, min(max(U{10..500},
    ceil(8 max(nx, ny) / min(nx, ny))), floor(nx ny / 100)) Voronoi cells at 0.5 lu node
    spacing (seeds redrawn while a cell would span the lattice), tau ~ U(0.55, 1.2), spring
    stiffness k ~ U(0.005, 0.05) at the initial lengths, body acceleration 1e-6 along x, and
    one species with the tiny workload's source/decay law (D = 0.1, source 1e-3 inside cells,
    decay 1e-4)."""
    rng = _rng(4, sim)
    lo, hi = math.log(side_lo), math.log(side_hi)
    nx = int(round(math.exp(rng.uniform(lo, hi))))
    ny = int(round(math.exp(rng.uniform(lo, hi))))
    # at least ~8 cells across the longer side keeps every cell narrower than the lattice
    n_min = math.ceil(8.0 * max(nx, ny) / min(nx, ny))
    n_cells = min(max(int(rng.integers(10, 501)), n_min), nx * ny // 100)
    tau = float(rng.uniform(0.55, 1.2))
    k = float(rng.uniform(0.005, 0.05))
    while True:                     # redraw the seeds while a cell spans the lattice
        offsets, xy = voronoi_tissue(nx, ny, n_cells, rng)
        span = max(max(np.ptp(xy[a:b, 0]) - nx, np.ptp(xy[a:b, 1]) - ny)
                   for a, b in zip(offsets[:-1], offsets[1:]))
        if span < -4.0:
            break
    w = Workload(name=f"sweep {sim}: {nx}x{ny} walls-y, {n_cells} cells, tau {tau:.3f}, k {k:.4f}",
                 nx=nx, ny=ny, bc_y=WALLS, tau=tau, rho0=1.0, body_accel=(1e-6, 0.0),
                 k_spring=k, delta_kernel=DELTA_COS4,
                 species=[Species(D=0.1, phi_ref=0.0, reaction=REACT_SOURCE_DECAY,
                                  c=(1e-3, 1e-4, 0.0, 0.0))],
                 steps=steps)
    return _attach_geometry(w, offsets, xy)


SWEEP_SIMS = 64

WORKLOADS = {"tiny": tiny_cell, "tissue": tissue, "large": large}

# parity-sized cell cases: ragged lattices, both boundary kinds, both kernels, every force law
PARITY_CASES = {
    "tiny": lambda: tiny_cell(),
    "walls": lambda: small_tissue(stretch=0.9, kappa_area=1e-3, phi_m=1e-3),
    "periodic": lambda: small_tissue(nx=150, ny=100, n_cells=9, bc_y=PERIODIC, n_species=2, seed=2,
                                     stretch=1.1),
    "peskin": lambda: small_tissue(nx=96, ny=70, n_cells=12, delta_kernel=DELTA_PESKIN4, seed=4, stretch=0.95),
}


def no_flux_tissue(static: bool = True, no_flux: bool = True, seed: int = 7, nx: int = 120, ny: int = 90,
                   n_cells: int = 8, steps: int = 100) -> Workload:
    """A small walled tissue whose one species (source inside the cells, linear decay) sees the
    membranes as no-flux boundaries (Section "Signalling"). ``static``: no forces and no body
    acceleration, so the fluid stays at rest and the membranes where they are; otherwise
    pre-stretched springs and a body acceleration move both."""
    w = small_tissue(nx=nx, ny=ny, n_cells=n_cells, n_species=1, seed=seed,
                     body=(0.0, 0.0) if static else (2e-5, 0.0),
                     k_spring=0.0 if static else 0.02, stretch=1.0 if static else 0.9, steps=steps)
    w.species[0].no_flux = no_flux
    w.name = f"no-flux tissue {nx}x{ny}, {n_cells} cells, {'static' if static else 'moving'}" + \
             ("" if no_flux else ", membranes invisible")
    return w


def mass_source_tissue(static: bool = False, mass_source: float = 1e-4, area_alpha: float = 1e-6,
                       target: float = 1.2, no_flux: bool = False, seed: int = 11, nx: int = 120,
                       ny: int = 90, n_cells: int = 8, steps: int = 60) -> Workload:
    """A small walled tissue with mass sources inside the cells (Section "Control of Cell
    Area"): every cell's reference area is ``target`` times the mean area nx ny / n_cells, so
    the area controller grows the smaller cells and shrinks the larger ones, on top of the
    constant source.  ``static``: no forces and no body acceleration; otherwise pre-stretched
    springs and a body acceleration.  ``no_flux``: the species sees the membranes as no-flux
    boundaries."""
    w = small_tissue(nx=nx, ny=ny, n_cells=n_cells, n_species=1, seed=seed,
                     body=(0.0, 0.0) if static else (2e-5, 0.0),
                     k_spring=0.0 if static else 0.02, stretch=1.0 if static else 0.9, steps=steps)
    w.mass_source = mass_source
    w.area_alpha = area_alpha
    w.species[0].no_flux = no_flux
    w.rest_area = np.full(n_cells, target * nx * ny / n_cells)
    w.name = f"mass-source tissue {nx}x{ny}, {n_cells} cells, source {mass_source:g}, alpha {area_alpha:g}" + \
             (", static" if static else "") + (", no-flux species" if no_flux else "")
    return w
