"""ctypes wrapper of the FP64 CPU oracle (``oracle/lbib_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg use this module; the library under ``paper_1503_06726_amd`` never
imports it.  It shares no code with the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "lbib_oracle.c")

PERIODIC, WALLS = 0, 1
DELTA_COS, DELTA_PESKIN = 0, 1
REACT_NONE, REACT_SOURCE_DECAY, REACT_SCHNAKENBERG = 0, 1, 2


def build(openmp: bool = True) -> str:
    """Compile the oracle with gcc (contraction off so products round as written)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off"]
    if openmp:
        cmd.append("-fopenmp")
    cmd += ["-o", LIB_PATH + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("bc_y", C.c_int32),
                ("delta_kernel", C.c_int32), ("n_species", C.c_int32),
                ("interp_new_u", C.c_int32),
                ("tau", C.c_double), ("rho0", C.c_double), ("body", C.c_double * 2),
                ("k_spring", C.c_double), ("phi_m", C.c_double), ("kappa_area", C.c_double),
                ("D", C.c_double * 2), ("reaction", C.c_int32 * 2),
                ("rc", (C.c_double * 4) * 2), ("wall_u_top", C.c_double), ("no_flux", C.c_int32 * 2),
                ("mass_source", C.c_double), ("area_alpha", C.c_double), ("mass_phi_gamma", C.c_double),
                ("pressure_ring", C.c_int32), ("interp_half_force", C.c_int32),
                ("no_flux_zeroth", C.c_int32), ("no_flux_bounce", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("ORACLE_LIB")      # a planted-mistake build (mutation tests)
    if not path:
        path = LIB_PATH
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            build()
    L = C.CDLL(path)
    dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
    ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
    P = C.POINTER(Params)
    L.orc_delta1d.restype = C.c_double
    L.orc_delta1d.argtypes = [C.c_int32, C.c_double]
    L.orc_equilibrium9.argtypes = [C.c_double, C.c_double, C.c_double, dp]
    L.orc_equilibrium5.argtypes = [C.c_double, C.c_double, C.c_double, dp]
    L.orc_reaction.restype = C.c_double
    L.orc_reaction.argtypes = [P, C.c_int32, dp, C.c_int32]
    L.orc_forces.argtypes = [P, C.c_int32, ip, dp, dp, dp, dp, dp]
    L.orc_spread.argtypes = [P, C.c_int64, dp, dp, dp, dp]
    L.orc_interp.argtypes = [P, C.c_int64, dp, dp, dp, dp]
    L.orc_raster.restype = C.c_int64
    L.orc_raster.argtypes = [P, C.c_int32, ip, dp, ip]
    L.orc_create.restype = C.c_void_p
    L.orc_create.argtypes = [P]
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_set_cells.restype = C.c_int32
    L.orc_set_cells.argtypes = [C.c_void_p, C.c_int32, ip, dp, C.c_void_p, C.c_void_p]
    L.orc_set_fields.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_step.argtypes = [C.c_void_p, C.c_int32]
    L.orc_set_source_cells.argtypes = [C.c_void_p, C.c_void_p]
    L.orc_set_node_sources.argtypes = [C.c_void_p, C.c_void_p]
    L.orc_set_pressure_nodes.argtypes = [C.c_void_p, C.c_void_p]
    L.orc_ade_step.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
    L.orc_source_map.argtypes = [C.c_void_p, C.c_void_p]
    L.orc_get_fields.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_get_populations.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_set_populations.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_get_last_spread.argtypes = [C.c_void_p, dp, dp]
    L.orc_get_forces.argtypes = [C.c_void_p, dp, dp]
    L.orc_invariants.argtypes = [C.c_void_p, dp]
    L.orc_link_crossings.argtypes = [P, C.c_int32, ip, dp, dp]
    L.orc_get_prev_moments.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_set_prev_moments.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_no_flux_values.argtypes = [C.c_void_p, C.c_int32, dp]
    L.orc_threads.restype = C.c_int32
    L.orc_threads.argtypes = []
    L.orc_set_threads.restype = None
    L.orc_set_threads.argtypes = [C.c_int32]
    _lib = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_params(d: dict, interp_new_u: bool = False, wall_u_top: float = 0.0) -> Params:
    """Build oracle parameters from a workload parameter dict."""
    p = Params()
    p.nx, p.ny, p.bc_y = int(d["nx"]), int(d["ny"]), int(d["bc_y"])
    p.delta_kernel = int(d.get("delta_kernel", 0))
    sp = d.get("species", [])
    p.n_species = len(sp)
    p.interp_new_u = int(bool(interp_new_u))
    p.tau, p.rho0 = float(d["tau"]), float(d.get("rho0", 1.0))
    b = d.get("body_accel", (0.0, 0.0))
    p.body[0], p.body[1] = float(b[0]), float(b[1])
    p.k_spring = float(d.get("k_spring", 0.0))
    p.phi_m = float(d.get("phi_m", 0.0))
    p.kappa_area = float(d.get("kappa_area", 0.0))
    for s, spc in enumerate(sp):
        p.D[s] = float(spc["D"])
        p.reaction[s] = int(spc.get("reaction", 0))
        for k, v in enumerate(spc.get("c", (0, 0, 0, 0))):
            p.rc[s][k] = float(v)
        p.no_flux[s] = 1 if spc.get("no_flux", False) else 0
    p.wall_u_top = float(wall_u_top)
    p.mass_source = float(d.get("mass_source", 0.0))
    p.area_alpha = float(d.get("area_alpha", 0.0))
    p.mass_phi_gamma = float(d.get("mass_phi_gamma", 0.0))
    p.pressure_ring = int(bool(d.get("pressure_ring", False)))
    p.interp_half_force = int(bool(d.get("interp_half_force", False)))
    p.no_flux_zeroth = int(bool(d.get("no_flux_zeroth", False)))
    p.no_flux_bounce = int(bool(d.get("no_flux_bounce", False)))
    return p


def threads() -> int:
    """OpenMP threads the oracle's lattice loops run on (1 without OpenMP)."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Run the oracle's lattice loops on n OpenMP threads."""
    lib().orc_set_threads(int(n))


def delta1d(kernel: int, r: float) -> float:
    return lib().orc_delta1d(kernel, float(r))


def equilibrium9(rho, ux, uy):
    out = np.zeros(9)
    lib().orc_equilibrium9(rho, ux, uy, out)
    return out


def equilibrium5(phi, ux, uy):
    out = np.zeros(5)
    lib().orc_equilibrium5(phi, ux, uy, out)
    return out


def forces(params: dict, offsets, xy, l0, A0):
    p = make_params(params)
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    F = np.zeros_like(xy)
    area = np.zeros(len(offsets) - 1)
    lib().orc_forces(C.byref(p), len(offsets) - 1, np.ascontiguousarray(offsets, np.int32), xy,
                     np.ascontiguousarray(l0, np.float64), np.ascontiguousarray(A0, np.float64), F, area)
    return F, area


def spread(params: dict, xy, F):
    p = make_params(params)
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(-1, 2)
    ex = np.zeros((p.ny, p.nx)); ey = np.zeros((p.ny, p.nx))
    lib().orc_spread(C.byref(p), xy.shape[0], xy, F, ex, ey)
    return ex, ey


def interp(params: dict, xy, ux, uy):
    p = make_params(params)
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    U = np.zeros_like(xy)
    lib().orc_interp(C.byref(p), xy.shape[0], xy, np.ascontiguousarray(ux, np.float64),
                     np.ascontiguousarray(uy, np.float64), U)
    return U


def raster(params: dict, offsets, xy):
    p = make_params(params)
    m = np.zeros((p.ny, p.nx), dtype=np.int32)
    ov = lib().orc_raster(C.byref(p), len(offsets) - 1, np.ascontiguousarray(offsets, np.int32),
                          np.ascontiguousarray(xy, np.float64).reshape(-1, 2), m)
    return m, int(ov)


def link_crossings(params: dict, offsets, xy):
    """[4, ny, nx] wall distances of the links crossed by membrane edges, for the populations
    arriving in +x, +y, -x, -y; +inf where no edge crosses the link."""
    p = make_params(params)
    q = np.zeros((4, p.ny, p.nx))
    lib().orc_link_crossings(C.byref(p), len(offsets) - 1, np.ascontiguousarray(offsets, np.int32),
                             np.ascontiguousarray(xy, np.float64).reshape(-1, 2), q)
    return q


class Sim:
    """One oracle simulation (FP64, CPU)."""

    def __init__(self, params: dict, interp_new_u: bool = False, wall_u_top: float = 0.0):
        self.params = params
        self.p = make_params(params, interp_new_u, wall_u_top)
        self.L = lib()
        self.h = self.L.orc_create(C.byref(self.p))
        self.n_nodes = 0
        self.nx, self.ny, self.S = self.p.nx, self.p.ny, self.p.n_species

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None

    def set_cells(self, offsets, xy, rest_len=None, rest_area=None):
        off = np.ascontiguousarray(offsets, np.int32)
        xy = np.ascontiguousarray(xy, np.float64).reshape(-1, 2)
        rl = None if rest_len is None else np.ascontiguousarray(rest_len, np.float64)
        ra = None if rest_area is None else np.ascontiguousarray(rest_area, np.float64)
        self.L.orc_set_cells(self.h, len(off) - 1, off, xy, _ptr(rl), _ptr(ra))
        self.n_nodes = xy.shape[0]
        self.n_cells = len(off) - 1

    def set_fields(self, rho=None, u=None, phi=None):
        r = None if rho is None else np.ascontiguousarray(rho, np.float64)
        uu = None if u is None else np.ascontiguousarray(u, np.float64)
        ph = None if phi is None else np.ascontiguousarray(phi, np.float64)
        self.L.orc_set_fields(self.h, _ptr(r), _ptr(uu), _ptr(ph))

    def step(self, n: int = 1):
        self.L.orc_step(self.h, int(n))

    def set_source_cells(self, src=None):
        """Cells whose interior the source/decay law treats as a source (None: all)."""
        a = None if src is None else np.ascontiguousarray(np.asarray(src) != 0, np.uint8)
        self.L.orc_set_source_cells(self.h, _ptr(a))

    def set_node_sources(self, rate=None):
        """[ny, nx] mass added per node and step (point sources), None: none."""
        a = None if rate is None else np.ascontiguousarray(rate, np.float64).reshape(self.ny, self.nx)
        self.L.orc_set_node_sources(self.h, _ptr(a))

    def set_pressure_nodes(self, flags=None):
        """[ny, nx] nodes held at rho0 (pressure points), None: none."""
        a = None if flags is None else np.ascontiguousarray(np.asarray(flags) != 0, np.uint8).reshape(self.ny, self.nx)
        self.L.orc_set_pressure_nodes(self.h, _ptr(a))

    def source_map(self) -> np.ndarray:
        """[ny, nx] int32, nonzero exactly inside a source cell (the source/decay law's map)."""
        m = np.zeros((self.ny, self.nx), np.int32)
        self.L.orc_source_map(self.h, _ptr(m))
        return m

    def ade_step(self, n: int = 1) -> np.ndarray:
        """n ADE-only iterations (u = 0, frozen fluid and membranes); returns the relative
        change ||phi^{k+1} - phi^k|| / ||phi^{k+1}|| per iteration and species, [n][S]."""
        ch = np.zeros((max(int(n), 1), max(self.S, 1)))
        self.L.orc_ade_step(self.h, int(n), _ptr(ch))
        return ch[:int(n), :self.S]

    def ade_steady(self, tol: float, max_iters: int, chunk: int = 256):
        """Iterate until every species' relative change is at most tol; returns (iterations,
        change history [k][S]).  iterations is 0 when max_iters pass without convergence."""
        hist = []
        done = 0
        while done < max_iters:
            n = min(chunk, max_iters - done)
            ch = self.ade_step(n)
            for k in range(n):
                hist.append(ch[k])
                if np.all(ch[k] <= tol):
                    # the state has advanced past the converged iteration: report, stop
                    return done + k + 1, np.array(hist)
            done += n
        return 0, np.array(hist)

    def get_fields(self):
        ny, nx, S = self.ny, self.nx, self.S
        rho = np.zeros((ny, nx)); u = np.zeros((2, ny, nx)); phi = np.zeros((max(S, 1), ny, nx))
        X = np.zeros((max(self.n_nodes, 1), 2)); m = np.zeros((ny, nx), np.int32)
        self.L.orc_get_fields(self.h, _ptr(rho), _ptr(u), _ptr(phi), _ptr(X), _ptr(m))
        return dict(rho=rho, u=u, phi=phi[:S], xy=X[:self.n_nodes], mask=m)

    def populations(self):
        f = np.zeros((9, self.ny, self.nx)); g = np.zeros((max(self.S, 1) * 5, self.ny, self.nx))
        self.L.orc_get_populations(self.h, _ptr(f), _ptr(g))
        return f, g[:5 * self.S].reshape(self.S, 5, self.ny, self.nx)

    def set_populations(self, f=None, g=None):
        ff = None if f is None else np.ascontiguousarray(f, np.float64)
        gg = None if g is None else np.ascontiguousarray(g, np.float64)
        self.L.orc_set_populations(self.h, _ptr(ff), _ptr(gg))

    def prev_moments(self):
        """(phi [S, ny, nx], u [2, ny, nx]) of the previous step, read by the no-flux
        replacement."""
        phi = np.zeros((max(self.S, 1), self.ny, self.nx)); u = np.zeros((2, self.ny, self.nx))
        self.L.orc_get_prev_moments(self.h, _ptr(phi), _ptr(u))
        return phi[:self.S], u

    def set_prev_moments(self, phi=None, u=None):
        ph = None if phi is None else np.ascontiguousarray(phi, np.float64)
        uu = None if u is None else np.ascontiguousarray(u, np.float64)
        self.L.orc_set_prev_moments(self.h, _ptr(ph), _ptr(uu))

    def no_flux_values(self, s: int = 0):
        """[4, ny, nx] populations the first-order no-flux condition gives the current state in
        directions +x, +y, -x, -y (NaN where no population is missing)."""
        out = np.zeros((4, self.ny, self.nx))
        self.L.orc_no_flux_values(self.h, int(s), out)
        return out

    def last_spread(self):
        ex = np.zeros((self.ny, self.nx)); ey = np.zeros((self.ny, self.nx))
        self.L.orc_get_last_spread(self.h, ex, ey)
        return ex, ey

    def forces(self):
        F = np.zeros((self.n_nodes, 2)); A = np.zeros(max(self.n_cells, 1))
        self.L.orc_get_forces(self.h, F, A)
        return F, A[:self.n_cells]

    def invariants(self):
        out = np.zeros(3 + self.S)
        self.L.orc_invariants(self.h, out)
        return out


def from_workload(w, **kw) -> Sim:
    """Oracle simulation initialised from a ``workloads.Workload``."""
    s = Sim(w.params_dict(), **kw)
    if w.n_cells:
        s.set_cells(w.offsets, w.xy, w.rest_len, w.rest_area)
        if getattr(w, "source_cells", None) is not None:
            s.set_source_cells(w.source_cells)
    if getattr(w, "node_sources", None) is not None:
        s.set_node_sources(w.node_sources)
    if getattr(w, "pressure_nodes", None) is not None:
        s.set_pressure_nodes(w.pressure_nodes)
    if w.rho_init is not None or w.u_init is not None or w.phi_init is not None:
        s.set_fields(w.rho_init, w.u_init, w.phi_init)
    return s
