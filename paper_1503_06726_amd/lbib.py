"""Thin ctypes binding of ``liblbib.so`` (C ABI in ``include/lbib.h``).

Argument marshalling only: every step of the coupled update runs in the library's HIP
kernels.  There is no fallback: if the library is not built, or no GPU is usable, the
calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbib.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENUMERIC = 0, -1, -2, -3, -4, -5
PERIODIC, WALLS = 0, 1
DELTA_COS4, DELTA_PESKIN4 = 0, 1
REACT_NONE, REACT_SOURCE_DECAY, REACT_SCHNAKENBERG = 0, 1, 2
STORAGE_FP32, STORAGE_FP16, STORAGE_BF16 = 0, 1, 2
SPECIES_NO_FLUX = 1
K_LATTICE, K_MEMBRANE, K_LISTS = range(3)
KERNEL_NAMES = ["lattice", "membrane", "lists"]

# every entry point declared in include/lbib.h
EXPORTS = ["lbib_validate_params", "lbib_validate_cells", "lbib_create", "lbib_set_cells",
           "lbib_set_fields", "lbib_step", "lbib_get_fields", "lbib_get_forces", "lbib_get_spread",
           "lbib_reduce", "lbib_sync", "lbib_set_timing", "lbib_get_timing", "lbib_device_bytes",
           "lbib_last_error", "lbib_status_string", "lbib_version", "lbib_destroy",
           "lbib_set_source_cells", "lbib_ade_steady", "lbib_ade_batch",
           "lbib_net_create", "lbib_net_param_count", "lbib_net_set_params", "lbib_net_get_params",
           "lbib_net_predict", "lbib_net_loss_grad", "lbib_net_train_step", "lbib_net_destroy",
           "lbib_batch_create", "lbib_batch_step", "lbib_batch_sync", "lbib_batch_get_tile",
           "lbib_batch_set_tile", "lbib_batch_get_groups", "lbib_batch_set_groups", "lbib_batch_autotune",
           "lbib_batch_last_error", "lbib_batch_destroy",
           "lbib_workspace_size", "lbib_bind_workspace", "lbib_workspace_nodes", "lbib_reduce_device",
           "lbib_get_monitor", "lbib_state_size", "lbib_save_state", "lbib_load_state",
           "lbib_set_node_sources", "lbib_set_pressure_nodes"]


class Species(C.Structure):
    _fields_ = [("D", C.c_double), ("phi_ref", C.c_double), ("reaction", C.c_int32),
                ("flags", C.c_int32), ("c", C.c_double * 4)]


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("bc_y", C.c_int32), ("delta_kernel", C.c_int32),
                ("tau", C.c_double), ("rho0", C.c_double), ("body_accel", C.c_double * 2),
                ("k_spring", C.c_double), ("phi_m", C.c_double), ("kappa_area", C.c_double),
                ("n_species", C.c_int32), ("storage", C.c_int32), ("species", Species * 2),
                ("mass_source", C.c_double), ("area_alpha", C.c_double), ("mass_phi_gamma", C.c_double),
                ("pressure_ring", C.c_int32), ("interp_half_force", C.c_int32),
                ("no_flux_zeroth", C.c_int32), ("no_flux_bounce", C.c_int32), ("monitor_every", C.c_int32),
                ("reserved", C.c_int32)]


class LbibError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str = ""):
        self.status = status
        super().__init__(f"{where}: {_status_name(status)} {msg}".strip())


_lib = None


def _status_name(s: int) -> str:
    return {0: "LBIB_OK", -1: "LBIB_EINVAL", -2: "LBIB_ENOMEM", -3: "LBIB_EDEVICE",
            -4: "LBIB_ESTATE", -5: "LBIB_ENUMERIC"}.get(int(s), f"status {s}")


def lib():
    """Load ``liblbib.so`` (built in-tree by ``paper_1503_06726_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(python -m paper_1503_06726_amd.build)")
    # PyTorch ships its own copy of the HIP runtime under the same soname as the system one the
    # library links; loading torch first makes the library bind to that copy, so that a process
    # using both has one runtime (loaded the other way round, torch's device initialisation
    # fails after the library's)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.c_void_p, C.c_void_p
    P = C.POINTER(Params)
    st = C.c_int
    L.lbib_validate_params.restype = st
    L.lbib_validate_params.argtypes = [P, C.c_char_p, C.c_size_t]
    L.lbib_validate_cells.restype = st
    L.lbib_validate_cells.argtypes = [P, C.c_int32, ip, dp, dp, dp, C.c_char_p, C.c_size_t]
    L.lbib_create.restype = st
    L.lbib_create.argtypes = [P, vp, C.POINTER(C.c_void_p)]
    L.lbib_set_cells.restype = st
    L.lbib_set_cells.argtypes = [vp, C.c_int32, ip, dp, dp, dp]
    L.lbib_set_fields.restype = st
    L.lbib_set_fields.argtypes = [vp, dp, dp, dp]
    L.lbib_step.restype = st
    L.lbib_step.argtypes = [vp, C.c_int32]
    L.lbib_get_fields.restype = st
    L.lbib_get_fields.argtypes = [vp, dp, dp, dp, dp, ip]
    L.lbib_get_forces.restype = st
    L.lbib_get_forces.argtypes = [vp, dp, dp]
    L.lbib_get_spread.restype = st
    L.lbib_get_spread.argtypes = [vp, dp]
    L.lbib_reduce.restype = st
    L.lbib_reduce.argtypes = [vp, dp]
    L.lbib_state_size.restype = st
    L.lbib_state_size.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.lbib_save_state.restype = st
    L.lbib_save_state.argtypes = [vp, vp, C.c_size_t]
    L.lbib_load_state.restype = st
    L.lbib_load_state.argtypes = [vp, vp, C.c_size_t]
    L.lbib_get_monitor.restype = st
    L.lbib_get_monitor.argtypes = [vp, dp, C.POINTER(C.c_int64)]
    L.lbib_reduce_device.restype = st
    L.lbib_reduce_device.argtypes = [vp, vp]
    L.lbib_sync.restype = st
    L.lbib_sync.argtypes = [vp]
    L.lbib_set_timing.restype = st
    L.lbib_set_timing.argtypes = [vp, C.c_int32]
    L.lbib_get_timing.restype = st
    L.lbib_get_timing.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.lbib_device_bytes.restype = st
    L.lbib_device_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.lbib_last_error.restype = C.c_char_p
    L.lbib_last_error.argtypes = [vp]
    L.lbib_status_string.restype = C.c_char_p
    L.lbib_status_string.argtypes = [C.c_int]
    L.lbib_version.restype = C.c_int32
    L.lbib_version.argtypes = []
    L.lbib_destroy.restype = None
    L.lbib_destroy.argtypes = [vp]
    L.lbib_workspace_size.restype = st
    L.lbib_workspace_size.argtypes = [P, C.c_int64, C.POINTER(C.c_size_t)]
    L.lbib_bind_workspace.restype = st
    L.lbib_bind_workspace.argtypes = [vp, vp, C.c_size_t]
    L.lbib_workspace_nodes.restype = st
    L.lbib_workspace_nodes.argtypes = [vp, C.POINTER(C.c_int64)]
    L.lbib_set_source_cells.restype = st
    L.lbib_set_source_cells.argtypes = [vp, vp]
    L.lbib_set_node_sources.restype = st
    L.lbib_set_node_sources.argtypes = [vp, vp]
    L.lbib_set_pressure_nodes.restype = st
    L.lbib_set_pressure_nodes.argtypes = [vp, vp]
    L.lbib_net_create.restype = st
    L.lbib_net_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, vp, C.POINTER(C.c_void_p)]
    L.lbib_net_param_count.restype = st
    L.lbib_net_param_count.argtypes = [vp, C.POINTER(C.c_int64)]
    L.lbib_net_set_params.restype = st
    L.lbib_net_set_params.argtypes = [vp, vp]
    L.lbib_net_get_params.restype = st
    L.lbib_net_get_params.argtypes = [vp, vp]
    L.lbib_net_predict.restype = st
    L.lbib_net_predict.argtypes = [vp, vp, C.c_int32, vp]
    L.lbib_net_loss_grad.restype = st
    L.lbib_net_loss_grad.argtypes = [vp, vp, vp, C.c_int32, C.POINTER(C.c_double), vp]
    L.lbib_net_train_step.restype = st
    L.lbib_net_train_step.argtypes = [vp, vp, vp, C.c_int32, C.c_float, C.POINTER(C.c_double)]
    L.lbib_net_destroy.restype = None
    L.lbib_net_destroy.argtypes = [vp]
    L.lbib_ade_batch.restype = st
    L.lbib_ade_batch.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp, vp, vp, C.c_int32,
                                 C.c_double, C.c_int64, C.c_int32, vp, vp]
    L.lbib_ade_steady.restype = st
    L.lbib_ade_steady.argtypes = [vp, C.c_double, C.c_int64, C.c_int32, C.POINTER(C.c_int64),
                                  C.POINTER(C.c_double)]
    L.lbib_batch_create.restype = st
    L.lbib_batch_create.argtypes = [C.POINTER(C.c_void_p), C.c_int32, vp, C.POINTER(C.c_void_p)]
    L.lbib_batch_step.restype = st
    L.lbib_batch_step.argtypes = [vp, C.c_int32]
    L.lbib_batch_sync.restype = st
    L.lbib_batch_sync.argtypes = [vp]
    L.lbib_batch_get_tile.restype = st
    L.lbib_batch_get_tile.argtypes = [vp, C.POINTER(C.c_int32)]
    L.lbib_batch_set_tile.restype = st
    L.lbib_batch_set_tile.argtypes = [vp, C.c_int32]
    L.lbib_batch_get_groups.restype = st
    L.lbib_batch_get_groups.argtypes = [vp, C.POINTER(C.c_int32)]
    L.lbib_batch_set_groups.restype = st
    L.lbib_batch_set_groups.argtypes = [vp, C.c_int32]
    L.lbib_batch_autotune.restype = st
    L.lbib_batch_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), vp]
    L.lbib_batch_last_error.restype = C.c_char_p
    L.lbib_batch_last_error.argtypes = [vp]
    L.lbib_batch_destroy.restype = None
    L.lbib_batch_destroy.argtypes = [vp]
    _lib = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_params(d: dict) -> Params:
    """lbib_params from a workload parameter dict (see ``workloads.Workload.params_dict``)."""
    p = Params()
    p.nx, p.ny, p.bc_y = int(d["nx"]), int(d["ny"]), int(d["bc_y"])
    p.delta_kernel = int(d.get("delta_kernel", DELTA_COS4))
    p.tau, p.rho0 = float(d["tau"]), float(d.get("rho0", 1.0))
    b = d.get("body_accel", (0.0, 0.0))
    p.body_accel[0], p.body_accel[1] = float(b[0]), float(b[1])
    p.k_spring = float(d.get("k_spring", 0.0))
    p.phi_m = float(d.get("phi_m", 0.0))
    p.kappa_area = float(d.get("kappa_area", 0.0))
    sp = d.get("species", [])
    p.n_species = len(sp)
    p.storage = int(d.get("storage", STORAGE_FP32))
    for s, spc in enumerate(sp[:2]):        # more than two is left to the validator to reject
        p.species[s].D = float(spc["D"])
        p.species[s].phi_ref = float(spc.get("phi_ref", 0.0))
        p.species[s].reaction = int(spc.get("reaction", REACT_NONE))
        p.species[s].flags = SPECIES_NO_FLUX if spc.get("no_flux", False) else 0
        for k, v in enumerate(spc.get("c", (0.0, 0.0, 0.0, 0.0))):
            p.species[s].c[k] = float(v)
    p.mass_source = float(d.get("mass_source", 0.0))
    p.area_alpha = float(d.get("area_alpha", 0.0))
    p.mass_phi_gamma = float(d.get("mass_phi_gamma", 0.0))
    p.pressure_ring = int(bool(d.get("pressure_ring", False)))
    p.interp_half_force = int(bool(d.get("interp_half_force", False)))
    p.no_flux_zeroth = int(bool(d.get("no_flux_zeroth", False)))
    p.no_flux_bounce = int(bool(d.get("no_flux_bounce", False)))
    p.monitor_every = int(d.get("monitor_every", 0))
    return p


def validate_params(d: dict):
    msg = C.create_string_buffer(256)
    p = make_params(d)
    s = lib().lbib_validate_params(C.byref(p), msg, 256)
    return s, msg.value.decode()


def validate_cells(d: dict, offsets, xy, rest_len=None, rest_area=None):
    msg = C.create_string_buffer(256)
    p = make_params(d)
    off = np.ascontiguousarray(offsets, np.int32)
    xy = np.ascontiguousarray(xy, np.float64).reshape(-1, 2)
    rl = None if rest_len is None else np.ascontiguousarray(rest_len, np.float64)
    ra = None if rest_area is None else np.ascontiguousarray(rest_area, np.float64)
    s = lib().lbib_validate_cells(C.byref(p), len(off) - 1, _p(off), _p(xy), _p(rl), _p(ra), msg, 256)
    return s, msg.value.decode()


def workspace_size(params: dict, n_nodes: int) -> int:
    """Bytes of a workspace for ``params`` and at most ``n_nodes`` membrane nodes
    (lbib_workspace_size)."""
    p = make_params(params)
    b = C.c_size_t()
    s = lib().lbib_workspace_size(C.byref(p), int(n_nodes), C.byref(b))
    if s != OK:
        raise LbibError(s, "lbib_workspace_size")
    return int(b.value)


class Simulation:
    """One lbib context: ``create`` on construction, ``destroy`` on ``close``.

    ``stream`` is a ``hipStream_t`` handle as an int (for instance
    ``torch.cuda.current_stream().cuda_stream``); None lets the library own a stream."""

    def __init__(self, params: dict, stream: int | None = None):
        self.L = lib()
        self.params = params
        self._p = make_params(params)
        h = C.c_void_p()
        s = self.L.lbib_create(C.byref(self._p), C.c_void_p(stream) if stream else None, C.byref(h))
        if s != OK:
            raise LbibError(s, "lbib_create")
        self.h = h
        self.nx, self.ny, self.S = self._p.nx, self._p.ny, self._p.n_species
        self.n_nodes = 0
        self.n_cells = 0

    # -- lifetime --------------------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.L.lbib_destroy(self.h)
            self.h = None
        self._ws_owner = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, s, where):
        if s != OK:
            raise LbibError(s, where, (self.L.lbib_last_error(self.h) or b"").decode())

    # -- calls of the C ABI -------------------------------------------------------------------
    def set_cells(self, offsets, xy, rest_len=None, rest_area=None):
        off = np.ascontiguousarray(offsets, np.int32)
        xy = np.ascontiguousarray(xy, np.float64).reshape(-1, 2)
        rl = None if rest_len is None else np.ascontiguousarray(rest_len, np.float64)
        ra = None if rest_area is None else np.ascontiguousarray(rest_area, np.float64)
        self._check(self.L.lbib_set_cells(self.h, len(off) - 1, _p(off), _p(xy), _p(rl), _p(ra)),
                    "lbib_set_cells")
        self.n_nodes = xy.shape[0]
        self.n_cells = len(off) - 1

    def set_fields(self, rho=None, u=None, phi=None):
        r = None if rho is None else np.ascontiguousarray(rho, np.float64)
        uu = None if u is None else np.ascontiguousarray(u, np.float64)
        ph = None if phi is None else np.ascontiguousarray(phi, np.float64)
        self._check(self.L.lbib_set_fields(self.h, _p(r), _p(uu), _p(ph)), "lbib_set_fields")

    def step(self, n: int = 1):
        self._check(self.L.lbib_step(self.h, int(n)), "lbib_step")

    def get_fields(self, rho=True, u=True, phi=True, xy=True, mask=True):
        ny, nx, S = self.ny, self.nx, self.S
        out = {}
        r = np.empty((ny, nx)) if rho else None
        uu = np.empty((2, ny, nx)) if u else None
        ph = np.empty((S, ny, nx)) if (phi and S) else None
        X = np.empty((self.n_nodes, 2)) if (xy and self.n_nodes) else None
        m = np.empty((ny, nx), np.int32) if mask else None
        self._check(self.L.lbib_get_fields(self.h, _p(r), _p(uu), _p(ph), _p(X), _p(m)), "lbib_get_fields")
        out["rho"], out["u"] = r, uu
        out["phi"] = ph if ph is not None else np.zeros((0, ny, nx))
        out["xy"] = X if X is not None else np.zeros((0, 2))
        out["mask"] = m
        return out

    def get_forces(self):
        F = np.zeros((max(self.n_nodes, 1), 2))
        A = np.zeros(max(self.n_cells, 1))
        self._check(self.L.lbib_get_forces(self.h, _p(F), _p(A)), "lbib_get_forces")
        return F[:self.n_nodes], A[:self.n_cells]

    def get_spread(self):
        e = np.empty((2, self.ny, self.nx))
        self._check(self.L.lbib_get_spread(self.h, _p(e)), "lbib_get_spread")
        return e

    def reduce(self):
        out = np.zeros(3 + self.S)
        self._check(self.L.lbib_reduce(self.h, _p(out)), "lbib_reduce")
        return out

    def save_state(self) -> bytes:
        """The solver state (lbib_save_state) as bytes, loadable with ``load_state``."""
        n = C.c_size_t()
        self._check(self.L.lbib_state_size(self.h, C.byref(n)), "lbib_state_size")
        buf = C.create_string_buffer(int(n.value))
        self._check(self.L.lbib_save_state(self.h, buf, n), "lbib_save_state")
        return buf.raw

    def load_state(self, state: bytes):
        """Continue from a state saved by ``save_state`` (lbib_load_state)."""
        buf = C.create_string_buffer(state, len(state))
        self._check(self.L.lbib_load_state(self.h, buf, len(state)), "lbib_load_state")
        # the header: magic, version and source flag, the parameters, then the cell and node counts
        n_cells, n_nodes = np.frombuffer(state, np.int64, 2, 16 + C.sizeof(Params))
        self.n_cells, self.n_nodes = int(n_cells), int(n_nodes)

    def monitor(self):
        """(sums, times taken) of the FP64 monitor (lbib_get_monitor); sums is None before the
        monitor has taken any."""
        out = np.zeros(3 + self.S)
        n = C.c_int64(0)
        self._check(self.L.lbib_get_monitor(self.h, _p(out), C.byref(n)), "lbib_get_monitor")
        return (out if n.value > 0 else None), int(n.value)

    def reduce_device(self, out_ptr: int):
        """Enqueue the sums of ``reduce`` into device memory at ``out_ptr`` (3 + S doubles,
        for instance a torch tensor's ``data_ptr()``) without allocating or synchronising
        (lbib_reduce_device)."""
        self._check(self.L.lbib_reduce_device(self.h, C.c_void_p(int(out_ptr))), "lbib_reduce_device")

    def set_source_cells(self, src=None):
        """Cells whose interior the source/decay law treats as a source (None: every cell)."""
        a = None if src is None else np.ascontiguousarray(np.asarray(src) != 0, np.uint8).ravel()
        if a is not None and self.n_cells and a.size != self.n_cells:   # (no cells: LBIB_ESTATE)
            raise ValueError(f"{self.n_cells} source flags are needed, not {a.size}")
        self._check(self.L.lbib_set_source_cells(self.h, _p(a)), "lbib_set_source_cells")

    def set_node_sources(self, rate=None):
        """Mass per node and step at every lattice node, [ny, nx] (point sources), None: none
        (lbib_set_node_sources)."""
        a = None if rate is None else np.ascontiguousarray(rate, np.float64)
        if a is not None and a.shape != (self.ny, self.nx):
            raise ValueError(f"node sources must have shape {(self.ny, self.nx)}, not {a.shape}")
        self._check(self.L.lbib_set_node_sources(self.h, _p(a)), "lbib_set_node_sources")

    def set_pressure_nodes(self, flags=None):
        """Lattice points held at rho0, [ny, nx] flags, None: none (lbib_set_pressure_nodes)."""
        a = None if flags is None else np.ascontiguousarray(np.asarray(flags) != 0, np.uint8)
        if a is not None and a.shape != (self.ny, self.nx):
            raise ValueError(f"pressure points must have shape {(self.ny, self.nx)}, not {a.shape}")
        self._check(self.L.lbib_set_pressure_nodes(self.h, _p(a)), "lbib_set_pressure_nodes")

    def ade_steady(self, tol: float, max_iters: int, fp64: bool = True):
        """ADE-only iterations (u = 0, frozen fluid and membranes) until the relative change of
        every species is at most tol; returns (iterations, last relative change)."""
        it, ch = C.c_int64(0), C.c_double(0.0)
        self._check(self.L.lbib_ade_steady(self.h, float(tol), int(max_iters), 1 if fp64 else 0,
                                           C.byref(it), C.byref(ch)), "lbib_ade_steady")
        return int(it.value), float(ch.value)

    def sync(self):
        self._check(self.L.lbib_sync(self.h), "lbib_sync")

    def set_timing(self, enable: bool):
        self._check(self.L.lbib_set_timing(self.h, int(bool(enable))), "lbib_set_timing")

    def get_timing(self, kernel: int):
        ms = C.c_double()
        n = C.c_int64()
        self._check(self.L.lbib_get_timing(self.h, int(kernel), C.byref(ms), C.byref(n)), "lbib_get_timing")
        return ms.value, n.value

    def bind_workspace(self, ptr: int | None, nbytes: int = 0, owner=None):
        """Move the state into caller device memory at ``ptr`` (lbib_bind_workspace); None moves
        it back into library memory.  ``owner`` (a torch tensor, say) is kept alive while bound."""
        self._check(self.L.lbib_bind_workspace(self.h, C.c_void_p(ptr) if ptr else None,
                                               int(nbytes) if ptr else 0), "lbib_bind_workspace")
        self._ws_owner = owner if ptr else None

    def workspace_nodes(self) -> int:
        """Node capacity of the bound workspace, -1 when none is bound."""
        n = C.c_int64()
        self._check(self.L.lbib_workspace_nodes(self.h, C.byref(n)), "lbib_workspace_nodes")
        return int(n.value)

    def device_bytes(self) -> int:
        b = C.c_size_t()
        self._check(self.L.lbib_device_bytes(self.h, C.byref(b)), "lbib_device_bytes")
        return int(b.value)


def ade_batch(nx: int, ny: int, bc_y: int, source, D, sigma, decay, phi0=None, tol: float = 1e-6,
              max_iters: int = 1_000_000, fp64: bool = True, stream: int | None = None):
    """Batched ADE-only steady states (see lbib_ade_batch); source [B, ny, nx] (nonzero inside a
    source cell), D / sigma / decay [B], phi0 [B, ny, nx] or None (zero start).  Returns
    (iterations [B] int64, final phi [B, ny, nx])."""
    L = lib()
    src = np.ascontiguousarray(np.asarray(source) != 0, np.uint8)
    B = src.shape[0]
    Dv = np.ascontiguousarray(D, np.float64).reshape(B)
    sv = np.ascontiguousarray(sigma, np.float64).reshape(B)
    dv = np.ascontiguousarray(decay, np.float64).reshape(B)
    phi = (np.zeros((B, ny, nx)) if phi0 is None else np.array(phi0, np.float64).reshape(B, ny, nx))
    phi = np.ascontiguousarray(phi)
    its = np.zeros(B, np.int64)
    s = L.lbib_ade_batch(int(nx), int(ny), int(bc_y), int(B), _p(src), _p(Dv), _p(sv), _p(dv), _p(phi),
                         1 if phi0 is None else 0, float(tol), int(max_iters), 1 if fp64 else 0, _p(its),
                         C.c_void_p(stream) if stream else None)
    if s != OK:
        raise LbibError(s, "lbib_ade_batch")
    return its, phi


class Batch:
    """Many Simulations stepped together (lbib_batch_*).  The batch holds references to its
    simulations, which stay usable for reads; ``close`` releases them."""

    def __init__(self, sims, stream: int | None = None):
        self.L = lib()
        self.h = None
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s.h.value for s in self.sims])
        hh = C.c_void_p()
        s = self.L.lbib_batch_create(arr, len(self.sims), C.c_void_p(stream) if stream else None, C.byref(hh))
        if s != OK:
            msgs = [(self.L.lbib_last_error(x.h) or b"").decode() for x in self.sims if x.h]
            raise LbibError(s, "lbib_batch_create", next((m for m in msgs if m), ""))
        self.h = hh
        self.updates_per_step = sum(x.nx * x.ny for x in self.sims)

    def close(self):
        if self.h:
            self.L.lbib_batch_destroy(self.h)
            self.h = None
        self.sims = []

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, s, where):
        if s != OK:
            raise LbibError(s, where, (self.L.lbib_batch_last_error(self.h) or b"").decode())

    def step(self, n: int = 1):
        self._check(self.L.lbib_batch_step(self.h, int(n)), "lbib_batch_step")

    def sync(self):
        self._check(self.L.lbib_batch_sync(self.h), "lbib_batch_sync")

    @property
    def tile(self) -> int:
        r = C.c_int32(0)
        self._check(self.L.lbib_batch_get_tile(self.h, C.byref(r)), "lbib_batch_get_tile")
        return int(r.value)

    def set_tile(self, rows: int):
        self._check(self.L.lbib_batch_set_tile(self.h, int(rows)), "lbib_batch_set_tile")

    @property
    def groups(self) -> int:
        g = C.c_int32(0)
        self._check(self.L.lbib_batch_get_groups(self.h, C.byref(g)), "lbib_batch_get_groups")
        return int(g.value)

    def set_groups(self, groups: int):
        self._check(self.L.lbib_batch_set_groups(self.h, int(groups)), "lbib_batch_set_groups")

    def autotune(self, periods: int = 2):
        """(chosen tile height, chosen groups, {(groups, height): ms per step} of the
        admissible configurations)."""
        r, g = C.c_int32(0), C.c_int32(0)
        ms = np.zeros(6)
        self._check(self.L.lbib_batch_autotune(self.h, int(periods), C.byref(r), C.byref(g), _p(ms)),
                    "lbib_batch_autotune")
        keys = [(1, 4), (1, 8), (1, 16), (2, 4), (2, 8), (2, 16)]
        return int(r.value), int(g.value), {k: float(v) for k, v in zip(keys, ms) if v >= 0}


class Net:
    """The steady-state surrogate network (lbib_net_*).  Tensors passed to predict / loss_grad /
    train_step are device addresses (e.g. ``torch.Tensor.data_ptr()`` of CUDA tensors):
    inputs [B, h, w, 8] float32, targets and outputs [B, h, w] float32."""

    def __init__(self, h: int, w: int, max_batch: int, stream: int | None = None):
        self.L = lib()
        self.h = None
        hh = C.c_void_p()
        s = self.L.lbib_net_create(int(h), int(w), int(max_batch), C.c_void_p(stream) if stream else None,
                                   C.byref(hh))
        if s != OK:
            raise LbibError(s, "lbib_net_create")
        self.h = hh
        n = C.c_int64(0)
        self.L.lbib_net_param_count(self.h, C.byref(n))
        self.n_params = int(n.value)

    def close(self):
        if self.h:
            self.L.lbib_net_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _check(self, s, where):
        if s != OK:
            raise LbibError(s, where)

    def set_params(self, p):
        a = np.ascontiguousarray(p, np.float32)
        assert a.size == self.n_params
        self._check(self.L.lbib_net_set_params(self.h, _p(a)), "lbib_net_set_params")

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.n_params, np.float32)
        self._check(self.L.lbib_net_get_params(self.h, _p(a)), "lbib_net_get_params")
        return a

    def predict(self, inputs_ptr: int, B: int, out_ptr: int):
        self._check(self.L.lbib_net_predict(self.h, C.c_void_p(inputs_ptr), int(B), C.c_void_p(out_ptr)),
                    "lbib_net_predict")

    def loss_grad(self, inputs_ptr: int, targets_ptr: int, B: int, want_grad: bool = True):
        loss = C.c_double(0.0)
        g = np.zeros(self.n_params, np.float32) if want_grad else None
        self._check(self.L.lbib_net_loss_grad(self.h, C.c_void_p(inputs_ptr), C.c_void_p(targets_ptr), int(B),
                                              C.byref(loss), _p(g)), "lbib_net_loss_grad")
        return float(loss.value), g

    def train_step(self, inputs_ptr: int, targets_ptr: int, B: int, lr: float) -> float:
        loss = C.c_double(0.0)
        self._check(self.L.lbib_net_train_step(self.h, C.c_void_p(inputs_ptr), C.c_void_p(targets_ptr), int(B),
                                               float(lr), C.byref(loss)), "lbib_net_train_step")
        return float(loss.value)


def from_workload(w, stream: int | None = None, storage: int | None = None) -> Simulation:
    """A Simulation initialised from a ``workloads.Workload`` (``storage`` overrides the
    population storage, one of the STORAGE_* constants)."""
    d = w.params_dict()
    if storage is not None:
        d["storage"] = storage
    s = Simulation(d, stream=stream)
    if w.rho_init is not None or w.u_init is not None or w.phi_init is not None:
        s.set_fields(w.rho_init, w.u_init, w.phi_init)
    if w.n_cells:
        s.set_cells(w.offsets, w.xy, w.rest_len, w.rest_area)
        if getattr(w, "source_cells", None) is not None:
            s.set_source_cells(w.source_cells)
    if getattr(w, "node_sources", None) is not None:
        s.set_node_sources(w.node_sources)
    if getattr(w, "pressure_nodes", None) is not None:
        s.set_pressure_nodes(w.pressure_nodes)
    return s
