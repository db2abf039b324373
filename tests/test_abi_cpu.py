"""C ABI checks that need no GPU: the library loads and exports every declared entry
point, the ctypes mirrors match the C struct layout, and the validation rules hold."""
import ctypes as C
import math
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_1503_06726_amd import lbib
from paper_1503_06726_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbib.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbib_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = lbib.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(lbib.EXPORTS) == names
    assert L.lbib_version() == 1
    assert L.lbib_status_string(-5) == b"LBIB_ENUMERIC"


def test_ctypes_layout_matches_header():
    src = r"""
    #include <stdio.h>
    #include <stddef.h>
    #include "lbib.h"
    int main(void) {
      printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(lbib_params), sizeof(lbib_species),
             offsetof(lbib_params, tau), offsetof(lbib_params, body_accel), offsetof(lbib_params, kappa_area),
             offsetof(lbib_params, n_species), offsetof(lbib_params, species), offsetof(lbib_species, c),
             offsetof(lbib_species, reaction), offsetof(lbib_params, mass_source), offsetof(lbib_params, area_alpha),
             offsetof(lbib_params, pressure_ring), offsetof(lbib_params, interp_half_force),
             offsetof(lbib_params, no_flux_zeroth), offsetof(lbib_params, mass_phi_gamma),
             offsetof(lbib_params, no_flux_bounce));
      return 0; }
    """
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "l")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    P, S = lbib.Params, lbib.Species
    want = [C.sizeof(P), C.sizeof(S), P.tau.offset, P.body_accel.offset, P.kappa_area.offset,
            P.n_species.offset, P.species.offset, S.c.offset, S.reaction.offset, P.mass_source.offset,
            P.area_alpha.offset, P.pressure_ring.offset, P.interp_half_force.offset, P.no_flux_zeroth.offset,
            P.mass_phi_gamma.offset, P.no_flux_bounce.offset]
    assert vals == want


GOOD = W.tiny_cell().params_dict()


@pytest.mark.parametrize("change,frag", [
    (dict(tau=0.5), "tau"), (dict(tau=float("nan")), "tau"), (dict(nx=3), "lattice"),
    (dict(ny=40000), "lattice"), (dict(bc_y=2), "bc_y"), (dict(delta_kernel=7), "delta_kernel"),
    (dict(rho0=0.0), "rho0"), (dict(body_accel=(float("inf"), 0.0)), "body"), (dict(storage=3), "storage"),
])
def test_bad_params_rejected(change, frag):
    d = dict(GOOD, **change)
    s, msg = lbib.validate_params(d)
    assert s == lbib.EINVAL and frag in msg


def test_species_rules():
    assert lbib.validate_params(GOOD)[0] == lbib.OK
    d = dict(GOOD, species=[dict(D=-0.1)])
    assert lbib.validate_params(d)[0] == lbib.EINVAL
    sch = (0.1, 0.9, 0.01, 0.0)
    d = dict(GOOD, species=[dict(D=0.1, reaction=2, c=sch)])
    s, msg = lbib.validate_params(d)
    assert s == lbib.EINVAL and "Schnakenberg" in msg
    d = dict(GOOD, species=[dict(D=0.1, reaction=2, c=sch), dict(D=0.2, reaction=2, c=(0.1, 0.8, 0.01, 0))])
    assert lbib.validate_params(d)[0] == lbib.EINVAL
    d = dict(GOOD, species=[dict(D=0.1, reaction=2, c=sch), dict(D=0.2, reaction=2, c=sch)])
    assert lbib.validate_params(d)[0] == lbib.OK
    d = dict(GOOD, species=[dict(D=0.1), dict(D=0.1), dict(D=0.1)])
    assert lbib.validate_params(d)[0] == lbib.EINVAL


def _square(x0, y0, s, cw=False):
    P = np.array([[x0, y0], [x0 + s, y0], [x0 + s, y0 + s], [x0, y0 + s]], float)
    return P[::-1].copy() if cw else P


def test_cell_validation():
    w = W.tiny_cell()
    assert lbib.validate_cells(GOOD, w.offsets, w.xy, w.rest_len, w.rest_area)[0] == lbib.OK
    off = np.array([0, 4], np.int32)
    s, msg = lbib.validate_cells(GOOD, off, _square(10.5, 10.5, 5, cw=True))
    assert s == lbib.EINVAL and "counter-clockwise" in msg
    bad = _square(10.5, 10.5, 5)
    bad[2, 0] = float("nan")
    assert lbib.validate_cells(GOOD, off, bad)[0] == lbib.EINVAL
    assert lbib.validate_cells(GOOD, np.array([0, 2], np.int32), _square(10, 10, 3)[:2])[0] == lbib.EINVAL
    assert lbib.validate_cells(GOOD, np.array([1, 4], np.int32), _square(10, 10, 3))[0] == lbib.EINVAL
    walls = dict(GOOD, bc_y=W.WALLS)
    s, msg = lbib.validate_cells(walls, off, _square(10.5, 1.0, 5))
    assert s == lbib.EINVAL and "wall" in msg
    assert lbib.validate_cells(walls, off, _square(10.5, 2.0, 5))[0] == lbib.OK
    s, msg = lbib.validate_cells(walls, off, _square(10.5, 57.0, 5))
    assert s == lbib.EINVAL
    big = W.circle_cell(32, 32, 20, 4097, 0.0, None)
    assert lbib.validate_cells(dict(GOOD, nx=128, ny=128), big[0], big[1])[0] == lbib.EINVAL
    big = W.circle_cell(32, 32, 20, 4096, 0.0, None)
    assert lbib.validate_cells(dict(GOOD, nx=128, ny=128), big[0], big[1])[0] == lbib.OK
    assert lbib.validate_cells(GOOD, off, _square(2.5, 10.5, 60.0))[0] == lbib.EINVAL   # spans the lattice
    rl = np.array([1.0, -1.0, 1.0, 1.0])
    assert lbib.validate_cells(GOOD, off, _square(10.5, 10.5, 5), rest_len=rl)[0] == lbib.EINVAL
    assert lbib.validate_cells(GOOD, np.zeros(1, np.int32), np.zeros((0, 2)))[0] == lbib.OK


def test_create_rejects_bad_params_before_touching_a_device():
    p = lbib.make_params(dict(GOOD, tau=0.4))
    h = C.c_void_p()
    assert lbib.lib().lbib_create(C.byref(p), None, C.byref(h)) == lbib.EINVAL
    assert not h.value
    assert lbib.lib().lbib_step(None, 1) == lbib.ESTATE
    assert lbib.lib().lbib_last_error(None) == b""
    lbib.lib().lbib_destroy(None)


def test_workload_inputs_pass_validation():
    cases = [W.tiny_cell(), W.small_tissue(), W.small_tissue(bc_y=W.PERIODIC, n_species=2, seed=3), W.tissue(),
             W.large()] + [f() for f in W.PARITY_CASES.values()]
    for w in cases:
        assert lbib.validate_params(w.params_dict())[0] == lbib.OK
        s, msg = lbib.validate_cells(w.params_dict(), w.offsets, w.xy, w.rest_len, w.rest_area)
        assert s == lbib.OK, msg


# ---- lbib_workspace_size: a pure host function of the parameters and the node capacity ----
def _ws(d, n):
    return lbib.workspace_size(d, n)


def test_workspace_size_covers_the_state():
    """At least the bytes of the state it holds (two population buffers per lattice, the
    membrane arrays per node), monotone in the node capacity, and only padding beyond that."""
    d = dict(W.small_tissue(nx=200, ny=130, n_species=1).params_dict())
    nx, ny, S = d["nx"], d["ny"], len(d["species"])
    pops = 2 * (9 + 5 * S) * ny * (-(-nx // 64) * 64) * 4          # FP32, rows padded to 64 columns
    base = _ws(d, 0)
    assert base >= pops
    assert base - pops < (3 + S) * nx * ny * 8 + 256 * 1024         # + staging of the moments, partial sums, bits
    sizes = [_ws(d, n) for n in (0, 3, 300, 3000, 30000, 300000)]
    assert sizes == sorted(sizes)
    per_node = (sizes[-1] - sizes[-2]) / 270000
    # position 16 + rest length 8 + stencil origins 8 + shares 72 + count 1 + record 16 + lists 36,
    # cells (<= n/3) 8 + 8 + 4 + 1 bytes each; and the staging grows once n exceeds (3+S) nx ny
    assert 150 <= per_node <= 200, per_node


def test_workspace_size_follows_storage_and_species():
    d = dict(W.small_tissue(nx=200, ny=130, n_species=1).params_dict())
    h = dict(d, storage=lbib.STORAGE_FP16)
    n0 = dict(d, species=[])
    assert _ws(h, 100) < _ws(d, 100)
    assert _ws(n0, 100) < _ws(d, 100)
    # FP16 halves the population buffers, nothing else
    nxp = -(-d["nx"] // 64) * 64
    saved = _ws(d, 100) - _ws(h, 100)
    want = 2 * (9 + 5) * d["ny"] * nxp * 2
    assert abs(saved - want) <= 4 * 256


def test_workspace_size_rejects_bad_input():
    d = dict(GOOD)
    with pytest.raises(lbib.LbibError) as e:
        _ws(d, -1)
    assert e.value.status == lbib.EINVAL
    with pytest.raises(lbib.LbibError) as e:
        _ws(dict(d, tau=0.5), 10)
    assert e.value.status == lbib.EINVAL


def test_species_flags_validated():
    d = dict(W.no_flux_tissue().params_dict())
    assert lbib.validate_params(d)[0] == lbib.OK
    assert d["species"][0]["no_flux"] is True
    p = lbib.make_params(d)
    assert p.species[0].flags == lbib.SPECIES_NO_FLUX
    p.species[0].flags = 2
    buf = C.create_string_buffer(256)
    assert lbib.lib().lbib_validate_params(C.byref(p), buf, 256) == lbib.EINVAL
    assert b"flags" in buf.value


def test_mass_source_constants_validated():
    d = dict(W.mass_source_tissue().params_dict())
    assert lbib.validate_params(d)[0] == lbib.OK
    p = lbib.make_params(d)
    assert p.mass_source == d["mass_source"] and p.area_alpha == d["area_alpha"]
    for field, bad, word in (("area_alpha", -1e-6, b"area_alpha"), ("mass_source", float("nan"), b"mass-source"),
                             ("area_alpha", float("inf"), b"mass-source"), ("pressure_ring", 2, b"pressure_ring"),
                             ("interp_half_force", 2, b"interp_half_force"), ("no_flux_zeroth", -1, b"no_flux_zeroth"),
                             ("reserved", 1, b"reserved")):
        q = lbib.make_params(d)
        setattr(q, field, bad)
        buf = C.create_string_buffer(256)
        assert lbib.lib().lbib_validate_params(C.byref(q), buf, 256) == lbib.EINVAL
        assert word in buf.value


def test_concentration_source_validated():
    """Case III's source (mass_phi_gamma) must be finite and needs a species to read."""
    d = dict(W.growth_case(3, 0).params_dict())
    assert d["mass_phi_gamma"] == 1e-4 and lbib.validate_params(d)[0] == lbib.OK
    q = lbib.make_params(d)
    q.mass_phi_gamma = float("nan")
    buf = C.create_string_buffer(256)
    assert lbib.lib().lbib_validate_params(C.byref(q), buf, 256) == lbib.EINVAL
    assert b"mass-source" in buf.value
    q = lbib.make_params(dict(d, species=[]))
    assert q.mass_phi_gamma == 1e-4
    assert lbib.lib().lbib_validate_params(C.byref(q), buf, 256) == lbib.EINVAL
    assert b"mass_phi_gamma" in buf.value


def test_bounce_back_no_flux_validated():
    """The bounce-back no-flux form is 0 or 1 and works on the first-order form's cut links."""
    d = dict(W.growth_case(3, 0, bounce=True).params_dict())
    assert lbib.validate_params(d)[0] == lbib.OK
    buf = C.create_string_buffer(256)
    for kw, word in ((dict(no_flux_zeroth=True), b"no_flux_zeroth"), (dict(), b"no_flux_bounce")):
        q = lbib.make_params(dict(d, **kw))
        if not kw:
            q.no_flux_bounce = 2
        assert lbib.lib().lbib_validate_params(C.byref(q), buf, 256) == lbib.EINVAL
        assert word in buf.value


def test_growth_cases_follow_the_table():
    """The growth validations' discretisation (Section "Validation", table of Cases I-III):
    lattice 100 * 2^l, diameter 10 * 2^l, tau = tau_D = 1, 10^4 * 4^l steps, the point source's
    1e-2 per step at every level; the laws double the area at T = 1 (Cases II, III) or add one
    unit of area (Case I: 10^4 * 4^l * 1e-2 lattice areas = (10 * 2^l)^2 lattice areas)."""
    for level in range(W.LEAKAGE_LEVELS):
        for case in W.GROWTH_CASES:
            w = W.growth_case(case, level)
            L = 100 * 2 ** level
            assert (w.nx, w.ny, w.tau, w.steps) == (L, L, 1.0, 10000 * 4 ** level)
            assert abs(3.0 * w.species[0].D + 0.5 - 1.0) < 1e-15 and w.pressure_ring
            A0 = math.pi * (5.0 * 2 ** level) ** 2
            law = W.growth_law(case, level, A0, w.steps)
            if case == 1:
                assert w.node_sources.sum() == 1e-2 and w.node_sources[L // 2, L // 2] == 1e-2
                assert abs(law - A0 - (10.0 * 2 ** level) ** 2) < 1e-9 * A0
            else:
                assert abs(law / A0 - 2.0) < 1e-12
            assert (w.mass_source != 0) == (case == 2) and (w.mass_phi_gamma != 0) == (case == 3)


def test_workspace_size_holds_the_cell_map_of_mass_sources():
    """Mass sources keep one 32-bit cell index per lattice node."""
    d = dict(W.small_tissue(nx=200, ny=130, n_species=1).params_dict())
    m = dict(d, mass_source=1e-4)
    extra = _ws(m, 100) - _ws(d, 100)
    assert 200 * 130 * 4 <= extra < 200 * 130 * 4 + 256
    assert _ws(dict(d, area_alpha=1e-6), 100) == _ws(m, 100)


def test_workspace_size_holds_the_first_order_no_flux_state():
    """The first-order no-flux condition keeps, per buffer parity, four wall distances and a
    blocked-link byte per lattice node, and the previous step's concentration and velocity;
    the zeroth-order form keeps none of them."""
    d = dict(W.no_flux_tissue().params_dict())
    z = dict(d, no_flux_zeroth=True)
    nn = d["nx"] * d["ny"]
    extra = _ws(d, 100) - _ws(z, 100)
    want = 2 * (16 * nn + (nn + 3) // 4 * 4 + 4 * nn + 8 * nn)
    assert want <= extra < want + 8 * 256
