"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula and compares it with itself: each one
checks an identity, a closed-form solution, a special case reducing to a textbook
result, a brute-force count, or a value printed in the paper.  Each test names
the passage it pins.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1503_06726_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as fh:
        return json.load(fh)


# ------------------------------------------------------------------------------------------
# lattice constants and equilibria (Suppl. "Lattice Boltzmann Method", Eq. standardequilibrium)
# ------------------------------------------------------------------------------------------

def test_equilibrium_at_rest_gives_paper_weights(gold):
    # at u = 0 the equilibrium is w_i rho, so the weights are the paper's (4/9, 1/9, 1/36)
    np.testing.assert_allclose(O.equilibrium9(1.0, 0.0, 0.0), gold["d2q9_weights"], rtol=0, atol=1e-16)
    np.testing.assert_allclose(O.equilibrium5(1.0, 0.0, 0.0), gold["d2q5_weights"], rtol=0, atol=1e-16)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments_exact(gold, seed):
    # zeroth, first and second moments of the D2Q9 equilibrium: rho, rho u, rho cs2 I + rho u u
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.1 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(2)
    v = np.array(gold["d2q9_velocities"], float)
    f = O.equilibrium9(rho, u[0], u[1])
    assert abs(f.sum() - rho) < 1e-15
    np.testing.assert_allclose(f @ v, rho * u, rtol=0, atol=1e-16)
    P = np.einsum("i,ia,ib->ab", f, v, v)
    np.testing.assert_allclose(P, rho * gold["cs2"] * np.eye(2) + rho * np.outer(u, u), rtol=0, atol=1e-15)
    # D2Q5: concentration and advective flux phi u, isotropic second moment phi cs2 I
    v5 = np.array(gold["d2q5_velocities"], float)
    phi = 0.3 + rng.random()
    g = O.equilibrium5(phi, u[0], u[1])
    assert abs(g.sum() - phi) < 1e-15
    np.testing.assert_allclose(g @ v5, phi * u, rtol=0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", g, v5, v5), phi * gold["cs2"] * np.eye(2),
                               rtol=0, atol=1e-15)


# ------------------------------------------------------------------------------------------
# delta kernel (Eq. 1Dkernel and the 2-D product; Peskin's 4-point kernel as the option)
# ------------------------------------------------------------------------------------------

def test_cosine_kernel_printed_values(gold):
    for r, val in gold["delta1d_cos"]["values"]:
        assert abs(O.delta1d(O.DELTA_COS, r) - val) < 1e-16
        assert abs(O.delta1d(O.DELTA_COS, -r) - val) < 1e-16


@pytest.mark.parametrize("kernel", [O.DELTA_COS, O.DELTA_PESKIN])
def test_kernel_moment_identities(kernel):
    for s in np.linspace(0.0, 0.999, 37):
        r = np.array([s + 1.0, s, s - 1.0, s - 2.0])          # distances to i0 .. i0+3
        phi = np.array([O.delta1d(kernel, x) for x in r])
        assert abs(phi.sum() - 1.0) < 1e-15                    # partition of unity
        assert abs(phi[0] + phi[2] - 0.5) < 1e-15              # even / odd sums
        assert abs(phi[1] + phi[3] - 0.5) < 1e-15
        assert abs((phi ** 2).sum() - 3.0 / 8.0) < 1e-15       # sum of squares
        m1 = (r * phi).sum()
        if kernel == O.DELTA_PESKIN:
            assert abs(m1) < 1e-15                             # first moment vanishes
        else:
            closed = s - 0.5 + (math.cos(math.pi * s / 2) - math.sin(math.pi * s / 2)) / 2
            assert abs(m1 - closed) < 1e-15
        # outside the support: zero
        assert O.delta1d(kernel, 2.0 + 1e-9) == 0.0


# ------------------------------------------------------------------------------------------
# membrane forces (Eq. membraneforce, Hookean springs, area pressure)
# ------------------------------------------------------------------------------------------

def _star(rng, n, cx=20.3, cy=17.7, r0=6.0, amp=2.0):
    th = np.sort(rng.uniform(0, 2 * np.pi, n))
    r = r0 + amp * rng.uniform(-1, 1, n)
    return np.stack([cx + r * np.cos(th), cy + r * np.sin(th)], 1)


def _two_cells(rng):
    a = _star(rng, 17)
    b = _star(rng, 23, cx=45.1, cy=30.2)
    return np.array([0, 17, 40], np.int32), np.concatenate([a, b])


def _energy(xy, off, l0, A0, k, phim, kap):
    E = 0.0
    for c in range(len(off) - 1):
        p = xy[off[c]:off[c + 1]]
        q = np.roll(p, -1, 0)
        L = np.hypot(*(q - p).T)
        A = 0.5 * np.sum(p[:, 0] * q[:, 1] - q[:, 0] * p[:, 1])
        E += 0.5 * k * np.sum((L - l0[off[c]:off[c + 1]]) ** 2) + phim * L.sum() + 0.5 * kap * (A - A0[c]) ** 2
    return E


@pytest.mark.parametrize("seed", range(3))
def test_forces_are_minus_energy_gradient(seed):
    # F = -dE/dX for E = sum k/2 (L - l0)^2 + phi_m * perimeter + kappa/2 (A - A0)^2,
    # checked by central differences: pins signs, edge/rest-length indexing, the area gradient
    rng = np.random.default_rng(seed)
    off, xy = _two_cells(rng)
    l0 = 0.8 * np.hypot(*(np.roll(xy, -1, 0) - xy).T) * rng.uniform(0.7, 1.3, len(xy))
    A0 = np.array([90.0, 140.0])
    prm = dict(nx=64, ny=64, bc_y=0, tau=1.0, k_spring=0.03, phi_m=0.01, kappa_area=2e-3)
    F, area = O.forces(prm, off, xy, l0, A0)
    h = 1e-6
    for i in range(len(xy)):
        for d in range(2):
            xp = xy.copy(); xp[i, d] += h
            xm = xy.copy(); xm[i, d] -= h
            g = (_energy(xp, off, l0, A0, 0.03, 0.01, 2e-3) - _energy(xm, off, l0, A0, 0.03, 0.01, 2e-3)) / (2 * h)
            assert abs(F[i, d] + g) < 2e-8


@pytest.mark.parametrize("seed", range(3))
def test_forces_free_of_net_force_and_torque(seed):
    rng = np.random.default_rng(10 + seed)
    off, xy = _two_cells(rng)
    l0 = rng.uniform(0.5, 3.0, len(xy))
    prm = dict(nx=64, ny=64, bc_y=0, tau=1.0, k_spring=0.05, phi_m=0.02, kappa_area=1e-3)
    F, _ = O.forces(prm, off, xy, l0, np.array([50.0, 300.0]))
    for c in range(2):
        s = slice(off[c], off[c + 1])
        assert np.abs(F[s].sum(0)).max() < 1e-13
        torque = np.sum(xy[s, 0] * F[s, 1] - xy[s, 1] * F[s, 0])
        assert abs(torque) < 1e-11


def test_shoelace_area_matches_picks_theorem():
    # integer-vertex polygons: A = I + B/2 - 1 with I, B counted by brute force
    polys = [np.array([[0, 0], [7, 0], [7, 3], [4, 6], [0, 5]], float),
             np.array([[1, 1], [9, 2], [6, 8], [5, 4], [2, 7]], float)]
    from math import gcd
    for P in polys:
        n = len(P)
        B = sum(gcd(int(abs(P[(k + 1) % n][0] - P[k][0])), int(abs(P[(k + 1) % n][1] - P[k][1]))) for k in range(n))
        I = 0
        for x in range(-1, 12):
            for y in range(-1, 12):
                # strict interior by winding angle (no vertex-ray ambiguity: integer points on edges excluded first)
                on = False
                for k in range(n):
                    a, b = P[k], P[(k + 1) % n]
                    cr = (b[0] - a[0]) * (y - a[1]) - (b[1] - a[1]) * (x - a[0])
                    if cr == 0 and min(a[0], b[0]) <= x <= max(a[0], b[0]) and min(a[1], b[1]) <= y <= max(a[1], b[1]):
                        on = True
                if on:
                    continue
                ang = 0.0
                for k in range(n):
                    a = np.arctan2(P[k][1] - y, P[k][0] - x)
                    b = np.arctan2(P[(k + 1) % n][1] - y, P[(k + 1) % n][0] - x)
                    d = b - a
                    d = (d + np.pi) % (2 * np.pi) - np.pi
                    ang += d
                I += int(round(ang / (2 * np.pi)) != 0)
        prm = dict(nx=32, ny=32, bc_y=0, tau=1.0)
        _, area = O.forces(prm, np.array([0, n], np.int32), P, np.ones(n), np.zeros(1))
        assert area[0] == I + B / 2 - 1


@pytest.mark.parametrize("N", [16, 64, 129])
def test_regular_polygon_radial_force(N):
    # tension phi_m: inward radial force of magnitude 2 phi_m sin(pi/N);
    # springs: 2 k (L - l0) sin(pi/N) with L = 2 R sin(pi/N)
    R = 7.5
    th = 2 * np.pi * np.arange(N) / N
    xy = np.stack([30 + R * np.cos(th), 31 + R * np.sin(th)], 1)
    radial = np.stack([np.cos(th), np.sin(th)], 1)
    prm = dict(nx=64, ny=64, bc_y=0, tau=1.0, phi_m=0.013)
    F, _ = O.forces(prm, np.array([0, N], np.int32), xy, np.ones(N), np.zeros(1))
    np.testing.assert_allclose(F, -2 * 0.013 * math.sin(math.pi / N) * radial, rtol=0, atol=1e-14)
    L = 2 * R * math.sin(math.pi / N)
    prm = dict(nx=64, ny=64, bc_y=0, tau=1.0, k_spring=0.02)
    F, _ = O.forces(prm, np.array([0, N], np.int32), xy, np.full(N, 0.9 * L), np.zeros(1))
    np.testing.assert_allclose(F, -2 * 0.02 * 0.1 * L * math.sin(math.pi / N) * radial, rtol=0, atol=1e-14)


# ------------------------------------------------------------------------------------------
# spreading and interpolation (Eqs. forcedistribution, conversion2)
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("bc,kernel", [(0, 0), (1, 0), (0, 1)])
def test_spread_interp_adjoint(bc, kernel):
    # sum_x e(x).v(x) == sum_l F_l . (Interp v)(X_l) for any v: pins stencil, wrap, weights
    rng = np.random.default_rng(3)
    nx, ny = 37, 29
    prm = dict(nx=nx, ny=ny, bc_y=bc, tau=1.0, delta_kernel=kernel)
    n = 60
    xy = np.stack([rng.uniform(-nx, 2 * nx, n), rng.uniform(0.2, ny - 0.2, n)], 1)
    if bc == 0:
        xy[:, 1] = rng.uniform(-ny, 2 * ny, n)
    F = rng.standard_normal((n, 2))
    ex, ey = O.spread(prm, xy, F)
    v = rng.standard_normal((2, ny, nx))
    U = O.interp(prm, xy, v[0], v[1])
    lhs = (ex * v[0]).sum() + (ey * v[1]).sum()
    rhs = (F * U).sum()
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))
    if bc == 0:
        np.testing.assert_allclose([ex.sum(), ey.sum()], F.sum(0), rtol=0, atol=1e-12)


def test_spread_single_node_weights_brute_force():
    # one node: e at every lattice point equals F delta1D(dx) delta1D(dy) with minimum-image dx
    prm = dict(nx=16, ny=12, bc_y=0, tau=1.0)
    X = np.array([[15.3, -0.6]])   # wraps in x and y
    F = np.array([[2.0, -1.0]])
    ex, ey = O.spread(prm, X, F)
    for j in range(12):
        for i in range(16):
            dx = (X[0, 0] - i + 8) % 16 - 8
            dy = (X[0, 1] - j + 6) % 12 - 6
            w = (0.25 * (1 + math.cos(math.pi * dx / 2)) if abs(dx) <= 2 else 0.0) * \
                (0.25 * (1 + math.cos(math.pi * dy / 2)) if abs(dy) <= 2 else 0.0)
            assert abs(ex[j, i] - 2.0 * w) < 1e-15 and abs(ey[j, i] + w) < 1e-15


@pytest.mark.parametrize("kernel", [O.DELTA_COS, O.DELTA_PESKIN])
def test_interp_linear_field(kernel):
    # Interp of a + b.x: exact for Peskin's kernel; shifted by the first moment M1 for the cosine one
    rng = np.random.default_rng(4)
    nx = ny = 40
    prm = dict(nx=nx, ny=ny, bc_y=0, tau=1.0, delta_kernel=kernel)
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    ux = 0.3 + 0.01 * xx - 0.02 * yy
    uy = -0.1 + 0.005 * yy
    xy = rng.uniform(5, 34, (50, 2))
    U = O.interp(prm, xy, ux, uy)

    def m1(s):
        return 0.0 if kernel == O.DELTA_PESKIN else s - 0.5 + (np.cos(np.pi * s / 2) - np.sin(np.pi * s / 2)) / 2

    ex_ = xy[:, 0] - m1(xy[:, 0] % 1.0)
    ey_ = xy[:, 1] - m1(xy[:, 1] % 1.0)
    np.testing.assert_allclose(U[:, 0], 0.3 + 0.01 * ex_ - 0.02 * ey_, rtol=0, atol=1e-14)
    np.testing.assert_allclose(U[:, 1], -0.1 + 0.005 * ey_, rtol=0, atol=1e-14)


# ------------------------------------------------------------------------------------------
# rasterisation of domain IDs (Section "Cell Representation")
# ------------------------------------------------------------------------------------------

def _winding_inside(P, x, y):
    ang = 0.0
    n = len(P)
    for k in range(n):
        a = math.atan2(P[k][1] - y, P[k][0] - x)
        b = math.atan2(P[(k + 1) % n][1] - y, P[(k + 1) % n][0] - x)
        d = (b - a + math.pi) % (2 * math.pi) - math.pi
        ang += d
    return round(ang / (2 * math.pi)) != 0


def test_half_integer_square_holds_100_nodes():
    P = np.array([[10.5, 10.5], [20.5, 10.5], [20.5, 20.5], [10.5, 20.5]])
    m, ov = O.raster(dict(nx=32, ny=32, bc_y=0, tau=1.0), np.array([0, 4], np.int32), P)
    assert (m == 1).sum() == 100 and ov == 0
    assert m[11:21, 11:21].min() == 1


@pytest.mark.parametrize("seed", range(4))
def test_raster_matches_winding_number(seed):
    rng = np.random.default_rng(seed)
    nx, ny = 48, 40
    bc = seed % 2
    cells = [_star(rng, 40, cx=14.37, cy=15.21, r0=7, amp=3), _star(rng, 31, cx=33.61, cy=24.83, r0=5, amp=2)]
    if bc == 0:
        cells.append(_star(rng, 25, cx=-1.27, cy=35.55, r0=4, amp=1))   # straddles x = 0 and y = ny
    off = np.zeros(len(cells) + 1, np.int32)
    off[1:] = np.cumsum([len(c) for c in cells])
    xy = np.concatenate(cells)
    m, ov = O.raster(dict(nx=nx, ny=ny, bc_y=bc, tau=1.0), off, xy)
    assert ov == 0
    for j in range(ny):
        for i in range(nx):
            want = 0
            for c, P in enumerate(cells):
                for sx in (-nx, 0, nx):
                    for sy in ((-ny, 0, ny) if bc == 0 else (0,)):
                        if _winding_inside(P, i - sx, j - sy):
                            want = c + 1
            assert m[j, i] == want, (i, j)


def test_raster_overlap_smallest_id_wins():
    A = np.array([[2.5, 2.5], [9.5, 2.5], [9.5, 9.5], [2.5, 9.5]])
    B = A + 3.0
    m, ov = O.raster(dict(nx=16, ny=16, bc_y=0, tau=1.0), np.array([0, 4, 8], np.int32), np.concatenate([A, B]))
    assert ov == 16            # the 4x4 overlap
    assert (m == 1).sum() == 49 and (m == 2).sum() == 49 - 16


# ------------------------------------------------------------------------------------------
# lattice Boltzmann: invariants and closed-form flows
# ------------------------------------------------------------------------------------------

def test_mass_exact_and_momentum_gain_equals_body_force():
    # periodic box: sum rho constant; with a uniform acceleration g the momentum gains rho g per node
    w = W.random_fields(W.Workload(name="t", nx=24, ny=20, bc_y=0, tau=0.7, body_accel=(3e-5, -1e-5)), seed=1)
    s = O.from_workload(w)
    inv0 = s.invariants()
    for _ in range(20):
        a = s.invariants()
        s.step(1)
        b = s.invariants()
        assert abs(b[0] - a[0]) < 1e-14 * a[0]
        assert abs((b[1] - a[1]) - a[0] * 3e-5) < 1e-13
        assert abs((b[2] - a[2]) + a[0] * 1e-5) < 1e-13
    assert abs(s.invariants()[0] - inv0[0]) < 1e-13 * inv0[0]


def test_momentum_identity_with_membrane_forces():
    # P^{n+1} - P^n = sum_x rho^n e^n exactly, with e the spread membrane force + body force
    w = W.small_tissue(nx=64, ny=48, n_cells=4, bc_y=0, n_species=0, stretch=0.8, body=(1e-5, 0))
    s = O.from_workload(w)
    for _ in range(5):
        rho = s.get_fields()["rho"]
        a = s.invariants()
        s.step(1)
        ex, ey = s.last_spread()
        b = s.invariants()
        assert abs((b[1] - a[1]) - (rho * ex).sum()) < 1e-12
        assert abs((b[2] - a[2]) - (rho * ey).sum()) < 1e-12
        assert abs(b[0] - a[0]) < 1e-11


def test_galilean_fixed_point_and_node_translation():
    # uniform equilibrium (rho0, U0) without forces is stationary; nodes move by exactly U0
    U0 = np.array([1.25e-3, -0.75e-3])
    w = W.small_tissue(nx=50, ny=40, n_cells=3, bc_y=0, n_species=0, k_spring=0.0, body=(0, 0))
    w.u_init = np.broadcast_to(U0[:, None, None], (2, 40, 50)).copy()
    s = O.from_workload(w)
    f0, _ = s.populations()
    s.step(10)
    f1, _ = s.populations()
    assert np.abs(f1 - f0).max() < 1e-16
    np.testing.assert_allclose(s.get_fields()["xy"], w.xy + 10 * U0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0, 1.3])
def test_poiseuille_closed_form(tau):
    # steady channel flow between halfway bounce-back walls driven by g:
    # u(y) = 3g/(2tau-1) (y+1/2)(H-1/2-y) + g (16 tau^2 - 20 tau + 3) / (4 (2 tau - 1));
    # the bulk curvature g/(2 nu) fixes nu = cs2 (tau - 1/2)
    H, g = 12, 1e-6
    s = O.Sim(dict(nx=1, ny=H, bc_y=1, tau=tau, body_accel=(g, 0.0)))
    s.step(40000)
    r = s.get_fields()
    y = np.arange(H)
    exact = 3 * g / (2 * tau - 1) * (y + 0.5) * (H - 0.5 - y) + g * (16 * tau ** 2 - 20 * tau + 3) / (4 * (2 * tau - 1))
    np.testing.assert_allclose(r["u"][0, :, 0], exact, rtol=1e-9, atol=0)
    assert np.abs(r["u"][1]).max() < 1e-8 * exact.max()
    assert np.abs(r["rho"] - 1.0).max() < 1e-10


def test_couette_linear_profile():
    # top wall moving at U_w (moving-wall bounce-back hook): u(y) = U_w (y + 1/2) / H exactly
    H, Uw = 10, 1e-4
    s = O.Sim(dict(nx=1, ny=H, bc_y=1, tau=0.9), wall_u_top=Uw)
    s.step(30000)
    u = s.get_fields()["u"][0, :, 0]
    np.testing.assert_allclose(u, Uw * (np.arange(H) + 0.5) / H, rtol=1e-9, atol=0)


def test_shear_wave_follows_linearised_operator(gold):
    # Fourier amplitudes of f evolve by M = diag(e^{-i k.v}) (I - (I - E)/tau), E_ij = w_i (1 + v_i.v_j / cs2),
    # the linearisation of Eq. (bgkequation) about rest; a 1e-7 wave must follow M^n to O(amplitude)
    nx, ny, tau, A = 4, 32, 0.8, 1e-7
    v = np.array(gold["d2q9_velocities"], float)
    w9 = np.array(gold["d2q9_weights"])
    E = w9[:, None] * (1.0 + (v @ v.T) / gold["cs2"])
    k = np.array([0.0, 2 * np.pi / ny])
    M = np.diag(np.exp(-1j * (v @ k))) @ (np.eye(9) - (np.eye(9) - E) / tau)
    y = np.arange(ny)
    u = np.zeros((2, ny, nx))
    u[0] = A * np.sin(2 * np.pi * y / ny)[:, None]
    s = O.Sim(dict(nx=nx, ny=ny, bc_y=0, tau=tau))
    s.set_fields(u=u)
    f0, _ = s.populations()
    fh0 = np.fft.fft(f0[:, :, 0], axis=1)[:, 1]
    for n in (1, 7, 60):
        s2 = O.Sim(dict(nx=nx, ny=ny, bc_y=0, tau=tau))
        s2.set_fields(u=u)
        s2.step(n)
        fn, _ = s2.populations()
        fhn = np.fft.fft(fn[:, :, 0], axis=1)[:, 1]
        pred = np.linalg.matrix_power(M, n) @ fh0
        assert np.abs(fhn - pred).max() < 1e-6 * np.abs(fh0).max()


# ------------------------------------------------------------------------------------------
# D2Q5 advection-diffusion (Suppl. "Lattice Boltzmann Method", D2Q5 equations)
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("tauD", [0.65, 0.8, 1.3])
def test_d2q5_second_moment_closed_form(tauD):
    # from equilibrium at rest, per-axis second moment:
    # M2(t) = M2(0) + t N/3 + (2N/3)(tau-1)[t - tau(1 - (1-1/tau)^t)]  (long-time slope 2 D N)
    n = 96
    D = (tauD - 0.5) / 3.0
    s = O.Sim(dict(nx=n, ny=n, bc_y=0, tau=1.0, species=[dict(D=D)]))
    yy, xx = np.mgrid[0:n, 0:n]
    phi = np.where((xx - 48) ** 2 + (yy - 48) ** 2 <= 12 ** 2, 1.0 + 0.2 * np.sin(0.4 * yy), 0.0)
    s.set_fields(phi=phi[None])

    def mom():
        f = s.get_fields()["phi"][0]
        return f.sum(), (f * (xx - 48.0) ** 2).sum(), (f * (yy - 48.0) ** 2).sum()

    N, mx0, my0 = mom()
    T = 40
    s.step(T)
    N1, mx, my = mom()
    assert abs(N1 - N) < 1e-12 * N
    inc = T * N / 3 + (2 * N / 3) * (tauD - 1) * (T - tauD * (1 - (1 - 1 / tauD) ** T))
    assert abs(mx - (mx0 + inc)) < 1e-12 * mx
    assert abs(my - (my0 + inc)) < 1e-12 * my


def test_d2q5_centroid_advects_with_fluid_velocity():
    # uniform fluid velocity U0 is transferred to the species: the centroid moves exactly t U0
    # (box large enough that the ballistic fronts, speed 1 lu/step, never wrap around)
    n, U0 = 128, np.array([0.02, -0.013])
    s = O.Sim(dict(nx=n, ny=n, bc_y=0, tau=0.9, species=[dict(D=0.05)]))
    yy, xx = np.mgrid[0:n, 0:n]
    phi = np.exp(-((xx - 64.0) ** 2 + (yy - 64.0) ** 2) / 20.0)
    s.set_fields(u=np.broadcast_to(U0[:, None, None], (2, n, n)).copy(), phi=phi[None])

    def cen():
        f = s.get_fields()["phi"][0]
        return np.array([(f * xx).sum(), (f * yy).sum()]) / f.sum()

    c0 = cen()
    s.step(25)
    np.testing.assert_allclose(cen(), c0 + 25 * U0, rtol=0, atol=1e-11)


def test_uniform_schnakenberg_reduces_to_forward_euler():
    # spatially uniform fields: streaming is the identity and collision keeps phi, so each
    # step is phi <- phi + R(phi) with R from the paper's Schnakenberg system (rate gamma)
    a, b, gam = 0.1, 0.9, 0.01
    sp = [dict(D=0.05, reaction=2, c=(a, b, gam, 0)), dict(D=0.2, reaction=2, c=(a, b, gam, 0))]
    s = O.Sim(dict(nx=6, ny=5, bc_y=1, tau=0.8, species=sp))
    R0, L0 = 1.3, 0.4
    s.set_fields(phi=np.stack([np.full((5, 6), R0), np.full((5, 6), L0)]))
    Rv, Lv = R0, L0
    for n in range(50):
        Rv, Lv = Rv + gam * (a - Rv + Rv * Rv * Lv), Lv + gam * (b - Rv * Rv * Lv)
    s.step(50)
    phi = s.get_fields()["phi"]
    np.testing.assert_allclose(phi[0], Rv, rtol=1e-13)
    np.testing.assert_allclose(phi[1], Lv, rtol=1e-13)


def test_ade_mass_budget_with_cell_source():
    # N^{n+1} = N^n + sum_x R: sigma on every node inside a cell, minus lambda * N
    w = W.tiny_cell()
    s = O.from_workload(w)
    sig, lam = 1e-3, 1e-4
    for _ in range(10):
        r = s.get_fields()
        N = r["phi"][0].sum()
        inside = (r["mask"] != 0).sum()
        s.step(1)
        N1 = s.get_fields()["phi"][0].sum()
        assert abs(N1 - (N + sig * inside - lam * N)) < 1e-14


# ------------------------------------------------------------------------------------------
# coupled step
# ------------------------------------------------------------------------------------------

def test_tiny_workload_invariants():
    w = W.tiny_cell()
    s = O.from_workload(w)
    m0 = s.invariants()[0]
    s.step(200)
    r = s.get_fields()
    assert abs(s.invariants()[0] - m0) < 1e-10
    assert np.isfinite(r["u"]).all() and np.abs(r["u"]).max() < 1e-2
    assert (r["mask"] == 1).sum() > 250


def test_laplace_pressure_of_tensioned_circle():
    # constant tension phi_m on a circle: virtual work gives dp = phi_m / (R cos(pi/N)),
    # so rho_in - rho_out = dp / cs2; IB smearing makes this a 5 % check (P: IB leakage remark)
    n, R, N, phim = 64, 12.0, 150, 2e-3
    th = 2 * np.pi * np.arange(N) / N
    xy = np.stack([32.0 + R * np.cos(th), 32.0 + R * np.sin(th)], 1)
    s = O.Sim(dict(nx=n, ny=n, bc_y=0, tau=1.0, phi_m=phim))
    s.set_cells(np.array([0, N], np.int32), xy)
    s.step(3000)
    r = s.get_fields()
    yy, xx = np.mgrid[0:n, 0:n]
    rr = np.hypot(xx - 32.0, yy - 32.0)
    rin = r["rho"][rr < R - 4].mean()
    rout = r["rho"][rr > R + 5].mean()
    X = r["xy"]
    Rnow = np.hypot(X[:, 0] - X[:, 0].mean(), X[:, 1] - X[:, 1].mean()).mean()
    dp = phim / (Rnow * math.cos(math.pi / N))
    # p = rho cs2 (Suppl. "Lattice Boltzmann Method")
    assert abs((rin - rout) / 3.0 - dp) < 0.05 * dp


# ---- half-force velocity (option; Eq. bgkequation's forcing, Section "Validation" Case IV) ----
def test_half_force_velocity_removes_the_static_drift():
    """A circle under constant tension relaxes towards a static balance: the pressure jump
    holds the membrane, and the momentum averaged over a step vanishes.  With the literal
    velocity u = sum f v / rho the pre-collision momentum at a forced node is -rho f / 2, so the
    membrane nodes drift at minus half the interpolated force density (outward for a contracting
    tension); the half-force-shifted velocity u + f/2 removes that drift, leaving only the slow
    inward leakage (the paper's shrinking Case IV cell)."""
    n, R, N, phim = 64, 12.0, 150, 2e-3
    th = 2 * np.pi * np.arange(N) / N
    xy = np.stack([32.0 + R * np.cos(th), 32.0 + R * np.sin(th)], 1)
    ratio = {}
    for hf in (False, True):
        s = O.Sim(dict(nx=n, ny=n, bc_y=0, tau=1.0, phi_m=phim, interp_half_force=hf))
        s.set_cells(np.array([0, N], np.int32), xy)
        s.step(2000)
        X0 = s.get_fields()["xy"]
        F, _ = s.forces()
        ex, ey = O.spread(s.params, X0, F)
        E = O.interp(s.params, X0, ex, ey)             # force density at the nodes
        s.step(50)
        X1 = s.get_fields()["xy"]
        c = X0.mean(0)
        rhat = (X0 - c) / np.linalg.norm(X0 - c, axis=1)[:, None]
        vr = float(((X1 - X0) / 50 * rhat).sum(1).mean())
        er = float((E * rhat).sum(1).mean())
        assert er < 0.0                                  # tension pulls inward
        ratio[hf] = vr / er
    assert -0.55 < ratio[False] < -0.40                 # drift of minus half the force density
    assert 0.0 < ratio[True] < 0.05                     # shifted: only a small inward leakage


# ---- no-flux membranes (Section "Signalling"; Suppl. "No-flux Boundary Condition for
# ---- Reaction-Advection-Diffusion Equations": the first-order form, and the zeroth-order option)
NF_FORMS = pytest.mark.parametrize("zeroth", [False, True], ids=["first-order", "zeroth-order"])


def _inside(o):
    return o.get_fields()["mask"] != 0


def _rect(x0, y0, x1, y1, h=0.5):
    """A CCW rectangle resampled at spacing h (input preparation)."""
    return W._resample(np.array([[x0, y0], [x1, y0], [x1, y1], [x0, y1]], float), h)


def test_link_crossings_of_an_axis_aligned_rectangle():
    """The wall distances of a rectangle with edges at x = 10.3, 30.7 and y = 20.6, 40.2, worked
    out by hand: the links of rows 21..40 cross the vertical edges, those of columns 11..30 the
    horizontal ones; every other link is free."""
    P = _rect(10.3, 20.6, 30.7, 40.2)
    q = O.link_crossings(dict(nx=48, ny=56, bc_y=0, tau=1.0), np.array([0, len(P)], np.int32), P)
    exp = np.full((4, 56, 48), np.inf)
    rows, cols = np.arange(21, 41), np.arange(11, 31)
    exp[0, rows, 11] = 11 - 10.3           # +x population of column 11, its link cut 0.7 back
    exp[2, rows, 10] = 10.3 - 10           # -x population of column 10
    exp[0, rows, 31] = 31 - 30.7
    exp[2, rows, 30] = 30.7 - 30
    exp[1, 21, cols] = 21 - 20.6           # +y population of row 21
    exp[3, 20, cols] = 20.6 - 20
    exp[1, 41, cols] = 41 - 40.2
    exp[3, 40, cols] = 40.2 - 40
    fin = np.isfinite(exp)
    assert np.array_equal(np.isfinite(q), fin)
    np.testing.assert_allclose(q[fin], exp[fin], rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_link_crossings_match_brute_force_segment_intersections(seed):
    """Jittered star polygons straddling the periodic edges: every lattice link is intersected
    with every polygon edge by the parametric segment formula (an independent computation), and
    the nearest intersection from each end must be the table's wall distance."""
    rng = np.random.default_rng(100 + seed)
    nx, ny = 30, 26
    cells, off = [], [0]
    for cx, cy in ((1.3 + 2 * rng.random(), 12.7), (17.2, 24.4 + rng.random())):
        m = 40
        th = 2 * np.pi * (np.arange(m) + 0.3 * rng.random(m)) / m
        r = 6.0 + 1.5 * rng.random(m)
        cells.append(np.stack([cx + r * np.cos(th), cy + r * np.sin(th)], 1))
        off.append(off[-1] + m)
    P = np.concatenate(cells)
    q = O.link_crossings(dict(nx=nx, ny=ny, bc_y=0, tau=1.0), np.array(off, np.int32), P)
    exp = np.full((4, ny, nx), np.inf)
    vx, vy = (1, 0, -1, 0), (0, 1, 0, -1)
    for c in range(2):
        Q = P[off[c]:off[c + 1]]
        for A, B in zip(Q, np.roll(Q, -1, 0)):
            lo, hi = np.floor(np.minimum(A, B)).astype(int) - 1, np.ceil(np.maximum(A, B)).astype(int) + 1
            for X in range(lo[0], hi[0] + 1):
                for Y in range(lo[1], hi[1] + 1):
                    for d in range(4):
                        # link from node (X, Y) back to (X - v, Y - v), a unit segment
                        ex, ey = -vx[d], -vy[d]
                        den = ex * (B[1] - A[1]) - ey * (B[0] - A[0])
                        if den == 0:
                            continue
                        t = ((A[0] - X) * (B[1] - A[1]) - (A[1] - Y) * (B[0] - A[0])) / den
                        u = ((A[0] - X) * ey - (A[1] - Y) * ex) / den
                        if 0 <= t <= 1 and 0 <= u < 1:
                            k = (d, Y % ny, X % nx)
                            exp[k] = min(exp[k], t)
    fin = np.isfinite(exp)
    assert np.array_equal(np.isfinite(q), fin)
    np.testing.assert_allclose(q[fin], exp[fin], rtol=0, atol=1e-12)


def test_first_order_boundary_values_are_exact_for_linear_fields():
    """The supplement's first-order interpolation and extrapolation are exact for linear fields:
    with the previous step's concentration linear in x and y and the velocity at rest, every
    replaced population is w_i phi(x); with a constant concentration and a velocity linear in
    the distance from a wall and zero on it, it is w_i (phi + 3 v_i . phi u(x)), at the nodes on
    both sides of that wall."""
    P = _rect(10.3, 20.6, 40.7, 50.2)
    nx = ny = 64
    d = dict(nx=nx, ny=ny, bc_y=0, tau=1.0, species=[dict(D=0.1, reaction=0, no_flux=True)])
    o = O.Sim(d)
    o.set_cells(np.array([0, len(P)], np.int32), P)
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    w = np.array([1 / 6.0] * 4)
    # (1) linear concentration, fluid at rest: the extrapolation gives phi at the node
    phi = 0.4 + 0.013 * xx - 0.007 * yy
    o.set_prev_moments(phi[None], np.zeros((2, ny, nx)))
    v = o.no_flux_values(0)
    q = O.link_crossings(d, np.array([0, len(P)], np.int32), P)
    assert np.array_equal(np.isfinite(v), np.isfinite(q))
    # nodes whose two steps on along the direction stay on their side (away from the corners)
    inner = np.zeros((ny, nx), bool)
    inner[23:48, 3:62] = True
    inner2 = np.zeros((ny, nx), bool)
    inner2[3:62, 13:38] = True
    for k in range(4):
        sel = np.isfinite(v[k]) & (inner if k in (0, 2) else inner2)
        assert sel.sum() >= 50
        np.testing.assert_allclose(v[k][sel], w[k] * phi[sel], rtol=0, atol=1e-14)
    # (2) constant concentration, velocity linear in x - 10.3 (zero on the left wall) and in
    # y - 20.6 (zero on the bottom wall): the interpolated momentum is phi u at the node
    phi0 = 0.8
    u = np.stack([2e-3 * (xx - 10.3), -3e-3 * (yy - 20.6)])
    o.set_prev_moments(np.full((1, ny, nx), phi0), u)
    v = o.no_flux_values(0)
    left = np.isfinite(v[0]) & inner & (xx < 20)        # +x population, node inside, x = 11
    right = np.isfinite(v[2]) & inner & (xx < 20)       # -x population, node outside, x = 10
    np.testing.assert_allclose(v[0][left], w[0] * (phi0 + 3 * phi0 * u[0][left]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(v[2][right], w[2] * (phi0 - 3 * phi0 * u[0][right]), rtol=0, atol=1e-15)
    bot = np.isfinite(v[1]) & inner2 & (yy < 30)
    top = np.isfinite(v[3]) & inner2 & (yy < 30)
    np.testing.assert_allclose(v[1][bot], w[1] * (phi0 + 3 * phi0 * u[1][bot]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(v[3][top], w[3] * (phi0 - 3 * phi0 * u[1][top]), rtol=0, atol=1e-15)
    assert left.sum() >= 20 and right.sum() >= 20 and bot.sum() >= 20 and top.sum() >= 20


def _neumann_error(level, bounce=False):
    """Diffusion (D = 1/6, fluid at rest) next to a flat no-flux wall at x = 10 s + 0.37 inside
    a long rectangular cell, from the even extension of a Gaussian (width 5 s, 8 s from the
    wall), after 400 s^2 steps; s = 2^level.  The Neumann solution on the half-line is the
    image pair of spreading Gaussians.  Returns the largest error relative to the peak on a
    middle row at the end, and the largest relative change of that row's mass at four times."""
    s = 2 ** level
    nx, ny = 120 * s, 24
    xw = 10 * s + 0.37
    P = _rect(xw, 3.41, 110 * s + 0.37, 20.41)
    D = 1.0 / 6.0
    xc, sg0 = xw + 8 * s, 5.0 * s
    o = O.Sim(dict(nx=nx, ny=ny, bc_y=0, tau=1.0, species=[dict(D=D, reaction=0, no_flux=True)],
                   no_flux_bounce=bounce))
    o.set_cells(np.array([0, len(P)], np.int32), P)
    x = np.arange(nx, dtype=float)
    ins = (x > xw) & (x < 110 * s + 0.37)

    def pair(sg):
        return np.exp(-(x - xc) ** 2 / (2 * sg * sg)) + np.exp(-(x - (2 * xw - xc)) ** 2 / (2 * sg * sg))
    phi = np.zeros((1, ny, nx))
    phi[0, 4:21] = np.where(ins, pair(sg0), 0.0)
    o.set_fields(phi=phi)
    T = 400 * s * s
    dm = 0.0
    for _ in range(4):
        o.step(T // 4)
        row = o.get_fields()["phi"][0, 12]
        dm = max(dm, abs(row[ins].sum() / phi[0, 12][ins].sum() - 1.0))
    sgt = math.sqrt(sg0 * sg0 + 2 * D * T)
    exact = np.where(ins, sg0 / sgt * pair(sgt), 0.0)
    return np.abs(row - exact).max() / exact.max(), dm


def test_first_order_no_flux_follows_the_neumann_solution():
    """Against the method-of-images solution of a no-flux (Neumann) wall: within 1 % of the peak
    and 1.5 % in mass at the coarse resolution, and both errors shrink at least as fast as
    first order when the lattice is refined twice (diffusive scaling)."""
    e0, m0 = _neumann_error(0)
    e1, m1 = _neumann_error(1)
    assert e0 < 0.01 and m0 < 0.015
    assert e1 < 0.6 * e0 and m1 < 0.7 * m0


def test_bounce_back_no_flux_follows_the_neumann_solution():
    """The bounce-back form against the same image solution: it keeps the row's mass to
    round-off, its profile error is below 0.3 % of the peak at the coarse resolution (the wall
    sits 0.37 of a link from the nodes, not midway) and shrinks at least as fast as first order
    under refinement."""
    e0, m0 = _neumann_error(0, bounce=True)
    e1, m1 = _neumann_error(1, bounce=True)
    assert e0 < 0.003 and m0 < 1e-12 and m1 < 1e-12
    assert e1 < 0.6 * e0


@NF_FORMS
def test_no_flux_keeps_a_uniform_field_uniform(zeroth):
    """A uniform concentration at rest is an equilibrium on both sides of every membrane, and
    the replacement equilibrium rebuilds exactly the populations that would have arrived: the
    field stays uniform (to round-off)."""
    w = W.no_flux_tissue(static=True)
    w.no_flux_zeroth = zeroth
    w.species[0].reaction = W.REACT_NONE
    w.phi_init = np.full((1, w.ny, w.nx), 0.7)
    o = O.from_workload(w)
    o.step(60)
    phi = o.get_fields()["phi"][0]
    assert np.max(np.abs(phi - 0.7)) < 1e-13


@NF_FORMS
def test_no_flux_confines_a_cell_source_to_the_cells(zeroth):
    """Static cells with a source inside them and the membranes as no-flux boundaries: the
    extracellular concentration stays exactly zero while the cells fill; with the membranes
    invisible, the source leaks out by diffusion."""
    w = W.no_flux_tissue(static=True, no_flux=True)
    w.no_flux_zeroth = zeroth
    o = O.from_workload(w)
    o.step(100)
    inside = _inside(o)
    phi = o.get_fields()["phi"][0]
    assert inside.any() and (~inside).any()
    assert np.all(phi[~inside] == 0.0)
    assert np.min(phi[inside]) > 0.0
    o2 = O.from_workload(W.no_flux_tissue(static=True, no_flux=False))
    o2.step(100)
    phi2 = o2.get_fields()["phi"][0]
    assert np.max(phi2[~inside]) > 1e-4 * np.max(phi2[inside])


@NF_FORMS
def test_no_flux_changes_only_nodes_next_to_a_membrane(zeroth):
    """After one step the no-flux run differs from the membranes-invisible run only at nodes
    with a blocked link (zeroth-order form: a lattice neighbour on the other side of a membrane;
    first-order form: a link a membrane edge crosses), or next to one; elsewhere the two agree
    exactly."""
    wa = W.no_flux_tissue(static=True, no_flux=True)
    wa.no_flux_zeroth = zeroth
    wb = W.no_flux_tissue(static=True, no_flux=False)
    phi0 = 0.1 + 0.05 * np.random.default_rng(3).random((1, wa.ny, wa.nx))
    wa.phi_init = phi0
    wb.phi_init = phi0
    oa, ob = O.from_workload(wa), O.from_workload(wb)
    if zeroth:
        inside = _inside(oa)
        edge = np.zeros_like(inside)
        for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
            nb = np.roll(inside, (dy, dx), axis=(0, 1))
            if dy:                      # walls in y: no link across the top and bottom rows
                nb[0 if dy == 1 else -1, :] = inside[0 if dy == 1 else -1, :]
            edge |= nb != inside
    else:
        edge = np.isfinite(O.link_crossings(wa.params_dict(), wa.offsets, wa.xy)).any(0)
    oa.step(1)
    ob.step(1)
    pa, pb = oa.get_fields()["phi"][0], ob.get_fields()["phi"][0]
    # a node's streamed value depends on its neighbours' replacement one step earlier
    near = edge.copy()
    for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        near |= np.roll(edge, (dy, dx), axis=(0, 1))
    if not zeroth:                      # the extrapolation reads two nodes on
        near2 = near.copy()
        for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
            near2 |= np.roll(near, (dy, dx), axis=(0, 1))
        near = near2
    assert np.array_equal(pa[~near], pb[~near])
    assert not np.array_equal(pa[edge], pb[edge])


# ---- mass sources and area control (Section "Control of Cell Area") ----
def _circle(n, cx, cy, r):
    t = 2.0 * np.pi * np.arange(n) / n
    return np.stack([cx + r * np.cos(t), cy + r * np.sin(t)], 1)


def _shoelace(P):
    x, y = P[:, 0], P[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def test_mass_source_moves_with_the_fluid():
    """A uniform flow at rest density, one static cell (no forces) with a constant source s:
    each node of the cell collides to f^eq(1, u0) + s f^eq(1, u0) = f^eq(1 + s, u0), so after
    one step nodes whose upstream neighbours all lie in the cell have density 1 + s and still
    the velocity u0, and nodes whose neighbours all lie outside keep density 1 and u0."""
    nx, ny, s = 48, 40, 1e-3
    u0 = (0.02, -0.01)
    o = O.Sim(dict(nx=nx, ny=ny, bc_y=0, tau=0.8, mass_source=s))
    cx, cy, R = 24.3, 20.1, 8.0
    o.set_cells(np.array([0, 48], np.int32), _circle(48, cx, cy, R))
    u = np.zeros((2, ny, nx))
    u[0], u[1] = u0
    o.set_fields(rho=np.ones((ny, nx)), u=u)
    o.step(1)
    f = o.get_fields()
    yy, xx = np.mgrid[0:ny, 0:nx]
    d = np.hypot(xx - cx, yy - cy)
    inner, outer = d < R - 2.5, d > R + 2.5
    assert inner.sum() > 60 and outer.sum() > 1000
    np.testing.assert_allclose(f["rho"][inner], 1.0 + s, rtol=0, atol=1e-14)
    np.testing.assert_allclose(f["rho"][outer], 1.0, rtol=0, atol=1e-14)
    for q in range(2):
        np.testing.assert_allclose(f["u"][q][inner | outer], u0[q], rtol=0, atol=1e-14)


def test_mass_source_adds_exactly_the_controlled_mass():
    """In a walled box (collision, forcing, streaming and halfway bounce-back all conserve
    mass) each step adds sum_k S_k N_k, S_k = s + alpha (A0_k - A_k) with A_k the shoelace area
    of the step's positions and N_k the nodes of cell k in the domain map, while springs and a
    body force move the cells."""
    w = W.mass_source_tissue(static=False, mass_source=2e-4, area_alpha=3e-6)
    off = w.offsets
    o = O.from_workload(w)
    for _ in range(8):
        f0 = o.get_fields()
        X, m = f0["xy"], f0["mask"]
        want = 0.0
        for k in range(w.n_cells):
            A = _shoelace(X[off[k]:off[k + 1]])
            want += (w.mass_source + w.area_alpha * (w.rest_area[k] - A)) * np.count_nonzero(m == k + 1)
        o.step(1)
        got = o.get_fields()["rho"].sum() - f0["rho"].sum()
        assert abs(got - want) < 1e-10 * f0["rho"].sum(), (got, want)


@pytest.mark.parametrize("A0", [420.0, 220.0])
def test_area_controller_follows_its_rate_law(A0):
    """One free circular cell (no membrane forces) under the area controller alone: the added
    mass S A per step becomes cell area, so A follows dA/dt = alpha (A0 - A) A.  The lattice
    fluid is weakly compressible (part of the mass raises the density instead), so the area
    stays within 15 % of the initial gap of that law's solution, and approaches A0
    monotonically from either side."""
    alpha = 2e-5
    o = O.Sim(dict(nx=64, ny=64, bc_y=0, tau=0.8, area_alpha=alpha))
    o.set_cells(np.array([0, 64], np.int32), _circle(64, 32.3, 31.7, 10.0), rest_area=np.array([A0]))
    A = _shoelace(o.get_fields()["xy"])
    gap0 = A0 - A
    law, prev = A, A
    for _ in range(5):
        o.step(80)
        for _k in range(80):
            law += alpha * (A0 - law) * law
        now = _shoelace(o.get_fields()["xy"])
        assert abs(now - law) < 0.15 * abs(gap0), (now, law)
        assert (now - prev) * gap0 > 0
        prev = now
    assert abs(A0 - prev) < 0.2 * abs(gap0)


# ---- pressure boundary (Suppl. "Pressure Boundary Condition for the Fluid Equations") ----
def test_pressure_ring_holds_rho0_and_keeps_the_velocity():
    """Random fields after a few steps: every ring node reports density rho0 and the velocity
    sum f v / sum f of its stored populations (the rescaling cancels in it); interior nodes
    report the plain moments."""
    nx, ny = 40, 30
    rng = np.random.default_rng(5)
    o = O.Sim(dict(nx=nx, ny=ny, bc_y=1, tau=0.7, rho0=1.0, pressure_ring=True, body_accel=(1e-5, 0.0)))
    o.set_fields(rho=1.0 + 0.01 * rng.random((ny, nx)), u=0.01 * rng.standard_normal((2, ny, nx)))
    o.step(5)
    F = o.get_fields()
    f, _ = o.populations()
    r = f.sum(0)
    vx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1]); vy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
    ux = np.tensordot(vx, f, 1) / r
    uy = np.tensordot(vy, f, 1) / r
    ring = np.zeros((ny, nx), bool)
    ring[0, :] = ring[-1, :] = ring[:, 0] = ring[:, -1] = True
    assert np.max(np.abs(F["rho"][ring] - 1.0)) < 1e-15
    assert np.max(np.abs(r[ring] - 1.0)) > 1e-5           # the stored populations were not rescaled yet
    np.testing.assert_array_equal(F["rho"][~ring], r[~ring])
    np.testing.assert_allclose(F["u"][0], ux, rtol=0, atol=1e-16)
    np.testing.assert_allclose(F["u"][1], uy, rtol=0, atol=1e-16)


def test_uniform_source_grows_a_cell_exponentially():
    """Case II of the supplement's validation: a free circular cell with a uniform mass source
    s per node and step in a domain whose boundary holds the pressure.  With an incompressible
    fluid and an impermeable membrane the area would follow A0 exp(s t); the lattice fluid and
    the immersed boundary lose a few per cent of it (compression, leakage), less on the finer
    lattice.  Without the pressure ring the closed box compresses instead."""
    s = 1e-3

    def run(n, R, nodes, ring):
        o = O.Sim(dict(nx=n, ny=n, bc_y=0, tau=1.0, mass_source=s, pressure_ring=ring))
        o.set_cells(np.array([0, nodes], np.int32), _circle(nodes, n / 2 + 0.3, n / 2 - 0.3, R))
        A0 = _shoelace(o.get_fields()["xy"])
        out = []
        for k in range(1, 8):
            o.step(100)
            out.append(_shoelace(o.get_fields()["xy"]) / A0)
        return np.array(out), o.get_fields()["rho"].mean()

    law = np.exp(s * 100 * np.arange(1, 8))
    coarse, rho_c = run(100, 10.0, 64, True)
    assert np.all(np.abs(coarse / law - 1.0) < 0.06), coarse / law
    assert coarse[-1] > 1.9                                  # doubled by t = 700 > ln 2 / s
    fine, _ = run(160, 16.0, 100, True)
    # past the start-up transient (the first 100 steps), the finer lattice is closer to the law
    assert np.all(np.abs(fine / law - 1.0)[1:] < np.abs(coarse / law - 1.0)[1:])
    closed, rho_closed = run(100, 10.0, 64, False)
    assert abs(rho_c - 1.0) < 3e-3 and rho_closed - 1.0 > 0.02
    assert closed[-1] < coarse[-1]


def test_node_sources_add_exactly_their_mass():
    """Per-node sources (point sources, validation Case I): every step adds the map's total to
    the lattice's mass, S f^eq(1, u) at each node, and, with the fluid at rest, no momentum."""
    nx, ny, n = 32, 24, 5
    rate = np.zeros((ny, nx))
    rate[5, 7] = 1e-3
    rate[17, 20] = 2.5e-3
    rate[0, 31] = 4e-4
    o = O.Sim(dict(nx=nx, ny=ny, bc_y=0, tau=0.8, rho0=1.0))
    o.set_node_sources(rate)
    m0 = o.invariants()[0]
    o.step(n)
    inv = o.invariants()
    assert abs(inv[0] - (m0 + n * rate.sum())) <= 1e-12 * m0
    assert np.max(np.abs(inv[1:3])) < 1e-12 * m0
    o.set_node_sources(None)                   # removed: mass stays
    o.step(3)
    assert abs(o.invariants()[0] - inv[0]) <= 1e-12 * m0


def test_pressure_points_hold_rho0():
    """Pressure points anywhere in the lattice (Suppl. "Pressure Boundary Condition for the
    Fluid Equations"): a flagged interior node reports rho0 after every step, as the outer ring
    does, and takes out part of the mass a point source puts in (a closed box without it keeps
    all of it)."""
    nx, ny = 40, 30
    rate = np.zeros((ny, nx))
    rate[8, 9] = 2e-3
    pm = np.zeros((ny, nx), np.uint8)
    pm[21, 30] = 1
    o = O.Sim(dict(nx=nx, ny=ny, bc_y=1, tau=0.9, rho0=1.0))
    o.set_node_sources(rate)
    o.set_pressure_nodes(pm)
    m0 = o.invariants()[0]
    for _ in range(4):
        o.step(250)
        assert abs(o.get_fields()["rho"][21, 30] - 1.0) < 1e-14
    kept = o.invariants()[0] - m0
    assert 0.0 < kept < 0.8 * 1000 * rate.sum()
    o.set_pressure_nodes(None)
    m1 = o.invariants()[0]
    o.step(100)
    assert abs(o.invariants()[0] - m1 - 100 * rate.sum()) <= 1e-12 * m1


def test_pressure_points_on_the_ring_equal_the_ring_option():
    """A pressure map that flags exactly the outer ring gives the pressure_ring option's run bit
    for bit (a source cell drives the flow)."""
    n = 48
    ring = np.zeros((n, n), np.uint8)
    ring[0, :] = ring[-1, :] = ring[:, 0] = ring[:, -1] = 1
    def run(use_map):
        o = O.Sim(dict(nx=n, ny=n, bc_y=0, tau=1.0, mass_source=2e-3, pressure_ring=not use_map))
        o.set_cells(np.array([0, 40], np.int32), _circle(40, n / 2 + 0.3, n / 2 - 0.3, 8.0))
        if use_map:
            o.set_pressure_nodes(ring)
        o.step(60)
        return o.get_fields(), o.invariants()
    (Fa, ia), (Fb, ib) = run(False), run(True)
    for k in ("rho", "u", "xy"):
        np.testing.assert_array_equal(Fa[k], Fb[k])
    np.testing.assert_array_equal(ia, ib)


def test_concentration_source_adds_gamma_phi():
    """Validation Case III's source: a node inside a cell gains mass_phi_gamma phi_0(x) per step,
    phi_0 its concentration of species 0 as the collision sees it (the reported field, after
    the no-flux replacement).  One step adds gamma times the species inside the cell."""
    n, gamma = 40, 3e-3
    cx, cy, R = 20.3, 19.7, 7.0
    yy, xx = np.mgrid[0:n, 0:n]
    phi = (1.0 + 0.2 * np.sin(0.3 * xx) * np.cos(0.2 * yy)) * (np.hypot(xx - cx, yy - cy) < R)
    p = dict(nx=n, ny=n, bc_y=0, tau=1.0, rho0=1.0, mass_phi_gamma=gamma,
             species=[dict(D=0.1, phi_ref=0.0, reaction=0, c=(0, 0, 0, 0), no_flux=True)])
    o = O.Sim(p)
    o.set_cells(np.array([0, 48], np.int32), _circle(48, cx, cy, R))
    o.set_fields(phi=phi[None])
    for _ in range(3):
        F = o.get_fields()
        inside = F["mask"] > 0
        want = gamma * F["phi"][0][inside].sum()
        m0 = o.invariants()[0]
        o.step(1)
        got = o.invariants()[0] - m0
        assert abs(got - want) <= 1e-10 * want, (got, want)


def test_point_source_grows_a_cell_linearly():
    """Validation Case I in lattice units (level 0 of the supplement's table: a cell of diameter
    10 in a 100 x 100 domain, tau = 1, the point source's 1e-2 per step at the centre node, the
    boundary held at rho0): the area grows by the source's rate, A = A0 + 1e-2 t, within 2 % of
    the increase over 300 steps (the membrane is a slightly leaky immersed boundary)."""
    n, R, nodes = 100, 5.0, 63
    cx, cy = n / 2 + 0.3, n / 2 - 0.3
    rate = np.zeros((n, n))
    rate[int(round(cy)), int(round(cx))] = 1e-2
    o = O.Sim(dict(nx=n, ny=n, bc_y=0, tau=1.0, rho0=1.0, pressure_ring=True))
    o.set_cells(np.array([0, nodes], np.int32), _circle(nodes, cx, cy, R))
    o.set_node_sources(rate)
    A0 = _shoelace(o.get_fields()["xy"])
    o.step(300)
    dA = _shoelace(o.get_fields()["xy"]) - A0
    assert abs(dA / 3.0 - 1.0) < 0.02, dA


def _area_and_species(o):
    F = o.get_fields()
    return _shoelace(F["xy"]), F["phi"][0], F["mask"] > 0


def test_bounce_back_no_flux_conserves_a_growing_cell_species():
    """The bounce-back form of the no-flux condition: what one side of a cut link sends, the
    other never receives, so while validation Case I's point source grows the cell (at the
    coarsest resolution) the species stays inside (the extracellular concentration exactly
    zero, also after the first step from the set fields) and its total is conserved to
    round-off.  The supplement's equilibrium forms lose more than 1 % of it meanwhile."""
    w = W.growth_case(1, 0, steps=1500, bounce=True)
    o = O.from_workload(w)
    _, ph, ins = _area_and_species(o)
    M0 = ph.sum()
    o.step(1)
    _, ph, ins = _area_and_species(o)
    assert np.all(ph[~ins] == 0.0)
    for _ in range(3):
        o.step(500)
        A, ph, ins = _area_and_species(o)
        assert np.all(ph[~ins] == 0.0)
        assert abs(ph.sum() - M0) <= 1e-12 * M0
    assert A > 1.06 * _shoelace(w.xy)                     # the cell did grow
    w.no_flux_bounce = False
    e = O.from_workload(w)
    e.step(1500)
    assert abs(e.get_fields()["phi"][0].sum() / M0 - 1.0) > 0.01


def test_bounce_back_keeps_a_resting_cell_exact():
    """A cell at rest (no forces, no flow) with the species at 1 inside and 0 outside: every
    population the bounce-back returns is the equilibrium the node sent, so the field does not
    change at all (to round-off)."""
    w = W.growth_case(1, 0, steps=200, bounce=True)
    w.node_sources = None
    o = O.from_workload(w)
    phi0 = o.get_fields()["phi"][0]
    o.step(200)
    assert np.max(np.abs(o.get_fields()["phi"][0] - phi0)) < 1e-13


def test_bounce_back_restart_from_populations_is_exact():
    """Populations restored mid-run carry their own history: the populations each node sent the
    step before are the ones that streamed into them (streaming with the wall reflection is a
    permutation), so a run restarted from its populations continues bit for bit.  Walls in y
    and a moving tissue exercise the wall reflection and moving cut links."""
    w = W.no_flux_tissue(static=False)
    w.no_flux_bounce = True
    a = O.from_workload(w)
    b = O.from_workload(w)
    a.step(30)
    b.step(15)
    f, g = b.populations()
    phi, u = b.prev_moments()
    X = b.get_fields()["xy"]
    c = O.from_workload(w)
    rest_len = w.rest_len if w.rest_len is not None else W.edge_lengths(w.offsets, w.xy)
    rest_area = w.rest_area if w.rest_area is not None else np.array(
        [_shoelace(w.xy[w.offsets[k]:w.offsets[k + 1]]) for k in range(w.n_cells)])
    c.set_cells(w.offsets, X, rest_len, rest_area)
    c.set_populations(f, g.reshape(-1, w.ny, w.nx))
    c.set_prev_moments(phi, u)
    c.step(15)
    A, C = a.get_fields(), c.get_fields()
    for k in ("rho", "u", "phi", "xy"):
        np.testing.assert_array_equal(A[k], C[k])
