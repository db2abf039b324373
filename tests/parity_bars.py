"""The parity bars of the GPU tests against the FP64 oracle (test infrastructure).

Relative L2 errors are taken on the quantities that carry the method's error, not on values
dominated by a constant: the velocity, the concentrations, the node displacement X - X0
(positions themselves are about 10^3 lattice units, so their relative error says nothing),
and the density deviation rho - rho0.

The density deviation is often far below what FP32 storage of the populations resolves (the
deviations f_i - w_i rho0 are stored in FP32, the oracle keeps every population in FP64), so
its bar has three parts:
  ||drho_gpu - drho_oracle||_2 <= tol ||drho_oracle||_2 + 3 eps sqrt(n) ||(|drho| + 2|u|)||_2
                                  + 9 eps64 rho0 sqrt(N),
with eps = 2^-24, eps64 = 2^-53 and N the nodes compared.  The second term is the rounding
of the stored deviations: each of the nine populations of a node is rounded at eps relative
every step; |f_i - w_i rho0| summed over i is
at most |drho| + 2|u| to first order in u (the equilibrium deviation is
w_i (drho + 3 rho v_i . u)); the nine roundings of a step add up in quadrature (a factor 3)
and the steps' roundings as a random walk (sqrt(n)), since the scheme conserves mass and the
rounding of the conserved density is never damped.  The last term is the oracle's own
resolution: it keeps absolute populations (about w_i rho0) in FP64, so its density deviation
carries the rounding of nine rho0-sized numbers at every node.  A real error of the method (a
wrong force weight, a wrong boundary) moves the density by the force or velocity scale itself,
orders of magnitude above this floor.
"""
import math

import numpy as np

TOL = 1e-5
EPS32 = 2.0 ** -24
EPS64 = 2.0 ** -53


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def drho_bound(drho_o, u_o, steps, tol=TOL, rho0=1.0):
    """Largest acceptable ||drho_gpu - drho_oracle||_2 (see the module docstring)."""
    drho_o = np.asarray(drho_o, float).ravel()
    u_o = np.asarray(u_o, float).reshape(2, -1)
    scale = np.abs(drho_o) + 2.0 * np.hypot(u_o[0], u_o[1])
    return (tol * float(np.linalg.norm(drho_o)) + 3.0 * EPS32 * math.sqrt(max(int(steps), 1)) * float(np.linalg.norm(scale))
            + 9.0 * EPS64 * rho0 * math.sqrt(drho_o.size))


def field_errors(G, R, rho0, X0, steps, S):
    """Errors of the GPU fields G against the oracle's R: relative L2 of u, phi, X - X0 and
    of rho - rho0, the absolute L2 error of rho - rho0 and its bar."""
    out = {}
    out["u"] = rel(G["u"], R["u"])
    if S:
        out["phi"] = rel(G["phi"], R["phi"])
    if X0 is not None and len(X0):
        out["X-X0"] = rel(G["xy"] - X0, R["xy"] - X0)
    dg, do = G["rho"] - rho0, R["rho"] - rho0
    out["drho"] = rel(dg, do)
    out["drho_abs"] = float(np.linalg.norm(dg - do))
    out["drho_bar"] = drho_bound(do, R["u"], steps, rho0=rho0)
    return out


def assert_fields(errs, tol=TOL, what=""):
    """Gate every relative error at tol and the density deviation at its bar."""
    for k in ("u", "phi", "X-X0"):
        if k in errs:
            assert errs[k] <= tol, (what, k, errs[k])
    assert errs["drho_abs"] <= errs["drho_bar"], (what, "rho - rho0", errs["drho_abs"], errs["drho_bar"])


def fmt(errs):
    return {k: f"{v:.2e}" for k, v in errs.items()}
