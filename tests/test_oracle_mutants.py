"""Plant plausible mistakes in the oracle (on the CPU) and check the pins catch each.

Every mutant is a one-token edit of ``oracle/lbib_oracle.c`` of the kind the pins
are meant to guard against: a dropped term, a wrong sign, a wrong index or weight,
a transposed operand.  Each is compiled to a temporary library and the pin suite is
run against it in a subprocess; the suite must fail.
"""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbib_oracle.c")

MUTANTS = {
    "equilibrium quadratic sign": ("(vu * vu - CS2 * uu)", "(vu * vu + CS2 * uu)"),
    "relaxation time inverted": ("c->f[i * nn + x] = fi - (fi - feq[i]) / p->tau + force;",
                                 "c->f[i * nn + x] = fi - (fi - feq[i]) * p->tau + force;"),
    "forcing without rho": ("double force = r * W9[i] *", "double force = W9[i] *"),
    "forcing without 1/cs2": ("(VX[i] * c->ex[x] + VY[i] * c->ey[x]) / CS2;", "(VX[i] * c->ex[x] + VY[i] * c->ey[x]);"),
    "opposite table wrong": ("OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6}", "OPP[9] = {0, 3, 4, 1, 2, 8, 7, 6, 5}"),
    "kernel width": ("cos(M_PI * a / 2.0)", "cos(M_PI * a / 4.0)"),
    "spread stencil origin": ("""    for (int64_t l = 0; l < n; ++l) {
        double x = X[2 * l], y = X[2 * l + 1];
        int64_t i0 = (int64_t)floor(x) - 1, j0 = (int64_t)floor(y) - 1;
        for (int bb = 0; bb < 4; ++bb) {
            int64_t j = j0 + bb;
            if (p->bc_y == ORC_WALLS) { if (j < 0 || j >= p->ny) continue; }
            else j = wrapi(j, p->ny);
            double wy = orc_delta1d(p->delta_kernel, y - (double)(j0 + bb));
            for (int aa = 0; aa < 4; ++aa) {
                int64_t i = wrapi(i0 + aa, p->nx);
                double w = orc_delta1d(p->delta_kernel, x - (double)(i0 + aa)) * wy;
                ex[""", """    for (int64_t l = 0; l < n; ++l) {
        double x = X[2 * l], y = X[2 * l + 1];
        int64_t i0 = (int64_t)floor(x), j0 = (int64_t)floor(y) - 1;
        for (int bb = 0; bb < 4; ++bb) {
            int64_t j = j0 + bb;
            if (p->bc_y == ORC_WALLS) { if (j < 0 || j >= p->ny) continue; }
            else j = wrapi(j, p->ny);
            double wy = orc_delta1d(p->delta_kernel, y - (double)(j0 + bb));
            for (int aa = 0; aa < 4; ++aa) {
                int64_t i = wrapi(i0 + aa, p->nx);
                double w = orc_delta1d(p->delta_kernel, x - (double)(i0 + aa)) * wy;
                ex["""),
    "interp transposed component": ("sy += w * uy[j * p->nx + i];", "sy += w * ux[j * p->nx + i];"),
    "tension sign": ("fx += p->phi_m * (dmx / Lm + dpx / Lp);", "fx += p->phi_m * (dmx / Lm - dpx / Lp);"),
    "spring rest-length index": ("p->k_spring * (Lm - l0[im]) * dmx / Lm;", "p->k_spring * (Lm - l0[i]) * dmx / Lm;"),
    "area force sign": ("double s = p->kappa_area * (A0[c] - A);", "double s = p->kappa_area * (A - A0[c]);"),
    "d2q5 rest weight": ("W5[5] = {1.0 / 3, 1.0 / 6", "W5[5] = {1.0 / 2, 1.0 / 6"),
    "d2q5 no advection": ("out[i] = phi * W5[i] * (1.0 + vu / CS2);", "out[i] = phi * W5[i];"),
    "schnakenberg term": ("if (s == 0) return c[2] * (c[0] - R + R * R * L);", "if (s == 0) return c[2] * (c[0] - R + R * L * L);"),
    "reaction without weights": ("+ W5[i] * R[s];", "+ R[s];"),
    "raster parity": ("if (cnt & 1) {", "if (cnt > 0) {"),
    "specular walls": ("c->fnew[OPP[i] * nn + src] = v;", "c->fnew[i * nn + src] = v;"),
    "diffusivity relation": ("tauD[s] = p->D[s] / CS2 + 0.5;", "tauD[s] = p->D[s] * CS2 + 0.5;"),
    "ade reaction without weights": ("+ R[s] * W5[i];", "+ R[s];"),
    "ade diffusivity relation": ("tauD[s] = 0.5 + p->D[s] / CS2;", "tauD[s] = 0.5 + p->D[s] * CS2;"),
    "ade change without root": ("(d2 == 0.0) ? 0.0 : sqrt(d2) / sqrt(p2);", "(d2 == 0.0) ? 0.0 : d2 / p2;"),
    "ade equilibrium weight": ("double geq = W5[i] * phi[s];", "double geq = W5[0] * phi[s];"),
    "ade specular walls": ("c->gnew[(5 * s + OPP[i]) * nn + src] = v;", "c->gnew[(5 * s + i) * nn + src] = v;"),
    "source subset ignored": ("    if (!c->src) {\n        orc_raster(", "    if (1) {\n        orc_raster("),
    "body force overwrites spread": ("c->ex[x] += p->body[0];", "c->ex[x] = p->body[0];"),
    "moments velocity sign": ("jx += fi * VX[i];\n            jy += fi * VY[i];\n        }\n        c->rho[x] = r;",
                              "jx -= fi * VX[i];\n            jy += fi * VY[i];\n        }\n        c->rho[x] = r;"),
    "no-flux boundary value without the missing weights": ("double phib = known / (1.0 - wm);", "double phib = known;"),
    "no-flux upstream neighbour reversed": ("int64_t yu = y - VY[i], xu = wrapi(x - VX[i], nx);",
                                            "int64_t yu = y + VY[i], xu = wrapi(x + VX[i], nx);"),
    "area controller sign": ("p->mass_source + p->area_alpha * (c->A0[k] - c->area[k]) +",
                             "p->mass_source + p->area_alpha * (c->area[k] - c->A0[k]) +"),
    "mass source added at rest": ("orc_equilibrium9(1.0, vx, vy, e1);", "orc_equilibrium9(1.0, 0.0, 0.0, e1);"),
    "no-flux extrapolation dropped": ("phib = ok2 ? 2.0 * ph[k1] - ph[k2] : ph[k1];", "phib = ok2 ? ph[k1] : ph[k1];"),
    "no-flux interpolation weight": ("double w = qq / (1.0 + qq);", "double w = 1.0 / (1.0 + qq);"),
    "no-flux wall distance from the far end": ("deposit(q, nn, 0, j * nx + wrapi(ir, nx), (double)ir - xc);",
                                               "deposit(q, nn, 0, j * nx + wrapi(ir, nx), xc - (double)(ir - 1));"),
    "no-flux momentum component sign": ("double v = W5[i] * (phib + (VX[i] * jbx + VY[i] * jby) / CS2);",
                                        "double v = W5[i] * (phib + (VX[i] * jbx - VY[i] * jby) / CS2);"),
    "no-flux downstream node reversed": ("int64_t k1 = ok1 ? wrapi(y1, ny) * nx + wrapi(x + VX[i], nx) : k;",
                                         "int64_t k1 = ok1 ? wrapi(y1, ny) * nx + wrapi(x - VX[i], nx) : k;"),
    "half-force shift sign": ("sh[x] = c->ux[x] + 0.5 * c->ex[x];", "sh[x] = c->ux[x] - 0.5 * c->ex[x];"),
    "pressure ring gamma inverted": ("double gamma = c->p.rho0 / r;\n        for (int i = 0; i < 9; ++i) c->f[i * nn + x] *= gamma;",
                                     "double gamma = r / c->p.rho0;\n        for (int i = 0; i < 9; ++i) c->f[i * nn + x] *= gamma;"),
    "node source dropped": ("if (c->nsrc) Sx += c->nsrc[x];", "if (c->nsrc) Sx += 0.0 * c->nsrc[x];"),
    "concentration source from the other species": ("+ p->mass_phi_gamma * phi[0];", "+ p->mass_phi_gamma * phi[1];"),
    "pressure map ignored": ("|| (c->pmap && c->pmap[x]);", "|| (c->pmap && 0);"),
    "bounce-back in the same direction": ("double v = c->gnew[(s * 5 + OPP[i]) * nn + k];",
                                          "double v = c->gnew[(s * 5 + i) * nn + k];"),
    "bounce-back of a set state unstreamed": ("    } else if (c->sent == 2) {\n        memcpy(c->gnew, c->g,",
                                              "    } else if (c->sent == 2) {\n        unstream_species(c, c->gnew); if (0) memcpy(c->gnew, c->g,"),
    "bounce-back restart from the set state's rule": ("        unstream_species(c, c->gnew);\n        c->sent = 1;",
                                                      "        memcpy(c->gnew, c->g, sizeof(double) * 5 * (size_t)p->n_species * (size_t)nn);\n        c->sent = 1;"),
}


def _run_mutant(name, old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutant '{name}' does not match exactly once"
    mpath = os.path.join(tmp, "".join(ch if ch.isalnum() else "_" for ch in name) + ".c")
    with open(mpath, "w") as fh:
        fh.write(src.replace(old, new))
    so = mpath[:-2] + ".so"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
                    "-I", os.path.join(ROOT, "oracle"), "-o", so, mpath, "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=so, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_ade.py"), "-m", "not slow"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_every_planted_mistake_is_caught():
    with tempfile.TemporaryDirectory() as tmp:
        with cf.ThreadPoolExecutor(max_workers=6) as ex:
            futs = [ex.submit(_run_mutant, k, o, n, tmp) for k, (o, n) in MUTANTS.items()]
            results = [f.result() for f in futs]
    survivors = [name for name, rc in results if rc == 0]
    assert not survivors, f"pins did not catch: {survivors}"
