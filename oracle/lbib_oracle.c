/* FP64 CPU oracle of one coupled LBM + IB time step of LBIBCell (arXiv:1503.06726).
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow reference the HIP library is checked
 * against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no code with the HIP library.
 *
 * Build: gcc -O2 -std=c99 -fPIC -shared -ffp-contract=off [-fopenmp]
 * (contraction off, so every product and sum rounds as written; OpenMP, when
 * enabled, only splits the lattice loops by rows, each element is still computed
 * by exactly the statements below).
 *
 * Readings of the paper taken here (where it is silent, garbled or ambiguous):
 *  - D2Q9 numbering: rest, +x, +y, -x, -y, then the diagonals (1,1), (-1,1),
 *    (-1,-1), (1,-1).  The printed diagonal formula has a misplaced parenthesis;
 *    the lattice is the standard one.
 *  - Equilibrium: the printed second-order term lacks c_s^2 and the identity; the
 *    standard form w rho [1 + v.u/cs2 + ((v.u)^2 - cs2 u.u)/(2 cs2^2)] is used.
 *  - Forcing: the literal first-order term dt w rho (v.f)/cs2 of Eq. (bgkequation),
 *    no (1 - 1/(2 tau)) prefactor, velocity u = sum f v / rho without a half-force
 *    shift; f is an acceleration field (spread force plus uniform body acceleration).
 *  - Time level of the interpolated velocity: u^n, the moments of f^n taken before
 *    collision (explicit Euler, the u(x,t) -> U(l,t) labels of Fig. "Algorithm
 *    Overview").  interp_new_u = 1 switches to u^{n+1} for comparison.
 *  - The species see the same u^n; the reaction term is added after collision as
 *    w_i R(phi^n, m^n) (explicit Euler, pre-collision phi), without a tau correction.
 *  - D2Q5 sound speed cs2 = 1/3 (consistent with w0 = 1/3, w1-4 = 1/6), so
 *    tau_D = D/cs2 + 1/2.
 *  - 2-D kernel: delta(r) = delta1D(r_x) delta1D(r_y) (the printed product repeats r).
 *    Stencil: i0 = floor(X) - 1, four points per axis, h = 1.  Nodal forces are
 *    spread without an arc-length weight.  Near walls, points outside the lattice
 *    are dropped.
 *  - Walls (not in the paper's hot path): halfway bounce-back, walls at y = -1/2 and
 *    y = ny - 1/2, for f and for every species (zero flux).  x is always periodic.
 *  - Domain IDs: crossing-number test at integer lattice coordinates, half-open in y
 *    ((a.y > y) != (b.y > y)), strict in x (x < x_crossing); positions are unwrapped,
 *    a cell is tested with its periodic images; overlapping cells: the smallest ID wins.
 *  - Source/decay law: R = sigma [m != 0] - lambda phi.  Schnakenberg:
 *    R_0 = gamma (a - phi0 + phi0^2 phi1), R_1 = gamma (b - phi0^2 phi1).
 *    With a source subset (orc_set_source_cells), [m != 0] becomes "inside at least one
 *    source cell": the crossing test run over the source cells alone.
 *  - Half-force velocity (option interp_half_force): the membrane nodes move with the
 *    interpolated u + f/2, the mean of the momentum before and after the step's forcing,
 *    instead of u; the fluid's collision and reported velocity keep u = sum f v / rho.
 *  - No-flux membranes (a species flag; Suppl. "No-flux Boundary Condition for
 *    Reaction-Advection-Diffusion Equations").  A D2Q5 link is blocked when a membrane edge
 *    crosses it; the crossing nearest to the node fixes the wall distance q in [0, 1] (as a
 *    fraction of the link).  The population that would have arrived across a blocked link is
 *    missing and becomes the equilibrium w_i (phi_b + 3 v_i . j_b) with
 *      j_b = q / (1 + q) phi(x + v_i) u(x + v_i)        (momentum interpolated linearly
 *            between the node one step on, in the direction of the missing population, and
 *            zero at the wall),
 *      phi_b = 2 phi(x + v_i) - phi(x + 2 v_i)          (density extrapolated linearly from
 *            the two nodes on),
 *    taking the moments of the previous step (the ones that step's collision saw), so that a
 *    lattice pass needs nothing of its own step's neighbours.  Where x + 2 v_i is not reachable
 *    (a wall, or a blocked link in between) phi_b = phi(x + v_i); where x + v_i is not,
 *    phi_b = phi(x) and j_b = 0.  Crossings follow the domain-ID test: an edge (A, B) crosses
 *    row y when (A.y > y) != (B.y > y) at x_c = A.x + (y - A.y)(B.x - A.x)/(B.y - A.y), which
 *    cuts the link between columns ceil(x_c) - 1 and ceil(x_c); columns likewise with x and y
 *    exchanged.  The zeroth-order form (option no_flux_zeroth) drops the interpolation and
 *    extrapolation: a population arriving across a membrane (the inside map [m != 0] of this
 *    step differs between the link's ends) becomes the zero-velocity equilibrium w_i phi_b,
 *    with phi_b the node's own concentration solved from the populations that did arrive.
 *    The bounce-back form (option no_flux_bounce, with the first-order form's cut links) is
 *    not the supplement's: the population that would arrive across a cut link becomes the
 *    one the node itself sent towards the membrane in the previous step (its post-collision
 *    population in the opposite direction).  What one side of a link sends the other never
 *    receives, so the species is conserved exactly, also while the membrane moves; the
 *    supplement's equilibrium forms lose the species a moving membrane sweeps over, where the
 *    paper's validations find the integrated concentration converging.  An equilibrium state
 *    set from outside (initial fields) has no previous step: each node is taken to have sent
 *    its own populations.  For populations restored mid-run, the previous post-collision
 *    populations are the ones that streamed into them (streaming and the wall reflection form
 *    a permutation, so they are recovered exactly).
 *    Each form is applied to the streamed populations before the moments of the step; the
 *    reported fields are the sums after the replacement.
 *  - Mass sources and area control (Section "Control of Cell Area"; the supplement's
 *    parameter table makes the lattice source a density per node and step): every node
 *    of cell k in the domain map gains S_k = mass_source + area_alpha (A0_k - A_k) per
 *    step, A_k the shoelace area of the step's positions.  Validation Case III's source,
 *    proportional to the species' concentration, adds mass_phi_gamma phi_0(x), phi_0 the
 *    node's concentration of species 0 as its collision sees it (after the no-flux
 *    replacement).  Case I's point source, and any other per-node source, is a map of
 *    rates per node and step added wherever set (orc_set_node_sources).  The paper does not
 *    say how a source enters the lattice Boltzmann equation; the added mass is taken to move
 *    with the local fluid, S f^eq_i(1, u) added after collision, so rho rises by S and u
 *    is unchanged.
 *  - Pressure boundary (Suppl. "Pressure Boundary Condition for the Fluid Equations"): the
 *    nodes of the lattice's outer ring (the iso-pressure outflow of the validation cases)
 *    and any flagged lattice point (orc_set_pressure_nodes) hold the density rho0; at the
 *    start of each step their populations are multiplied by rho0 / rho (the velocity is
 *    unchanged).  Reported fields and sums are those after the rescaling.
 *  - ADE-only iteration (the steady-state measurement): the species lattices advance
 *    with u = 0 while the fluid, the membranes and the domain map stay frozen; the
 *    relative change after iteration k is ||phi^k - phi^{k-1}||_2 / ||phi^k||_2, with
 *    phi^k = sum_i g_i after k collide-and-stream iterations (0 when both norms vanish).
 */
#include "lbib_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- lattice constants (Suppl. "Lattice Boltzmann Method", D2Q9 and D2Q5 footnotes) ---- */
static const int VX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int VY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const double W5[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
static const double CS2 = 1.0 / 3.0;

struct orc_ctx {
    orc_params p;
    int64_t nn;                   /* nx * ny */
    double *f, *fnew;             /* [9][ny][nx], state f^n (pre-collision) */
    double *g, *gnew;             /* [S][5][ny][nx] */
    double *rho, *ux, *uy;        /* moments of f^n of the current step */
    double *ex, *ey;              /* spread force + body acceleration of the current step */
    int32_t *mask;                /* domain IDs of X^n */
    int32_t n_cells;
    int64_t n_nodes;
    int32_t *off;
    double *X, *F, *l0, *A0, *area;
    uint8_t *src;                 /* [n_cells] source cells of the source/decay law, NULL: all */
    double *phi_prev;             /* [S][ny][nx] concentrations the previous collision saw */
    double *ux_prev, *uy_prev;    /* velocity the previous collision used */
    double *q;                    /* [4][ny][nx] wall distances of blocked links (first-order no-flux) */
    double *nsrc;                 /* [ny][nx] mass source per node and step (point sources), NULL: none */
    int sent;                     /* what gnew holds for the bounce-back no-flux form: 1 the previous
                                     step's post-collision species populations; 0 nothing yet (a
                                     state restored mid-run: unstream it); 2 nothing yet, the state
                                     is an equilibrium set from outside (its own populations) */
    uint8_t *pmap;                /* [ny][nx] pressure points held at rho0, NULL: none */
};

static int64_t wrapi(int64_t i, int64_t n) { int64_t r = i % n; return r < 0 ? r + n : r; }

/* ------------------------------------------------------------------------------------
 * Eq. (1Dkernel): delta1D(r) = (1 + cos(pi |r| / 2)) / 4 for |r| <= 2, else 0.
 * The alternative is Peskin's standard 4-point kernel (the one named in his 2002
 * review), offered because the cosine kernel has a nonzero first moment.
 * ---------------------------------------------------------------------------------- */
double orc_delta1d(int32_t kernel, double r)
{
    double a = fabs(r);
    if (kernel == ORC_DELTA_PESKIN) {
        if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
        if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
        return 0.0;
    }
    if (a <= 2.0) return 0.25 * (1.0 + cos(M_PI * a / 2.0));
    return 0.0;
}

/* Eq. (standardequilibrium), with the garbled second-order term read as
 * ((v_i.u)^2 - cs2 u.u) / (2 cs2^2). */
void orc_equilibrium9(double rho, double ux, double uy, double out[9])
{
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        double vu = VX[i] * ux + VY[i] * uy;
        out[i] = W9[i] * rho * (1.0 + vu / CS2 + (vu * vu - CS2 * uu) / (2.0 * CS2 * CS2));
    }
}

/* D2Q5 equilibrium with the fluid's velocity: g_i^eq = phi w_i (1 + v_i.u / cs2). */
void orc_equilibrium5(double phi, double ux, double uy, double out[5])
{
    for (int i = 0; i < 5; ++i) {
        double vu = VX[i] * ux + VY[i] * uy;
        out[i] = phi * W5[i] * (1.0 + vu / CS2);
    }
}

/* Reaction terms (the paper's CDESolver hook; Schnakenberg from "Turing Patterning").
 * phi: the S local concentrations; m: the local domain ID. */
double orc_reaction(const orc_params* p, int32_t s, const double* phi, int32_t m)
{
    const double* c = p->rc[s];
    switch (p->reaction[s]) {
    case ORC_REACT_SOURCE_DECAY:
        return (m != 0 ? c[0] : 0.0) - c[1] * phi[s];
    case ORC_REACT_SCHNAKENBERG: {
        double R = phi[0], L = phi[1];
        if (s == 0) return c[2] * (c[0] - R + R * R * L);
        return c[2] * (c[1] - R * R * L);
    }
    default:
        return 0.0;
    }
}

/* ------------------------------------------------------------------------------------
 * Membrane forces, per node, in the paper's per-node form:
 *  tension   F_i = phi_m ( (x_{i-1}-x_i)/|x_{i-1}-x_i| + (x_{i+1}-x_i)/|x_{i+1}-x_i| )
 *            (Eq. membraneforce);
 *  springs   F_i = k (|x_{i+1}-x_i| - l0_i) unit(x_{i+1}-x_i)
 *                + k (|x_{i-1}-x_i| - l0_{i-1}) unit(x_{i-1}-x_i)
 *            (Hookean membrane springs; l0_i is the rest length of edge (i, i+1));
 *  area      F_i = kappa_A (A0 - A) dA/dX_i, A = 1/2 sum (x_k y_{k+1} - x_{k+1} y_k)
 *            (gradient of kappa_A (A - A0)^2 / 2; not in the paper, used by the tiny
 *            workload's area pressure).
 * ---------------------------------------------------------------------------------- */
void orc_forces(const orc_params* p, int32_t n_cells, const int32_t* off, const double* X,
                const double* l0, const double* A0, double* F, double* area)
{
    for (int32_t c = 0; c < n_cells; ++c) {
        int64_t a = off[c], b = off[c + 1], n = b - a;
        double A = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            int64_t i = a + k, j = a + (k + 1) % n;
            A += X[2 * i] * X[2 * j + 1] - X[2 * j] * X[2 * i + 1];
        }
        A *= 0.5;
        if (area) area[c] = A;
        for (int64_t k = 0; k < n; ++k) {
            int64_t i = a + k, ip = a + (k + 1) % n, im = a + (k + n - 1) % n;
            double dpx = X[2 * ip] - X[2 * i], dpy = X[2 * ip + 1] - X[2 * i + 1];
            double dmx = X[2 * im] - X[2 * i], dmy = X[2 * im + 1] - X[2 * i + 1];
            double Lp = sqrt(dpx * dpx + dpy * dpy), Lm = sqrt(dmx * dmx + dmy * dmy);
            double fx = 0.0, fy = 0.0;
            /* tension */
            fx += p->phi_m * (dmx / Lm + dpx / Lp);
            fy += p->phi_m * (dmy / Lm + dpy / Lp);
            /* springs */
            fx += p->k_spring * (Lp - l0[i]) * dpx / Lp + p->k_spring * (Lm - l0[im]) * dmx / Lm;
            fy += p->k_spring * (Lp - l0[i]) * dpy / Lp + p->k_spring * (Lm - l0[im]) * dmy / Lm;
            /* area pressure */
            double s = p->kappa_area * (A0[c] - A);
            fx += s * 0.5 * (X[2 * ip + 1] - X[2 * im + 1]);
            fy += s * 0.5 * (X[2 * im] - X[2 * ip]);
            F[2 * i] = fx;
            F[2 * i + 1] = fy;
        }
    }
}

/* Eq. (forcedistribution) discretised: f(x) += F_l delta(x - X_l) over the 4x4
 * stencil i0 = floor(X) - 1 .. i0 + 3, nodes in index order.  ex/ey accumulate. */
void orc_spread(const orc_params* p, int64_t n, const double* X, const double* F,
                double* ex, double* ey)
{
    for (int64_t l = 0; l < n; ++l) {
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
                ex[j * p->nx + i] += w * F[2 * l];
                ey[j * p->nx + i] += w * F[2 * l + 1];
            }
        }
    }
}

/* Eq. (conversion2) discretised: U_l = sum_x u(x) delta(x - X_l), same stencil. */
void orc_interp(const orc_params* p, int64_t n, const double* X, const double* ux,
                const double* uy, double* U)
{
    for (int64_t l = 0; l < n; ++l) {
        double x = X[2 * l], y = X[2 * l + 1];
        int64_t i0 = (int64_t)floor(x) - 1, j0 = (int64_t)floor(y) - 1;
        double sx = 0.0, sy = 0.0;
        for (int bb = 0; bb < 4; ++bb) {
            int64_t j = j0 + bb;
            if (p->bc_y == ORC_WALLS) { if (j < 0 || j >= p->ny) continue; }
            else j = wrapi(j, p->ny);
            double wy = orc_delta1d(p->delta_kernel, y - (double)(j0 + bb));
            for (int aa = 0; aa < 4; ++aa) {
                int64_t i = wrapi(i0 + aa, p->nx);
                double w = orc_delta1d(p->delta_kernel, x - (double)(i0 + aa)) * wy;
                sx += w * ux[j * p->nx + i];
                sy += w * uy[j * p->nx + i];
            }
        }
        U[2 * l] = sx;
        U[2 * l + 1] = sy;
    }
}

/* Domain IDs on the lattice (Section "Cell Representation": the domain on the left
 * of each CCW connection carries the cell's ID, zero is the extracellular space).
 * For each cell in ascending ID, each lattice node (integer coordinates) of its
 * bounding box, in unwrapped coordinates (which covers the periodic images), is
 * inside when the number of edges crossed by the ray to +x is odd; a node keeps the
 * first (smallest) ID that claims it.  Returns the number of nodes claimed twice. */
int64_t orc_raster(const orc_params* p, int32_t n_cells, const int32_t* off, const double* X,
                   int32_t* mask)
{
    int64_t overlaps = 0;
    int64_t nx = p->nx, ny = p->ny;
    memset(mask, 0, sizeof(int32_t) * (size_t)(nx * ny));
    double* xc = NULL;
    size_t cap = 0;
    for (int32_t c = 0; c < n_cells; ++c) {
        int64_t a = off[c], b = off[c + 1], n = b - a;
        double xmin = X[2 * a], xmax = xmin, ymin = X[2 * a + 1], ymax = ymin;
        for (int64_t k = a; k < b; ++k) {
            if (X[2 * k] < xmin) xmin = X[2 * k];
            if (X[2 * k] > xmax) xmax = X[2 * k];
            if (X[2 * k + 1] < ymin) ymin = X[2 * k + 1];
            if (X[2 * k + 1] > ymax) ymax = X[2 * k + 1];
        }
        if ((size_t)n > cap) { cap = (size_t)n; xc = (double*)realloc(xc, cap * sizeof(double)); }
        for (int64_t py = (int64_t)ceil(ymin); py <= (int64_t)floor(ymax); ++py) {
            /* crossings of this row: (a.y > py) != (b.y > py) */
            int64_t nc = 0;
            for (int64_t k = 0; k < n; ++k) {
                const double* A = &X[2 * (a + k)];
                const double* B = &X[2 * (a + (k + 1) % n)];
                if ((A[1] > (double)py) != (B[1] > (double)py))
                    xc[nc++] = A[0] + ((double)py - A[1]) * (B[0] - A[0]) / (B[1] - A[1]);
            }
            if (nc == 0) continue;
            int64_t jj;
            if (p->bc_y == ORC_WALLS) { if (py < 0 || py >= ny) continue; jj = py; }
            else jj = wrapi(py, ny);
            for (int64_t px = (int64_t)ceil(xmin); px <= (int64_t)floor(xmax); ++px) {
                int64_t cnt = 0;
                for (int64_t q = 0; q < nc; ++q)
                    if ((double)px < xc[q]) ++cnt;
                if (cnt & 1) {
                    int32_t* m = &mask[jj * nx + wrapi(px, nx)];
                    if (*m == 0) *m = c + 1;
                    else ++overlaps;
                }
            }
        }
    }
    free(xc);
    return overlaps;
}

/* Wall distances of the D2Q5 links crossed by membrane edges (Suppl. "No-flux Boundary
 * Condition ..."; the crossings follow the domain-ID test of Section "Cell Representation").
 * q[d][y][x], d = 0..3 for directions +x, +y, -x, -y, is the distance from node (x, y) to the
 * nearest crossing on the link to its upstream neighbour (x, y) - v_{d+1}, as a fraction of the
 * link, or +inf where no edge crosses that link.  An edge (A, B) crossing row y at x_c cuts the
 * link between columns ceil(x_c) - 1 and ceil(x_c): the right node (population arriving in +x)
 * is ceil(x_c) - x_c away, the left one (arriving in -x) x_c - ceil(x_c) + 1; columns likewise.
 * Links to rows beyond a wall do not exist. */
static void deposit(double* q, int64_t nn, int d, int64_t k, double v)
{
    if (v < q[d * nn + k]) q[d * nn + k] = v;
}

void orc_link_crossings(const orc_params* p, int32_t n_cells, const int32_t* off, const double* X,
                        double* q)
{
    int64_t nx = p->nx, ny = p->ny, nn = nx * ny;
    for (int64_t k = 0; k < 4 * nn; ++k) q[k] = INFINITY;
    for (int32_t c = 0; c < n_cells; ++c) {
        int64_t a = off[c], n = off[c + 1] - a;
        for (int64_t k = 0; k < n; ++k) {
            const double* A = &X[2 * (a + k)];
            const double* B = &X[2 * (a + (k + 1) % n)];
            /* rows y with (A.y > y) != (B.y > y): the horizontal links of row y */
            int64_t lo = (int64_t)floor(fmin(A[1], B[1])), hi = (int64_t)floor(fmax(A[1], B[1]));
            for (int64_t py = lo; py <= hi; ++py) {
                double yy = (double)py;
                if ((A[1] > yy) == (B[1] > yy)) continue;
                int64_t j;
                if (p->bc_y == ORC_WALLS) { if (py < 0 || py >= ny) continue; j = py; }
                else j = wrapi(py, ny);
                double xc = A[0] + (yy - A[1]) * (B[0] - A[0]) / (B[1] - A[1]);
                int64_t ir = (int64_t)ceil(xc);
                deposit(q, nn, 0, j * nx + wrapi(ir, nx), (double)ir - xc);
                deposit(q, nn, 2, j * nx + wrapi(ir - 1, nx), xc - (double)(ir - 1));
            }
            /* columns x with (A.x > x) != (B.x > x): the vertical links of column x */
            lo = (int64_t)floor(fmin(A[0], B[0]));
            hi = (int64_t)floor(fmax(A[0], B[0]));
            for (int64_t px = lo; px <= hi; ++px) {
                double xx = (double)px;
                if ((A[0] > xx) == (B[0] > xx)) continue;
                double yc = A[1] + (xx - A[0]) * (B[1] - A[1]) / (B[0] - A[0]);
                int64_t jt = (int64_t)ceil(yc), i = wrapi(px, nx);
                if (p->bc_y == ORC_WALLS) {
                    if (jt >= 1 && jt < ny) {   /* both rows jt - 1 and jt inside the lattice */
                        deposit(q, nn, 1, jt * nx + i, (double)jt - yc);
                        deposit(q, nn, 3, (jt - 1) * nx + i, yc - (double)(jt - 1));
                    }
                } else {
                    deposit(q, nn, 1, wrapi(jt, ny) * nx + i, (double)jt - yc);
                    deposit(q, nn, 3, wrapi(jt - 1, ny) * nx + i, yc - (double)(jt - 1));
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------------------
 * simulation context
 * ---------------------------------------------------------------------------------- */
orc_ctx* orc_create(const orc_params* p)
{
    orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
    c->p = *p;
    c->nn = (int64_t)p->nx * p->ny;
    size_t nn = (size_t)c->nn;
    int S = p->n_species;
    c->f = (double*)malloc(sizeof(double) * 9 * nn);
    c->fnew = (double*)malloc(sizeof(double) * 9 * nn);
    c->g = (double*)malloc(sizeof(double) * (size_t)(5 * (S > 0 ? S : 1)) * nn);
    c->gnew = (double*)malloc(sizeof(double) * (size_t)(5 * (S > 0 ? S : 1)) * nn);
    c->rho = (double*)malloc(sizeof(double) * nn);
    c->ux = (double*)malloc(sizeof(double) * nn);
    c->uy = (double*)malloc(sizeof(double) * nn);
    c->ex = (double*)calloc(nn, sizeof(double));
    c->ey = (double*)calloc(nn, sizeof(double));
    c->mask = (int32_t*)calloc(nn, sizeof(int32_t));
    c->phi_prev = (double*)calloc((size_t)(S > 0 ? S : 1) * nn, sizeof(double));
    c->ux_prev = (double*)calloc(nn, sizeof(double));
    c->uy_prev = (double*)calloc(nn, sizeof(double));
    c->q = (double*)malloc(sizeof(double) * 4 * nn);
    for (size_t k = 0; k < 4 * nn; ++k) c->q[k] = INFINITY;
    orc_set_fields(c, NULL, NULL, NULL);
    return c;
}

void orc_destroy(orc_ctx* c)
{
    if (!c) return;
    free(c->f); free(c->fnew); free(c->g); free(c->gnew);
    free(c->rho); free(c->ux); free(c->uy); free(c->ex); free(c->ey); free(c->mask);
    free(c->off); free(c->X); free(c->F); free(c->l0); free(c->A0); free(c->area);
    free(c->src);
    free(c->phi_prev); free(c->ux_prev); free(c->uy_prev); free(c->q);
    free(c->nsrc); free(c->pmap);
    free(c);
}

int32_t orc_set_cells(orc_ctx* c, int32_t n_cells, const int32_t* off, const double* X,
                      const double* rest_len, const double* rest_area)
{
    free(c->off); free(c->X); free(c->F); free(c->l0); free(c->A0); free(c->area);
    free(c->src);
    c->src = NULL;
    c->n_cells = n_cells;
    c->n_nodes = off[n_cells];
    size_t N = (size_t)c->n_nodes;
    c->off = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_cells + 1));
    memcpy(c->off, off, sizeof(int32_t) * (size_t)(n_cells + 1));
    c->X = (double*)malloc(sizeof(double) * 2 * (N ? N : 1));
    c->F = (double*)calloc(2 * (N ? N : 1), sizeof(double));
    c->l0 = (double*)malloc(sizeof(double) * (N ? N : 1));
    c->A0 = (double*)malloc(sizeof(double) * (size_t)(n_cells ? n_cells : 1));
    c->area = (double*)malloc(sizeof(double) * (size_t)(n_cells ? n_cells : 1));
    memcpy(c->X, X, sizeof(double) * 2 * N);
    for (int32_t q = 0; q < n_cells; ++q) {
        int64_t a = off[q], b = off[q + 1], n = b - a;
        double A = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            int64_t i = a + k, j = a + (k + 1) % n;
            double dx = X[2 * j] - X[2 * i], dy = X[2 * j + 1] - X[2 * i + 1];
            c->l0[i] = rest_len ? rest_len[i] : sqrt(dx * dx + dy * dy);
            A += X[2 * i] * X[2 * j + 1] - X[2 * j] * X[2 * i + 1];
        }
        c->A0[q] = rest_area ? rest_area[q] : 0.5 * A;
    }
    return 0;
}

/* The "previous step" moments of a state set from outside (initial fields, populations): the
 * sums of its populations. */
static void prev_from_populations(orc_ctx* c)
{
    int64_t nn = c->nn;
    c->sent = 0;
    for (int64_t x = 0; x < nn; ++x) {
        double r = 0.0, jx = 0.0, jy = 0.0;
        for (int i = 0; i < 9; ++i) {
            double fi = c->f[i * nn + x];
            r += fi; jx += fi * VX[i]; jy += fi * VY[i];
        }
        c->ux_prev[x] = jx / r;
        c->uy_prev[x] = jy / r;
        for (int s = 0; s < c->p.n_species; ++s) {
            double sum = 0.0;
            for (int i = 0; i < 5; ++i) sum += c->g[(s * 5 + i) * nn + x];
            c->phi_prev[s * nn + x] = sum;
        }
    }
}

/* Equilibrium initial state: f = f^eq(rho, u), g_s = g^eq(phi_s, u).  NULL fields take
 * rho0, zero velocity and zero concentration. */
void orc_set_fields(orc_ctx* c, const double* rho, const double* u, const double* phi)
{
    int64_t nn = c->nn;
    double e9[9], e5[5];
    for (int64_t x = 0; x < nn; ++x) {
        double r = rho ? rho[x] : c->p.rho0;
        double vx = u ? u[x] : 0.0, vy = u ? u[nn + x] : 0.0;
        orc_equilibrium9(r, vx, vy, e9);
        for (int i = 0; i < 9; ++i) c->f[i * nn + x] = e9[i];
        for (int s = 0; s < c->p.n_species; ++s) {
            orc_equilibrium5(phi ? phi[s * nn + x] : 0.0, vx, vy, e5);
            for (int i = 0; i < 5; ++i) c->g[(s * 5 + i) * nn + x] = e5[i];
        }
    }
    prev_from_populations(c);
    c->sent = 2;
}

void orc_set_source_cells(orc_ctx* c, const uint8_t* src)
{
    free(c->src);
    c->src = NULL;
    if (!src || c->n_cells == 0) return;
    c->src = (uint8_t*)malloc((size_t)c->n_cells);
    memcpy(c->src, src, (size_t)c->n_cells);
}

/* Point (or any per-node) mass sources: node x gains rate[x] per step, added as
 * rate[x] f^eq_i(1, u) after the collision like the cells' sources; NULL removes them. */
void orc_set_node_sources(orc_ctx* c, const double* rate)
{
    free(c->nsrc);
    c->nsrc = NULL;
    if (!rate) return;
    c->nsrc = (double*)malloc(sizeof(double) * (size_t)c->nn);
    memcpy(c->nsrc, rate, sizeof(double) * (size_t)c->nn);
}

/* Pressure points anywhere in the lattice (Suppl. "Pressure Boundary Condition for the Fluid
 * Equations"): every flagged node is held at rho0 as the outer ring is; NULL removes them. */
void orc_set_pressure_nodes(orc_ctx* c, const uint8_t* flags)
{
    free(c->pmap);
    c->pmap = NULL;
    if (!flags) return;
    c->pmap = (uint8_t*)malloc((size_t)c->nn);
    memcpy(c->pmap, flags, (size_t)c->nn);
}

/* The map the source/decay law reads: domain IDs of all cells, or, with a source subset,
 * nonzero exactly at the nodes inside at least one source cell (the same crossing test
 * over the source cells alone). */
static void source_map(orc_ctx* c, int32_t* m)
{
    if (!c->src) {
        orc_raster(&c->p, c->n_cells, c->off, c->X, m);
        return;
    }
    int32_t ns = 0;
    int64_t nodes = 0;
    for (int32_t q = 0; q < c->n_cells; ++q)
        if (c->src[q]) { ++ns; nodes += c->off[q + 1] - c->off[q]; }
    int32_t* off = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ns + 1));
    double* X = (double*)malloc(sizeof(double) * 2 * (size_t)(nodes ? nodes : 1));
    off[0] = 0;
    int32_t k = 0;
    for (int32_t q = 0; q < c->n_cells; ++q) {
        if (!c->src[q]) continue;
        int64_t a = c->off[q], n = c->off[q + 1] - a;
        memcpy(X + 2 * (int64_t)off[k], c->X + 2 * a, sizeof(double) * 2 * (size_t)n);
        off[k + 1] = off[k] + (int32_t)n;
        ++k;
    }
    orc_raster(&c->p, ns, off, X, m);
    free(off);
    free(X);
}

void orc_source_map(orc_ctx* c, int32_t* out)
{
    source_map(c, out);
}

static int cell_sources(const orc_params* p)
{
    return p->mass_source != 0.0 || p->area_alpha != 0.0 || p->mass_phi_gamma != 0.0;
}

static int needs_mask(const orc_params* p)
{
    for (int s = 0; s < p->n_species; ++s)
        if (p->reaction[s] == ORC_REACT_SOURCE_DECAY || (p->no_flux[s] && p->no_flux_zeroth)) return 1;
    return cell_sources(p);
}

static int any_no_flux(const orc_params* p)
{
    int nf = 0;
    for (int s = 0; s < p->n_species; ++s) nf |= p->no_flux[s];
    return nf;
}

/* No-flux membranes for a species (Section "Signalling"; Suppl. "No-flux Boundary Condition
 * for Reaction-Advection-Diffusion Equations"), zeroth-order reading: a population that
 * arrived at x across a membrane (its upstream node x - v_i lies inside a cell and x does
 * not, or the reverse; m is the domain map of this step's positions) is missing and becomes
 * the equilibrium at the wall's zero velocity, w_i phi_b, with phi_b the node's own
 * concentration: phi_b = (populations that arrived) + (sum of the missing w_i) phi_b.  A
 * population reflected by a wall is not missing. */
static void no_flux_replace(orc_ctx* c, const int32_t* m, double* g)
{
    const orc_params* p = &c->p;
    int64_t nx = p->nx, ny = p->ny, nn = c->nn;
    for (int s = 0; s < p->n_species; ++s) {
        if (!p->no_flux[s]) continue;
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t k = y * nx + x;
                int in = m[k] != 0;
                double known = g[(s * 5) * nn + k], wm = 0.0;
                int miss[5] = {0, 0, 0, 0, 0};
                for (int i = 1; i < 5; ++i) {
                    int64_t yu = y - VY[i], xu = wrapi(x - VX[i], nx);
                    int across = 0;
                    if (!(p->bc_y == ORC_WALLS && (yu < 0 || yu >= ny)))
                        across = (m[wrapi(yu, ny) * nx + xu] != 0) != in;
                    if (across) { miss[i] = 1; wm += W5[i]; }
                    else known += g[(s * 5 + i) * nn + k];
                }
                if (wm == 0.0) continue;
                double phib = known / (1.0 - wm);
                for (int i = 1; i < 5; ++i)
                    if (miss[i]) g[(s * 5 + i) * nn + k] = W5[i] * phib;
            }
    }
}

/* No-flux membranes, the supplement's first-order condition (see the readings above): every
 * population whose link is blocked (q finite) becomes w_i (phi_b + 3 v_i . j_b), from the wall
 * distance q and the previous step's moments of the nodes one and two steps on along v_i.
 * out receives, per species s and direction i, the replacement value (or leaves g alone when
 * out is NULL and writes into g). */
static void no_flux_first(orc_ctx* c, const double* q, double* g, int only_s, double* out)
{
    const orc_params* p = &c->p;
    int64_t nx = p->nx, ny = p->ny, nn = c->nn;
    for (int s = 0; s < p->n_species; ++s) {
        if (!p->no_flux[s] || (only_s >= 0 && s != only_s)) continue;
        const double* ph = c->phi_prev + s * nn;
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t k = y * nx + x;
                for (int i = 1; i < 5; ++i) {
                    double qq = q[(i - 1) * nn + k];
                    if (qq == INFINITY) continue;
                    /* the nodes one and two steps on in the direction of the missing population,
                     * each reachable when it lies inside the lattice and no membrane blocks the
                     * link leading to it */
                    int64_t y1 = y + VY[i], y2 = y + 2 * VY[i];
                    int ok1 = 1, ok2 = 1;
                    if (p->bc_y == ORC_WALLS) {
                        if (y1 < 0 || y1 >= ny) ok1 = 0;
                        if (y2 < 0 || y2 >= ny) ok2 = 0;
                    }
                    int64_t k1 = ok1 ? wrapi(y1, ny) * nx + wrapi(x + VX[i], nx) : k;
                    int64_t k2 = ok2 ? wrapi(y2, ny) * nx + wrapi(x + 2 * VX[i], nx) : k;
                    if (ok1 && q[(i - 1) * nn + k1] != INFINITY) ok1 = 0;
                    if (!ok1 || q[(i - 1) * nn + k2] != INFINITY) ok2 = 0;
                    double phib, jbx = 0.0, jby = 0.0;
                    if (!ok1) {
                        phib = ph[k];
                    } else {
                        double w = qq / (1.0 + qq);
                        jbx = w * ph[k1] * c->ux_prev[k1];
                        jby = w * ph[k1] * c->uy_prev[k1];
                        phib = ok2 ? 2.0 * ph[k1] - ph[k2] : ph[k1];
                    }
                    double v = W5[i] * (phib + (VX[i] * jbx + VY[i] * jby) / CS2);
                    if (out) out[(i - 1) * nn + k] = v;
                    else g[(s * 5 + i) * nn + k] = v;
                }
            }
    }
}

/* The populations that streamed into the current state, unstreamed: sent[i][x] is the
 * population node x sent in direction i (free flight to x + v_i, or back to x itself in the
 * opposite direction where x + v_i lies beyond a wall). */
static void unstream_species(orc_ctx* c, double* sent)
{
    const orc_params* p = &c->p;
    int64_t nx = p->nx, ny = p->ny, nn = c->nn;
    for (int s = 0; s < p->n_species; ++s)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x)
                for (int i = 0; i < 5; ++i) {
                    int64_t yd = y + VY[i], xd = wrapi(x + VX[i], nx);
                    double v;
                    if (p->bc_y == ORC_WALLS && (yd < 0 || yd >= ny))
                        v = c->g[(s * 5 + OPP[i]) * nn + y * nx + x];
                    else
                        v = c->g[(s * 5 + i) * nn + wrapi(yd, ny) * nx + xd];
                    sent[(s * 5 + i) * nn + y * nx + x] = v;
                }
}

/* No-flux membranes in the bounce-back form: every population whose link is cut (q finite)
 * becomes the population the node sent in the opposite direction in the previous step.  An
 * equilibrium state set from outside has no previous step: each node is taken to have sent
 * its own populations.  out as in no_flux_first. */
static void no_flux_bounce(orc_ctx* c, const double* q, double* g, int only_s, double* out)
{
    const orc_params* p = &c->p;
    int64_t nn = c->nn;
    if (c->sent == 0) {
        unstream_species(c, c->gnew);
        c->sent = 1;
    } else if (c->sent == 2) {
        memcpy(c->gnew, c->g, sizeof(double) * 5 * (size_t)p->n_species * (size_t)nn);
    }
    for (int s = 0; s < p->n_species; ++s) {
        if (!p->no_flux[s] || (only_s >= 0 && s != only_s)) continue;
        for (int64_t k = 0; k < nn; ++k)
            for (int i = 1; i < 5; ++i) {
                if (q[(i - 1) * nn + k] == INFINITY) continue;
                double v = c->gnew[(s * 5 + OPP[i]) * nn + k];
                if (out) out[(i - 1) * nn + k] = v;
                else g[(s * 5 + i) * nn + k] = v;
            }
    }
}

static void moments(orc_ctx* c)
{
    int64_t nn = c->nn;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < nn; ++x) {
        double r = 0.0, jx = 0.0, jy = 0.0;
        for (int i = 0; i < 9; ++i) {
            double fi = c->f[i * nn + x];
            r += fi;
            jx += fi * VX[i];
            jy += fi * VY[i];
        }
        c->rho[x] = r;
        c->ux[x] = jx / r;
        c->uy[x] = jy / r;
    }
}

/* One coupled step, in the order of Fig. "Algorithm Overview":
 *  1 membrane forces F(X^n); 2 spread F -> f(x) (+ body acceleration);
 *  3 domain IDs m^n of X^n (only when a reaction reads them);
 *  4 collision of fluid (Eq. bgkequation) and species (D2Q5 equation) with u^n;
 *  5 streaming (free flight), halfway bounce-back at walls;
 *  6 interpolation of u^n to the nodes (Eq. conversion2) and explicit move. */
/* is node x (row-major index) on the lattice's outer ring? */
static int on_ring(const orc_params* p, int64_t x)
{
    int64_t i = x % p->nx, j = x / p->nx;
    return i == 0 || i == p->nx - 1 || j == 0 || j == p->ny - 1;
}

/* is node x a pressure point: on the outer ring (pressure_ring) or flagged in the map? */
static int pressure_node(const orc_ctx* c, int64_t x)
{
    return (c->p.pressure_ring && on_ring(&c->p, x)) || (c->pmap && c->pmap[x]);
}

/* Pressure boundary: the populations of every pressure point scaled by gamma = rho0 / rho, so
 * the node's density becomes rho0 and its velocity sum f v / sum f stays as it was. */
static void pressure_ring(orc_ctx* c)
{
    int64_t nn = c->nn;
    for (int64_t x = 0; x < nn; ++x) {
        if (!pressure_node(c, x)) continue;
        double r = 0.0;
        for (int i = 0; i < 9; ++i) r += c->f[i * nn + x];
        double gamma = c->p.rho0 / r;
        for (int i = 0; i < 9; ++i) c->f[i * nn + x] *= gamma;
    }
}

static void step_once(orc_ctx* c)
{
    const orc_params* p = &c->p;
    int64_t nx = p->nx, ny = p->ny, nn = c->nn;
    int S = p->n_species;

    /* 0: pressure boundary on the outer ring and at the pressure points */
    if (p->pressure_ring || c->pmap) pressure_ring(c);

    /* 1-2: forces and spreading */
    memset(c->ex, 0, sizeof(double) * (size_t)nn);
    memset(c->ey, 0, sizeof(double) * (size_t)nn);
    if (c->n_cells > 0) {
        orc_forces(p, c->n_cells, c->off, c->X, c->l0, c->A0, c->F, c->area);
        orc_spread(p, c->n_nodes, c->X, c->F, c->ex, c->ey);
    }
    for (int64_t x = 0; x < nn; ++x) { c->ex[x] += p->body[0]; c->ey[x] += p->body[1]; }

    /* 3: domain IDs (the map the source term and no-flux membranes read); populations that
     * arrived across a no-flux membrane are replaced before the moments */
    if (needs_mask(p)) source_map(c, c->mask);
    else memset(c->mask, 0, sizeof(int32_t) * (size_t)nn);
    if (any_no_flux(p) && c->n_cells > 0) {
        if (p->no_flux_zeroth) {
            no_flux_replace(c, c->mask, c->g);
        } else {
            orc_link_crossings(p, c->n_cells, c->off, c->X, c->q);
            if (p->no_flux_bounce) no_flux_bounce(c, c->q, c->g, -1, NULL);
            else no_flux_first(c, c->q, c->g, -1, NULL);
        }
    }

    /* the cell of every node for the mass sources: the domain map, or, when a source subset
     * narrowed that map, the crossing test over all cells */
    const int mass = cell_sources(p);
    int32_t* cell_map = c->mask;
    if (mass && c->src) {
        cell_map = (int32_t*)malloc(sizeof(int32_t) * (size_t)nn);
        orc_raster(p, c->n_cells, c->off, c->X, cell_map);
    }

    /* 4: moments and collision (post-collision values into f / g in place) */
    moments(c);
    double tauD[2];
    for (int s = 0; s < S; ++s) tauD[s] = p->D[s] / CS2 + 0.5;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < nn; ++x) {
        double feq[9], geq[5], phi[2] = {0.0, 0.0}, R[2];
        double r = c->rho[x], vx = c->ux[x], vy = c->uy[x];
        orc_equilibrium9(r, vx, vy, feq);
        for (int i = 0; i < 9; ++i) {
            double fi = c->f[i * nn + x];
            double force = r * W9[i] * (VX[i] * c->ex[x] + VY[i] * c->ey[x]) / CS2;
            c->f[i * nn + x] = fi - (fi - feq[i]) / p->tau + force;
        }
        for (int s = 0; s < S; ++s) {
            double sum = 0.0;
            for (int i = 0; i < 5; ++i) sum += c->g[(s * 5 + i) * nn + x];
            phi[s] = sum;
            c->phi_prev[s * nn + x] = sum;      /* read by the next step's no-flux replacement */
        }
        /* mass sources, moving with the fluid: the node's cell (the map holds cell + 1) gives
         * S_k + mass_phi_gamma phi_0(x), the node-source map its own rate */
        double Sx = 0.0;
        if (mass && cell_map[x] > 0) {
            int32_t k = cell_map[x] - 1;
            Sx = p->mass_source + p->area_alpha * (c->A0[k] - c->area[k]) + p->mass_phi_gamma * phi[0];
        }
        if (c->nsrc) Sx += c->nsrc[x];
        if (Sx != 0.0) {
            double e1[9];
            orc_equilibrium9(1.0, vx, vy, e1);
            for (int i = 0; i < 9; ++i) c->f[i * nn + x] += Sx * e1[i];
        }
        c->ux_prev[x] = vx;
        c->uy_prev[x] = vy;
        for (int s = 0; s < S; ++s) R[s] = orc_reaction(p, s, phi, c->mask[x]);
        for (int s = 0; s < S; ++s) {
            orc_equilibrium5(phi[s], vx, vy, geq);
            for (int i = 0; i < 5; ++i) {
                double gi = c->g[(s * 5 + i) * nn + x];
                c->g[(s * 5 + i) * nn + x] = gi - (gi - geq[i]) / tauD[s] + W5[i] * R[s];
            }
        }
    }

    if (cell_map != c->mask) free(cell_map);

    /* 5: streaming f(x + v_i, t + 1) = f*(x, t); a population leaving through a wall
     * returns to its node in the opposite direction (halfway bounce-back). */
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < ny; ++y) {
        for (int64_t x = 0; x < nx; ++x) {
            int64_t src = y * nx + x;
            for (int i = 0; i < 9; ++i) {
                int64_t xd = wrapi(x + VX[i], nx), yd = y + VY[i];
                double v = c->f[i * nn + src];
                if (p->bc_y == ORC_WALLS && (yd < 0 || yd >= ny)) {
                    if (yd >= ny && p->wall_u_top != 0.0)
                        v -= 2.0 * W9[i] * c->rho[src] * (VX[i] * p->wall_u_top) / CS2;
                    c->fnew[OPP[i] * nn + src] = v;
                } else {
                    c->fnew[i * nn + wrapi(yd, ny) * nx + xd] = v;
                }
            }
            for (int s = 0; s < S; ++s) {
                for (int i = 0; i < 5; ++i) {
                    int64_t xd = wrapi(x + VX[i], nx), yd = y + VY[i];
                    double v = c->g[(s * 5 + i) * nn + src];
                    if (p->bc_y == ORC_WALLS && (yd < 0 || yd >= ny))
                        c->gnew[(s * 5 + OPP[i]) * nn + src] = v;
                    else
                        c->gnew[(s * 5 + i) * nn + wrapi(yd, ny) * nx + xd] = v;
                }
            }
        }
    }
    double* t = c->f; c->f = c->fnew; c->fnew = t;
    t = c->g; c->g = c->gnew; c->gnew = t;
    c->sent = 1;                          /* gnew: this step's post-collision populations */

    /* 6: interpolate and move (positions stay unwrapped) */
    if (c->n_nodes > 0) {
        double* U = (double*)malloc(sizeof(double) * 2 * (size_t)c->n_nodes);
        if (p->interp_new_u) {
            /* alternative reading: the velocity after advancing the fluid */
            double *r2 = c->rho, *x2 = c->ux, *y2 = c->uy;
            double* tmp = (double*)malloc(sizeof(double) * 3 * (size_t)nn);
            c->rho = tmp; c->ux = tmp + nn; c->uy = tmp + 2 * nn;
            moments(c);
            orc_interp(p, c->n_nodes, c->X, c->ux, c->uy, U);
            c->rho = r2; c->ux = x2; c->uy = y2;
            free(tmp);
        } else if (p->interp_half_force) {
            /* the half-force-shifted velocity u + f/2: the mean of the momentum before and
             * after the forcing term of this step (f the spread and body acceleration) */
            double* sh = (double*)malloc(sizeof(double) * 2 * (size_t)nn);
            for (int64_t x = 0; x < nn; ++x) {
                sh[x] = c->ux[x] + 0.5 * c->ex[x];
                sh[nn + x] = c->uy[x] + 0.5 * c->ey[x];
            }
            orc_interp(p, c->n_nodes, c->X, sh, sh + nn, U);
            free(sh);
        } else {
            orc_interp(p, c->n_nodes, c->X, c->ux, c->uy, U);
        }
        for (int64_t l = 0; l < 2 * c->n_nodes; ++l) c->X[l] += U[l];
        free(U);
    }
}

void orc_step(orc_ctx* c, int32_t n)
{
    for (int32_t k = 0; k < n; ++k) step_once(c);
}

/* n ADE-only iterations: every species collides with u = 0 (D2Q5 equilibrium w_i phi) plus
 * its reaction, then streams with halfway bounce-back at walls; the fluid, the nodes and the
 * domain map stay as they are.  change (NULL to skip) receives, per iteration k and species
 * s, ||phi^{k+1} - phi^k||_2 / ||phi^{k+1}||_2 at change[k * S + s]. */
void orc_ade_step(orc_ctx* c, int32_t n, double* change)
{
    const orc_params* p = &c->p;
    int64_t nx = p->nx, ny = p->ny, nn = c->nn;
    int S = p->n_species;
    if (S == 0) return;
    double tauD[2];
    for (int s = 0; s < S; ++s) tauD[s] = 0.5 + p->D[s] / CS2;
    if (needs_mask(p)) source_map(c, c->mask);
    else memset(c->mask, 0, sizeof(int32_t) * (size_t)nn);
    double* phi_old = (double*)malloc(sizeof(double) * (size_t)(S * nn));
    for (int32_t k = 0; k < n; ++k) {
        for (int s = 0; s < S; ++s)
            for (int64_t x = 0; x < nn; ++x) {
                double sum = 0.0;
                for (int i = 0; i < 5; ++i) sum += c->g[(s * 5 + i) * nn + x];
                phi_old[s * nn + x] = sum;
            }
        /* collision in place */
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < nn; ++x) {
            double phi[2] = {0.0, 0.0}, R[2];
            for (int s = 0; s < S; ++s) phi[s] = phi_old[s * nn + x];
            for (int s = 0; s < S; ++s) R[s] = orc_reaction(p, s, phi, c->mask[x]);
            for (int s = 0; s < S; ++s)
                for (int i = 0; i < 5; ++i) {
                    double gi = c->g[(s * 5 + i) * nn + x];
                    double geq = W5[i] * phi[s];
                    c->g[(s * 5 + i) * nn + x] = gi - (gi - geq) / tauD[s] + R[s] * W5[i];
                }
        }
        /* streaming */
#pragma omp parallel for schedule(static)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t src = y * nx + x;
                for (int s = 0; s < S; ++s)
                    for (int i = 0; i < 5; ++i) {
                        int64_t xd = wrapi(x + VX[i], nx), yd = y + VY[i];
                        double v = c->g[(s * 5 + i) * nn + src];
                        if (p->bc_y == ORC_WALLS && (yd < 0 || yd >= ny))
                            c->gnew[(5 * s + OPP[i]) * nn + src] = v;
                        else
                            c->gnew[(s * 5 + i) * nn + wrapi(yd, ny) * nx + xd] = v;
                    }
            }
        double* t = c->g; c->g = c->gnew; c->gnew = t;
        c->sent = 0;                      /* an ADE-only iteration, not a coupled step */
        if (change) {
            for (int s = 0; s < S; ++s) {
                double d2 = 0.0, p2 = 0.0;
                for (int64_t x = 0; x < nn; ++x) {
                    double sum = 0.0;
                    for (int i = 0; i < 5; ++i) sum += c->g[(s * 5 + i) * nn + x];
                    double d = sum - phi_old[s * nn + x];
                    d2 += d * d;
                    p2 += sum * sum;
                }
                change[(int64_t)k * S + s] = (d2 == 0.0) ? 0.0 : sqrt(d2) / sqrt(p2);
            }
        }
    }
    free(phi_old);
}

void orc_get_fields(orc_ctx* c, double* rho, double* u, double* phi, double* X, int32_t* mask)
{
    int64_t nn = c->nn;
    /* the concentrations the next collision sees: with no-flux membranes, the populations
     * that arrived across one are replaced first (on a copy; the replacement is the one the
     * next step makes) */
    double* g = c->g;
    int nf = 0;
    for (int s = 0; s < c->p.n_species; ++s) nf |= c->p.no_flux[s];
    if (phi && nf && c->n_cells > 0) {
        size_t bytes = sizeof(double) * 5 * (size_t)c->p.n_species * (size_t)nn;
        g = (double*)malloc(bytes);
        memcpy(g, c->g, bytes);
        if (c->p.no_flux_zeroth) {
            int32_t* m = (int32_t*)malloc(sizeof(int32_t) * (size_t)nn);
            source_map(c, m);
            no_flux_replace(c, m, g);
            free(m);
        } else {
            double* q = (double*)malloc(sizeof(double) * 4 * (size_t)nn);
            orc_link_crossings(&c->p, c->n_cells, c->off, c->X, q);
            if (c->p.no_flux_bounce) no_flux_bounce(c, q, g, -1, NULL);
            else no_flux_first(c, q, g, -1, NULL);
            free(q);
        }
    }
    for (int64_t x = 0; x < nn; ++x) {
        double r = 0.0, jx = 0.0, jy = 0.0;
        for (int i = 0; i < 9; ++i) {
            double fi = c->f[i * nn + x];
            r += fi; jx += fi * VX[i]; jy += fi * VY[i];
        }
        if (pressure_node(c, x)) {
            /* as the next step's rescaling leaves the node */
            double gamma = c->p.rho0 / r;
            r *= gamma; jx *= gamma; jy *= gamma;
        }
        if (rho) rho[x] = r;
        if (u) { u[x] = jx / r; u[nn + x] = jy / r; }
        if (phi) {
            for (int s = 0; s < c->p.n_species; ++s) {
                double sum = 0.0;
                for (int i = 0; i < 5; ++i) sum += g[(s * 5 + i) * nn + x];
                phi[s * nn + x] = sum;
            }
        }
    }
    if (g != c->g) free(g);
    if (X && c->n_nodes) memcpy(X, c->X, sizeof(double) * 2 * (size_t)c->n_nodes);
    if (mask) orc_raster(&c->p, c->n_cells, c->off, c->X, mask);
}

void orc_get_populations(const orc_ctx* c, double* f, double* g)
{
    if (f) memcpy(f, c->f, sizeof(double) * 9 * (size_t)c->nn);
    if (g && c->p.n_species) memcpy(g, c->g, sizeof(double) * 5 * (size_t)c->p.n_species * (size_t)c->nn);
}

void orc_set_populations(orc_ctx* c, const double* f, const double* g)
{
    if (f) memcpy(c->f, f, sizeof(double) * 9 * (size_t)c->nn);
    if (g && c->p.n_species) memcpy(c->g, g, sizeof(double) * 5 * (size_t)c->p.n_species * (size_t)c->nn);
    prev_from_populations(c);
}

void orc_get_prev_moments(const orc_ctx* c, double* phi, double* u)
{
    int64_t nn = c->nn;
    if (phi && c->p.n_species) memcpy(phi, c->phi_prev, sizeof(double) * (size_t)c->p.n_species * (size_t)nn);
    if (u) {
        memcpy(u, c->ux_prev, sizeof(double) * (size_t)nn);
        memcpy(u + nn, c->uy_prev, sizeof(double) * (size_t)nn);
    }
}

void orc_set_prev_moments(orc_ctx* c, const double* phi, const double* u)
{
    int64_t nn = c->nn;
    if (phi && c->p.n_species) memcpy(c->phi_prev, phi, sizeof(double) * (size_t)c->p.n_species * (size_t)nn);
    if (u) {
        memcpy(c->ux_prev, u, sizeof(double) * (size_t)nn);
        memcpy(c->uy_prev, u + nn, sizeof(double) * (size_t)nn);
    }
}

void orc_no_flux_values(orc_ctx* c, int32_t s, double* out)
{
    int64_t nn = c->nn;
    for (int64_t k = 0; k < 4 * nn; ++k) out[k] = NAN;
    if (c->n_cells == 0 || s < 0 || s >= c->p.n_species || !c->p.no_flux[s]) return;
    double* q = (double*)malloc(sizeof(double) * 4 * (size_t)nn);
    orc_link_crossings(&c->p, c->n_cells, c->off, c->X, q);
    if (c->p.no_flux_bounce) no_flux_bounce(c, q, c->g, s, out);
    else no_flux_first(c, q, c->g, s, out);
    free(q);
}

void orc_get_last_spread(const orc_ctx* c, double* ex, double* ey)
{
    memcpy(ex, c->ex, sizeof(double) * (size_t)c->nn);
    memcpy(ey, c->ey, sizeof(double) * (size_t)c->nn);
}

void orc_get_forces(orc_ctx* c, double* F, double* area)
{
    if (c->n_cells == 0) return;
    orc_forces(&c->p, c->n_cells, c->off, c->X, c->l0, c->A0, F, area);
}

void orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads((int)n);
#else
    (void)n;
#endif
}

int32_t orc_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_invariants(const orc_ctx* c, double* out)
{
    /* long double accumulators: the sums are used to check conservation to round-off */
    int64_t nn = c->nn;
    long double m = 0.0L, px = 0.0L, py = 0.0L;
    for (int64_t x = 0; x < nn; ++x) {
        double gamma = 1.0;
        if (pressure_node(c, x)) {
            double r = 0.0;
            for (int i = 0; i < 9; ++i) r += c->f[i * nn + x];
            gamma = c->p.rho0 / r;
        }
        for (int i = 0; i < 9; ++i) {
            double fi = gamma * c->f[i * nn + x];
            m += fi; px += fi * VX[i]; py += fi * VY[i];
        }
    }
    out[0] = (double)m; out[1] = (double)px; out[2] = (double)py;
    for (int s = 0; s < c->p.n_species; ++s) {
        long double t = 0.0L;
        for (int64_t x = 0; x < nn; ++x)
            for (int i = 0; i < 5; ++i) t += c->g[(s * 5 + i) * nn + x];
        out[3 + s] = (double)t;
    }
}
