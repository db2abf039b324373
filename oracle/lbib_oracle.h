/* FP64 CPU oracle of the coupled lattice-Boltzmann / immersed-boundary time step
 * of LBIBCell (Tanaka, Sichau & Iber, arXiv:1503.06726).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain reference that the HIP
 * library is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header, table
 * or constant with the HIP library, and neither side includes the other.
 *
 * Everything is in lattice units (dx = dt = 1), double precision, plain loops.
 *
 * Paper passages followed (section / equation names of the paper):
 *   D2Q9 lattice, BGK collision with body force .... Suppl. "Lattice Boltzmann Method",
 *                                                    Eq. (bgkequation), footnote on D2Q9
 *   second-order equilibrium ........................ Eq. (standardequilibrium)
 *   density and momentum moments, p = rho cs^2 ...... Suppl. "Lattice Boltzmann Method"
 *   D2Q5 advection-diffusion LB, its equilibrium ...... Suppl. "Lattice Boltzmann Method",
 *     with the fluid's u, D = cs^2 (tau_D - 1/2)        D2Q5 footnote and equations
 *   force spreading / velocity interpolation ......... Suppl. "Immersed Boundary Method",
 *                                                    Eqs. (forcedistribution), (conversion2)
 *   1-D cosine kernel and its 4x4 tensor product ..... Eq. (1Dkernel) and the 2-D product
 *   membrane tension ................................. Eq. (membraneforce)
 *   Hookean membrane springs ......................... Section "Membrane Tension"
 *   domain IDs on the lattice ........................ Section "Cell Representation",
 *                                                    Fig. "Elements of the Geometry Representation"
 *   Schnakenberg kinetics ............................ Section "Turing Patterning ..."
 *   loop order (forces, spread, fluid, interpolate,
 *   move, signalling) ................................ Fig. "Algorithm Overview"
 *
 * Readings where the paper is silent are listed with each function in the .c file.
 */
#ifndef LBIB_ORACLE_H
#define LBIB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PERIODIC = 0, ORC_WALLS = 1 };
enum { ORC_DELTA_COS = 0, ORC_DELTA_PESKIN = 1 };
enum { ORC_REACT_NONE = 0, ORC_REACT_SOURCE_DECAY = 1, ORC_REACT_SCHNAKENBERG = 2 };

typedef struct {
    int32_t nx, ny;
    int32_t bc_y;                /* ORC_PERIODIC or ORC_WALLS (halfway bounce-back at y=-1/2, ny-1/2) */
    int32_t delta_kernel;        /* ORC_DELTA_COS (paper) or ORC_DELTA_PESKIN */
    int32_t n_species;           /* 0..2 */
    int32_t interp_new_u;        /* 0: interpolate u of f^n (default); 1: u of f^{n+1} */
    double tau, rho0;
    double body[2];              /* uniform acceleration added to the spread field */
    double k_spring, phi_m, kappa_area;
    double D[2];                 /* diffusivities */
    int32_t reaction[2];
    double rc[2][4];             /* reaction constants, see orc_reaction() */
    double wall_u_top;           /* x-velocity of the top wall (moving-wall test hook) */
    int32_t no_flux[2];          /* 1: the cell membranes are no-flux boundaries for species s */
    double mass_source;          /* constant mass source per node inside a cell and step */
    double area_alpha;           /* area controller: S_k = mass_source + area_alpha (A0_k - A_k) */
    double mass_phi_gamma;       /* + mass_phi_gamma phi_0(x) at every node inside a cell */
    int32_t pressure_ring;       /* 1: the lattice's outer ring is a pressure boundary at rho0 */
    int32_t interp_half_force;   /* 1: interpolate u + f/2 (the half-force-shifted velocity) */
    int32_t no_flux_zeroth;      /* 1: the zeroth-order form of the no-flux condition */
    int32_t no_flux_bounce;      /* 1: the bounce-back form (cut links; conserves the species) */
    int32_t reserved;
} orc_params;

typedef struct orc_ctx orc_ctx;

/* building blocks (also used directly by the pins) */
double orc_delta1d(int32_t kernel, double r);
void   orc_equilibrium9(double rho, double ux, double uy, double out[9]);
void   orc_equilibrium5(double phi, double ux, double uy, double out[5]);
double orc_reaction(const orc_params* p, int32_t s, const double* phi, int32_t m);
void   orc_forces(const orc_params* p, int32_t n_cells, const int32_t* off, const double* X,
                  const double* l0, const double* A0, double* F, double* area);
void   orc_spread(const orc_params* p, int64_t n, const double* X, const double* F,
                  double* ex, double* ey);
void   orc_interp(const orc_params* p, int64_t n, const double* X, const double* ux,
                  const double* uy, double* U);
int64_t orc_raster(const orc_params* p, int32_t n_cells, const int32_t* off, const double* X,
                   int32_t* mask);
void   orc_link_crossings(const orc_params* p, int32_t n_cells, const int32_t* off, const double* X,
                          double* q);                       /* [4][ny][nx] wall distances, +inf: none */

/* a whole simulation */
orc_ctx* orc_create(const orc_params* p);
void     orc_destroy(orc_ctx* c);
int32_t  orc_set_cells(orc_ctx* c, int32_t n_cells, const int32_t* off, const double* X,
                       const double* rest_len, const double* rest_area);
void     orc_set_fields(orc_ctx* c, const double* rho, const double* u, const double* phi);
void     orc_step(orc_ctx* c, int32_t n);
void     orc_set_source_cells(orc_ctx* c, const uint8_t* src);     /* [n_cells] flags, NULL: all */
void     orc_set_node_sources(orc_ctx* c, const double* rate);     /* [ny][nx] mass per node and step, NULL: none */
void     orc_set_pressure_nodes(orc_ctx* c, const uint8_t* flags); /* [ny][nx] nodes held at rho0, NULL: none */
void     orc_ade_step(orc_ctx* c, int32_t n, double* change);      /* ADE-only, u = 0; change [n][S] */
void     orc_source_map(orc_ctx* c, int32_t* out);                  /* [ny][nx], nonzero inside a source cell */
void     orc_get_fields(orc_ctx* c, double* rho, double* u, double* phi, double* X, int32_t* mask);
void     orc_get_populations(const orc_ctx* c, double* f, double* g);
void     orc_set_populations(orc_ctx* c, const double* f, const double* g);
void     orc_get_last_spread(const orc_ctx* c, double* ex, double* ey);
void     orc_get_forces(orc_ctx* c, double* F, double* area);
void     orc_invariants(const orc_ctx* c, double* out);   /* sum rho, sum rho*ux, sum rho*uy, sum phi_s */
/* no-flux membranes, first-order form: the moments of the previous step the replacement reads
 * ([S][ny][nx] concentrations, [2][ny][nx] velocity), and the replacement populations the
 * current state would receive ([4][ny][nx] for directions 1..4, NaN where none is missing) */
void     orc_get_prev_moments(const orc_ctx* c, double* phi, double* u);
void     orc_set_prev_moments(orc_ctx* c, const double* phi, const double* u);
void     orc_no_flux_values(orc_ctx* c, int32_t s, double* out);
int32_t  orc_threads(void);                               /* OpenMP threads the lattice loops use */
void     orc_set_threads(int32_t n);                      /* set them (n > 0) */

#ifdef __cplusplus
}
#endif
#endif
