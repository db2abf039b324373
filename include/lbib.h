/* lbib -- MI355X (gfx950) library for the coupled lattice-Boltzmann / immersed-boundary
 * time step of the LBIBCell method (Tanaka, Sichau & Iber, arXiv:1503.06726).
 *
 * One step advances, on one GPU:
 *   - the D2Q9 BGK fluid with the immersed-boundary body force
 *       (Suppl. "Lattice Boltzmann Method", Eq. bgkequation, Eq. standardequilibrium);
 *   - one D2Q5 advection-diffusion(-reaction) lattice per morphogen species, fed with the
 *     fluid's velocity (Suppl. "Lattice Boltzmann Method", D2Q5 equations; reaction laws of
 *     the "Turing Patterning" section and a source/decay law);
 *   - the polygonal cell membranes: forces (Eq. membraneforce, Hookean springs, area
 *     pressure), spreading to the lattice (Eq. forcedistribution) and interpolation back with
 *     the 4x4 cosine kernel (Eq. 1Dkernel), explicit node advection (Eq. conversion2);
 *   - the domain-ID map (Section "Cell Representation": the ID of the cell on the left of each
 *     counter-clockwise connection, zero outside all cells).
 *
 * Units: lattice units, dx = dt = 1, c_s^2 = 1/3.  x is periodic; y is periodic or bounded by
 * no-slip halfway bounce-back walls at y = -1/2 and y = ny - 1/2.
 *
 * Layouts (all caller buffers are C-contiguous, row-major):
 *   scalar field    [ny][nx], index y*nx + x
 *   vector field    [2][ny][nx] (x component plane, then y component plane)
 *   species fields  [n_species][ny][nx]
 *   node positions  [N][2] (x, y) doubles, unwrapped in x (and in y when periodic)
 *   cells           CSR: offsets[n_cells+1], offsets[0] = 0; nodes offsets[c] .. offsets[c+1]-1
 *                   form cell c+1's polygon in counter-clockwise order; edge k joins node k to
 *                   its cyclic successor in the same cell.
 *
 * Ownership: every input is copied before the call returns; outputs go to caller buffers.
 * The context owns its device memory (hipMalloc), or keeps its state in a workspace the caller
 * binds (lbib_bind_workspace), and launches on the stream given at creation.
 *
 * Errors: every call returns an lbib_status; nothing prints or aborts.  A call that fails
 * validation leaves the context unchanged.  lbib_last_error() gives a message.
 *
 * Threading: a context is not thread-safe.  lbib_step() is asynchronous on the context's
 * stream; calls that return data synchronise that stream.
 */
#ifndef LBIB_H
#define LBIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBIB_VERSION 1

typedef enum {
    LBIB_OK = 0,
    LBIB_EINVAL = -1,    /* an argument failed validation */
    LBIB_ENOMEM = -2,    /* device or host allocation failed */
    LBIB_EDEVICE = -3,   /* no usable GPU, or a HIP call failed */
    LBIB_ESTATE = -4,    /* call made in the wrong state (e.g. NULL context) */
    LBIB_ENUMERIC = -5   /* non-finite state detected (monitor or node positions) */
} lbib_status;

enum { LBIB_PERIODIC = 0, LBIB_WALLS = 1 };
enum { LBIB_DELTA_COS4 = 0,      /* the paper's kernel (1 + cos(pi r / 2)) / 4, |r| <= 2 */
       LBIB_DELTA_PESKIN4 = 1 }; /* Peskin's standard 4-point kernel (zero first moment) */
enum { LBIB_REACT_NONE = 0,
       LBIB_REACT_SOURCE_DECAY = 1,   /* R = c[0] * [inside any cell] - c[1] * phi            */
       LBIB_REACT_SCHNAKENBERG = 2 }; /* species 0: R = c[2] (c[0] - u + u^2 v),
                                         species 1: R = c[2] (c[1] - u^2 v), u = phi_0, v = phi_1;
                                         both species must name it, with equal c[0..2] */
/* Population storage (collision always in FP32).  Populations are kept as deviations from
 * rest, f_i - w_i rho0 and g_i - w_i phi_ref.  FP16 and BF16 store the deviation divided by
 * w_i and multiplied by 2^10, which keeps FP16 clear of its subnormal range; FP16 then holds
 * |deviation / w_i| up to 63. */
enum { LBIB_STORAGE_FP32 = 0, LBIB_STORAGE_FP16 = 1, LBIB_STORAGE_BF16 = 2 };

/* Species flags.
 * LBIB_SPECIES_NO_FLUX: the cell membranes are no-flux boundaries for the species (Section
 * "Signalling": compounds that exist only inside or only outside the cells; Suppl. "No-flux
 * Boundary Condition for Reaction-Advection-Diffusion Equations": missing populations are
 * replaced by equilibria, the momentum interpolated to first order between the fluid and zero
 * at the wall, the density extrapolated to first order from the fluid).  By default the
 * supplement's first-order condition: a D2Q5 link is blocked when a membrane edge cuts it (the
 * crossing rule of the domain IDs, applied to rows for the horizontal links and to columns for
 * the vertical ones); the cut nearest to the node puts the wall at a distance q in [0, 1] of
 * the link.  A population arriving over a blocked link becomes w_i (phi_b + 3 v_i . j_b) with
 *   j_b = q / (1 + q) phi(x + v_i) u(x + v_i)     (interpolated between the node one step on,
 *                                                  in the population's direction, and the wall)
 *   phi_b = 2 phi(x + v_i) - phi(x + 2 v_i)       (extrapolated from the two nodes on),
 * taken from the previous step's collision (its concentration and fluid velocity); where the
 * node two steps on lies beyond a wall or behind a cut link, phi_b = phi(x + v_i); where the
 * node one step on does, phi_b = phi(x) of the previous step and j_b = 0.  Cells in contact are
 * separated (a link between them is cut twice).  With no_flux_zeroth = 1 in lbib_params the
 * zeroth-order form applies instead: a link crosses a membrane when one of its nodes lies inside
 * a cell and the other does not (the inside-cell map of the step's positions), and the
 * population becomes w_i phi_b at zero velocity, phi_b = sum_known g_j / (1 - sum_missing w_i)
 * the node's own concentration; cells then need one lattice unit of extracellular space
 * between them.  In both forms a concentration confined to one side stays there exactly.  Not
 * with a source subset (lbib_set_source_cells), a batch, or lbib_ade_steady (LBIB_EINVAL /
 * LBIB_ESTATE). */
enum { LBIB_SPECIES_NO_FLUX = 1 };

typedef struct {
    double D;          /* diffusivity, > 0; relaxation time tau_D = 3 D + 1/2 */
    double phi_ref;    /* storage reference concentration (deviation storage); any finite value */
    int32_t reaction;  /* LBIB_REACT_* */
    int32_t flags;     /* LBIB_SPECIES_* (0: the membranes are invisible to the species) */
    double c[4];       /* reaction constants (per step), see LBIB_REACT_* */
} lbib_species;

typedef struct {
    int32_t nx, ny;          /* lattice size, 4 .. 32767 each */
    int32_t bc_y;            /* LBIB_PERIODIC or LBIB_WALLS */
    int32_t delta_kernel;    /* LBIB_DELTA_* */
    double tau;              /* fluid relaxation time, > 1/2; nu = (tau - 1/2) / 3 */
    double rho0;             /* reference density (initial density and storage reference), > 0 */
    double body_accel[2];    /* uniform acceleration added to the spread force field */
    double k_spring;         /* Hookean membrane spring constant (0 disables) */
    double phi_m;            /* constant membrane tension (0 disables) */
    double kappa_area;       /* area-pressure stiffness: energy kappa_A (A - A0)^2 / 2 (0 disables) */
    int32_t n_species;       /* 0, 1 or 2 */
    int32_t storage;         /* LBIB_STORAGE_* */
    lbib_species species[2];
    /* Mass sources and area control (Section "Control of Cell Area": a proportional
     * controller S_k = alpha (A0_k - A_k) of each cell's area; Suppl. Table of parameters:
     * the lattice source is a density added per node and step).  Every lattice node inside
     * cell k (the domain map of the step's positions; a node inside two cells belongs to the
     * lower index) gains S_k = mass_source + area_alpha (A0_k - A_k) per step, A0_k the
     * cell's reference area (lbib_set_cells) and A_k its area at the step's positions.  The
     * added mass moves with the local fluid: S_k f_i^eq(1, u) joins the post-collision
     * populations, so the node's density rises by S_k and its velocity is unchanged.  Both 0
     * disable the source.  Not with a source subset (lbib_set_source_cells) or a batch
     * (LBIB_EINVAL / LBIB_ESTATE). */
    double mass_source;      /* constant mass source per inside node and step (Case II's uniform source) */
    double area_alpha;       /* proportional constant alpha of the area controller, >= 0 */
    /* Validation Case III (Section "Validation"): a uniform source inside the cell whose
     * strength is proportional to the species' concentration.  Every node inside a cell gains
     * mass_phi_gamma phi_0(x) per step as well, phi_0(x) its concentration of species 0 as its
     * collision sees it (after a no-flux replacement).  Needs n_species >= 1 when nonzero; not
     * with a source subset or a batch, as above. */
    double mass_phi_gamma;
    /* Pressure boundary (Suppl. "Pressure Boundary Condition for the Fluid Equations"; the
     * iso-pressure outflow of the validation cases): with pressure_ring = 1 every node of the
     * lattice's outer ring (columns 0 and nx-1, rows 0 and ny-1) is a point of prescribed
     * density rho0.  Its streamed populations are rescaled by gamma = rho0 / rho before the
     * collision; the velocity is unchanged, since gamma cancels in it.  Reported fields and
     * sums are those after the rescaling.  This is the mass sink that lets cells grow under
     * mass sources.  Not with a batch (LBIB_EINVAL). */
    int32_t pressure_ring;   /* 0 or 1 */
    /* The velocity the membrane nodes move with (Eq. conversion2 applied to the fluid of
     * Eq. bgkequation).  0 (default): u = sum f v / rho, the moments of the populations before
     * the collision.  1: the half-force-shifted u + f/2, the mean of the momentum before and
     * after the step's forcing term (f the spread membrane force plus the body acceleration);
     * with it a membrane in static balance does not drift, and a circle under constant tension
     * shrinks slowly by leakage, as in the paper's validation Case IV (with 0 it drifts outward
     * by half the interpolated force density per step).  The fluid's collision, the species'
     * advection and the reported velocity keep u = sum f v / rho either way.  Not with a batch
     * (LBIB_EINVAL). */
    int32_t interp_half_force;   /* 0 or 1 */
    int32_t no_flux_zeroth;  /* 0: the first-order no-flux condition; 1: its zeroth-order form */
    /* The bounce-back form of the no-flux condition (0 or 1; with no_flux_zeroth = 0).  Not the
     * supplement's equilibrium replacement: a population that would arrive across a cut link
     * becomes the one the node itself sent towards the membrane the step before (its
     * post-collision population in the opposite direction).  Neither side of a cut link receives
     * what the other sends, so the species is conserved exactly while membranes move, where the
     * equilibrium forms lose the species a moving membrane sweeps over (Section "Validation":
     * the paper finds the integrated concentration of its growing cells converging).  At the
     * first step after the fields are set (lbib_create, lbib_set_fields) each node is taken to
     * have sent its own populations; that step is launched outside the step graphs. */
    int32_t no_flux_bounce;
    /* The FP64 monitor: 0 (default) off, or a positive multiple of LBIB_GRAPH_STEPS.  The global
     * sums of lbib_reduce (sum rho, sum rho u, sum phi_s) are then taken on the device at the
     * end of every (monitor_every / LBIB_GRAPH_STEPS)-th period of LBIB_GRAPH_STEPS steps
     * completed by lbib_step since the last lbib_set_cells (or the creation), inside the step
     * graphs it replays; periods are aligned to the rebuilds of the per-tile node lists, so with
     * cells set at step 0 the sums follow steps monitor_every, 2 monitor_every, ...  Steps a batch
     * takes do not count.  lbib_get_monitor returns the latest.  A sum that is not finite sets
     * the context's error state (see lbib_step). */
    int32_t monitor_every;
    int32_t reserved;        /* 0 */
} lbib_params;

/* Steps per captured graph of lbib_step, and the period of the per-tile node lists. */
#define LBIB_GRAPH_STEPS 16

typedef struct lbib_ctx lbib_ctx;

/* Validate parameters without touching a GPU.  msg (optional) receives a reason.
 * Returns LBIB_OK or LBIB_EINVAL. */
lbib_status lbib_validate_params(const lbib_params* p, char* msg, size_t msg_len);

/* Validate a cell set (same rules as lbib_set_cells) without touching a GPU. */
lbib_status lbib_validate_cells(const lbib_params* p, int32_t n_cells, const int32_t* offsets,
                                const double* xy, const double* rest_len, const double* rest_area,
                                char* msg, size_t msg_len);

/* Create a context on the current HIP device.  hip_stream is a hipStream_t to launch on
 * (NULL: the library creates its own).  The lattice starts at rest: rho = rho0, u = 0,
 * every concentration 0, no cells.  On failure *out is NULL and the status says why
 * (LBIB_EINVAL, LBIB_EDEVICE when no GPU is usable, LBIB_ENOMEM). */
lbib_status lbib_create(const lbib_params* p, void* hip_stream, lbib_ctx** out);

/* Caller-owned device memory for the solver states (Section "Input and Output": the fluid
 * and reaction-advection-diffusion solver states, the geometry points and their connections;
 * Figure "Iterative Processing in the Solver": these states persist from one iteration to the
 * next).  A workspace holds, in one caller allocation, every array a context keeps between
 * calls: both population buffers of the fluid and species lattices, the inside-cell bits, the
 * tile lists and counters, the reduction partials, a staging area for read-backs, and the
 * membrane arrays (positions, rest lengths and areas, spreading records, velocity shares,
 * per-tile node lists, source-cell flags) for up to a stated number of nodes.
 *
 * lbib_workspace_size: bytes of a workspace for a context with parameters p whose cell sets
 * have at most n_nodes membrane nodes in total (any number of cells).  Pure host function; the
 * value depends on p and n_nodes only.  LBIB_EINVAL for invalid parameters or n_nodes < 0. */
lbib_status lbib_workspace_size(const lbib_params* p, int64_t n_nodes, size_t* bytes);

/* Move the context's state into the caller's workspace [device_ptr, device_ptr + bytes).
 *   device_ptr  device memory of the context's device (hipMalloc, or a torch tensor's
 *               storage), 256-byte aligned, with bytes inside one allocation; or NULL with
 *               bytes = 0 to move the state back into memory the library allocates
 *   bytes       at least lbib_workspace_size(p, N) for the current node count N; the node
 *               capacity is the largest n with lbib_workspace_size(p, n) <= bytes
 * The state is copied (the simulation continues unchanged, bit for bit) on the context's
 * stream, which is synchronised; the library's own memory for it is then released, or, when
 * moving from one workspace to another, the old workspace is no longer used and may be freed.
 * While bound, lbib_set_cells with more nodes than the capacity returns LBIB_ENOMEM (state
 * unchanged), and nothing of the state is allocated or freed by the library.  lbib_ade_steady
 * still allocates its own working set for the length of that call.
 * The caller keeps the workspace alive and untouched until the context is destroyed or moved
 * elsewhere; the contents are the library's and their layout is private.
 * Errors: LBIB_EINVAL for a misaligned pointer, memory that is not device memory of the
 * context's device, a range past the end of its allocation, or a range overlapping the
 * workspace currently bound; LBIB_ENOMEM when bytes is below what the current state needs;
 * LBIB_ESTATE while a batch has adopted the context, or while node sources or pressure points
 * are set (they stay in the library's memory).  On failure the context is unchanged. */
lbib_status lbib_bind_workspace(lbib_ctx* ctx, void* device_ptr, size_t bytes);

/* Membrane nodes the bound workspace holds, or -1 when no workspace is bound. */
lbib_status lbib_workspace_nodes(const lbib_ctx* ctx, int64_t* n_nodes);

/* Set the membranes (Section "Cell Representation": closed CCW polygons, the cell's ID is
 * c+1 for the c-th polygon, 0 is the extracellular space).
 *   offsets   [n_cells+1] host int32, CSR as above; 0 <= n_cells <= 65535;
 *             3 .. 4096 nodes per cell, at most 2e8 nodes in total
 *   xy        [N][2] host doubles, N = offsets[n_cells]; finite, |coordinate| < 2^20
 *   rest_len  [N] host doubles (edge k's rest length) or NULL for the initial edge lengths
 *   rest_area [n_cells] host doubles or NULL for the initial areas
 * Rejected (LBIB_EINVAL): clockwise or degenerate polygons (signed area <= 0), non-finite
 * values, bad offsets, a polygon spanning nx (or ny when periodic) or more, and with walls
 * any node closer than 2 lattice units to a wall (y < 1.5 or y > ny - 2.5).
 * Computes the forces of the new positions and the domain-ID map. */
lbib_status lbib_set_cells(lbib_ctx* ctx, int32_t n_cells, const int32_t* offsets, const double* xy,
                           const double* rest_len, const double* rest_area);

/* Reset the lattice to equilibrium populations f^eq(rho, u), g^eq(phi_s, u)
 * (Eq. standardequilibrium and the D2Q5 equilibrium).  Host doubles:
 *   rho [ny][nx] or NULL (rho0), u [2][ny][nx] or NULL (0), phi [S][ny][nx] or NULL (0). */
lbib_status lbib_set_fields(lbib_ctx* ctx, const double* rho, const double* u, const double* phi);

/* Enqueue n >= 0 coupled steps on the context's stream (asynchronous).  Each step, from
 * state (f^n, g^n, X^n): spread the membrane forces F(X^n) plus the body acceleration, collide
 * the fluid and every species with u^n = sum f^n v / rho^n and the domain IDs of X^n, stream,
 * then move every node by the interpolated u^n (Fig. "Algorithm Overview").  Whole periods of
 * LBIB_GRAPH_STEPS steps, aligned to the per-tile node lists, replay a captured graph.
 * Watchdog: the device flags a node position or force that became non-finite, a node that
 * moved more than 2 lattice units between list rebuilds (its spread force would be lost), and,
 * with the monitor on, a lattice sum that is not finite; every period ends by copying the flags
 * to pinned host memory.  lbib_step returns LBIB_ENUMERIC, and enqueues no further step, once
 * flags raised by work that has completed are visible there; every call that reads data
 * returns LBIB_ENUMERIC for them as well.  lbib_set_cells clears them. */
lbib_status lbib_step(lbib_ctx* ctx, int32_t n);

/* Copy the current state to host buffers (NULL skips an output); synchronises the stream.
 * Section "Input and Output": the fluid and the reaction-advection-diffusion solver states
 * (here their moments) and the geometry points.
 *   rho [ny][nx], u [2][ny][nx], phi [S][ny][nx] doubles (moments of the current populations),
 *   xy [N][2] doubles (current node positions), cell_id_map [ny][nx] int32 (domain IDs).
 * Returns LBIB_ENUMERIC (after copying) when the device has flagged a node position or force
 * that became non-finite, a node that moved more than 2 lattice units between two rebuilds of
 * the per-tile node lists (its stencil may then reach tiles that do not list it: part of its
 * spread force and interpolated velocity is lost), or a non-finite monitor sum. */
lbib_status lbib_get_fields(lbib_ctx* ctx, double* rho, double* u, double* phi, double* xy,
                            int32_t* cell_id_map);

/* Membrane forces F(X) of the current positions ([N][2] doubles, NULL skips) and the
 * cell areas ([n_cells] doubles, NULL skips); synchronises. */
lbib_status lbib_get_forces(lbib_ctx* ctx, double* F, double* area);

/* The force field the next step will use: the current forces spread to the lattice plus the
 * body acceleration, as [2][ny][nx] doubles (Eq. forcedistribution); synchronises. */
lbib_status lbib_get_spread(lbib_ctx* ctx, double* e);

/* Mark the cells whose interior is a source for the source/decay law (R = c[0] [inside a
 * source cell] - c[1] phi): src[n_cells] host bytes, nonzero = source; NULL restores the
 * default, every cell.  A node inside several cells is inside a source cell when any of them
 * is one.  The cells must be set (LBIB_ESTATE otherwise); lbib_set_cells resets the choice.
 * A subset (src not NULL) is refused with LBIB_EINVAL when a species has no-flux membranes or
 * mass sources are on: they read the same inside map.  Synchronises. */
lbib_status lbib_set_source_cells(lbib_ctx* ctx, const uint8_t* src);

/* Mass sources at lattice nodes (Section "Validation", Case I: a constant point mass source in
 * the cell), and any other per-node source.  rate[ny][nx] (host, row-major, copied before
 * return) is the mass added at each node per step; a node gains it as rate f_i^eq(1, u) after
 * its collision, like a cell's source (see mass_source), whether or not it lies inside a cell.
 * The rates are kept in FP32 on the device.  NULL removes them.  LBIB_EINVAL for a rate that
 * is not finite in FP32; LBIB_ESTATE while a workspace is bound or a batch holds the context. */
lbib_status lbib_set_node_sources(lbib_ctx* ctx, const double* rate);

/* Pressure points anywhere in the lattice (Suppl. "Pressure Boundary Condition for the Fluid
 * Equations": lattice points with prescribed pressure, the sinks of growing tissues).
 * flags[ny][nx] (host, row-major, copied before return): every node with a nonzero flag is
 * held at density rho0 as the outer ring is with pressure_ring (its streamed populations
 * rescaled by rho0 / rho before the collision, the velocity unchanged; reported fields and
 * sums those after the rescaling).  NULL removes them.  LBIB_ESTATE while a workspace is bound
 * or a batch holds the context. */
lbib_status lbib_set_pressure_nodes(lbib_ctx* ctx, const uint8_t* flags);

/* ADE-only iterations towards the steady state of the species (the "iterations to steady"
 * measurement).  Every species lattice collides with u = 0 (equilibrium w_i phi) plus its
 * reaction and streams (D2Q5 equations, halfway bounce-back at walls) while the fluid, the
 * membranes and the source map stay frozen, starting from the current species state (set it
 * with lbib_set_fields: zero, or a warm start), until for every species
 *   ||phi^k - phi^{k-1}||_2 <= tol ||phi^k||_2,
 * phi^k being the concentration after k iterations, or until k = max_iters.
 *   fp64     1: iterate in FP64 (the state is copied to an FP64 working set and back);
 *            0: iterate in FP32
 *   iters    receives the first k meeting the criterion, 0 if none did within max_iters
 *   change   receives the last relative change evaluated (maximum over species), or NULL
 * Iterations run in captured batches of 128, so the species state left behind may be up to
 * 127 iterations past k.  tol must be finite and >= 0, max_iters >= 0 (LBIB_EINVAL);
 * LBIB_ENUMERIC if a change becomes non-finite.  Synchronises. */
lbib_status lbib_ade_steady(lbib_ctx* ctx, double tol, int64_t max_iters, int32_t fp64, int64_t* iters,
                            double* change);

/* Batched ADE-only steady states (no context): `batch` independent single-species problems on
 * one nx x ny lattice (x periodic, y per bc_y), each iterated as in lbib_ade_steady with the
 * source/decay law R = sigma[b] m_b(x) - decay[b] phi and relaxation tau_D = 3 D[b] + 1/2.
 *   source   [batch][ny][nx] host bytes, m_b(x) = 1 where nonzero (inside a source cell)
 *   phi      [batch][ny][nx] host doubles: the start (equilibrium populations w_i phi),
 *            ignored when zero_start != 0; on return the final concentrations
 *   iters    [batch] out: the first k with ||phi^k - phi^{k-1}||_2 <= tol ||phi^k||_2, 0 when
 *            max_iters passed first
 *   fp64     1 iterates in FP64, 0 in FP32;  hip_stream as in lbib_create (NULL: private)
 * All problems advance together in captured batches of 64 iterations; a converged problem
 * stops after the batch in which it converged, so its returned field may be up to 63
 * iterations past its k.  Device memory is allocated for the call and freed before it
 * returns.  LBIB_EINVAL for bad sizes or parameters, LBIB_ENUMERIC if a change became
 * non-finite (the other problems still finish).  Synchronises. */
lbib_status lbib_ade_batch(int32_t nx, int32_t ny, int32_t bc_y, int32_t batch, const uint8_t* source,
                           const double* D, const double* sigma, const double* decay, double* phi,
                           int32_t zero_start, double tol, int64_t max_iters, int32_t fp64, int64_t* iters,
                           void* hip_stream);

/* ---------------------------------------------------------------------------------------
 * Batched stepping of many independent simulations (parameter sweeps).  The paper runs one
 * tissue at a time; a batch adopts existing contexts, of any lattice sizes and cell counts,
 * and advances them together: each kernel of the step (Fig. "Algorithm Overview": lattice
 * pass with spreading and interpolation, node advection and forces, list rebuild) runs once
 * per step over every simulation of a group, and whole list periods (16 steps) replay one
 * captured HIP graph.  The simulations form one group, or two groups of about equal lattice
 * size whose step chains run on two streams (one group's latency-bound membrane and list
 * kernels then overlap the other's lattice pass).  Each simulation's arithmetic is that of
 * lbib_step: with the default tile height (8 rows) a batched simulation is bit-identical to
 * the same simulation stepped alone, in either grouping; another tile height changes only the
 * grouping of the interpolation sums (round-off level).
 * While adopted, a context's own lbib_step, lbib_set_cells, lbib_set_fields,
 * lbib_set_source_cells, lbib_set_node_sources, lbib_set_pressure_nodes and lbib_ade_steady
 * return LBIB_ESTATE; its reads (lbib_get_fields,
 * lbib_get_forces, lbib_get_spread, lbib_reduce, lbib_sync) wait for the batch's last
 * enqueued work.  Destroying an adopted context leaves the batch unusable (LBIB_ESTATE).
 * --------------------------------------------------------------------------------------- */
typedef struct lbib_batch lbib_batch;

/* Adopt n >= 1 contexts (host array of distinct, non-adopted contexts on the current device,
 * each with cells set, all with the same species count, storage type and source law).  Any
 * context between list rebuilds has its lists rebuilt first.  hip_stream as in lbib_create
 * (the batch's work runs there).  The contexts stay owned by the caller and must outlive the
 * batch.  LBIB_EINVAL for a bad set, and for a context with no-flux species, mass sources
 * (cell or node sources), the pressure ring or pressure points (the batched pass has none of
 * them); *out is NULL on failure. */
lbib_status lbib_batch_create(lbib_ctx* const* sims, int32_t n, void* hip_stream, lbib_batch** out);

/* Enqueue n >= 0 steps of every simulation on the batch's stream (asynchronous). */
lbib_status lbib_batch_step(lbib_batch* b, int32_t n);

/* Wait for the batch's work and check every simulation's error flags (LBIB_ENUMERIC, naming
 * the simulation, when a node became non-finite or outran its list margin). */
lbib_status lbib_batch_sync(lbib_batch* b);

/* Lattice tile height (rows; tiles are 64 columns wide) of the batched lattice pass: 4, 8
 * (default) or 16.  4 needs walls or ny divisible by 4 in every simulation (LBIB_EINVAL).
 * Changing it is allowed only after a whole number of 16-step periods (LBIB_ESTATE); the
 * lists are rebuilt for the new tiles. */
lbib_status lbib_batch_get_tile(const lbib_batch* b, int32_t* rows);
lbib_status lbib_batch_set_tile(lbib_batch* b, int32_t rows);

/* Number of groups (1, the default, or 2; LBIB_EINVAL otherwise).  Changing it is allowed only
 * after a whole number of 16-step periods (LBIB_ESTATE). */
lbib_status lbib_batch_get_groups(const lbib_batch* b, int32_t* groups);
lbib_status lbib_batch_set_groups(lbib_batch* b, int32_t groups);

/* Autotuner: time `periods` 16-step periods (after one warm-up period) of the batch at every
 * admissible tile height in one and in two groups, on a copy of the simulations' state that is
 * restored afterwards (the simulations do not advance), and keep the fastest.  rows and groups
 * (each NULL or one host int32) receive it; ms_per_step (NULL, or 6 host doubles) receives the
 * time per step of heights 4, 8, 16 in one group, then in two (-1 where not admissible).
 * Needs device memory for one copy of every simulation's state; only after a whole number of
 * periods (LBIB_ESTATE); synchronises. */
lbib_status lbib_batch_autotune(lbib_batch* b, int32_t periods, int32_t* rows, int32_t* groups, double* ms_per_step);

/* Last error message of the batch (never NULL). */
const char* lbib_batch_last_error(const lbib_batch* b);

/* Release the contexts (waiting for the batch's work; lists of a non-default tile height are
 * rebuilt for the contexts' own steps) and free the batch.  NULL is ignored. */
void lbib_batch_destroy(lbib_batch* b);

/* ---------------------------------------------------------------------------------------
 * Learned warm start of the steady state: a convolutional surrogate (four-level U-Net on BF16
 * with FP32 accumulation) mapping, per lattice node, eight input channels (the caller's
 * features; the warm-start module uses source mask, cell-boundary mask, normalised diffusivity,
 * normalised log decay and the domain's source fraction, and leaves three at zero) to the
 * dimensionless steady concentration phi * decay / source, trained and evaluated entirely by
 * the library's kernels.  It is not a
 * passage of the paper: it seeds the D2Q5 populations, and lbib_ade_steady / lbib_ade_batch
 * still iterate to the same tolerance, so a poor prediction costs iterations, not accuracy.
 *
 * Architecture (15 convolutions, all 3x3, zero padding, stride 1; ReLU after each but the
 * last; channels in parentheses; "pool" is a 2x2 average, "up" a 2x nearest upsample, "+" adds
 * the encoder output of the same level after the convolution's ReLU):
 *   input(8, zero-padded to 16) -c0-> (32) -c1-> s0(32) pool -c2-> (64) -c3-> s1(64) pool
 *   -c4-> (128) -c5-> s2(128) pool -c6-> (256) -c7-> (256) up -c8-> (128) + s2 -c9-> (128)
 *   up -c10-> (64) + s1 -c11-> (64) up -c12-> (32) + s0 -c13-> (32) -c14-> (16); output = channel 0
 * Parameters, packed in layer order l = 0..14: W_l [Cout][9 Cin] (index (3 ky + kx) Cin + ci,
 * reading the input at (y + ky - 1, x + kx - 1)), then b_l [Cout].  FP32 host arrays.
 * Tensors handed to the calls below are DEVICE pointers: inputs [B][h][w][8] float, targets
 * and predictions [B][h][w] float.  h and w are multiples of 8.  Loss: mean over nodes of
 * (prediction - target)^2.  Training uses Adam (0.9, 0.999, 1e-8) on FP32 master weights.
 * --------------------------------------------------------------------------------------- */
typedef struct lbib_net lbib_net;

/* Create a network for h x w inputs and batches of at most max_batch, all parameters zero.
 * hip_stream as in lbib_create.  LBIB_EINVAL for bad sizes. */
lbib_status lbib_net_create(int32_t h, int32_t w, int32_t max_batch, void* hip_stream, lbib_net** out);
/* Number of packed parameters. */
lbib_status lbib_net_param_count(const lbib_net* net, int64_t* count);
/* Copy in / out all parameters (host FP32, packed as above); setting resets Adam's moments.
 * LBIB_EINVAL for non-finite values. */
lbib_status lbib_net_set_params(lbib_net* net, const float* params);
lbib_status lbib_net_get_params(lbib_net* net, float* params);
/* Predictions for B <= max_batch inputs (device pointers); synchronises. */
lbib_status lbib_net_predict(lbib_net* net, const float* inputs, int32_t B, float* out);
/* Loss and, when grad (host, packed like the parameters) is not NULL, its gradient for one
 * batch; synchronises. */
lbib_status lbib_net_loss_grad(lbib_net* net, const float* inputs, const float* targets, int32_t B, double* loss,
                               float* grad);
/* One Adam step with learning rate lr on one batch; *loss (optional) is the batch loss before
 * the step.  Synchronises for the loss. */
lbib_status lbib_net_train_step(lbib_net* net, const float* inputs, const float* targets, int32_t B, float lr,
                                double* loss);
/* Free the network (NULL is ignored). */
void lbib_net_destroy(lbib_net* net);

/* Global sums over the lattice in FP64, deterministic:
 *   out[0] = sum rho, out[1] = sum rho ux, out[2] = sum rho uy, out[3+s] = sum phi_s.
 * out has 3 + n_species doubles.  Returns LBIB_ENUMERIC if any sum is not finite. */
lbib_status lbib_reduce(lbib_ctx* ctx, double* out);

/* The sums of lbib_reduce, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine) and does not synchronise: it
 * enqueues on the context's stream the same two kernels as lbib_reduce, which write
 * out_device[0 .. 2 + n_species] in the same order, bit for bit the values lbib_reduce returns
 * for the same state.
 *   out_device  device memory of the context's device, 3 + n_species doubles, caller-owned;
 *               valid once the context's stream has reached the call
 * The per-block partial sums live in a scratch array that the library holds in each GPU's
 * memory for the life of the process: 4096 partials of 5 doubles (160 KiB), enough for any
 * lattice (each block loops over its share of the nodes).  Every context on a GPU shares that
 * GPU's scratch, and it keeps the last call's partials: calls on one GPU that overlap (on
 * different streams, or from different threads) race and must be ordered by the caller.
 * No check for non-finite sums is made (the values stay on the device).
 * Errors: LBIB_ESTATE for a NULL context; LBIB_EINVAL for a NULL pointer or memory that is not
 * device memory of the context's device; LBIB_EDEVICE when the scratch has no device address
 * or a launch fails. */
lbib_status lbib_reduce_device(lbib_ctx* ctx, double* out_device);

/* Saving and resuming a run (Section "Input and Output": the solver states are saved in a
 * format the software can load to continue).  The state is everything a step reads that is
 * not a function of the node positions: the current populations of the fluid and species
 * lattices as stored (deviations in the storage type), the first-order no-flux condition's
 * previous-step concentrations and velocities, the cells (offsets, positions, rest lengths and
 * areas, source flags), the node sources and pressure points, the monitor's latest sums and
 * period count, and the error flags.  On
 * loading, the forces, spreading records, per-tile node lists, inside-cell bits, cell map and
 * link cuts are rebuilt from the positions as lbib_set_cells builds them, and the lists start
 * a new period; the run then continues bit for bit as it would have (the list period decides
 * only which tiles list a node, which does not change any sum).
 *   lbib_state_size: bytes of the current state (it depends on the parameters and the node
 *                    count).
 *   lbib_save_state: copy the state into the host buffer [buf, buf + bytes); synchronises.
 *                    LBIB_EINVAL when bytes is short.
 *   lbib_load_state: replace the context's state by a saved one.  The context must have been
 *                    created with the same parameters (LBIB_EINVAL otherwise, or for a short or
 *                    foreign buffer); the cells are validated as by lbib_set_cells.  Synchronises;
 *                    LBIB_ESTATE while a batch has adopted the context.  A failure may leave the
 *                    node maps and cells replaced and the populations unchanged.  A state with node sources
 *                    or pressure points is refused with LBIB_ESTATE while a workspace is
 *                    bound (the workspace does not hold them). */
lbib_status lbib_state_size(lbib_ctx* ctx, size_t* bytes);
lbib_status lbib_save_state(lbib_ctx* ctx, void* buf, size_t bytes);
lbib_status lbib_load_state(lbib_ctx* ctx, const void* buf, size_t bytes);

/* The latest sums of the FP64 monitor (lbib_params.monitor_every): out [3 + n_species] doubles
 * as lbib_reduce's, *taken the number of times the monitor has taken them since the last
 * lbib_set_cells (0, out untouched, when it has not yet).  Synchronises.  LBIB_ESTATE when the
 * monitor is off; LBIB_ENUMERIC (after copying) when a sum is not finite. */
lbib_status lbib_get_monitor(lbib_ctx* ctx, double* out, int64_t* taken);

/* Wait for all queued work on the context's stream. */
lbib_status lbib_sync(lbib_ctx* ctx);

/* Per-kernel timing with HIP events on the context's stream (0 disables, default).
 * Ids: LBIB_K_LATTICE (the lattice pass), LBIB_K_MEMBRANE (interpolation, advection, forces,
 * domain IDs), LBIB_K_LISTS (rebuilding the per-tile lists of membrane nodes, every few steps).
 * lbib_get_timing synchronises and returns the summed milliseconds and the number of timed
 * launches since timing was last enabled. */
enum { LBIB_K_LATTICE = 0, LBIB_K_MEMBRANE = 1, LBIB_K_LISTS = 2, LBIB_K_COUNT = 3 };
lbib_status lbib_set_timing(lbib_ctx* ctx, int32_t enable);
lbib_status lbib_get_timing(lbib_ctx* ctx, int32_t kernel, double* total_ms, int64_t* launches);

/* Bytes of device memory the library has allocated for the context (a bound workspace is
 * the caller's and is not counted). */
lbib_status lbib_device_bytes(const lbib_ctx* ctx, size_t* bytes);

/* Last error message of the context (never NULL; "" when none). */
const char* lbib_last_error(const lbib_ctx* ctx);

/* Name of a status code. */
const char* lbib_status_string(lbib_status s);

/* Library version (LBIB_VERSION). */
int32_t lbib_version(void);

/* Free the context and its device memory (waits for its stream).  NULL is ignored. */
void lbib_destroy(lbib_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBIB_H */
