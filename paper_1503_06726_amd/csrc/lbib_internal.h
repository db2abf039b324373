// Host-side context and kernel launch wrappers of the lbib library.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string>
#include <vector>

#include "lbib.h"
#include "lbib_device.h"

namespace lbib {

// validation (pure C++, no HIP calls; validate.cpp)
lbib_status check_params(const lbib_params* p, std::string& msg);
lbib_status check_cells(const lbib_params* p, int32_t n_cells, const int32_t* offsets, const double* xy,
                        const double* rest_len, const double* rest_area, std::string& msg);

struct TimedLaunch {
    int kernel;
    hipEvent_t start, stop;
};

}  // namespace lbib

struct lbib_batch;

struct lbib_ctx {
    lbib_params p{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    int64_t nn = 0;          // nx * ny
    int S = 0;               // species
    int ntx = 0, nlty = 0, nltiles = 0;   // lattice tiles (TILE_X x LTILE_Y): columns, rows, total
    int tile_cap = 0;                     // tiles of the shortest tile shape (sizes the tile arrays)
    bool mask_needed = false;
    bool nf_fresh = true;    // the state was set from outside and has not stepped (bounce-back no-flux)

    // lattice state: post-collision deviations (FP32, FP16 or BF16), A/B buffers
    void* f[2] = {nullptr, nullptr};
    void* g[2] = {nullptr, nullptr};
    size_t pop_bytes = 4;            // bytes per stored population
    // chunked arrays (lbib_device.h): ntx chunks of TILE_X columns per row
    int gchunk() const { return 5 * S * lbib::TILE_X; }
    int64_t frow() const { return (int64_t)ntx * 9 * lbib::TILE_X; }
    int64_t grow() const { return (int64_t)ntx * gchunk(); }
    size_t f_elems() const { return (size_t)p.ny * (size_t)frow(); }
    size_t g_elems() const { return (size_t)p.ny * (size_t)grow(); }
    int cur = 0;
    unsigned* inside[2] = {nullptr, nullptr};   // inside-any-cell bits [ny][wpr], by parity cur
    unsigned* cmap = nullptr;   // mass sources: [ny][nx] index of the cell each node lies in (~0: none)
    // no-flux membranes in the first-order form, by parity cur (NULL otherwise): wall distances
    // [4][nn] and blocked-link bytes [nn] (4-byte padded) of the positions the pass of parity cur
    // reads, the concentration deviations [S][nn] and velocities [nn] its collision saw last
    float* nfq[2] = {nullptr, nullptr};
    uint8_t* nfm[2] = {nullptr, nullptr};
    float* nfphi[2] = {nullptr, nullptr};
    float2* nfu[2] = {nullptr, nullptr};
    size_t nfm_bytes() const { return ((size_t)nn + 3) / 4 * 4; }
    int wpr = 0;                     // 32-bit words per lattice row
    int64_t ny_words() const { return (int64_t)p.ny * wpr; }

    // membranes
    int32_t n_cells = 0;
    int64_t n_nodes = 0;
    int max_cell_nodes = 0;
    int* d_off = nullptr;
    double2* d_X = nullptr;
    double* d_l0 = nullptr;
    double* d_A0 = nullptr;
    double* d_area = nullptr;
    int* d_ijlist = nullptr;         // stencil origin of each node at the last list build
    float2* d_part = nullptr;        // [MAX_NODE_TILES][N] velocity shares by tile rank and node
    uint8_t* d_cnt = nullptr;        // [N] tiles each node is listed in
    float4* d_rec = nullptr;         // [N] spreading records (fractional offset, force)
    int* d_rec_ij = nullptr;         // [N] current stencil origins
    int* d_list = nullptr;           // [N * MAX_NODE_TILES] per-tile node lists
    float* d_nsrc = nullptr;         // [ny][nx] mass source per node and step (NULL: none)
    uint8_t* d_pmap = nullptr;       // [ny][nx] pressure points (NULL: none)
    int* d_t_count = nullptr;        // [tile_cap], zero between list builds
    int* d_t_off = nullptr;          // [tile_cap + 1]
    int* d_t_cur = nullptr;          // [tile_cap] fill cursors
    int* d_err = nullptr;            // device error flags
    uint8_t* d_src = nullptr;        // [n_cells] source cells of the source/decay law (NULL: all)
    int steps_since_lists = 0;

    // staging
    double* d_stage = nullptr;
    size_t stage_bytes = 0;
    double* d_mon = nullptr;         // FP64 monitor: [0] sums taken, [1 ..] the latest sums
    int64_t period_count = 0;        // periods of LIST_PERIOD steps completed since the last lbib_set_cells
    int* h_err = nullptr;            // the error flags mirrored to pinned host memory
    int* h_err_dev = nullptr;        // its device address
    double* d_partial = nullptr;     // reduction partials
    size_t partial_count = 0;
    bool scratch_ok = false;         // the static reduction scratch has an address on this device

    size_t device_bytes = 0;         // bytes the library allocated itself

    // caller-owned workspace (lbib_bind_workspace): while ws is set, every persistent array
    // above lives in it, in the order of the workspace layout, and none is allocated or freed
    // by the library
    char* ws = nullptr;
    size_t ws_bytes = 0;
    size_t ws_node_base = 0;         // byte offset of the node part
    int64_t ws_node_cap = 0;         // membrane nodes the node part holds
    size_t ws_stage_doubles = 0;     // staging capacity
    uint8_t* ws_src = nullptr;       // the source-cell slot of the node part

    // captured step sequences: GRAPH_STEPS steps starting right after a list build, one graph
    // per parity (cur) of the population buffers at the start
    bool use_graphs = true;
    hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [parity][monitor at the end]
    hipStream_t capture_stream = nullptr;

    // a batch that has adopted this context steps it on the batch's stream; reads wait for
    // the batch's last work (done), changes are refused until the batch releases it
    lbib_batch* batch = nullptr;
    hipEvent_t batch_done = nullptr;

    // timing
    bool timing = false;
    std::vector<lbib::TimedLaunch> pending;
    std::vector<hipEvent_t> free_events;
    double t_ms[LBIB_K_COUNT] = {};
    int64_t t_count[LBIB_K_COUNT] = {};
};

namespace lbib {

// species whose cell membranes are no-flux boundaries (bit s for species s)
inline int no_flux_bits(const lbib_params& p)
{
    int b = 0;
    for (int s = 0; s < p.n_species; ++s)
        if (p.species[s].flags & LBIB_SPECIES_NO_FLUX) b |= 1 << s;
    return b;
}

// does the step keep the first-order no-flux state (a no-flux species, not the zeroth-order form)?
inline bool no_flux_first(const lbib_params& p) { return no_flux_bits(p) != 0 && !p.no_flux_zeroth; }

// does the step add mass inside the cells (constant source or area controller)?
inline bool mass_sources(const lbib_params& p)
{
    return p.mass_source != 0.0 || p.area_alpha != 0.0 || p.mass_phi_gamma != 0.0;
}

// does a step read the cell areas (area pressure, area controller)?
inline bool area_in_step(const lbib_params& p) { return p.kappa_area != 0.0 || mass_sources(p); }

// kernel launchers (return the launch error)
hipError_t launch_lattice(lbib_ctx* c, const LatticeArgs& a, bool nodes, bool mask);
hipError_t launch_spread_inspect(lbib_ctx* c, const LatticeArgs& a);
hipError_t launch_init(lbib_ctx* c, const double* stage_rho, const double* stage_u, const double* stage_phi,
                       int has_rho, int has_u, int has_phi);
hipError_t launch_moments(lbib_ctx* c, double* out);
// partial: reduce_blocks(nn) x 5 doubles; with the monitor, count (out = count + 1) and err
hipError_t launch_reduce(lbib_ctx* c, double* partial, double* out_dev, double* count = nullptr, int* err = nullptr);
hipError_t launch_err_mirror(lbib_ctx* c, int* host_dev);
int reduce_blocks(int64_t nn);
// the file-scope scratch of the reduction that allocates nothing (k_lattice.hip): its device
// address on a device, resolved once per device by reduce_scratch_init (with that device current)
hipError_t reduce_scratch_init(int device);
double* reduce_scratch_ptr(int device);
int reduce_scratch_blocks();
hipError_t launch_membrane(lbib_ctx* c, const MembraneArgs& a);
hipError_t launch_lists(lbib_ctx* c, const ListArgs& a, int which);   // 0 count, 1 scan, 2 fill
// batched forms: one launch over (simulation, work unit) items named by device tables
hipError_t launch_lattice_batch(const LatticeArgs* tab, const int2* work, int nwork, int S, int storage, int rows,
                                bool mask, hipStream_t stream);
hipError_t launch_membrane_batch(const MembraneArgs* tab, const int2* work, int nwork, int max_cell_nodes,
                                 hipStream_t stream);
hipError_t launch_lists_batch(const ListArgs* tab, const int2* work, int nwork, int nsims, int which,
                              hipStream_t stream);
hipError_t launch_forces_out(lbib_ctx* c, float2* F);
hipError_t launch_raster(lbib_ctx* c, const RasterArgs& a);
hipError_t launch_fill_i32(lbib_ctx* c, int* p, int64_t n, int v);
hipError_t launch_fill_u16(lbib_ctx* c, uint16_t* p, int64_t n);
hipError_t launch_fill_f32(lbib_ctx* c, float* p, int64_t n);
hipError_t launch_ade(lbib_ctx* c, const AdeArgs& a, bool fp64, hipStream_t stream);
hipError_t launch_ade_copy(lbib_ctx* c, void* work, bool fp64, bool to_work);
unsigned ade_blocks(int64_t nn);
hipError_t launch_ade_hist(const double* partial, int nblocks, int S, double* hist, int slots, hipStream_t stream);

// batched single-species ADE-only iterations (k_ade.hip)
hipError_t ade_batch_launch(const AdeBatchArgs& a, bool fp64, hipStream_t s);
hipError_t ade_batch_hist_launch(const AdeBatchArgs& a, double* hist, hipStream_t s);
hipError_t ade_batch_init_launch(const double* phi, void* g, int64_t nn, int nx, int ny, int walls, int B, bool fp64,
                                 hipStream_t s);
hipError_t ade_batch_phi_launch(const void* g, double* phi, int64_t nn, int nx, int ny, int walls, int B, bool fp64,
                                hipStream_t s);

}  // namespace lbib

namespace lbib {

// kernel arguments of a context at a given buffer parity / tile height (api.hip)
LatticeArgs lattice_args_at(lbib_ctx* c, int cur);
MembraneArgs membrane_args_at(lbib_ctx* c, int cur, int advect);
ListArgs list_args_h(lbib_ctx* c, int lty);
lbib_status build_lists(lbib_ctx* c);
lbib_status check_err_flag(lbib_ctx* c);
const char* err_text(int flags);

}  // namespace lbib

// Many contexts stepped together (batch.hip): each launch of the step covers every simulation
// of a group, with per-simulation arguments in device tables (one per buffer parity).  With two
// groups the groups' step chains run on two streams, so that one group's latency-bound
// membrane and list kernels overlap the other's bandwidth-bound lattice pass.
struct lbib_batch_group {
    std::vector<int> sims;           // indices into lbib_batch::sims
    lbib::LatticeArgs* d_lat[2] = {nullptr, nullptr};    // [group sims] per parity
    lbib::MembraneArgs* d_mem[2] = {nullptr, nullptr};
    lbib::ListArgs* d_list = nullptr;
    int2* d_lat_work = nullptr;      // (group simulation, tile)
    int2* d_mem_work = nullptr;      // (group simulation, cell)
    int2* d_node_work = nullptr;     // (group simulation, block of LIST_THREADS nodes)
    int n_lat_work = 0, n_mem_work = 0, n_node_work = 0;
    int max_cell_nodes = 0;
};

struct lbib_batch {
    std::vector<lbib_ctx*> sims;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t side = nullptr;      // the second group's stream
    hipEvent_t fork = nullptr, join = nullptr;
    hipEvent_t done = nullptr;
    std::string err;
    bool broken = false;             // an adopted context was destroyed

    int S = 0, storage = 0;
    bool mask = false;
    int lty = 0;                     // lattice tile height (rows) of the batched pass
    int ngroups = 1;
    int since = 0;                   // steps since the last list build
    int par = 0;                     // parity of the steps taken (buffer parity relative to cur0)
    std::vector<int> cur0;
    std::vector<lbib_batch_group> groups;
    int64_t updates_per_step = 0;    // lattice nodes of all simulations

    hipGraphExec_t graph = nullptr;  // LIST_PERIOD steps from an aligned state
    hipStream_t capture_stream = nullptr;
};
