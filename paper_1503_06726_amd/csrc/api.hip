// C ABI of the lbib library: context management, validation, the step loop and data
// movement.  All device work is issued on the context's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "lbib_internal.h"

using namespace lbib;

namespace {

#define LBIB_HIP(ctx, call)                                                                   \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            (ctx)->err = std::string(#call) + " failed: " + hipGetErrorString(e_);            \
            return e_ == hipErrorOutOfMemory ? LBIB_ENOMEM : LBIB_EDEVICE;                    \
        }                                                                                     \
    } while (0)

template <typename T>
lbib_status dev_alloc(lbib_ctx* c, T** p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        c->err = std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) + " bytes failed: " +
                 hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? LBIB_ENOMEM : LBIB_EDEVICE;
    }
    c->device_bytes += count * sizeof(T);
    return LBIB_OK;
}

template <typename T>
void dev_free(lbib_ctx* c, T*& p, size_t count)
{
    if (p) {
        (void)hipFree((void*)p);
        c->device_bytes -= (count ? count : 1) * sizeof(T);
    }
    p = nullptr;
}

// persistent arrays: a bound workspace owns their memory, so only the pointer is dropped
template <typename T>
void state_free(lbib_ctx* c, T*& p, size_t count)
{
    if (c->ws)
        p = nullptr;
    else
        dev_free(c, p, count);
}

#define LBIB_TRY(expr)                  \
    do {                                \
        lbib_status s_ = (expr);        \
        if (s_ != LBIB_OK) return s_;   \
    } while (0)

// -------------------------------------------------------------------------------------
// timing
// -------------------------------------------------------------------------------------
hipEvent_t take_event(lbib_ctx* c)
{
    if (!c->free_events.empty()) {
        hipEvent_t e = c->free_events.back();
        c->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

lbib_status harvest(lbib_ctx* c)
{
    if (c->pending.empty()) return LBIB_OK;
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    for (auto& t : c->pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
            c->t_ms[t.kernel] += ms;
            c->t_count[t.kernel] += 1;
        }
        c->free_events.push_back(t.start);
        c->free_events.push_back(t.stop);
    }
    c->pending.clear();
    return LBIB_OK;
}

struct Timed {
    lbib_ctx* c;
    int kernel;
    hipEvent_t start = nullptr, stop = nullptr;
    Timed(lbib_ctx* ctx, int k) : c(ctx), kernel(k)
    {
        if (!c->timing) return;
        start = take_event(c);
        stop = take_event(c);
        if (start) (void)hipEventRecord(start, c->stream);
    }
    ~Timed()
    {
        if (!c->timing || !start || !stop) return;
        (void)hipEventRecord(stop, c->stream);
        c->pending.push_back({kernel, start, stop});
    }
};

// -------------------------------------------------------------------------------------
// kernel argument builders
// -------------------------------------------------------------------------------------
}  // namespace

namespace lbib {

LatticeArgs lattice_args_at(lbib_ctx* c, int cur)
{
    LatticeArgs a;
    std::memset(&a, 0, sizeof a);
    const lbib_params& p = c->p;
    a.fsrc = c->f[cur];
    a.fdst = c->f[1 - cur];
    a.gsrc = c->g[cur];
    a.gdst = c->g[1 - cur];
    a.nn = c->nn;
    a.frow = c->frow();
    a.grow = c->grow();
    a.gchunk = c->gchunk();
    a.nx = p.nx;
    a.ny = p.ny;
    a.walls = p.bc_y == LBIB_WALLS;
    a.ntx = c->ntx;
    a.omega = (float)(1.0 / p.tau);
    a.rho0 = (float)p.rho0;
    for (int s = 0; s < 2; ++s) {
        const lbib_species& sp = p.species[s];
        const double tau_s = 3.0 * sp.D + 0.5;    // D = cs2 (tau_D - 1/2), cs2 = 1/3
        a.omega_s_d[s] = s < c->S ? 1.0 / tau_s : 0.0;
        a.omega_s[s] = (float)a.omega_s_d[s];
        a.phi_ref_d[s] = sp.phi_ref;
        a.phi_ref[s] = (float)sp.phi_ref;
        a.react[s] = s < c->S ? sp.reaction : 0;
        for (int k = 0; k < 4; ++k) {
            a.rc_d[s][k] = sp.c[k];
            a.rc[s][k] = (float)sp.c[k];
        }
    }
    a.bodyx = (float)p.body_accel[0];
    a.bodyy = (float)p.body_accel[1];
    a.omega_d = 1.0 / p.tau;
    a.bodyx_d = p.body_accel[0];
    a.bodyy_d = p.body_accel[1];
    a.kernel = p.delta_kernel;
    a.t_off = c->n_cells ? c->d_t_off : nullptr;
    a.t_list = c->d_list;
    a.rec = c->d_rec;
    a.rec_ij = c->d_rec_ij;
    a.part = c->d_part;
    a.n_nodes = c->n_nodes;
    a.inside = c->inside[cur];
    a.inside_clr = c->inside[1 - cur];
    a.wpr = c->wpr;
    a.noflux = c->n_cells ? no_flux_bits(p) : 0;
    a.cmap = c->n_cells ? c->cmap : nullptr;
    a.A0 = c->d_A0;
    a.area = c->d_area;
    a.msrc = p.mass_source;
    a.alpha = p.area_alpha;
    a.pring = p.pressure_ring;
    a.gamma = p.mass_phi_gamma;
    a.nsrc = c->d_nsrc;
    a.pmap = c->d_pmap;
    if (a.noflux && c->nfq[0]) {
        a.nfq = c->nfq[cur];
        a.nfm = c->nfm[cur];
        a.nfphi = c->nfphi[cur];
        a.nfu = c->nfu[cur];
        a.nfphi_out = c->nfphi[1 - cur];
        a.nfu_out = c->nfu[1 - cur];
        a.nf_bb = p.no_flux_bounce ? (c->nf_fresh ? 2 : 1) : 0;
    }
    a.e_out = nullptr;
    return a;
}

MembraneArgs membrane_args_at(lbib_ctx* c, int cur, int advect)
{
    MembraneArgs a;
    std::memset(&a, 0, sizeof a);
    a.off = c->d_off;
    a.X = c->d_X;
    a.l0 = c->d_l0;
    a.A0 = c->d_A0;
    a.area = c->d_area;
    a.part = c->d_part;
    a.cnt = c->d_cnt;
    a.n_nodes = c->n_nodes;
    a.ij_list = c->d_ijlist;
    a.rec = c->d_rec;
    a.rec_ij = c->d_rec_ij;
    a.inside = c->inside[cur];
    a.src = c->d_src;
    a.cmap = c->cmap;
    a.wpr = c->wpr;
    a.err = c->d_err;
    a.nn = c->nn;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.walls = c->p.bc_y == LBIB_WALLS;
    a.kernel = c->p.delta_kernel;
    a.k_spring = c->p.k_spring;
    a.phi_m = c->p.phi_m;
    a.kappa = c->p.kappa_area;
    a.advect = advect;
    a.raster = c->mask_needed ? 1 : 0;
    a.need_area = area_in_step(c->p) ? 1 : 0;
    if (c->nfq[0]) {
        a.nfq = c->nfq[cur];
        a.nfm = (unsigned*)c->nfm[cur];
        a.nfq_old = c->nfq[1 - cur];
        a.nfm_old = c->nfm[1 - cur];
    }
    return a;
}

// lists for lattice tiles of lty rows
ListArgs list_args_h(lbib_ctx* c, int lty)
{
    ListArgs a;
    std::memset(&a, 0, sizeof a);
    a.X = c->d_X;
    a.ij_list = c->d_ijlist;
    a.count = c->d_t_count;
    a.off = c->d_t_off;
    a.cursor = c->d_t_cur;
    a.list = c->d_list;
    a.cnt = c->d_cnt;
    a.n = c->n_nodes;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.walls = c->p.bc_y == LBIB_WALLS;
    a.ntx = c->ntx;
    a.nlty = (c->p.ny + lty - 1) / lty;
    a.ntiles = c->ntx * a.nlty;
    a.lty = lty;
    a.lty_shift = 0;
    while ((1 << a.lty_shift) < lty) ++a.lty_shift;
    return a;
}

}  // namespace lbib

namespace {

LatticeArgs lattice_args(lbib_ctx* c) { return lattice_args_at(c, c->cur); }
MembraneArgs membrane_args(lbib_ctx* c, int advect) { return membrane_args_at(c, c->cur, advect); }
ListArgs list_args(lbib_ctx* c) { return list_args_h(c, LTILE_Y); }

RasterArgs raster_args(lbib_ctx* c, uint16_t* ids)
{
    RasterArgs a;
    a.off = c->d_off;
    a.X = c->d_X;
    a.mask = ids;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.walls = c->p.bc_y == LBIB_WALLS;
    return a;
}

#define LBIB_LAUNCH(ctx, call)                                                               \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) {                                                              \
            (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);                  \
            return LBIB_EDEVICE;                                                             \
        }                                                                                    \
    } while (0)

}  // namespace

// List every node in the lattice tiles its stencil can reach from its current position
// (within the drift margin).
lbib_status lbib::build_lists(lbib_ctx* c)
{
    Timed tm(c, LBIB_K_LISTS);
    const ListArgs a = list_args(c);
    for (int which = 0; which < 3; ++which) LBIB_LAUNCH(c, launch_lists(c, a, which));
    c->steps_since_lists = 0;
    return LBIB_OK;
}

namespace {

// interpolation and advection (advect = 1), forces and records of the new positions, and,
// when a reaction reads it, the domain map
lbib_status membrane(lbib_ctx* c, int advect)
{
    Timed tm(c, LBIB_K_MEMBRANE);
    LBIB_LAUNCH(c, launch_membrane(c, membrane_args(c, advect)));
    return LBIB_OK;
}

lbib_status ensure_stage(lbib_ctx* c, size_t doubles)
{
    if (c->stage_bytes >= doubles * sizeof(double)) return LBIB_OK;
    if (c->ws) {
        // the workspace's staging area is sized for every read-back of its node capacity
        c->err = "the workspace's staging area holds " + std::to_string(c->ws_stage_doubles) +
                 " doubles; " + std::to_string(doubles) + " are needed";
        return LBIB_ENOMEM;
    }
    if (c->d_stage) {
        LBIB_HIP(c, hipStreamSynchronize(c->stream));
        dev_free(c, c->d_stage, c->stage_bytes / sizeof(double));
        c->stage_bytes = 0;
    }
    LBIB_TRY(dev_alloc(c, &c->d_stage, doubles));
    c->stage_bytes = doubles * sizeof(double);
    return LBIB_OK;
}

}  // namespace

// The error flags that completed device work has copied to pinned host memory (no
// synchronisation): LBIB_ENUMERIC once any is set.
static lbib_status host_flags(lbib_ctx* c)
{
    const int h = c->h_err ? __atomic_load_n(c->h_err, __ATOMIC_ACQUIRE) : 0;
    if (!h) return LBIB_OK;
    c->err = std::string("stepping stopped: ") + lbib::err_text(h);
    return LBIB_ENUMERIC;
}

const char* lbib::err_text(int h)
{
    if (h & ERR_NONFINITE) return "a membrane node position or force became non-finite";
    if (h & ERR_MARGIN) return "a membrane node moved more than 2 lattice units between list rebuilds (velocity too large)";
    if (h & ERR_FIELDS) return "a lattice sum of the monitor is not finite";
    return "device error flag";
}

lbib_status lbib::check_err_flag(lbib_ctx* c)
{
    int h = 0;
    LBIB_HIP(c, hipMemcpyAsync(&h, c->d_err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    if (h) {
        c->err = err_text(h);
        return LBIB_ENUMERIC;
    }
    return LBIB_OK;
}

namespace {

void free_nodes(lbib_ctx* c)
{
    const size_t N = (size_t)c->n_nodes, C = (size_t)c->n_cells;
    state_free(c, c->d_off, C + 1);
    state_free(c, c->d_X, N);
    state_free(c, c->d_l0, N);
    state_free(c, c->d_A0, C);
    state_free(c, c->d_area, C);
    state_free(c, c->d_ijlist, N);
    state_free(c, c->d_part, N * MAX_NODE_TILES);
    state_free(c, c->d_cnt, N);
    state_free(c, c->d_rec, N);
    state_free(c, c->d_rec_ij, N);
    state_free(c, c->d_list, N * MAX_NODE_TILES);
    state_free(c, c->d_src, C);
    c->ws_src = nullptr;
    c->n_nodes = 0;
    c->n_cells = 0;
    c->max_cell_nodes = 0;
    c->mask_needed = false;
    c->steps_since_lists = 0;
}

void free_all(lbib_ctx* c)
{
    free_nodes(c);
    const size_t nn = (size_t)c->nn;
    for (int b = 0; b < 2; ++b) {
        char* fb = (char*)c->f[b];
        char* gb = (char*)c->g[b];
        state_free(c, fb, c->f_elems() * c->pop_bytes);
        state_free(c, gb, c->g_elems() * c->pop_bytes);
        c->f[b] = c->g[b] = nullptr;
    }
    for (int b = 0; b < 2; ++b) state_free(c, c->inside[b], (size_t)c->ny_words());
    state_free(c, c->cmap, (size_t)c->nn);
    for (int b = 0; b < 2; ++b) {
        state_free(c, c->nfq[b], 4 * (size_t)c->nn);
        state_free(c, c->nfm[b], c->nfm_bytes());
        state_free(c, c->nfphi[b], (size_t)c->S * (size_t)c->nn);
        state_free(c, c->nfu[b], (size_t)c->nn);
    }
    dev_free(c, c->d_nsrc, (size_t)c->nn);       // never in a workspace
    dev_free(c, c->d_pmap, (size_t)c->nn);
    state_free(c, c->d_t_count, (size_t)c->tile_cap);
    state_free(c, c->d_t_off, (size_t)c->tile_cap + 1);
    state_free(c, c->d_t_cur, (size_t)c->tile_cap);
    state_free(c, c->d_err, 1);
    state_free(c, c->d_mon, 8);
    state_free(c, c->d_partial, c->partial_count * 5);
    if (c->d_stage) state_free(c, c->d_stage, c->stage_bytes / sizeof(double));
    c->stage_bytes = 0;
    for (auto& t : c->pending) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    c->pending.clear();
    for (auto e : c->free_events) (void)hipEventDestroy(e);
    c->free_events.clear();
    if (c->h_err) (void)hipHostFree(c->h_err);
    c->h_err = c->h_err_dev = nullptr;
}

// -------------------------------------------------------------------------------------
// workspace layout: the persistent arrays in a fixed order, each piece starting on a
// WS_ALIGN boundary.  The lattice part depends on the parameters only; the node part follows
// it and is laid out for the current nodes and cells (every piece grows with N and C, and
// C <= N / 3 since a cell has at least 3 nodes, so a part sized for N nodes holds any set of
// at most N nodes).
// -------------------------------------------------------------------------------------
enum Piece {
    PC_F0, PC_F1, PC_G0, PC_G1, PC_IN0, PC_IN1, PC_CMAP,
    PC_NFQ0, PC_NFQ1, PC_NFM0, PC_NFM1, PC_NFPHI0, PC_NFPHI1, PC_NFU0, PC_NFU1,
    PC_TCOUNT, PC_TOFF, PC_TCUR, PC_ERR, PC_MON, PC_PARTIAL, PC_STAGE,
    PC_OFF, PC_X, PC_L0, PC_A0, PC_AREA, PC_IJ, PC_PART, PC_CNT, PC_REC, PC_RECIJ, PC_LIST, PC_SRC,
    PC_COUNT
};
constexpr int PC_NODE0 = PC_OFF;
constexpr size_t WS_ALIGN = 256;

size_t ws_round(size_t b) { return (b + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }

// lattice geometry of a context (everything the layout and the launches derive from params)
void set_geometry(lbib_ctx* c, const lbib_params* p)
{
    c->p = *p;
    c->nn = (int64_t)p->nx * p->ny;
    c->S = p->n_species;
    c->ntx = (p->nx + TILE_X - 1) / TILE_X;
    c->nlty = (p->ny + LTILE_Y - 1) / LTILE_Y;
    c->nltiles = c->ntx * c->nlty;
    c->tile_cap = c->ntx * ((p->ny + MIN_LTILE_Y - 1) / MIN_LTILE_Y);
    c->wpr = (p->nx + 31) / 32;
    c->partial_count = 4096;
    c->pop_bytes = (p->storage == LBIB_STORAGE_FP32) ? 4 : 2;
}

// staging a workspace provides: the largest read-back (moments, spread field, node forces)
size_t ws_stage_doubles(const lbib_ctx& c, int64_t node_cap)
{
    return std::max<size_t>({(size_t)c.nn * (size_t)(3 + c.S), (size_t)node_cap, 8});
}

void piece_bytes(const lbib_ctx& c, int64_t n_nodes, int64_t n_cells, size_t stage_doubles, size_t b[PC_COUNT])
{
    const size_t N = (size_t)n_nodes, C = (size_t)n_cells;
    b[PC_F0] = b[PC_F1] = c.f_elems() * c.pop_bytes;
    b[PC_G0] = b[PC_G1] = c.S ? c.g_elems() * c.pop_bytes : 0;
    b[PC_IN0] = b[PC_IN1] = (size_t)c.ny_words() * sizeof(unsigned);
    b[PC_CMAP] = mass_sources(c.p) ? (size_t)c.nn * sizeof(unsigned) : 0;
    const bool nf1 = no_flux_first(c.p);
    b[PC_NFQ0] = b[PC_NFQ1] = nf1 ? 4 * (size_t)c.nn * sizeof(float) : 0;
    b[PC_NFM0] = b[PC_NFM1] = nf1 ? c.nfm_bytes() : 0;
    b[PC_NFPHI0] = b[PC_NFPHI1] = nf1 ? (size_t)c.S * (size_t)c.nn * sizeof(float) : 0;
    b[PC_NFU0] = b[PC_NFU1] = nf1 ? (size_t)c.nn * sizeof(float2) : 0;
    b[PC_TCOUNT] = b[PC_TCUR] = (size_t)c.tile_cap * sizeof(int);
    b[PC_TOFF] = ((size_t)c.tile_cap + 1) * sizeof(int);
    b[PC_ERR] = sizeof(int);
    b[PC_MON] = 8 * sizeof(double);
    b[PC_PARTIAL] = c.partial_count * 5 * sizeof(double);
    b[PC_STAGE] = stage_doubles * sizeof(double);
    b[PC_OFF] = N ? (C + 1) * sizeof(int) : 0;
    b[PC_X] = N * sizeof(double2);
    b[PC_L0] = N * sizeof(double);
    b[PC_A0] = b[PC_AREA] = C * sizeof(double);
    b[PC_IJ] = b[PC_RECIJ] = N * sizeof(int);
    b[PC_PART] = N * MAX_NODE_TILES * sizeof(float2);
    b[PC_CNT] = N;
    b[PC_REC] = N * sizeof(float4);
    b[PC_LIST] = N * MAX_NODE_TILES * sizeof(int);
    b[PC_SRC] = C;
}

void** piece_slot(lbib_ctx* c, int i)
{
    switch (i) {
    case PC_F0: return &c->f[0];
    case PC_F1: return &c->f[1];
    case PC_G0: return &c->g[0];
    case PC_G1: return &c->g[1];
    case PC_IN0: return reinterpret_cast<void**>(&c->inside[0]);
    case PC_IN1: return reinterpret_cast<void**>(&c->inside[1]);
    case PC_CMAP: return reinterpret_cast<void**>(&c->cmap);
    case PC_NFQ0: return reinterpret_cast<void**>(&c->nfq[0]);
    case PC_NFQ1: return reinterpret_cast<void**>(&c->nfq[1]);
    case PC_NFM0: return reinterpret_cast<void**>(&c->nfm[0]);
    case PC_NFM1: return reinterpret_cast<void**>(&c->nfm[1]);
    case PC_NFPHI0: return reinterpret_cast<void**>(&c->nfphi[0]);
    case PC_NFPHI1: return reinterpret_cast<void**>(&c->nfphi[1]);
    case PC_NFU0: return reinterpret_cast<void**>(&c->nfu[0]);
    case PC_NFU1: return reinterpret_cast<void**>(&c->nfu[1]);
    case PC_TCOUNT: return reinterpret_cast<void**>(&c->d_t_count);
    case PC_TOFF: return reinterpret_cast<void**>(&c->d_t_off);
    case PC_TCUR: return reinterpret_cast<void**>(&c->d_t_cur);
    case PC_ERR: return reinterpret_cast<void**>(&c->d_err);
    case PC_MON: return reinterpret_cast<void**>(&c->d_mon);
    case PC_PARTIAL: return reinterpret_cast<void**>(&c->d_partial);
    case PC_STAGE: return reinterpret_cast<void**>(&c->d_stage);
    case PC_OFF: return reinterpret_cast<void**>(&c->d_off);
    case PC_X: return reinterpret_cast<void**>(&c->d_X);
    case PC_L0: return reinterpret_cast<void**>(&c->d_l0);
    case PC_A0: return reinterpret_cast<void**>(&c->d_A0);
    case PC_AREA: return reinterpret_cast<void**>(&c->d_area);
    case PC_IJ: return reinterpret_cast<void**>(&c->d_ijlist);
    case PC_PART: return reinterpret_cast<void**>(&c->d_part);
    case PC_CNT: return reinterpret_cast<void**>(&c->d_cnt);
    case PC_REC: return reinterpret_cast<void**>(&c->d_rec);
    case PC_RECIJ: return reinterpret_cast<void**>(&c->d_rec_ij);
    case PC_LIST: return reinterpret_cast<void**>(&c->d_list);
    default: return reinterpret_cast<void**>(&c->d_src);
    }
}

// bytes of a workspace holding the lattice part and a node part for node_cap nodes
size_t ws_total(const lbib_ctx& c, int64_t node_cap)
{
    size_t b[PC_COUNT];
    piece_bytes(c, node_cap, node_cap / 3, ws_stage_doubles(c, node_cap), b);
    size_t t = 0;
    for (int i = 0; i < PC_COUNT; ++i) t += ws_round(b[i]);
    return t;
}

size_t ws_lattice_part(const lbib_ctx& c, size_t stage_doubles)
{
    size_t b[PC_COUNT];
    piece_bytes(c, 0, 0, stage_doubles, b);
    size_t t = 0;
    for (int i = 0; i < PC_NODE0; ++i) t += ws_round(b[i]);
    return t;
}

// node pieces of the bound workspace for N nodes in C cells (N <= ws_node_cap)
void carve_nodes(lbib_ctx* c, int64_t N, int64_t C)
{
    size_t b[PC_COUNT];
    piece_bytes(*c, N, C, 0, b);
    size_t off = c->ws_node_base;
    for (int i = PC_NODE0; i < PC_COUNT; ++i) {
        void* q = b[i] ? (void*)(c->ws + off) : nullptr;
        if (i == PC_SRC)
            c->ws_src = (uint8_t*)q;     // claimed by lbib_set_source_cells
        else
            *piece_slot(c, i) = q;
        off += ws_round(b[i]);
    }
}

lbib_status alloc_nodes(lbib_ctx* c, size_t N, size_t C)
{
    if (c->ws) {
        carve_nodes(c, (int64_t)N, (int64_t)C);
        return LBIB_OK;
    }
    lbib_status s = dev_alloc(c, &c->d_off, C + 1);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_X, N);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_l0, N);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_A0, C);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_area, C);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_ijlist, N);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_part, N * MAX_NODE_TILES);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_cnt, N);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_rec, N);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_rec_ij, N);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_list, N * MAX_NODE_TILES);
    return s;
}

// Moves every persistent array into the workspace [base, base + bytes) with room for
// node_cap nodes, or, with base NULL, into memory the library allocates.  The contents are
// copied on the context's stream; the old memory is released only after all copies
// succeeded, so on failure the context is unchanged.
lbib_status relocate(lbib_ctx* c, char* base, size_t bytes, int64_t node_cap)
{
    const size_t stage_d = base ? ws_stage_doubles(*c, node_cap) : 0;
    size_t b[PC_COUNT];
    piece_bytes(*c, c->n_nodes, c->n_cells, stage_d, b);
    void* nw[PC_COUNT] = {};
    uint8_t* new_src_slot = nullptr;
    size_t new_bytes = 0;
    lbib_status s = LBIB_OK;
    if (base) {
        size_t off = 0;
        for (int i = 0; i < PC_COUNT; ++i) {
            if (i == PC_NODE0) off = ws_lattice_part(*c, stage_d);
            if (b[i]) nw[i] = base + off;
            off += ws_round(b[i]);
        }
        new_src_slot = (uint8_t*)nw[PC_SRC];
        if (!c->d_src) nw[PC_SRC] = nullptr;
    } else {
        for (int i = 0; i < PC_COUNT && s == LBIB_OK; ++i) {
            if (!b[i] || i == PC_STAGE || (i == PC_SRC && !c->d_src)) continue;
            hipError_t e = hipMalloc(&nw[i], b[i]);
            if (e != hipSuccess) {
                nw[i] = nullptr;
                c->err = std::string("hipMalloc of ") + std::to_string(b[i]) + " bytes failed: " +
                         hipGetErrorString(e);
                s = e == hipErrorOutOfMemory ? LBIB_ENOMEM : LBIB_EDEVICE;
            } else {
                new_bytes += b[i];
            }
        }
    }
    for (int i = 0; i < PC_COUNT && s == LBIB_OK; ++i) {
        void* old = *piece_slot(c, i);
        if (i == PC_STAGE || !old || !nw[i]) continue;
        hipError_t e = hipMemcpyAsync(nw[i], old, b[i], hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) {
            c->err = std::string("hipMemcpyAsync of the state failed: ") + hipGetErrorString(e);
            s = LBIB_EDEVICE;
        }
    }
    if (s == LBIB_OK) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            c->err = std::string("hipStreamSynchronize failed: ") + hipGetErrorString(e);
            s = LBIB_EDEVICE;
        }
    }
    if (s != LBIB_OK) {
        if (!base)
            for (int i = 0; i < PC_COUNT; ++i)
                if (nw[i]) (void)hipFree(nw[i]);
        return s;
    }
    if (!c->ws) {
        for (int i = 0; i < PC_COUNT; ++i) {
            void* old = *piece_slot(c, i);
            if (old) (void)hipFree(old);
        }
    }
    for (int i = 0; i < PC_COUNT; ++i) *piece_slot(c, i) = nw[i];
    c->device_bytes = new_bytes;
    c->ws = base;
    c->ws_bytes = base ? bytes : 0;
    c->ws_node_cap = base ? node_cap : 0;
    c->ws_node_base = base ? ws_lattice_part(*c, stage_d) : 0;
    c->ws_stage_doubles = stage_d;
    c->ws_src = new_src_slot;
    c->stage_bytes = stage_d * sizeof(double);
    return LBIB_OK;
}

bool any_source_decay(const lbib_params& p)
{
    for (int s = 0; s < p.n_species; ++s)
        if (p.species[s].reaction == LBIB_REACT_SOURCE_DECAY) return true;
    return false;
}

// no-flux membranes, first-order form: no link of buffer b cut (wall distances +inf)
lbib_status clear_cuts(lbib_ctx* c, int b)
{
    if (!c->nfq[b]) return LBIB_OK;
    LBIB_LAUNCH(c, launch_fill_i32(c, (int*)c->nfq[b], 4 * c->nn, 0x7F800000));
    LBIB_LAUNCH(c, launch_fill_i32(c, (int*)c->nfm[b], (int64_t)(c->nfm_bytes() / 4), 0));
    return LBIB_OK;
}

lbib_status init_fields(lbib_ctx* c, const double* rho, const double* u, const double* phi)
{
    const size_t nn = (size_t)c->nn;
    const size_t need = nn * (size_t)((rho ? 1 : 0) + (u ? 2 : 0) + (phi ? c->S : 0));
    double *d_rho = nullptr, *d_u = nullptr, *d_phi = nullptr;
    if (need) {
        LBIB_TRY(ensure_stage(c, need));
        double* q = c->d_stage;
        if (rho) {
            d_rho = q;
            LBIB_HIP(c, hipMemcpyAsync(d_rho, rho, nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
            q += nn;
        }
        if (u) {
            d_u = q;
            LBIB_HIP(c, hipMemcpyAsync(d_u, u, 2 * nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
            q += 2 * nn;
        }
        if (phi && c->S) {
            d_phi = q;
            LBIB_HIP(c, hipMemcpyAsync(d_phi, phi, (size_t)c->S * nn * sizeof(double), hipMemcpyHostToDevice,
                                       c->stream));
        }
    }
    LBIB_LAUNCH(c, launch_init(c, d_rho, d_u, d_phi, d_rho != nullptr, d_u != nullptr, d_phi != nullptr));
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    c->nf_fresh = true;
    return LBIB_OK;
}

// is the monitor due at the end of the period that brings the count of periods to `period`?
bool monitor_due(const lbib_ctx* c, int64_t period)
{
    return c->p.monitor_every > 0 && period % (c->p.monitor_every / GRAPH_STEPS) == 0;
}

// one coupled step, launched directly on the context's stream
lbib_status one_step(lbib_ctx* c)
{
    const bool nodes = c->n_cells > 0;
    {
        Timed tm(c, LBIB_K_LATTICE);
        LBIB_LAUNCH(c, launch_lattice(c, lattice_args(c), nodes, c->mask_needed));
    }
    c->nf_fresh = false;
    c->cur = 1 - c->cur;
    if (nodes) LBIB_TRY(membrane(c, 1));
    if (++c->steps_since_lists >= LIST_PERIOD) {       // a period ends: lists rebuilt, monitor
        if (nodes) LBIB_TRY(build_lists(c));
        c->steps_since_lists = 0;
        if (monitor_due(c, ++c->period_count))         // FP64 sums of the new state
            LBIB_LAUNCH(c, launch_reduce(c, c->d_partial, c->d_mon + 1, c->d_mon, c->d_err));
    }
    if (c->timing && c->pending.size() > 4096) LBIB_TRY(harvest(c));
    return LBIB_OK;
}

void drop_graphs(lbib_ctx* c)
{
    for (int i = 0; i < 2; ++i)
        for (int m = 0; m < 2; ++m)
            if (c->graph[i][m]) {
                (void)hipGraphExecDestroy(c->graph[i][m]);
                c->graph[i][m] = nullptr;
            }
}

// Capture GRAPH_STEPS steps (kernels only: no memsets or copies) on a private stream.  The
// kernels' arguments follow the buffer parity, which is back where it started after the
// period, so the host-side state is restored once the capture ends.
lbib_status capture_steps(lbib_ctx* c, hipGraphExec_t* out)
{
    if (!c->capture_stream) LBIB_HIP(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    const int cur0 = c->cur, since0 = c->steps_since_lists;
    const int64_t count0 = c->period_count;
    hipStream_t user = c->stream;
    c->stream = c->capture_stream;
    hipGraph_t graph = nullptr;
    lbib_status st = LBIB_OK;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = LBIB_EDEVICE;
    } else {
        for (int k = 0; k < GRAPH_STEPS && st == LBIB_OK; ++k) st = one_step(c);
        if (st == LBIB_OK && launch_err_mirror(c, c->h_err_dev) != hipSuccess) st = LBIB_EDEVICE;
        hipError_t e = hipStreamEndCapture(c->stream, &graph);
        if (st == LBIB_OK && e != hipSuccess) st = LBIB_EDEVICE;
    }
    c->stream = user;
    c->cur = cur0;
    c->steps_since_lists = since0;
    c->period_count = count0;
    if (st == LBIB_OK && hipGraphInstantiate(out, graph, nullptr, nullptr, 0) != hipSuccess) st = LBIB_EDEVICE;
    if (graph) (void)hipGraphDestroy(graph);
    if (st != LBIB_OK) {
        *out = nullptr;
        c->use_graphs = false;          // fall back to direct launches
        if (c->err.empty()) c->err = "step graph capture failed; using direct launches";
        return LBIB_OK;
    }
    return LBIB_OK;
}

// A context adopted by a batch is stepped on the batch's stream: changes are refused, reads
// wait for the batch's last work.
lbib_status refuse_if_batched(lbib_ctx* c)
{
    if (!c->batch) return LBIB_OK;
    c->err = "the context is stepped by a batch; destroy the batch first";
    return LBIB_ESTATE;
}

lbib_status join_batch(lbib_ctx* c)
{
    if (c->batch && c->batch_done) LBIB_HIP(c, hipStreamWaitEvent(c->stream, c->batch_done, 0));
    return LBIB_OK;
}

}  // namespace

// =======================================================================================
// C ABI
// =======================================================================================
extern "C" {

int32_t lbib_version(void) { return LBIB_VERSION; }

const char* lbib_status_string(lbib_status s)
{
    switch (s) {
    case LBIB_OK: return "LBIB_OK";
    case LBIB_EINVAL: return "LBIB_EINVAL";
    case LBIB_ENOMEM: return "LBIB_ENOMEM";
    case LBIB_EDEVICE: return "LBIB_EDEVICE";
    case LBIB_ESTATE: return "LBIB_ESTATE";
    case LBIB_ENUMERIC: return "LBIB_ENUMERIC";
    }
    return "LBIB_UNKNOWN";
}

const char* lbib_last_error(const lbib_ctx* ctx)
{
    if (!ctx) return "";
    return ctx->err.c_str();
}

lbib_status lbib_create(const lbib_params* p, void* hip_stream, lbib_ctx** out)
{
    if (!out) return LBIB_EINVAL;
    *out = nullptr;
    std::string msg;
    if (check_params(p, msg) != LBIB_OK) return LBIB_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return LBIB_EDEVICE;

    lbib_ctx* c = new (std::nothrow) lbib_ctx();
    if (!c) return LBIB_ENOMEM;
    set_geometry(c, p);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return LBIB_EDEVICE;
    }
    // the device address of the reduction scratch on this device (lbib_reduce_device); a
    // failure is reported by that call, not here
    c->scratch_ok = reduce_scratch_init(c->device) == hipSuccess;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return LBIB_EDEVICE;
        }
        c->own_stream = true;
    }
    lbib_status s = LBIB_OK;
    for (int b = 0; b < 2 && s == LBIB_OK; ++b) {
        char* fb = nullptr;
        char* gb = nullptr;
        s = dev_alloc(c, &fb, c->f_elems() * c->pop_bytes);
        c->f[b] = fb;
        if (s == LBIB_OK && c->S) {
            s = dev_alloc(c, &gb, c->g_elems() * c->pop_bytes);
            c->g[b] = gb;
        }
    }
    for (int b = 0; b < 2 && s == LBIB_OK; ++b) s = dev_alloc(c, &c->inside[b], (size_t)c->ny_words());
    if (s == LBIB_OK && mass_sources(c->p)) {
        s = dev_alloc(c, &c->cmap, (size_t)c->nn);
        if (s == LBIB_OK && launch_fill_i32(c, (int*)c->cmap, c->nn, -1) != hipSuccess) s = LBIB_EDEVICE;
    }
    if (s == LBIB_OK && no_flux_first(c->p))
        for (int b = 0; b < 2 && s == LBIB_OK; ++b) {
            s = dev_alloc(c, &c->nfq[b], 4 * (size_t)c->nn);
            if (s == LBIB_OK) s = dev_alloc(c, &c->nfm[b], c->nfm_bytes());
            if (s == LBIB_OK) s = dev_alloc(c, &c->nfphi[b], (size_t)c->S * (size_t)c->nn);
            if (s == LBIB_OK) s = dev_alloc(c, &c->nfu[b], (size_t)c->nn);
            if (s == LBIB_OK) s = clear_cuts(c, b);
        }
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_t_count, (size_t)c->tile_cap);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_t_off, (size_t)c->tile_cap + 1);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_t_cur, (size_t)c->tile_cap);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_err, 1);
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_mon, 8);
    if (s == LBIB_OK && (hipHostMalloc((void**)&c->h_err, sizeof(int), hipHostMallocMapped) != hipSuccess ||
                         hipHostGetDevicePointer((void**)&c->h_err_dev, c->h_err, 0) != hipSuccess)) {
        c->h_err_dev = nullptr;
        s = LBIB_EDEVICE;
    }
    if (s == LBIB_OK) *(volatile int*)c->h_err = 0;
    if (s == LBIB_OK) s = dev_alloc(c, &c->d_partial, c->partial_count * 5);
    if (s == LBIB_OK && (launch_fill_i32(c, (int*)c->inside[0], c->ny_words(), 0) != hipSuccess ||
                         launch_fill_i32(c, (int*)c->inside[1], c->ny_words(), 0) != hipSuccess ||
                         launch_fill_i32(c, c->d_t_count, c->tile_cap, 0) != hipSuccess ||
                         launch_fill_i32(c, c->d_t_off, c->tile_cap + 1, 0) != hipSuccess ||
                         launch_fill_i32(c, c->d_err, 1, 0) != hipSuccess ||
                         launch_fill_i32(c, (int*)c->d_mon, 16, 0) != hipSuccess))
        s = LBIB_EDEVICE;
    if (s == LBIB_OK) s = init_fields(c, nullptr, nullptr, nullptr);
    if (s != LBIB_OK) {
        (void)hipStreamSynchronize(c->stream);
        free_all(c);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return s;
    }
    *out = c;
    return LBIB_OK;
}

void lbib_destroy(lbib_ctx* c)
{
    if (!c) return;
    if (c->batch) {
        // the batch can no longer step; its work on this context ends first
        (void)hipStreamSynchronize(c->batch->stream);
        c->batch->broken = true;
        for (auto& q : c->batch->sims)
            if (q == c) q = nullptr;
        c->batch = nullptr;
    }
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    free_all(c);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

lbib_status lbib_set_cells(lbib_ctx* c, int32_t n_cells, const int32_t* off, const double* xy,
                           const double* rest_len, const double* rest_area)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(refuse_if_batched(c));
    std::string msg;
    if (check_cells(&c->p, n_cells, off, xy, rest_len, rest_area, msg) != LBIB_OK) {
        c->err = msg;
        return LBIB_EINVAL;
    }
    if (c->ws && (int64_t)off[n_cells] > c->ws_node_cap) {
        c->err = "the bound workspace holds " + std::to_string(c->ws_node_cap) + " membrane nodes; " +
                 std::to_string(off[n_cells]) + " were given";
        return LBIB_ENOMEM;
    }
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    free_nodes(c);
    c->steps_since_lists = 0;
    c->period_count = 0;
    if (n_cells == 0) return LBIB_OK;
    const size_t N = (size_t)off[n_cells], C = (size_t)n_cells;

    // rest lengths / areas default to the initial ones
    std::vector<double> l0(N), A0(C);
    int max_n = 0;
    for (size_t q = 0; q < C; ++q) {
        const size_t a = (size_t)off[q], n = (size_t)off[q + 1] - a;
        if ((int)n > max_n) max_n = (int)n;
        double A = 0.0;
        for (size_t k = 0; k < n; ++k) {
            const size_t i = a + k, j = a + (k + 1) % n;
            const double dx = xy[2 * j] - xy[2 * i], dy = xy[2 * j + 1] - xy[2 * i + 1];
            l0[i] = rest_len ? rest_len[i] : std::sqrt(dx * dx + dy * dy);
            A += (xy[2 * i] - xy[2 * a]) * (xy[2 * j + 1] - xy[2 * a + 1]) -
                 (xy[2 * j] - xy[2 * a]) * (xy[2 * i + 1] - xy[2 * a + 1]);
        }
        A0[q] = rest_area ? rest_area[q] : 0.5 * A;
    }
    lbib_status s = alloc_nodes(c, N, C);
    c->n_cells = n_cells;
    c->n_nodes = (int64_t)N;
    if (s != LBIB_OK) {
        free_nodes(c);
        return s;
    }
    c->max_cell_nodes = max_n;
    // the step keeps the inside map (and, with mass sources, the cell map)
    c->mask_needed = any_source_decay(c->p) || (no_flux_bits(c->p) != 0 && c->p.no_flux_zeroth) ||
                     mass_sources(c->p);
    LBIB_HIP(c, hipMemcpyAsync(c->d_off, off, (C + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream));
    LBIB_HIP(c, hipMemcpyAsync(c->d_X, xy, N * sizeof(double2), hipMemcpyHostToDevice, c->stream));
    LBIB_HIP(c, hipMemcpyAsync(c->d_l0, l0.data(), N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    LBIB_HIP(c, hipMemcpyAsync(c->d_A0, A0.data(), C * sizeof(double), hipMemcpyHostToDevice, c->stream));
    LBIB_LAUNCH(c, launch_fill_i32(c, c->d_t_count, c->tile_cap, 0));
    LBIB_LAUNCH(c, launch_fill_i32(c, c->d_err, 1, 0));
    LBIB_LAUNCH(c, launch_fill_i32(c, (int*)c->d_mon, 16, 0));
    c->period_count = 0;
    if (c->mask_needed)
        for (int b = 0; b < 2; ++b) LBIB_LAUNCH(c, launch_fill_i32(c, (int*)c->inside[b], c->ny_words(), 0));
    if (c->cmap) LBIB_LAUNCH(c, launch_fill_i32(c, (int*)c->cmap, c->nn, -1));   // claims of earlier cells
    for (int b = 0; b < 2; ++b) LBIB_TRY(clear_cuts(c, b));                     // cuts of earlier cells
    LBIB_TRY(build_lists(c));
    LBIB_TRY(membrane(c, 0));
    LBIB_LAUNCH(c, launch_err_mirror(c, c->h_err_dev));
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    return check_err_flag(c);
}

lbib_status lbib_set_fields(lbib_ctx* c, const double* rho, const double* u, const double* phi)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(refuse_if_batched(c));
    const int64_t nn = c->nn;
    for (int64_t i = 0; rho && i < nn; ++i)
        if (!std::isfinite(rho[i]) || !(rho[i] > 0.0)) {
            c->err = "rho must be finite and positive";
            return LBIB_EINVAL;
        }
    for (int64_t i = 0; u && i < 2 * nn; ++i)
        if (!std::isfinite(u[i])) {
            c->err = "u must be finite";
            return LBIB_EINVAL;
        }
    for (int64_t i = 0; phi && i < (int64_t)c->S * nn; ++i)
        if (!std::isfinite(phi[i])) {
            c->err = "phi must be finite";
            return LBIB_EINVAL;
        }
    return init_fields(c, rho, u, phi);
}

lbib_status lbib_step(lbib_ctx* c, int32_t n)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(refuse_if_batched(c));
    if (n < 0) {
        c->err = "negative step count";
        return LBIB_EINVAL;
    }
    LBIB_TRY(host_flags(c));
    bool direct = false;
    while (n > 0) {
        // whole periods of GRAPH_STEPS steps, aligned to the list rebuilds, replay a captured
        // graph (not while timing kernels, nor for the first step of a state set from outside
        // under the bounce-back no-flux form); with the monitor due at the period's last step,
        // the graph that ends with it
        const bool fresh_bb = c->nf_fresh && c->p.no_flux_bounce && no_flux_first(c->p);
        if (c->use_graphs && !c->timing && !fresh_bb && n >= GRAPH_STEPS && c->steps_since_lists == 0) {
            hipGraphExec_t& g = c->graph[c->cur][monitor_due(c, c->period_count + 1) ? 1 : 0];
            if (!g) LBIB_TRY(capture_steps(c, &g));
            if (g) {
                LBIB_TRY(host_flags(c));
                LBIB_HIP(c, hipGraphLaunch(g, c->stream));
                n -= GRAPH_STEPS;        // buffer parities are the same again after the period
                ++c->period_count;
                direct = false;
                continue;
            }
        }
        LBIB_TRY(one_step(c));
        direct = true;
        --n;
    }
    if (direct) LBIB_LAUNCH(c, launch_err_mirror(c, c->h_err_dev));   // graphs end with one
    return LBIB_OK;
}

lbib_status lbib_get_fields(lbib_ctx* c, double* rho, double* u, double* phi, double* xy, int32_t* cell_id_map)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(join_batch(c));
    const size_t nn = (size_t)c->nn;
    if (rho || u || (phi && c->S)) {
        LBIB_TRY(ensure_stage(c, nn * (size_t)(3 + c->S)));
        LBIB_LAUNCH(c, launch_moments(c, c->d_stage));
        if (rho)
            LBIB_HIP(c, hipMemcpyAsync(rho, c->d_stage, nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        if (u)
            LBIB_HIP(c, hipMemcpyAsync(u, c->d_stage + nn, 2 * nn * sizeof(double), hipMemcpyDeviceToHost,
                                       c->stream));
        if (phi && c->S)
            LBIB_HIP(c, hipMemcpyAsync(phi, c->d_stage + 3 * nn, (size_t)c->S * nn * sizeof(double),
                                       hipMemcpyDeviceToHost, c->stream));
    }
    if (xy && c->n_nodes)
        LBIB_HIP(c, hipMemcpyAsync(xy, c->d_X, (size_t)c->n_nodes * sizeof(double2), hipMemcpyDeviceToHost,
                                   c->stream));
    if (cell_id_map) {
        // the ID map is built on demand from the current positions
        LBIB_HIP(c, hipStreamSynchronize(c->stream));         // the stage may hold the moments
        uint16_t* ids = nullptr;
        LBIB_TRY(ensure_stage(c, (nn + 3) / 4));
        ids = (uint16_t*)c->d_stage;
        LBIB_LAUNCH(c, launch_fill_u16(c, ids, c->nn));
        if (c->n_cells) LBIB_LAUNCH(c, launch_raster(c, raster_args(c, ids)));
        std::vector<uint16_t> h(nn);
        LBIB_HIP(c, hipMemcpyAsync(h.data(), ids, nn * sizeof(uint16_t), hipMemcpyDeviceToHost, c->stream));
        LBIB_HIP(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < nn; ++i) cell_id_map[i] = h[i];
    }
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    return check_err_flag(c);
}

lbib_status lbib_get_forces(lbib_ctx* c, double* F, double* area)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(join_batch(c));
    if (!c->n_cells) return LBIB_OK;
    if (area && !area_in_step(c->p)) {
        // the step does not keep the areas: the membrane kernel at the current positions
        // (everything else it writes is the same function of them) computes them
        MembraneArgs a = membrane_args_at(c, c->cur, 0);
        a.need_area = 1;
        LBIB_LAUNCH(c, launch_membrane(c, a));
    }
    const size_t N = (size_t)c->n_nodes;
    if (F) {
        LBIB_TRY(ensure_stage(c, N));
        LBIB_LAUNCH(c, launch_forces_out(c, (float2*)c->d_stage));
        std::vector<float> h(2 * N);
        LBIB_HIP(c, hipMemcpyAsync(h.data(), c->d_stage, N * sizeof(float2), hipMemcpyDeviceToHost, c->stream));
        LBIB_HIP(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < 2 * N; ++i) F[i] = h[i];
    }
    if (area)
        LBIB_HIP(c, hipMemcpyAsync(area, c->d_area, (size_t)c->n_cells * sizeof(double), hipMemcpyDeviceToHost,
                                   c->stream));
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    return LBIB_OK;
}

lbib_status lbib_get_spread(lbib_ctx* c, double* e)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(join_batch(c));
    if (!e) return LBIB_EINVAL;
    const size_t nn = (size_t)c->nn;
    LBIB_TRY(ensure_stage(c, 2 * nn));
    LatticeArgs a = lattice_args(c);
    a.e_out = c->d_stage;
    if (!c->n_cells) a.t_off = nullptr;
    LBIB_LAUNCH(c, launch_spread_inspect(c, a));
    LBIB_HIP(c, hipMemcpyAsync(e, c->d_stage, 2 * nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    return LBIB_OK;
}

lbib_status lbib_reduce(lbib_ctx* c, double* out)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(join_batch(c));
    if (!out) return LBIB_EINVAL;
    const int nv = 3 + c->S;
    LBIB_TRY(ensure_stage(c, 8));
    LBIB_LAUNCH(c, launch_reduce(c, c->d_partial, c->d_stage));
    LBIB_HIP(c, hipMemcpyAsync(out, c->d_stage, (size_t)nv * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    for (int v = 0; v < nv; ++v)
        if (!std::isfinite(out[v])) {
            c->err = "non-finite lattice sum";
            return LBIB_ENUMERIC;
        }
    return LBIB_OK;
}

lbib_status lbib_reduce_device(lbib_ctx* c, double* out_device)
{
    if (!c) return LBIB_ESTATE;
    if (!out_device) {
        c->err = "out_device is NULL";
        return LBIB_EINVAL;
    }
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, out_device) != hipSuccess || at.type != hipMemoryTypeDevice ||
        at.device != c->device) {
        (void)hipGetLastError();
        c->err = "out_device is not device memory of the context's device";
        return LBIB_EINVAL;
    }
    double* scratch = c->scratch_ok ? reduce_scratch_ptr(c->device) : nullptr;
    if (!scratch) {
        c->err = "the reduction scratch has no device address on this device";
        return LBIB_EDEVICE;
    }
    if (reduce_blocks(c->nn) > reduce_scratch_blocks()) {
        c->err = "the lattice needs more reduction blocks than the scratch holds";
        return LBIB_EINVAL;
    }
    LBIB_TRY(join_batch(c));
    LBIB_LAUNCH(c, launch_reduce(c, scratch, out_device));
    return LBIB_OK;
}

lbib_status lbib_get_monitor(lbib_ctx* c, double* out, int64_t* step)
{
    if (!c) return LBIB_ESTATE;
    if (!out || !step) return LBIB_EINVAL;
    if (c->p.monitor_every <= 0) {
        c->err = "the monitor is off (monitor_every = 0)";
        return LBIB_ESTATE;
    }
    LBIB_TRY(join_batch(c));
    double h[8];
    LBIB_HIP(c, hipMemcpyAsync(h, c->d_mon, sizeof h, hipMemcpyDeviceToHost, c->stream));
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    const int64_t taken = (int64_t)h[0];
    *step = taken;
    if (taken <= 0) return LBIB_OK;
    const int nv = 3 + c->S;
    for (int v = 0; v < nv; ++v) out[v] = h[1 + v];
    for (int v = 0; v < nv; ++v)
        if (!std::isfinite(out[v])) {
            c->err = "non-finite lattice sum";
            return LBIB_ENUMERIC;
        }
    return LBIB_OK;
}

// ---------------------------------------------------------------------------------------
// Solver state for saving and resuming (Section "Input and Output"): a header, then the
// current populations of both lattices as stored (chunked deviations in the storage type),
// the first-order no-flux planes, the cells (offsets, positions, rest lengths and areas,
// source flags).  Everything else a step reads (forces, spreading records, node lists, the
// inside-cell bits, the cell map, the link cuts) is a function of the positions and is rebuilt
// on loading, as lbib_set_cells builds it.
// ---------------------------------------------------------------------------------------
namespace {

struct StateHeader {
    char magic[8];
    int32_t version, has_src;
    lbib_params p;
    int64_t n_cells, n_nodes, period_count;
    int32_t err, nf1;
    double mon[8];
    uint64_t bytes_f, bytes_g, bytes_nfphi, bytes_nfu;
    uint64_t bytes_nsrc, bytes_pmap;     // node sources (FP32) and pressure points, 0 when unset
    int32_t fresh, unused;               // not stepped since its fields were set
};
constexpr char STATE_MAGIC[8] = {'L', 'B', 'I', 'B', 'S', 'T', 'A', 'T'};
constexpr int32_t STATE_VERSION = 3;

void state_layout(const lbib_ctx* c, StateHeader& h)
{
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, STATE_MAGIC, 8);
    h.version = STATE_VERSION;
    h.p = c->p;
    h.n_cells = c->n_cells;
    h.n_nodes = c->n_nodes;
    h.period_count = c->period_count;
    h.has_src = c->d_src ? 1 : 0;
    h.nf1 = c->nfq[0] ? 1 : 0;
    h.bytes_f = c->f_elems() * c->pop_bytes;
    h.bytes_g = c->S ? c->g_elems() * c->pop_bytes : 0;
    h.bytes_nfphi = h.nf1 ? (uint64_t)c->S * (uint64_t)c->nn * sizeof(float) : 0;
    h.bytes_nfu = h.nf1 ? (uint64_t)c->nn * sizeof(float2) : 0;
    h.bytes_nsrc = c->d_nsrc ? (uint64_t)c->nn * sizeof(float) : 0;
    h.bytes_pmap = c->d_pmap ? (uint64_t)c->nn : 0;
    h.fresh = c->nf_fresh ? 1 : 0;
}

// Node sources: rate[nn] FP32 mass per node and step, any alignment (NULL removes them).
lbib_status set_node_sources_f32(lbib_ctx* c, const void* rate)
{
    const size_t nn = (size_t)c->nn;
    std::vector<float> r;
    if (rate) {
        r.resize(nn);
        std::memcpy(r.data(), rate, nn * sizeof(float));
        for (size_t i = 0; i < nn; ++i)
            if (!std::isfinite(r[i])) {
                c->err = "node source rate " + std::to_string(i) + " is not finite";
                return LBIB_EINVAL;
            }
    }
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);                 // the captured launches hold the map (and the kernel form)
    if (!rate) {
        dev_free(c, c->d_nsrc, nn);
        return LBIB_OK;
    }
    if (!c->d_nsrc) LBIB_TRY(dev_alloc(c, &c->d_nsrc, nn));
    LBIB_HIP(c, hipMemcpyAsync(c->d_nsrc, r.data(), nn * sizeof(float), hipMemcpyHostToDevice, c->stream));
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    return LBIB_OK;
}

// Pressure points: flags[nn], nonzero = held at rho0, stored as 0/1 (NULL removes them).
lbib_status set_pressure_map(lbib_ctx* c, const uint8_t* flags)
{
    const size_t nn = (size_t)c->nn;
    std::vector<uint8_t> m;
    if (flags) {
        m.resize(nn);
        for (size_t i = 0; i < nn; ++i) m[i] = flags[i] ? 1 : 0;
    }
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    if (!flags) {
        dev_free(c, c->d_pmap, nn);
        return LBIB_OK;
    }
    if (!c->d_pmap) LBIB_TRY(dev_alloc(c, &c->d_pmap, nn));
    LBIB_HIP(c, hipMemcpyAsync(c->d_pmap, m.data(), nn, hipMemcpyHostToDevice, c->stream));
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    return LBIB_OK;
}

size_t state_bytes(const StateHeader& h)
{
    const size_t N = (size_t)h.n_nodes, C = (size_t)h.n_cells;
    size_t b = sizeof(StateHeader) + h.bytes_f + h.bytes_g + h.bytes_nfphi + h.bytes_nfu;
    if (C) b += (C + 1) * sizeof(int32_t) + N * (2 * sizeof(double) + sizeof(double)) + C * sizeof(double);
    if (h.has_src) b += C;
    return b + h.bytes_nsrc + h.bytes_pmap;
}

}  // namespace

lbib_status lbib_state_size(lbib_ctx* c, size_t* bytes)
{
    if (!c) return LBIB_ESTATE;
    if (!bytes) return LBIB_EINVAL;
    StateHeader h;
    state_layout(c, h);
    *bytes = state_bytes(h);
    return LBIB_OK;
}

lbib_status lbib_save_state(lbib_ctx* c, void* buf, size_t bytes)
{
    if (!c) return LBIB_ESTATE;
    StateHeader h;
    state_layout(c, h);
    if (!buf || bytes < state_bytes(h)) {
        c->err = "the buffer holds " + std::to_string(bytes) + " bytes; the state needs " +
                 std::to_string(buf ? state_bytes(h) : 0);
        return LBIB_EINVAL;
    }
    LBIB_TRY(join_batch(c));
    int hd[2] = {0, 0};
    LBIB_HIP(c, hipMemcpyAsync(hd, c->d_err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    LBIB_HIP(c, hipMemcpyAsync(h.mon, c->d_mon, sizeof h.mon, hipMemcpyDeviceToHost, c->stream));
    char* q = (char*)buf + sizeof(StateHeader);
    auto take = [&](const void* dev, size_t n) -> hipError_t {
        if (!n) return hipSuccess;
        const hipError_t e = hipMemcpyAsync(q, dev, n, hipMemcpyDeviceToHost, c->stream);
        q += n;
        return e;
    };
    LBIB_HIP(c, take(c->f[c->cur], h.bytes_f));
    LBIB_HIP(c, take(c->g[c->cur], h.bytes_g));
    LBIB_HIP(c, take(c->nfphi[c->cur], h.bytes_nfphi));
    LBIB_HIP(c, take(c->nfu[c->cur], h.bytes_nfu));
    if (c->n_cells) {
        const size_t N = (size_t)c->n_nodes, C = (size_t)c->n_cells;
        LBIB_HIP(c, take(c->d_off, (C + 1) * sizeof(int32_t)));
        LBIB_HIP(c, take(c->d_X, N * sizeof(double2)));
        LBIB_HIP(c, take(c->d_l0, N * sizeof(double)));
        LBIB_HIP(c, take(c->d_A0, C * sizeof(double)));
        if (h.has_src) LBIB_HIP(c, take(c->d_src, C));
    }
    LBIB_HIP(c, take(c->d_nsrc, h.bytes_nsrc));
    LBIB_HIP(c, take(c->d_pmap, h.bytes_pmap));
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    h.err = hd[0];
    std::memcpy(buf, &h, sizeof h);
    return LBIB_OK;
}

lbib_status lbib_load_state(lbib_ctx* c, const void* buf, size_t bytes)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(refuse_if_batched(c));
    StateHeader h;
    if (!buf || bytes < sizeof h) {
        c->err = "the buffer is shorter than a state header";
        return LBIB_EINVAL;
    }
    std::memcpy(&h, buf, sizeof h);
    StateHeader mine;
    state_layout(c, mine);
    if (std::memcmp(h.magic, STATE_MAGIC, 8) != 0 || h.version != STATE_VERSION) {
        c->err = "not a saved lbib state of this version";
        return LBIB_EINVAL;
    }
    // every named field of the parameters (the struct has no padding before its last field)
    const size_t pfields = offsetof(lbib_params, reserved) + sizeof(int32_t);
    if (std::memcmp(&h.p, &c->p, pfields) != 0 || h.bytes_f != mine.bytes_f ||
        h.bytes_g != mine.bytes_g || h.nf1 != mine.nf1 || h.bytes_nfphi != mine.bytes_nfphi ||
        h.bytes_nfu != mine.bytes_nfu) {
        c->err = "the saved state was made with other parameters";
        return LBIB_EINVAL;
    }
    // the limits lbib_set_cells enforces, checked before anything is sized from them
    if (h.n_cells < 0 || h.n_cells > 65535 || h.n_nodes < 0 || h.n_nodes > 200000000) {
        c->err = "the saved cell counts are out of range";
        return LBIB_EINVAL;
    }
    if ((h.bytes_nsrc && h.bytes_nsrc != (uint64_t)c->nn * sizeof(float)) ||
        (h.bytes_pmap && h.bytes_pmap != (uint64_t)c->nn)) {
        c->err = "the saved node maps do not fit the lattice";
        return LBIB_EINVAL;
    }
    if (bytes < state_bytes(h)) {
        c->err = "the buffer is shorter than the saved state";
        return LBIB_EINVAL;
    }
    if ((h.bytes_nsrc || h.bytes_pmap) && c->ws) {
        c->err = "node sources or pressure points cannot be loaded while a workspace is bound";
        return LBIB_ESTATE;
    }
    const char* q = (const char*)buf + sizeof(StateHeader) + h.bytes_f + h.bytes_g + h.bytes_nfphi + h.bytes_nfu;
    // the node maps follow the cells
    const char* qmaps = q;
    if (h.n_cells)
        qmaps += (h.n_cells + 1) * sizeof(int32_t) + h.n_nodes * 3 * sizeof(double) + h.n_cells * sizeof(double) +
                 (h.has_src ? h.n_cells : 0);
    LBIB_TRY(set_node_sources_f32(c, h.bytes_nsrc ? (const float*)qmaps : nullptr));
    LBIB_TRY(set_pressure_map(c, h.bytes_pmap ? (const uint8_t*)(qmaps + h.bytes_nsrc) : nullptr));
    if (h.n_cells) {
        const size_t N = (size_t)h.n_nodes, C = (size_t)h.n_cells;
        std::vector<int32_t> off(C + 1);
        std::vector<double> xy(2 * N), l0(N), A0(C);
        std::memcpy(off.data(), q, (C + 1) * sizeof(int32_t));
        q += (C + 1) * sizeof(int32_t);
        std::memcpy(xy.data(), q, 2 * N * sizeof(double));
        q += 2 * N * sizeof(double);
        std::memcpy(l0.data(), q, N * sizeof(double));
        q += N * sizeof(double);
        std::memcpy(A0.data(), q, C * sizeof(double));
        q += C * sizeof(double);
        if ((size_t)off[C] != N) {
            c->err = "the saved cells are inconsistent";
            return LBIB_EINVAL;
        }
        LBIB_TRY(lbib_set_cells(c, (int32_t)C, off.data(), xy.data(), l0.data(), A0.data()));
        if (h.has_src) LBIB_TRY(lbib_set_source_cells(c, (const uint8_t*)q));
    } else {
        const int32_t none = 0;
        LBIB_TRY(lbib_set_cells(c, 0, &none, nullptr, nullptr, nullptr));
    }
    const char* p = (const char*)buf + sizeof(StateHeader);
    auto give = [&](void* dev, size_t n) -> hipError_t {
        if (!n) return hipSuccess;
        const hipError_t e = hipMemcpyAsync(dev, p, n, hipMemcpyHostToDevice, c->stream);
        p += n;
        return e;
    };
    LBIB_HIP(c, give(c->f[c->cur], h.bytes_f));
    LBIB_HIP(c, give(c->g[c->cur], h.bytes_g));
    LBIB_HIP(c, give(c->nfphi[c->cur], h.bytes_nfphi));
    LBIB_HIP(c, give(c->nfu[c->cur], h.bytes_nfu));
    LBIB_HIP(c, hipMemcpyAsync(c->d_mon, h.mon, sizeof h.mon, hipMemcpyHostToDevice, c->stream));
    LBIB_HIP(c, hipMemcpyAsync(c->d_err, &h.err, sizeof(int), hipMemcpyHostToDevice, c->stream));
    LBIB_LAUNCH(c, launch_err_mirror(c, c->h_err_dev));
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    c->period_count = h.period_count;
    c->nf_fresh = h.fresh != 0;
    return LBIB_OK;
}

lbib_status lbib_set_node_sources(lbib_ctx* c, const double* rate)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(refuse_if_batched(c));
    if (rate && c->ws) {
        c->err = "node sources cannot be set while a workspace is bound";
        return LBIB_ESTATE;
    }
    std::vector<float> r;
    if (rate) {
        r.resize((size_t)c->nn);
        for (int64_t i = 0; i < c->nn; ++i) {
            if (!std::isfinite(rate[i])) {
                c->err = "node source rate " + std::to_string(i) + " is not finite";
                return LBIB_EINVAL;
            }
            r[(size_t)i] = (float)rate[i];
        }
    }
    return set_node_sources_f32(c, rate ? r.data() : nullptr);
}

lbib_status lbib_set_pressure_nodes(lbib_ctx* c, const uint8_t* flags)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(refuse_if_batched(c));
    if (flags && c->ws) {
        c->err = "pressure points cannot be set while a workspace is bound";
        return LBIB_ESTATE;
    }
    return set_pressure_map(c, flags);
}

lbib_status lbib_set_source_cells(lbib_ctx* c, const uint8_t* src)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(refuse_if_batched(c));
    if (c->n_cells == 0) {
        c->err = "no cells are set";
        return LBIB_ESTATE;
    }
    if (src && no_flux_bits(c->p)) {
        c->err = "a source subset cannot be combined with no-flux membranes (they share the inside map)";
        return LBIB_EINVAL;
    }
    if (src && mass_sources(c->p)) {
        c->err = "a source subset cannot be combined with mass sources (they share the inside map)";
        return LBIB_EINVAL;
    }
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    if (src) {
        if (!c->d_src) {
            if (c->ws)
                c->d_src = c->ws_src;
            else
                LBIB_TRY(dev_alloc(c, &c->d_src, (size_t)c->n_cells));
        }
        LBIB_HIP(c, hipMemcpyAsync(c->d_src, src, (size_t)c->n_cells, hipMemcpyHostToDevice, c->stream));
    } else {
        state_free(c, c->d_src, (size_t)c->n_cells);
    }
    if (c->mask_needed) {
        // rebuild the source bits of the current positions (forces and records are recomputed
        // from the same positions, unchanged)
        LBIB_LAUNCH(c, launch_fill_i32(c, (int*)c->inside[c->cur], c->ny_words(), 0));
        if (c->cmap) LBIB_LAUNCH(c, launch_fill_i32(c, (int*)c->cmap, c->nn, -1));
        LBIB_TRY(membrane(c, 0));
    }
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    return check_err_flag(c);
}

lbib_status lbib_ade_steady(lbib_ctx* c, double tol, int64_t max_iters, int32_t fp64, int64_t* iters,
                            double* change)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(refuse_if_batched(c));
    if (iters) *iters = 0;
    if (change) *change = NAN;
    if (c->S == 0) {
        c->err = "no species to iterate";
        return LBIB_EINVAL;
    }
    if (no_flux_bits(c->p)) {
        c->err = "the ADE-only iteration has no no-flux membranes";
        return LBIB_EINVAL;
    }
    if (!std::isfinite(tol) || tol < 0.0 || max_iters < 0) {
        c->err = "tol must be finite and >= 0, max_iters >= 0";
        return LBIB_EINVAL;
    }
    if (max_iters == 0) return LBIB_OK;
    constexpr int H = 128;                       // passes per captured batch (even)
    const bool dbl = fp64 != 0;
    const size_t wbytes = dbl ? sizeof(double) : sizeof(float);
    const size_t nw = (size_t)5 * c->S * (size_t)c->nn;
    const unsigned nb = ade_blocks(c->nn);
    char* work[2] = {nullptr, nullptr};
    double *phi_prev = nullptr, *partial = nullptr, *hist = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<double> h((size_t)H * c->S);
    lbib_status st = LBIB_OK;
    int64_t found = 0, done = 0;
    double last = NAN;
    int wc = 0;
    AdeArgs a;
    std::memset(&a, 0, sizeof a);
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < 2 && st == LBIB_OK; ++b) st = dev_alloc(c, &work[b], nw * wbytes);
    if (st == LBIB_OK) st = dev_alloc(c, &phi_prev, (size_t)c->S * (size_t)c->nn);
    if (st == LBIB_OK) st = dev_alloc(c, &partial, (size_t)H * nb * 4);
    if (st == LBIB_OK) st = dev_alloc(c, &hist, (size_t)H * c->S);
    if (st != LBIB_OK) goto out;
    a.phi_prev = phi_prev;
    a.inside = c->inside[c->cur];
    a.wpr = c->wpr;
    a.partial = partial;
    a.nn = c->nn;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.walls = c->p.bc_y == LBIB_WALLS;
    a.S = c->S;
    for (int s = 0; s < 2; ++s) {
        const lbib_species& sp = c->p.species[s];
        a.omega_s[s] = s < c->S ? 1.0 / (3.0 * sp.D + 0.5) : 0.0;
        a.phi_ref[s] = sp.phi_ref;
        a.react[s] = s < c->S ? sp.reaction : 0;
        for (int k = 0; k < 4; ++k) a.rc[s][k] = sp.c[k];
    }
    if (launch_ade_copy(c, work[0], dbl, true) != hipSuccess) {
        st = LBIB_EDEVICE;
        goto out;
    }
    // first pass: phi^0 into phi_prev (no change yet), the state advances to iteration 1
    a.src = work[0];
    a.dst = work[1];
    a.track = 0;
    if (launch_ade(c, a, dbl, c->stream) != hipSuccess) {
        st = LBIB_EDEVICE;
        goto out;
    }
    wc = 1;
    // H tracked passes per batch, captured once (the buffer parity repeats after H)
    if (!c->capture_stream &&
        hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        st = LBIB_EDEVICE;
        goto out;
    }
    {
        hipGraph_t graph = nullptr;
        bool ok = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        for (int i = 0; i < H && ok; ++i) {
            a.src = work[(wc + i) & 1];
            a.dst = work[(wc + i + 1) & 1];
            a.track = 1;
            a.hslot = i;
            ok = launch_ade(c, a, dbl, c->capture_stream) == hipSuccess;
        }
        if (ok) ok = launch_ade_hist(partial, (int)nb, c->S, hist, H, c->capture_stream) == hipSuccess;
        const bool ended = hipStreamEndCapture(c->capture_stream, &graph) == hipSuccess;
        ok = ok && ended && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        if (!ok) {
            c->err = "ADE batch capture failed";
            st = LBIB_EDEVICE;
            goto out;
        }
    }
    while (done < max_iters && !found) {
        if (hipGraphLaunch(exec, c->stream) != hipSuccess ||
            hipMemcpyAsync(h.data(), hist, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            c->err = "ADE batch failed";
            st = LBIB_EDEVICE;
            goto out;
        }
        for (int i = 0; i < H; ++i) {
            const int64_t k = done + 1 + i;                  // the pass computed phi^k
            if (k > max_iters) break;
            double ch = 0.0;
            for (int s = 0; s < c->S; ++s) ch = std::fmax(ch, h[(size_t)i * c->S + s]);
            last = ch;
            if (!std::isfinite(ch)) {
                c->err = "non-finite concentration in the ADE iteration";
                st = LBIB_ENUMERIC;
                break;
            }
            if (ch <= tol) {
                found = k;
                break;
            }
        }
        if (st != LBIB_OK) break;
        done += H;
    }
    if (launch_ade_copy(c, work[wc], dbl, false) != hipSuccess) st = LBIB_EDEVICE;
    if (hipStreamSynchronize(c->stream) != hipSuccess && st == LBIB_OK) st = LBIB_EDEVICE;
    if (iters) *iters = found;
    if (change) *change = last;
out:
    (void)hipStreamSynchronize(c->stream);
    if (exec) (void)hipGraphExecDestroy(exec);
    for (int b = 0; b < 2; ++b) dev_free(c, work[b], nw * wbytes);
    dev_free(c, phi_prev, (size_t)c->S * (size_t)c->nn);
    dev_free(c, partial, (size_t)H * nb * 4);
    dev_free(c, hist, (size_t)H * c->S);
    return st;
}

lbib_status lbib_ade_batch(int32_t nx, int32_t ny, int32_t bc_y, int32_t batch, const uint8_t* source,
                           const double* D, const double* sigma, const double* decay, double* phi, int32_t zero_start,
                           double tol, int64_t max_iters, int32_t fp64, int64_t* iters, void* hip_stream)
{
    if (nx < 4 || nx > 32767 || ny < 4 || ny > 32767 || (bc_y != LBIB_PERIODIC && bc_y != LBIB_WALLS) || batch < 1 ||
        batch > 65535 || !source || !D || !sigma || !decay || !phi || !iters || !std::isfinite(tol) || tol < 0.0 ||
        max_iters < 0)
        return LBIB_EINVAL;
    for (int b = 0; b < batch; ++b)
        if (!std::isfinite(D[b]) || !(D[b] > 0.0) || !std::isfinite(sigma[b]) || !std::isfinite(decay[b]))
            return LBIB_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return LBIB_EDEVICE;
    for (int b = 0; b < batch; ++b) iters[b] = 0;

    constexpr int H = ADE_BATCH_SLOTS;
    const int64_t nn = (int64_t)nx * ny;
    const bool dbl = fp64 != 0;
    const size_t wbytes = dbl ? sizeof(double) : sizeof(float);
    const int nblocks = (int)ade_blocks(nn);
    hipStream_t st = (hipStream_t)hip_stream, cap = nullptr;
    bool own = false;
    lbib_status res = LBIB_OK;
    char *work[2] = {nullptr, nullptr}, *src = nullptr;
    double *phi_prev = nullptr, *partial = nullptr, *hist = nullptr, *prm = nullptr, *dphi = nullptr;
    int* active = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<double> hh((size_t)H * batch), p((size_t)3 * batch);
    std::vector<int> act((size_t)batch, 1);
    AdeBatchArgs a;
    std::memset(&a, 0, sizeof a);
    int64_t done = 0, left = batch;
    int wc = 0;
    auto fail = [&](lbib_status s) { res = s; };
#define ADE_B_HIP(call)                                                               \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            fail(e_ == hipErrorOutOfMemory ? LBIB_ENOMEM : LBIB_EDEVICE);             \
            goto out;                                                                 \
        }                                                                             \
    } while (0)
    if (!st) {
        ADE_B_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        own = true;
    }
    ADE_B_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) ADE_B_HIP(hipMalloc((void**)&work[b], (size_t)5 * batch * nn * wbytes));
    ADE_B_HIP(hipMalloc((void**)&src, (size_t)batch * nn));
    ADE_B_HIP(hipMalloc((void**)&phi_prev, (size_t)batch * nn * sizeof(double)));
    ADE_B_HIP(hipMalloc((void**)&dphi, (size_t)batch * nn * sizeof(double)));
    ADE_B_HIP(hipMalloc((void**)&partial, (size_t)H * batch * nblocks * 2 * sizeof(double)));
    ADE_B_HIP(hipMalloc((void**)&hist, (size_t)H * batch * sizeof(double)));
    ADE_B_HIP(hipMalloc((void**)&prm, (size_t)3 * batch * sizeof(double)));
    ADE_B_HIP(hipMalloc((void**)&active, (size_t)batch * sizeof(int)));
    for (int b = 0; b < batch; ++b) {
        p[b] = 1.0 / (3.0 * D[b] + 0.5);
        p[batch + b] = sigma[b];
        p[2 * batch + b] = decay[b];
    }
    ADE_B_HIP(hipMemcpyAsync(src, source, (size_t)batch * nn, hipMemcpyHostToDevice, st));
    ADE_B_HIP(hipMemcpyAsync(prm, p.data(), p.size() * sizeof(double), hipMemcpyHostToDevice, st));
    ADE_B_HIP(hipMemcpyAsync(active, act.data(), act.size() * sizeof(int), hipMemcpyHostToDevice, st));
    if (!zero_start)
        ADE_B_HIP(hipMemcpyAsync(dphi, phi, (size_t)batch * nn * sizeof(double), hipMemcpyHostToDevice, st));
    ADE_B_HIP(ade_batch_init_launch(zero_start ? nullptr : dphi, work[0], nn, nx, ny, bc_y == LBIB_WALLS, batch, dbl, st));

    a.phi_prev = phi_prev;
    a.source = (const uint8_t*)src;
    a.omega = prm;
    a.sigma = prm + batch;
    a.decay = prm + 2 * batch;
    a.active = active;
    a.partial = partial;
    a.nn = nn;
    a.nx = nx;
    a.ny = ny;
    a.walls = bc_y == LBIB_WALLS;
    a.B = batch;
    a.nblocks = nblocks;
    // first pass: phi^0 into phi_prev, the state advances to iteration 1
    a.src = work[0];
    a.dst = work[1];
    a.track = 0;
    ADE_B_HIP(ade_batch_launch(a, dbl, st));
    wc = 1;
    ADE_B_HIP(hipStreamSynchronize(st));
    ADE_B_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    {
        bool ok = true;
        for (int i = 0; i < H && ok; ++i) {
            a.src = work[(wc + i) & 1];
            a.dst = work[(wc + i + 1) & 1];
            a.track = 1;
            a.hslot = i;
            ok = ade_batch_launch(a, dbl, cap) == hipSuccess;
        }
        if (ok) ok = ade_batch_hist_launch(a, hist, cap) == hipSuccess;
        const bool ended = hipStreamEndCapture(cap, &graph) == hipSuccess;
        if (!ok || !ended || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            fail(LBIB_EDEVICE);
            goto out;
        }
    }
    while (done < max_iters && left > 0) {
        ADE_B_HIP(hipGraphLaunch(exec, st));
        ADE_B_HIP(hipMemcpyAsync(hh.data(), hist, hh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        ADE_B_HIP(hipStreamSynchronize(st));
        bool changed = false;
        for (int b = 0; b < batch; ++b) {
            if (!act[b]) continue;
            for (int i = 0; i < H; ++i) {
                const int64_t k = done + 1 + i;             // the pass computed phi^k
                if (k > max_iters) break;
                const double ch = hh[(size_t)i * batch + b];
                if (!std::isfinite(ch)) {
                    res = LBIB_ENUMERIC;
                    act[b] = 0;
                    changed = true;
                    break;
                }
                if (ch <= tol) {
                    iters[b] = k;
                    act[b] = 0;
                    changed = true;
                    break;
                }
            }
            if (!act[b]) --left;
        }
        if (changed) ADE_B_HIP(hipMemcpyAsync(active, act.data(), act.size() * sizeof(int), hipMemcpyHostToDevice, st));
        done += H;
    }
    ADE_B_HIP(ade_batch_phi_launch(work[wc], dphi, nn, nx, ny, bc_y == LBIB_WALLS, batch, dbl, st));
    ADE_B_HIP(hipMemcpyAsync(phi, dphi, (size_t)batch * nn * sizeof(double), hipMemcpyDeviceToHost, st));
    ADE_B_HIP(hipStreamSynchronize(st));
#undef ADE_B_HIP
out:
    if (st) (void)hipStreamSynchronize(st);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (int b = 0; b < 2; ++b)
        if (work[b]) (void)hipFree(work[b]);
    if (src) (void)hipFree(src);
    if (phi_prev) (void)hipFree(phi_prev);
    if (dphi) (void)hipFree(dphi);
    if (partial) (void)hipFree(partial);
    if (hist) (void)hipFree(hist);
    if (prm) (void)hipFree(prm);
    if (active) (void)hipFree(active);
    if (cap) (void)hipStreamDestroy(cap);
    if (own) (void)hipStreamDestroy(st);
    return res;
}

lbib_status lbib_sync(lbib_ctx* c)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(join_batch(c));
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    return LBIB_OK;
}

lbib_status lbib_set_timing(lbib_ctx* c, int32_t enable)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(harvest(c));
    c->timing = enable != 0;
    for (int k = 0; k < LBIB_K_COUNT; ++k) {
        c->t_ms[k] = 0.0;
        c->t_count[k] = 0;
    }
    return LBIB_OK;
}

lbib_status lbib_get_timing(lbib_ctx* c, int32_t kernel, double* total_ms, int64_t* launches)
{
    if (!c) return LBIB_ESTATE;
    if (kernel < 0 || kernel >= LBIB_K_COUNT) return LBIB_EINVAL;
    LBIB_TRY(harvest(c));
    if (total_ms) *total_ms = c->t_ms[kernel];
    if (launches) *launches = c->t_count[kernel];
    return LBIB_OK;
}

lbib_status lbib_workspace_size(const lbib_params* p, int64_t n_nodes, size_t* bytes)
{
    if (!bytes) return LBIB_EINVAL;
    *bytes = 0;
    std::string msg;
    if (check_params(p, msg) != LBIB_OK || n_nodes < 0) return LBIB_EINVAL;
    lbib_ctx g;
    set_geometry(&g, p);
    *bytes = ws_total(g, n_nodes);
    return LBIB_OK;
}

lbib_status lbib_bind_workspace(lbib_ctx* c, void* device_ptr, size_t bytes)
{
    if (!c) return LBIB_ESTATE;
    LBIB_TRY(refuse_if_batched(c));
    char* base = (char*)device_ptr;
    if (!base) {
        if (bytes) {
            c->err = "a NULL workspace must have 0 bytes";
            return LBIB_EINVAL;
        }
        if (!c->ws) return LBIB_OK;
    } else {
        if ((uintptr_t)base % WS_ALIGN) {
            c->err = "the workspace must start on a " + std::to_string(WS_ALIGN) + "-byte boundary";
            return LBIB_EINVAL;
        }
        if (c->ws && base < c->ws + c->ws_bytes && c->ws < base + bytes) {
            c->err = "the new workspace overlaps the bound one";
            return LBIB_EINVAL;
        }
        hipPointerAttribute_t at{};
        if (hipPointerGetAttributes(&at, base) != hipSuccess || at.type != hipMemoryTypeDevice ||
            at.device != c->device) {
            (void)hipGetLastError();
            c->err = "the workspace is not device memory of the context's device";
            return LBIB_EINVAL;
        }
        void* abase = nullptr;
        size_t asize = 0;
        if (hipMemGetAddressRange(&abase, &asize, base) != hipSuccess ||
            base + bytes > (char*)abase + asize) {
            (void)hipGetLastError();
            c->err = "the workspace extends past the end of its allocation";
            return LBIB_EINVAL;
        }
    }
    if (base && (c->d_nsrc || c->d_pmap)) {
        c->err = "node sources or pressure points are set; the workspace does not hold them";
        return LBIB_ESTATE;
    }
    int64_t cap = 0;
    if (base) {
        const size_t need = ws_total(*c, c->n_nodes);
        if (bytes < need) {
            c->err = "the workspace has " + std::to_string(bytes) + " bytes; " + std::to_string(need) +
                     " are needed for the lattice and " + std::to_string(c->n_nodes) + " membrane nodes";
            return LBIB_ENOMEM;
        }
        // largest node capacity that fits (ws_total grows with it by >= 16 bytes a node)
        int64_t lo = c->n_nodes, hi = (int64_t)(bytes / 16) + 1;
        while (hi - lo > 1) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (ws_total(*c, mid) <= bytes)
                lo = mid;
            else
                hi = mid;
        }
        cap = lo;
    }
    LBIB_HIP(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    return relocate(c, base, bytes, cap);
}

lbib_status lbib_workspace_nodes(const lbib_ctx* c, int64_t* n_nodes)
{
    if (!c || !n_nodes) return LBIB_EINVAL;
    *n_nodes = c->ws ? c->ws_node_cap : -1;
    return LBIB_OK;
}

lbib_status lbib_device_bytes(const lbib_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return LBIB_ESTATE;
    *bytes = c->device_bytes;
    return LBIB_OK;
}

}  // extern "C"
