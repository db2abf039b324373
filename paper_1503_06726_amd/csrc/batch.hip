// Batched stepping: many independent simulations (contexts of any lattice size and cell count)
// advanced together.  Every kernel of the coupled step runs once per step for the whole batch:
// a work table lists (simulation, tile), (simulation, cell) or (simulation, node block) items
// and a per-simulation argument table, one per buffer parity, names each simulation's buffers.
// Whole list periods are captured as one HIP graph and replayed.  The simulations form one or
// two groups of about equal lattice size; two groups step as two chains on two streams (one
// graph), so that one group's latency-bound membrane and list kernels run beside the other's
// bandwidth-bound lattice pass.  The arithmetic is that of the single-simulation kernels (the
// same device functions), so with the default tile shape a batched simulation is
// bit-identical to the same simulation stepped alone, whatever the grouping.
#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <set>
#include <vector>

#include "lbib_internal.h"

using namespace lbib;

namespace {

#define BATCH_HIP(b, call)                                                                    \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            (b)->err = std::string(#call) + " failed: " + hipGetErrorString(e_);              \
            return e_ == hipErrorOutOfMemory ? LBIB_ENOMEM : LBIB_EDEVICE;                    \
        }                                                                                     \
    } while (0)

#define BATCH_TRY(expr)                 \
    do {                                \
        lbib_status s_ = (expr);        \
        if (s_ != LBIB_OK) return s_;   \
    } while (0)

constexpr int TILE_CHOICES[3] = {4, 8, 16};   // lattice tile heights (rows) the batched pass offers

template <typename T>
void free_dev(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

// (re)place a host table in device memory; the stream is idle when this runs
template <typename T>
lbib_status upload(lbib_batch* b, T*& d, const std::vector<T>& h)
{
    free_dev(d);
    BATCH_HIP(b, hipMalloc((void**)&d, std::max<size_t>(1, h.size()) * sizeof(T)));
    if (!h.empty()) BATCH_HIP(b, hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, b->stream));
    BATCH_HIP(b, hipStreamSynchronize(b->stream));
    return LBIB_OK;
}

// Tiles of 4 rows are admitted only where a node's rows cannot wrap onto a narrow last tile
// row (walls, or ny a multiple of 4): the list build's three-tile-row bound needs it.
bool tile_ok(const lbib_ctx* c, int lty)
{
    if (lty == 8 || lty == 16) return true;
    if (lty == 4) return c->p.bc_y == LBIB_WALLS || c->p.ny % 4 == 0;
    return false;
}

bool tile_ok_all(const lbib_batch* b, int lty)
{
    for (const lbib_ctx* c : b->sims)
        if (!tile_ok(c, lty)) return false;
    return true;
}

void drop_graph(lbib_batch* b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
}

void free_groups(lbib_batch* b)
{
    for (lbib_batch_group& g : b->groups) {
        for (int p = 0; p < 2; ++p) {
            free_dev(g.d_lat[p]);
            free_dev(g.d_mem[p]);
        }
        free_dev(g.d_list);
        free_dev(g.d_lat_work);
        free_dev(g.d_mem_work);
        free_dev(g.d_node_work);
    }
    b->groups.clear();
}

// the simulations split into ngroups groups of about equal lattice size (largest first, each
// into the lightest group), then, per group, the argument tables of both parities, the list
// table and the work tables for tile height lty
lbib_status build_tables(lbib_batch* b, int lty)
{
    const int n = (int)b->sims.size();
    const int G = std::max(1, std::min(b->ngroups, n));
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->sims[x]->nn > b->sims[y]->nn; });
    std::vector<std::vector<int>> members(G);
    std::vector<int64_t> load(G, 0);
    for (int s : order) {
        const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        members[g].push_back(s);
        load[g] += b->sims[s]->nn;
    }
    free_groups(b);
    b->groups.resize(G);
    for (int g = 0; g < G; ++g) {
        lbib_batch_group& grp = b->groups[g];
        grp.sims = members[g];
        std::sort(grp.sims.begin(), grp.sims.end());
        std::vector<LatticeArgs> lat[2];
        std::vector<MembraneArgs> mem[2];
        std::vector<ListArgs> lst;
        std::vector<int2> wl, wm, wn;
        for (int gs = 0; gs < (int)grp.sims.size(); ++gs) {
            const int s = grp.sims[gs];
            lbib_ctx* c = b->sims[s];
            for (int p = 0; p < 2; ++p) {
                lat[p].push_back(lattice_args_at(c, b->cur0[s] ^ p));
                // the membrane pass of a step reads and writes the buffers of the step's end
                mem[p].push_back(membrane_args_at(c, b->cur0[s] ^ p ^ 1, 1));
            }
            const ListArgs la = list_args_h(c, lty);
            lst.push_back(la);
            for (int t = 0; t < la.ntiles; ++t) wl.push_back(make_int2(gs, tile_of_block(t, la.ntx, la.nlty)));
            for (int q = 0; q < c->n_cells; ++q) wm.push_back(make_int2(gs, q));
            const int64_t nb = (c->n_nodes + LIST_THREADS - 1) / LIST_THREADS;
            for (int64_t q = 0; q < nb; ++q) wn.push_back(make_int2(gs, (int)q));
            grp.max_cell_nodes = std::max(grp.max_cell_nodes, c->max_cell_nodes);
        }
        if (wl.size() > 0x7FFFFFFF || wm.size() > 0x7FFFFFFF || wn.size() > 0x7FFFFFFF) {
            b->err = "batch too large for one launch";
            return LBIB_EINVAL;
        }
        for (int p = 0; p < 2; ++p) {
            BATCH_TRY(upload(b, grp.d_lat[p], lat[p]));
            BATCH_TRY(upload(b, grp.d_mem[p], mem[p]));
        }
        BATCH_TRY(upload(b, grp.d_list, lst));
        BATCH_TRY(upload(b, grp.d_lat_work, wl));
        BATCH_TRY(upload(b, grp.d_mem_work, wm));
        BATCH_TRY(upload(b, grp.d_node_work, wn));
        grp.n_lat_work = (int)wl.size();
        grp.n_mem_work = (int)wm.size();
        grp.n_node_work = (int)wn.size();
    }
    b->lty = lty;
    return LBIB_OK;
}

hipStream_t group_stream(const lbib_batch* b, int g) { return g == 0 ? b->stream : b->side; }

#define BATCH_LAUNCH(b, call)                                                                \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) {                                                              \
            (b)->err = std::string(#call) + ": " + hipGetErrorString(e_);                    \
            return LBIB_EDEVICE;                                                             \
        }                                                                                    \
    } while (0)

lbib_status lists(lbib_batch* b)
{
    for (int g = 0; g < (int)b->groups.size(); ++g) {
        const lbib_batch_group& grp = b->groups[g];
        for (int which = 0; which < 3; ++which)
            BATCH_LAUNCH(b, launch_lists_batch(grp.d_list, grp.d_node_work, grp.n_node_work, (int)grp.sims.size(),
                                               which, group_stream(b, g)));
    }
    b->since = 0;
    return LBIB_OK;
}

// one coupled step of every simulation: lattice pass, membrane pass, and every LIST_PERIOD
// steps the list build (the order of a single context's step), each group on its stream
lbib_status one_step(lbib_batch* b)
{
    const int p = b->par;
    for (int g = 0; g < (int)b->groups.size(); ++g) {
        const lbib_batch_group& grp = b->groups[g];
        const hipStream_t st = group_stream(b, g);
        BATCH_LAUNCH(b, launch_lattice_batch(grp.d_lat[p], grp.d_lat_work, grp.n_lat_work, b->S, b->storage,
                                             b->lty / TILE_Y, b->mask, st));
        BATCH_LAUNCH(b, launch_membrane_batch(grp.d_mem[p], grp.d_mem_work, grp.n_mem_work, grp.max_cell_nodes, st));
    }
    b->par ^= 1;
    if (++b->since >= LIST_PERIOD) BATCH_TRY(lists(b));
    return LBIB_OK;
}

// the second group's stream starts after, and the batch's stream continues after, all work so far
lbib_status fork_groups(lbib_batch* b)
{
    if (b->groups.size() < 2) return LBIB_OK;
    BATCH_HIP(b, hipEventRecord(b->fork, b->stream));
    BATCH_HIP(b, hipStreamWaitEvent(b->side, b->fork, 0));
    return LBIB_OK;
}

lbib_status join_groups(lbib_batch* b)
{
    if (b->groups.size() < 2) return LBIB_OK;
    BATCH_HIP(b, hipEventRecord(b->join, b->side));
    BATCH_HIP(b, hipStreamWaitEvent(b->stream, b->join, 0));
    return LBIB_OK;
}

// LIST_PERIOD steps from an aligned state (since = par = 0, which they are again at the end);
// the groups' chains fork at the start and join at the end of the period
lbib_status capture(lbib_batch* b)
{
    if (!b->capture_stream) BATCH_HIP(b, hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
    hipStream_t user = b->stream;
    b->stream = b->capture_stream;
    hipGraph_t g = nullptr;
    lbib_status st = LBIB_OK;
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = LBIB_EDEVICE;
    } else {
        st = fork_groups(b);
        for (int k = 0; k < LIST_PERIOD && st == LBIB_OK; ++k) st = one_step(b);
        if (st == LBIB_OK) st = join_groups(b);
        const hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (st == LBIB_OK && e != hipSuccess) st = LBIB_EDEVICE;
    }
    b->stream = user;
    b->par = 0;
    b->since = 0;
    if (st == LBIB_OK && hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0) != hipSuccess) st = LBIB_EDEVICE;
    if (g) (void)hipGraphDestroy(g);
    if (st != LBIB_OK) {
        b->graph = nullptr;
        if (b->err.empty()) b->err = "batch step graph capture failed";
    }
    return st;
}

// advance n steps; whole aligned periods replay the captured graph, other steps are launched
// directly (up to the next list build, or the remainder)
lbib_status advance(lbib_batch* b, int64_t n)
{
    while (n > 0) {
        if (n >= LIST_PERIOD && b->since == 0) {
            if (!b->graph) BATCH_TRY(capture(b));
            BATCH_HIP(b, hipGraphLaunch(b->graph, b->stream));
            n -= LIST_PERIOD;
            continue;
        }
        const int64_t m = std::min<int64_t>(n, LIST_PERIOD - b->since);
        BATCH_TRY(fork_groups(b));
        for (int64_t k = 0; k < m; ++k) BATCH_TRY(one_step(b));
        BATCH_TRY(join_groups(b));
        n -= m;
    }
    return LBIB_OK;
}

// the adopted contexts' host-side step state follows the batch
void publish(lbib_batch* b)
{
    for (size_t s = 0; s < b->sims.size(); ++s) {
        lbib_ctx* c = b->sims[s];
        c->cur = b->cur0[s] ^ b->par;
        c->steps_since_lists = b->since;
    }
    (void)hipEventRecord(b->done, b->stream);
}

// switch the tile height at an aligned state: new tables, lists rebuilt from the current
// positions (as a build at the last list step with this height would have made them)
lbib_status set_tile(lbib_batch* b, int lty)
{
    BATCH_HIP(b, hipStreamSynchronize(b->stream));
    drop_graph(b);
    BATCH_TRY(build_tables(b, lty));
    BATCH_TRY(fork_groups(b));
    BATCH_TRY(lists(b));
    BATCH_TRY(join_groups(b));
    return LBIB_OK;
}

// regroup at an aligned state (the lists stay as they are)
lbib_status set_groups(lbib_batch* b, int ngroups)
{
    BATCH_HIP(b, hipStreamSynchronize(b->stream));
    drop_graph(b);
    b->ngroups = ngroups;
    return build_tables(b, b->lty);
}

// copy of the state a step starts from: populations of the current parity, positions,
// spreading records, inside-any-cell bits, areas and error flags
struct Snapshot {
    std::vector<char*> buf;
    std::vector<size_t> bytes;
};

struct Part {
    void* p;
    size_t n;
};

std::vector<Part> state_parts(lbib_ctx* c)
{
    const size_t N = (size_t)c->n_nodes, C = (size_t)c->n_cells;
    return {{c->f[c->cur], c->f_elems() * c->pop_bytes},
            {c->g[c->cur], c->g_elems() * c->pop_bytes},
            {c->d_X, N * sizeof(double2)},
            {c->d_rec, N * sizeof(float4)},
            {c->d_rec_ij, N * sizeof(int)},
            {c->inside[c->cur], (size_t)c->ny_words() * sizeof(unsigned)},
            {c->d_area, C * sizeof(double)},
            {c->d_err, sizeof(int)}};
}

lbib_status snapshot(lbib_batch* b, Snapshot& snap, bool restore)
{
    if (!restore) {
        snap.buf.assign(b->sims.size(), nullptr);
        snap.bytes.assign(b->sims.size(), 0);
    }
    for (size_t s = 0; s < b->sims.size(); ++s) {
        const std::vector<Part> parts = state_parts(b->sims[s]);
        if (!restore) {
            size_t tot = 0;
            for (const Part& q : parts) tot += (q.n + 255) & ~size_t(255);
            BATCH_HIP(b, hipMalloc((void**)&snap.buf[s], tot));
            snap.bytes[s] = tot;
        }
        size_t o = 0;
        for (const Part& q : parts) {
            if (q.n && q.p) {
                if (restore)
                    BATCH_HIP(b, hipMemcpyAsync(q.p, snap.buf[s] + o, q.n, hipMemcpyDeviceToDevice, b->stream));
                else
                    BATCH_HIP(b, hipMemcpyAsync(snap.buf[s] + o, q.p, q.n, hipMemcpyDeviceToDevice, b->stream));
            }
            o += (q.n + 255) & ~size_t(255);
        }
    }
    BATCH_HIP(b, hipStreamSynchronize(b->stream));
    return LBIB_OK;
}

void free_snapshot(Snapshot& snap)
{
    for (char*& p : snap.buf) free_dev(p);
    snap.buf.clear();
}

lbib_status usable(lbib_batch* b)
{
    if (b->broken) {
        b->err = "a simulation of the batch was destroyed";
        return LBIB_ESTATE;
    }
    return LBIB_OK;
}

}  // namespace

extern "C" {

lbib_status lbib_batch_create(lbib_ctx* const* sims, int32_t n, void* hip_stream, lbib_batch** out)
{
    if (!out) return LBIB_EINVAL;
    *out = nullptr;
    if (!sims || n < 1) return LBIB_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LBIB_EDEVICE;
    std::set<const lbib_ctx*> seen;
    for (int s = 0; s < n; ++s) {
        lbib_ctx* c = sims[s];
        if (!c || c->batch || !seen.insert(c).second) return LBIB_EINVAL;   // null, adopted or repeated
        const lbib_ctx* c0 = sims[0];
        if (c->n_cells <= 0 || c->device != dev || c->S != c0->S || c->p.storage != c0->p.storage ||
            c->mask_needed != c0->mask_needed) {
            c->err = "a batch needs simulations with cells, on the current device, with one species count, "
                     "storage type and source law";
            return LBIB_EINVAL;
        }
        if (no_flux_bits(c->p)) {
            c->err = "the batched pass has no no-flux membranes";
            return LBIB_EINVAL;
        }
        if (mass_sources(c->p) || c->p.pressure_ring || c->d_nsrc || c->d_pmap) {
            c->err = "the batched pass has no mass sources or pressure boundaries";
            return LBIB_EINVAL;
        }
        if (c->p.interp_half_force) {
            c->err = "the batched pass interpolates u, not the half-force-shifted velocity";
            return LBIB_EINVAL;
        }
    }
    lbib_batch* b = new (std::nothrow) lbib_batch();
    if (!b) return LBIB_ENOMEM;
    b->sims.assign(sims, sims + n);
    b->S = sims[0]->S;
    b->storage = sims[0]->p.storage;
    b->mask = sims[0]->mask_needed;
    lbib_status st = LBIB_OK;
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return LBIB_EDEVICE;
    } else {
        b->own_stream = true;
    }
    if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess)
        st = LBIB_EDEVICE;
    // every simulation starts aligned: its lists built at the current positions
    for (int s = 0; s < n && st == LBIB_OK; ++s) {
        lbib_ctx* c = sims[s];
        if (c->steps_since_lists != 0) st = build_lists(c);
        if (st == LBIB_OK && hipStreamSynchronize(c->stream) != hipSuccess) st = LBIB_EDEVICE;
        b->cur0.push_back(c->cur);
        b->updates_per_step += c->nn;
    }
    if (st == LBIB_OK) st = build_tables(b, LTILE_Y);
    if (st != LBIB_OK) {
        lbib_batch_destroy(b);
        return st;
    }
    for (lbib_ctx* c : b->sims) {
        c->batch = b;
        c->batch_done = b->done;
    }
    publish(b);
    *out = b;
    return LBIB_OK;
}

void lbib_batch_destroy(lbib_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->side) (void)hipStreamSynchronize(b->side);
    for (lbib_ctx* c : b->sims) {
        if (!c || c->batch != b) continue;
        c->batch = nullptr;
        c->batch_done = nullptr;
        // lists of another tile height are rebuilt for the context's own pass
        if (b->lty != LTILE_Y && b->lty != 0) {
            (void)build_lists(c);
            (void)hipStreamSynchronize(c->stream);
        }
    }
    drop_graph(b);
    free_groups(b);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

const char* lbib_batch_last_error(const lbib_batch* b)
{
    if (!b) return "";
    return b->err.c_str();
}

lbib_status lbib_batch_step(lbib_batch* b, int32_t n)
{
    if (!b) return LBIB_ESTATE;
    BATCH_TRY(usable(b));
    if (n < 0) {
        b->err = "negative step count";
        return LBIB_EINVAL;
    }
    const lbib_status st = advance(b, n);
    publish(b);
    return st;
}

lbib_status lbib_batch_sync(lbib_batch* b)
{
    if (!b) return LBIB_ESTATE;
    BATCH_TRY(usable(b));
    BATCH_HIP(b, hipStreamSynchronize(b->stream));
    for (size_t s = 0; s < b->sims.size(); ++s) {
        int h = 0;
        BATCH_HIP(b, hipMemcpyAsync(&h, b->sims[s]->d_err, sizeof(int), hipMemcpyDeviceToHost, b->stream));
        BATCH_HIP(b, hipStreamSynchronize(b->stream));
        if (h) {
            b->err = "simulation " + std::to_string(s) +
                     ((h & ERR_NONFINITE) ? ": a membrane node position or force became non-finite"
                                          : ": a membrane node moved more than 2 lattice units between list rebuilds");
            return LBIB_ENUMERIC;
        }
    }
    return LBIB_OK;
}

lbib_status lbib_batch_get_tile(const lbib_batch* b, int32_t* rows)
{
    if (!b || !rows) return LBIB_EINVAL;
    *rows = b->lty;
    return LBIB_OK;
}

lbib_status lbib_batch_set_tile(lbib_batch* b, int32_t rows)
{
    if (!b) return LBIB_ESTATE;
    BATCH_TRY(usable(b));
    if (!tile_ok_all(b, rows)) {
        b->err = "tile height must be 8 or 16, or 4 where every simulation has walls or ny divisible by 4";
        return LBIB_EINVAL;
    }
    if (b->since != 0 || b->par != 0) {
        b->err = "the tile height can change only after a whole number of list periods";
        return LBIB_ESTATE;
    }
    if (rows == b->lty) return LBIB_OK;
    BATCH_TRY(set_tile(b, rows));
    publish(b);
    return LBIB_OK;
}

lbib_status lbib_batch_get_groups(const lbib_batch* b, int32_t* groups)
{
    if (!b || !groups) return LBIB_EINVAL;
    *groups = (int32_t)b->groups.size();
    return LBIB_OK;
}

lbib_status lbib_batch_set_groups(lbib_batch* b, int32_t groups)
{
    if (!b) return LBIB_ESTATE;
    BATCH_TRY(usable(b));
    if (groups != 1 && groups != 2) {
        b->err = "a batch steps in 1 or 2 groups";
        return LBIB_EINVAL;
    }
    if (b->since != 0 || b->par != 0) {
        b->err = "the grouping can change only after a whole number of list periods";
        return LBIB_ESTATE;
    }
    if (groups == (int)b->groups.size()) return LBIB_OK;
    BATCH_TRY(set_groups(b, groups));
    publish(b);
    return LBIB_OK;
}

lbib_status lbib_batch_autotune(lbib_batch* b, int32_t periods, int32_t* rows, int32_t* groups, double* ms_per_step)
{
    if (!b) return LBIB_ESTATE;
    BATCH_TRY(usable(b));
    if (periods < 1) {
        b->err = "periods must be at least 1";
        return LBIB_EINVAL;
    }
    if (b->since != 0 || b->par != 0) {
        b->err = "autotuning starts only after a whole number of list periods";
        return LBIB_ESTATE;
    }
    for (int k = 0; k < 6 && ms_per_step; ++k) ms_per_step[k] = -1.0;
    BATCH_HIP(b, hipStreamSynchronize(b->stream));
    Snapshot snap;
    lbib_status st = snapshot(b, snap, false);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == LBIB_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = LBIB_EDEVICE;
    const int start = b->lty, start_groups = (int)b->groups.size();
    int best = start, best_groups = start_groups;
    double best_ms = -1.0;
    const int max_groups = b->sims.size() >= 2 ? 2 : 1;
    for (int gi = 0; gi < max_groups && st == LBIB_OK; ++gi) {
        b->ngroups = gi + 1;
        for (int k = 0; k < 3 && st == LBIB_OK; ++k) {
            const int lty = TILE_CHOICES[k];
            if (!tile_ok_all(b, lty)) continue;
            st = set_tile(b, lty);
            if (st == LBIB_OK) st = advance(b, LIST_PERIOD);            // warm-up (captures the graph)
            if (st == LBIB_OK && hipEventRecord(e0, b->stream) != hipSuccess) st = LBIB_EDEVICE;
            if (st == LBIB_OK) st = advance(b, (int64_t)periods * LIST_PERIOD);
            if (st == LBIB_OK && hipEventRecord(e1, b->stream) != hipSuccess) st = LBIB_EDEVICE;
            if (st == LBIB_OK && hipEventSynchronize(e1) != hipSuccess) st = LBIB_EDEVICE;
            float ms = 0.0f;
            if (st == LBIB_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = LBIB_EDEVICE;
            if (st != LBIB_OK) break;
            const double per = (double)ms / ((double)periods * LIST_PERIOD);
            if (ms_per_step) ms_per_step[3 * gi + k] = per;
            if (best_ms < 0.0 || per < best_ms) {
                best_ms = per;
                best = lty;
                best_groups = gi + 1;
            }
            st = snapshot(b, snap, true);                              // back to the starting state
        }
    }
    if (st == LBIB_OK) {
        b->ngroups = best_groups;
        st = set_tile(b, best);
    } else if (!snap.buf.empty() && snap.buf[0]) {
        // a failed candidate: back to the starting state, grouping and tile height, lists rebuilt
        (void)hipStreamSynchronize(b->stream);
        (void)hipStreamSynchronize(b->side);
        (void)snapshot(b, snap, true);
        b->ngroups = start_groups;
        (void)set_tile(b, start);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    free_snapshot(snap);
    if (st == LBIB_OK && rows) *rows = best;
    if (st == LBIB_OK && groups) *groups = best_groups;
    publish(b);
    return st;
}

}  // extern "C"
