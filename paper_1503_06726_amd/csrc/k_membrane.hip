// Membrane kernels of the coupled step (gfx950).
//
// k_membrane: one workgroup (three wavefronts) per cell.  In a time step it
//   1. adds the node's interpolated velocity U (Eq. conversion2 with the kernel of
//      Eq. 1Dkernel; the lattice pass leaves one share per listed tile, added here in the
//      order of the node's tiles) and moves the node explicitly, X^{n+1} = X^n + U
//      (positions in FP64);
//   2. stages the cell's new positions in LDS and reduces the polygon area (shoelace, FP64,
//      fixed-order wave and LDS reduction);
//   3. when a reaction, no-flux membranes or mass sources read it, ORs the cell's interior
//      into the inside-any-cell bit map (rasterised from the LDS positions); with mass
//      sources it also claims the interior's nodes in the cell map;
//   4. evaluates the nodal forces in the paper's per-node form: constant tension
//      (Eq. membraneforce), Hookean springs, area pressure kappa (A0 - A) dA/dX, refreshes
//      the node's spreading record (fractional offset, force, stencil origin) and stores the
//      new position; a node that drifted beyond its list margin raises an error flag.
// Every global store comes after the last workgroup barrier, which would otherwise wait for
// them.
// k_list_count / k_list_scan / k_list_fill rebuild the per-tile node lists (every few steps).
// The *_batch forms run the same per-cell, per-node and per-simulation work for many
// independent simulations in one launch, each work item naming its simulation's arguments.
#include "lbib_internal.h"
#include "lbib_raster.h"

namespace lbib {

__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// has the stencil origin (i0, j0) moved at most LIST_MARGIN from its value at the last list
// build (packed in ijb)?  Then every tile its stencil reaches still lists the node.
__device__ inline bool within_margin(int i0, int j0, int ijb, int nx, int ny, int walls)
{
    const int ib = ijb & 0xFFFF, jb = ijb >> 16;
    int di = i0 - ib;
    if (di > nx / 2) di -= nx;
    else if (di < -(nx / 2)) di += nx;
    if (di > LIST_MARGIN || di < -LIST_MARGIN) return false;
    int dj;
    if (walls) {
        dj = j0 - jb;
    } else {
        dj = j0 - jb;
        if (dj > ny / 2) dj -= ny;
        else if (dj < -(ny / 2)) dj += ny;
    }
    return dj <= LIST_MARGIN && dj >= -LIST_MARGIN;
}

// a value known to be equal in every lane, moved to scalar registers
__device__ inline double uniform(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Block-wide sum of one double and minima of four (fixed order: waves, then LDS slots); the
// results are uniform.
__device__ inline void block_reduce5(double& sum, double m[4], double* red)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    sum = wave_sum(sum);
#pragma unroll
    for (int q = 0; q < 4; ++q) m[q] = wave_min(m[q]);
    if (lane == 0) {
        red[wid * 5] = sum;
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wid * 5 + 1 + q] = m[q];
    }
    __syncthreads();
    sum = red[0];
#pragma unroll
    for (int q = 0; q < 4; ++q) m[q] = red[1 + q];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
        sum += red[w * 5];
#pragma unroll
        for (int q = 0; q < 4; ++q) m[q] = fmin(m[q], red[w * 5 + 1 + q]);
    }
    sum = uniform(sum);
#pragma unroll
    for (int q = 0; q < 4; ++q) m[q] = uniform(m[q]);
}

// One cell per workgroup: xs holds the cell's positions (dynamic LDS), red the reduction
// slots, bm the raster bitmap.
template <int NT, int NB, bool NF1 = false>
__device__ __forceinline__ void membrane_cell(const MembraneArgs& a, const int c, double2* xs, double* red,
                                              unsigned* bm)
{
    const int t = threadIdx.x;
    const int beg = a.off[c];
    const int n = a.off[c + 1] - beg;
    const int64_t N = a.n_nodes;
    if (a.raster)
        for (int i = t; i < RASTER_WORDS_FUSED; i += NT) bm[i] = 0u;
    if constexpr (NF1) {
        // no-flux membranes, first-order form: the links the cell's edges cut at the previous
        // positions leave the buffers the lattice pass of this step has read (a cell's nodes
        // are written by its own workgroup only, at the end, so these are still the old ones)
        if (a.advect)
            for (int k = t; k < n; k += NT) {
                const double2 A = a.X[beg + k], B = a.X[beg + ((k + 1 == n) ? 0 : k + 1)];
                if (!(finite2(A.x, A.y) && finite2(B.x, B.y))) continue;
                edge_link_cuts(A, B, a.nx, a.ny, a.walls, [&](int d, int64_t node, float) {
                    a.nfq_old[(int64_t)d * a.nn + node] = INFINITY;
                    a.nfm_old[node] = 0;
                });
            }
    }

    // 1. move: X^{n+1} = X^n + U, U interpolated by the lattice pass as one share per listed
    //    tile, added in the order of the node's tiles; stage the new positions in LDS and track
    //    their bounding box.  A lane takes NB nodes per pass and issues all their loads first
    //    (a lane past the end loads the cell's last node and discards it: no branches around
    //    the loads).  The first four shares are read with the count (a node has at most four
    //    tiles unless its list range wraps onto a narrow last tile); slots beyond the count are
    //    never added.  Positions reach global memory only at the end: a workgroup barrier
    //    waits for every outstanding store.
    double bb[4] = {INFINITY, INFINITY, INFINITY, INFINITY};     // min x, min y, -max x, -max y
    for (int base = 0; base < n; base += NT * NB) {
        double2 X[NB];
        float2 sh[NB][4];
        int nt[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int64_t l = beg + min(base + j * NT + t, n - 1);
            X[j] = a.X[l];
            nt[j] = 0;
            if (a.advect) {
                nt[j] = a.cnt[l];
#pragma unroll
                for (int q = 0; q < 4; ++q) sh[j][q] = a.part[q * N + l];
            }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int k = base + j * NT + t;
            if (k >= n) continue;
            double2 x = X[j];
            if (a.advect) {
                double ux = 0.0, uy = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (nt[j] > q) {
                        ux += (double)sh[j][q].x;
                        uy += (double)sh[j][q].y;
                    }
                for (int q = 4; q < nt[j]; ++q) {
                    const float2 sq = a.part[q * N + beg + k];
                    ux += (double)sq.x;
                    uy += (double)sq.y;
                }
                if (finite2(x.x, x.y)) {
                    x.x += ux;
                    x.y += uy;
                }
            }
            xs[k] = x;
            bb[0] = fmin(bb[0], x.x);
            bb[1] = fmin(bb[1], x.y);
            bb[2] = fmin(bb[2], -x.x);
            bb[3] = fmin(bb[3], -x.y);
        }
    }
    if (!a.need_area) {
        // without the area, the bounding box alone: each wavefront's goes to LDS before the
        // barrier the positions need anyway (no second barrier for a block reduction)
#pragma unroll
        for (int q = 0; q < 4; ++q) bb[q] = wave_min(bb[q]);
        if ((t & 63) == 0)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[(t >> 6) * 5 + 1 + q] = bb[q];
    }
    __syncthreads();

    if constexpr (NF1) {
        // the links the edges cut at the new positions: the wall distance (the smallest over the
        // cuts of a link: non-negative floats order as their bit patterns) and the blocked bit
        for (int k = t; k < n; k += NT) {
            const double2 A = xs[k], B = xs[(k + 1 == n) ? 0 : k + 1];
            if (!(finite2(A.x, A.y) && finite2(B.x, B.y))) continue;
            edge_link_cuts(A, B, a.nx, a.ny, a.walls, [&](int d, int64_t node, float q) {
                atomicMin((unsigned*)&a.nfq[(int64_t)d * a.nn + node], __float_as_uint(q));
                atomicOr(&a.nfm[node >> 2], (1u << d) << (8 * (int)(node & 3)));
            });
        }
    }

    // 2. shoelace area about the first node (translation invariant, less cancellation), when the
    //    step reads it (area pressure, area controller) or it is asked for
    double A = 0.0, s_area = 0.0;
    if (a.need_area) {
        const double ox = uniform(xs[0].x), oy = uniform(xs[0].y);
        double A2 = 0.0;
        for (int k = t; k < n; k += NT) {
            const int kn = (k + 1 == n) ? 0 : k + 1;
            A2 += (xs[k].x - ox) * (xs[kn].y - oy) - (xs[kn].x - ox) * (xs[k].y - oy);
        }
        block_reduce5(A2, bb, red);
        A = 0.5 * A2;
        s_area = a.kappa * (a.A0[c] - A);
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double m = red[1 + q];
            for (int w = 1; w < NT / 64; ++w) m = fmin(m, red[w * 5 + 1 + q]);
            bb[q] = uniform(m);
        }
    }

    // 3. inside-any-cell bits of the new positions (the bitmap was cleared above); with a
    //    source subset only the source cells are rasterised.  No barrier follows the last
    //    chunk, so its atomics drain during the force pass.
    if (a.raster && !(a.src && !a.src[c])) {
        const RasterBox b = raster_box(bb[0], bb[1], -bb[2], -bb[3], a.nx, a.ny);
        if (b.ok) {                                                  // uniform across the group
            int CH = RASTER_WORDS_FUSED / b.WW;
            if (CH < 1) CH = 1;
            if (CH > b.H) CH = b.H;
            for (int r0 = 0; r0 < b.H; r0 += CH) {
                const int rows = (b.H - r0 < CH) ? b.H - r0 : CH;
                if (r0 > 0) {
                    for (int i = t; i < rows * b.WW; i += NT) bm[i] = 0u;
                    __syncthreads();
                }
                raster_toggle(xs, n, b, r0, rows, bm);
                __syncthreads();
                raster_prefix(bm, rows, b.WW);
                __syncthreads();
                raster_or_bits(bm, b, r0, rows, a.inside, a.wpr, a.nx, a.ny, a.walls);
                if (a.cmap) raster_claim_cells(bm, b, r0, rows, (unsigned)c, a.cmap, a.nx, a.ny, a.walls);
                if (r0 + CH < b.H) __syncthreads();
            }
        }
    }

    // 4. forces, spreading records and the new positions (no barrier follows: the stores
    //    drain while the workgroup retires); rest lengths and list origins of a lane's NB
    //    nodes are loaded first
    int flags = 0;
    for (int base = 0; base < n; base += NT * NB) {
        double lpv[NB], lmv[NB];
        int kyv[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int k = min(base + j * NT + t, n - 1);
            lpv[j] = a.l0[beg + k];
            lmv[j] = a.l0[beg + (k == 0 ? n - 1 : k - 1)];
            kyv[j] = a.ij_list[beg + k];
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int k = base + j * NT + t;
            if (k >= n) continue;
            const int kp = (k + 1 == n) ? 0 : k + 1;
            const int km = (k == 0) ? n - 1 : k - 1;
            const double lp = lpv[j], lm = lmv[j];
            const double2 X = xs[k], Xp = xs[kp], Xm = xs[km];
            const double dpx = Xp.x - X.x, dpy = Xp.y - X.y;
            const double dmx = Xm.x - X.x, dmy = Xm.y - X.y;
            const double Lp = sqrt(dpx * dpx + dpy * dpy), Lm = sqrt(dmx * dmx + dmy * dmy);
            // tension phi_m along both edges; springs k (L - l0) along each edge
            const double sp = (a.phi_m + a.k_spring * (Lp - lp)) / Lp;
            const double sm = (a.phi_m + a.k_spring * (Lm - lm)) / Lm;
            double Fx = sp * dpx + sm * dmx;
            double Fy = sp * dpy + sm * dmy;
            // area pressure: dA/dX_k = ((y_{k+1} - y_{k-1}) / 2, (x_{k-1} - x_{k+1}) / 2)
            Fx += s_area * 0.5 * (Xp.y - Xm.y);
            Fy += s_area * 0.5 * (Xm.x - Xp.x);
            const int s = beg + k;
            if (a.advect) a.X[s] = X;
            if (finite2(X.x, X.y) && finite2(Fx, Fy)) {
                const double fx = floor(X.x), fy = floor(X.y);
                int i0, j0;
                stencil_origin(X.x, X.y, a.nx, a.ny, a.walls, i0, j0);
                a.rec[s] = make_float4((float)(X.x - fx), (float)(X.y - fy), (float)Fx, (float)Fy);
                a.rec_ij[s] = pack_ij(i0, j0);
                if (!within_margin(i0, j0, kyv[j], a.nx, a.ny, a.walls)) flags |= ERR_MARGIN;
            } else {
                a.rec[s] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                a.rec_ij[s] = 0;
                flags |= ERR_NONFINITE;
            }
        }
    }
    if (t == 0 && a.need_area) a.area[c] = A;
    if (flags) atomicOr(a.err, flags);
}

// Three wavefronts per cell with two nodes per lane: a pass covers 384 nodes, and 6 waves per
// SIMD keep every workgroup of a 2000-cell step resident at once (more nodes per pass cost
// the registers that residency needs; a cell beyond a pass takes another)
template <bool NF1>
__global__ __launch_bounds__(MEMBRANE_THREADS) __attribute__((amdgpu_waves_per_eu(6))) void k_membrane(MembraneArgs a)
{
    extern __shared__ double2 xs[];
    __shared__ double red[5 * (MEMBRANE_THREADS / 64)];
    __shared__ unsigned bm[RASTER_WORDS_FUSED];
    membrane_cell<MEMBRANE_THREADS, MEMBRANE_BATCH, NF1>(a, blockIdx.x, xs, red, bm);
}

// Batched form: one (simulation, cell) work item per workgroup, the simulation's arguments
// from a device table.  The cells of many simulations take several rounds of workgroups,
// where two wavefronts per cell with three nodes per lane keep more cells in flight.
__global__ __launch_bounds__(MEMBRANE_THREADS_MANY) __attribute__((amdgpu_waves_per_eu(5))) void k_membrane_batch(const MembraneArgs* __restrict__ tab,
                                                                     const int2* __restrict__ work)
{
    extern __shared__ double2 xs[];
    __shared__ double red[5 * (MEMBRANE_THREADS_MANY / 64)];
    __shared__ unsigned bm[RASTER_WORDS_FUSED];
    const int2 wk = work[blockIdx.x];
    const MembraneArgs a = tab[wk.x];
    membrane_cell<MEMBRANE_THREADS_MANY, MEMBRANE_BATCH_MANY>(a, wk.y, xs, red, bm);
}

// ---------------------------------------------------------------------------------------
// per-tile node lists
// ---------------------------------------------------------------------------------------

// Lattice tiles a node with stencil origin (i0, j0) is listed in: every tile that meets
// columns i0 - M .. i0 + 3 + M and rows j0 - M .. j0 + 3 + M (M = LIST_MARGIN; columns cyclic,
// rows cyclic or, next to walls, only those inside the lattice), each once.  Eight
// consecutive columns touch at most three tile columns (the last tile may be narrow and the
// range may wrap), and so do eight rows for tiles of at least 8 rows, or of 4 rows when the
// rows do not wrap onto a narrow last tile (walls, or ny a multiple of 4; the host admits no
// other tile height).  Tiles come out row by row in ascending order of the range, so the list
// build is a pure function of the origin and the tile shape.
__device__ inline int node_tiles(int i0, int j0, const ListArgs& a, int tiles[MAX_NODE_TILES])
{
    constexpr int M = LIST_MARGIN;
    int cols[3], nc = 0, rows[3], nr = 0;
#pragma unroll
    for (int q = -M; q <= 3 + M; ++q) {
        const int cc = wrap_i(i0 + q, a.nx) / TILE_X;
        bool seen = false;
        for (int k = 0; k < nc; ++k) seen = seen || cols[k] == cc;
        if (!seen && nc < 3) cols[nc++] = cc;
    }
#pragma unroll
    for (int q = -M; q <= 3 + M; ++q) {
        int j = j0 + q;
        if (a.walls) {
            if (j < 0 || j >= a.ny) continue;
        } else {
            j = wrap_i(j, a.ny);
        }
        const int rr = j >> a.lty_shift;                      // j >= 0 here
        bool seen = false;
        for (int k = 0; k < nr; ++k) seen = seen || rows[k] == rr;
        if (!seen && nr < 3) rows[nr++] = rr;
    }
    int n = 0;
    for (int r = 0; r < nr; ++r)
        for (int k = 0; k < nc; ++k) tiles[n++] = rows[r] * a.ntx + cols[k];
    return n;
}

// Wavefront-aggregated increment: every live lane adds 1 to counter[key].  Lanes are grouped
// into runs of consecutive lanes with the same key (consecutive membrane nodes mostly share a
// tile); the first lane of each run adds the run length with one atomic, all runs at once.
// Returns the counter's previous value plus the lane's rank within its run (when RET).
template <bool RET>
__device__ inline int wave_claim(int* counter, int key, bool live)
{
    const int lane = threadIdx.x & 63;
    const int k = live ? key : -1;
    const int prev = __shfl_up(k, 1, 64);
    const bool head = lane == 0 || prev != k;
    const unsigned long long heads = __ballot(head);
    const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const int first = 63 - __clzll((long long)(heads & upto));            // head of the lane's run
    int pos = 0;
    if (head && live) {
        const unsigned long long above = heads & ~upto;
        const int next = above ? __ffsll((long long)above) - 1 : 64;    // head of the next run
        if constexpr (RET) pos = atomicAdd(&counter[key], next - lane);
        else atomicAdd(&counter[key], next - lane);
    }
    if constexpr (RET) pos = __shfl(pos, first, 64) + (lane - first);
    return pos;
}

// stencil origin of every node at this build, and the length of every tile's list (node l
// of a block whose wavefronts all take part)
__device__ __forceinline__ void list_count_node(const ListArgs& a, const int64_t l)
{
    const bool live = l < a.n;
    int tiles[MAX_NODE_TILES];
    int nt = 0;
    if (live) {
        const double2 X = a.X[l];
        int ij = 0;
        if (finite2(X.x, X.y)) {
            int i0, j0;
            stencil_origin(X.x, X.y, a.nx, a.ny, a.walls, i0, j0);
            ij = pack_ij(i0, j0);
            nt = node_tiles(i0, j0, a, tiles);
        }
        a.ij_list[l] = ij;
    }
    for (int k = 0; k < MAX_NODE_TILES; ++k) {
        const bool on = live && k < nt;
        if (!__ballot(on)) break;
        (void)wave_claim<false>(a.count, on ? tiles[k] : 0, on);
    }
}

__global__ void k_list_count(ListArgs a)
{
    list_count_node(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// batched: work items (simulation, block of LIST_THREADS nodes)
__global__ __launch_bounds__(LIST_THREADS) void k_list_count_batch(const ListArgs* __restrict__ tab,
                                                                   const int2* __restrict__ work)
{
    const int2 wk = work[blockIdx.x];
    const ListArgs a = tab[wk.x];
    list_count_node(a, (int64_t)wk.y * LIST_THREADS + threadIdx.x);
}

// exclusive scan of the list lengths into offsets (and fill cursors); counts are cleared for
// the next build (one workgroup per simulation)
__device__ __forceinline__ void list_scan(const ListArgs& a, int* buf, int* wsum, int& carry_sh)
{
    constexpr int CHUNK = SCAN_THREADS * SCAN_PER_THREAD;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    if (t == 0) carry_sh = 0;
    for (int base = 0; base < a.ntiles; base += CHUNK) {
        for (int i = t; i < CHUNK; i += SCAN_THREADS) {
            const int b = base + i;
            int v = 0;
            if (b < a.ntiles) {
                v = a.count[b];
                a.count[b] = 0;
            }
            buf[i] = v;
        }
        __syncthreads();
        int s = 0;
        for (int q = 0; q < SCAN_PER_THREAD; ++q) s += buf[t * SCAN_PER_THREAD + q];
        // inclusive scan across the wavefront
        int incl = s;
        for (int o = 1; o < 64; o <<= 1) {
            const int up = __shfl_up(incl, o, 64);
            if (lane >= o) incl += up;
        }
        if (lane == 63) wsum[wid] = incl;
        __syncthreads();
        int pre = carry_sh;
        for (int w = 0; w < wid; ++w) pre += wsum[w];
        int run = pre + incl - s;
        for (int q = 0; q < SCAN_PER_THREAD; ++q) {
            const int v = buf[t * SCAN_PER_THREAD + q];
            buf[t * SCAN_PER_THREAD + q] = run;
            run += v;
        }
        __syncthreads();
        for (int i = t; i < CHUNK; i += SCAN_THREADS) {
            const int b = base + i;
            if (b < a.ntiles) {
                a.off[b] = buf[i];
                a.cursor[b] = buf[i];
            }
        }
        if (t == SCAN_THREADS - 1) carry_sh = run;
        __syncthreads();
    }
    if (t == 0) a.off[a.ntiles] = carry_sh;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_list_scan(ListArgs a)
{
    __shared__ int buf[SCAN_THREADS * SCAN_PER_THREAD];
    __shared__ int wsum[SCAN_THREADS / 64];
    __shared__ int carry_sh;
    list_scan(a, buf, wsum, carry_sh);
}

__global__ __launch_bounds__(SCAN_THREADS) void k_list_scan_batch(const ListArgs* __restrict__ tab)
{
    __shared__ int buf[SCAN_THREADS * SCAN_PER_THREAD];
    __shared__ int wsum[SCAN_THREADS / 64];
    __shared__ int carry_sh;
    const ListArgs a = tab[blockIdx.x];
    list_scan(a, buf, wsum, carry_sh);
}

// every node enters the lists of its tiles, each entry naming the node and the rank of the
// tile among the node's tiles (order within a list is immaterial: the lattice pass sums
// forces in fixed point, and each velocity share goes to its own [rank][node] slot)
__device__ __forceinline__ void list_fill_node(const ListArgs& a, const int64_t l)
{
    const bool live = l < a.n;
    int tiles[MAX_NODE_TILES];
    int nt = 0;
    if (live) {
        const double2 X = a.X[l];
        if (finite2(X.x, X.y)) {
            const int ij = a.ij_list[l];
            nt = node_tiles(ij & 0xFFFF, ij >> 16, a, tiles);
        }
    }
    if (live) a.cnt[l] = (uint8_t)nt;
    for (int k = 0; k < MAX_NODE_TILES; ++k) {
        const bool on = live && k < nt;
        if (!__ballot(on)) break;
        const int p = wave_claim<true>(a.cursor, on ? tiles[k] : 0, on);
        if (on) a.list[p] = (int)(((unsigned)l << 4) | (unsigned)k);
    }
}

__global__ void k_list_fill(ListArgs a)
{
    list_fill_node(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(LIST_THREADS) void k_list_fill_batch(const ListArgs* __restrict__ tab,
                                                                  const int2* __restrict__ work)
{
    const int2 wk = work[blockIdx.x];
    const ListArgs a = tab[wk.x];
    list_fill_node(a, (int64_t)wk.y * LIST_THREADS + threadIdx.x);
}

// forces of every node, read back from the records (inspection)
__global__ void k_forces_out(const float4* __restrict__ rec, float2* __restrict__ F, int64_t n)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const float4 r = rec[l];
    F[l] = make_float2(r.z, r.w);
}

__global__ void k_fill_i32(int* p, int64_t n, int v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u16(uint16_t* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_fill_f32(float* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

hipError_t launch_membrane(lbib_ctx* c, const MembraneArgs& a)
{
    const size_t lds = sizeof(double2) * (size_t)(c->max_cell_nodes > 0 ? c->max_cell_nodes : 1);
    if (a.nfq)
        hipLaunchKernelGGL(k_membrane<true>, dim3((unsigned)c->n_cells), dim3(MEMBRANE_THREADS), lds, c->stream, a);
    else
        hipLaunchKernelGGL(k_membrane<false>, dim3((unsigned)c->n_cells), dim3(MEMBRANE_THREADS), lds, c->stream, a);
    return hipGetLastError();
}

hipError_t launch_lists(lbib_ctx* c, const ListArgs& a, int which)
{
    const unsigned nb = (unsigned)((a.n + LIST_THREADS - 1) / LIST_THREADS);
    if (which == 0) hipLaunchKernelGGL(k_list_count, dim3(nb), dim3(LIST_THREADS), 0, c->stream, a);
    else if (which == 1) hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(SCAN_THREADS), 0, c->stream, a);
    else hipLaunchKernelGGL(k_list_fill, dim3(nb), dim3(LIST_THREADS), 0, c->stream, a);
    return hipGetLastError();
}

hipError_t launch_membrane_batch(const MembraneArgs* tab, const int2* work, int nwork, int max_cell_nodes,
                                 hipStream_t stream)
{
    if (nwork <= 0) return hipSuccess;
    const size_t lds = sizeof(double2) * (size_t)(max_cell_nodes > 0 ? max_cell_nodes : 1);
    hipLaunchKernelGGL(k_membrane_batch, dim3((unsigned)nwork), dim3(MEMBRANE_THREADS_MANY), lds, stream, tab, work);
    return hipGetLastError();
}

hipError_t launch_lists_batch(const ListArgs* tab, const int2* work, int nwork, int nsims, int which,
                              hipStream_t stream)
{
    if (which == 1) {
        if (nsims > 0) hipLaunchKernelGGL(k_list_scan_batch, dim3((unsigned)nsims), dim3(SCAN_THREADS), 0, stream, tab);
    } else if (nwork > 0) {
        if (which == 0) hipLaunchKernelGGL(k_list_count_batch, dim3((unsigned)nwork), dim3(LIST_THREADS), 0, stream, tab, work);
        else hipLaunchKernelGGL(k_list_fill_batch, dim3((unsigned)nwork), dim3(LIST_THREADS), 0, stream, tab, work);
    }
    return hipGetLastError();
}

hipError_t launch_forces_out(lbib_ctx* c, float2* F)
{
    const unsigned nb = (unsigned)((c->n_nodes + 255) / 256);
    hipLaunchKernelGGL(k_forces_out, dim3(nb), dim3(256), 0, c->stream, (const float4*)c->d_rec, F, c->n_nodes);
    return hipGetLastError();
}

hipError_t launch_fill_i32(lbib_ctx* c, int* p, int64_t n, int v)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u16(lbib_ctx* c, uint16_t* p, int64_t n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, p, n);
    return hipGetLastError();
}

hipError_t launch_fill_f32(lbib_ctx* c, float* p, int64_t n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, p, n);
    return hipGetLastError();
}

}  // namespace lbib
