// Device-side definitions shared by the lbib HIP kernels (gfx950).
//
// Storage: every population is kept as a deviation from its rest value,
// df_i = f_i - w_i rho0 and dg_i = g_i - w_i phi_ref, in arrays chunked by TILE_X columns:
// a lattice row is a run of chunks, each holding the Q planes of its 64 columns one after the
// other ([ny][ceil(nx / 64)][Q][64], x fastest; the last chunk of a row is padded).  A
// workgroup's loads and stores then fall into a few contiguous kilobyte runs instead of 2Q
// separate streams, which DRAM serves markedly faster.  Q = 9 for the fluid and 5 S for the
// species (species s in planes 5 s .. 5 s + 4).  The arrays hold post-collision,
// pre-streaming values; a lattice pass pulls f_i(x) = f*_i(x - v_i) (or, across a wall,
// f*_opp(i)(x)), collides, and stores f*_i(x) in place of x in the other buffer.
//
// Immersed-boundary nodes are listed per lattice tile (TILE_X x LTILE_Y nodes): every few
// steps (LIST_PERIOD) each node enters the list of every tile that its 4x4 stencil can reach
// while its stencil origin (floor(X) - 1) stays within LIST_MARGIN lattice units of the origin
// it had then.  The membrane kernel refreshes each node's spreading record at the node's own
// index every step and flags a node that drifted further.  Each list entry also receives,
// every step, the tile's share of its node's interpolated velocity; the membrane kernel adds
// a node's shares in the order of its tiles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbib.h"

namespace lbib {

// workgroup of the lattice pass: 64 x 4 threads (one 64-wide wavefront per row), each thread
// taking RPT rows, so a lattice tile is TILE_X x LTILE_Y nodes
constexpr int TILE_X = 64;
constexpr int TILE_Y = 4;
constexpr int TILE_N = TILE_X * TILE_Y;
constexpr int RPT = 2;                // rows per thread of a single simulation's pass
constexpr int LTILE_Y = TILE_Y * RPT;
constexpr int MIN_LTILE_Y = TILE_Y;   // the shortest tile (one row per thread) sizes the tile arrays

constexpr int LIST_MARGIN = 2;       // lattice units a node may drift between list rebuilds
constexpr int LIST_PERIOD = 16;      // steps between list rebuilds (nodes may move 2/16 lu per step)
constexpr int MAX_NODE_TILES = 9;    // tiles one node can be listed in (3 columns x 3 rows at most)
constexpr int GRAPH_STEPS = LBIB_GRAPH_STEPS;   // steps per captured graph (a multiple of LIST_PERIOD)

constexpr int MEMBRANE_THREADS = 192;             // three wavefronts per cell
constexpr int MEMBRANE_BATCH = 2;               // nodes per lane whose loads are issued together
constexpr int MEMBRANE_THREADS_MANY = 128;        // the batched form: two wavefronts per cell,
constexpr int MEMBRANE_BATCH_MANY = 3;           // three nodes per lane (several rounds of cells)
constexpr int MAX_CELL_NODES = 4096;            // LDS holds one cell's positions as double2
constexpr int RASTER_THREADS = 256;
constexpr int RASTER_WORDS_FUSED = 1024;        // 4 KB bitmap inside the membrane kernel
constexpr int RASTER_WORDS = 8192;              // 32 KB bitmap in the standalone rasteriser
constexpr int SCAN_THREADS = 1024;
constexpr int LIST_THREADS = 256;             // nodes per workgroup of the list build
constexpr int SCAN_PER_THREAD = 8;

// Spread forces are summed in 64-bit fixed point (integer addition is associative, so the
// sum does not depend on the order the nodes arrive in): value = integer * 2^-48.
constexpr float FIX_SCALE = 281474976710656.0f;          // 2^48
constexpr float FIX_INV = 1.0f / 281474976710656.0f;     // 2^-48 (exact)
constexpr float FIX_CLAMP = 16384.0f;                    // |contribution| bound, keeps sums in range

// error flags (device int, OR-ed)
constexpr int ERR_NONFINITE = 1;     // a node position or force became non-finite
constexpr int ERR_MARGIN = 2;        // a node drifted beyond its list margin
constexpr int ERR_FIELDS = 4;        // a monitor sum of the lattice was not finite

// Element (plane p, row y, column x) of a chunked population array whose rows hold `row`
// elements and whose chunks hold `chunk` = Q * TILE_X elements.
__device__ inline int64_t pop_at(int64_t row, int chunk, int p, int y, int x)
{
    return (int64_t)y * row + (int64_t)(x / TILE_X) * chunk + p * TILE_X + (x % TILE_X);
}

struct LatticeArgs {
    const void* __restrict__ fsrc;    // 9 planes of the storage type, chunked
    void* __restrict__ fdst;
    const void* __restrict__ gsrc;    // 5 * S planes, chunked
    void* __restrict__ gdst;
    int64_t nn;                       // nx * ny
    int64_t frow, grow;               // elements per lattice row of the fluid / species arrays
    int gchunk;                       // elements per chunk of the species array (5 S TILE_X)
    int nx, ny, walls, ntx;
    float omega, rho0;
    double omega_d, bodyx_d, bodyy_d;   // the same in FP64 (the FP32-storage collision's arithmetic)
    float omega_s[2], phi_ref[2];
    double omega_s_d[2], phi_ref_d[2];
    int react[2];
    float rc[2][4];
    double rc_d[2][4];
    float bodyx, bodyy;
    int kernel;
    // immersed boundary: node lists per lattice tile, spreading records per node
    const int* __restrict__ t_off;     // [ntiles + 1] list offsets (NULL: no nodes)
    const int* __restrict__ t_list;    // entries: node index << 4 | the tile's rank among the node's tiles
    const float4* __restrict__ rec;    // [N] (sx, sy, Fx, Fy): fractional offset and force
    const int* __restrict__ rec_ij;    // [N] packed stencil origin (i0 | j0 << 16)
    float2* __restrict__ part;         // [MAX_NODE_TILES][N] share of the node's velocity per tile
    int64_t n_nodes;
    const unsigned* __restrict__ inside;   // inside-any-cell bits of this step, rows of wpr words
    unsigned* __restrict__ inside_clr;     // the other buffer, cleared for the membrane kernel
    int wpr;
    int noflux;                            // bit s: the membranes are no-flux boundaries for species s
    // mass sources: the cell each node lies in (read and reset to ~0 here; NULL: no sources),
    // S_k = msrc + alpha (A0_k - A_k) from the reference and current areas
    unsigned* __restrict__ cmap;
    const double* __restrict__ A0;
    const double* __restrict__ area;
    double msrc, alpha;
    double gamma;                          // + gamma phi_0(x) at nodes inside a cell
    int nf_bb;                             // no-flux over cut links: 0 first-order replacement,
                                           // 1 bounce-back from the node's own slots, 2 bounce-back
                                           // of a state set from outside (its pulled populations)
    int pring;                             // the outer ring of nodes is held at density rho0
    const float* __restrict__ nsrc;        // [ny][nx] mass per node and step (NULL: none)
    const uint8_t* __restrict__ pmap;      // [ny][nx] pressure points held at rho0 (NULL: none)
    // no-flux membranes in the first-order form (nfq NULL: none): wall distances [4][nn] and
    // blocked-link bytes [nn] of this step's positions, the concentration deviations [S][nn] and
    // velocities [nn] the previous step's collision saw (read) and this step's (written)
    const float* __restrict__ nfq;
    const uint8_t* __restrict__ nfm;
    const float* __restrict__ nfphi;
    const float2* __restrict__ nfu;
    float* __restrict__ nfphi_out;
    float2* __restrict__ nfu_out;
    // inspection output (spread field only)
    double* __restrict__ e_out;
};

struct MembraneArgs {
    const int* __restrict__ off;
    double2* __restrict__ X;
    const double* __restrict__ l0;
    const double* __restrict__ A0;
    double* __restrict__ area;
    const float2* __restrict__ part;   // [MAX_NODE_TILES][N] velocity shares (from the lattice pass)
    const uint8_t* __restrict__ cnt;   // [N] number of tiles each node is listed in
    int64_t n_nodes;
    const int* __restrict__ ij_list;   // packed stencil origin of each node at the last list build
    float4* __restrict__ rec;          // [N]
    int* __restrict__ rec_ij;          // [N]
    unsigned* __restrict__ inside;     // inside-any-cell bits, OR-ed into when raster != 0
    const uint8_t* __restrict__ src;   // [n_cells] source cells (NULL: every cell is rasterised)
    unsigned* __restrict__ cmap;       // mass sources: [ny][nx] cell of each node, the lowest index
                                       // claiming it (reset to ~0 by the lattice pass); NULL: none
    int wpr;
    int* __restrict__ err;
    int64_t nn;
    int nx, ny, walls, kernel;
    double k_spring, phi_m, kappa;
    int advect;
    int raster;
    int need_area;                     // compute (and store) the cell areas
    // no-flux membranes in the first-order form (NULL: none): the crossings of the new
    // positions go into nfq (atomic minimum of the wall distance) and nfm (blocked-link bits,
    // OR-ed into 32-bit words of four node bytes); those of the previous positions are cleared
    // from the other pair of buffers, which the lattice pass of this step has read
    float* __restrict__ nfq;
    unsigned* __restrict__ nfm;
    float* __restrict__ nfq_old;
    uint8_t* __restrict__ nfm_old;
};

struct ListArgs {
    const double2* __restrict__ X;
    int* __restrict__ ij_list;         // stencil origin of each node at this build
    int* __restrict__ count;           // [ntiles], zero between builds (the scan clears it)
    int* __restrict__ off;             // [ntiles + 1]
    int* __restrict__ cursor;          // [ntiles] fill positions
    int* __restrict__ list;            // [N * MAX_NODE_TILES] capacity: node << 4 | rank of the tile
    uint8_t* __restrict__ cnt;         // [N] tiles the node is listed in
    int64_t n;
    int nx, ny, walls, ntx, nlty, ntiles;
    int lty;                           // rows per lattice tile (TILE_Y times the rows per thread)
    int lty_shift;                     // log2(lty): tile heights are powers of two
};

// ADE-only iteration (species with u = 0, fluid and membranes frozen) in a working set of
// WT (float or double) deviations dg = g - w phi_ref, planes [S][5][ny][nx]
struct AdeArgs {
    const void* __restrict__ src;
    void* __restrict__ dst;
    double* __restrict__ phi_prev;     // [S][ny][nx] phi of the previous pass
    const unsigned* __restrict__ inside;   // source bits (source/decay law)
    int wpr;
    double* __restrict__ partial;      // [slots][nblocks][4] per-block sums of each pass
    int64_t nn;
    int nx, ny, walls, S;
    double omega_s[2], phi_ref[2];
    int react[2];
    double rc[2][4];
    int hslot;                         // history slot of this pass
    int track;                         // 0: first pass (phi_prev is only written)
};

// batched ADE-only iterations: B single-species problems (source/decay, u = 0) on one lattice
// size, absolute populations in the working type
constexpr int ADE_BATCH_SLOTS = 64;   // passes per captured batch of the batched solver
struct AdeBatchArgs {
    const void* __restrict__ src;      // [B][5][ny][nx] working populations (absolute values)
    void* __restrict__ dst;
    double* __restrict__ phi_prev;     // [B][ny][nx]
    const uint8_t* __restrict__ source;   // [B][ny][nx] 1 inside a source cell
    const double* __restrict__ omega;  // [B] 1 / tau_D
    const double* __restrict__ sigma;  // [B] source rate
    const double* __restrict__ decay;  // [B]
    const int* __restrict__ active;    // [B] 0 once converged
    double* __restrict__ partial;      // [slots][B][nblocks][2]
    int64_t nn;
    int nx, ny, walls, B, nblocks;
    int hslot, track;
};

struct RasterArgs {
    const int* __restrict__ off;
    const double2* __restrict__ X;
    uint16_t* __restrict__ mask;
    int nx, ny, walls;
};

// ---------------------------------------------------------------------------------------
// 1-D kernel weights for the four stencil points i0 .. i0+3 of a node whose fractional
// offset is s = X - floor(X) in [0, 1), i0 = floor(X) - 1, i.e. at distances
// r = s+1, s, s-1, s-2.
// Cosine kernel (Eq. 1Dkernel): with c = cos(pi s/2), n = sin(pi s/2) the four values are
// (1-n)/4, (1+c)/4, (1+n)/4, (1-c)/4.
// Peskin's 4-point kernel: with q = sqrt(1 + 4s - 4s^2) they are
// (3-2s-q)/8, (3-2s+q)/8, (1+2s+q)/8, (1+2s-q)/8.
// The sine and cosine of t = pi s/2 in [0, pi/2) come from their Taylor series, through the
// t^11 and t^12 terms: the first omitted terms, t^13/13! and t^14/14!, stay below 6e-8 and
// 7e-9, under the FP32 rounding of the results, and the sums w0 + w2 = w1 + w3 = 1/2 hold
// whatever the values.
// ---------------------------------------------------------------------------------------
__host__ __device__ inline void delta_weights(int kernel, float s, float w[4])
{
    if (kernel == 0) {
        const float t = 1.5707963267948966f * s, t2 = t * t;
        const float sn = t * (1.0f + t2 * (-1.0f / 6 + t2 * (1.0f / 120 + t2 * (-1.0f / 5040 +
                         t2 * (1.0f / 362880 + t2 * (-1.0f / 39916800))))));
        const float cs = 1.0f + t2 * (-0.5f + t2 * (1.0f / 24 + t2 * (-1.0f / 720 + t2 * (1.0f / 40320 +
                         t2 * (-1.0f / 3628800 + t2 * (1.0f / 479001600))))));
        w[0] = 0.25f * (1.0f - sn);
        w[1] = 0.25f * (1.0f + cs);
        w[2] = 0.25f * (1.0f + sn);
        w[3] = 0.25f * (1.0f - cs);
    } else {
        float q = sqrtf(1.0f + 4.0f * s - 4.0f * s * s);
        w[0] = 0.125f * (3.0f - 2.0f * s - q);
        w[1] = 0.125f * (3.0f - 2.0f * s + q);
        w[2] = 0.125f * (1.0f + 2.0f * s + q);
        w[3] = 0.125f * (1.0f + 2.0f * s - q);
    }
}

// i mod n for 32-bit i; the common case (one period off at most) avoids a division
__device__ inline int wrap_i(int i, int n)
{
    if (i >= n) {
        i -= n;
        if (i >= n) i %= n;
    } else if (i < 0) {
        i += n;
        if (i < 0) {
            i %= n;
            if (i < 0) i += n;
        }
    }
    return i;
}

// finite and small enough for 32-bit stencil arithmetic (|coordinate| < 2^30)
__device__ inline bool finite2(double x, double y)
{
    return fabs(x) < 1073741824.0 && fabs(y) < 1073741824.0;
}

// stencil origin of a node (finite2 positions): column wrapped into [0, nx); row wrapped
// (periodic) or, next to walls, clamped to [-4, ny] (rows outside the lattice receive nothing)
__device__ inline void stencil_origin(double x, double y, int nx, int ny, int walls, int& i0, int& j0)
{
    i0 = wrap_i((int)floor(x) - 1, nx);
    const int j = (int)floor(y) - 1;
    if (walls) j0 = j < -4 ? -4 : (j > ny ? ny : j);
    else j0 = wrap_i(j, ny);
}

// The D2Q5 links a membrane edge (A, B) cuts (Suppl. "No-flux Boundary Condition for
// Reaction-Advection-Diffusion Equations"), by the crossing rule of the domain IDs: the edge
// crosses row y when (A.y > y) != (B.y > y), at x_c = A.x + (y - A.y)(B.x - A.x)/(B.y - A.y),
// cutting the link between columns ceil(x_c) - 1 and ceil(x_c); columns likewise with x and y
// exchanged (links to rows beyond a wall do not exist).  For each cut, emit(d, node, q) names
// the node whose population arriving in direction d (0..3: +x, +y, -x, -y) crosses the edge
// and its distance q to the cut, as a fraction of the link.  Contraction is off, so the
// abscissae round as written (the same values as the rasteriser's).
template <typename F>
__device__ inline void edge_link_cuts(double2 A, double2 B, int nx, int ny, int walls, F&& emit)
{
#pragma clang fp contract(off)
    const int ylo = (int)floor(fmin(A.y, B.y)), yhi = (int)floor(fmax(A.y, B.y));
    for (int py = ylo; py <= yhi && py - ylo <= ny; ++py) {
        const double yy = (double)py;
        if ((A.y > yy) == (B.y > yy)) continue;
        int j;
        if (walls) {
            if (py < 0 || py >= ny) continue;
            j = py;
        } else {
            j = wrap_i(py, ny);
        }
        const double xc = A.x + (yy - A.y) * (B.x - A.x) / (B.y - A.y);
        const double ir = ceil(xc);
        const int i = wrap_i((int)ir, nx), il = (i == 0) ? nx - 1 : i - 1;
        emit(0, (int64_t)j * nx + i, (float)(ir - xc));
        emit(2, (int64_t)j * nx + il, (float)(xc - (ir - 1.0)));
    }
    const int xlo = (int)floor(fmin(A.x, B.x)), xhi = (int)floor(fmax(A.x, B.x));
    for (int px = xlo; px <= xhi && px - xlo <= nx; ++px) {
        const double xx = (double)px;
        if ((A.x > xx) == (B.x > xx)) continue;
        const double yc = A.y + (xx - A.x) * (B.y - A.y) / (B.x - A.x);
        const double jt = ceil(yc);
        const int i = wrap_i(px, nx), jtop = (int)jt;
        int j1, j0;
        if (walls) {
            if (jtop < 1 || jtop >= ny) continue;             // both rows inside the lattice
            j1 = jtop;
            j0 = jtop - 1;
        } else {
            j1 = wrap_i(jtop, ny);
            j0 = (j1 == 0) ? ny - 1 : j1 - 1;
        }
        emit(1, (int64_t)j1 * nx + i, (float)(jt - yc));
        emit(3, (int64_t)j0 * nx + i, (float)(yc - (jt - 1.0)));
    }
}

__device__ inline int pack_ij(int i0, int j0)
{
    return (i0 & 0xFFFF) | (int)((unsigned)(j0 & 0xFFFF) << 16);
}

// ---------------------------------------------------------------------------------------
// population storage: FP32 keeps the plain deviation; FP16 / BF16 keep deviation / w_i * 2^10
// ---------------------------------------------------------------------------------------
template <int ST> struct Pop;
template <> struct Pop<0> {
    using T = float;
    __device__ static float ld(T v, float) { return v; }
    __device__ static T st(float v, float) { return v; }
};
template <> struct Pop<1> {
    using T = _Float16;
    __device__ static float ld(T v, float inv) { return (float)v * inv; }
    __device__ static T st(float v, float sc) { return (T)(v * sc); }
};
template <> struct Pop<2> {
    using T = __bf16;
    __device__ static float ld(T v, float inv) { return (float)v * inv; }
    __device__ static T st(float v, float sc) { return (T)(v * sc); }
};
// storage scale 2^10 / w_i (exact integers) and its inverse, D2Q9 and D2Q5
__device__ constexpr float SC9[9] = {2304.0f, 9216.0f, 9216.0f, 9216.0f, 9216.0f, 36864.0f, 36864.0f, 36864.0f, 36864.0f};
__device__ constexpr float IS9[9] = {1.0f / 2304.0f, 1.0f / 9216.0f, 1.0f / 9216.0f, 1.0f / 9216.0f, 1.0f / 9216.0f,
                                     1.0f / 36864.0f, 1.0f / 36864.0f, 1.0f / 36864.0f, 1.0f / 36864.0f};
__device__ constexpr float SC5[5] = {3072.0f, 6144.0f, 6144.0f, 6144.0f, 6144.0f};
__device__ constexpr float IS5[5] = {1.0f / 3072.0f, 1.0f / 6144.0f, 1.0f / 6144.0f, 1.0f / 6144.0f, 1.0f / 6144.0f};


// Tile of a workgroup.  The dispatcher deals workgroups round-robin over the 8 XCDs.  Tiles
// go out by bands of two tile rows, so the whole chip sweeps one band of the lattice at a time
// (the HBM channels see neighbouring addresses); when the column count allows, each XCD takes
// a contiguous eighth of the columns and keeps those columns in every band, visiting the two
// rows of a column one after the other.  An XCD's L2 then serves the halo columns that
// horizontally adjacent tiles share, and the records and halo rows of vertically adjacent
// ones.  At 2048^2 this order beats plain row-major order by 3 % and giving each XCD a
// contiguous eighth of the lattice by 7 %.  With an odd number of tile rows the band is one
// row; with a column count that is not a multiple of 8, the order is plain row-major.  The
// batched pass lists each simulation's tiles in the same order (the dealing then only
// rotates which XCD takes which group).
__host__ __device__ inline int tile_of_block(int bid, int ntx, int nlty)
{
    if (ntx & 7) return bid;
    const int g = ntx >> 3, xcd = bid & 7, k = bid >> 3;
    if (nlty & 1) return (k / g) * ntx + xcd * g + (k % g);
    const int row = (k / (2 * g)) * 2 + (k & 1), col = xcd * g + (k >> 1) % g;
    return row * ntx + col;
}

}  // namespace lbib
