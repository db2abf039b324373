// Lattice kernels of the coupled step (gfx950).
//
// k_lattice: one fused pass per time step over the whole lattice, one 64x8 tile per
// workgroup.  Per tile:
//   1. per lattice node: pull the D2Q9 populations (streaming of Eq. bgkequation, halfway
//      bounce-back at walls) and take rho and u = sum f v / rho (u staged in LDS);
//   2. for every membrane node in the tile's list: spread its force over the stencil points
//      inside the tile (Eq. forcedistribution with the kernel of Eq. 1Dkernel), summed in LDS
//      in 64-bit fixed point so the result does not depend on node order, and store the
//      tile's share of the node's interpolated velocity (Eq. conversion2) in the node's slot
//      for this tile;
//   3. collide with the BGK operator and the body-force term w_i rho (v_i . e) / cs2, store;
//   4. per species: pull the D2Q5 populations, take phi, add the reaction, collide towards
//      phi w_i (1 + v_i . u / cs2) with the fluid's u, store; the source term reads the
//      inside-any-cell bit of the node (the word-aligned bits of the other buffer are cleared
//      here for the membrane kernel to fill).
// The pass reads every population once and writes it once: it is HBM-bandwidth bound.
#include "lbib_internal.h"

#include <mutex>

namespace lbib {

// D2Q9 weights (Suppl. "Lattice Boltzmann Method": 4/9, 1/9 x4, 1/36 x4)
#define W0 (4.0f / 9.0f)
#define W1 (1.0f / 9.0f)
#define W5 (1.0f / 36.0f)
// D2Q5 weights: 1/3, 1/6 x4
#define Q0 (1.0f / 3.0f)
#define Q1 (1.0f / 6.0f)

// Arithmetic of the fluid's moments and collision.  With FP32 storage it runs in FP64: in a
// steadily forced flow every node's populations change by the same small increment each step,
// so the FP32 rounding of the collision's intermediate products would repeat with the same
// sign at every node and step and add up to a drift of the velocity (about 1e-5 relative after
// 1,000 steps of a channel starting up under a body force, growing linearly); in FP64 only the
// rounding of the stored deviations is left.  The same holds for a species fed by a steady
// source.  The 16-bit storage forms keep FP32 arithmetic (their storage rounding is far
// larger).
template <int ST> struct Arith {
    using T = float;
    __device__ static float body(float f, double) { return f; }
    __device__ static float fix(long long v) { return __ll2float_rn(v) * FIX_INV; }
    __device__ static float c(float f, double) { return f; }
};
template <> struct Arith<0> {
    using T = double;
    __device__ static double body(float, double d) { return d; }
    __device__ static double fix(long long v) { return (double)v * (double)FIX_INV; }   // exact below 2^53
    __device__ static double c(float, double d) { return d; }
};

template <typename Rt> struct Moments {
    Rt drho, rho, ux, uy;
};
// density deviation, density and velocity u = sum f v / rho of a node's D2Q9 deviations
template <typename Rt>
__device__ inline Moments<Rt> moments(const float f[9], float rho0)
{
    Rt fr[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) fr[i] = (Rt)f[i];
    Moments<Rt> m;
    m.drho = ((fr[0] + fr[1]) + (fr[2] + fr[3])) + ((fr[4] + fr[5]) + (fr[6] + fr[7])) + fr[8];
    m.rho = (Rt)rho0 + m.drho;
    const Rt jx = (fr[1] - fr[3]) + (fr[5] - fr[6]) + (fr[8] - fr[7]);
    const Rt jy = (fr[2] - fr[4]) + (fr[5] + fr[6]) - (fr[7] + fr[8]);
    const Rt inv = (Rt)1 / m.rho;
    m.ux = jx * inv;
    m.uy = jy * inv;
    return m;
}

struct Nbr {
    int y, ym, yp;        // rows y, y-1, y+1 (clamped at walls)
    int x, xm, xp;        // columns x, x-1, x+1 (periodic)
    bool bot, top;        // y-1 (y+1) lies beyond a wall
};

__device__ inline Nbr neighbours(int x, int y, int nx, int ny, int walls)
{
    Nbr n;
    n.x = x;
    n.y = y;
    n.xm = (x == 0) ? nx - 1 : x - 1;
    n.xp = (x == nx - 1) ? 0 : x + 1;
    if (walls) {
        n.bot = (y == 0);
        n.top = (y == ny - 1);
        n.ym = n.bot ? y : y - 1;
        n.yp = n.top ? y : y + 1;
    } else {
        n.bot = n.top = false;
        n.ym = (y == 0) ? ny - 1 : y - 1;
        n.yp = (y == ny - 1) ? 0 : y + 1;
    }
    return n;
}

// bit of node (x, y) in the inside-cell map (x, y inside the lattice)
__device__ inline unsigned inside_bit(const LatticeArgs& a, int x, int y)
{
    return (a.inside[(int64_t)y * a.wpr + (x >> 5)] >> (x & 31)) & 1u;
}

// offset of column x within its row of a chunked array (chunk = Q TILE_X elements)
__device__ inline int chunk_col(int x, int chunk) { return (x / TILE_X) * chunk + (x % TILE_X); }

// Element `idx` of a row whose base address is the same for the whole wavefront: the base
// stays in scalar registers and each lane adds a 32-bit byte offset (a row holds far fewer
// than 2^30 elements), which spares the 64-bit address arithmetic per load and store.
template <typename T>
__device__ inline const T& row_at(const T* base, int idx)
{
    return *(const T*)((const char*)base + (unsigned)((unsigned)idx * (unsigned)sizeof(T)));
}
// The same element loaded with the non-temporal hint, for the planes whose cache lines one
// tile reads whole (v_x = 0: each line holds the 64 columns of one chunk, and every element
// is pulled by a node of the same tile).  The lines of the other planes are shared by two
// horizontally adjacent tiles (one column crosses the chunk edge) and keep the default
// policy, so the second tile still finds them in the L2; the lines the hint spares leave room
// for them and for the node data the membrane kernel reads next.
template <typename T>
__device__ inline T row_nt(const T* base, int idx)
{
    const T* q = (const T*)((const char*)base + (unsigned)((unsigned)idx * (unsigned)sizeof(T)));
    if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_nontemporal_load((const unsigned*)q));
    else return __builtin_bit_cast(T, __builtin_nontemporal_load((const unsigned short*)q));
}
template <typename T>
__device__ inline T* row_ptr(T* base, int idx)
{
    return (T*)((char*)base + (unsigned)((unsigned)idx * (unsigned)sizeof(T)));
}

// f_i(x) = s_i(x - v_i); across a wall the population returns reversed: s_opp(i)(x).
// Velocities: 0 rest, 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1), 5 (1,1), 6 (-1,1), 7 (-1,-1), 8 (1,-1).
// Values come back as FP32 deviations (w_opp(i) = w_i, so the storage scale matches).
// s: the chunked fluid array (rows of `row` elements, chunks of 9 TILE_X).
template <int ST>
__device__ inline void pull9(const void* sv, int64_t row, const Nbr& n, float f[9])
{
    using T = typename Pop<ST>::T;
    constexpr int C = 9 * TILE_X, P = TILE_X;
    const T* __restrict__ s = (const T*)sv;
    const T* rc = s + (int64_t)n.y * row;
    const T* rm = s + (int64_t)n.ym * row;
    const T* rp = s + (int64_t)n.yp * row;
    const int cx = chunk_col(n.x, C), cm = chunk_col(n.xm, C), cp = chunk_col(n.xp, C);
    // across a wall the row is the node's own and the plane the opposite one
    f[0] = Pop<ST>::ld(row_nt(rc, cx), IS9[0]);
    f[1] = Pop<ST>::ld(row_at(rc, cm + P), IS9[1]);
    f[2] = Pop<ST>::ld(row_nt(n.bot ? rc : rm, cx + (n.bot ? 4 : 2) * P), IS9[2]);
    f[3] = Pop<ST>::ld(row_at(rc, cp + 3 * P), IS9[3]);
    f[4] = Pop<ST>::ld(row_nt(n.top ? rc : rp, cx + (n.top ? 2 : 4) * P), IS9[4]);
    f[5] = Pop<ST>::ld(row_at(n.bot ? rc : rm, n.bot ? cx + 7 * P : cm + 5 * P), IS9[5]);
    f[6] = Pop<ST>::ld(row_at(n.bot ? rc : rm, n.bot ? cx + 8 * P : cp + 6 * P), IS9[6]);
    f[7] = Pop<ST>::ld(row_at(n.top ? rc : rp, n.top ? cx + 5 * P : cp + 7 * P), IS9[7]);
    f[8] = Pop<ST>::ld(row_at(n.top ? rc : rp, n.top ? cx + 6 * P : cm + 8 * P), IS9[8]);
}

// one species: s points at the species' first plane within the chunked species array
// (rows of `row` elements, chunks of `chunk` = 5 S TILE_X)
template <int ST>
__device__ inline void pull5(const void* sv, int64_t row, int chunk, const Nbr& n, float g[5])
{
    using T = typename Pop<ST>::T;
    constexpr int P = TILE_X;
    const T* __restrict__ s = (const T*)sv;
    const T* rc = s + (int64_t)n.y * row;
    const T* rm = s + (int64_t)n.ym * row;
    const T* rp = s + (int64_t)n.yp * row;
    const int cx = chunk_col(n.x, chunk), cm = chunk_col(n.xm, chunk), cp = chunk_col(n.xp, chunk);
    g[0] = Pop<ST>::ld(row_nt(rc, cx), IS5[0]);
    g[1] = Pop<ST>::ld(row_at(rc, cm + P), IS5[1]);
    g[2] = Pop<ST>::ld(row_nt(n.bot ? rc : rm, cx + (n.bot ? 4 : 2) * P), IS5[2]);
    g[3] = Pop<ST>::ld(row_at(rc, cp + 3 * P), IS5[3]);
    g[4] = Pop<ST>::ld(row_nt(n.top ? rc : rp, cx + (n.top ? 2 : 4) * P), IS5[4]);
}

// streaming store that bypasses the caches' retention (the next pass reads it from HBM)
template <typename T>
__device__ inline void store_nt(T* p, T v)
{
    if constexpr (sizeof(T) == 4) __builtin_nontemporal_store(__builtin_bit_cast(unsigned, v), (unsigned*)p);
    else __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v), (unsigned short*)p);
}

__device__ inline unsigned long long to_fixed(float v)
{
    v = fminf(fmaxf(v, -FIX_CLAMP), FIX_CLAMP);
    return (unsigned long long)__float2ll_rn(v * FIX_SCALE);
}

// A node's force component F in fixed point (F 2^48), split for the weighted contributions
struct FixedForce {
    int hi;           // signed upper word
    unsigned lo;      // lower word
};

__device__ inline FixedForce fixed_force(float v)
{
    const long long q = (long long)to_fixed(v);
    int hi = (int)(q >> 32);
    // an empty asm statement: the compiler then treats hi as a plain 32-bit integer and
    // multiplies it with one signed 32 x 32 -> 64 multiply-add, not a 64-bit product
    asm volatile("" : "+v"(hi));
    return {hi, (unsigned)q};
}

// floor(F 2^48 * wq / 2^32) for a stencil weight wq = w 2^32 (0 <= w <= 1/4, so wq < 2^31):
// the spread contribution w F in the same fixed point, from two integer products (exact but
// for the floor): a signed 32 x 32 -> 64 multiply-add of the upper word and the high half of
// the lower word's product
__device__ inline unsigned long long weighted_fixed(FixedForce f, unsigned wq)
{
    return (unsigned long long)((long long)f.hi * (long long)(int)wq + (long long)__umulhi(f.lo, wq));
}

constexpr float WQ_SCALE = 4294967296.0f;   // 2^32

constexpr int SPREAD_UNROLL = 1;   // listed nodes per thread whose loads are issued together

// The tile's LDS arrays (spread force accumulators, staged velocity) hold rows of TILE_X + 1
// entries: with the padding, stencil points of different rows in the same column fall into
// different LDS banks (the membrane nodes a wavefront couples lie close together, so unpadded
// rows made their atomics collide in the same banks).
constexpr int LDS_ROW = TILE_X + 1;

// LDS slot of row r of thread t (thread t covers column t % TILE_X of rows t / TILE_X + r TILE_Y)
__device__ inline int lds_slot(int t, int r) { return (t / TILE_X + r * TILE_Y) * LDS_ROW + (t % TILE_X); }

// Load one chunk of the tile's listed nodes [beg, end): list entry (node << 4 | rank of this
// tile among the node's tiles; -1, which names no node, past the end), stencil origin, record.
__device__ inline void load_candidates(const LatticeArgs& a, int k0, int end, int ij[SPREAD_UNROLL],
                                       float4 rc[SPREAD_UNROLL], int ent[SPREAD_UNROLL])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < SPREAD_UNROLL; ++u) {
        const int k = k0 + u * TILE_N + t;
        ij[u] = 0x7FFF7FFF;                              // far away: never hits
        ent[u] = -1;
        if (k < end) {
            const int e = a.t_list[k];
            const int node = (int)((unsigned)e >> 4);
            ent[u] = e;
            ij[u] = a.rec_ij[node];
            rc[u] = a.rec[node];
        }
    }
}

// The same in two halves, so that other loads can be issued between them: the list entries
// of the chunk, then (once they are back) the stencil origins and records they name.
__device__ inline void load_entries(const LatticeArgs& a, int k0, int end, int ent[SPREAD_UNROLL])
{
#pragma unroll
    for (int u = 0; u < SPREAD_UNROLL; ++u) {
        const int k = k0 + u * TILE_N + (int)threadIdx.x;
        ent[u] = (k < end) ? a.t_list[k] : -1;
    }
}

// (loads without branches: a lane past the end reads node 0's record and discards it, which
// lets the compiler wait for exactly the loads each use needs)
__device__ inline void load_records(const LatticeArgs& a, const int ent[SPREAD_UNROLL], int ij[SPREAD_UNROLL],
                                    float4 rc[SPREAD_UNROLL])
{
#pragma unroll
    for (int u = 0; u < SPREAD_UNROLL; ++u) {
        const int node = (ent[u] != -1) ? (int)((unsigned)ent[u] >> 4) : 0;
        const int v = a.rec_ij[node];
        rc[u] = a.rec[node];
        ij[u] = (ent[u] != -1) ? v : 0x7FFF7FFF;        // far away: never hits
    }
}

// slot of a list entry's velocity share: [rank of the tile][node]
__device__ inline int64_t share_slot(const LatticeArgs& a, int e)
{
    return (int64_t)(e & 15) * a.n_nodes + (int64_t)((unsigned)e >> 4);
}

// Couple one chunk of listed nodes with the tile [x0, x1) x [y0, y1) (LDS rows TILE_X apart):
// spread each node's force into the LDS accumulators (Eq. forcedistribution), and, when
// INTERP, compute the node's share of the interpolated velocity from the tile's u (LDS) over
// the tile's own stencil points (Eq. conversion2) into Ud (zero when the stencil misses).
// The caller stores the shares by node and tile rank; DEFER leaves that to after the tile's
// population stores, because a workgroup barrier waits for every outstanding global memory
// operation and the shares are not needed before the end.
template <bool INTERP, bool DEFER = false, bool SPREAD = true>
__device__ inline void couple_chunk(const LatticeArgs& a, int x0, int x1, int y0, int y1,
                                    const int ij[SPREAD_UNROLL], const float4 rc[SPREAD_UNROLL],
                                    const int ent[SPREAD_UNROLL], unsigned long long* accx, unsigned long long* accy,
                                    const float2* us, float2* Ud = nullptr)
{
#pragma unroll
    for (int u = 0; u < SPREAD_UNROLL; ++u) {
        if constexpr (INTERP) Ud[u] = make_float2(0.0f, 0.0f);
        const int i0 = ij[u] & 0xFFFF;
        const int j0 = ij[u] >> 16;                      // sign-extended 16-bit row
        // tile coordinates of the four stencil columns and rows (each wrapped on its own,
        // so a stencil that wraps onto the same tile twice is still counted correctly)
        int lx[4], ly[4];
        unsigned hx = 0u, hy = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int i = i0 + q;
            if (i >= a.nx) i -= a.nx;
            lx[q] = i - x0;
            if ((unsigned)lx[q] < (unsigned)(x1 - x0)) hx |= 1u << q;
            int j = j0 + q;
            bool ok = true;
            if (a.walls) ok = j >= 0 && j < a.ny;
            else if (j >= a.ny) j -= a.ny;
            ly[q] = j - y0;
            if (ok && (unsigned)ly[q] < (unsigned)(y1 - y0)) hy |= 1u << q;
        }
        if (!hx || !hy) continue;
        const float4 r = rc[u];
        float wx[4], wy[4];
        delta_weights(a.kernel, r.x, wx);
        delta_weights(a.kernel, r.y, wy);
        FixedForce fx{0, 0u}, fy{0, 0u};
        if constexpr (SPREAD) {
            fx = fixed_force(r.z);
            fy = fixed_force(r.w);
        }
        float Ux = 0.0f, Uy = 0.0f;
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
            if (!((hy >> bb) & 1u)) continue;
            float sx = 0.0f, sy = 0.0f;
            // the row's four columns without branches: a column outside the tile adds zero to
            // the row's first slot and contributes nothing to the velocity
#pragma unroll
            for (int aa = 0; aa < 4; ++aa) {
                const bool in = (hx >> aa) & 1u;
                const int o = ly[bb] * LDS_ROW + (in ? lx[aa] : 0);
                float2 uv;
                if constexpr (INTERP) uv = us[o];          // read first: the atomics need not wait for it
                if constexpr (SPREAD) {
                    const unsigned wq = in ? (unsigned)(wx[aa] * wy[bb] * WQ_SCALE) : 0u;
                    atomicAdd(&accx[o], weighted_fixed(fx, wq));
                    atomicAdd(&accy[o], weighted_fixed(fy, wq));
                }
                if constexpr (INTERP) {
                    sx += in ? wx[aa] * uv.x : 0.0f;
                    sy += in ? wx[aa] * uv.y : 0.0f;
                }
            }
            if constexpr (INTERP) {
                Ux += wy[bb] * sx;
                Uy += wy[bb] * sy;
            }
        }
        if constexpr (INTERP) Ud[u] = make_float2(Ux, Uy);
    }
    if constexpr (INTERP && !DEFER) {
#pragma unroll
        for (int u = 0; u < SPREAD_UNROLL; ++u)
            if (ent[u] != -1) a.part[share_slot(a, ent[u])] = Ud[u];
    }
}

// No-flux membranes, the supplement's first-order condition, at node (x, y) for one species:
// every population whose link a membrane edge cuts (bit d of the node's byte mk; d = 0..3 for
// +x, +y, -x, -y) is replaced by the equilibrium w (phi_b + 3 v . j_b), in deviations
// w (dphi_b + 3 v . j_b), with the momentum j_b interpolated between the node one step on in
// the population's direction and zero at the wall, j_b = q / (1 + q) phi_1 u_1 (q the wall
// distance as a fraction of the link), and the density extrapolated linearly from the nodes one
// and two steps on, dphi_b = 2 dphi_1 - dphi_2.  The values are those of the previous step's
// collision (planes written by the previous pass).  A node two steps on that lies beyond a wall
// or behind a cut link gives dphi_b = dphi_1; a node one step on that does, dphi_b = the node's
// own dphi and j_b = 0.
template <typename Args>
__device__ inline void nf_first_replace(const Args& a, int s, int x, int y, unsigned mk, float g[5])
{
    const int64_t k = (int64_t)y * a.nx + x;
    const float* __restrict__ ph = a.nfphi + (int64_t)s * a.nn;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        if (!((mk >> d) & 1u)) continue;
        const int vx = (d == 0) ? 1 : (d == 2) ? -1 : 0;
        const int vy = (d == 1) ? 1 : (d == 3) ? -1 : 0;
        int y1 = y + vy, y2 = y + 2 * vy;
        bool ok1 = true, ok2 = true;
        if (a.walls) {
            ok1 = y1 >= 0 && y1 < a.ny;
            ok2 = y2 >= 0 && y2 < a.ny;
        } else {
            y1 = wrap_i(y1, a.ny);
            y2 = wrap_i(y2, a.ny);
        }
        const int64_t k1 = ok1 ? (int64_t)y1 * a.nx + wrap_i(x + vx, a.nx) : k;
        const int64_t k2 = ok2 ? (int64_t)y2 * a.nx + wrap_i(x + 2 * vx, a.nx) : k;
        if (ok1 && ((a.nfm[k1] >> d) & 1u)) ok1 = false;
        if (!ok1 || ((a.nfm[k2] >> d) & 1u)) ok2 = false;
        float db, jv = 0.0f;
        if (!ok1) {
            db = ph[k];
        } else {
            const float q = a.nfq[(int64_t)d * a.nn + k];
            const float d1 = ph[k1];
            const float2 u1 = a.nfu[k1];
            jv = q / (1.0f + q) * ((float)a.phi_ref[s] + d1) * ((float)vx * u1.x + (float)vy * u1.y);
            db = ok2 ? 2.0f * d1 - ph[k2] : d1;
        }
        g[1 + d] = Q1 * (db + 3.0f * jv);
    }
}

// No-flux membranes in the bounce-back form (over the first-order form's cut links, bits d of
// mk for the populations 1 + d): a population that would arrive across a cut link becomes the
// one the node sent in the opposite direction the step before, its post-collision population
// stored in its own slot of the source buffer gs (nf_bb = 1).  A state set from outside has
// not streamed yet: each node is taken to have sent its own populations, which the pull has
// just brought in as g (nf_bb = 2).  What one side of a cut link sends, the other never
// receives, so the species is conserved exactly.
template <int ST, typename Args>
__device__ inline void nf_bounce(const Args& a, const void* gs, int s, int x, int y, unsigned mk, float g[5])
{
    float sent[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) sent[i] = g[i];
    if (a.nf_bb == 1) {
        const typename Pop<ST>::T* p = (const typename Pop<ST>::T*)gs;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const int o = 1 + ((d + 2) & 3);           // the direction opposite to 1 + d
            if ((mk >> d) & 1u) sent[o] = Pop<ST>::ld(p[pop_at(a.grow, a.gchunk, 5 * s + o, y, x)], IS5[o]);
        }
    }
#pragma unroll
    for (int d = 0; d < 4; ++d)
        if ((mk >> d) & 1u) g[1 + d] = sent[1 + ((d + 2) & 3)];
}

// One lattice tile of TILE_X x LTILE_Y nodes per workgroup; thread (lx, ly) handles rows
// ly, ly + TILE_Y, ...  Order: listed nodes' records and the population loads issued; moments
// (rho, u) of every row, u staged in LDS; listed nodes coupled (force spread into LDS, velocity
// interpolated to the nodes); collision with the spread force and stores.
template <int S, bool NODES, bool MASK, int ST, int RP, int NF = 0, bool MS = false, bool HF = false>
__device__ __forceinline__ void lattice_tile(const LatticeArgs& a, const int tile)
{
    constexpr int LY = TILE_Y * RP;
    constexpr int NL = NODES ? LDS_ROW * LY : 1;
    const int tcol = tile % a.ntx, trow = tile / a.ntx;
    const int x0 = tcol * TILE_X, y0 = trow * LY;
    const int x1 = min(x0 + TILE_X, a.nx), y1 = min(y0 + LY, a.ny);
    const int t = threadIdx.x;
    const int x = x0 + (t % TILE_X);

    __shared__ unsigned long long accx[NL], accy[NL];
    __shared__ float2 us[NL];

    // Load order: the first chunk's list entries, the populations, then the records the entries
    // name.  Loads complete in order, so waiting for the entries does not wait for the
    // populations, and the entry -> record round trip overlaps the population loads.
    int lbeg = 0, lend = 0;
    int cij[SPREAD_UNROLL], cnd[SPREAD_UNROLL];
    float4 crc[SPREAD_UNROLL];
    float2 Ud[SPREAD_UNROLL];
    if constexpr (NODES) {
        lbeg = a.t_off[tile];
        lend = a.t_off[tile + 1];
        load_entries(a, lbeg, lend, cnd);
#pragma unroll
        for (int r = 0; r < RP; ++r) {
            accx[lds_slot(t, r)] = 0ull;
            accy[lds_slot(t, r)] = 0ull;
        }
    }

    Nbr n[RP];
    bool active[RP];
    float f[RP][9];
    float g[RP][S > 0 ? S : 1][5];
    int m[RP];
    unsigned miss[RP];            // no-flux membranes: D2Q5 directions 1..4 that arrived across one
                                  // (first-order form: bits 0..3, the node's cut links)
    unsigned cell[RP];            // mass sources: the cell the node lies in (~0: none)
    // every lane loads (lanes beyond a ragged edge read the last column / row and discard it):
    // without branches around the loads the compiler waits for exactly the ones each use needs
#pragma unroll
    for (int r = 0; r < RP; ++r) {
        const int y = y0 + t / TILE_X + r * TILE_Y;
        active[r] = x < a.nx && y < a.ny;
        const int xl = min(x, a.nx - 1);
        const int yl = __builtin_amdgcn_readfirstlane(min(y, a.ny - 1));   // one row per wavefront
        n[r] = neighbours(xl, yl, a.nx, a.ny, a.walls);
        pull9<ST>(a.fsrc, a.frow, n[r], f[r]);
#pragma unroll
        for (int s = 0; s < S; ++s)
            pull5<ST>((const typename Pop<ST>::T*)a.gsrc + 5 * s * TILE_X, a.grow, a.gchunk, n[r], g[r][s]);
        m[r] = 0;
        if constexpr (MASK) {
            // the row's two bit words are the same for the whole wavefront: scalar loads
            const unsigned* row = a.inside + (int64_t)yl * a.wpr + (x0 >> 5);
            const unsigned w0 = row[0];
            const unsigned w1 = (x0 + 32 < a.nx) ? row[1] : 0u;
            m[r] = (((x & 32) ? w1 : w0) >> (x & 31)) & 1u;
        }
        miss[r] = 0u;
        if constexpr (NF == 2) miss[r] = a.nfm[(int64_t)yl * a.nx + xl];
        if constexpr (NF == 1) {
            // direction i arrives from x - v_i: +x from x-1, +y from y-1, -x from x+1, -y from
            // y+1; it crossed a membrane when the inside map differs between the two nodes
            // (a population reflected by a wall did not)
            const Nbr& q = n[r];
            const unsigned me = inside_bit(a, q.x, q.y);
            unsigned ms = 0u;
            if (inside_bit(a, q.xm, q.y) != me) ms |= 2u;
            if (!q.bot && inside_bit(a, q.x, q.ym) != me) ms |= 4u;
            if (inside_bit(a, q.xp, q.y) != me) ms |= 8u;
            if (!q.top && inside_bit(a, q.x, q.yp) != me) ms |= 16u;
            miss[r] = ms;
        }
        cell[r] = ~0u;
        if constexpr (MS) {
            if (a.cmap) cell[r] = a.cmap[(int64_t)yl * a.nx + xl];
        }
    }
    if constexpr (NODES) load_records(a, cnd, cij, crc);

    // moments of every row: rho^n, u^n = sum f v / rho (taken again by the collision from the
    // same populations, so no FP64 value stays live across the coupling)
    using Rt = typename Arith<ST>::T;
#pragma unroll
    for (int r = 0; r < RP; ++r) {
        if constexpr (MS) {
            // pressure boundary on the outer ring and at the pressure points: f_i -> gamma f_i
            // with gamma = rho0 / rho, in deviations d_i -> gamma (d_i - w_i drho); the
            // velocity is unchanged
            const int y = y0 + t / TILE_X + r * TILE_Y;
            const bool ring = a.pring && (x == 0 || x == a.nx - 1 || y == 0 || y == a.ny - 1);
            if (ring || (a.pmap && a.pmap[(int64_t)n[r].y * a.nx + n[r].x])) {
                float* fr = f[r];
                const float d = ((fr[0] + fr[1]) + (fr[2] + fr[3])) + ((fr[4] + fr[5]) + (fr[6] + fr[7])) + fr[8];
                const float gm = a.rho0 / (a.rho0 + d);
                fr[0] = gm * (fr[0] - W0 * d);
#pragma unroll
                for (int i = 1; i < 5; ++i) fr[i] = gm * (fr[i] - W1 * d);
#pragma unroll
                for (int i = 5; i < 9; ++i) fr[i] = gm * (fr[i] - W5 * d);
            }
        }
        if constexpr (NODES) {
            const Moments<Rt> mo = moments<Rt>(f[r], a.rho0);
            us[lds_slot(t, r)] = make_float2((float)mo.ux, (float)mo.uy);
        }
    }

    if constexpr (NODES && HF) {
        // the nodes move with the half-force-shifted velocity u + e/2: every listed node is
        // spread first, the tile's velocity is restaged with the complete force, then the
        // nodes interpolate it (the first chunk's records stay in registers for the second pass)
        __syncthreads();
        couple_chunk<false>(a, x0, x1, y0, y1, cij, crc, cnd, accx, accy, us);
        int cij0[SPREAD_UNROLL], cnd0[SPREAD_UNROLL];
        float4 crc0[SPREAD_UNROLL];
#pragma unroll
        for (int u = 0; u < SPREAD_UNROLL; ++u) {
            cij0[u] = cij[u];
            cnd0[u] = cnd[u];
            crc0[u] = crc[u];
        }
        for (int k0 = lbeg + SPREAD_UNROLL * TILE_N; k0 < lend; k0 += SPREAD_UNROLL * TILE_N) {
            load_candidates(a, k0, lend, cij, crc, cnd);
            couple_chunk<false>(a, x0, x1, y0, y1, cij, crc, cnd, accx, accy, us);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RP; ++r) {
            const int l = lds_slot(t, r);
            const float ex = a.bodyx + __ll2float_rn((long long)accx[l]) * FIX_INV;
            const float ey = a.bodyy + __ll2float_rn((long long)accy[l]) * FIX_INV;
            const float2 u0 = us[l];
            us[l] = make_float2(u0.x + 0.5f * ex, u0.y + 0.5f * ey);
        }
        __syncthreads();
        couple_chunk<true, true, false>(a, x0, x1, y0, y1, cij0, crc0, cnd0, accx, accy, us, Ud);
        if (lend - lbeg > SPREAD_UNROLL * TILE_N) {
            float2 Ux[SPREAD_UNROLL];
            for (int k0 = lbeg + SPREAD_UNROLL * TILE_N; k0 < lend; k0 += SPREAD_UNROLL * TILE_N) {
                load_candidates(a, k0, lend, cij, crc, cnd);
                couple_chunk<true, false, false>(a, x0, x1, y0, y1, cij, crc, cnd, accx, accy, us, Ux);
            }
        }
#pragma unroll
        for (int u = 0; u < SPREAD_UNROLL; ++u) cnd[u] = cnd0[u];
        // the collision reads the accumulators, final since the barrier above
    } else if constexpr (NODES) {
        __syncthreads();
        couple_chunk<true, true>(a, x0, x1, y0, y1, cij, crc, cnd, accx, accy, us, Ud);
        if (lend - lbeg > SPREAD_UNROLL * TILE_N) {
            int ent0[SPREAD_UNROLL];                      // the first chunk's entries, stored last
#pragma unroll
            for (int u = 0; u < SPREAD_UNROLL; ++u) ent0[u] = cnd[u];
            float2 Ux[SPREAD_UNROLL];
            for (int k0 = lbeg + SPREAD_UNROLL * TILE_N; k0 < lend; k0 += SPREAD_UNROLL * TILE_N) {
                load_candidates(a, k0, lend, cij, crc, cnd);
                couple_chunk<true>(a, x0, x1, y0, y1, cij, crc, cnd, accx, accy, us, Ux);
            }
#pragma unroll
            for (int u = 0; u < SPREAD_UNROLL; ++u) cnd[u] = ent0[u];
        }
        __syncthreads();
    }

#pragma unroll
    for (int r = 0; r < RP; ++r) {
        if (!active[r]) continue;
        if constexpr (S > 0) {
            // populations that arrived across a no-flux membrane are replaced first: the
            // concentration-driven mass source reads the replaced concentration
            if constexpr (NF == 2) {
                if (miss[r]) {
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        if (!((a.noflux >> s) & 1)) continue;
                        if (a.nf_bb) nf_bounce<ST>(a, a.gsrc, s, x, n[r].y, miss[r], g[r][s]);
                        else nf_first_replace(a, s, x, n[r].y, miss[r], g[r][s]);
                    }
                }
            }
            if constexpr (NF == 1) {
                // populations that arrived across a no-flux membrane become the equilibrium at
                // the wall's zero velocity, w_i phi_b, phi_b the node's own concentration:
                // in deviations, dphi_b = (sum of the arrived dg_j) / (1 - sum of missing w_i)
                if (miss[r]) {
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        if (!((a.noflux >> s) & 1)) continue;
                        float known = g[r][s][0], wm = 0.0f;
#pragma unroll
                        for (int i = 1; i < 5; ++i) {
                            if ((miss[r] >> i) & 1u) wm += Q1;
                            else known += g[r][s][i];
                        }
                        const float db = known / (1.0f - wm);
#pragma unroll
                        for (int i = 1; i < 5; ++i)
                            if ((miss[r] >> i) & 1u) g[r][s][i] = Q1 * db;
                    }
                }
            }
        }
        // the spread force: fixed point to the arithmetic type (exact in FP64)
        Rt ex = Arith<ST>::body(a.bodyx, a.bodyx_d), ey = Arith<ST>::body(a.bodyy, a.bodyy_d);
        if constexpr (NODES) {
            const int l = lds_slot(t, r);
            ex += Arith<ST>::fix((long long)accx[l]);
            ey += Arith<ST>::fix((long long)accy[l]);
        }
        const float* fr = f[r];              // converted where used (exact)
        const Moments<Rt> mo = moments<Rt>(f[r], a.rho0);
        const Rt drho = mo.drho, rho = mo.rho, ux = mo.ux, uy = mo.uy;
        const Rt usq = (Rt)1.5 * (ux * ux + uy * uy);
        const Rt om = Arith<ST>::body(a.omega, a.omega_d), om1 = (Rt)1 - om;
        const Rt w0 = Arith<ST>::c(W0, 4.0 / 9.0), w1 = Arith<ST>::c(W1, 1.0 / 9.0), w5 = Arith<ST>::c(W5, 1.0 / 36.0);
        // force term 3 w_i rho (v_i . e)
        const Rt fx = (Rt)3 * rho * ex, fy = (Rt)3 * rho * ey;
        if constexpr (MS) {
            // mass source S of the node's cell, added as S f_i^eq(1, u) (the added mass moves
            // with the fluid): the even part gains w_i S (1 + 4.5 vu^2 - 1.5 u^2), the odd part
            // w_i 3 S vu, so rho om becomes rr = rho om + S in both
            Rt sig = (Rt)0;
            if (cell[r] != ~0u) {
                const unsigned k = cell[r];
                sig = (Rt)(a.msrc + a.alpha * (a.A0[k] - a.area[k]));
                if constexpr (S > 0) {
                    if (a.gamma != 0.0) {
                        // + gamma phi_0(x), the species' concentration as its collision sees it
                        // (summed as the species' moments below)
                        const float* g0 = g[r][0];
                        const Rt dphi0 = (((Rt)g0[0] + (Rt)g0[1]) + ((Rt)g0[2] + (Rt)g0[3])) + (Rt)g0[4];
                        sig += (Rt)a.gamma * (Arith<ST>::body(a.phi_ref[0], a.phi_ref_d[0]) + dphi0);
                    }
                }
                a.cmap[(int64_t)n[r].y * a.nx + x] = ~0u;        // reset for the next step's claims
            }
            if (a.nsrc) sig += (Rt)a.nsrc[(int64_t)n[r].y * a.nx + x];
            using T = typename Pop<ST>::T;
            constexpr int P = TILE_X;
            T* __restrict__ d = row_ptr((T*)a.fdst + (int64_t)n[r].y * a.frow, chunk_col(x, 9 * TILE_X));
            const Rt rr = om * rho + sig, od0 = om * drho + sig, rs = (Rt)3 * rr, c45 = (Rt)4.5;
            store_nt(d, Pop<ST>::st((float)(om1 * fr[0] + w0 * (od0 - rr * usq)), SC9[0]));
            Rt vu, ev, od;
            vu = ux;      ev = w1 * (od0 + rr * (c45 * vu * vu - usq)); od = w1 * (rs * vu + fx);
            store_nt(d + P,     Pop<ST>::st((float)(om1 * fr[1] + ev + od), SC9[1]));
            store_nt(d + 3 * P, Pop<ST>::st((float)(om1 * fr[3] + ev - od), SC9[3]));
            vu = uy;      ev = w1 * (od0 + rr * (c45 * vu * vu - usq)); od = w1 * (rs * vu + fy);
            store_nt(d + 2 * P, Pop<ST>::st((float)(om1 * fr[2] + ev + od), SC9[2]));
            store_nt(d + 4 * P, Pop<ST>::st((float)(om1 * fr[4] + ev - od), SC9[4]));
            vu = ux + uy; ev = w5 * (od0 + rr * (c45 * vu * vu - usq)); od = w5 * (rs * vu + fx + fy);
            store_nt(d + 5 * P, Pop<ST>::st((float)(om1 * fr[5] + ev + od), SC9[5]));
            store_nt(d + 7 * P, Pop<ST>::st((float)(om1 * fr[7] + ev - od), SC9[7]));
            vu = uy - ux; ev = w5 * (od0 + rr * (c45 * vu * vu - usq)); od = w5 * (rs * vu + fy - fx);
            store_nt(d + 6 * P, Pop<ST>::st((float)(om1 * fr[6] + ev + od), SC9[6]));
            store_nt(d + 8 * P, Pop<ST>::st((float)(om1 * fr[8] + ev - od), SC9[8]));
        } else {
            // equilibrium deviation w_i (drho + rho (3 vu + 4.5 vu^2 - 1.5 u^2)), vu = v_i . u,
            // for pairs of opposite directions: the part even in v_i is shared, the odd part
            // (with the force term) changes sign
            using T = typename Pop<ST>::T;
            constexpr int P = TILE_X;
            T* __restrict__ d = row_ptr((T*)a.fdst + (int64_t)n[r].y * a.frow, chunk_col(x, 9 * TILE_X));
            const Rt rs = (Rt)3 * om * rho, c45 = (Rt)4.5;
            store_nt(d, Pop<ST>::st((float)(om1 * fr[0] + om * w0 * (drho - rho * usq)), SC9[0]));
            Rt vu, ev, od;
            vu = ux;      ev = om * w1 * (drho + rho * (c45 * vu * vu - usq)); od = w1 * (rs * vu + fx);
            store_nt(d + P,     Pop<ST>::st((float)(om1 * fr[1] + ev + od), SC9[1]));
            store_nt(d + 3 * P, Pop<ST>::st((float)(om1 * fr[3] + ev - od), SC9[3]));
            vu = uy;      ev = om * w1 * (drho + rho * (c45 * vu * vu - usq)); od = w1 * (rs * vu + fy);
            store_nt(d + 2 * P, Pop<ST>::st((float)(om1 * fr[2] + ev + od), SC9[2]));
            store_nt(d + 4 * P, Pop<ST>::st((float)(om1 * fr[4] + ev - od), SC9[4]));
            vu = ux + uy; ev = om * w5 * (drho + rho * (c45 * vu * vu - usq)); od = w5 * (rs * vu + fx + fy);
            store_nt(d + 5 * P, Pop<ST>::st((float)(om1 * fr[5] + ev + od), SC9[5]));
            store_nt(d + 7 * P, Pop<ST>::st((float)(om1 * fr[7] + ev - od), SC9[7]));
            vu = uy - ux; ev = om * w5 * (drho + rho * (c45 * vu * vu - usq)); od = w5 * (rs * vu + fy - fx);
            store_nt(d + 6 * P, Pop<ST>::st((float)(om1 * fr[6] + ev + od), SC9[6]));
            store_nt(d + 8 * P, Pop<ST>::st((float)(om1 * fr[8] + ev - od), SC9[8]));
        }

        if constexpr (MASK)
            if ((x & 31) == 0) a.inside_clr[(int64_t)(y0 + t / TILE_X + r * TILE_Y) * a.wpr + (x >> 5)] = 0u;
        if constexpr (S > 0) {
            // the species' moments and collision, in the fluid's arithmetic type
            Rt dphi[S], phi[S], rct[S];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const float* gs = g[r][s];
                dphi[s] = (((Rt)gs[0] + (Rt)gs[1]) + ((Rt)gs[2] + (Rt)gs[3])) + (Rt)gs[4];
                phi[s] = Arith<ST>::body(a.phi_ref[s], a.phi_ref_d[s]) + dphi[s];
            }
            if constexpr (NF == 2) {
                // what this collision sees, for the next step's replacement
                const int64_t k = (int64_t)n[r].y * a.nx + x;
#pragma unroll
                for (int s = 0; s < S; ++s) a.nfphi_out[(int64_t)s * a.nn + k] = (float)dphi[s];
                a.nfu_out[k] = make_float2((float)ux, (float)uy);
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const float* c = a.rc[s];
                const double* cd = a.rc_d[s];
                const Rt c0 = Arith<ST>::body(c[0], cd[0]), c1 = Arith<ST>::body(c[1], cd[1]);
                if (a.react[s] == 1) {
                    rct[s] = (m[r] != 0 ? c0 : (Rt)0) - c1 * phi[s];
                } else if (a.react[s] == 2 && S == 2) {
                    const Rt c2 = Arith<ST>::body(c[2], cd[2]);
                    const Rt u2v = phi[0] * phi[0] * phi[S - 1];
                    rct[s] = (s == 0) ? c2 * (c0 - phi[0] + u2v) : c2 * (c1 - u2v);
                } else {
                    rct[s] = (Rt)0;
                }
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const Rt os = Arith<ST>::body(a.omega_s[s], a.omega_s_d[s]), os1 = (Rt)1 - os;
                const Rt p3 = (Rt)3 * phi[s];
                const Rt q0 = Arith<ST>::c(Q0, 1.0 / 3.0), q1 = Arith<ST>::c(Q1, 1.0 / 6.0);
                const float* gg = g[r][s];
                using T = typename Pop<ST>::T;
                constexpr int P = TILE_X;
                T* __restrict__ d = row_ptr((T*)a.gdst + (int64_t)n[r].y * a.grow, chunk_col(x, a.gchunk) + 5 * s * P);
                // equilibrium deviation w_i (dphi + 3 phi v_i . u) and reaction w_i R, by pairs of
                // opposite directions (shared even part, odd part of changing sign)
                const Rt ev = q1 * (os * dphi[s] + rct[s]), ox = q1 * os * p3 * ux, oy = q1 * os * p3 * uy;
                store_nt(d,         Pop<ST>::st((float)(os1 * gg[0] + q0 * (os * dphi[s] + rct[s])), SC5[0]));
                store_nt(d + P,     Pop<ST>::st((float)(os1 * gg[1] + ev + ox), SC5[1]));
                store_nt(d + 2 * P, Pop<ST>::st((float)(os1 * gg[2] + ev + oy), SC5[2]));
                store_nt(d + 3 * P, Pop<ST>::st((float)(os1 * gg[3] + ev - ox), SC5[3]));
                store_nt(d + 4 * P, Pop<ST>::st((float)(os1 * gg[4] + ev - oy), SC5[4]));
            }
        }
    }

    // the first chunk's velocity shares, deferred past the barrier
    if constexpr (NODES) {
#pragma unroll
        for (int u = 0; u < SPREAD_UNROLL; ++u)
            if (cnd[u] != -1) a.part[share_slot(a, cnd[u])] = Ud[u];
    }
}

// Waves per SIMD the lattice pass is compiled for: the register budget that keeps the
// population loads of RP rows in flight without spilling (96 VGPRs at two rows and one species
// with FP32 arithmetic; the FP64 collision of the FP32 storage form needs 128; a budget that
// spills costs far more than a wave).
constexpr int lattice_waves(int S, int RP, int ST)
{
    return RP == 1 ? (ST == 0 ? 5 : 6) : RP == 2 ? ((S <= 1 && ST != 0) ? 5 : 4) : (ST == 0 ? 2 : 3);
}

template <int S, bool NODES, bool MASK, int ST, int NF = 0, bool MS = false, bool HF = false>
__global__ __launch_bounds__(TILE_N) __attribute__((amdgpu_waves_per_eu(lattice_waves(S, RPT, ST)))) void k_lattice(LatticeArgs a)
{
    lattice_tile<S, NODES, MASK, ST, RPT, NF, MS, HF>(a, tile_of_block((int)blockIdx.x, a.ntx, (a.ny + LTILE_Y - 1) / LTILE_Y));
}

// Batched form: every workgroup takes one (simulation, tile) work item; the simulation's
// arguments come from a device table (independent lattices of any sizes in one launch), and
// the tile height TILE_Y RP is a parameter of the launch.
template <int S, bool NODES, bool MASK, int ST, int RP>
__global__ __launch_bounds__(TILE_N) __attribute__((amdgpu_waves_per_eu(lattice_waves(S, RP, ST)))) void k_lattice_batch(const LatticeArgs* __restrict__ tab,
                                                          const int2* __restrict__ work)
{
    const int2 wk = work[blockIdx.x];
    const LatticeArgs a = tab[wk.x];
    lattice_tile<S, NODES, MASK, ST, RP>(a, wk.y);
}

// The spread force field alone (inspection): same tiling and summation as k_lattice.
__global__ __launch_bounds__(TILE_N) void k_spread_inspect(LatticeArgs a)
{
    constexpr int LY = LTILE_Y;
    const int tile = blockIdx.x;
    const int tcol = tile % a.ntx, trow = tile / a.ntx;
    const int x0 = tcol * TILE_X, y0 = trow * LY;
    const int x1 = min(x0 + TILE_X, a.nx), y1 = min(y0 + LY, a.ny);
    const int t = threadIdx.x;
    __shared__ unsigned long long accx[LDS_ROW * LY], accy[LDS_ROW * LY];
    for (int r = 0; r < RPT; ++r) {
        accx[lds_slot(t, r)] = 0ull;
        accy[lds_slot(t, r)] = 0ull;
    }
    __syncthreads();
    if (a.t_off) {
        const int lbeg = a.t_off[tile], lend = a.t_off[tile + 1];
        int cij[SPREAD_UNROLL], cnd[SPREAD_UNROLL];
        float4 crc[SPREAD_UNROLL];
        for (int k0 = lbeg; k0 < lend; k0 += SPREAD_UNROLL * TILE_N) {
            load_candidates(a, k0, lend, cij, crc, cnd);
            couple_chunk<false>(a, x0, x1, y0, y1, cij, crc, cnd, accx, accy, nullptr);
        }
    }
    __syncthreads();
    for (int r = 0; r < RPT; ++r) {
        const int x = x0 + (t % TILE_X), y = y0 + t / TILE_X + r * TILE_Y;
        if (x >= a.nx || y >= a.ny) continue;
        const int l = lds_slot(t, r);
        const int64_t o = (int64_t)y * a.nx + x;
        a.e_out[o] = (double)(__ll2float_rn((long long)accx[l]) * FIX_INV + a.bodyx);
        a.e_out[a.nn + o] = (double)(__ll2float_rn((long long)accy[l]) * FIX_INV + a.bodyy);
    }
}

// Equilibrium initial state, written in the stored (pre-streaming) layout so that the next
// pull yields f_i(x) = f_i^eq(rho(x), u(x)): s_i(x - v_i) = f_i^eq(x), or across a wall
// s_opp(i)(x) = f_i^eq(x).
struct InitArgs {
    void* f;                          // chunked arrays
    void* g;
    const double* rho;                // planar [ny][nx] inputs
    const double* u;
    const double* phi;
    int64_t nn;
    int64_t frow, grow;
    int gchunk;
    int nx, ny, walls, S;
    double rho0;
    double phi_ref[2];
    float* nfphi;                     // first-order no-flux membranes: the state's concentration
    float2* nfu;                      // deviations and velocities as the previous step's (or NULL)
};

template <int ST>
__global__ void k_init(InitArgs a)
{
    using T = typename Pop<ST>::T;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.nn) return;
    const int x = (int)(idx % a.nx), y = (int)(idx / a.nx);
    const int vx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int vy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    const double w9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    const double w5[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
    const double rho = a.rho ? a.rho[idx] : a.rho0;
    const double ux = a.u ? a.u[idx] : 0.0, uy = a.u ? a.u[a.nn + idx] : 0.0;
    const double drho = rho - a.rho0;
    const double usq = 1.5 * (ux * ux + uy * uy);
    T* f = (T*)a.f;
    for (int i = 0; i < 9; ++i) {
        const double vu = vx[i] * ux + vy[i] * uy;
        const T val = Pop<ST>::st((float)(w9[i] * (drho + rho * (3.0 * vu + 4.5 * vu * vu - usq))), SC9[i]);
        const int sy = y - vy[i];
        if (a.walls && (sy < 0 || sy >= a.ny)) {
            f[pop_at(a.frow, 9 * TILE_X, opp[i], y, x)] = val;
        } else {
            const int sx = (x - vx[i] + a.nx) % a.nx;
            const int syy = (sy + a.ny) % a.ny;
            f[pop_at(a.frow, 9 * TILE_X, i, syy, sx)] = val;
        }
    }
    if (a.nfu) a.nfu[idx] = make_float2((float)ux, (float)uy);
    for (int s = 0; s < a.S; ++s) {
        const double phi = a.phi ? a.phi[(int64_t)s * a.nn + idx] : 0.0;
        const double dphi = phi - a.phi_ref[s];
        if (a.nfphi) a.nfphi[(int64_t)s * a.nn + idx] = (float)dphi;
        T* gs = (T*)a.g;
        for (int i = 0; i < 5; ++i) {
            const double vu = vx[i] * ux + vy[i] * uy;
            const T val = Pop<ST>::st((float)(w5[i] * (dphi + 3.0 * phi * vu)), SC5[i]);
            const int sy = y - vy[i];
            if (a.walls && (sy < 0 || sy >= a.ny)) {
                gs[pop_at(a.grow, a.gchunk, 5 * s + opp[i], y, x)] = val;
            } else {
                const int sx = (x - vx[i] + a.nx) % a.nx;
                const int syy = (sy + a.ny) % a.ny;
                gs[pop_at(a.grow, a.gchunk, 5 * s + i, syy, sx)] = val;
            }
        }
    }
}

// Moments of the current state in FP64: planes rho, ux, uy, phi_0 .. phi_{S-1}.
struct MomentArgs {
    const void* f;                    // chunked arrays
    const void* g;
    double* out;                      // planar outputs
    int64_t nn;
    int64_t frow, grow;
    int gchunk;
    int nx, ny, walls, S;
    double rho0;
    double phi_ref[2];
    const unsigned* inside;           // inside-cell map of the current positions (no-flux membranes)
    int wpr;
    int noflux;                       // bit s: no-flux membranes for species s
    int pring;                        // the outer ring is held at rho0 (pressure boundary)
    const uint8_t* pmap;              // pressure points held at rho0 (NULL: none)
    int nf_bb;                        // the no-flux form over cut links, as in LatticeArgs
    // no-flux membranes in the first-order form (nfq NULL: the zeroth-order form): the buffers
    // the next lattice pass reads
    const float* nfq;
    const uint8_t* nfm;
    const float* nfphi;
    const float2* nfu;
};

template <int ST>
__device__ inline void node_moments(const MomentArgs& a, int x, int y, double& drho, double& jx,
                                    double& jy, double dphi[2])
{
    const Nbr n = neighbours(x, y, a.nx, a.ny, a.walls);
    float f[9];
    pull9<ST>(a.f, a.frow, n, f);
    drho = 0.0;
    for (int i = 0; i < 9; ++i) drho += (double)f[i];
    jx = ((double)f[1] - f[3]) + ((double)f[5] - f[6]) + ((double)f[8] - f[7]);
    jy = ((double)f[2] - f[4]) + ((double)f[5] + f[6]) - ((double)f[7] + f[8]);
    if ((a.pring && (x == 0 || x == a.nx - 1 || y == 0 || y == a.ny - 1)) || (a.pmap && a.pmap[(int64_t)y * a.nx + x])) {
        // the density the next collision sees at a pressure point: rho0, momentum rescaled
        const double gm = a.rho0 / (a.rho0 + drho);
        jx *= gm;
        jy *= gm;
        drho = 0.0;
    }
    unsigned miss = 0u;
    if (a.noflux && a.nfq) {
        miss = a.nfm[(int64_t)y * a.nx + x];
    } else if (a.noflux) {
        // populations that arrived across a no-flux membrane (as in the lattice pass)
        auto bit = [&](int xx, int yy) { return (a.inside[(int64_t)yy * a.wpr + (xx >> 5)] >> (xx & 31)) & 1u; };
        const unsigned me = bit(n.x, n.y);
        if (bit(n.xm, n.y) != me) miss |= 2u;
        if (!n.bot && bit(n.x, n.ym) != me) miss |= 4u;
        if (bit(n.xp, n.y) != me) miss |= 8u;
        if (!n.top && bit(n.x, n.yp) != me) miss |= 16u;
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {          // constant indices: dphi stays in registers
        if (s >= a.S) break;
        float g[5];
        pull5<ST>((const typename Pop<ST>::T*)a.g + 5 * s * TILE_X, a.grow, a.gchunk, n, g);
        if (miss && ((a.noflux >> s) & 1) && a.nfq) {
            // the concentration the next collision sees: the populations over cut links replaced
            if (a.nf_bb) nf_bounce<ST>(a, a.g, s, x, y, miss, g);
            else nf_first_replace(a, s, x, y, miss, g);
            double t = 0.0;
            for (int i = 0; i < 5; ++i) t += (double)g[i];
            dphi[s] = t;
            continue;
        }
        if (miss && ((a.noflux >> s) & 1)) {
            // the concentration the next collision sees: the missing populations become
            // w_i phi_b, so the sum is (sum of the arrived ones) / (1 - sum of the missing w_i)
            double known = (double)g[0], wm = 0.0;
            for (int i = 1; i < 5; ++i) {
                if ((miss >> i) & 1u) wm += 1.0 / 6.0;
                else known += (double)g[i];
            }
            dphi[s] = known / (1.0 - wm);
            continue;
        }
        double t = 0.0;
        for (int i = 0; i < 5; ++i) t += (double)g[i];
        dphi[s] = t;
    }
}

template <int ST>
__global__ void k_moments(MomentArgs a)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.nn) return;
    const int x = (int)(idx % a.nx), y = (int)(idx / a.nx);
    double drho, jx, jy, dphi[2] = {0.0, 0.0};
    node_moments<ST>(a, x, y, drho, jx, jy, dphi);
    const double rho = a.rho0 + drho;
    a.out[idx] = rho;
    a.out[a.nn + idx] = jx / rho;
    a.out[2 * a.nn + idx] = jy / rho;
    for (int s = 0; s < a.S; ++s) a.out[(3 + s) * a.nn + idx] = a.phi_ref[s] + dphi[s];
}

// Deterministic FP64 sums: fixed node-to-thread assignment, fixed LDS tree, then one block
// adds the per-block partials in order.
constexpr int RED_THREADS = 256;
constexpr int RED_MAXV = 5;

// Work items are 64-column segments of one lattice row, one wavefront per item (coalesced
// rows, no per-node index division); a wavefront takes items w, w + W, w + 2W, ... (W the
// wavefronts of the grid), four at a time so that their loads are in flight together.
template <int ST>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_partial(MomentArgs a, double* partial)
{
    __shared__ double sh[RED_MAXV][RED_THREADS];
    constexpr int U = 4;
    const int nv = 3 + a.S;
    double acc[RED_MAXV] = {0, 0, 0, 0, 0};
    const int ncx = (a.nx + 63) / 64;
    const int items = a.ny * ncx;
    const int lane = threadIdx.x & 63;
    const int wstride = (int)gridDim.x * (RED_THREADS / 64);
    const int w0 = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (RED_THREADS / 64) + (int)(threadIdx.x >> 6));
    for (int it0 = w0; it0 < items; it0 += U * wstride) {
        double v[U][RED_MAXV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int k = 0; k < RED_MAXV; ++k) v[u][k] = 0.0;
            const int it = it0 + u * wstride;
            if (it < items) {
                const int y = it / ncx, x = (it - y * ncx) * 64 + lane;
                if (x < a.nx) node_moments<ST>(a, x, y, v[u][0], v[u][1], v[u][2], &v[u][3]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < RED_MAXV; ++k) acc[k] += v[u][k];
    }
    for (int v = 0; v < nv; ++v) sh[v][threadIdx.x] = acc[v];
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int v = 0; v < nv; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int v = 0; v < nv; ++v) partial[(int64_t)blockIdx.x * RED_MAXV + v] = sh[v][0];
}

// Final stage, one workgroup: thread t adds the partials of blocks t, t + RED_THREADS, ... in
// that order, then a fixed LDS tree adds the threads' sums; the order depends on nblocks only,
// so the result is the same from run to run.
// With the monitor (count non-NULL) the workgroup also counts the sums taken (count[0] += 1,
// out = count + 1) and flags a sum that is not finite in err.
__global__ __launch_bounds__(RED_THREADS) void k_reduce_final(const double* partial, int nblocks, int nv,
                                                              double rho_total, double phi_tot0, double phi_tot1,
                                                              double* out, double* count, int* err)
{
    __shared__ double sh[RED_MAXV][RED_THREADS];
    double acc[RED_MAXV] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += RED_THREADS)
        for (int v = 0; v < nv; ++v) acc[v] += partial[(int64_t)b * RED_MAXV + v];
    for (int v = 0; v < nv; ++v) sh[v][threadIdx.x] = acc[v];
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int v = 0; v < nv; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double v[RED_MAXV] = {rho_total + sh[0][0], sh[1][0], sh[2][0], phi_tot0 + sh[3][0], phi_tot1 + sh[4][0]};
        bool finite = true;
        for (int k = 0; k < nv; ++k) {
            out[k] = v[k];
            finite = finite && isfinite(v[k]);
        }
        if (count) count[0] += 1.0;
        if (err && !finite) atomicOr(err, ERR_FIELDS);
    }
}

// The context's error flags copied to host-visible memory (pinned, mapped), which lbib_step
// reads without synchronising.
__global__ void k_err_mirror(const int* err, int* host)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int v = __atomic_load_n(err, __ATOMIC_RELAXED);
        __hip_atomic_store(host, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

hipError_t launch_err_mirror(lbib_ctx* c, int* host_dev)
{
    hipLaunchKernelGGL(k_err_mirror, dim3(1), dim3(64), 0, c->stream, (const int*)c->d_err, host_dev);
    return hipGetLastError();
}

// Block partials of the sums for the entry point that allocates nothing: a file-scope array
// each GPU holds once for the life of the process (REDUCE_SCRATCH_BLOCKS partials of RED_MAXV
// doubles, 160 KiB).  Host code names it only through the device address that
// hipGetSymbolAddress returns for the current device (reduce_scratch_ptr).
constexpr int REDUCE_SCRATCH_BLOCKS = 4096;
static __device__ __align__(256) double scratch[REDUCE_SCRATCH_BLOCKS * RED_MAXV];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_dev[SCRATCH_MAX_DEVICES] = {};
}  // namespace

hipError_t reduce_scratch_init(int device)
{
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_dev[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_dev[device] = (double*)ptr;
    return hipSuccess;
}

double* reduce_scratch_ptr(int device)
{
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    return scratch_dev[device];
}

int reduce_scratch_blocks() { return REDUCE_SCRATCH_BLOCKS; }

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
// Forms of the lattice pass: NF (no-flux membranes: 0 none, 1 zeroth-order form reading the
// inside bits, 2 the first-order form), MS (mass sources or the pressure ring), HF (the nodes
// move with the half-force-shifted velocity); the plain form carries none of their code.
template <int S, int ST, int NF, bool MS>
static hipError_t launch_form(lbib_ctx* c, const LatticeArgs& a, bool nodes, bool mask, bool hf)
{
    dim3 grid((unsigned)c->nltiles), block(TILE_N);
    constexpr bool MASK_ONLY = NF == 1 || MS;        // these forms read the inside bits or the cell map
#define LL(N, M, H) hipLaunchKernelGGL((k_lattice<S, N, M, ST, NF, MS, H>), grid, block, 0, c->stream, a)
    if (nodes) {
        if (hf) {
            if (mask || MASK_ONLY) LL(true, true, true);
            else LL(true, false, true);
        } else {
            if (mask || MASK_ONLY) LL(true, true, false);
            else LL(true, false, false);
        }
    } else if constexpr (NF == 0) {
        if (mask || MASK_ONLY) LL(false, true, false);
        else LL(false, false, false);
    }
#undef LL
    return hipGetLastError();
}

template <int S, int ST>
static hipError_t launch_lattice_s(lbib_ctx* c, const LatticeArgs& a, bool nodes, bool mask)
{
    const bool hf = c->p.interp_half_force != 0;
    // mass sources (the cell map), node sources, the pressure ring or pressure points
    const bool ms = (a.cmap && nodes) || a.pring || a.nsrc || a.pmap;
    if constexpr (S > 0) {
        if (a.noflux && nodes) {
            if (a.nfq) return ms ? launch_form<S, ST, 2, true>(c, a, nodes, mask, hf)
                                 : launch_form<S, ST, 2, false>(c, a, nodes, mask, hf);
            return ms ? launch_form<S, ST, 1, true>(c, a, nodes, mask, hf) : launch_form<S, ST, 1, false>(c, a, nodes, mask, hf);
        }
    }
    return ms ? launch_form<S, ST, 0, true>(c, a, nodes, mask, hf) : launch_form<S, ST, 0, false>(c, a, nodes, mask, hf);
}

template <int ST>
static hipError_t launch_lattice_st(lbib_ctx* c, const LatticeArgs& a, bool nodes, bool mask)
{
    switch (c->S) {
    case 0: return launch_lattice_s<0, ST>(c, a, nodes, mask);
    case 1: return launch_lattice_s<1, ST>(c, a, nodes, mask);
    default: return launch_lattice_s<2, ST>(c, a, nodes, mask);
    }
}

hipError_t launch_lattice(lbib_ctx* c, const LatticeArgs& a, bool nodes, bool mask)
{
    switch (c->p.storage) {
    case LBIB_STORAGE_FP16: return launch_lattice_st<1>(c, a, nodes, mask);
    case LBIB_STORAGE_BF16: return launch_lattice_st<2>(c, a, nodes, mask);
    default: return launch_lattice_st<0>(c, a, nodes, mask);
    }
}

template <int S, int ST, int RP>
static hipError_t launch_lattice_batch_r(const LatticeArgs* tab, const int2* work, int nwork, bool mask,
                                         hipStream_t stream)
{
    dim3 grid((unsigned)nwork), block(TILE_N);
    if (mask) hipLaunchKernelGGL((k_lattice_batch<S, true, true, ST, RP>), grid, block, 0, stream, tab, work);
    else hipLaunchKernelGGL((k_lattice_batch<S, true, false, ST, RP>), grid, block, 0, stream, tab, work);
    return hipGetLastError();
}

template <int S, int ST>
static hipError_t launch_lattice_batch_s(const LatticeArgs* tab, const int2* work, int nwork, int rows, bool mask,
                                         hipStream_t stream)
{
    if (rows == 1) return launch_lattice_batch_r<S, ST, 1>(tab, work, nwork, mask, stream);
    if (rows == 4) return launch_lattice_batch_r<S, ST, 4>(tab, work, nwork, mask, stream);
    return launch_lattice_batch_r<S, ST, 2>(tab, work, nwork, mask, stream);
}

hipError_t launch_lattice_batch(const LatticeArgs* tab, const int2* work, int nwork, int S, int storage, int rows,
                                bool mask, hipStream_t stream)
{
    if (nwork <= 0) return hipSuccess;
#define LB(SS, TT) return launch_lattice_batch_s<SS, TT>(tab, work, nwork, rows, mask, stream)
    if (storage == LBIB_STORAGE_FP16) {
        if (S == 0) LB(0, 1);
        if (S == 1) LB(1, 1);
        LB(2, 1);
    }
    if (storage == LBIB_STORAGE_BF16) {
        if (S == 0) LB(0, 2);
        if (S == 1) LB(1, 2);
        LB(2, 2);
    }
    if (S == 0) LB(0, 0);
    if (S == 1) LB(1, 0);
    LB(2, 0);
#undef LB
}

hipError_t launch_spread_inspect(lbib_ctx* c, const LatticeArgs& a)
{
    hipLaunchKernelGGL(k_spread_inspect, dim3((unsigned)c->nltiles), dim3(TILE_N), 0, c->stream, a);
    return hipGetLastError();
}

hipError_t launch_init(lbib_ctx* c, const double* rho, const double* u, const double* phi, int has_rho,
                       int has_u, int has_phi)
{
    InitArgs a;
    a.f = c->f[c->cur];
    a.g = c->g[c->cur];
    a.rho = has_rho ? rho : nullptr;
    a.u = has_u ? u : nullptr;
    a.phi = has_phi ? phi : nullptr;
    a.nn = c->nn;
    a.frow = c->frow();
    a.grow = c->grow();
    a.gchunk = c->gchunk();
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.walls = c->p.bc_y == LBIB_WALLS;
    a.S = c->S;
    a.rho0 = c->p.rho0;
    a.phi_ref[0] = c->p.species[0].phi_ref;
    a.phi_ref[1] = c->p.species[1].phi_ref;
    a.nfphi = c->nfphi[c->cur];
    a.nfu = c->nfu[c->cur];
    const unsigned nb = (unsigned)((c->nn + 255) / 256);
    switch (c->p.storage) {
    case LBIB_STORAGE_FP16: hipLaunchKernelGGL(k_init<1>, dim3(nb), dim3(256), 0, c->stream, a); break;
    case LBIB_STORAGE_BF16: hipLaunchKernelGGL(k_init<2>, dim3(nb), dim3(256), 0, c->stream, a); break;
    default: hipLaunchKernelGGL(k_init<0>, dim3(nb), dim3(256), 0, c->stream, a); break;
    }
    return hipGetLastError();
}

static MomentArgs moment_args(lbib_ctx* c, double* out)
{
    MomentArgs a;
    a.f = c->f[c->cur];
    a.g = c->g[c->cur];
    a.out = out;
    a.nn = c->nn;
    a.frow = c->frow();
    a.grow = c->grow();
    a.gchunk = c->gchunk();
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.walls = c->p.bc_y == LBIB_WALLS;
    a.S = c->S;
    a.rho0 = c->p.rho0;
    a.phi_ref[0] = c->p.species[0].phi_ref;
    a.phi_ref[1] = c->p.species[1].phi_ref;
    a.inside = c->inside[c->cur];
    a.wpr = c->wpr;
    a.noflux = c->n_cells ? no_flux_bits(c->p) : 0;
    a.pring = c->p.pressure_ring;
    a.pmap = c->d_pmap;
    const bool nf1 = a.noflux && c->nfq[0];
    a.nfq = nf1 ? c->nfq[c->cur] : nullptr;
    a.nfm = nf1 ? c->nfm[c->cur] : nullptr;
    a.nfphi = nf1 ? c->nfphi[c->cur] : nullptr;
    a.nfu = nf1 ? c->nfu[c->cur] : nullptr;
    a.nf_bb = nf1 && c->p.no_flux_bounce ? (c->nf_fresh ? 2 : 1) : 0;
    return a;
}

hipError_t launch_moments(lbib_ctx* c, double* out)
{
    MomentArgs a = moment_args(c, out);
    const unsigned nb = (unsigned)((c->nn + 255) / 256);
    switch (c->p.storage) {
    case LBIB_STORAGE_FP16: hipLaunchKernelGGL(k_moments<1>, dim3(nb), dim3(256), 0, c->stream, a); break;
    case LBIB_STORAGE_BF16: hipLaunchKernelGGL(k_moments<2>, dim3(nb), dim3(256), 0, c->stream, a); break;
    default: hipLaunchKernelGGL(k_moments<0>, dim3(nb), dim3(256), 0, c->stream, a); break;
    }
    return hipGetLastError();
}

// blocks of the partial stage for a lattice of nn nodes: 16 nodes per thread, at most
// REDUCE_SCRATCH_BLOCKS (a grid-stride loop covers the rest)
int reduce_blocks(int64_t nn)
{
    int64_t nb = (nn + RED_THREADS * 16 - 1) / (RED_THREADS * 16);
    if (nb > REDUCE_SCRATCH_BLOCKS) nb = REDUCE_SCRATCH_BLOCKS;
    return nb < 1 ? 1 : (int)nb;
}

hipError_t launch_reduce(lbib_ctx* c, double* partial, double* out_dev, double* count, int* err)
{
    MomentArgs a = moment_args(c, nullptr);
    const int nblocks = reduce_blocks(c->nn);
    switch (c->p.storage) {
    case LBIB_STORAGE_FP16:
        hipLaunchKernelGGL(k_reduce_partial<1>, dim3(nblocks), dim3(RED_THREADS), 0, c->stream, a, partial);
        break;
    case LBIB_STORAGE_BF16:
        hipLaunchKernelGGL(k_reduce_partial<2>, dim3(nblocks), dim3(RED_THREADS), 0, c->stream, a, partial);
        break;
    default:
        hipLaunchKernelGGL(k_reduce_partial<0>, dim3(nblocks), dim3(RED_THREADS), 0, c->stream, a, partial);
        break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double rho_total = c->p.rho0 * (double)c->nn;
    const double p0 = c->p.species[0].phi_ref * (double)c->nn;
    const double p1 = c->p.species[1].phi_ref * (double)c->nn;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, c->stream, (const double*)partial, nblocks,
                       3 + c->S, rho_total, p0, p1, out_dev, count, err);
    return hipGetLastError();
}

}  // namespace lbib
