// Membrane kernels of the coupled step (gfx950).
//
// k_membrane: one workgroup per cell.  In a time step it
//   1. interpolates u^n to each node over the 4x4 stencil (Eq. conversion2 with the kernel
//      of Eq. 1Dkernel) and moves the node explicitly, X^{n+1} = X^n + U (positions in FP64);
//   2. stages the cell's new positions in LDS and reduces the polygon area (shoelace, FP64,
//      fixed-order wave and LDS reduction);
//   3. evaluates the nodal forces in the paper's per-node form: constant tension
//      (Eq. membraneforce), Hookean springs, area pressure kappa (A0 - A) dA/dX, and
//      refreshes the node's spreading record (fractional offset, force, stencil origin) in
//      its bin slot; a node that drifted beyond its bin margin raises an error flag;
//   4. when a reaction reads them, rasterises the cell's domain IDs from the LDS positions.
// k_bin_count / k_bin_scan / k_bin_scatter rebuild the bins (every few steps).
#include "lbib_internal.h"
#include "lbib_raster.h"

namespace lbib {

__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// has the stencil origin (i0, j0) moved at most BIN_MARGIN from its value at the last
// rebinning (packed in ijb)?  Then it is still inside its bin's widened tile.
__device__ inline bool within_margin(int i0, int j0, int ijb, int nx, int ny, int walls)
{
    const int ib = ijb & 0xFFFF, jb = ijb >> 16;
    int di = i0 - ib;
    if (di > nx / 2) di -= nx;
    else if (di < -(nx / 2)) di += nx;
    if (di > BIN_MARGIN || di < -BIN_MARGIN) return false;
    int dj;
    if (walls) {
        const int jr = j0 < 0 ? 0 : (j0 >= ny ? ny - 1 : j0);
        const int jbr = jb < 0 ? 0 : (jb >= ny ? ny - 1 : jb);
        dj = jr - jbr;
    } else {
        dj = j0 - jb;
        if (dj > ny / 2) dj -= ny;
        else if (dj < -(ny / 2)) dj += ny;
    }
    return dj <= BIN_MARGIN && dj >= -BIN_MARGIN;
}

constexpr int MEM_UNROLL = 2;     // nodes per thread whose loads are issued together

__global__ __launch_bounds__(MEMBRANE_THREADS) void k_membrane(MembraneArgs a)
{
    extern __shared__ double2 xs[];
    __shared__ double red[16];
    __shared__ unsigned bm[RASTER_WORDS_FUSED];
    const int c = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int beg = a.off[c];
    const int n = a.off[c + 1] - beg;

    // 1. move: X^{n+1} = X^n + U, U interpolated by the lattice pass (fixed point, cleared here)
    for (int base = 0; base < n; base += MEM_UNROLL * MEMBRANE_THREADS) {
        double2 X[MEM_UNROLL];
        unsigned long long ux[MEM_UNROLL], uy[MEM_UNROLL];
#pragma unroll
        for (int u = 0; u < MEM_UNROLL; ++u) {
            const int k = base + u * MEMBRANE_THREADS + t;
            if (k >= n) continue;
            X[u] = a.X[beg + k];
            if (a.advect) {
                ux[u] = a.U_acc[2 * (int64_t)(beg + k)];
                uy[u] = a.U_acc[2 * (int64_t)(beg + k) + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < MEM_UNROLL; ++u) {
            const int k = base + u * MEMBRANE_THREADS + t;
            if (k >= n) continue;
            if (a.advect) {
                a.U_acc[2 * (int64_t)(beg + k)] = 0ull;
                a.U_acc[2 * (int64_t)(beg + k) + 1] = 0ull;
                if (finite2(X[u].x, X[u].y)) {
                    X[u].x += (double)(long long)ux[u] * UFIX_INV;
                    X[u].y += (double)(long long)uy[u] * UFIX_INV;
                    a.X[beg + k] = X[u];
                }
            }
            xs[k] = X[u];
        }
    }
    __syncthreads();

    // 2. shoelace area about the first node (translation invariant, less cancellation)
    const double ox = xs[0].x, oy = xs[0].y;
    double part = 0.0;
    for (int k = t; k < n; k += MEMBRANE_THREADS) {
        const int kn = (k + 1 == n) ? 0 : k + 1;
        part += (xs[k].x - ox) * (xs[kn].y - oy) - (xs[kn].x - ox) * (xs[k].y - oy);
    }
    part = wave_sum(part);
    if (lane == 0) red[wid] = part;
    __syncthreads();
    double A2 = 0.0;
    for (int w = 0; w < MEMBRANE_THREADS / 64; ++w) A2 += red[w];
    const double A = 0.5 * A2;
    if (t == 0) a.area[c] = A;
    const double s_area = a.kappa * (a.A0[c] - A);

    // 3. forces and spreading records
    int flags = 0;
    for (int base = 0; base < n; base += MEM_UNROLL * MEMBRANE_THREADS) {
        double lp[MEM_UNROLL], lm[MEM_UNROLL];
        int sl[MEM_UNROLL], ky[MEM_UNROLL];
#pragma unroll
        for (int u = 0; u < MEM_UNROLL; ++u) {
            const int k = base + u * MEMBRANE_THREADS + t;
            if (k >= n) continue;
            const int km = (k == 0) ? n - 1 : k - 1;
            lp[u] = a.l0[beg + k];
            lm[u] = a.l0[beg + km];
            sl[u] = a.slot[beg + k];
            ky[u] = a.ij_bin[beg + k];
        }
#pragma unroll
        for (int u = 0; u < MEM_UNROLL; ++u) {
            const int k = base + u * MEMBRANE_THREADS + t;
            if (k >= n) continue;
            const int kp = (k + 1 == n) ? 0 : k + 1;
            const int km = (k == 0) ? n - 1 : k - 1;
            const double2 X = xs[k], Xp = xs[kp], Xm = xs[km];
            const double dpx = Xp.x - X.x, dpy = Xp.y - X.y;
            const double dmx = Xm.x - X.x, dmy = Xm.y - X.y;
            const double Lp = sqrt(dpx * dpx + dpy * dpy), Lm = sqrt(dmx * dmx + dmy * dmy);
            // tension phi_m along both edges; springs k (L - l0) along each edge
            const double sp = (a.phi_m + a.k_spring * (Lp - lp[u])) / Lp;
            const double sm = (a.phi_m + a.k_spring * (Lm - lm[u])) / Lm;
            double Fx = sp * dpx + sm * dmx;
            double Fy = sp * dpy + sm * dmy;
            // area pressure: dA/dX_k = ((y_{k+1} - y_{k-1}) / 2, (x_{k-1} - x_{k+1}) / 2)
            Fx += s_area * 0.5 * (Xp.y - Xm.y);
            Fy += s_area * 0.5 * (Xm.x - Xp.x);
            const int s = sl[u];
            if (finite2(X.x, X.y) && finite2(Fx, Fy)) {
                const double fx = floor(X.x), fy = floor(X.y);
                int i0, j0;
                stencil_origin(X.x, X.y, a.nx, a.ny, a.walls, i0, j0);
                a.rec[s] = make_float4((float)(X.x - fx), (float)(X.y - fy), (float)Fx, (float)Fy);
                a.rec_ij[s] = pack_ij(i0, j0);
                if (!within_margin(i0, j0, ky[u], a.nx, a.ny, a.walls)) flags |= ERR_MARGIN;
            } else {
                a.rec[s] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                a.rec_ij[s] = 0;
                flags |= ERR_NONFINITE;
            }
        }
    }
    if (flags) atomicOr(a.err, flags);

    // 4. domain IDs of the new positions
    if (a.raster) raster_cell(xs, n, (uint16_t)(c + 1), a.mask, a.nx, a.ny, a.walls, bm, RASTER_WORDS_FUSED, red);
}

// ---------------------------------------------------------------------------------------
// rebinning
// ---------------------------------------------------------------------------------------

// bin of every node; a wavefront issues one counter increment per distinct bin among its
// lanes (consecutive nodes of a membrane mostly share a tile) and hands out ranks within it
__global__ void k_bin_count(BinArgs a)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = l < a.n;
    int key = -1;
    if (live) {
        const double2 X = a.X[l];
        key = 0;
        int ij = 0;
        if (finite2(X.x, X.y)) {
            int i0, j0;
            stencil_origin(X.x, X.y, a.nx, a.ny, a.walls, i0, j0);
            key = bin_of(i0, j0, a.ny, a.ntx);
            ij = pack_ij(i0, j0);
        }
        a.ij_bin[l] = ij;
    }
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned long long todo = __ballot(live);
    int rank = 0;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lkey = __shfl(key, leader, 64);
        const unsigned long long grp = __ballot(live && key == lkey);
        int base = 0;
        if (lane == leader) base = atomicAdd(&a.count[lkey], __popcll(grp));
        base = __shfl(base, leader, 64);
        if (live && key == lkey) rank = base + __popcll(grp & below);
        todo &= ~grp;
    }
    if (live) {
        a.key[l] = key;
        a.rank[l] = rank;
    }
}

// exclusive scan of the bin counts into offsets; counts are cleared for the next rebinning
__global__ __launch_bounds__(SCAN_THREADS) void k_bin_scan(BinArgs a)
{
    constexpr int CHUNK = SCAN_THREADS * SCAN_PER_THREAD;
    __shared__ int buf[CHUNK];
    __shared__ int wsum[SCAN_THREADS / 64];
    __shared__ int carry_sh;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    if (t == 0) carry_sh = 0;
    for (int base = 0; base < a.nbins; base += CHUNK) {
        for (int i = t; i < CHUNK; i += SCAN_THREADS) {
            const int b = base + i;
            int v = 0;
            if (b < a.nbins) {
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
            if (b < a.nbins) a.off[b] = buf[i];
        }
        if (t == SCAN_THREADS - 1) carry_sh = run;
        __syncthreads();
    }
    if (t == 0) a.off[a.nbins] = carry_sh;
}

// new slot of every node; its record moves there from the old slot when copy is set
__global__ void k_bin_scatter(BinArgs a)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.n) return;
    const int s = a.off[a.key[l]] + a.rank[l];
    a.rec_node[s] = (int)l;
    if (a.copy) {
        const int o = a.slot[l];
        a.rec_new[s] = a.rec_old[o];
        a.ij_new[s] = a.ij_old[o];
    }
    a.slot[l] = s;
}

// forces of every node, read back from the records (inspection)
__global__ void k_forces_out(const int* __restrict__ slot, const float4* __restrict__ rec, float2* __restrict__ F,
                             int64_t n)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const float4 r = rec[slot[l]];
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
    hipLaunchKernelGGL(k_membrane, dim3((unsigned)c->n_cells), dim3(MEMBRANE_THREADS), lds, c->stream, a);
    return hipGetLastError();
}

hipError_t launch_rebin(lbib_ctx* c, const BinArgs& a, int which)
{
    const unsigned nb = (unsigned)((a.n + 255) / 256);
    if (which == 0) hipLaunchKernelGGL(k_bin_count, dim3(nb), dim3(256), 0, c->stream, a);
    else if (which == 1) hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(SCAN_THREADS), 0, c->stream, a);
    else hipLaunchKernelGGL(k_bin_scatter, dim3(nb), dim3(256), 0, c->stream, a);
    return hipGetLastError();
}

hipError_t launch_forces_out(lbib_ctx* c, float2* F)
{
    const unsigned nb = (unsigned)((c->n_nodes + 255) / 256);
    hipLaunchKernelGGL(k_forces_out, dim3(nb), dim3(256), 0, c->stream, (const int*)c->d_slot,
                       (const float4*)c->d_rec[c->rec_cur], F, c->n_nodes);
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
