// Membrane kernels of the coupled step (gfx950).
//
// k_membrane: one workgroup per cell.  In a time step it
//   1. interpolates u^n to each node over the 4x4 stencil (Eq. conversion2 with the kernel
//      of Eq. 1Dkernel) and moves the node explicitly, X^{n+1} = X^n + U (positions in FP64);
//   2. stages the cell's new positions in LDS and reduces the polygon area (shoelace, FP64,
//      fixed-order tree);
//   3. evaluates the nodal forces in the paper's per-node form: constant tension
//      (Eq. membraneforce), Hookean springs, area pressure kappa (A0 - A) dA/dX;
//   4. files the node under the lattice tile of its stencil origin for the next spreading.
// k_bin_scan / k_bin_scatter turn the per-tile counts into a CSR of node records.
#include "lbib_internal.h"

namespace lbib {

__device__ inline float2 interp_u(const MembraneArgs& a, double X, double Y)
{
    const double fx = floor(X), fy = floor(Y);
    float wx[4], wy[4];
    delta_weights(a.kernel, (float)(X - fx), wx);
    delta_weights(a.kernel, (float)(Y - fy), wy);
    const int i0 = wrap_ll((long long)fx - 1, a.nx);
    const long long j0 = (long long)fy - 1;
    float ux = 0.0f, uy = 0.0f;
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
        int j;
        if (a.walls) {
            const long long jj = j0 + bb;
            if (jj < 0 || jj >= a.ny) continue;
            j = (int)jj;
        } else {
            j = wrap_ll(j0 + bb, a.ny);
        }
        const float* row = a.uband + (int64_t)j * a.nx;
        float sx = 0.0f, sy = 0.0f;
#pragma unroll
        for (int aa = 0; aa < 4; ++aa) {
            int i = i0 + aa;
            if (i >= a.nx) i -= a.nx;
            sx += wx[aa] * row[i];
            sy += wx[aa] * row[a.nn + i];
        }
        ux += wy[bb] * sx;
        uy += wy[bb] * sy;
    }
    return make_float2(ux, uy);
}

// finite and small enough for the integer stencil arithmetic (|coordinate| < 2^40)
__device__ inline bool finite2(double x, double y)
{
    return fabs(x) < 1099511627776.0 && fabs(y) < 1099511627776.0;
}

__global__ __launch_bounds__(MEMBRANE_THREADS) void k_membrane(MembraneArgs a)
{
    extern __shared__ double2 xs[];
    __shared__ double red[MEMBRANE_THREADS];
    const int c = blockIdx.x;
    const int t = threadIdx.x;
    const int beg = a.off[c];
    const int n = a.off[c + 1] - beg;

    for (int k = t; k < n; k += MEMBRANE_THREADS) {
        double2 X = a.X[beg + k];
        if (a.advect) {
            if (finite2(X.x, X.y)) {
                const float2 U = interp_u(a, X.x, X.y);
                X.x += (double)U.x;
                X.y += (double)U.y;
                a.X[beg + k] = X;
            }
        }
        xs[k] = X;
    }
    __syncthreads();

    // shoelace area about the first node (translation invariant, less cancellation)
    const double ox = xs[0].x, oy = xs[0].y;
    double part = 0.0;
    for (int k = t; k < n; k += MEMBRANE_THREADS) {
        const int kn = (k + 1 == n) ? 0 : k + 1;
        part += (xs[k].x - ox) * (xs[kn].y - oy) - (xs[kn].x - ox) * (xs[k].y - oy);
    }
    red[t] = part;
    __syncthreads();
    for (int w = MEMBRANE_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const double A = 0.5 * red[0];
    if (t == 0) a.area[c] = A;
    const double s_area = a.kappa * (a.A0[c] - A);

    for (int k = t; k < n; k += MEMBRANE_THREADS) {
        const int kp = (k + 1 == n) ? 0 : k + 1;
        const int km = (k == 0) ? n - 1 : k - 1;
        const double2 X = xs[k], Xp = xs[kp], Xm = xs[km];
        const double dpx = Xp.x - X.x, dpy = Xp.y - X.y;
        const double dmx = Xm.x - X.x, dmy = Xm.y - X.y;
        const double Lp = sqrt(dpx * dpx + dpy * dpy), Lm = sqrt(dmx * dmx + dmy * dmy);
        // unit vectors towards the successor and the predecessor
        const double tpx = dpx / Lp, tpy = dpy / Lp, tmx = dmx / Lm, tmy = dmy / Lm;
        // tension phi_m along both edges; springs k (L - l0) along each edge
        const double sp = a.phi_m + a.k_spring * (Lp - a.l0[beg + k]);
        const double sm = a.phi_m + a.k_spring * (Lm - a.l0[beg + km]);
        double Fx = sp * tpx + sm * tmx;
        double Fy = sp * tpy + sm * tmy;
        // area pressure: dA/dX_k = ((y_{k+1} - y_{k-1}) / 2, (x_{k-1} - x_{k+1}) / 2)
        Fx += s_area * 0.5 * (Xp.y - Xm.y);
        Fy += s_area * 0.5 * (Xm.x - Xp.x);
        const int node = beg + k;
        int key = 0;
        if (finite2(X.x, X.y) && finite2(Fx, Fy)) {
            a.F[node] = make_float2((float)Fx, (float)Fy);
            key = bin_key(X.x, X.y, a.nx, a.ny, a.walls, a.ntx);
        } else {
            a.F[node] = make_float2(0.0f, 0.0f);
            atomicOr(a.err, 1);
        }
        a.key[node] = key;
        a.rank[node] = atomicAdd(&a.bin_count[key], 1);
    }
}

// Exclusive scan of the per-tile counts into CSR offsets (one workgroup; runs of
// SCAN_THREADS * 4 counts per pass with a running carry).
__global__ __launch_bounds__(SCAN_THREADS) void k_bin_scan(const int* __restrict__ count, int* __restrict__ off,
                                                           int nbins)
{
    __shared__ int sh[SCAN_THREADS];
    __shared__ int carry_sh;
    const int t = threadIdx.x;
    if (t == 0) carry_sh = 0;
    __syncthreads();
    for (int base = 0; base < nbins; base += SCAN_THREADS * 4) {
        int v[4], s = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = base + t * 4 + q;
            v[q] = (i < nbins) ? count[i] : 0;
            s += v[q];
        }
        sh[t] = s;
        __syncthreads();
        // Hillis-Steele inclusive scan of the per-thread sums
        for (int d = 1; d < SCAN_THREADS; d <<= 1) {
            const int add = (t >= d) ? sh[t - d] : 0;
            __syncthreads();
            sh[t] += add;
            __syncthreads();
        }
        const int carry = carry_sh;
        int run = carry + sh[t] - s;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = base + t * 4 + q;
            if (i < nbins) off[i] = run;
            run += v[q];
        }
        __syncthreads();
        if (t == SCAN_THREADS - 1) carry_sh = carry + sh[t];
        __syncthreads();
    }
    if (t == 0) off[nbins] = carry_sh;
}

// Node records in bin order: (frac x, frac y, Fx, Fy) and the packed stencil origin.
__global__ void k_bin_scatter(ScatterArgs a)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.n) return;
    const double2 X = a.X[l];
    const int slot = a.bin_off[a.key[l]] + a.rank[l];
    float4 r = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    int ij = 0;
    if (finite2(X.x, X.y)) {
        const double fx = floor(X.x), fy = floor(X.y);
        const float2 F = a.F[l];
        r = make_float4((float)(X.x - fx), (float)(X.y - fy), F.x, F.y);
        const int i0 = wrap_ll((long long)fx - 1, a.nx);
        long long j0 = (long long)fy - 1;
        if (a.walls) {
            if (j0 < -4) j0 = -4;
            if (j0 > a.ny) j0 = a.ny;
        } else {
            j0 = wrap_ll(j0, a.ny);
        }
        ij = (i0 & 0xFFFF) | (int)((unsigned)(j0 & 0xFFFF) << 16);
    }
    a.rec[slot] = r;
    a.rec_ij[slot] = ij;
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

hipError_t launch_scan(lbib_ctx* c)
{
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(SCAN_THREADS), 0, c->stream, (const int*)c->d_bin_count,
                       c->d_bin_off, c->nbins);
    return hipGetLastError();
}

hipError_t launch_scatter(lbib_ctx* c, const ScatterArgs& a)
{
    const unsigned nb = (unsigned)((a.n + 255) / 256);
    hipLaunchKernelGGL(k_bin_scatter, dim3(nb), dim3(256), 0, c->stream, a);
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
