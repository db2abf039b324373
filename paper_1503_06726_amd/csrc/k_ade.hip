// ADE-only iterations of the species lattices (gfx950), the steady-state measurement: every
// species collides with u = 0 (D2Q5 equilibrium w_i phi, Suppl. "Lattice Boltzmann Method")
// plus its reaction and streams with halfway bounce-back at walls, while the fluid, the
// membranes and the domain map stay frozen.  The iteration runs in a working set of float or
// double deviations; each pass also leaves per-block sums of (phi^k - phi^{k-1})^2 and
// (phi^k)^2, which one kernel per batch of passes turns into the relative changes
// ||phi^k - phi^{k-1}||_2 / ||phi^k||_2 (fixed-order sums: deterministic).
#include "lbib_internal.h"

namespace lbib {

constexpr int ADE_THREADS = 256;

template <typename WT>
__device__ inline void pull5w(const WT* __restrict__ s, int64_t nn, int x, int y, int nx, int ny, int walls, WT g[5])
{
    const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    const int64_t rc = (int64_t)y * nx;
    bool bot = false, top = false;
    int ym, yp;
    if (walls) {
        bot = (y == 0);
        top = (y == ny - 1);
        ym = bot ? y : y - 1;
        yp = top ? y : y + 1;
    } else {
        ym = (y == 0) ? ny - 1 : y - 1;
        yp = (y == ny - 1) ? 0 : y + 1;
    }
    // g_i(x) = s_i(x - v_i); across a wall the population returns reversed: s_opp(i)(x)
    g[0] = s[rc + x];
    g[1] = s[nn + rc + xm];
    g[2] = bot ? s[4 * nn + rc + x] : s[2 * nn + (int64_t)ym * nx + x];
    g[3] = s[3 * nn + rc + xp];
    g[4] = top ? s[2 * nn + rc + x] : s[4 * nn + (int64_t)yp * nx + x];
}

template <typename WT>
__global__ __launch_bounds__(ADE_THREADS) void k_ade(AdeArgs a)
{
    __shared__ double sh[4][ADE_THREADS];
    const int t = threadIdx.x;
    const int64_t idx = (int64_t)blockIdx.x * ADE_THREADS + t;
    const WT w0 = WT(1) / WT(3), w1 = WT(1) / WT(6);
    double d2[2] = {0.0, 0.0}, p2[2] = {0.0, 0.0};
    if (idx < a.nn) {
        const int x = (int)(idx % a.nx), y = (int)(idx / a.nx);
        const WT* src = (const WT*)a.src;
        WT* dst = (WT*)a.dst;
        WT g[2][5], dphi[2], phi[2];
        for (int s = 0; s < a.S; ++s) {
            pull5w<WT>(src + (int64_t)5 * s * a.nn, a.nn, x, y, a.nx, a.ny, a.walls, g[s]);
            dphi[s] = ((g[s][0] + g[s][1]) + (g[s][2] + g[s][3])) + g[s][4];
            phi[s] = (WT)a.phi_ref[s] + dphi[s];
        }
        const int m = (int)((a.inside[(int64_t)y * a.wpr + (x >> 5)] >> (x & 31)) & 1u);
        for (int s = 0; s < a.S; ++s) {
            WT R = WT(0);
            if (a.react[s] == LBIB_REACT_SOURCE_DECAY) {
                R = (m ? (WT)a.rc[s][0] : WT(0)) - (WT)a.rc[s][1] * phi[s];
            } else if (a.react[s] == LBIB_REACT_SCHNAKENBERG && a.S == 2) {
                const WT u2v = phi[0] * phi[0] * phi[1];
                R = (s == 0) ? (WT)a.rc[s][2] * ((WT)a.rc[s][0] - phi[0] + u2v) : (WT)a.rc[s][2] * ((WT)a.rc[s][1] - u2v);
            }
            const WT om = (WT)a.omega_s[s], om1 = WT(1) - om;
            WT* d = dst + (int64_t)5 * s * a.nn + idx;
            // deviation form: dg_i <- dg_i - omega (dg_i - w_i dphi) + w_i R
            d[0] = om1 * g[s][0] + om * w0 * dphi[s] + w0 * R;
            for (int i = 1; i < 5; ++i) d[i * a.nn] = om1 * g[s][i] + om * w1 * dphi[s] + w1 * R;
            const double ph = (double)phi[s];
            double* pp = a.phi_prev + (int64_t)s * a.nn + idx;
            if (a.track) {
                const double df = ph - *pp;
                d2[s] = df * df;
                p2[s] = ph * ph;
            }
            *pp = ph;
        }
    }
    if (!a.track) return;                                   // uniform: no reduction on the first pass

    // per-block sums (fixed tree) into the pass's slot; k_ade_hist adds the blocks in order
    for (int q = 0; q < 2; ++q) {
        sh[2 * q][t] = d2[q];
        sh[2 * q + 1][t] = p2[q];
    }
    __syncthreads();
    for (int w = ADE_THREADS / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int v = 0; v < 4; ++v) sh[v][t] += sh[v][t + w];
        __syncthreads();
    }
    if (t < 4) a.partial[((int64_t)a.hslot * gridDim.x + blockIdx.x) * 4 + t] = sh[t][0];
}

// relative change of every species for each pass of a batch: one workgroup per pass adds
// its per-block sums in block order (fixed tree)
__global__ __launch_bounds__(ADE_THREADS) void k_ade_hist(const double* __restrict__ partial, int nblocks, int S,
                                                          double* __restrict__ hist)
{
    __shared__ double sh[4][ADE_THREADS];
    const int t = threadIdx.x, slot = blockIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = t; b < nblocks; b += ADE_THREADS)
        for (int v = 0; v < 4; ++v) acc[v] += partial[((int64_t)slot * nblocks + b) * 4 + v];
    for (int v = 0; v < 4; ++v) sh[v][t] = acc[v];
    __syncthreads();
    for (int w = ADE_THREADS / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int v = 0; v < 4; ++v) sh[v][t] += sh[v][t + w];
        __syncthreads();
    }
    if (t == 0)
        for (int s = 0; s < S; ++s) {
            const double dd = sh[2 * s][0], pp = sh[2 * s + 1][0];
            hist[(int64_t)slot * S + s] = (dd == 0.0) ? 0.0 : sqrt(dd) / sqrt(pp);
        }
}

// working set <- the context's populations (storage ST), and back
template <int ST, typename WT>
__global__ void k_ade_load(const void* __restrict__ g, WT* __restrict__ w, int64_t nn, int nx, int64_t grow,
                           int gchunk, int S)
{
    using T = typename Pop<ST>::T;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nn) return;
    const int x = (int)(idx % nx), y = (int)(idx / nx);
    const T* gs = (const T*)g;
    for (int s = 0; s < S; ++s)
        for (int i = 0; i < 5; ++i) {
            const int64_t o = ((int64_t)5 * s + i) * nn + idx;
            w[o] = (WT)Pop<ST>::ld(gs[pop_at(grow, gchunk, 5 * s + i, y, x)], IS5[i]);
        }
}

template <int ST, typename WT>
__global__ void k_ade_store(const WT* __restrict__ w, void* __restrict__ g, int64_t nn, int nx, int64_t grow,
                            int gchunk, int S)
{
    using T = typename Pop<ST>::T;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nn) return;
    const int x = (int)(idx % nx), y = (int)(idx / nx);
    T* gs = (T*)g;
    for (int s = 0; s < S; ++s)
        for (int i = 0; i < 5; ++i) {
            const int64_t o = ((int64_t)5 * s + i) * nn + idx;
            gs[pop_at(grow, gchunk, 5 * s + i, y, x)] = Pop<ST>::st((float)w[o], SC5[i]);
        }
}

hipError_t launch_ade(lbib_ctx* c, const AdeArgs& a, bool fp64, hipStream_t stream)
{
    const unsigned nb = (unsigned)((a.nn + ADE_THREADS - 1) / ADE_THREADS);
    if (fp64) hipLaunchKernelGGL(k_ade<double>, dim3(nb), dim3(ADE_THREADS), 0, stream, a);
    else hipLaunchKernelGGL(k_ade<float>, dim3(nb), dim3(ADE_THREADS), 0, stream, a);
    return hipGetLastError();
}

template <typename WT>
static hipError_t ade_copy(lbib_ctx* c, void* work, bool to_work)
{
    const unsigned nb = (unsigned)((c->nn + 255) / 256);
    const void* g = c->g[c->cur];
    WT* w = (WT*)work;
    switch (c->p.storage) {
    case LBIB_STORAGE_FP16:
        if (to_work) hipLaunchKernelGGL((k_ade_load<1, WT>), dim3(nb), dim3(256), 0, c->stream, g, w, c->nn, c->p.nx, c->grow(), c->gchunk(), c->S);
        else hipLaunchKernelGGL((k_ade_store<1, WT>), dim3(nb), dim3(256), 0, c->stream, w, c->g[c->cur], c->nn, c->p.nx, c->grow(), c->gchunk(), c->S);
        break;
    case LBIB_STORAGE_BF16:
        if (to_work) hipLaunchKernelGGL((k_ade_load<2, WT>), dim3(nb), dim3(256), 0, c->stream, g, w, c->nn, c->p.nx, c->grow(), c->gchunk(), c->S);
        else hipLaunchKernelGGL((k_ade_store<2, WT>), dim3(nb), dim3(256), 0, c->stream, w, c->g[c->cur], c->nn, c->p.nx, c->grow(), c->gchunk(), c->S);
        break;
    default:
        if (to_work) hipLaunchKernelGGL((k_ade_load<0, WT>), dim3(nb), dim3(256), 0, c->stream, g, w, c->nn, c->p.nx, c->grow(), c->gchunk(), c->S);
        else hipLaunchKernelGGL((k_ade_store<0, WT>), dim3(nb), dim3(256), 0, c->stream, w, c->g[c->cur], c->nn, c->p.nx, c->grow(), c->gchunk(), c->S);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_ade_copy(lbib_ctx* c, void* work, bool fp64, bool to_work)
{
    return fp64 ? ade_copy<double>(c, work, to_work) : ade_copy<float>(c, work, to_work);
}

unsigned ade_blocks(int64_t nn) { return (unsigned)((nn + ADE_THREADS - 1) / ADE_THREADS); }

hipError_t launch_ade_hist(const double* partial, int nblocks, int S, double* hist, int slots, hipStream_t stream)
{
    hipLaunchKernelGGL(k_ade_hist, dim3((unsigned)slots), dim3(ADE_THREADS), 0, stream, partial, nblocks, S, hist);
    return hipGetLastError();
}

}  // namespace lbib

// ---------------------------------------------------------------------------------------
// batched ADE-only iterations: B independent single-species problems of one lattice size
// (source/decay law, u = 0), one grid row per sample; a converged sample stops updating.
// ---------------------------------------------------------------------------------------
namespace lbib {


template <typename WT>
__global__ __launch_bounds__(ADE_THREADS) void k_ade_batch(AdeBatchArgs a)
{
    __shared__ double sh[2][ADE_THREADS];
    const int b = blockIdx.y, t = threadIdx.x;
    if (!a.active[b]) return;                                // uniform across the block
    const int64_t idx = (int64_t)blockIdx.x * ADE_THREADS + t;
    const WT w0 = WT(1) / WT(3), w1 = WT(1) / WT(6);
    double d2 = 0.0, p2 = 0.0;
    if (idx < a.nn) {
        const int x = (int)(idx % a.nx), y = (int)(idx / a.nx);
        const WT* src = (const WT*)a.src + (int64_t)5 * b * a.nn;
        WT* dst = (WT*)a.dst + (int64_t)5 * b * a.nn;
        WT g[5];
        pull5w<WT>(src, a.nn, x, y, a.nx, a.ny, a.walls, g);
        const WT phi = ((g[0] + g[1]) + (g[2] + g[3])) + g[4];
        const WT R = (a.source[(int64_t)b * a.nn + idx] ? (WT)a.sigma[b] : WT(0)) - (WT)a.decay[b] * phi;
        const WT om = (WT)a.omega[b], om1 = WT(1) - om;
        // g_i <- g_i - omega (g_i - w_i phi) + w_i R
        dst[idx] = om1 * g[0] + om * w0 * phi + w0 * R;
        for (int i = 1; i < 5; ++i) dst[i * a.nn + idx] = om1 * g[i] + om * w1 * phi + w1 * R;
        const double ph = (double)phi;
        double* pp = a.phi_prev + (int64_t)b * a.nn + idx;
        if (a.track) {
            const double df = ph - *pp;
            d2 = df * df;
            p2 = ph * ph;
        }
        *pp = ph;
    }
    if (!a.track) return;
    sh[0][t] = d2;
    sh[1][t] = p2;
    __syncthreads();
    for (int w = ADE_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] += sh[0][t + w];
            sh[1][t] += sh[1][t + w];
        }
        __syncthreads();
    }
    if (t < 2) a.partial[(((int64_t)a.hslot * a.B + b) * a.nblocks + blockIdx.x) * 2 + t] = sh[t][0];
}

// relative change per (pass, sample): one workgroup each, blocks added in order
__global__ __launch_bounds__(ADE_THREADS) void k_ade_batch_hist(const double* __restrict__ partial, int nblocks, int B,
                                                                const int* __restrict__ active, double* __restrict__ hist)
{
    __shared__ double sh[2][ADE_THREADS];
    const int t = threadIdx.x, slot = blockIdx.x, b = blockIdx.y;
    if (!active[b]) {
        if (t == 0) hist[(int64_t)slot * B + b] = -1.0;        // not iterated in this pass
        return;
    }
    double acc[2] = {0.0, 0.0};
    for (int k = t; k < nblocks; k += ADE_THREADS)
        for (int v = 0; v < 2; ++v) acc[v] += partial[(((int64_t)slot * B + b) * nblocks + k) * 2 + v];
    sh[0][t] = acc[0];
    sh[1][t] = acc[1];
    __syncthreads();
    for (int w = ADE_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] += sh[0][t + w];
            sh[1][t] += sh[1][t + w];
        }
        __syncthreads();
    }
    if (t == 0) hist[(int64_t)slot * B + b] = (sh[0][0] == 0.0) ? 0.0 : sqrt(sh[0][0]) / sqrt(sh[1][0]);
}

// equilibrium start g_i = w_i phi (u = 0), written in the stored (pre-streaming) layout so
// that the first pull yields g_i(x) = w_i phi(x): s_i(x - v_i) = w_i phi(x), or, across a wall,
// s_opp(i)(x) = w_i phi(x); and read-back of phi = sum_i g_i
template <typename WT>
__global__ void k_ade_batch_init(const double* __restrict__ phi, WT* __restrict__ g, int64_t nn, int nx, int ny,
                                 int walls, int B)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (idx >= nn) return;
    const int x = (int)(idx % nx), y = (int)(idx / nx);
    const int vx[5] = {0, 1, 0, -1, 0}, vy[5] = {0, 0, 1, 0, -1}, opp[5] = {0, 3, 4, 1, 2};
    const double p = phi ? phi[(int64_t)b * nn + idx] : 0.0;
    WT* gb = g + (int64_t)5 * b * nn;
    for (int i = 0; i < 5; ++i) {
        const WT v = (WT)(p * (i == 0 ? 1.0 / 3.0 : 1.0 / 6.0));
        const int sy = y - vy[i];
        if (walls && (sy < 0 || sy >= ny)) {
            gb[(int64_t)opp[i] * nn + idx] = v;
        } else {
            const int sx = (x - vx[i] + nx) % nx, syy = (sy + ny) % ny;
            gb[(int64_t)i * nn + (int64_t)syy * nx + sx] = v;
        }
    }
}

template <typename WT>
__global__ void k_ade_batch_phi(const WT* __restrict__ g, double* __restrict__ phi, int64_t nn, int nx, int ny,
                                int walls, int B)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (idx >= nn) return;
    // the stored values are post-collision: phi is the sum of the populations pulled to the node
    WT q[5];
    pull5w<WT>(g + (int64_t)5 * b * nn, nn, (int)(idx % nx), (int)(idx / nx), nx, ny, walls, q);
    phi[(int64_t)b * nn + idx] = (double)(((q[0] + q[1]) + (q[2] + q[3])) + q[4]);
}

}  // namespace lbib

namespace lbib {

hipError_t ade_batch_launch(const AdeBatchArgs& a, bool fp64, hipStream_t s)
{
    const dim3 grid((unsigned)a.nblocks, (unsigned)a.B);
    if (fp64) hipLaunchKernelGGL(k_ade_batch<double>, grid, dim3(ADE_THREADS), 0, s, a);
    else hipLaunchKernelGGL(k_ade_batch<float>, grid, dim3(ADE_THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t ade_batch_hist_launch(const AdeBatchArgs& a, double* hist, hipStream_t s)
{
    hipLaunchKernelGGL(k_ade_batch_hist, dim3(ADE_BATCH_SLOTS, (unsigned)a.B), dim3(ADE_THREADS), 0, s,
                       (const double*)a.partial, a.nblocks, a.B, a.active, hist);
    return hipGetLastError();
}

hipError_t ade_batch_init_launch(const double* phi, void* g, int64_t nn, int nx, int ny, int walls, int B, bool fp64,
                                 hipStream_t s)
{
    const dim3 grid((unsigned)((nn + 255) / 256), (unsigned)B);
    if (fp64) hipLaunchKernelGGL(k_ade_batch_init<double>, grid, dim3(256), 0, s, phi, (double*)g, nn, nx, ny, walls, B);
    else hipLaunchKernelGGL(k_ade_batch_init<float>, grid, dim3(256), 0, s, phi, (float*)g, nn, nx, ny, walls, B);
    return hipGetLastError();
}

hipError_t ade_batch_phi_launch(const void* g, double* phi, int64_t nn, int nx, int ny, int walls, int B, bool fp64,
                                hipStream_t s)
{
    const dim3 grid((unsigned)((nn + 255) / 256), (unsigned)B);
    if (fp64)
        hipLaunchKernelGGL(k_ade_batch_phi<double>, grid, dim3(256), 0, s, (const double*)g, phi, nn, nx, ny, walls, B);
    else hipLaunchKernelGGL(k_ade_batch_phi<float>, grid, dim3(256), 0, s, (const float*)g, phi, nn, nx, ny, walls, B);
    return hipGetLastError();
}

}  // namespace lbib
