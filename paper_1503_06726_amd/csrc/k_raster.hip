// Domain-ID rasterisation (Section "Cell Representation": lattice nodes inside cell c carry
// its ID c+1, the extracellular space 0).  Built with floating-point contraction off so the
// crossing abscissae round exactly as in a plain evaluation of the formula below.
//
// One workgroup per cell.  A lattice node (px, py) at integer coordinates is inside when an
// odd number of polygon edges cross the horizontal ray from it to +x, an edge (A, B) crossing
// row py when (A.y > py) != (B.y > py), at x_c = A.x + (py - A.y)(B.x - A.x)/(B.y - A.y), and
// the node counting it when px < x_c.  Each row's crossing count to the right is odd exactly
// when the count of crossings with ceil(x_c) <= px is odd (every row meets a closed polygon
// an even number of times), so each crossing toggles one bit at column ceil(x_c) of an LDS
// bitmap over the cell's bounding box, a prefix XOR along each row gives the parity, and the
// odd pixels receive the cell's ID.  XOR is order-independent, so the result is deterministic.
// The kernel writes only pixels inside its cell; the lattice pass clears the map beforehand.
#include "lbib_internal.h"

#pragma clang fp contract(off)

namespace lbib {

__global__ __launch_bounds__(RASTER_THREADS) void k_raster(RasterArgs a)
{
    __shared__ unsigned bm[RASTER_LDS_WORDS];
    __shared__ double rmin[4][RASTER_THREADS];
    const int c = blockIdx.x;
    const int t = threadIdx.x;
    const int beg = a.off[c];
    const int n = a.off[c + 1] - beg;
    const uint16_t id = (uint16_t)(c + 1);

    // bounding box (min x, min y, -max x, -max y)
    double b0 = INFINITY, b1 = INFINITY, b2 = INFINITY, b3 = INFINITY;
    for (int k = t; k < n; k += RASTER_THREADS) {
        const double2 X = a.X[beg + k];
        b0 = fmin(b0, X.x);
        b1 = fmin(b1, X.y);
        b2 = fmin(b2, -X.x);
        b3 = fmin(b3, -X.y);
    }
    rmin[0][t] = b0;
    rmin[1][t] = b1;
    rmin[2][t] = b2;
    rmin[3][t] = b3;
    __syncthreads();
    for (int w = RASTER_THREADS / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int q = 0; q < 4; ++q) rmin[q][t] = fmin(rmin[q][t], rmin[q][t + w]);
        __syncthreads();
    }
    const double xmin = rmin[0][0], ymin = rmin[1][0], xmax = -rmin[2][0], ymax = -rmin[3][0];
    if (!(isfinite(xmin) && isfinite(ymin) && isfinite(xmax) && isfinite(ymax))) return;
    if (xmax - xmin >= (double)a.nx || ymax - ymin >= (double)a.ny) return;   // invalid cell
    const long long cx0 = (long long)ceil(xmin);
    const int W = (int)((long long)ceil(xmax) - cx0);        // pixel columns cx0 .. cx0 + W - 1
    const long long ry0 = (long long)ceil(ymin);
    const int H = (int)((long long)ceil(ymax) - ry0);        // rows ry0 .. ry0 + H - 1
    if (W <= 0 || H <= 0) return;
    const int WW = (W + 31) / 32;
    int CH = RASTER_LDS_WORDS / WW;                          // rows per pass
    if (CH < 1) CH = 1;                                      // (W <= nx <= 32767 keeps WW <= 1024)
    if (CH > H) CH = H;

    for (int r0 = 0; r0 < H; r0 += CH) {
        const int rows = (H - r0 < CH) ? H - r0 : CH;
        for (int i = t; i < rows * WW; i += RASTER_THREADS) bm[i] = 0u;
        __syncthreads();
        // each edge toggles one bit per row it crosses
        for (int k = t; k < n; k += RASTER_THREADS) {
            const double2 A = a.X[beg + k];
            const double2 B = a.X[beg + ((k + 1 == n) ? 0 : k + 1)];
            const double lo = fmin(A.y, B.y), hi = fmax(A.y, B.y);
            long long ya = (long long)ceil(lo), yb = (long long)ceil(hi) - 1;
            if (ya < ry0 + r0) ya = ry0 + r0;
            if (yb > ry0 + r0 + rows - 1) yb = ry0 + r0 + rows - 1;
            for (long long py = ya; py <= yb; ++py) {
                const double yy = (double)py;
                if ((A.y > yy) == (B.y > yy)) continue;
                const double xc = A.x + (yy - A.y) * (B.x - A.x) / (B.y - A.y);
                long long col = (long long)ceil(xc) - cx0;
                if (col < 0) col = 0;
                if (col >= W) continue;
                const int rr = (int)(py - ry0 - r0);
                atomicXor(&bm[rr * WW + (int)(col >> 5)], 1u << (col & 31));
            }
        }
        __syncthreads();
        // prefix XOR along each row: bit k becomes the parity of toggles at columns <= k
        for (int rr = t; rr < rows; rr += RASTER_THREADS) {
            unsigned carry = 0u;
            for (int w = 0; w < WW; ++w) {
                unsigned v = bm[rr * WW + w];
                v ^= v << 1;
                v ^= v << 2;
                v ^= v << 4;
                v ^= v << 8;
                v ^= v << 16;
                v ^= carry;
                bm[rr * WW + w] = v;
                carry = (v >> 31) ? 0xFFFFFFFFu : 0u;
            }
        }
        __syncthreads();
        for (int i = t; i < rows * W; i += RASTER_THREADS) {
            const int rr = i / W, col = i - rr * W;
            if (!((bm[rr * WW + (col >> 5)] >> (col & 31)) & 1u)) continue;
            const long long py = ry0 + r0 + rr;
            int j;
            if (a.walls) {
                if (py < 0 || py >= a.ny) continue;
                j = (int)py;
            } else {
                j = wrap_ll(py, a.ny);
            }
            const int ix = wrap_ll(cx0 + col, a.nx);
            a.mask[(int64_t)j * a.nx + ix] = id;
        }
        __syncthreads();
    }
}

hipError_t launch_raster(lbib_ctx* c, const RasterArgs& a)
{
    hipLaunchKernelGGL(k_raster, dim3((unsigned)c->n_cells), dim3(RASTER_THREADS), 0, c->stream, a);
    return hipGetLastError();
}

}  // namespace lbib
