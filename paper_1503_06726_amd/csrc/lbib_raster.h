// Domain-ID rasterisation of one cell by one workgroup (Section "Cell Representation": lattice
// nodes inside cell c carry its ID c+1, the extracellular space 0).
//
// A lattice node (px, py) at integer coordinates is inside when an odd number of polygon
// edges cross the horizontal ray from it to +x; an edge (A, B) crosses row py when
// (A.y > py) != (B.y > py), at x_c = A.x + (py - A.y)(B.x - A.x)/(B.y - A.y), and the node
// counts it when px < x_c.  Every row meets a closed polygon an even number of times, so the
// count to the right is odd exactly when the count with ceil(x_c) <= px is odd: each crossing
// toggles the bit at column ceil(x_c) of a bitmap over the cell's bounding box, a prefix XOR
// along the row gives the parity, and odd pixels receive the ID.  XOR is order-independent,
// so the result is deterministic.  Floating-point contraction is off in this function so the
// crossing abscissae round exactly as the formula is written.  Only pixels inside the cell
// are written; the lattice pass clears the map beforehand.
#pragma once

#include "lbib_device.h"

namespace lbib {

__device__ inline double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// P: the cell's n positions (global or LDS); bm: `words` LDS words; red: >= 16 LDS doubles.
// Called by every thread of a 256-thread workgroup.
__device__ inline void raster_cell(const double2* P, int n, uint16_t id, uint16_t* __restrict__ mask, int nx,
                                   int ny, int walls, unsigned* bm, int words, double* red)
{
#pragma clang fp contract(off)
    const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wid = t >> 6;
    // bounding box: min x, min y, -max x, -max y
    double b0 = INFINITY, b1 = INFINITY, b2 = INFINITY, b3 = INFINITY;
    for (int k = t; k < n; k += nt) {
        const double2 X = P[k];
        b0 = fmin(b0, X.x);
        b1 = fmin(b1, X.y);
        b2 = fmin(b2, -X.x);
        b3 = fmin(b3, -X.y);
    }
    b0 = wave_min(b0);
    b1 = wave_min(b1);
    b2 = wave_min(b2);
    b3 = wave_min(b3);
    __syncthreads();                         // red may still be in use by the caller
    if (lane == 0) {
        red[wid * 4 + 0] = b0;
        red[wid * 4 + 1] = b1;
        red[wid * 4 + 2] = b2;
        red[wid * 4 + 3] = b3;
    }
    __syncthreads();
    const int nw = nt >> 6;
    double xmin = red[0], ymin = red[1], nxmax = red[2], nymax = red[3];
    for (int w = 1; w < nw; ++w) {
        xmin = fmin(xmin, red[w * 4 + 0]);
        ymin = fmin(ymin, red[w * 4 + 1]);
        nxmax = fmin(nxmax, red[w * 4 + 2]);
        nymax = fmin(nymax, red[w * 4 + 3]);
    }
    const double xmax = -nxmax, ymax = -nymax;
    if (!(finite2(xmin, ymin) && finite2(xmax, ymax))) return;          // uniform across the group
    if (xmax - xmin >= (double)nx || ymax - ymin >= (double)ny) return;  // invalid cell
    const long long cx0 = (long long)ceil(xmin);
    const int W = (int)((long long)ceil(xmax) - cx0);   // pixel columns cx0 .. cx0 + W - 1
    const long long ry0 = (long long)ceil(ymin);
    const int H = (int)((long long)ceil(ymax) - ry0);   // rows ry0 .. ry0 + H - 1
    if (W <= 0 || H <= 0) return;
    const int WW = (W + 31) / 32;
    int CH = words / WW;                                // rows per pass
    if (CH < 1) CH = 1;                                 // (W < nx <= 32767 keeps WW <= 1024)
    if (CH > H) CH = H;

    for (int r0 = 0; r0 < H; r0 += CH) {
        const int rows = (H - r0 < CH) ? H - r0 : CH;
        for (int i = t; i < rows * WW; i += nt) bm[i] = 0u;
        __syncthreads();
        for (int k = t; k < n; k += nt) {
            const double2 A = P[k];
            const double2 B = P[(k + 1 == n) ? 0 : k + 1];
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
        for (int rr = t; rr < rows; rr += nt) {
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
        // one wavefront per row, lanes along the row
        const int cw = wrap_i((int)cx0, nx);
        for (int rr = wid; rr < rows; rr += nt >> 6) {
            const int py = (int)(ry0 + r0 + rr);
            int j;
            if (walls) {
                if (py < 0 || py >= ny) continue;
                j = py;
            } else {
                j = wrap_i(py, ny);
            }
            uint16_t* row = mask + (int64_t)j * nx;
            for (int col = lane; col < W; col += 64) {
                if (!((bm[rr * WW + (col >> 5)] >> (col & 31)) & 1u)) continue;
                int ix = cw + col;
                if (ix >= nx) ix -= nx;
                row[ix] = id;
            }
        }
        __syncthreads();
    }
}

}  // namespace lbib
