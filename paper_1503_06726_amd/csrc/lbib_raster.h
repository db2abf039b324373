// Domain-ID rasterisation of one cell by one workgroup (Section "Cell Representation": lattice
// nodes inside cell c carry its ID c+1, the extracellular space 0).
//
// A lattice node (px, py) at integer coordinates is inside when an odd number of polygon
// edges cross the horizontal ray from it to +x; an edge (A, B) crosses row py when
// (A.y > py) != (B.y > py), at x_c = A.x + (py - A.y)(B.x - A.x)/(B.y - A.y), and the node
// counts it when px < x_c.  Every row meets a closed polygon an even number of times, so the
// count to the right is odd exactly when the count with ceil(x_c) <= px is odd: each crossing
// toggles the bit at column ceil(x_c) of a bitmap over the cell's bounding box, and a prefix
// XOR along the row gives the parity.  XOR is order-independent, so the result is
// deterministic.  Floating-point contraction is off where the crossing abscissae are computed,
// so they round exactly as the formula is written.
//
// Two outputs: the domain-ID map (odd pixels receive the cell's ID), or the inside map, one
// bit per lattice node (rows of wpr 32-bit words) into which the cell's rows are OR-ed whole
// words at a time; its bit is 1 where some cell's ID would be nonzero.  Only pixels inside the
// cell are written; the caller clears the map beforehand.
#pragma once

#include "lbib_device.h"

namespace lbib {

__device__ inline double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Pixel box of a cell: columns cx0 .. cx0 + W - 1 (unwrapped), rows ry0 .. ry0 + H - 1, WW
// bitmap words per row.  ok is false for an empty box or an invalid (non-finite or too wide)
// cell, which is not rasterised.
struct RasterBox {
    int cx0, W, WW, ry0, H;
    bool ok;
};

__device__ inline RasterBox raster_box(double xmin, double ymin, double xmax, double ymax, int nx, int ny)
{
    RasterBox b{0, 0, 1, 0, 0, false};
    if (!(finite2(xmin, ymin) && finite2(xmax, ymax))) return b;
    if (xmax - xmin >= (double)nx || ymax - ymin >= (double)ny) return b;
    b.cx0 = (int)ceil(xmin);
    b.W = (int)ceil(xmax) - b.cx0;
    b.ry0 = (int)ceil(ymin);
    b.H = (int)ceil(ymax) - b.ry0;
    b.WW = (b.W + 31) / 32;
    b.ok = b.W > 0 && b.H > 0;
    return b;
}

// Toggle the crossings of the cell's edges with box rows r0 .. r0 + rows - 1 (bitmap rows 0 ..).
__device__ inline void raster_toggle(const double2* P, int n, const RasterBox& b, int r0, int rows, unsigned* bm)
{
#pragma clang fp contract(off)
    const int t = threadIdx.x, nt = blockDim.x;
    const int ylo = b.ry0 + r0, yhi = b.ry0 + r0 + rows - 1;
    for (int k = t; k < n; k += nt) {
        const double2 A = P[k];
        const double2 B = P[(k + 1 == n) ? 0 : k + 1];
        int ya = (int)ceil(fmin(A.y, B.y)), yb = (int)ceil(fmax(A.y, B.y)) - 1;
        if (ya < ylo) ya = ylo;
        if (yb > yhi) yb = yhi;
        for (int py = ya; py <= yb; ++py) {
            const double yy = (double)py;
            if ((A.y > yy) == (B.y > yy)) continue;
            const double xc = A.x + (yy - A.y) * (B.x - A.x) / (B.y - A.y);
            int col = (int)ceil(xc) - b.cx0;
            if (col < 0) col = 0;
            if (col >= b.W) continue;
            atomicXor(&bm[(py - ylo) * b.WW + (col >> 5)], 1u << (col & 31));
        }
    }
}

// prefix XOR along each bitmap row: bit k becomes the parity of the toggles at columns <= k
__device__ inline void raster_prefix(unsigned* bm, int rows, int WW)
{
    for (int rr = threadIdx.x; rr < rows; rr += blockDim.x) {
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
}

// lattice row of box row py, or -1 beyond a wall
__device__ inline int raster_row(int py, int ny, int walls)
{
    if (walls) return (py < 0 || py >= ny) ? -1 : py;
    return wrap_i(py, ny);
}

// write the ID into the odd pixels of box rows r0 .. r0 + rows - 1 (one wavefront per row)
__device__ inline void raster_write_ids(const unsigned* bm, const RasterBox& b, int r0, int rows, uint16_t id,
                                        uint16_t* __restrict__ ids, int nx, int ny, int walls)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int cw = wrap_i(b.cx0, nx);
    for (int rr = wid; rr < rows; rr += nw) {
        const int j = raster_row(b.ry0 + r0 + rr, ny, walls);
        if (j < 0) continue;
        uint16_t* row = ids + (int64_t)j * nx;
        for (int col = lane; col < b.W; col += 64) {
            if (!((bm[rr * b.WW + (col >> 5)] >> (col & 31)) & 1u)) continue;
            int ix = cw + col;
            if (ix >= nx) ix -= nx;
            row[ix] = id;
        }
    }
}

// claim the odd pixels of box rows r0 .. r0 + rows - 1 for cell `cell` in the cell map: the
// lowest index claiming a node keeps it (atomic minimum over a map reset to ~0), so the result
// does not depend on the order of the cells' workgroups (one wavefront per row)
__device__ inline void raster_claim_cells(const unsigned* bm, const RasterBox& b, int r0, int rows, unsigned cell,
                                          unsigned* __restrict__ cmap, int nx, int ny, int walls)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int cw = wrap_i(b.cx0, nx);
    for (int rr = wid; rr < rows; rr += nw) {
        const int j = raster_row(b.ry0 + r0 + rr, ny, walls);
        if (j < 0) continue;
        unsigned* row = cmap + (int64_t)j * nx;
        for (int col = lane; col < b.W; col += 64) {
            if (!((bm[rr * b.WW + (col >> 5)] >> (col & 31)) & 1u)) continue;
            int ix = cw + col;
            if (ix >= nx) ix -= nx;
            atomicMin(&row[ix], cell);
        }
    }
}

// Bits of relative columns c0 .. c0 + 31 of bitmap row `row` (WW words, W valid columns);
// columns outside 0 .. W - 1 read as 0.
__device__ inline unsigned bitmap_bits(const unsigned* row, int WW, int W, int c0)
{
    const int w = c0 >> 5, sh = c0 & 31;                // floor division for negative c0
    const unsigned lo = (w >= 0 && w < WW) ? row[w] : 0u;
    const unsigned hi = (w + 1 >= 0 && w + 1 < WW) ? row[w + 1] : 0u;
    unsigned v = sh ? (lo >> sh) | (hi << (32 - sh)) : lo;
    if (c0 < 0) v &= (c0 <= -32) ? 0u : (0xFFFFFFFFu << (-c0));
    const int left = W - c0;                            // valid columns from c0 on
    if (left < 32) v &= (left <= 0) ? 0u : (0xFFFFFFFFu >> (32 - left));
    return v;
}

// OR the odd pixels of box rows r0 .. r0 + rows - 1 into the inside map.  A row's columns
// cw .. cw + W - 1 (cw = cx0 mod nx) wrap at nx into at most two runs of whole words; every
// (row, word) pair goes to its own thread.
__device__ inline void raster_or_bits(const unsigned* bm, const RasterBox& b, int r0, int rows,
                                      unsigned* __restrict__ bits, int wpr, int nx, int ny, int walls)
{
    const int cw = wrap_i(b.cx0, nx);
    const int e0 = (cw + b.W < nx) ? cw + b.W : nx;     // first run [cw, e0)
    const int g0 = cw >> 5;
    const int n0 = ((e0 - 1) >> 5) - g0 + 1;
    const int e1 = cw + b.W - nx;                       // second run [0, e1), if e1 > 0
    const int n1 = (e1 > 0) ? ((e1 - 1) >> 5) + 1 : 0;
    const int per_row = n0 + n1;
    for (int q = threadIdx.x; q < rows * per_row; q += blockDim.x) {
        const int rr = q / per_row, qq = q - rr * per_row;
        const int j = raster_row(b.ry0 + r0 + rr, ny, walls);
        if (j < 0) continue;
        int g, lo, hi, rel;
        if (qq < n0) {
            g = g0 + qq;
            lo = cw;
            hi = e0;
            rel = 32 * g - cw;                          // relative column of the word's bit 0
        } else {
            g = qq - n0;
            lo = 0;
            hi = e1;
            rel = 32 * g + (nx - cw);
        }
        unsigned v = bitmap_bits(bm + rr * b.WW, b.WW, b.W, rel);
        const int b0 = lo - 32 * g, b1 = hi - 32 * g;   // valid bit range [b0, b1)
        if (b0 > 0) v &= 0xFFFFFFFFu << b0;
        if (b1 < 32) v &= (b1 <= 0) ? 0u : (0xFFFFFFFFu >> (32 - b1));
        if (v) atomicOr(&bits[(int64_t)j * wpr + g], v);
    }
}

// Whole-cell rasterisation into the ID map.  P: the cell's n positions; bm: `words` LDS words;
// red: >= 4 * (blockDim.x / 64) LDS doubles.  Called by every thread of the workgroup.
__device__ inline void raster_cell_ids(const double2* P, int n, uint16_t id, uint16_t* __restrict__ ids, int nx,
                                       int ny, int walls, unsigned* bm, int words, double* red)
{
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
    const RasterBox b = raster_box(xmin, ymin, -nxmax, -nymax, nx, ny);
    if (!b.ok) return;                                  // uniform across the group
    int CH = words / b.WW;                              // rows per pass (W <= nx keeps WW <= 1024)
    if (CH < 1) CH = 1;
    if (CH > b.H) CH = b.H;
    for (int r0 = 0; r0 < b.H; r0 += CH) {
        const int rows = (b.H - r0 < CH) ? b.H - r0 : CH;
        for (int i = t; i < rows * b.WW; i += nt) bm[i] = 0u;
        __syncthreads();
        raster_toggle(P, n, b, r0, rows, bm);
        __syncthreads();
        raster_prefix(bm, rows, b.WW);
        __syncthreads();
        raster_write_ids(bm, b, r0, rows, id, ids, nx, ny, walls);
        __syncthreads();
    }
}

}  // namespace lbib
