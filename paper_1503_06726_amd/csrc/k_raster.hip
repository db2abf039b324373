// Standalone domain-ID rasterisation, one workgroup per cell (the ID map is built on demand;
// the time step keeps only the inside-any-cell bits).  The per-cell algorithm is in
// lbib_raster.h.
#include "lbib_internal.h"
#include "lbib_raster.h"

namespace lbib {

__global__ __launch_bounds__(RASTER_THREADS) void k_raster(RasterArgs a)
{
    __shared__ unsigned bm[RASTER_WORDS];
    __shared__ double red[16];
    const int c = blockIdx.x;
    const int beg = a.off[c];
    const int n = a.off[c + 1] - beg;
    raster_cell_ids(a.X + beg, n, (uint16_t)(c + 1), a.mask, a.nx, a.ny, a.walls, bm, RASTER_WORDS, red);
}

hipError_t launch_raster(lbib_ctx* c, const RasterArgs& a)
{
    hipLaunchKernelGGL(k_raster, dim3((unsigned)c->n_cells), dim3(RASTER_THREADS), 0, c->stream, a);
    return hipGetLastError();
}

}  // namespace lbib
