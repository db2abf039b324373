// Convolutional surrogate of the species' steady state (gfx950): a four-level U-Net on BF16
// activations and weights with FP32 accumulation on MFMA, trained by the kernels below (forward,
// backward, Adam).  It maps per-node features of a static tissue (source mask, cell-boundary
// mask, diffusivity, decay, source fraction; eight input channels) to the dimensionless steady
// concentration phi * decay / source, which seeds the D2Q5 populations before the ADE-only
// iteration runs to its tolerance.
//
// Tensors are NHWC with the channel count a multiple of 16.  A 3x3 convolution (zero padding,
// stride 1) is an implicit GEMM: M = output pixels, N = output channels, K = 9 * Cin ordered
// k = tap * Cin + ci with tap = 3 ky + kx reading the input at (y + ky - 1, x + kx - 1).
// Weights are stored [Cout][9 Cin] (k contiguous).  Convolutions whose input has a multiple of
// 32 channels and every weight gradient run on MFMA 16x16x32 (below); the first layer's 16-channel
// input takes MFMA 16x16x16 (bf16), where lane l supplies A[l % 16][4 (l / 16) + i] and
// B[4 (l / 16) + i][l % 16] and holds D[4 (l / 16) + i][l % 16].
#include "lbib_internal.h"

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

namespace lbib {
namespace net {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint16_t bf16;

__device__ __host__ inline float bf2f(bf16 h)
{
    union { uint32_t u; float f; } c;
    c.u = (uint32_t)h << 16;
    return c.f;
}

// round to nearest even (NaN stays NaN)
__device__ __host__ inline bf16 f2bf(float f)
{
    union { uint32_t u; float f; } c;
    c.f = f;
    if ((c.u & 0x7F800000u) == 0x7F800000u && (c.u & 0x007FFFFFu)) return (bf16)((c.u >> 16) | 0x40u);
    const uint32_t r = c.u + 0x7FFFu + ((c.u >> 16) & 1u);
    return (bf16)(r >> 16);
}

constexpr int THREADS = 256;

// Eight channels (16 bytes) at a time: every channel count is a multiple of 16.
struct bf8 {
    uint4 v;
    __device__ float get(int q) const { return bf2f(((const bf16*)&v)[q]); }
    __device__ void set(int q, float f) { ((bf16*)&v)[q] = f2bf(f); }
};
__device__ inline bf8 ld8(const bf16* p) { return bf8{*(const uint4*)p}; }
__device__ inline void st8(bf16* p, const bf8& x) { *(uint4*)p = x.v; }

// ---------------------------------------------------------------------------------------
// 3x3 convolution, forward, LDS-tiled: a workgroup computes CT_BM = 128 output pixels x BN
// output channels.  K (9 taps x Cin) is walked in steps of KC channels of one tap; each step
// stages the 128 x KC slice of the input patches and the BN x KC slice of the weights in LDS
// (the next step's slices are fetched into registers while the current ones are multiplied),
// and each wave multiplies 32 pixels x BN channels on MFMA 16x16x16.  Rows of the LDS tiles
// are padded by 8 elements (16 bytes) to spread the fragment reads over the banks.
// ---------------------------------------------------------------------------------------
constexpr int CT_BM = 128;

template <int BN, int KC, bool RELU, bool OUT_F32>
__global__ __launch_bounds__(THREADS) void k_conv_tile(const bf16* __restrict__ in, const bf16* __restrict__ W,
                                                       const float* __restrict__ bias, void* __restrict__ out, int P,
                                                       int H, int Wd, int Cin, int Cout)
{
    constexpr int AROW = KC + 8;
    constexpr int PPR = KC / 8;                                   // 16-byte pieces per row
    constexpr int AP = (CT_BM * PPR + THREADS - 1) / THREADS;     // A pieces per thread
    constexpr int BPIECES = BN * PPR;
    constexpr int BPT = (BPIECES + THREADS - 1) / THREADS;        // B pieces per thread
    constexpr int NJ = BN / 16;
    __shared__ __attribute__((aligned(16))) bf16 As[CT_BM * AROW];
    __shared__ __attribute__((aligned(16))) bf16 Bs[BN * AROW];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int m = l & 15, kq = l >> 4;
    const int p0 = blockIdx.x * CT_BM;
    const int co0 = blockIdx.y * BN;
    const int K = 9 * Cin;
    const int hw = H * Wd;

    // the pieces this thread moves: A (pixel row, channel offset), B (channel row, offset)
    int arow[AP], acol[AP], an[AP], ay[AP], ax[AP];
    bool aok[AP];
#pragma unroll
    for (int i = 0; i < AP; ++i) {
        const int idx = t + i * THREADS;
        arow[i] = idx / PPR;
        acol[i] = (idx % PPR) * 8;
        const int p = p0 + arow[i];
        aok[i] = idx < CT_BM * PPR && p < P;
        const int pp = aok[i] ? p : 0;
        an[i] = pp / hw;
        const int rem = pp - an[i] * hw;
        ay[i] = rem / Wd;
        ax[i] = rem - ay[i] * Wd;
    }
    int brow[BPT], bcol[BPT];
    bool bok[BPT];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int idx = t + i * THREADS;
        bok[i] = idx < BPIECES;
        brow[i] = bok[i] ? idx / PPR : 0;
        bcol[i] = (idx % PPR) * 8;
    }
    uint4 ra[AP], rb[BPT];
    auto fetch = [&](int step) {
        const int tap = step / (Cin / KC), c0 = (step % (Cin / KC)) * KC;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
#pragma unroll
        for (int i = 0; i < AP; ++i) {
            const int yy = ay[i] + dy, xx = ax[i] + dx;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (aok[i] && yy >= 0 && yy < H && xx >= 0 && xx < Wd)
                v = *(const uint4*)(in + ((int64_t)(an[i] * H + yy) * Wd + xx) * Cin + c0 + acol[i]);
            ra[i] = v;
        }
#pragma unroll
        for (int i = 0; i < BPT; ++i)
            if (bok[i]) rb[i] = *(const uint4*)(W + (int64_t)(co0 + brow[i]) * K + tap * Cin + c0 + bcol[i]);
    };
    auto stash = [&]() {
#pragma unroll
        for (int i = 0; i < AP; ++i)
            if (t + i * THREADS < CT_BM * PPR) *(uint4*)(As + arow[i] * AROW + acol[i]) = ra[i];
#pragma unroll
        for (int i = 0; i < BPT; ++i)
            if (bok[i]) *(uint4*)(Bs + brow[i] * AROW + bcol[i]) = rb[i];
    };

    v4f acc[2][NJ];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    const int nsteps = 9 * (Cin / KC);
    fetch(0);
    for (int st = 0; st < nsteps; ++st) {
        stash();
        __syncthreads();
        if (st + 1 < nsteps) fetch(st + 1);
#pragma unroll
        for (int k0 = 0; k0 < KC; k0 += 16) {
            v4s b[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) b[j] = *(const v4s*)(Bs + (16 * j + m) * AROW + k0 + 4 * kq);
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const v4s a = *(const v4s*)(As + (32 * w + 16 * i + m) * AROW + k0 + 4 * kq);
#pragma unroll
                for (int j = 0; j < NJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int co = co0 + 16 * j + m;
        const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int po = p0 + 32 * w + 16 * i + 4 * kq + e;
                if (po >= P) continue;
                float v = acc[i][j][e] + bv;
                if (RELU) v = fmaxf(v, 0.0f);
                if (OUT_F32) ((float*)out)[(int64_t)po * Cout + co] = v;
                else ((bf16*)out)[(int64_t)po * Cout + co] = f2bf(v);
            }
    }
}

// four pixels' value of one channel, packed for one LDS store
__device__ inline uint2 pack4(const uint4 v[4], int q)
{
    const bf16 e0 = ((const bf16*)&v[0])[q], e1 = ((const bf16*)&v[1])[q];
    const bf16 e2 = ((const bf16*)&v[2])[q], e3 = ((const bf16*)&v[3])[q];
    return make_uint2((uint32_t)e0 | ((uint32_t)e1 << 16), (uint32_t)e2 | ((uint32_t)e3 << 16));
}

// ---------------------------------------------------------------------------------------
// The same two products on gfx950's MFMA 16x16x32 (bf16), for channel counts that are multiples
// of 32.  Lane l supplies A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16], i < 8 (16
// bytes each, one LDS read), and holds D[4 (l / 16) + i][l % 16], i < 4.
// ---------------------------------------------------------------------------------------
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ inline v4f mfma32(const bf16* a, const bf16* b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(*(const v8bf*)a, *(const v8bf*)b, c, 0, 0, 0);
}

// 3x3 convolution, forward (and data gradient with flipped weights), Cin a multiple of 32: a
// workgroup computes an 8 x 32 pixel tile of one image x BN output channels; wave w takes tile
// rows 2w and 2w + 1 (four 16-pixel MFMA row tiles).  Per chunk of 32 input channels it stages
// the tile's 10 x 34 halo of inputs (zero outside the image) and the chunk's weights of all nine
// taps in LDS once, then runs the nine taps from LDS (each tap's A fragment is the halo shifted
// by the tap), so every input is fetched once per chunk instead of once per tap.  LDS rows are
// padded by 8 elements (16 bytes).  The output-channel tiles of one pixel tile run on the same
// XCD one after another (consecutive workgroups go to the eight XCDs in turn), so the tile's
// inputs come from that XCD's L2 after the first.
constexpr int HT_Y = 8, HT_X = 32;
constexpr int HT_HY = HT_Y + 2, HT_HX = HT_X + 2;
constexpr int HT_ROW = 32 + 8;

template <int BN, bool RELU, bool OUT_F32>
__global__ __launch_bounds__(THREADS) void k_conv_halo(const bf16* __restrict__ in, const bf16* __restrict__ W,
                                                       const float* __restrict__ bias, void* __restrict__ out, int H,
                                                       int Wd, int Cin, int Cout, int ntiles)
{
    const int nct = Cout / BN;
    const int xcd = (int)blockIdx.x & 7, rr = (int)blockIdx.x >> 3;
    const int ptile = (rr / nct) * 8 + xcd;
    if (ptile >= ntiles) return;
    constexpr int NJ = BN / 16;
    constexpr int APIECES = HT_HY * HT_HX * 4;                      // 16-byte pieces of the halo
    constexpr int BPIECES = 9 * BN * 4;
    __shared__ __attribute__((aligned(16))) bf16 As[HT_HY * HT_HX * HT_ROW];
    __shared__ __attribute__((aligned(16))) bf16 Bs[9 * BN * HT_ROW];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int m = l & 15, kq = l >> 4;
    const int tx_n = (Wd + HT_X - 1) / HT_X, ty_n = (H + HT_Y - 1) / HT_Y;
    const int img = ptile / (tx_n * ty_n);
    const int tr = ptile - img * tx_n * ty_n;
    const int y0 = (tr / tx_n) * HT_Y, x0 = (tr % tx_n) * HT_X;
    const int co0 = (rr % nct) * BN;
    const int K = 9 * Cin;
    const bf16* src = in + (int64_t)img * H * Wd * Cin;

    // the chunk's pieces this thread moves: all loads of a chunk are issued before any is
    // stored, and the next chunk's while the current one multiplies
    constexpr int AT = (APIECES + THREADS - 1) / THREADS;
    constexpr int BT = (BPIECES + THREADS - 1) / THREADS;
    uint4 ra[AT], rb[BT];
    auto fetch = [&](int c0) {
#pragma unroll
        for (int q = 0; q < AT; ++q) {
            const int pc = t + q * THREADS;
            const int hp = pc >> 2, c8 = (pc & 3) * 8;
            const int hy = hp / HT_HX, hx = hp - hy * HT_HX;
            const int y = y0 + hy - 1, x = x0 + hx - 1;
            ra[q] = make_uint4(0u, 0u, 0u, 0u);
            if (pc < APIECES && y >= 0 && y < H && x >= 0 && x < Wd)
                ra[q] = *(const uint4*)(src + ((int64_t)y * Wd + x) * Cin + c0 + c8);
        }
#pragma unroll
        for (int q = 0; q < BT; ++q) {
            const int pc = t + q * THREADS;
            const int r = pc >> 2, c8 = (pc & 3) * 8;                // r = tap * BN + co
            const int tap = r / BN, co = r - tap * BN;
            rb[q] = make_uint4(0u, 0u, 0u, 0u);
            if (pc < BPIECES) rb[q] = *(const uint4*)(W + (int64_t)(co0 + co) * K + tap * Cin + c0 + c8);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < AT; ++q) {
            const int pc = t + q * THREADS;
            if (pc < APIECES) *(uint4*)(As + (pc >> 2) * HT_ROW + (pc & 3) * 8) = ra[q];
        }
#pragma unroll
        for (int q = 0; q < BT; ++q) {
            const int pc = t + q * THREADS;
            if (pc < BPIECES) *(uint4*)(Bs + (pc >> 2) * HT_ROW + (pc & 3) * 8) = rb[q];
        }
    };

    v4f acc[4][NJ];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    fetch(0);
    for (int c0 = 0; c0 < Cin; c0 += 32) {
        stash();
        __syncthreads();
        if (c0 + 32 < Cin) fetch(c0 + 32);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int hp = (2 * w + (i >> 1) + dy) * HT_HX + 16 * (i & 1) + m + dx;
                const bf16* a = As + hp * HT_ROW + 8 * kq;
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    acc[i][j] = mfma32(a, Bs + (tap * BN + 16 * j + m) * HT_ROW + 8 * kq, acc[i][j]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int co = co0 + 16 * j + m;
        const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int y = y0 + 2 * w + (i >> 1);
            if (y >= H) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = x0 + 16 * (i & 1) + 4 * kq + e;
                if (x >= Wd) continue;
                float v = acc[i][j][e] + bv;
                if (RELU) v = fmaxf(v, 0.0f);
                const int64_t po = ((int64_t)img * H + y) * Wd + x;
                if (OUT_F32) ((float*)out)[po * Cout + co] = v;
                else ((bf16*)out)[po * Cout + co] = f2bf(v);
            }
        }
    }
}

// weight gradient on MFMA 16x16x32: dW[co][k] += sum_p dZ[p][co] patch[p][k] for a tile of BM
// output channels x BK values of k over a chunk of pixels, PX pixels per step.  Both operands
// are staged transposed ([co][pixel], [k][pixel]) so that a lane's fragment is eight
// consecutive pixels; a staging piece is 4 pixels x 8 channels (four 16-byte loads, eight
// 8-byte LDS stores), the threads take the step's pieces in turn, and the next step's pieces
// are loaded while the current step multiplies.  Wave w owns k values [w BK / 4, (w + 1) BK / 4).
// Chunks of pixels are added atomically.  The first k tile also sums the bias gradient
// db[co] += sum_p dZ[p][co].  Workgroups are dealt so that all (k, co) tiles of one pixel chunk
// run on the same XCD one after another (the GPU deals consecutive workgroups to its eight
// XCDs in turn): the chunk's inputs and gradients then come from that XCD's L2 after the
// first tile, not again from HBM.
// ROWS: the image width is a multiple of PX and chunks hold whole PX-pixel row segments, so a
// step's image and row are the same for the whole workgroup and a pixel's address is a row base
// plus its column (the general form tracks every pixel's image, row and column).
template <int BM, int BK, int PX, bool ROWS>
__global__ __launch_bounds__(THREADS) void k_wgrad_m32(const bf16* __restrict__ in, const bf16* __restrict__ dZ,
                                                       float* __restrict__ dW, float* __restrict__ db, int P, int H,
                                                       int Wd, int Cin, int Cout, int chunk, int nkt, int tiles,
                                                       int nchunk)
{
    __shared__ float bred[THREADS];
    const int xcd = (int)blockIdx.x & 7, r = (int)blockIdx.x >> 3;
    const int tile = r % tiles, ch = (r / tiles) * 8 + xcd;
    if (ch >= nchunk) return;
    const int kt = tile % nkt, ct = tile / nkt;
    constexpr int PR = PX + 8;                                         // padded LDS row (pixels)
    constexpr int NI = BM / 16;
    constexpr int NJ = BK / 64;                                        // 16-wide k tiles per wave
    constexpr int PA = (PX / 4) * (BM / 8);                            // dZ pieces
    constexpr int PB = (PX / 4) * (BK / 8);                            // patch pieces
    constexpr int PT = (PA + PB + THREADS - 1) / THREADS;
    __shared__ __attribute__((aligned(16))) bf16 At[BM * PR];          // dZ^T
    __shared__ __attribute__((aligned(16))) bf16 Bt[BK * PR];          // patch^T
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int m = l & 15, kq = l >> 4;
    const int K = 9 * Cin;
    const int k0 = kt * BK, co0 = ct * BM;
    const int pbeg = ch * chunk, pend = min(P, pbeg + chunk);
    const int hw = H * Wd;
    v4f acc[NI][NJ];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    const bool bias_tile = kt == 0;
    // this thread's pieces: kind (0 dZ, 1 patch, 2 patch beyond K, -1 none), first pixel of the
    // four, first channel (dZ) or k (patch), and the patch's tap offsets and input channel
    // Piece order within each operand: four channel groups (64 contiguous bytes of one pixel)
    // fastest, then the PX / 4 pixel quads, then the remaining channel groups.  A store
    // instruction then writes four rows eight apart (two bank halves) x 16 pixel quads (128
    // bytes): every bank twice, no conflicts; a load instruction reads whole 64-byte segments.
    auto piece = [](int pc, int groups, int& quad, int& c8) {
        const int lo = groups < 4 ? groups : 4;
        const int rest = pc / lo;
        quad = (rest % (PX / 4)) * 4;
        c8 = ((rest / (PX / 4)) * lo + pc % lo) * 8;
    };
    int kind[PT], px4[PT], cp[PT], dyo[PT], dxo[PT], ci[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        const int pc = t + q * THREADS;
        kind[q] = -1;
        px4[q] = cp[q] = dyo[q] = dxo[q] = ci[q] = 0;
        if (pc < PA) {
            kind[q] = 0;
            piece(pc, BM / 8, px4[q], cp[q]);
        } else if (pc < PA + PB) {
            const int pb = pc - PA;
            piece(pb, BK / 8, px4[q], cp[q]);
            kind[q] = 2;
            if (k0 + cp[q] < K) {
                kind[q] = 1;
                const int tap = (k0 + cp[q]) / Cin;
                ci[q] = k0 + cp[q] - tap * Cin;
                dyo[q] = tap / 3 - 1;
                dxo[q] = tap % 3 - 1;
            }
        }
    }
    // image, row and column of each patch piece's first pixel, advanced by PX pixels per step
    // (no division inside the loop)
    int pn[PT], py[PT], pxx[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        const int p = pbeg + px4[q];
        pn[q] = p / hw;
        const int rem = p - pn[q] * hw;
        py[q] = rem / Wd;
        pxx[q] = rem - py[q] * Wd;
    }
    uint4 v[PT][4];
    // row-segment form: the step's segment starts at pixel pb; (image row, first column) of it
    int srow = pbeg / Wd, scol = pbeg - srow * Wd;
    auto fetch_rows = [&](int pb) {
        const int n = srow / H, y = srow - n * H;
#pragma unroll
        for (int q = 0; q < PT; ++q) {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[q][j] = make_uint4(0u, 0u, 0u, 0u);
            if (kind[q] == 0) {
                const bf16* r = dZ + (int64_t)(pb + px4[q]) * Cout + co0 + cp[q];
                if (pb < pend)
#pragma unroll
                    for (int j = 0; j < 4; ++j) v[q][j] = *(const uint4*)(r + (int64_t)j * Cout);
            } else if (kind[q] == 1) {
                const int yy = y + dyo[q];
                if (pb < pend && yy >= 0 && yy < H) {
                    const bf16* r = in + (int64_t)(n * H + yy) * Wd * Cin + ci[q];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int xx = scol + px4[q] + j + dxo[q];
                        if (xx >= 0 && xx < Wd) v[q][j] = *(const uint4*)(r + xx * Cin);
                    }
                }
            }
        }
        scol += PX;
        if (scol == Wd) {
            scol = 0;
            ++srow;
        }
    };
    auto fetch = [&](int pb) {
        if constexpr (ROWS) {
            fetch_rows(pb);
            return;
        }
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            int n = pn[q], y = py[q], x = pxx[q];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[q][j] = make_uint4(0u, 0u, 0u, 0u);
                const int p = pb + px4[q] + j;
                if (p < pend) {
                    if (kind[q] == 0) {
                        v[q][j] = *(const uint4*)(dZ + (int64_t)p * Cout + co0 + cp[q]);
                    } else if (kind[q] == 1) {
                        const int yy = y + dyo[q], xx = x + dxo[q];
                        if (yy >= 0 && yy < H && xx >= 0 && xx < Wd)
                            v[q][j] = *(const uint4*)(in + ((int64_t)(n * H + yy) * Wd + xx) * Cin + ci[q]);
                    }
                }
                if (++x == Wd) {
                    x = 0;
                    if (++y == H) {
                        y = 0;
                        ++n;
                    }
                }
            }
            // the next step's first pixel: PX on from this one
            int xx = pxx[q] + PX;
            while (xx >= Wd) {
                xx -= Wd;
                if (++py[q] == H) {
                    py[q] = 0;
                    ++pn[q];
                }
            }
            pxx[q] = xx;
        }
    };
    if constexpr (ROWS) (void)pn, (void)py, (void)pxx;
    fetch(pbeg);
    for (int pb = pbeg; pb < pend; pb += PX) {
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            if (kind[q] < 0) continue;
            bf16* dst = kind[q] == 0 ? At + cp[q] * PR + px4[q] : Bt + cp[q] * PR + px4[q];
#pragma unroll
            for (int c = 0; c < 8; ++c) *(uint2*)(dst + c * PR) = pack4(v[q], c);
        }
        __syncthreads();
        if (pb + PX < pend) fetch(pb + PX);
        if (bias_tile) {
            // NSEG threads per channel, each adding SEG pixels (a multiple of eight: one LDS read
            // per eight)
            constexpr int NSEG = (PX / 8) < (THREADS / BM) ? (PX / 8) : (THREADS / BM);
            constexpr int SEG = PX / NSEG;
            if (t / BM < NSEG) {
                const bf16* r = At + (t % BM) * PR + (t / BM) * SEG;
#pragma unroll
                for (int q = 0; q < SEG; q += 8) {
                    const bf8 x = ld8(r + q);
#pragma unroll
                    for (int e = 0; e < 8; ++e) bsum += x.get(e);
                }
            }
        }
#pragma unroll
        for (int r0 = 0; r0 < PX; r0 += 32) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const bf16* b = Bt + (w * (BK / 4) + 16 * j + m) * PR + r0 + 8 * kq;
#pragma unroll
                for (int i = 0; i < NI; ++i) acc[i][j] = mfma32(At + (16 * i + m) * PR + r0 + 8 * kq, b, acc[i][j]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int k = k0 + w * (BK / 4) + 16 * j + m;
        if (k < K)
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int co = co0 + 16 * i + 4 * kq + e;
                    if (acc[i][j][e] != 0.0f) atomicAdd(&dW[(int64_t)co * K + k], acc[i][j][e]);
                }
    }
    if (bias_tile) {
        // the THREADS / BM segments of each channel, added in segment order
        bred[t] = bsum;
        __syncthreads();
        if (t < BM) {
            float b = 0.0f;
            for (int sgm = 0; sgm < THREADS / BM; ++sgm) b += bred[sgm * BM + t];
            if (b != 0.0f) atomicAdd(&db[co0 + t], b);
        }
    }
}

// ---------------------------------------------------------------------------------------
// elementwise pieces
// ---------------------------------------------------------------------------------------
// inputs [B][H][W][8] float -> [B][H][W][16] bf16 (channels 8..15 zero)
__global__ void k_pack_input(const float* __restrict__ src, bf16* __restrict__ dst, int64_t npix)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * 16) return;
    const int64_t p = i >> 4;
    const int c = (int)(i & 15);
    dst[i] = c < 8 ? f2bf(src[p * 8 + c]) : (bf16)0;
}


// 2x2 average pool: [B][H][W][C] -> [B][H/2][W/2][C]
__global__ void k_pool(const bf16* __restrict__ in, bf16* __restrict__ out, int B, int H, int Wd, int C)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int h2 = H / 2, w2 = Wd / 2, C8 = C / 8;
    if (i >= (int64_t)B * h2 * w2 * C8) return;
    const int c = (int)(i % C8) * 8;
    const int64_t q = i / C8;
    const int x = (int)(q % w2), y = (int)((q / w2) % h2), n = (int)(q / ((int64_t)w2 * h2));
    const bf16* s = in + ((int64_t)(n * H + 2 * y) * Wd + 2 * x) * C + c;
    const bf8 a = ld8(s), b = ld8(s + C), d = ld8(s + (int64_t)Wd * C), e = ld8(s + (int64_t)Wd * C + C);
    bf8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o.set(k, 0.25f * ((a.get(k) + b.get(k)) + (d.get(k) + e.get(k))));
    st8(out + q * C + c, o);
}

// gradient of the pool: dIn (+)= dOut / 4 at the four inputs
__global__ void k_pool_bwd(const bf16* __restrict__ dout, bf16* __restrict__ din, int B, int H, int Wd, int C, int add)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int C8 = C / 8;
    if (i >= (int64_t)B * H * Wd * C8) return;
    const int c = (int)(i % C8) * 8;
    const int64_t q = i / C8;
    const int x = (int)(q % Wd), y = (int)((q / Wd) % H), n = (int)(q / ((int64_t)Wd * H));
    const bf8 g = ld8(dout + ((int64_t)(n * (H / 2) + y / 2) * (Wd / 2) + x / 2) * C + c);
    bf8 o{make_uint4(0u, 0u, 0u, 0u)};
    if (add) o = ld8(din + q * C + c);
#pragma unroll
    for (int k = 0; k < 8; ++k) o.set(k, 0.25f * g.get(k) + (add ? o.get(k) : 0.0f));
    st8(din + q * C + c, o);
}

// nearest 2x upsample: [B][H][W][C] -> [B][2H][2W][C]
__global__ void k_up(const bf16* __restrict__ in, bf16* __restrict__ out, int B, int H, int Wd, int C)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int H2 = 2 * H, W2 = 2 * Wd, C8 = C / 8;
    if (i >= (int64_t)B * H2 * W2 * C8) return;
    const int c = (int)(i % C8) * 8;
    const int64_t q = i / C8;
    const int x = (int)(q % W2), y = (int)((q / W2) % H2), n = (int)(q / ((int64_t)W2 * H2));
    st8(out + q * C + c, ld8(in + ((int64_t)(n * H + y / 2) * Wd + x / 2) * C + c));
}

// gradient of the upsample: dIn = sum of the four dOut
__global__ void k_up_bwd(const bf16* __restrict__ dout, bf16* __restrict__ din, int B, int H, int Wd, int C)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int C8 = C / 8;
    if (i >= (int64_t)B * H * Wd * C8) return;
    const int c = (int)(i % C8) * 8;
    const int64_t q = i / C8;
    const int x = (int)(q % Wd), y = (int)((q / Wd) % H), n = (int)(q / ((int64_t)Wd * H));
    const int64_t W2 = 2 * Wd;
    const bf16* s = dout + ((int64_t)(n * 2 * H + 2 * y) * W2 + 2 * x) * C + c;
    const bf8 a = ld8(s), b = ld8(s + C), d = ld8(s + W2 * C), e = ld8(s + W2 * C + C);
    bf8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o.set(k, (a.get(k) + b.get(k)) + (d.get(k) + e.get(k)));
    st8(din + q * C + c, o);
}

// n8: number of eight-channel groups
__global__ void k_add(const bf16* __restrict__ a, const bf16* __restrict__ b, bf16* __restrict__ out, int64_t n8)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const bf8 x = ld8(a + 8 * i), y = ld8(b + 8 * i);
    bf8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o.set(k, x.get(k) + y.get(k));
    st8(out + 8 * i, o);
}

// dZ = dY * [Y > 0]
__global__ void k_relu_bwd(const bf16* __restrict__ dy, const bf16* __restrict__ y, bf16* __restrict__ dz, int64_t n8)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const bf8 g = ld8(dy + 8 * i), v = ld8(y + 8 * i);
    bf8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) ((bf16*)&o.v)[k] = v.get(k) > 0.0f ? ((const bf16*)&g.v)[k] : (bf16)0;
    st8(dz + 8 * i, o);
}

// weights for the data gradient: Wf[ci][tap * Cout + co] = W[co][(8 - tap) * Cin + ci]
__global__ void k_flip(const bf16* __restrict__ W, bf16* __restrict__ Wf, int Cin, int Cout)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)9 * Cin * Cout) return;
    const int ci = (int)(i / (9 * Cout));
    const int r = (int)(i - (int64_t)ci * 9 * Cout);
    const int tap = r / Cout, co = r - tap * Cout;
    Wf[i] = W[(int64_t)co * 9 * Cin + (8 - tap) * Cin + ci];
}

// mean squared error of channel 0 of pred [npix][16] against tgt [npix]; dPred [npix][16]
// (bf16, channels 1..15 zero) and per-block partial sums of the squared error
__global__ __launch_bounds__(THREADS) void k_mse(const float* __restrict__ pred, const float* __restrict__ tgt,
                                                 bf16* __restrict__ dpred, double* __restrict__ part, int64_t npix,
                                                 float scale)
{
    __shared__ double sh[THREADS];
    const int64_t i = (int64_t)blockIdx.x * THREADS + threadIdx.x;
    double e2 = 0.0;
    if (i < npix) {
        const float d = pred[i * 16] - tgt[i];
        e2 = (double)d * d;
        dpred[i * 16] = f2bf(2.0f * d * scale);
        for (int c = 1; c < 16; ++c) dpred[i * 16 + c] = 0;
    }
    sh[threadIdx.x] = e2;
    __syncthreads();
    for (int w = THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_take_ch0(const float* __restrict__ pred, float* __restrict__ out, int64_t npix)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npix) out[i] = pred[i * 16];
}

// Adam on FP32 master weights; the BF16 copy used by the forward pass follows
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, bf16* __restrict__ wb, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float v = w[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    w[i] = v;
    if (wb) wb[i] = f2bf(v);
}

__global__ void k_to_bf16(const float* __restrict__ w, bf16* __restrict__ wb, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = f2bf(w[i]);
}

__global__ void k_zero_f32(float* __restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

inline unsigned nblk(int64_t n, int t = THREADS) { return (unsigned)((n + t - 1) / t); }

}  // namespace net
}  // namespace lbib

// =======================================================================================
// the network object
// =======================================================================================
using namespace lbib::net;

namespace {

constexpr int NL = 15;
// (Cin, Cout, resolution divisor) of the 15 convolutions, in order
const int LAYER_CIN[NL] = {16, 32, 32, 64, 64, 128, 128, 256, 256, 128, 128, 64, 64, 32, 32};
const int LAYER_COUT[NL] = {32, 32, 64, 64, 128, 128, 256, 256, 128, 128, 64, 64, 32, 32, 16};
const int LAYER_DIV[NL] = {1, 1, 2, 2, 4, 4, 8, 8, 4, 4, 2, 2, 1, 1, 1};

}  // namespace

struct lbib_net {
    int H = 0, Wd = 0, maxB = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int64_t nparam = 0;
    int64_t woff[NL], boff[NL];            // offsets of W_l and b_l in the packed parameters
    float *w32 = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
    bf16* wbf = nullptr;                    // BF16 copy (biases included, unused)
    bf16* wflip = nullptr;                  // scratch for the flipped weights of one layer
    int64_t adam_t = 0;
    // activations (B max) and their gradients
    bf16* act[40] = {};
    bf16* gr[40] = {};
    float* pred = nullptr;                  // [B][H][W][16]
    double* part = nullptr;
    std::vector<void*> allocs;
};

namespace {

// activation slots
enum {
    X0, A0, S0, P0, A1, S1, P1, A2, S2, P2, A3, B3, U3, R8, U2, V2, UP2, R10, U1, V1, UP1, R12, U0, V0, NACT
};

struct Shape {
    int div, C;
};
const Shape ACT_SHAPE[NACT] = {
    {1, 16}, {1, 32}, {1, 32}, {2, 32}, {2, 64}, {2, 64}, {4, 64}, {4, 128}, {4, 128}, {8, 128}, {8, 256}, {8, 256},
    {4, 256}, {4, 128}, {4, 128}, {4, 128}, {2, 128}, {2, 64}, {2, 64}, {2, 64}, {1, 64}, {1, 32}, {1, 32}, {1, 32}};

int64_t act_elems(const lbib_net* n, int s, int B)
{
    const int64_t h = n->H / ACT_SHAPE[s].div, w = n->Wd / ACT_SHAPE[s].div;
    return (int64_t)B * h * w * ACT_SHAPE[s].C;
}

template <typename T>
bool nalloc(lbib_net* n, T** p, size_t count)
{
    if (hipMalloc((void**)p, (count ? count : 1) * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return false;
    }
    n->allocs.push_back((void*)*p);
    return true;
}

#define NET_K(call)                                       \
    do {                                                  \
        call;                                             \
        if (hipGetLastError() != hipSuccess) return false; \
    } while (0)

template <int BN, int KC>
bool conv_tile(hipStream_t s, const bf16* in, void* out, bool relu, bool out_f32, const bf16* W, const float* bias,
               int P, int H, int Wd, int Cin, int Cout)
{
    const dim3 grid((unsigned)((P + CT_BM - 1) / CT_BM), (unsigned)(Cout / BN));
    if (out_f32) {
        NET_K(hipLaunchKernelGGL((k_conv_tile<BN, KC, false, true>), grid, dim3(THREADS), 0, s, in, W, bias, out, P, H, Wd,
                                 Cin, Cout));
    } else if (relu) {
        NET_K(hipLaunchKernelGGL((k_conv_tile<BN, KC, true, false>), grid, dim3(THREADS), 0, s, in, W, bias, out, P, H, Wd,
                                 Cin, Cout));
    } else {
        NET_K(hipLaunchKernelGGL((k_conv_tile<BN, KC, false, false>), grid, dim3(THREADS), 0, s, in, W, bias, out, P, H,
                                 Wd, Cin, Cout));
    }
    return true;
}

template <int BN>
bool conv_halo(hipStream_t s, const bf16* in, void* out, bool relu, bool out_f32, const bf16* W, const float* bias,
               int B, int H, int Wd, int Cin, int Cout)
{
    const int ntiles = B * ((H + HT_Y - 1) / HT_Y) * ((Wd + HT_X - 1) / HT_X);
    const dim3 grid((unsigned)((ntiles + 7) / 8 * 8 * (Cout / BN)));
    if (out_f32) {
        NET_K(hipLaunchKernelGGL((k_conv_halo<BN, false, true>), grid, dim3(THREADS), 0, s, in, W, bias, out, H, Wd,
                                 Cin, Cout, ntiles));
    } else if (relu) {
        NET_K(hipLaunchKernelGGL((k_conv_halo<BN, true, false>), grid, dim3(THREADS), 0, s, in, W, bias, out, H, Wd,
                                 Cin, Cout, ntiles));
    } else {
        NET_K(hipLaunchKernelGGL((k_conv_halo<BN, false, false>), grid, dim3(THREADS), 0, s, in, W, bias, out, H, Wd,
                                 Cin, Cout, ntiles));
    }
    return true;
}

// Cin and Cout are multiples of 16 (the activations' channel counts); Cin a multiple of 32 takes
// the halo-tiled MFMA 16x16x32 kernel
bool conv_fwd(lbib_net* n, int l, const bf16* in, void* out, int B, bool relu, bool out_f32, const bf16* W,
              const float* bias, int Cin, int Cout)
{
    const int div = LAYER_DIV[l];
    const int H = n->H / div, Wd = n->Wd / div;
    const int P = B * H * Wd;
    hipStream_t s = n->stream;
    if (Cin % 32 == 0) {
        if (Cout % 64 == 0) return conv_halo<64>(s, in, out, relu, out_f32, W, bias, B, H, Wd, Cin, Cout);
        if (Cout % 32 == 0) return conv_halo<32>(s, in, out, relu, out_f32, W, bias, B, H, Wd, Cin, Cout);
        return conv_halo<16>(s, in, out, relu, out_f32, W, bias, B, H, Wd, Cin, Cout);
    }
    const bool k32 = Cin % 32 == 0;
    if (Cout % 64 == 0) return k32 ? conv_tile<64, 32>(s, in, out, relu, out_f32, W, bias, P, H, Wd, Cin, Cout)
                                   : conv_tile<64, 16>(s, in, out, relu, out_f32, W, bias, P, H, Wd, Cin, Cout);
    if (Cout % 32 == 0) return k32 ? conv_tile<32, 32>(s, in, out, relu, out_f32, W, bias, P, H, Wd, Cin, Cout)
                                   : conv_tile<32, 16>(s, in, out, relu, out_f32, W, bias, P, H, Wd, Cin, Cout);
    return k32 ? conv_tile<16, 32>(s, in, out, relu, out_f32, W, bias, P, H, Wd, Cin, Cout)
               : conv_tile<16, 16>(s, in, out, relu, out_f32, W, bias, P, H, Wd, Cin, Cout);
}

const bf16* WB(lbib_net* n, int l) { return n->wbf + n->woff[l]; }
const float* BIAS(lbib_net* n, int l) { return n->w32 + n->boff[l]; }

bool forward(lbib_net* n, const float* inputs, int B)
{
    hipStream_t s = n->stream;
    const int64_t npix = (int64_t)B * n->H * n->Wd;
    auto A = [&](int k) { return n->act[k]; };
    NET_K(hipLaunchKernelGGL(k_pack_input, dim3(nblk(npix * 16)), dim3(THREADS), 0, s, inputs, A(X0), npix));
    auto conv = [&](int l, int in, int out, bool relu) {
        return conv_fwd(n, l, A(in), A(out), B, relu, false, WB(n, l), BIAS(n, l), LAYER_CIN[l], LAYER_COUT[l]);
    };
    auto pool = [&](int in, int out) {
        const int div = ACT_SHAPE[in].div;
        hipLaunchKernelGGL(k_pool, dim3(nblk(act_elems(n, out, B) / 8)), dim3(THREADS), 0, s, A(in), A(out), B,
                           n->H / div, n->Wd / div, ACT_SHAPE[in].C);
        return hipGetLastError() == hipSuccess;
    };
    auto up = [&](int in, int out) {
        const int div = ACT_SHAPE[in].div;
        hipLaunchKernelGGL(k_up, dim3(nblk(act_elems(n, out, B) / 8)), dim3(THREADS), 0, s, A(in), A(out), B,
                           n->H / div, n->Wd / div, ACT_SHAPE[in].C);
        return hipGetLastError() == hipSuccess;
    };
    auto add = [&](int a, int b, int out) {
        hipLaunchKernelGGL(k_add, dim3(nblk(act_elems(n, out, B) / 8)), dim3(THREADS), 0, s, A(a), A(b), A(out),
                           act_elems(n, out, B) / 8);
        return hipGetLastError() == hipSuccess;
    };
    bool ok = conv(0, X0, A0, true) && conv(1, A0, S0, true) && pool(S0, P0) && conv(2, P0, A1, true) &&
              conv(3, A1, S1, true) && pool(S1, P1) && conv(4, P1, A2, true) && conv(5, A2, S2, true) &&
              pool(S2, P2) && conv(6, P2, A3, true) && conv(7, A3, B3, true) && up(B3, U3) &&
              conv(8, U3, R8, true) && add(R8, S2, U2) && conv(9, U2, V2, true) && up(V2, UP2) &&
              conv(10, UP2, R10, true) && add(R10, S1, U1) && conv(11, U1, V1, true) && up(V1, UP1) &&
              conv(12, UP1, R12, true) && add(R12, S0, U0) && conv(13, U0, V0, true) &&
              conv_fwd(n, 14, A(V0), n->pred, B, false, true, WB(n, 14), BIAS(n, 14), 32, 16);
    return ok;
}

// The weight-gradient tiling of layer l at batch B: output-channel and k tile sizes, pixels per
// chunk and the number of chunks (up to about 4096 workgroups in all, at least ~1024 pixels each)
struct WgradPlan {
    int BM, BK, nkt, tiles, chunk, nchunk;
    int px;                   // row-segment step (32, 64 or 128 pixels), 0: the general form
};
constexpr int WG_STEP_PX = 128;
WgradPlan wgrad_plan(const lbib_net* n, int l, int B)
{
    const int div = LAYER_DIV[l];
    const int P = B * (n->H / div) * (n->Wd / div);
    const int Cout = LAYER_COUT[l], K = 9 * LAYER_CIN[l];
    WgradPlan w;
    w.BM = Cout >= 128 ? 128 : Cout;
    // k tiles of 128 only where they divide K and the output channels fill 128-row tiles of
    // the dZ operand; elsewhere 64 (a partial last k tile multiplies zeros, and with few output
    // channels the patch staging dominates either way)
    w.BK = (K >= 576 && K % 128 == 0 && Cout > 64) ? 128 : 64;
    w.nkt = (K + w.BK - 1) / w.BK;
    w.tiles = w.nkt * (Cout / w.BM);
    const int Wd = n->Wd / div;
    w.px = Wd % 128 == 0 ? 128 : Wd % 64 == 0 ? 64 : Wd % 32 == 0 ? 32 : 0;
    const int step = w.px ? w.px : WG_STEP_PX;
    w.nchunk = std::max(1, std::min(4096 / w.tiles, (P + 1023) / 1024));
    w.chunk = (P + w.nchunk - 1) / w.nchunk;
    w.chunk = (w.chunk + step - 1) / step * step;
    w.nchunk = (P + w.chunk - 1) / w.chunk;
    return w;
}

// gradient of convolution l: given dZ (gradient of its pre-activation output) and its input,
// add to dW/db and, when din is set, write the input gradient
bool conv_bwd(lbib_net* n, int l, const bf16* in, const bf16* dz, bf16* din, int B)
{
    hipStream_t s = n->stream;
    const int div = LAYER_DIV[l];
    const int H = n->H / div, Wd = n->Wd / div, P = B * H * Wd;
    const int Cin = LAYER_CIN[l], Cout = LAYER_COUT[l], K = 9 * Cin;
    float* dW = n->grad + n->woff[l];
    float* db = n->grad + n->boff[l];
    const WgradPlan pl = wgrad_plan(n, l, B);
    const int BM = pl.BM, BK = pl.BK;
    const dim3 grid((unsigned)(pl.tiles * ((pl.nchunk + 7) / 8) * 8));
#define NET_WG(bm, bk, px, rows) NET_K(hipLaunchKernelGGL((k_wgrad_m32<bm, bk, px, rows>), grid, dim3(THREADS), 0, s, in, dz, dW, db, P, H, Wd, Cin, Cout, pl.chunk, pl.nkt, pl.tiles, pl.nchunk))
#define NET_WG_BM(bk, px, rows)                          \
    do {                                                 \
        if (BM == 128) NET_WG(128, bk, px, rows);        \
        else if (BM == 64) NET_WG(64, bk, px, rows);     \
        else if (BM == 32) NET_WG(32, bk, px, rows);     \
        else NET_WG(16, bk, px, rows);                   \
    } while (0)
#define NET_WG_BK(px, rows)                              \
    do {                                                 \
        if (BK == 128) NET_WG_BM(128, px, rows);         \
        else NET_WG_BM(64, px, rows);                    \
    } while (0)
    if (pl.px == 0) NET_WG_BK(WG_STEP_PX, false);
    else if (pl.px == 128) NET_WG_BK(128, true);
    else if (pl.px == 64) NET_WG_BK(64, true);
    else NET_WG_BK(32, true);
#undef NET_WG_BK
#undef NET_WG_BM
#undef NET_WG
    if (din) {
        NET_K(hipLaunchKernelGGL(k_flip, dim3(nblk((int64_t)9 * Cin * Cout)), dim3(THREADS), 0, s, WB(n, l), n->wflip, Cin,
                                 Cout));
        if (!conv_fwd(n, l, dz, din, B, false, false, n->wflip, nullptr, Cout, Cin)) return false;
    }
    return true;
}

bool backward(lbib_net* n, int B)
{
    hipStream_t s = n->stream;
    auto A = [&](int k) { return n->act[k]; };
    auto G = [&](int k) { return n->gr[k]; };
    auto relu_bwd = [&](int y, bf16* dy, bf16* dz) {
        const int64_t e = act_elems(n, y, B);
        hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(e / 8)), dim3(THREADS), 0, s, dy, A(y), dz, e / 8);
        return hipGetLastError() == hipSuccess;
    };
    auto up_bwd = [&](int up_out, int in_slot, bf16* dout, bf16* din) {
        const int div = ACT_SHAPE[in_slot].div;
        hipLaunchKernelGGL(k_up_bwd, dim3(nblk(act_elems(n, in_slot, B) / 8)), dim3(THREADS), 0, s, dout, din, B,
                           n->H / div, n->Wd / div, ACT_SHAPE[in_slot].C);
        (void)up_out;
        return hipGetLastError() == hipSuccess;
    };
    auto pool_bwd = [&](int in_slot, bf16* dout, bf16* din, int add) {
        const int div = ACT_SHAPE[in_slot].div;
        hipLaunchKernelGGL(k_pool_bwd, dim3(nblk(act_elems(n, in_slot, B) / 8)), dim3(THREADS), 0, s, dout, din, B,
                           n->H / div, n->Wd / div, ACT_SHAPE[in_slot].C, add);
        return hipGetLastError() == hipSuccess;
    };
    // gradient buffers: gr[k] holds d(loss)/d(act[k]); gr[NACT] is the head's dZ, gr[NACT + 1]
    // a scratch dZ of the largest size
    bf16* dz = n->gr[NACT + 1];
    bf16* dhead = n->gr[NACT];
    bool ok = true;
    // head (no activation): dZ = dPred
    ok = ok && conv_bwd(n, 14, A(V0), dhead, G(V0), B);
    // level 0 decoder
    ok = ok && relu_bwd(V0, G(V0), dz) && conv_bwd(n, 13, A(U0), dz, G(U0), B);
    // U0 = R12 + S0: both receive G(U0)
    ok = ok && relu_bwd(R12, G(U0), dz) && conv_bwd(n, 12, A(UP1), dz, G(UP1), B);
    ok = ok && up_bwd(UP1, V1, G(UP1), G(V1));
    ok = ok && relu_bwd(V1, G(V1), dz) && conv_bwd(n, 11, A(U1), dz, G(U1), B);
    ok = ok && relu_bwd(R10, G(U1), dz) && conv_bwd(n, 10, A(UP2), dz, G(UP2), B);
    ok = ok && up_bwd(UP2, V2, G(UP2), G(V2));
    ok = ok && relu_bwd(V2, G(V2), dz) && conv_bwd(n, 9, A(U2), dz, G(U2), B);
    ok = ok && relu_bwd(R8, G(U2), dz) && conv_bwd(n, 8, A(U3), dz, G(U3), B);
    ok = ok && up_bwd(U3, B3, G(U3), G(B3));
    // bottom
    ok = ok && relu_bwd(B3, G(B3), dz) && conv_bwd(n, 7, A(A3), dz, G(A3), B);
    ok = ok && relu_bwd(A3, G(A3), dz) && conv_bwd(n, 6, A(P2), dz, G(P2), B);
    // S2 gets the skip gradient G(U2) plus the pool's
    ok = ok && hipMemcpyAsync(G(S2), G(U2), act_elems(n, S2, B) * sizeof(bf16), hipMemcpyDeviceToDevice, s) == hipSuccess;
    ok = ok && pool_bwd(S2, G(P2), G(S2), 1);
    ok = ok && relu_bwd(S2, G(S2), dz) && conv_bwd(n, 5, A(A2), dz, G(A2), B);
    ok = ok && relu_bwd(A2, G(A2), dz) && conv_bwd(n, 4, A(P1), dz, G(P1), B);
    ok = ok && hipMemcpyAsync(G(S1), G(U1), act_elems(n, S1, B) * sizeof(bf16), hipMemcpyDeviceToDevice, s) == hipSuccess;
    ok = ok && pool_bwd(S1, G(P1), G(S1), 1);
    ok = ok && relu_bwd(S1, G(S1), dz) && conv_bwd(n, 3, A(A1), dz, G(A1), B);
    ok = ok && relu_bwd(A1, G(A1), dz) && conv_bwd(n, 2, A(P0), dz, G(P0), B);
    ok = ok && hipMemcpyAsync(G(S0), G(U0), act_elems(n, S0, B) * sizeof(bf16), hipMemcpyDeviceToDevice, s) == hipSuccess;
    ok = ok && pool_bwd(S0, G(P0), G(S0), 1);
    ok = ok && relu_bwd(S0, G(S0), dz) && conv_bwd(n, 1, A(A0), dz, G(A0), B);
    ok = ok && relu_bwd(A0, G(A0), dz) && conv_bwd(n, 0, A(X0), dz, nullptr, B);
    return ok;
}

// loss and gradient of the current parameters on one batch; grad holds d(loss)/d(params)
bool loss_grad(lbib_net* n, const float* inputs, const float* targets, int B, double* loss)
{
    hipStream_t s = n->stream;
    if (!forward(n, inputs, B)) return false;
    const int64_t npix = (int64_t)B * n->H * n->Wd;
    const unsigned nb = nblk(npix);
    NET_K(hipLaunchKernelGGL(k_mse, dim3(nb), dim3(THREADS), 0, s, n->pred, targets, n->gr[NACT], n->part, npix,
                             1.0f / (float)npix));
    NET_K(hipLaunchKernelGGL(k_zero_f32, dim3(nblk(n->nparam)), dim3(THREADS), 0, s, n->grad, n->nparam));
    if (!backward(n, B)) return false;
    std::vector<double> h(nb);
    if (hipMemcpyAsync(h.data(), n->part, nb * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
    if (hipStreamSynchronize(s) != hipSuccess) return false;
    double t = 0.0;
    for (double v : h) t += v;
    if (loss) *loss = t / (double)npix;
    return true;
}

}  // namespace

extern "C" {

lbib_status lbib_net_create(int32_t h, int32_t w, int32_t max_batch, void* hip_stream, lbib_net** out)
{
    if (!out) return LBIB_EINVAL;
    *out = nullptr;
    if (h < 8 || w < 8 || h % 8 || w % 8 || h > 4096 || w > 4096 || max_batch < 1 || max_batch > 1024)
        return LBIB_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return LBIB_EDEVICE;
    lbib_net* n = new (std::nothrow) lbib_net();
    if (!n) return LBIB_ENOMEM;
    n->H = h;
    n->Wd = w;
    n->maxB = max_batch;
    if (hip_stream) n->stream = (hipStream_t)hip_stream;
    else {
        if (hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking) != hipSuccess) {
            delete n;
            return LBIB_EDEVICE;
        }
        n->own_stream = true;
    }
    int64_t off = 0;
    int64_t maxw = 0;
    for (int l = 0; l < NL; ++l) {
        n->woff[l] = off;
        off += (int64_t)LAYER_COUT[l] * 9 * LAYER_CIN[l];
        n->boff[l] = off;
        off += LAYER_COUT[l];
        maxw = std::max(maxw, (int64_t)LAYER_COUT[l] * 9 * LAYER_CIN[l]);
    }
    n->nparam = off;
    bool ok = nalloc(n, &n->w32, off) && nalloc(n, &n->grad, off) && nalloc(n, &n->m1, off) && nalloc(n, &n->m2, off) &&
              nalloc(n, &n->wbf, off) && nalloc(n, &n->wflip, maxw);
    int64_t maxe = 0;
    for (int k = 0; k < NACT && ok; ++k) {
        ok = nalloc(n, &n->act[k], act_elems(n, k, max_batch)) && nalloc(n, &n->gr[k], act_elems(n, k, max_batch));
        maxe = std::max(maxe, act_elems(n, k, max_batch));
    }
    const int64_t npix = (int64_t)max_batch * h * w;
    ok = ok && nalloc(n, &n->gr[NACT], npix * 16) && nalloc(n, &n->gr[NACT + 1], maxe) && nalloc(n, &n->pred, npix * 16) &&
         nalloc(n, &n->part, (size_t)nblk(npix));
    if (ok) {
        hipLaunchKernelGGL(k_zero_f32, dim3(nblk(off)), dim3(THREADS), 0, n->stream, n->w32, off);
        hipLaunchKernelGGL(k_zero_f32, dim3(nblk(off)), dim3(THREADS), 0, n->stream, n->m1, off);
        hipLaunchKernelGGL(k_zero_f32, dim3(nblk(off)), dim3(THREADS), 0, n->stream, n->m2, off);
        hipLaunchKernelGGL(k_to_bf16, dim3(nblk(off)), dim3(THREADS), 0, n->stream, n->w32, n->wbf, off);
        ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(n->stream) == hipSuccess;
    }
    if (!ok) {
        lbib_net_destroy(n);
        return LBIB_ENOMEM;
    }
    *out = n;
    return LBIB_OK;
}

void lbib_net_destroy(lbib_net* n)
{
    if (!n) return;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    for (void* p : n->allocs) (void)hipFree(p);
    if (n->own_stream) (void)hipStreamDestroy(n->stream);
    delete n;
}

lbib_status lbib_net_param_count(const lbib_net* n, int64_t* count)
{
    if (!n || !count) return LBIB_EINVAL;
    *count = n->nparam;
    return LBIB_OK;
}

lbib_status lbib_net_set_params(lbib_net* n, const float* params)
{
    if (!n || !params) return LBIB_EINVAL;
    for (int64_t i = 0; i < n->nparam; ++i)
        if (!std::isfinite(params[i])) return LBIB_EINVAL;
    if (hipMemcpyAsync(n->w32, params, n->nparam * sizeof(float), hipMemcpyHostToDevice, n->stream) != hipSuccess)
        return LBIB_EDEVICE;
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n->nparam)), dim3(THREADS), 0, n->stream, n->w32, n->wbf, n->nparam);
    hipLaunchKernelGGL(k_zero_f32, dim3(nblk(n->nparam)), dim3(THREADS), 0, n->stream, n->m1, n->nparam);
    hipLaunchKernelGGL(k_zero_f32, dim3(nblk(n->nparam)), dim3(THREADS), 0, n->stream, n->m2, n->nparam);
    n->adam_t = 0;
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(n->stream) != hipSuccess) return LBIB_EDEVICE;
    return LBIB_OK;
}

lbib_status lbib_net_get_params(lbib_net* n, float* params)
{
    if (!n || !params) return LBIB_EINVAL;
    if (hipMemcpyAsync(params, n->w32, n->nparam * sizeof(float), hipMemcpyDeviceToHost, n->stream) != hipSuccess ||
        hipStreamSynchronize(n->stream) != hipSuccess)
        return LBIB_EDEVICE;
    return LBIB_OK;
}

lbib_status lbib_net_predict(lbib_net* n, const float* inputs, int32_t B, float* out)
{
    if (!n || !inputs || !out || B < 1 || B > n->maxB) return LBIB_EINVAL;
    if (!forward(n, inputs, B)) return LBIB_EDEVICE;
    const int64_t npix = (int64_t)B * n->H * n->Wd;
    hipLaunchKernelGGL(k_take_ch0, dim3(nblk(npix)), dim3(THREADS), 0, n->stream, n->pred, out, npix);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(n->stream) != hipSuccess) return LBIB_EDEVICE;
    return LBIB_OK;
}

lbib_status lbib_net_loss_grad(lbib_net* n, const float* inputs, const float* targets, int32_t B, double* loss,
                               float* grad)
{
    if (!n || !inputs || !targets || B < 1 || B > n->maxB) return LBIB_EINVAL;
    if (!loss_grad(n, inputs, targets, B, loss)) return LBIB_EDEVICE;
    if (grad && (hipMemcpyAsync(grad, n->grad, n->nparam * sizeof(float), hipMemcpyDeviceToHost, n->stream) != hipSuccess ||
                 hipStreamSynchronize(n->stream) != hipSuccess))
        return LBIB_EDEVICE;
    return LBIB_OK;
}

lbib_status lbib_net_train_step(lbib_net* n, const float* inputs, const float* targets, int32_t B, float lr,
                                double* loss)
{
    if (!n || !inputs || !targets || B < 1 || B > n->maxB || !std::isfinite(lr) || !(lr > 0.0f)) return LBIB_EINVAL;
    if (!loss_grad(n, inputs, targets, B, loss)) return LBIB_EDEVICE;
    n->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)n->adam_t), c2 = 1.0f - std::pow(b2, (float)n->adam_t);
    hipLaunchKernelGGL(k_adam, dim3(nblk(n->nparam)), dim3(THREADS), 0, n->stream, n->w32, n->grad, n->m1, n->m2,
                       n->wbf, n->nparam, lr, b1, b2, 1e-8f, c1, c2);
    if (hipGetLastError() != hipSuccess) return LBIB_EDEVICE;
    return LBIB_OK;
}

}  // extern "C"
