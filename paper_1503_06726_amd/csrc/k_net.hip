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
// Weights are stored [Cout][9 Cin] (k contiguous).  MFMA 16x16x16 (bf16): lane l supplies
// A[l % 16][4 (l / 16) + i] and B[4 (l / 16) + i][l % 16] and holds D[4 (l / 16) + i][l % 16].
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

// ---------------------------------------------------------------------------------------
// weight gradient, LDS-tiled: dW[co][k] += sum_p dZ[p][co] patch[p][k] for a tile of BM output
// channels x 64 values of k over a chunk of pixels, 64 pixels per step.  Both operands are
// staged transposed ([co][pixel], [k][pixel]) so that a lane's MFMA fragment is four
// consecutive pixels; a staging thread moves 4 pixels x 8 channels and writes each channel's
// four pixels with one 8-byte LDS store.  Each wave owns 16 values of k.  Chunks of pixels are
// added atomically.  The first k tile also sums the bias gradient db[co] += sum_p dZ[p][co].
// ---------------------------------------------------------------------------------------
constexpr int WG_PX = 64;

// four pixels' value of one channel, packed for one LDS store
__device__ inline uint2 pack4(const uint4 v[4], int q)
{
    const bf16 e0 = ((const bf16*)&v[0])[q], e1 = ((const bf16*)&v[1])[q];
    const bf16 e2 = ((const bf16*)&v[2])[q], e3 = ((const bf16*)&v[3])[q];
    return make_uint2((uint32_t)e0 | ((uint32_t)e1 << 16), (uint32_t)e2 | ((uint32_t)e3 << 16));
}

template <int BM>
__global__ __launch_bounds__(THREADS) void k_conv_wgrad_tile(const bf16* __restrict__ in, const bf16* __restrict__ dZ,
                                                             float* __restrict__ dW, float* __restrict__ db, int P,
                                                             int H, int Wd, int Cin, int Cout, int chunk)
{
    constexpr int PR = WG_PX + 8;                                      // padded LDS row (pixels)
    constexpr int NI = BM / 16;
    constexpr int NA = (WG_PX / 4) * (BM / 8);                         // dZ pieces (<= 128)
    constexpr int NB = (WG_PX / 4) * 8;                                // patch pieces (128)
    __shared__ __attribute__((aligned(16))) bf16 At[BM * PR];          // dZ^T
    __shared__ __attribute__((aligned(16))) bf16 Bt[64 * PR];          // patch^T
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int m = l & 15, kq = l >> 4;
    const int K = 9 * Cin;
    const int k0 = blockIdx.x * 64, co0 = blockIdx.y * BM;
    const int pbeg = blockIdx.z * chunk, pend = min(P, pbeg + chunk);
    const int hw = H * Wd;
    v4f acc[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    const bool bias_tile = db && blockIdx.x == 0;
    // the staging piece of this thread: threads [0, NA) move dZ, [128, 128 + NB) the patches
    const bool isA = t < NA, isB = t >= 128 && t - 128 < NB;
    const int pa = isA ? t : t - 128;
    const int px4 = (pa / (isA ? BM / 8 : 8)) * 4;                     // first of the four pixels
    const int cp = (pa % (isA ? BM / 8 : 8)) * 8;                      // first channel / k
    int tap = 0, ci = 0;
    if (isB && k0 + cp < K) {
        tap = (k0 + cp) / Cin;
        ci = k0 + cp - tap * Cin;
    }
    for (int pb = pbeg; pb < pend; pb += WG_PX) {
        uint4 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = make_uint4(0u, 0u, 0u, 0u);
            const int p = pb + px4 + j;
            if (p >= pend) continue;
            if (isA) {
                v[j] = *(const uint4*)(dZ + (int64_t)p * Cout + co0 + cp);
            } else if (isB && k0 + cp < K) {
                const int n = p / hw, rem = p - n * hw, y = rem / Wd, x = rem - y * Wd;
                const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
                if (yy >= 0 && yy < H && xx >= 0 && xx < Wd)
                    v[j] = *(const uint4*)(in + ((int64_t)(n * H + yy) * Wd + xx) * Cin + ci);
            }
        }
        if (isA) {
#pragma unroll
            for (int q = 0; q < 8; ++q) *(uint2*)(At + (cp + q) * PR + px4) = pack4(v, q);
        } else if (isB) {
#pragma unroll
            for (int q = 0; q < 8; ++q) *(uint2*)(Bt + (cp + q) * PR + px4) = pack4(v, q);
        }
        __syncthreads();
        if (bias_tile && t < BM)
            for (int px = 0; px < WG_PX; ++px) bsum += bf2f(At[t * PR + px]);
#pragma unroll
        for (int r0 = 0; r0 < WG_PX; r0 += 16) {
            const v4s b = *(const v4s*)(Bt + (16 * w + m) * PR + r0 + 4 * kq);
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                const v4s a = *(const v4s*)(At + (16 * i + m) * PR + r0 + 4 * kq);
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[i], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    const int k = k0 + 16 * w + m;
    if (k < K)
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int co = co0 + 16 * i + 4 * kq + e;
                if (acc[i][e] != 0.0f) atomicAdd(&dW[(int64_t)co * K + k], acc[i][e]);
            }
    if (bias_tile && t < BM && bsum != 0.0f) atomicAdd(&db[co0 + t], bsum);
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

// The elementwise layers move eight channels (16 bytes) per thread: every channel count is a
// multiple of 16.
struct bf8 {
    uint4 v;
    __device__ float get(int q) const { return bf2f(((const bf16*)&v)[q]); }
    __device__ void set(int q, float f) { ((bf16*)&v)[q] = f2bf(f); }
};
__device__ inline bf8 ld8(const bf16* p) { return bf8{*(const uint4*)p}; }
__device__ inline void st8(bf16* p, const bf8& x) { *(uint4*)p = x.v; }

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

// Cin and Cout are multiples of 16 (the activations' channel counts)
bool conv_fwd(lbib_net* n, int l, const bf16* in, void* out, int B, bool relu, bool out_f32, const bf16* W,
              const float* bias, int Cin, int Cout)
{
    const int div = LAYER_DIV[l];
    const int H = n->H / div, Wd = n->Wd / div;
    const int P = B * H * Wd;
    hipStream_t s = n->stream;
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
    // pixel chunks: about 2048 workgroups in all, at least ~1024 pixels each
    const int BM = Cout >= 64 ? 64 : Cout;
    const int tiles = ((K + 63) / 64) * (Cout / BM);
    int nchunk = std::max(1, std::min(2048 / tiles, (P + 1023) / 1024));
    int chunk = (P + nchunk - 1) / nchunk;
    chunk = (chunk + WG_PX - 1) / WG_PX * WG_PX;
    nchunk = (P + chunk - 1) / chunk;
    const dim3 grid((unsigned)((K + 63) / 64), (unsigned)(Cout / BM), (unsigned)nchunk);
    if (BM == 64)
        NET_K(hipLaunchKernelGGL(k_conv_wgrad_tile<64>, grid, dim3(THREADS), 0, s, in, dz, dW, db, P, H, Wd, Cin, Cout, chunk));
    else if (BM == 32)
        NET_K(hipLaunchKernelGGL(k_conv_wgrad_tile<32>, grid, dim3(THREADS), 0, s, in, dz, dW, db, P, H, Wd, Cin, Cout, chunk));
    else
        NET_K(hipLaunchKernelGGL(k_conv_wgrad_tile<16>, grid, dim3(THREADS), 0, s, in, dz, dW, db, P, H, Wd, Cin, Cout, chunk));
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
