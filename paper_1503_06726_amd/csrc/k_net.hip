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

constexpr int NT_MAX = 4;
constexpr int THREADS = 256;

// ---------------------------------------------------------------------------------------
// 3x3 convolution, forward: out[p][co] = act(sum_k patch[p][k] W[co][k] + bias[co])
// block: 64 pixels (4 waves x 16) x 16 NT output channels
// ---------------------------------------------------------------------------------------
template <int NT, bool RELU, bool OUT_F32>
__global__ __launch_bounds__(THREADS) void k_conv_fwd(const bf16* __restrict__ in, const bf16* __restrict__ W,
                                                      const float* __restrict__ bias, void* __restrict__ out, int P,
                                                      int H, int Wd, int Cin, int Cout)
{
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = l & 15, kq = l >> 4;
    const int p = blockIdx.x * 64 + w * 16 + m;                  // this lane's A row (pixel)
    const int co0 = blockIdx.y * 16 * NT;
    const int K = 9 * Cin;
    const int hw = H * Wd;
    const int n = p / hw, rem = p - n * hw, y = rem / Wd, x = rem - y * Wd;
    v4f acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int tap = 0; tap < 9; ++tap) {
        const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
        const bool ok = p < P && yy >= 0 && yy < H && xx >= 0 && xx < Wd;
        const bf16* arow = in + ((int64_t)(n * H + yy) * Wd + xx) * Cin + 4 * kq;
        const bf16* brow = W + (int64_t)(co0 + m) * K + tap * Cin + 4 * kq;
        for (int ci0 = 0; ci0 < Cin; ci0 += 16) {
            v4s a = v4s{0, 0, 0, 0};
            if (ok) a = *(const v4s*)(arow + ci0);
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const v4s b = *(const v4s*)(brow + (int64_t)16 * j * K + ci0);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = co0 + 16 * j + m;
        const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int po = blockIdx.x * 64 + w * 16 + 4 * kq + i;
            if (po >= P) continue;
            float v = acc[j][i] + bv;
            if (RELU) v = fmaxf(v, 0.0f);
            if (OUT_F32) ((float*)out)[(int64_t)po * Cout + co] = v;
            else ((bf16*)out)[(int64_t)po * Cout + co] = f2bf(v);
        }
    }
}

// ---------------------------------------------------------------------------------------
// weight gradient: dW[co][k] += sum_p dZ[p][co] patch[p][k]  (MFMA over 16-pixel steps), and
// the bias gradient db[co] += sum_p dZ[p][co].  block: 4 waves, each a share of the pixel chunk;
// a wave's tile is 16 output channels x 16 NT values of k; partial tiles are added atomically.
// ---------------------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(THREADS) void k_conv_wgrad(const bf16* __restrict__ in, const bf16* __restrict__ dZ,
                                                        float* __restrict__ dW, float* __restrict__ db, int P, int H,
                                                        int Wd, int Cin, int Cout, int chunk)
{
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = l & 15, kq = l >> 4;
    const int K = 9 * Cin;
    const int k0 = blockIdx.x * 16 * NT, co0 = blockIdx.y * 16;
    const int pbeg = blockIdx.z * chunk, pend = min(P, pbeg + chunk);
    const int hw = H * Wd;
    v4f acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    // k columns of this lane for each j: tap and channel
    int tapj[NT], cij[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int k = k0 + 16 * j + m;
        tapj[j] = k / Cin;
        cij[j] = k - tapj[j] * Cin;
    }
    for (int pb = pbeg + 16 * w; pb < pend; pb += 64) {
        v4s a;
        short bj[NT][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int pp = pb + 4 * kq + i;
            bf16 dz = 0;
            if (pp < pend) dz = dZ[(int64_t)pp * Cout + co0 + m];
            a[i] = (short)dz;
            const int n = pp / hw, rem = pp - n * hw, y = rem / Wd, x = rem - y * Wd;
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const int yy = y + tapj[j] / 3 - 1, xx = x + tapj[j] % 3 - 1;
                bf16 v = 0;
                if (pp < pend && yy >= 0 && yy < H && xx >= 0 && xx < Wd)
                    v = in[((int64_t)(n * H + yy) * Wd + xx) * Cin + cij[j]];
                bj[j][i] = (short)v;
            }
        }
        // lane (m, kq) holds dZ of channel co0 + m at 4 of the 16 pixels: the four lane groups
        // together cover them all, once (the first k tile only)
        if (db && blockIdx.x == 0) bsum += bf2f((bf16)a[0]) + bf2f((bf16)a[1]) + bf2f((bf16)a[2]) + bf2f((bf16)a[3]);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const v4s b = v4s{bj[j][0], bj[j][1], bj[j][2], bj[j][3]};
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = co0 + 4 * kq + i, k = k0 + 16 * j + m;
            if (acc[j][i] != 0.0f) atomicAdd(&dW[(int64_t)co * K + k], acc[j][i]);
        }
    if (db && blockIdx.x == 0 && bsum != 0.0f) atomicAdd(&db[co0 + m], bsum);
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
    const int h2 = H / 2, w2 = Wd / 2;
    if (i >= (int64_t)B * h2 * w2 * C) return;
    const int c = (int)(i % C);
    const int64_t q = i / C;
    const int x = (int)(q % w2), y = (int)((q / w2) % h2), n = (int)(q / ((int64_t)w2 * h2));
    const bf16* s = in + ((int64_t)(n * H + 2 * y) * Wd + 2 * x) * C + c;
    const float v = (bf2f(s[0]) + bf2f(s[C])) + (bf2f(s[(int64_t)Wd * C]) + bf2f(s[(int64_t)Wd * C + C]));
    out[i] = f2bf(0.25f * v);
}

// gradient of the pool: dIn (+)= dOut / 4 at the four inputs
__global__ void k_pool_bwd(const bf16* __restrict__ dout, bf16* __restrict__ din, int B, int H, int Wd, int C, int add)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)B * H * Wd * C) return;
    const int c = (int)(i % C);
    const int64_t q = i / C;
    const int x = (int)(q % Wd), y = (int)((q / Wd) % H), n = (int)(q / ((int64_t)Wd * H));
    float v = 0.25f * bf2f(dout[((int64_t)(n * (H / 2) + y / 2) * (Wd / 2) + x / 2) * C + c]);
    if (add) v += bf2f(din[i]);
    din[i] = f2bf(v);
}

// nearest 2x upsample: [B][H][W][C] -> [B][2H][2W][C]
__global__ void k_up(const bf16* __restrict__ in, bf16* __restrict__ out, int B, int H, int Wd, int C)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int H2 = 2 * H, W2 = 2 * Wd;
    if (i >= (int64_t)B * H2 * W2 * C) return;
    const int c = (int)(i % C);
    const int64_t q = i / C;
    const int x = (int)(q % W2), y = (int)((q / W2) % H2), n = (int)(q / ((int64_t)W2 * H2));
    out[i] = in[((int64_t)(n * H + y / 2) * Wd + x / 2) * C + c];
}

// gradient of the upsample: dIn = sum of the four dOut
__global__ void k_up_bwd(const bf16* __restrict__ dout, bf16* __restrict__ din, int B, int H, int Wd, int C)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)B * H * Wd * C) return;
    const int c = (int)(i % C);
    const int64_t q = i / C;
    const int x = (int)(q % Wd), y = (int)((q / Wd) % H), n = (int)(q / ((int64_t)Wd * H));
    const int64_t W2 = 2 * Wd;
    const bf16* s = dout + ((int64_t)(n * 2 * H + 2 * y) * W2 + 2 * x) * C + c;
    din[i] = f2bf((bf2f(s[0]) + bf2f(s[C])) + (bf2f(s[W2 * C]) + bf2f(s[W2 * C + C])));
}

__global__ void k_add(const bf16* __restrict__ a, const bf16* __restrict__ b, bf16* __restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf(bf2f(a[i]) + bf2f(b[i]));
}

// dZ = dY * [Y > 0]
__global__ void k_relu_bwd(const bf16* __restrict__ dy, const bf16* __restrict__ y, bf16* __restrict__ dz, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dz[i] = bf2f(y[i]) > 0.0f ? dy[i] : (bf16)0;
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

bool conv_fwd(lbib_net* n, int l, const bf16* in, void* out, int B, bool relu, bool out_f32, const bf16* W,
              const float* bias, int Cin, int Cout)
{
    const int div = LAYER_DIV[l];
    const int H = n->H / div, Wd = n->Wd / div;
    const int P = B * H * Wd;
    const int NT = (Cout % 64 == 0) ? 4 : (Cout % 32 == 0 ? 2 : 1);
    const dim3 grid((unsigned)((P + 63) / 64), (unsigned)(Cout / (16 * NT)));
    hipStream_t s = n->stream;
    if (out_f32) {
        NET_K(hipLaunchKernelGGL((k_conv_fwd<1, false, true>), dim3(grid.x, Cout / 16), dim3(THREADS), 0, s, in, W,
                                 bias, out, P, H, Wd, Cin, Cout));
        return true;
    }
    if (NT == 4) {
        if (relu) NET_K(hipLaunchKernelGGL((k_conv_fwd<4, true, false>), grid, dim3(THREADS), 0, s, in, W, bias, out, P, H, Wd, Cin, Cout));
        else NET_K(hipLaunchKernelGGL((k_conv_fwd<4, false, false>), grid, dim3(THREADS), 0, s, in, W, bias, out, P, H, Wd, Cin, Cout));
    } else if (NT == 2) {
        if (relu) NET_K(hipLaunchKernelGGL((k_conv_fwd<2, true, false>), grid, dim3(THREADS), 0, s, in, W, bias, out, P, H, Wd, Cin, Cout));
        else NET_K(hipLaunchKernelGGL((k_conv_fwd<2, false, false>), grid, dim3(THREADS), 0, s, in, W, bias, out, P, H, Wd, Cin, Cout));
    } else {
        if (relu) NET_K(hipLaunchKernelGGL((k_conv_fwd<1, true, false>), grid, dim3(THREADS), 0, s, in, W, bias, out, P, H, Wd, Cin, Cout));
        else NET_K(hipLaunchKernelGGL((k_conv_fwd<1, false, false>), grid, dim3(THREADS), 0, s, in, W, bias, out, P, H, Wd, Cin, Cout));
    }
    return true;
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
        hipLaunchKernelGGL(k_pool, dim3(nblk(act_elems(n, out, B))), dim3(THREADS), 0, s, A(in), A(out), B,
                           n->H / div, n->Wd / div, ACT_SHAPE[in].C);
        return hipGetLastError() == hipSuccess;
    };
    auto up = [&](int in, int out) {
        const int div = ACT_SHAPE[in].div;
        hipLaunchKernelGGL(k_up, dim3(nblk(act_elems(n, out, B))), dim3(THREADS), 0, s, A(in), A(out), B,
                           n->H / div, n->Wd / div, ACT_SHAPE[in].C);
        return hipGetLastError() == hipSuccess;
    };
    auto add = [&](int a, int b, int out) {
        hipLaunchKernelGGL(k_add, dim3(nblk(act_elems(n, out, B))), dim3(THREADS), 0, s, A(a), A(b), A(out),
                           act_elems(n, out, B));
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
    const int chunk = 4096;
    const unsigned nz = (unsigned)((P + chunk - 1) / chunk);
    float* dW = n->grad + n->woff[l];
    float* db = n->grad + n->boff[l];
    if (K % 64 == 0)
        NET_K(hipLaunchKernelGGL(k_conv_wgrad<4>, dim3(K / 64, Cout / 16, nz), dim3(THREADS), 0, s, in, dz, dW, db, P, H,
                                 Wd, Cin, Cout, chunk));
    else
        NET_K(hipLaunchKernelGGL(k_conv_wgrad<1>, dim3(K / 16, Cout / 16, nz), dim3(THREADS), 0, s, in, dz, dW, db, P, H,
                                 Wd, Cin, Cout, chunk));
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
        hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(e)), dim3(THREADS), 0, s, dy, A(y), dz, e);
        return hipGetLastError() == hipSuccess;
    };
    auto up_bwd = [&](int up_out, int in_slot, bf16* dout, bf16* din) {
        const int div = ACT_SHAPE[in_slot].div;
        hipLaunchKernelGGL(k_up_bwd, dim3(nblk(act_elems(n, in_slot, B))), dim3(THREADS), 0, s, dout, din, B,
                           n->H / div, n->Wd / div, ACT_SHAPE[in_slot].C);
        (void)up_out;
        return hipGetLastError() == hipSuccess;
    };
    auto pool_bwd = [&](int in_slot, bf16* dout, bf16* din, int add) {
        const int div = ACT_SHAPE[in_slot].div;
        hipLaunchKernelGGL(k_pool_bwd, dim3(nblk(act_elems(n, in_slot, B))), dim3(THREADS), 0, s, dout, din, B,
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
