// vdi_mlp.hip -- the threshold regressor of the learned path: a 64-128-128-1
// MLP with GELU, bf16 weights and activations, fp32 accumulation on the
// matrix cores (v_mfma_f32_16x16x16_bf16), trained with Adam by the kernels
// below.  The MLP maps a brick-ray's 64-bin opacity histogram to log2(gamma).
//
// Parameters live in one flat array (fp32 master copy and bf16 copy, same
// offsets): W1 [128][64] (out, in), b1 [128], W2 [128][128], b2 [128], w3 [128],
// b3 [1].  Matrices are read from the bf16 copy, biases from the fp32 copy.
//
// MFMA 16x16x16 fragments (64 lanes, lane l = 16*g + i):
//   A (M x K): lane holds A[i][4g .. 4g+3]
//   B (K x N): lane holds B[4g .. 4g+3][i]
//   D (M x N): lane holds D[4g .. 4g+3][i]
#include "vdi_internal.h"
#include "vdi_kernels.h"

namespace vdi {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kIn = 64, kHid = 128;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kHid;
constexpr int kRowsPerBlock = 64;   // 4 waves x 16 rows

__device__ inline uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// GELU(z) = z * Phi(z) with the normal CDF Phi(z) = 1 - erfc(z / sqrt 2) / 2.
// erfc(x) for x >= 0 by the rational approximation of Abramowitz and Stegun,
// formula 7.1.26 (t = 1 / (1 + p x), erfc(x) = t (a1 + t (a2 + ... t a5)) exp(-x^2),
// absolute error at most 1.5e-7), evaluated on |z| with Phi(-z) = 1 - Phi(z);
// exp(-x^2) is also the density term of the derivative.
__device__ inline void normal_parts(float z, float& cdf, float& pdf)
{
    const float x = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
    const float poly =
        t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
    const float e = __builtin_amdgcn_exp2f(-(x * x) * 1.4426950408889634f);   // exp(-x^2) = exp(-z^2 / 2)
    const float half_erfc = 0.5f * poly * e;
    cdf = z >= 0.0f ? 1.0f - half_erfc : half_erfc;
    pdf = e * 0.39894228040143268f;                                          // 1 / sqrt(2 pi)
}
__device__ inline float gelu(float z)
{
    float c, d;
    normal_parts(z, c, d);
    return z * c;
}
__device__ inline float gelu_grad(float z)
{
    float c, d;
    normal_parts(z, c, d);
    return fmaf(z, d, c);
}

__device__ inline floatx4 mfma16(bf16x4 a, bf16x4 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ inline bf16x4 load4(const uint16_t* p)
{
    // 8-byte aligned by construction of every caller
    return *(const bf16x4*)p;
}

}  // namespace

// acts per row: z1[128] f32, z2[128] f32, h1[128] bf16 (64 words), h2[128] bf16 (64 words)
constexpr int kActFloats = 128 + 128 + 64 + 64;

// Forward pass.  Persistent: each block stages W1 and W2 in LDS once and
// walks row tiles with a grid stride; a wave takes 32 rows per step (two
// 16-row fragments sharing every weight fragment it reads).  Each layer is
// computed transposed, Z^T = W X^T (A operand: a 16x16 weight tile, B: the
// rows), so the accumulator a lane holds -- Z[row i][units 4g .. 4g+3] -- is
// exactly the B fragment of the next layer after GELU and bf16 rounding: the
// hidden activations never leave registers.  rows_dev, when given, holds the
// row count on the device; out_idx, when given, maps row r to y[out_idx[r]].
constexpr int kFwdRowsPerWave = 32;
constexpr int kFwdRowsPerBlock = 4 * kFwdRowsPerWave;

__global__ __launch_bounds__(256) void mlp_fwd_kernel(const uint16_t* __restrict__ wb, const float* __restrict__ wf,
                                                      const uint16_t* __restrict__ x, int rows_host,
                                                      const int* __restrict__ rows_dev, int row_off,
                                                      const int* __restrict__ out_idx, float* __restrict__ y,
                                                      float* __restrict__ acts)
{
    __shared__ __align__(16) uint16_t sW1[kHid * kIn];
    __shared__ __align__(16) uint16_t sW2[kHid * kHid];
    // rows: rows_host, or those of the device count past row_off (at most rows_host)
    const int rows = rows_dev ? max(0, min(rows_host, *rows_dev - row_off)) : rows_host;
    if (blockIdx.x * kFwdRowsPerBlock >= rows) return;
    for (int e = threadIdx.x; e < kHid * kIn / 8; e += blockDim.x)
        ((uint4*)sW1)[e] = ((const uint4*)(wb + oW1))[e];
    for (int e = threadIdx.x; e < kHid * kHid / 8; e += blockDim.x)
        ((uint4*)sW2)[e] = ((const uint4*)(wb + oW2))[e];
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, g = l >> 4;
    const float b3 = wf[oB3];
    for (int base = blockIdx.x * kFwdRowsPerBlock; base < rows; base += gridDim.x * kFwdRowsPerBlock) {
        const int r0 = base + w * kFwdRowsPerWave;
        int row[2];
        bf16x4 xa[2][4];
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            row[tt] = r0 + tt * 16 + i;
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                xa[tt][ks] = row[tt] < rows ? load4(x + (size_t)row[tt] * kIn + ks * 16 + g * 4) : bf16x4{0, 0, 0, 0};
        }
        // layer 1: Z1^T = W1 X^T; lane (g, i) gets units nt*16 + 4g .. +3 of row i
        bf16x4 h1[2][8];
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) {
            floatx4 acc[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const bf16x4 wa = load4(sW1 + (nt * 16 + i) * kIn + ks * 16 + g * 4);
#pragma unroll
                for (int tt = 0; tt < 2; ++tt) acc[tt] = mfma16(wa, xa[tt][ks], acc[tt]);
            }
            const int u0 = nt * 16 + 4 * g;
            const float4 bias = *(const float4*)(wf + oB1 + u0);
            const float bv[4] = { bias.x, bias.y, bias.z, bias.w };
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                float z[4];
                uint16_t hb[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    z[v] = acc[tt][v] + bv[v];
                    hb[v] = f2bf(gelu(z[v]));
                }
                h1[tt][nt] = bf16x4{(short)hb[0], (short)hb[1], (short)hb[2], (short)hb[3]};
                if (acts && row[tt] < rows) {
                    float* ar = acts + (size_t)row[tt] * kActFloats;
                    *(float4*)(ar + u0) = make_float4(z[0], z[1], z[2], z[3]);
                    *(bf16x4*)((uint16_t*)(ar + 256) + u0) = h1[tt][nt];
                }
            }
        }
        // layer 2: Z2^T = W2 H1^T, then y = w3 . GELU(Z2) + b3
        float part[2] = {0.0f, 0.0f};
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) {
            floatx4 acc[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                const bf16x4 wa = load4(sW2 + (nt * 16 + i) * kHid + ks * 16 + g * 4);
#pragma unroll
                for (int tt = 0; tt < 2; ++tt) acc[tt] = mfma16(wa, h1[tt][ks], acc[tt]);
            }
            const int u0 = nt * 16 + 4 * g;
            const float4 bias = *(const float4*)(wf + oB2 + u0);
            const float bv[4] = { bias.x, bias.y, bias.z, bias.w };
            const bf16x4 w3 = load4(wb + oW3 + u0);
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                float z[4];
                uint16_t hb[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    z[v] = acc[tt][v] + bv[v];
                    hb[v] = f2bf(gelu(z[v]));
                    part[tt] = fmaf(bf2f(hb[v]), bf2f((uint16_t)w3[v]), part[tt]);
                }
                if (acts && row[tt] < rows) {
                    float* ar = acts + (size_t)row[tt] * kActFloats;
                    *(float4*)(ar + 128 + u0) = make_float4(z[0], z[1], z[2], z[3]);
                    *(bf16x4*)((uint16_t*)(ar + 320) + u0) = bf16x4{(short)hb[0], (short)hb[1], (short)hb[2], (short)hb[3]};
                }
            }
        }
        // row i's 128 units are spread over the four lanes i, i+16, i+32, i+48
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            part[tt] += __shfl_xor(part[tt], 16, 64);
            part[tt] += __shfl_xor(part[tt], 32, 64);
            if (g == 0 && row[tt] < rows) y[out_idx ? out_idx[row[tt]] : row[tt]] = part[tt] + b3;
        }
    }
}

// Backward for one block of 64 rows: data gradients and the block's partial
// parameter gradients (written to partial[blockIdx.x][kParams]).
__global__ __launch_bounds__(256) void mlp_bwd_kernel(const uint16_t* __restrict__ wb, const uint16_t* __restrict__ x,
                                                      const float* __restrict__ acts, const float* __restrict__ dy,
                                                      int rows, float* __restrict__ partial)
{
    __shared__ __align__(16) uint16_t sW2t[kHid * (kHid + 8)];     // W2 transposed: [k][n]
    __shared__ __align__(16) uint16_t sDz2[kRowsPerBlock * (kHid + 8)];
    __shared__ __align__(16) uint16_t sDz1[kRowsPerBlock * (kHid + 8)];
    __shared__ __align__(16) uint16_t sH1[kRowsPerBlock * (kHid + 8)];
    __shared__ __align__(16) uint16_t sX[kRowsPerBlock * (kIn + 8)];
    __shared__ float sColB2[4][kHid], sColB1[4][kHid], sW3[4][kHid], sB3[4];
    constexpr int LD = kHid + 8, LDX = kIn + 8;

    for (int e = threadIdx.x; e < kHid * kHid; e += blockDim.x) {
        int n = e / kHid, k = e % kHid;
        sW2t[k * LD + n] = wb[oW2 + e];
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, g = l >> 4;
    const int rb = blockIdx.x * kRowsPerBlock;
    // stage x and h1 of the block's rows (zeros past the end)
    for (int e = threadIdx.x; e < kRowsPerBlock * kIn; e += blockDim.x) {
        int r = e / kIn, c = e % kIn;
        sX[r * LDX + c] = rb + r < rows ? x[(size_t)(rb + r) * kIn + c] : (uint16_t)0;
    }
    for (int e = threadIdx.x; e < kRowsPerBlock * kHid; e += blockDim.x) {
        int r = e / kHid, c = e % kHid;
        sH1[r * LD + c] = rb + r < rows ? ((const uint16_t*)(acts + (size_t)(rb + r) * kActFloats + 256))[c]
                                        : (uint16_t)0;
    }
    __syncthreads();

    // dz2 = dy * w3 * gelu'(z2), in A-fragment order: row i of this wave, cols ks*16 + 4g + v
    const int r0 = rb + w * 16;
    const int ra = r0 + i;
    const float dyr = ra < rows ? dy[ra] : 0.0f;
    bf16x4 adz2[8];
    float colb2[8][4];
    float w3p[8][4];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int col = ks * 16 + 4 * g + v;
            float d = 0.0f, hv = 0.0f;
            if (ra < rows) {
                const float* ar = acts + (size_t)ra * kActFloats;
                d = dyr * bf2f(wb[oW3 + col]) * gelu_grad(ar[128 + col]);
                hv = bf2f(((const uint16_t*)(ar + 320))[col]);
            }
            uint16_t db = f2bf(d);
            adz2[ks][v] = (short)db;
            sDz2[(w * 16 + i) * LD + col] = db;
            colb2[ks][v] = d;
            w3p[ks][v] = dyr * hv;
        }
    }
    // column sums over the wave's 16 rows (lanes sharing g): bias and w3 grads
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float s = colb2[ks][v], t = w3p[ks][v];
#pragma unroll
            for (int d = 8; d >= 1; d >>= 1) {
                s += __shfl_xor(s, d, 64);
                t += __shfl_xor(t, d, 64);
            }
            if (i == 0) {
                sColB2[w][ks * 16 + 4 * g + v] = s;
                sW3[w][ks * 16 + 4 * g + v] = t;
            }
        }
    }
    {
        float s = dyr;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
        // each row counted 4 times (lanes 16g+i for g = 0..3 share row i)
        if (l == 0) sB3[w] = 0.25f * s;
    }
    // dh1 = dz2 W2 (contraction over n); dz1 = dh1 * gelu'(z1), D layout: rows 4g+v, col kt*16+i
    float colb1[8];
#pragma unroll
    for (int kt = 0; kt < 8; ++kt) {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) acc = mfma16(adz2[ks], load4(sW2t + (kt * 16 + i) * LD + ks * 16 + g * 4), acc);
        const int col = kt * 16 + i;
        float s = 0.0f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = r0 + 4 * g + v;
            float d = 0.0f;
            if (row < rows) d = acc[v] * gelu_grad(acts[(size_t)row * kActFloats + col]);
            sDz1[(w * 16 + 4 * g + v) * LD + col] = f2bf(d);
            s += d;
        }
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        colb1[kt] = s;
    }
    if (g == 0) {
#pragma unroll
        for (int kt = 0; kt < 8; ++kt) sColB1[w][kt * 16 + i] = colb1[kt];
    }
    __syncthreads();

    float* out = partial + (size_t)blockIdx.x * (oB3 + 1);
    // gW2[n][k] = sum_r dz2[r][n] h1[r][k]: M = n, N = k, K = the block's 64 rows.
    // A[n][r] = dz2[r][n] -> lane needs dz2[r0' + 4g + v][n0 + i]; B[r][k] = h1[r][k] -> h1[r0' + 4g + v][k0 + i].
    // Wave w owns n-tiles {2w, 2w+1} x all 8 k-tiles.
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int nt = 2 * w + t;
        floatx4 acc[8];
#pragma unroll
        for (int kt = 0; kt < 8; ++kt) acc[kt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int rs = 0; rs < 4; ++rs) {
            bf16x4 av;
#pragma unroll
            for (int v = 0; v < 4; ++v) av[v] = (short)sDz2[(rs * 16 + 4 * g + v) * LD + nt * 16 + i];
#pragma unroll
            for (int kt = 0; kt < 8; ++kt) {
                bf16x4 bv;
#pragma unroll
                for (int v = 0; v < 4; ++v) bv[v] = (short)sH1[(rs * 16 + 4 * g + v) * LD + kt * 16 + i];
                acc[kt] = mfma16(av, bv, acc[kt]);
            }
        }
        // D[n][k]: lane holds rows n = nt*16 + 4g + v, col k = kt*16 + i
#pragma unroll
        for (int kt = 0; kt < 8; ++kt)
#pragma unroll
            for (int v = 0; v < 4; ++v) out[oW2 + (nt * 16 + 4 * g + v) * kHid + kt * 16 + i] = acc[kt][v];
    }
    // gW1[o][c] = sum_r dz1[r][o] x[r][c]: wave w owns o-tiles {2w, 2w+1} x 4 c-tiles.
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int ot = 2 * w + t;
        floatx4 acc[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int rs = 0; rs < 4; ++rs) {
            bf16x4 av;
#pragma unroll
            for (int v = 0; v < 4; ++v) av[v] = (short)sDz1[(rs * 16 + 4 * g + v) * LD + ot * 16 + i];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                bf16x4 bv;
#pragma unroll
                for (int v = 0; v < 4; ++v) bv[v] = (short)sX[(rs * 16 + 4 * g + v) * LDX + ct * 16 + i];
                acc[ct] = mfma16(av, bv, acc[ct]);
            }
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) out[oW1 + (ot * 16 + 4 * g + v) * kIn + ct * 16 + i] = acc[ct][v];
    }
    // biases and w3: fixed-order sums over the 4 waves
    for (int c = threadIdx.x; c < kHid; c += blockDim.x) {
        out[oB2 + c] = ((sColB2[0][c] + sColB2[1][c]) + sColB2[2][c]) + sColB2[3][c];
        out[oB1 + c] = ((sColB1[0][c] + sColB1[1][c]) + sColB1[2][c]) + sColB1[3][c];
        out[oW3 + c] = ((sW3[0][c] + sW3[1][c]) + sW3[2][c]) + sW3[3][c];
    }
    if (threadIdx.x == 0) out[oB3] = ((sB3[0] + sB3[1]) + sB3[2]) + sB3[3];
}

// Sum of the per-block partial gradients in block order (deterministic).
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ partial, int nblocks,
                                                         float* __restrict__ grad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > oB3) return;
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * (oB3 + 1) + p];
    grad[p] = s;
}

// Adam on the fp32 master weights; refreshes the bf16 copy.
__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ wf, uint16_t* __restrict__ wb,
                                                       const float* __restrict__ grad, float* __restrict__ m,
                                                       float* __restrict__ v, float lr, float b1, float b2, float eps,
                                                       float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > oB3) return;
    const float gr = grad[p];
    const float mm = b1 * m[p] + (1.0f - b1) * gr;
    const float vv = b2 * v[p] + (1.0f - b2) * gr * gr;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / c1, vh = vv / c2;
    const float nw = wf[p] - lr * mh / (sqrtf(vh) + eps);
    wf[p] = nw;
    wb[p] = f2bf(nw);
}

// Gradient of the regression loss 0.5 * sum_i (y_i - log2(gamma_i))^2 with
// respect to y, scaled: dy_i = scale * (y_i - log2(gamma_i)); per block of 256
// rows the loss summed in fp64 in a fixed order (for reporting).
__global__ __launch_bounds__(256) void mlp_mse_kernel(const float* __restrict__ y, const float* __restrict__ gamma,
                                                      int rows, float scale, float* __restrict__ dy,
                                                      double* __restrict__ loss_part)
{
    __shared__ double ls[256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (i < rows) {
        const float d = y[i] - log2f(gamma[i]);
        dy[i] = d * scale;
        l = 0.5 * (double)d * (double)d;
    }
    ls[threadIdx.x] = l;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) ls[threadIdx.x] += ls[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss_part) loss_part[blockIdx.x] = ls[0];
}

// The bf16 copy of the fp32 master parameters (round to nearest even).
__global__ __launch_bounds__(256) void mlp_pack_kernel(const float* __restrict__ wf, uint16_t* __restrict__ wb)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p <= oB3) wb[p] = f2bf(wf[p]);
}

// One 16x16x16 product through the matrix core, for checking the fragment layout.
__global__ void mfma_probe_kernel(const uint16_t* A, const uint16_t* B, float* D)
{
    const int l = threadIdx.x, i = l & 15, g = l >> 4;
    bf16x4 a, b;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        a[v] = (short)A[i * 16 + 4 * g + v];   // A[i][4g+v]
        b[v] = (short)B[(4 * g + v) * 16 + i]; // B[4g+v][i]
    }
    floatx4 d = mfma16(a, b, floatx4{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
    for (int v = 0; v < 4; ++v) D[(4 * g + v) * 16 + i] = d[v];
}

int mlp_params() { return oB3 + 1; }
int mlp_act_floats() { return kActFloats; }
int mlp_rows_per_block() { return kRowsPerBlock; }

void launch_mlp_fwd(const uint16_t* wb, const float* wf, const uint16_t* x, int rows, const int* rows_dev,
                    const int* out_idx, int max_blocks, float* y, float* acts, hipStream_t s, int row_off)
{
    int nb = (rows + kFwdRowsPerBlock - 1) / kFwdRowsPerBlock;
    nb = std::max(1, std::min(nb, max_blocks));
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(nb), dim3(256), 0, s, wb, wf, x, rows, rows_dev, row_off, out_idx, y,
                       acts);
}

void launch_mlp_bwd(const uint16_t* wb, const uint16_t* x, const float* acts, const float* dy, int rows,
                    float* partial, float* grad, hipStream_t s)
{
    int nb = (rows + kRowsPerBlock - 1) / kRowsPerBlock;
    hipLaunchKernelGGL(mlp_bwd_kernel, dim3(nb), dim3(256), 0, s, wb, x, acts, dy, rows, partial);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((oB3 + 1 + 255) / 256), dim3(256), 0, s, partial, nb, grad);
}

void launch_mlp_adam(float* wf, uint16_t* wb, const float* grad, float* m, float* v, float lr, float b1, float b2,
                     float eps, int step, hipStream_t s)
{
    float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((oB3 + 1 + 255) / 256), dim3(256), 0, s, wf, wb, grad, m, v, lr, b1,
                       b2, eps, c1, c2);
}

void launch_mlp_mse(const float* y, const float* gamma, int rows, float scale, float* dy, double* loss_part,
                    hipStream_t s)
{
    hipLaunchKernelGGL(mlp_mse_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, y, gamma, rows, scale, dy,
                       loss_part);
}

void launch_mlp_pack(const float* wf, uint16_t* wb, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_pack_kernel, dim3((oB3 + 1 + 255) / 256), dim3(256), 0, s, wf, wb);
}

void launch_mfma_probe(const uint16_t* A, const uint16_t* B, float* D, hipStream_t s)
{
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, s, A, B, D);
}

}  // namespace vdi
