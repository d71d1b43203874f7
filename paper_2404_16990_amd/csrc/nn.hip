// HIP kernels of the block-proposal network (definitions in nn.hpp):
//  - training: masked-conv forward with an MFMA BF16 GEMM (FP32 accumulate),
//    loss, backward (data and weight gradients as GEMMs), Adam;
//  - the incremental autoregressive pass that scores a given block or samples
//    a new one site by site with exactly the same arithmetic, accumulating
//    log q in FP64 from uint32 thresholds;
//  - gathering blocks from packed lattices, the Metropolis-Hastings decision
//    and write-back, and training-block extraction.
#include <math.h>

#include "device.hpp"
#include "nn.hpp"
#include "nn_launch.hpp"

namespace ising {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (inputs are finite)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// tanh from the hardware exp2 and reciprocal: tanh|x| = (1 - e)/(1 + e), e = exp(-2|x|).
// Every kernel of the network uses this one definition, so training, scoring
// and sampling evaluate the same function.
__device__ __forceinline__ float net_tanh(float x)
{
    const float e = __builtin_amdgcn_exp2f(-2.8853900817779268f * fabsf(x));  // 2 log2(e)
    const float t = (1.f - e) * __builtin_amdgcn_rcpf(1.f + e);
    return copysignf(t, x);
}

__device__ __forceinline__ float net_sigmoid(float x)
{
    return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(-1.4426950408889634f * x));
}

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t *p)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 zero_bf16x8()
{
    const uint4 v = make_uint4(0u, 0u, 0u, 0u);
    return __builtin_bit_cast(bf16x8, v);
}

// ---------------------------------------------------------------------------
// parameters -> BF16 GEMM operands
// ---------------------------------------------------------------------------
__global__ void k_cast_weights(const float *__restrict__ params, uint16_t *__restrict__ wt,
                               uint16_t *__restrict__ wtt)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // over 3 * C * KB
    if (idx >= 3 * C * KB)
        return;
    const int l = idx / (C * KB), r = idx - l * C * KB;
    const int c = r / KB, k = r - c * KB;          // output channel, K index t*C + c'
    const float w = params[off_w(l + 2) + k * C + c];  // W_l[t][c'][c]
    const uint16_t b = f2bf(w);
    wt[(l * C + c) * KB + k] = b;
    wtt[(l * KB + k) * C + c] = b;
}

// ---------------------------------------------------------------------------
// generic C[M][N] = sum_k A[m][k] * Bt[n][k]   (BF16 in, FP32 out)
// 256 threads, 64x64 tile, each wave a 32x32 quarter of 2x2 MFMA 16x16x32.
// Requires K % 32 == 0 and 16-byte aligned rows (lda, ldb multiples of 8).
// ---------------------------------------------------------------------------
// blockIdx.z = s sums k in [s kchunk, min(K, (s + 1) kchunk)) into the slice
// Cm + s M ldc (split-K partials; one slice when gridDim.z = 1).
__global__ __launch_bounds__(256) void k_gemm_nt(const uint16_t *__restrict__ A, int lda,
                                                 const uint16_t *__restrict__ Bt, int ldb,
                                                 float *__restrict__ Cm, int ldc, int M, int N, int K, int kchunk)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    Cm += (size_t)blockIdx.z * M * ldc;
    const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    floatx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k = kb; k < ke; k += 32) {
        bf16x8 av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int row = m0 + a * 16 + r;
            av[a] = row < M ? load_bf16x8(A + (size_t)row * lda + k + kq) : zero_bf16x8();
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int col = n0 + b * 16 + r;
            bv[b] = col < N ? load_bf16x8(Bt + (size_t)col * ldb + k + kq) : zero_bf16x8();
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = m0 + a * 16 + 4 * (lane >> 4) + i;
                const int col = n0 + b * 16 + r;
                if (row < M && col < N)
                    Cm[(size_t)row * ldc + col] = acc[a][b][i];
            }
}

// C[i] = sum over s = 0..S-1 of part[s][i], in that order
__global__ void k_sum_splits(const float *__restrict__ part, int S, int n, float *__restrict__ Cm)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    float v = 0.f;
    for (int s = 0; s < S; ++s)
        v += part[(size_t)s * n + i];
    Cm[i] = v;
}

// ---------------------------------------------------------------------------
// training forward
// ---------------------------------------------------------------------------
__device__ __forceinline__ float boundary_field(const int8_t *bnd, int Bs, int i, int j, const float *u)
{
    float f = 0.f;
    if (i == 0)
        f += (float)bnd[j] * u[0];
    if (i == Bs - 1)
        f += (float)bnd[Bs + j] * u[1];
    if (j == 0)
        f += (float)bnd[2 * Bs + i] * u[2];
    if (j == Bs - 1)
        f += (float)bnd[3 * Bs + i] * u[3];
    return f;
}

__global__ void k_layer1(const float *__restrict__ params, const int8_t *__restrict__ x,
                         const int8_t *__restrict__ bnd, const float *__restrict__ kc, int nblk, int Bs,
                         int Ppad, float *__restrict__ h, uint16_t *__restrict__ hb)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Ppad * C)
        return;
    const int p = idx / C, c = idx - p * C;
    const int BB = Bs * Bs;
    float v = 0.f;
    if (p < nblk * BB) {
        const int n = p / BB, k = p - n * BB, i = k / Bs, j = k - i * Bs;
        float pre = kc[n] * params[OFF_V1 + c] + params[OFF_B1 + c];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int ii = i + tap_di(t), jj = j + tap_dj(t);
            if (ii >= 0 && jj >= 0 && jj < Bs)
                pre += (float)x[n * BB + ii * Bs + jj] * params[OFF_W1 + t * C + c];
        }
        const float u[4] = {params[OFF_U1 + c], params[OFF_U1 + C + c], params[OFF_U1 + 2 * C + c],
                            params[OFF_U1 + 3 * C + c]};
        pre += boundary_field(bnd + n * 4 * Bs, Bs, i, j, u);
        v = net_tanh(pre);
    }
    h[idx] = v;
    hb[idx] = f2bf(v);
}

// xcol[p][t*C + c'] = hb[p + tap t][c'] inside the block, else 0; also transposed
__global__ void k_im2col(const uint16_t *__restrict__ hb, int nblk, int Bs, int Ppad,
                         uint16_t *__restrict__ xcol, uint16_t *__restrict__ xcolt)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // over Ppad * 5 * (C / 8)
    if (idx >= Ppad * 5 * (C / 8))
        return;
    const int p = idx / (5 * (C / 8));
    const int r = idx - p * 5 * (C / 8);
    const int t = r / (C / 8), c8 = (r - t * (C / 8)) * 8;
    const int BB = Bs * Bs;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (p < nblk * BB) {
        const int n = p / BB, k = p - n * BB, i = k / Bs, j = k - i * Bs;
        const int ii = i + tap_di(t), jj = j + tap_dj(t);
        if (ii >= 0 && jj >= 0 && jj < Bs)
            v = *reinterpret_cast<const uint4 *>(hb + (size_t)(n * BB + ii * Bs + jj) * C + c8);
    }
    *reinterpret_cast<uint4 *>(xcol + (size_t)p * KB + t * C + c8) = v;
    const uint16_t *e = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
    for (int q = 0; q < 8; ++q)
        xcolt[(size_t)(t * C + c8 + q) * Ppad + p] = e[q];
}

__global__ void k_bias_tanh(const float *__restrict__ pre, const float *__restrict__ bias, int Pvalid,
                            int Ppad, float *__restrict__ h, uint16_t *__restrict__ hb)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Ppad * C)
        return;
    const int p = idx / C, c = idx - p * C;
    const float v = p < Pvalid ? net_tanh(pre[idx] + bias[c]) : 0.f;
    h[idx] = v;
    if (hb)
        hb[idx] = f2bf(v);
}

__global__ void k_head(const float *__restrict__ h4, const float *__restrict__ params, int Pvalid,
                       float *__restrict__ logits)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= Pvalid)
        return;
    float s = params[OFF_BO];
    for (int c = 0; c < C; ++c)
        s = fmaf(h4[(size_t)p * C + c], params[OFF_WO + c], s);
    logits[p] = s;
}

// per-position loss softplus(-x l) into partial sums; dlogit = -x sigmoid(-x l) / P
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ logits, const int8_t *__restrict__ x,
                                              int Pvalid, int Ppad, float *__restrict__ dlogit,
                                              float *__restrict__ partial)
{
    __shared__ float red[256];
    const int p = blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (p < Ppad) {
        float d = 0.f;
        if (p < Pvalid) {
            const float xv = (float)x[p];
            const float z = -xv * logits[p];
            l = z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z));
            d = -xv / (1.f + expf(-z)) / (float)Pvalid;  // -x sigmoid(z)
        }
        dlogit[p] = d;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum(const float *__restrict__ partial, int n, float scale,
                                             float *__restrict__ out)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256)
        s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k)
            red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[0] = red[0] * scale;
}

// ---------------------------------------------------------------------------
// training backward
// ---------------------------------------------------------------------------
// dpre4 = dlogit * wo * (1 - h4^2), in fp32, bf16 and transposed bf16
__global__ void k_dpre_head(const float *__restrict__ h4, const float *__restrict__ dlogit,
                            const float *__restrict__ params, int Ppad, float *__restrict__ dpre,
                            uint16_t *__restrict__ dpreb, uint16_t *__restrict__ dpret)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Ppad * C)
        return;
    const int p = idx / C, c = idx - p * C;
    const float hv = h4[idx];
    const float d = dlogit[p] * params[OFF_WO + c] * (1.f - hv * hv);
    dpre[idx] = d;
    const uint16_t b = f2bf(d);
    dpreb[idx] = b;
    dpret[(size_t)c * Ppad + p] = b;
}

// partial column sums: partial[blk][c] = sum over this block's rows of A[p][c] * (w ? w[p] : 1)
__global__ __launch_bounds__(256) void k_colsum(const float *__restrict__ A, const float *__restrict__ w,
                                                int rows, int rows_per_blk, float *__restrict__ partial)
{
    // 256 threads = 4 row groups x 64 columns
    __shared__ float red[4][C];
    const int c = threadIdx.x & (C - 1), g = threadIdx.x >> 6;
    const int r0 = blockIdx.x * rows_per_blk;
    const int r1 = min(r0 + rows_per_blk, rows);
    float s = 0.f;
    for (int r = r0 + g; r < r1; r += 4)
        s += A[(size_t)r * C + c] * (w ? w[r] : 1.f);
    red[g][c] = s;
    __syncthreads();
    if (g == 0)
        partial[blockIdx.x * C + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

// out[j] (+)= sum_b partial[b][j], j < width; fixed order
__global__ void k_reduce_cols(const float *__restrict__ partial, int nb, int width, float *__restrict__ out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= width)
        return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b)
        s += partial[(size_t)b * width + j];
    out[j] = s;
}

// grad[W_l][t][c'][c] = wgrad[c][t*C + c']
__global__ void k_scatter_wgrad(const float *__restrict__ wgrad, int l, float *__restrict__ grad)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= C * KB)
        return;
    const int c = idx / KB, k = idx - c * KB;
    grad[off_w(l) + k * C + c] = wgrad[idx];
}

// dh[q][c'] = sum_t dxcol[q - tap t][t*C + c'];  dpre = dh (1 - h^2)
__global__ void k_col2im(const float *__restrict__ dxcol, const float *__restrict__ hprev, int nblk, int Bs,
                         int Ppad, float *__restrict__ dpre, uint16_t *__restrict__ dpreb,
                         uint16_t *__restrict__ dpret)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Ppad * C)
        return;
    const int q = idx / C, c = idx - q * C;
    const int BB = Bs * Bs;
    float dh = 0.f;
    if (q < nblk * BB) {
        const int n = q / BB, k = q - n * BB, i = k / Bs, j = k - i * Bs;
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            // source position p with p + tap t = q
            const int ii = i - tap_di(t), jj = j - tap_dj(t);
            if (ii < Bs && jj >= 0 && jj < Bs)
                dh += dxcol[(size_t)(n * BB + ii * Bs + jj) * KB + t * C + c];
        }
    }
    const float hv = hprev[idx];
    const float d = dh * (1.f - hv * hv);
    dpre[idx] = d;
    const uint16_t b = f2bf(d);
    dpreb[idx] = b;
    dpret[(size_t)c * Ppad + q] = b;
}

// layer-1 gradients: 10 rows (W1 taps 0..3, U1 f 0..3, v1, b1) x C, partial over positions
__global__ __launch_bounds__(256) void k_layer1_grad(const float *__restrict__ dpre1, const int8_t *__restrict__ x,
                                                     const int8_t *__restrict__ bnd, const float *__restrict__ kc,
                                                     int nblk, int Bs, int rows_per_blk, float *__restrict__ partial)
{
    __shared__ float red[4][10][C];
    const int c = threadIdx.x & (C - 1), g = threadIdx.x >> 6;
    const int BB = Bs * Bs, P = nblk * BB;
    const int r0 = blockIdx.x * rows_per_blk, r1 = min(r0 + rows_per_blk, P);
    float acc[10];
#pragma unroll
    for (int q = 0; q < 10; ++q)
        acc[q] = 0.f;
    for (int p = r0 + g; p < r1; p += 4) {
        const int n = p / BB, k = p - n * BB, i = k / Bs, j = k - i * Bs;
        const float d = dpre1[(size_t)p * C + c];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int ii = i + tap_di(t), jj = j + tap_dj(t);
            if (ii >= 0 && jj >= 0 && jj < Bs)
                acc[t] += (float)x[n * BB + ii * Bs + jj] * d;
        }
        const int8_t *bn = bnd + n * 4 * Bs;
        if (i == 0)
            acc[4] += (float)bn[j] * d;
        if (i == Bs - 1)
            acc[5] += (float)bn[Bs + j] * d;
        if (j == 0)
            acc[6] += (float)bn[2 * Bs + i] * d;
        if (j == Bs - 1)
            acc[7] += (float)bn[3 * Bs + i] * d;
        acc[8] += kc[n] * d;
        acc[9] += d;
    }
#pragma unroll
    for (int q = 0; q < 10; ++q)
        red[g][q][c] = acc[q];
    __syncthreads();
    if (g == 0)
        for (int q = 0; q < 10; ++q)
            partial[(size_t)blockIdx.x * 10 * C + q * C + c] = red[0][q][c] + red[1][q][c] + red[2][q][c] + red[3][q][c];
}

__global__ void k_adam(float *__restrict__ params, const float *__restrict__ grad, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    params[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// Autoregressive passes.  Both evaluate the conditional of every site k of a
// block given the sites before it and the boundary with one per-site
// arithmetic: layer 1 on the VALU (layer1_site), layers 2..4 as MFMA tiles
// whose 16 rows are 16 sequences at one site and whose K runs over the taps
// in a fixed order, the logit head summed in a fixed tree, and the uint32
// threshold (site_threshold).  A matrix-core product row depends only on its
// own A row, so a block scored by k_nn_score gets bit for bit the log q that
// k_nn_sample assigned when it drew it.
//  - k_nn_sample: 16 sequences per workgroup, one site per step (a site
//    depends on the one drawn just before it);
//  - k_nn_score: 16 given blocks per workgroup, one block row per step (a
//    site only looks at the row above and at sites to its left, all known),
//    so each wave runs Bs independent MFMA chains per layer.
// Each wave owns 16 output channels of layers 2..4, whose BF16 weights it
// keeps in registers for the whole pass.
// ---------------------------------------------------------------------------
constexpr int SEQ_PER_WG = 16;
constexpr int RING_ROW = C + 8;  // padded row (bf16 elements) against LDS bank conflicts

struct ArWeights {
    bf16x8 w[3][10];  // layers 2..4: this lane's B-operand slices (output channel cw)
    float bias[3], wo_c, bo;
    float w1[4], u1[4], v1, b1;  // layer 1 of channel tid & 63
};

__device__ __forceinline__ void load_ar_weights(const NetDev &net, int wave, int lane, ArWeights &p)
{
    const float *P = net.params;
    const int cw = 16 * wave + (lane & 15);
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int q = 0; q < 10; ++q)
            p.w[l][q] = load_bf16x8(net.wt + ((size_t)l * C + cw) * KB + q * 32 + 8 * (lane >> 4));
#pragma unroll
    for (int l = 0; l < 3; ++l)
        p.bias[l] = P[off_b(l + 2) + cw];
    p.wo_c = P[OFF_WO + cw];
    p.bo = P[OFF_BO];
    const int c1 = lane;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        p.w1[t] = P[OFF_W1 + t * C + c1];
        p.u1[t] = P[OFF_U1 + t * C + c1];
    }
    p.v1 = P[OFF_V1 + c1];
    p.b1 = P[OFF_B1 + c1];
}

// Layer-1 output (BF16) of channel lane at site (i, j) of one sequence: x
// holds the sequence's known sites; the site at position ov_pos (if any)
// is taken from ov_val instead.
template <int BS>
__device__ __forceinline__ uint16_t layer1_site(const int8_t *x, int ov_pos, float ov_val, const int8_t *bnd,
                                                float kc, int i, int j, const ArWeights &p)
{
    float pre = __builtin_fmaf(kc, p.v1, p.b1);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int ii = i + tap_di(t), jj = j + tap_dj(t);
        if (ii >= 0 && jj >= 0 && jj < BS) {
            const int pos = ii * BS + jj;
            pre = __builtin_fmaf(pos == ov_pos ? ov_val : (float)x[pos], p.w1[t], pre);
        }
    }
    pre += boundary_field(bnd, BS, i, j, p.u1);
    return f2bf(net_tanh(pre));
}

// uint32 threshold of a site from its logit: clamp(floor(sigmoid * 2^32), 1,
// 2^32 - 1).  The product with 2^32 is exact in FP32 and the conversion
// truncates, so this is the floor of the exact product.
__device__ __forceinline__ uint32_t site_threshold(float logit)
{
    const float scaled = net_sigmoid(logit) * 4294967296.0f;
    const uint32_t t = scaled >= 4294967296.0f ? 0xffffffffu : (uint32_t)scaled;
    return t > 1u ? t : 1u;
}

// Sum of the logit head over this wave's 16 channels for the 4 rows this
// lane holds (fixed butterfly over the 16 lanes of a row group); lane 0 of
// each group writes out[row].
__device__ __forceinline__ void head_rows(const floatx4 &acc, const ArWeights &p, int lane, float *out)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float v = net_tanh(acc[r] + p.bias[2]) * p.wo_c;
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        if ((lane & 15) == 0)
            out[4 * (lane >> 4) + r] = v;
    }
}

__device__ __forceinline__ float head_logit(const float *h0, const float *h1, const float *h2, const float *h3,
                                            int row, float bo)
{
    return ((h0[row] + h1[row]) + (h2[row] + h3[row])) + bo;
}

// log q = sum_k log(thr_k or 2^32 - thr_k) - BB * 32 ln 2 in FP64, summed in a
// fixed order: 16 parts of 4 consecutive sites, then the parts in order.
__device__ __forceinline__ void logq_parts(const int8_t (*xs)[64], const uint32_t (*thr)[64], int BB, int tid,
                                           double (*part)[16])
{
    const int s = tid >> 4, pt = tid & 15;
    double acc = 0.0;
    for (int k = pt * 4; k < pt * 4 + 4 && k < BB; ++k) {
        const double t = (double)thr[s][k];
        acc += log(xs[s][k] > 0 ? t : 4294967296.0 - t);
    }
    part[s][pt] = acc;
}

__device__ __forceinline__ double logq_total(const double *part, int BB)
{
    double sum = 0.0;
    for (int pt = 0; pt < 16; ++pt)
        sum += part[pt];
    return sum - (double)BB * 32.0 * 0.69314718055994530942;
}

template <int BS>
__global__ __launch_bounds__(256) void k_nn_sample(NetDev net, SeqDev seq, int first, int n_seq)
{
    constexpr int BB = BS * BS;
    __shared__ __attribute__((aligned(16))) uint16_t ring[3][RING][SEQ_PER_WG][RING_ROW];
    __shared__ float head_part[4][SEQ_PER_WG];
    __shared__ int8_t xs[SEQ_PER_WG][64];
    __shared__ int8_t bs[SEQ_PER_WG][32];
    __shared__ uint32_t ut[SEQ_PER_WG][64];  // site uniform; replaced by the site's threshold once drawn
    __shared__ float ks[SEQ_PER_WG];
    __shared__ double lq_part[SEQ_PER_WG][16];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int s0 = first + blockIdx.x * SEQ_PER_WG, end = first + n_seq;

    for (int i = tid; i < SEQ_PER_WG * 64; i += 256)
        xs[i >> 6][i & 63] = 0;
    for (int i = tid; i < SEQ_PER_WG * 32; i += 256) {
        const int s = i >> 5, k = i & 31;
        bs[s][k] = (s0 + s < end && k < 4 * BS) ? seq.bnd[(size_t)(s0 + s) * 4 * BS + k] : (int8_t)0;
    }
    if (tid < SEQ_PER_WG)
        ks[tid] = s0 + tid < end ? seq.coupling[s0 + tid] : 0.f;
    // site uniforms: word site & 3 of Philox(ctr = (site >> 2, round, replica, 3)),
    // site = blk * BB + k; BB is a multiple of 4, so one call serves sites 4m..4m+3
    for (int i = tid; i < SEQ_PER_WG * 16; i += 256) {
        const int s = i >> 4, m = i & 15;
        if (s0 + s < end && 4 * m < BB) {
            const uint32_t *kk = seq.key + 4 * (size_t)(s0 + s);
            const uint32_t site0 = seq.blk[s0 + s] * (uint32_t)BB + 4u * m;
            uint32_t o[4];
            philox4x32_10(site0 >> 2, kk[3], kk[2], 3u, kk[0], kk[1], o);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                ut[s][4 * m + r] = o[r];
        }
    }
    ArWeights p;
    load_ar_weights(net, wave & 3, lane, p);
    const int cw = 16 * wave + (lane & 15);
    __syncthreads();

    for (int k = 0; k <= BB; ++k) {
        const int i = k / BS, j = k - i * BS, slot = k % RING;
        // draw site k - 1 of this wave's sequences (every lane of the wave
        // evaluates the same decision; lane 0 records it), then layer 1 of site k
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int s = wave + 4 * q;
            float xprev = 0.f;
            if (k > 0) {
                const uint32_t thr = site_threshold(
                    head_logit(head_part[0], head_part[1], head_part[2], head_part[3], s, p.bo));
                const int8_t xv = ut[s][k - 1] < thr ? (int8_t)1 : (int8_t)-1;
                xprev = (float)xv;
                if (lane == 0) {
                    xs[s][k - 1] = xv;
                    ut[s][k - 1] = thr;
                }
            }
            if (k < BB)
                ring[0][slot][s][lane] = layer1_site<BS>(&xs[s][0], k - 1, xprev, &bs[s][0], ks[s], i, j, p);
        }
        __syncthreads();
        if (k == BB)
            break;
        // layers 2..4 on the matrix cores; layer 4 feeds the logit head directly
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 10; ++q) {
                const int t = q >> 1, half = q & 1;
                const int ii = i + tap_di(t), jj = j + tap_dj(t);
                bf16x8 a = zero_bf16x8();
                if (ii >= 0 && jj >= 0 && jj < BS) {
                    const int pslot = (k + tap_di(t) * BS + tap_dj(t) + RING) % RING;
                    a = load_bf16x8(&ring[l][pslot][lane & 15][half * 32 + 8 * (lane >> 4)]);
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, p.w[l][q], acc, 0, 0, 0);
            }
            if (l < 2) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    ring[l + 1][slot][4 * (lane >> 4) + r][cw] = f2bf(net_tanh(acc[r] + p.bias[l]));
            } else {
                head_rows(acc, p, lane, head_part[wave]);
            }
            __syncthreads();
        }
    }
    logq_parts(xs, ut, BB, tid, lq_part);
    __syncthreads();
    for (int i = tid; i < SEQ_PER_WG * 64; i += 256) {
        const int s = i >> 6, k = i & 63;
        if (s0 + s < end && k < BB)
            seq.x[(size_t)(s0 + s) * BB + k] = xs[s][k];
    }
    if (tid < SEQ_PER_WG && s0 + tid < end)
        seq.logq[s0 + tid] = logq_total(lq_part[tid], BB);
}

// 512 threads: wave w computes output channels 16 (w & 3) .. +15 for the
// sites j of a row with j / (BS / 2) == w >> 2 (half the row's tiles).
template <int BS>
__global__ __launch_bounds__(512) void k_nn_score(NetDev net, SeqDev seq, int n_seq)
{
    constexpr int BB = BS * BS, HT = BS / 2;  // tiles per wave
    // layer outputs of the current and the previous block row: [layer][row & 1][site j][sequence][channel]
    __shared__ __attribute__((aligned(16))) uint16_t rows[3][2][BS][SEQ_PER_WG][RING_ROW];
    __shared__ float head_part[4][BS][SEQ_PER_WG];
    __shared__ int8_t xs[SEQ_PER_WG][64];
    __shared__ int8_t bs[SEQ_PER_WG][32];
    __shared__ uint32_t thr_s[SEQ_PER_WG][64];
    __shared__ float ks[SEQ_PER_WG];
    __shared__ double lq_part[SEQ_PER_WG][16];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int nsl = wave & 3, j0 = (wave >> 2) * HT;
    const int s0 = blockIdx.x * SEQ_PER_WG;

    for (int i = tid; i < SEQ_PER_WG * 64; i += 512) {
        const int s = i >> 6, k = i & 63;
        xs[s][k] = (s0 + s < n_seq && k < BB) ? seq.x[(size_t)(s0 + s) * BB + k] : (int8_t)0;
    }
    for (int i = tid; i < SEQ_PER_WG * 32; i += 512) {
        const int s = i >> 5, k = i & 31;
        bs[s][k] = (s0 + s < n_seq && k < 4 * BS) ? seq.bnd[(size_t)(s0 + s) * 4 * BS + k] : (int8_t)0;
    }
    if (tid < SEQ_PER_WG)
        ks[tid] = s0 + tid < n_seq ? seq.coupling[s0 + tid] : 0.f;
    ArWeights p;
    load_ar_weights(net, nsl, lane, p);
    const int cw = 16 * nsl + (lane & 15);
    __syncthreads();

    for (int i = 0; i < BS; ++i) {
        const int par = i & 1;
        // layer 1 of row i: channel lane, sequences wave and wave + 8, every site
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int s = wave + 8 * q;
#pragma unroll
            for (int j = 0; j < BS; ++j)
                rows[0][par][j][s][lane] = layer1_site<BS>(&xs[s][0], -1, 0.f, &bs[s][0], ks[s], i, j, p);
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            floatx4 acc[HT];
#pragma unroll
            for (int jt = 0; jt < HT; ++jt)
                acc[jt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 10; ++q) {
                const int t = q >> 1, half = q & 1;
                const int ii = i + tap_di(t);
#pragma unroll
                for (int jt = 0; jt < HT; ++jt) {
                    const int jj = j0 + jt + tap_dj(t);
                    bf16x8 a = zero_bf16x8();
                    if (ii >= 0 && jj >= 0 && jj < BS)
                        a = load_bf16x8(&rows[l][ii & 1][jj][lane & 15][half * 32 + 8 * (lane >> 4)]);
                    acc[jt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, p.w[l][q], acc[jt], 0, 0, 0);
                }
            }
#pragma unroll
            for (int jt = 0; jt < HT; ++jt) {
                if (l < 2) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        rows[l + 1][par][j0 + jt][4 * (lane >> 4) + r][cw] =
                            f2bf(net_tanh(acc[jt][r] + p.bias[l]));
                } else {
                    head_rows(acc[jt], p, lane, head_part[nsl][j0 + jt]);
                }
            }
            __syncthreads();
        }
        if (tid < SEQ_PER_WG * BS) {
            const int s = tid / BS, j = tid - s * BS;
            thr_s[s][i * BS + j] = site_threshold(
                head_logit(head_part[0][j], head_part[1][j], head_part[2][j], head_part[3][j], s, p.bo));
        }
    }
    __syncthreads();
    if (tid < 256)
        logq_parts(xs, thr_s, BB, tid, lq_part);
    __syncthreads();
    if (tid < SEQ_PER_WG && s0 + tid < n_seq)
        seq.logq[s0 + tid] = logq_total(lq_part[tid], BB);
}

// ---------------------------------------------------------------------------
// lattice <-> blocks
// ---------------------------------------------------------------------------
__device__ __forceinline__ int spin_at(const RepDev &d, uint32_t x, uint32_t y)
{
    const uint32_t c = (x + y) & 1u, k = x >> 1;
    const uint32_t w = d.plane0[c * d.Ly * d.W + y * d.W + (k >> 5)];
    return ((w >> (k & 31)) & 1u) ? 1 : -1;
}

// block (bx, by) of a replica -> its spins and boundary
__device__ void read_block(const RepDev &d, int Bs, uint32_t bx, uint32_t by, int8_t *x, int8_t *bnd)
{
    const uint32_t x0 = bx * Bs, y0 = by * Bs;
    for (int i = 0; i < Bs; ++i)
        for (int j = 0; j < Bs; ++j)
            x[i * Bs + j] = (int8_t)spin_at(d, x0 + j, y0 + i);
    const uint32_t yu = y0 == 0 ? d.Ly - 1 : y0 - 1, yd = (y0 + Bs) % d.Ly;
    const uint32_t xl = x0 == 0 ? d.Lx - 1 : x0 - 1, xr = (x0 + Bs) % d.Lx;
    for (int j = 0; j < Bs; ++j) {
        bnd[j] = (int8_t)spin_at(d, x0 + j, yu);
        bnd[Bs + j] = (int8_t)spin_at(d, x0 + j, yd);
    }
    for (int i = 0; i < Bs; ++i) {
        bnd[2 * Bs + i] = (int8_t)spin_at(d, xl, y0 + i);
        bnd[3 * Bs + i] = (int8_t)spin_at(d, xr, y0 + i);
    }
}

// colour-`colour` block number idx of a replica -> (bx, by); blocks alternate in colour
__device__ __forceinline__ void block_coords(uint32_t idx, uint32_t nbx, uint32_t colour, uint32_t *bx, uint32_t *by)
{
    const uint32_t half = nbx / 2;
    *by = idx / half;
    *bx = 2 * (idx - *by * half) + ((*by + colour) & 1u);
}

// Boundary spin q of block (bx, by): top row, bottom row, left column, right
// column, Bs each, periodic.
__device__ __forceinline__ int8_t boundary_spin(const RepDev &d, int Bs, uint32_t bx, uint32_t by, int q)
{
    const uint32_t x0 = bx * Bs, y0 = by * Bs;
    const int side = q / Bs, m = q - side * Bs;
    uint32_t x, y;
    if (side < 2) {
        x = x0 + m;
        y = side == 0 ? (y0 == 0 ? d.Ly - 1 : y0 - 1) : (y0 + Bs) % d.Ly;
    } else {
        y = y0 + m;
        x = side == 2 ? (x0 == 0 ? d.Lx - 1 : x0 - 1) : (x0 + Bs) % d.Lx;
    }
    return (int8_t)spin_at(d, x, y);
}

// One wave per block of the round: sequence b scores the current block,
// sequence count + b draws the proposal with the same boundary.  Lane k reads
// site k and boundary spin k.
__global__ __launch_bounds__(256) void k_block_gather(const RepDev *__restrict__ reps, const double *__restrict__ kcoup,
                                                      int Bs, uint32_t colour, uint32_t round, uint32_t first,
                                                      uint32_t count, uint32_t per_rep, SeqDev seq)
{
    const uint32_t b = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= count)
        return;
    const uint32_t g = first + b, r = g / per_rep, idx = g - r * per_rep;
    const RepDev d = reps[r];
    const uint32_t nbx = d.Lx / Bs;
    uint32_t bx, by;
    block_coords(idx, nbx, colour, &bx, &by);
    const int BB = Bs * Bs;
    if (lane < BB) {
        const int i = lane / Bs, j = lane - i * Bs;
        seq.x[(size_t)b * BB + lane] = (int8_t)spin_at(d, bx * Bs + j, by * Bs + i);
    }
    if (lane < 4 * Bs) {
        const int8_t v = boundary_spin(d, Bs, bx, by, lane);
        seq.bnd[(size_t)b * 4 * Bs + lane] = v;
        seq.bnd[(size_t)(count + b) * 4 * Bs + lane] = v;
    }
    if (lane < 2) {
        const size_t s = b + (size_t)lane * count;
        seq.coupling[s] = (float)kcoup[r];
        seq.key[4 * s + 0] = d.seed_lo;
        seq.key[4 * s + 1] = d.seed_hi;
        seq.key[4 * s + 2] = d.replica;
        seq.key[4 * s + 3] = round;
        seq.blk[s] = by * nbx + bx;
    }
}

// Metropolis-Hastings for each gathered block, one wave per block: lane k
// adds the change of the bonds of site k to its right and lower neighbours
// inside the block and to the boundary; the exact integer sum decides with
// log A = K dB + log q(current) - log q(proposal) against a 53-bit uniform.
// Accepted proposals are XORed into the packed planes (only this block's
// bits; same-colour blocks never share a bond, so concurrent blocks do not
// interact).
__global__ __launch_bounds__(256) void k_block_mh(const RepDev *__restrict__ reps, const double *__restrict__ kcoup,
                                                  int Bs, uint32_t colour, uint32_t round, uint32_t first,
                                                  uint32_t count, uint32_t per_rep, SeqDev seq,
                                                  unsigned long long *__restrict__ accepts)
{
    const uint32_t b = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= count)
        return;
    const uint32_t g = first + b, r = g / per_rep, idx = g - r * per_rep;
    const RepDev d = reps[r];
    const uint32_t nbx = d.Lx / Bs;
    uint32_t bx, by;
    block_coords(idx, nbx, colour, &bx, &by);
    const int BB = Bs * Bs;
    const int8_t *s = seq.x + (size_t)b * BB;
    const int8_t *sp = seq.x + (size_t)(count + b) * BB;
    const int8_t *bn = seq.bnd + (size_t)b * 4 * Bs;
    int dB = 0, changed = 0;
    if (lane < BB) {
        const int i = lane / Bs, j = lane - i * Bs, k = lane;
        const int a = s[k], ap = sp[k];
        changed = a != ap;
        if (j + 1 < Bs)
            dB += ap * sp[k + 1] - a * s[k + 1];
        if (i + 1 < Bs)
            dB += ap * sp[k + Bs] - a * s[k + Bs];
        if (i == 0)
            dB += (ap - a) * bn[j];
        if (i == Bs - 1)
            dB += (ap - a) * bn[Bs + j];
        if (j == 0)
            dB += (ap - a) * bn[2 * Bs + i];
        if (j == Bs - 1)
            dB += (ap - a) * bn[3 * Bs + i];
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        dB += __shfl_xor(dB, m, 64);
    // log of pi(s') q(s) / (pi(s) q(s')), pi ~ exp(K B)
    const double logA = kcoup[r] * (double)dB + seq.logq[b] - seq.logq[count + b];
    uint32_t o[4];
    philox4x32_10(by * nbx + bx, round, d.replica, 4u, d.seed_lo, d.seed_hi, o);
    const double u = (double)(((uint64_t)o[0] << 21) | (o[1] >> 11)) * 1.1102230246251565404e-16;  // 2^-53
    const bool accept = logA >= 0.0 || u < exp(logA);
    if (!accept)
        return;
    if (lane == 0)
        atomicAdd(&accepts[r], 1ull);
    if (changed) {
        const int i = lane / Bs, j = lane - i * Bs;
        const uint32_t x = bx * Bs + j, y = by * Bs + i, c = (x + y) & 1u, kk = x >> 1;
        atomicXor(&d.plane0[c * d.Ly * d.W + y * d.W + (kk >> 5)], 1u << (kk & 31));
    }
}

// training samples: block position of sample i of replica r drawn from
// Philox(ctr = {i, draw, replica, 5})
__global__ void k_extract(const RepDev *__restrict__ reps, const double *__restrict__ kcoup, int Bs,
                          uint32_t per_rep, uint32_t count, uint32_t draw, int8_t *__restrict__ x,
                          int8_t *__restrict__ bnd, float *__restrict__ kout)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count)
        return;
    const uint32_t r = q / per_rep, i = q - r * per_rep;
    const RepDev d = reps[r];
    uint32_t o[4];
    philox4x32_10(i, draw, d.replica, 5u, d.seed_lo, d.seed_hi, o);
    const uint32_t bx = o[0] % (d.Lx / Bs), by = o[1] % (d.Ly / Bs);
    read_block(d, Bs, bx, by, x + (size_t)q * Bs * Bs, bnd + (size_t)q * 4 * Bs);
    kout[q] = (float)kcoup[r];
}

// Minibatch drawn on the device: row i of training step k is
// floor(u * n_rows / 2^32) with u the first word of Philox(ctr = (i, k, 0, 6),
// key = seed); one workgroup of 64 threads copies one row.
__global__ __launch_bounds__(64) void k_gather_rows(const int8_t *__restrict__ x, const int8_t *__restrict__ bnd,
                                                    const float *__restrict__ kc, uint32_t n_rows, int BB, int NB,
                                                    uint32_t step, uint32_t seed_lo, uint32_t seed_hi,
                                                    int8_t *__restrict__ tx, int8_t *__restrict__ tb,
                                                    float *__restrict__ tk)
{
    const uint32_t i = blockIdx.x;
    uint32_t o[4];
    philox4x32_10(i, step, 0u, 6u, seed_lo, seed_hi, o);
    const size_t row = (size_t)(((uint64_t)o[0] * n_rows) >> 32);
    for (int j = threadIdx.x; j < BB; j += 64)
        tx[(size_t)i * BB + j] = x[row * BB + j];
    for (int j = threadIdx.x; j < NB; j += 64)
        tb[(size_t)i * NB + j] = bnd[row * NB + j];
    if (threadIdx.x == 0)
        tk[i] = kc[row];
}

// standalone sampled sequences: Philox key and block id of sequence i
__global__ void k_seq_setup(SeqDev seq, int n, uint32_t seed_lo, uint32_t seed_hi, uint32_t replica, uint32_t round,
                            uint32_t blk0)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    seq.key[4 * i + 0] = seed_lo;
    seq.key[4 * i + 1] = seed_hi;
    seq.key[4 * i + 2] = replica;
    seq.key[4 * i + 3] = round;
    seq.blk[i] = blk0 + (uint32_t)i;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t cast_weights(const NetDev &net, hipStream_t st)
{
    hipLaunchKernelGGL(k_cast_weights, dim3(blocks_for(3L * C * KB, 256)), dim3(256), 0, st, net.params, net.wt,
                       net.wtt);
    return hipGetLastError();
}

hipError_t gemm_nt(const uint16_t *A, int lda, const uint16_t *Bt, int ldb, float *Cm, int ldc, int M, int N,
                   int K, hipStream_t st)
{
    hipLaunchKernelGGL(k_gemm_nt, dim3(blocks_for(N, 64), blocks_for(M, 64), 1), dim3(256), 0, st, A, lda, Bt, ldb,
                       Cm, ldc, M, N, K, K);
    return hipGetLastError();
}

// Split-K product for a small output and a long K (the weight gradients):
// partials of kchunk-long K ranges go to part[S][M][N], then a fixed-order sum.
static hipError_t gemm_nt_splitk(const uint16_t *A, int lda, const uint16_t *Bt, int ldb, float *part, float *Cm,
                                 int M, int N, int K, int kchunk, hipStream_t st)
{
    const int S = (K + kchunk - 1) / kchunk;
    hipLaunchKernelGGL(k_gemm_nt, dim3(blocks_for(N, 64), blocks_for(M, 64), S), dim3(256), 0, st, A, lda, Bt, ldb,
                       part, N, M, N, K, kchunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sum_splits, dim3(blocks_for((long)M * N, 256)), dim3(256), 0, st, part, S, M * N, Cm);
    return hipGetLastError();
}

// forward of nblk blocks; logits[P]; returns the padded position count in *ppad
hipError_t forward(const NetDev &net, const TrainWs &ws, const int8_t *x, const int8_t *bnd, const float *kc,
                   int nblk, int Bs, hipStream_t st)
{
    const int Pv = nblk * Bs * Bs, Pp = (Pv + 63) / 64 * 64;
    hipLaunchKernelGGL(k_layer1, dim3(blocks_for((long)Pp * C, 256)), dim3(256), 0, st, net.params, x, bnd, kc,
                       nblk, Bs, Pp, ws.h[0], ws.hb[0]);
    for (int l = 2; l <= 4; ++l) {
        const int li = l - 2;
        hipLaunchKernelGGL(k_im2col, dim3(blocks_for((long)Pp * 5 * (C / 8), 256)), dim3(256), 0, st,
                           ws.hb[li], nblk, Bs, Pp, ws.xcol[li], ws.xcolt[li]);
        hipError_t e = gemm_nt(ws.xcol[li], KB, net.wt + (size_t)li * C * KB, KB, ws.pre, C, Pp, C, KB, st);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_bias_tanh, dim3(blocks_for((long)Pp * C, 256)), dim3(256), 0, st, ws.pre,
                           net.params + off_b(l), Pv, Pp, ws.h[l - 1], l < 4 ? ws.hb[l - 1] : (uint16_t *)nullptr);
    }
    hipLaunchKernelGGL(k_head, dim3(blocks_for(Pv, 256)), dim3(256), 0, st, ws.h[3], net.params, Pv, ws.logits);
    const int nb = blocks_for(Pp, 256);
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, st, ws.logits, x, Pv, Pp, ws.dlogit, ws.partial);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, ws.partial, nb, 1.f / (float)Pv, ws.loss);
    return hipGetLastError();
}

hipError_t backward(const NetDev &net, const TrainWs &ws, const int8_t *x, const int8_t *bnd, const float *kc,
                    int nblk, int Bs, hipStream_t st)
{
    const int Pv = nblk * Bs * Bs, Pp = (Pv + 63) / 64 * 64;
    const int rows_per_blk = 256;
    const int nbr = blocks_for(Pp, rows_per_blk);
    // head: dwo = sum_p h4[p] dlogit[p]; dbo = sum_p dlogit[p]
    hipLaunchKernelGGL(k_colsum, dim3(nbr), dim3(256), 0, st, ws.h[3], ws.dlogit, Pp, rows_per_blk, ws.partial);
    hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(C), 0, st, ws.partial, nbr, C, net.grad + OFF_WO);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, ws.dlogit, Pp, 1.f, net.grad + OFF_BO);
    hipLaunchKernelGGL(k_dpre_head, dim3(blocks_for((long)Pp * C, 256)), dim3(256), 0, st, ws.h[3], ws.dlogit,
                       net.params, Pp, ws.dpre, ws.dpreb, ws.dpret);
    for (int l = 4; l >= 2; --l) {
        const int li = l - 2;
        hipLaunchKernelGGL(k_colsum, dim3(nbr), dim3(256), 0, st, ws.dpre, (const float *)nullptr, Pp, rows_per_blk,
                           ws.partial);
        hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(C), 0, st, ws.partial, nbr, C, net.grad + off_b(l));
        // weight gradient [C][KB] = dpre^T (C x P) . xcol (P x KB), split over P in
        // chunks of 512 positions; the partials use ws.pre, which is free here
        // (S C KB <= Pp KB floats)
        hipError_t e = gemm_nt_splitk(ws.dpret, Pp, ws.xcolt[li], Pp, ws.pre, ws.wgrad, C, KB, Pp, 512, st);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_scatter_wgrad, dim3(blocks_for((long)C * KB, 256)), dim3(256), 0, st, ws.wgrad, l,
                           net.grad);
        // data gradient [P][KB] = dpre (P x C) . W (C x KB)
        e = gemm_nt(ws.dpreb, C, net.wtt + (size_t)li * KB * C, C, ws.pre, KB, Pp, KB, C, st);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_col2im, dim3(blocks_for((long)Pp * C, 256)), dim3(256), 0, st, ws.pre, ws.h[l - 2],
                           nblk, Bs, Pp, ws.dpre, ws.dpreb, ws.dpret);
    }
    hipLaunchKernelGGL(k_layer1_grad, dim3(nbr), dim3(256), 0, st, ws.dpre, x, bnd, kc, nblk, Bs, rows_per_blk,
                       ws.partial);
    // rows: W1 taps (4), U1 (4), v1, b1 -> contiguous in the flat vector starting at OFF_W1
    hipLaunchKernelGGL(k_reduce_cols, dim3(blocks_for(10 * C, 256)), dim3(256), 0, st, ws.partial, nbr, 10 * C,
                       net.grad + OFF_W1);
    return hipGetLastError();
}

hipError_t adam(const NetDev &net, float lr, int step, hipStream_t st)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(N_PARAMS, 256)), dim3(256), 0, st, net.params, net.grad, net.adam_m,
                       net.adam_v, N_PARAMS, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

template <int BS>
static hipError_t ar_pass_bs(const NetDev &net, const SeqDev &seq, int n_score, int n_sample, hipStream_t st)
{
    if (n_score > 0) {
        hipLaunchKernelGGL(k_nn_score<BS>, dim3(blocks_for(n_score, SEQ_PER_WG)), dim3(512), 0, st, net, seq,
                           n_score);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (n_sample > 0) {
        hipLaunchKernelGGL(k_nn_sample<BS>, dim3(blocks_for(n_sample, SEQ_PER_WG)), dim3(256), 0, st, net, seq,
                           n_score, n_sample);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t ar_pass(const NetDev &net, const SeqDev &seq, int n_score, int n_sample, int Bs, hipStream_t st)
{
    switch (Bs) {
    case 2: return ar_pass_bs<2>(net, seq, n_score, n_sample, st);
    case 4: return ar_pass_bs<4>(net, seq, n_score, n_sample, st);
    case 8: return ar_pass_bs<8>(net, seq, n_score, n_sample, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t block_gather(const RepDev *reps, const double *kcoup, int Bs, uint32_t colour, uint32_t round,
                        uint32_t first, uint32_t count, uint32_t per_rep, const SeqDev &seq, hipStream_t st)
{
    hipLaunchKernelGGL(k_block_gather, dim3(blocks_for(count, 4)), dim3(256), 0, st, reps, kcoup, Bs, colour,
                       round, first, count, per_rep, seq);
    return hipGetLastError();
}

hipError_t block_mh(const RepDev *reps, const double *kcoup, int Bs, uint32_t colour, uint32_t round,
                    uint32_t first, uint32_t count, uint32_t per_rep, const SeqDev &seq, int64_t *accepts,
                    hipStream_t st)
{
    hipLaunchKernelGGL(k_block_mh, dim3(blocks_for(count, 4)), dim3(256), 0, st, reps, kcoup, Bs, colour, round,
                       first, count, per_rep, seq, reinterpret_cast<unsigned long long *>(accepts));
    return hipGetLastError();
}

hipError_t seq_setup(const SeqDev &seq, int n, uint64_t seed, uint32_t replica, uint32_t round, uint32_t blk0,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_seq_setup, dim3(blocks_for(n, 256)), dim3(256), 0, st, seq, n,
                       (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), replica, round, blk0);
    return hipGetLastError();
}

hipError_t gather_rows(const TrainWs &ws, const int8_t *x, const int8_t *bnd, const float *kc, uint32_t n_rows,
                       int batch, int Bs, uint32_t step, uint64_t seed, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_rows, dim3(batch), dim3(64), 0, st, x, bnd, kc, n_rows, Bs * Bs, 4 * Bs, step,
                       (uint32_t)seed, (uint32_t)(seed >> 32), ws.tx, ws.tbnd, ws.tcoup);
    return hipGetLastError();
}

hipError_t extract(const RepDev *reps, const double *kcoup, int Bs, uint32_t per_rep, uint32_t count,
                   uint32_t draw, int8_t *x, int8_t *bnd, float *kout, hipStream_t st)
{
    hipLaunchKernelGGL(k_extract, dim3(blocks_for(count, 256)), dim3(256), 0, st, reps, kcoup, Bs, per_rep, count,
                       draw, x, bnd, kout);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace ising
