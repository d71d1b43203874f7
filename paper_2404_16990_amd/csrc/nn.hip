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

// float -> bfloat16 bits, round to nearest even (inputs are finite): one
// v_cvt_pk_bf16_f32 on gfx950
__device__ __forceinline__ uint16_t f2bf(float f)
{
    return __builtin_bit_cast(uint16_t, (__bf16)f);
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
// parameters -> BF16 matrix-core operands
// ---------------------------------------------------------------------------
__global__ void k_cast_weights(const float *__restrict__ params, uint16_t *__restrict__ wt,
                               uint16_t *__restrict__ wtd)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // over 3 * C * KB
    if (idx >= 3 * C * KB)
        return;
    const int l = idx / (C * KB), r = idx - l * C * KB;
    const int c = r / KB, k = r - c * KB;          // output channel, K index t*C + c'
    const int t = k / C, ci = k - t * C;
    const uint16_t b = f2bf(params[off_w(l + 2) + k * C + c]);  // W_l[t][c'][c]
    wt[(l * C + c) * KB + k] = b;
    wtd[(l * C + ci) * KB + t * C + c] = b;
}

// ---------------------------------------------------------------------------
// Masked 3x3 convolution of a layer as an implicit GEMM on the matrix cores
// (BF16 operands, FP32 accumulation).  K = 5 taps x 64 channels in the order
// t*C + c; a row's A is read straight from the activation rows at the tap
// offsets (zero where the tap leaves the block), so no unfolded copy exists.
//  forward (BWD = false), rows p, columns c:
//    pre[p][c] = sum_t sum_c' in[p + off(t)][c'] W_t[c'][c]   (B = wt)
//    out = tanh(pre + bias) and its BF16 copy (rows past Pvalid: 0)
//  data gradient (BWD = true), rows q, columns c':
//    dh[q][c'] = sum_t sum_c in[q - off(t)][c] W_t[c'][c]     (B = wtd)
//    out = dh (1 - hprev^2) and its BF16 copy
// 256 threads per 64 rows x 64 columns; each wave a 32 x 32 quarter of 2 x 2
// MFMA 16x16x32 tiles.
// ---------------------------------------------------------------------------
template <bool BWD>
__global__ __launch_bounds__(256) void k_conv(const uint16_t *__restrict__ in, const uint16_t *__restrict__ Bt,
                                              const float *__restrict__ bias, const float *__restrict__ hprev,
                                              int Pvalid, int Bs, float *__restrict__ out,
                                              uint16_t *__restrict__ outb)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = blockIdx.x * 64 + (wave >> 1) * 32, n0 = (wave & 1) * 32;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const int BB = Bs * Bs;
    int base[2], ri[2], rj[2];
    bool live[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int p = m0 + a * 16 + r;
        live[a] = p < Pvalid;
        const int n = p / BB, k = p - n * BB;
        base[a] = n * BB;
        ri[a] = k / Bs;
        rj[a] = k - ri[a] * Bs;
    }
    floatx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        const int t = q >> 1, half = q & 1;
        const int di = BWD ? -tap_di(t) : tap_di(t), dj = BWD ? -tap_dj(t) : tap_dj(t);
        bf16x8 av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int ii = ri[a] + di, jj = rj[a] + dj;
            av[a] = (live[a] && ii >= 0 && ii < Bs && jj >= 0 && jj < Bs)
                        ? load_bf16x8(in + (size_t)(base[a] + ii * Bs + jj) * C + half * 32 + kq)
                        : zero_bf16x8();
        }
#pragma unroll
        for (int b = 0; b < 2; ++b)
            bv[b] = load_bf16x8(Bt + (size_t)(n0 + b * 16 + r) * KB + q * 32 + kq);
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
                const int p = m0 + a * 16 + 4 * (lane >> 4) + i, c = n0 + b * 16 + r;
                const size_t idx = (size_t)p * C + c;
                float v;
                if (BWD) {
                    const float hv = hprev[idx];
                    v = acc[a][b][i] * (1.f - hv * hv);
                } else {
                    v = p < Pvalid ? net_tanh(acc[a][b][i] + bias[c]) : 0.f;
                }
                out[idx] = v;
                if (outb)
                    outb[idx] = f2bf(v);
            }
}

// ---------------------------------------------------------------------------
// Weight gradient of a layer, split over positions (the K of the product):
//   part[s][c][t*C + c'] = sum over the positions p of split s of
//                          dpreb[p][c] in[p + off(t)][c']   (0 where the tap leaves the block)
// Each step stages 32 positions of both operands in LDS, transposed, so a
// matrix-core operand (8 consecutive positions of one channel) is one 16-byte
// read.  Grid: 5 taps x splits; each wave a 32 x 32 quarter of the 64 x 64 tile.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t *__restrict__ dpreb, const uint16_t *__restrict__ in,
                                               int Pvalid, int Bs, float *__restrict__ part)
{
    constexpr int ROW = 40;  // 32 positions + padding (bf16 elements; rows stay 16-byte aligned)
    __shared__ __attribute__((aligned(16))) uint16_t at[C][ROW];
    __shared__ __attribute__((aligned(16))) uint16_t bt[C][ROW];
    const int t = blockIdx.x, s = blockIdx.y;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = (wave >> 1) * 32, n0 = (wave & 1) * 32;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const int pl = tid >> 3, c8 = (tid & 7) * 8;  // staging: position in step, channel chunk
    const int BB = Bs * Bs;
    floatx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int p_begin = s * WGRAD_CHUNK, p_end = min(p_begin + WGRAD_CHUNK, Pvalid);
    for (int p0 = p_begin; p0 < p_end; p0 += 32) {
        const int p = p0 + pl;
        uint4 va = make_uint4(0u, 0u, 0u, 0u), vb = va;
        if (p < p_end) {
            va = *reinterpret_cast<const uint4 *>(dpreb + (size_t)p * C + c8);
            const int n = p / BB, k = p - n * BB, i = k / Bs, j = k - i * Bs;
            const int ii = i + tap_di(t), jj = j + tap_dj(t);
            if (ii >= 0 && jj >= 0 && jj < Bs)
                vb = *reinterpret_cast<const uint4 *>(in + (size_t)(n * BB + ii * Bs + jj) * C + c8);
        }
        const uint16_t *ea = reinterpret_cast<const uint16_t *>(&va);
        const uint16_t *eb = reinterpret_cast<const uint16_t *>(&vb);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            at[c8 + q][pl] = ea[q];
            bt[c8 + q][pl] = eb[q];
        }
        __syncthreads();
        bf16x8 av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
            av[a] = load_bf16x8(&at[m0 + a * 16 + r][kq]);
#pragma unroll
        for (int b = 0; b < 2; ++b)
            bv[b] = load_bf16x8(&bt[n0 + b * 16 + r][kq]);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = m0 + a * 16 + 4 * (lane >> 4) + i, ci = n0 + b * 16 + r;
                part[((size_t)s * C + c) * KB + t * C + ci] = acc[a][b][i];
            }
}

// grad W_l[t][c'][c] = sum over splits s (in order) of part[s][c][t*C + c']
__global__ void k_wgrad_sum(const float *__restrict__ part, int S, int l, float *__restrict__ grad)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= C * KB)
        return;
    const int c = idx / KB, k = idx - c * KB;
    float v = 0.f;
    for (int s = 0; s < S; ++s)
        v += part[(size_t)s * C * KB + idx];
    grad[off_w(l) + k * C + c] = v;
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
// dpre4 = dlogit * wo * (1 - h4^2), in fp32 and bf16
__global__ void k_dpre_head(const float *__restrict__ h4, const float *__restrict__ dlogit,
                            const float *__restrict__ params, int Ppad, float *__restrict__ dpre,
                            uint16_t *__restrict__ dpreb)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Ppad * C)
        return;
    const int p = idx / C, c = idx - p * C;
    const float hv = h4[idx];
    const float d = dlogit[p] * params[OFF_WO + c] * (1.f - hv * hv);
    dpre[idx] = d;
    dpreb[idx] = f2bf(d);
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

// Adam step number t = (steps taken) + 1 from the device counter, so a
// captured training step stays valid for every replay; the bias corrections
// 1 - beta^t are formed in FP64 from the exact decimal betas.
__global__ void k_adam(float *__restrict__ params, const float *__restrict__ grad, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps,
                       const uint32_t *__restrict__ steps_taken)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double t = (double)*steps_taken + 1.0;
    const float c1 = (float)(1.0 - pow(0.9, t)), c2 = (float)(1.0 - pow(0.999, t));
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
// arithmetic: every layer as matrix-core tiles of 16 rows (layer 1 in FP32,
// layer1_tile; layers 2..4 in BF16 with K running over the taps in a fixed
// order), the logit head summed in a fixed tree, and the uint32 threshold
// (site_threshold).  A matrix-core product row depends only on its own A
// row, so a block scored by
// k_nn_score gets bit for bit the log q that k_nn_sample assigned when it
// drew it.
//  - k_nn_sample: 16 sequences per workgroup, one site per step (a site
//    depends on the one drawn just before it); a tile's rows are the 16
//    sequences at one site;
//  - k_nn_score: every site of its blocks at once, one layer at a time (all
//    spins are given); a tile's rows are 16 (block, site) pairs.
// Each wave owns 16 output channels of layers 2..4, whose BF16 weights it
// keeps in registers for the whole pass.
// ---------------------------------------------------------------------------
constexpr int SEQ_PER_WG = 16;
constexpr int RING_ROW = C + 8;  // padded row (bf16 elements) against LDS bank conflicts

struct ArWeights {
    bf16x8 w[3][10];  // layers 2..4: this lane's B-operand slices (output channel cw)
    float bias[3], wo_c, bo;
    float l1w[3];     // layer 1: this lane's B operands (channel cw, input k = lane >> 4 of each group)
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
    const int k = lane >> 4;
    p.l1w[0] = P[OFF_W1 + k * C + cw];
    p.l1w[1] = P[OFF_U1 + k * C + cw];
    p.l1w[2] = k == 0 ? P[OFF_V1 + cw] : (k == 1 ? P[OFF_B1 + cw] : 0.f);
}

// Layer 1 of a tile of 16 rows on the matrix cores (FP32 operands,
// v_mfma_f32_16x16x4_f32, three K groups of 4): a row's inputs are its four
// spin taps (0 outside the block), its four boundary features (the boundary
// spin beside the site on that edge: top, bottom, left, right; else 0), then
// K and 1; the B operands are W1, U1 and (v1, b1) of this wave's 16 channels.
// Lane (row lane & 15, input k = lane >> 4) passes its three inputs; the
// result holds pre1 of rows 4 (lane >> 4) + r, channel cw.
__device__ __forceinline__ floatx4 layer1_tile(float in_tap, float in_bnd, float in_k, const ArWeights &p)
{
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(in_tap, p.l1w[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(in_bnd, p.l1w[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(in_k, p.l1w[2], acc, 0, 0, 0);
    return acc;
}

// The three layer-1 inputs number k (0..3) of site (i, j) of a block: x holds
// the block's known sites (the one at position ov_pos, if any, is ov_val
// instead), bnd its boundary (top row, bottom row, left column, right column).
template <int BS>
__device__ __forceinline__ void layer1_inputs(const int8_t *x, int ov_pos, float ov_val, const int8_t *bnd,
                                              float kc, int i, int j, int k, float *in_tap, float *in_bnd,
                                              float *in_k)
{
    const int ii = i + tap_di(k), jj = j + tap_dj(k);
    float v = 0.f;
    if (ii >= 0 && jj >= 0 && jj < BS) {
        const int pos = ii * BS + jj;
        v = pos == ov_pos ? ov_val : (float)x[pos];
    }
    *in_tap = v;
    float b = 0.f;
    if (k == 0 && i == 0)
        b = (float)bnd[j];
    else if (k == 1 && i == BS - 1)
        b = (float)bnd[BS + j];
    else if (k == 2 && j == 0)
        b = (float)bnd[2 * BS + i];
    else if (k == 3 && j == BS - 1)
        b = (float)bnd[3 * BS + i];
    *in_bnd = b;
    *in_k = k == 0 ? kc : (k == 1 ? 1.f : 0.f);
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

// v + the value of the lane selected by a DPP control (in-register cross-lane
// read; out-of-row sources read 0)
template <int CTRL>
__device__ __forceinline__ float add_dpp(float v)
{
    return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}

// Sum of the logit head over this wave's 16 channels for the 4 rows this
// lane holds: within each row of 16 lanes, pairs, then quads (quad
// permutations), then lane + 4 and lane + 8 (row shifts), so lane 0 of the
// row holds ((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7)) + (the same
// for lanes 8..15), a fixed order; it writes out[row].
__device__ __forceinline__ void head_rows(const floatx4 &acc, const ArWeights &p, int lane, float *out)
{
    // the product is rounded before the sums in every kernel that inlines
    // this (no contraction into fused multiply-adds)
#pragma clang fp contract(off)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float v = net_tanh(acc[r] + p.bias[2]) * p.wo_c;
        v = add_dpp<0xb1>(v);   // quad_perm [1, 0, 3, 2]: lane ^ 1
        v = add_dpp<0x4e>(v);   // quad_perm [2, 3, 0, 1]: lane ^ 2
        v = add_dpp<0x104>(v);  // row_shl 4: lane + 4
        v = add_dpp<0x108>(v);  // row_shl 8: lane + 8
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

    // every lane draws for the sequence of its tile row; the threshold of the
    // site drawn in one step is recorded (over its uniform) in the next step,
    // after every wave has read that uniform
    const int srow = lane & 15, kin = lane >> 4;
    uint32_t thr_prev = 0u;
    for (int k = 0; k <= BB; ++k) {
        const int i = k / BS, j = k - i * BS, slot = k % RING;
        // draw site k - 1 (every wave, every lane of a row the same decision;
        // wave 0 records it), then layer 1 of site k for the wave's channels
        float xprev = 0.f;
        if (k > 0) {
            const uint32_t thr = site_threshold(
                head_logit(head_part[0], head_part[1], head_part[2], head_part[3], srow, p.bo));
            const int8_t xv = ut[srow][k - 1] < thr ? (int8_t)1 : (int8_t)-1;
            xprev = (float)xv;
            if (wave == 0 && kin == 0) {
                xs[srow][k - 1] = xv;
                if (k > 1)
                    ut[srow][k - 2] = thr_prev;
            }
            thr_prev = thr;
        }
        if (k < BB) {
            float in_tap, in_bnd, in_k;
            layer1_inputs<BS>(&xs[srow][0], k - 1, xprev, &bs[srow][0], ks[srow], i, j, kin, &in_tap, &in_bnd,
                              &in_k);
            const floatx4 pre = layer1_tile(in_tap, in_bnd, in_k, p);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                ring[0][slot][4 * kin + r][cw] = f2bf(net_tanh(pre[r]));
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
    if (wave == 0 && kin == 0)
        ut[srow][BB - 1] = thr_prev;
    __syncthreads();
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

// Scoring has no site-to-site dependency (every spin is given), so a
// workgroup holds all SCORE_POS positions of its blocks in LDS and runs the
// network one layer at a time: layer 1 for every position on the VALU, then
// for layers 2..4 wave w (output channels 16w .. 16w+15, weights in
// registers) walks the position tiles of 16 rows, four independent MFMA
// chains at a time.  A row of a tile is one (block, site) pair; its A row is
// the previous layer at the site's five taps (zero outside the block), its B
// operands and K order are the sampler's, and a matrix-core product row
// depends only on its own A row, so every site gets the sampler's logit and
// threshold bit for bit.
constexpr int SCORE_POS = 256;  // positions per workgroup (a multiple of 64)
constexpr int SCORE_TILES = 4;  // MFMA chains a wave runs together

template <int BS>
__global__ __launch_bounds__(256) void k_nn_score(NetDev net, SeqDev seq, int n_seq)
{
    constexpr int BB = BS * BS;
    constexpr int G = SCORE_POS / BB < 16 ? SCORE_POS / BB : 16;  // blocks per workgroup
    constexpr int P = G * BB;                                      // positions (a multiple of 64)
    constexpr int MT = P / 16;                                     // tiles of 16 positions
    static_assert(P % 64 == 0 && MT % SCORE_TILES == 0, "whole tile groups");
    // activations of the layer being read and the layer being written (ping-pong);
    // after layer 4 the first holds the head partials, the thresholds and the log-q parts
    __shared__ __attribute__((aligned(16))) uint16_t hbuf[2][P][RING_ROW];
    __shared__ int8_t xs[G][64];
    __shared__ int8_t bs[G][32];
    __shared__ float ks[G];
    float(*head_part)[P] = reinterpret_cast<float(*)[P]>(&hbuf[1][0][0]);              // [4][P]
    uint32_t(*thr_s)[64] = reinterpret_cast<uint32_t(*)[64]>(&hbuf[0][0][0]);         // [G][64]
    double(*lq_part)[16] = reinterpret_cast<double(*)[16]>(&hbuf[0][0][0] + G * 64 * 2);  // [G][16]

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int s0 = blockIdx.x * G;

    for (int i = tid; i < G * 64; i += 256) {
        const int s = i >> 6, k = i & 63;
        xs[s][k] = (s0 + s < n_seq && k < BB) ? seq.x[(size_t)(s0 + s) * BB + k] : (int8_t)0;
    }
    for (int i = tid; i < G * 32; i += 256) {
        const int s = i >> 5, k = i & 31;
        bs[s][k] = (s0 + s < n_seq && k < 4 * BS) ? seq.bnd[(size_t)(s0 + s) * 4 * BS + k] : (int8_t)0;
    }
    if (tid < G)
        ks[tid] = s0 + tid < n_seq ? seq.coupling[s0 + tid] : 0.f;
    ArWeights p;
    load_ar_weights(net, wave, lane, p);
    const int cw = 16 * wave + (lane & 15);
    __syncthreads();

    // layer 1: this wave's 16 channels for every tile of 16 positions
    for (int m = 0; m < MT; ++m) {
        const int pos = 16 * m + (lane & 15);  // this lane's row
        const int s = pos / BB, k = pos - s * BB, i = k / BS, j = k - i * BS;
        float in_tap, in_bnd, in_k;
        layer1_inputs<BS>(&xs[s][0], -1, 0.f, &bs[s][0], ks[s], i, j, lane >> 4, &in_tap, &in_bnd, &in_k);
        const floatx4 pre = layer1_tile(in_tap, in_bnd, in_k, p);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            hbuf[0][16 * m + 4 * (lane >> 4) + r][cw] = f2bf(net_tanh(pre[r]));
    }
    __syncthreads();

    // layers 2..4: this wave's 16 output channels for every position
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const uint16_t(*hin)[RING_ROW] = hbuf[l & 1];
        uint16_t(*hout)[RING_ROW] = hbuf[(l + 1) & 1];
        for (int m0 = 0; m0 < MT; m0 += SCORE_TILES) {
            floatx4 acc[SCORE_TILES];
            int src[SCORE_TILES], si[SCORE_TILES], sj[SCORE_TILES];
#pragma unroll
            for (int u = 0; u < SCORE_TILES; ++u) {
                acc[u] = floatx4{0.f, 0.f, 0.f, 0.f};
                const int pos = 16 * (m0 + u) + (lane & 15);  // this lane's A row
                const int s = pos / BB, k = pos - s * BB;
                si[u] = k / BS;
                sj[u] = k - si[u] * BS;
                src[u] = s * BB;
            }
#pragma unroll
            for (int q = 0; q < 10; ++q) {
                const int t = q >> 1, half = q & 1;
#pragma unroll
                for (int u = 0; u < SCORE_TILES; ++u) {
                    const int ii = si[u] + tap_di(t), jj = sj[u] + tap_dj(t);
                    bf16x8 a = zero_bf16x8();
                    if (ii >= 0 && jj >= 0 && jj < BS)
                        a = load_bf16x8(&hin[src[u] + ii * BS + jj][half * 32 + 8 * (lane >> 4)]);
                    acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, p.w[l][q], acc[u], 0, 0, 0);
                }
            }
#pragma unroll
            for (int u = 0; u < SCORE_TILES; ++u) {
                const int row0 = 16 * (m0 + u) + 4 * (lane >> 4);
                if (l < 2) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        hout[row0 + r][cw] = f2bf(net_tanh(acc[u][r] + p.bias[l]));
                } else {
                    // hout is the other buffer, free now: head partials of this wave
                    head_rows(acc[u], p, lane, &head_part[wave][16 * (m0 + u)]);
                }
            }
        }
        __syncthreads();
    }

    // thresholds (position pos = s * BB + k) and log q, in the sampler's order
    for (int pos = tid; pos < P; pos += 256) {
        const int s = pos / BB, k = pos - s * BB;
        thr_s[s][k] = site_threshold(head_logit(head_part[0], head_part[1], head_part[2], head_part[3], pos, p.bo));
    }
    __syncthreads();
    for (int idx = tid; idx < G * 16; idx += 256)
        logq_parts(xs, thr_s, BB, idx, lq_part);
    __syncthreads();
    if (tid < G && s0 + tid < n_seq)
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
                                                    const uint32_t *__restrict__ steps_taken, uint32_t seed_lo,
                                                    uint32_t seed_hi, int8_t *__restrict__ tx,
                                                    int8_t *__restrict__ tb, float *__restrict__ tk)
{
    const uint32_t i = blockIdx.x, step = *steps_taken;
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

// one training step taken (after its Adam update)
__global__ void k_step_advance(uint32_t *steps_taken)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *steps_taken += 1u;
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
                       net.wtd);
    return hipGetLastError();
}

hipError_t forward(const NetDev &net, const TrainWs &ws, const int8_t *x, const int8_t *bnd, const float *kc,
                   int nblk, int Bs, hipStream_t st)
{
    const int Pv = nblk * Bs * Bs, Pp = (Pv + 63) / 64 * 64;
    hipLaunchKernelGGL(k_layer1, dim3(blocks_for((long)Pp * C, 256)), dim3(256), 0, st, net.params, x, bnd, kc,
                       nblk, Bs, Pp, ws.h[0], ws.hb[0]);
    for (int l = 2; l <= 4; ++l) {
        const int li = l - 2;
        hipLaunchKernelGGL(k_conv<false>, dim3(Pp / 64), dim3(256), 0, st, ws.hb[li], net.wt + (size_t)li * C * KB,
                           net.params + off_b(l), (const float *)nullptr, Pv, Bs, ws.h[l - 1],
                           l < 4 ? ws.hb[l - 1] : (uint16_t *)nullptr);
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
    const int splits = (Pv + WGRAD_CHUNK - 1) / WGRAD_CHUNK;
    // head: dwo = sum_p h4[p] dlogit[p]; dbo = sum_p dlogit[p]
    hipLaunchKernelGGL(k_colsum, dim3(nbr), dim3(256), 0, st, ws.h[3], ws.dlogit, Pp, rows_per_blk, ws.partial);
    hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(C), 0, st, ws.partial, nbr, C, net.grad + OFF_WO);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, ws.dlogit, Pp, 1.f, net.grad + OFF_BO);
    hipLaunchKernelGGL(k_dpre_head, dim3(blocks_for((long)Pp * C, 256)), dim3(256), 0, st, ws.h[3], ws.dlogit,
                       net.params, Pp, ws.dpre[0], ws.dpreb[0]);
    for (int l = 4; l >= 2; --l) {
        const int li = l - 2, cur = l & 1, nxt = cur ^ 1;  // layer 4 reads buffer 0
        hipLaunchKernelGGL(k_colsum, dim3(nbr), dim3(256), 0, st, ws.dpre[cur], (const float *)nullptr, Pp,
                           rows_per_blk, ws.partial);
        hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(C), 0, st, ws.partial, nbr, C, net.grad + off_b(l));
        // weight gradient against this layer's input (BF16 activations of layer l - 1)
        hipLaunchKernelGGL(k_wgrad, dim3(5, splits), dim3(256), 0, st, ws.dpreb[cur], ws.hb[li], Pv, Bs, ws.wpart);
        hipLaunchKernelGGL(k_wgrad_sum, dim3(blocks_for((long)C * KB, 256)), dim3(256), 0, st, ws.wpart, splits, l,
                           net.grad);
        // gradient of layer l - 1's pre-activation
        hipLaunchKernelGGL(k_conv<true>, dim3(Pp / 64), dim3(256), 0, st, ws.dpreb[cur],
                           net.wtd + (size_t)li * C * KB, (const float *)nullptr, ws.h[l - 2], Pv, Bs, ws.dpre[nxt],
                           ws.dpreb[nxt]);
    }
    // layer 2 wrote dpre1 into buffer 1
    hipLaunchKernelGGL(k_layer1_grad, dim3(nbr), dim3(256), 0, st, ws.dpre[1], x, bnd, kc, nblk, Bs, rows_per_blk,
                       ws.partial);
    // rows: W1 taps (4), U1 (4), v1, b1 -> contiguous in the flat vector starting at OFF_W1
    hipLaunchKernelGGL(k_reduce_cols, dim3(blocks_for(10 * C, 256)), dim3(256), 0, st, ws.partial, nbr, 10 * C,
                       net.grad + OFF_W1);
    return hipGetLastError();
}

hipError_t adam(const NetDev &net, float lr, hipStream_t st)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(N_PARAMS, 256)), dim3(256), 0, st, net.params, net.grad, net.adam_m,
                       net.adam_v, N_PARAMS, lr, b1, b2, eps, (const uint32_t *)net.step);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, st, net.step);
    return hipGetLastError();
}

template <int BS>
static hipError_t ar_pass_bs(const NetDev &net, const SeqDev &seq, int n_score, int n_sample, hipStream_t st)
{
    if (n_score > 0) {
        constexpr int G = SCORE_POS / (BS * BS) < 16 ? SCORE_POS / (BS * BS) : 16;
        hipLaunchKernelGGL(k_nn_score<BS>, dim3(blocks_for(n_score, G)), dim3(256), 0, st, net, seq, n_score);
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

hipError_t gather_rows(const NetDev &net, const TrainWs &ws, const int8_t *x, const int8_t *bnd, const float *kc,
                       uint32_t n_rows, int batch, int Bs, uint64_t seed, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_rows, dim3(batch), dim3(64), 0, st, x, bnd, kc, n_rows, Bs * Bs, 4 * Bs,
                       (const uint32_t *)net.step,
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
