// HIP kernels of the block-proposal network (definitions in nn.hpp):
//  - training, three kernels a step: the forward and backward of each
//    64-position tile (masked convolutions and their data gradients as
//    implicit GEMMs on the BF16 matrix cores, FP32 accumulation), the weight
//    gradients of all layers, and the reduction with Adam;
//  - the incremental autoregressive passes that score a given block or
//    sample a new one site by site with exactly the same arithmetic,
//    accumulating log q in FP64 from uint32 thresholds; in a block round the
//    scorer reads the current blocks from the packed lattice and the sampler
//    ends with the Metropolis-Hastings decision and write-back;
//  - training-block extraction from the packed lattices.
#include <math.h>

#include "device.hpp"
#include "nn.hpp"
#include "nn_launch.hpp"

namespace ising {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// float -> bfloat16 bits, round to nearest even (inputs are finite): one
// v_cvt_pk_bf16_f32 on gfx950
__device__ __forceinline__ uint16_t f2bf(float f)
{
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

// two floats -> two bfloat16 (round to nearest even) in one v_cvt_pk_bf16_f32:
// a in the low half, b in the high half
__device__ __forceinline__ uint32_t f2bf2(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){a, b}, bf16x2));
}

// v[0..3] in BF16 to p[0], p[RS], p[2 RS], p[3 RS] (one column of four rows of
// a row-major array): two conversions, the high halves stored straight from
// the upper 16 bits
template <int RS>
__device__ __forceinline__ void store_col4(uint16_t *p, float v0, float v1, float v2, float v3)
{
    const uint32_t lo = f2bf2(v0, v1), hi = f2bf2(v2, v3);
    p[0] = (uint16_t)lo;
    p[RS] = (uint16_t)(lo >> 16);
    p[2 * RS] = (uint16_t)hi;
    p[3 * RS] = (uint16_t)(hi >> 16);
}

// tanh(x + b) from the hardware exp2 and reciprocal: tanh y = 1 - 2 / (1 + e^{2y}),
// with 2 log2(e) (x + b) formed by one fused multiply-add from sb = tanh_bias(b)
// (sb = 0: tanh x).  exp2 overflows to +inf (reciprocal 0) or underflows to 0
// far from the origin, so the ends are exactly +1 and -1; near 0 the error is
// absolute, about one ulp of 1.  Three vector operations and two
// transcendentals: the activations of every layer go through it, and it is
// the largest share of the vector-unit work of the network kernels.  Every
// kernel of the network uses this one definition, so training, scoring and
// sampling evaluate the same function.
constexpr float TANH_K = 2.8853900817779268f;  // 2 log2(e)
__device__ __forceinline__ float tanh_bias(float b) { return TANH_K * b; }
__device__ __forceinline__ float net_tanh(float x, float sb = 0.f)
{
    const float e = __builtin_amdgcn_exp2f(fmaf(x, TANH_K, sb));  // e^{2(x + b)}
    return fmaf(-2.f, __builtin_amdgcn_rcpf(1.f + e), 1.f);
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
// Training step, fused per tile of 64 positions.  Blocks of 2x2, 4x4 and 8x8
// sites hold 4, 16 and 64 positions, so a tile holds whole blocks and every
// tap of the masked convolutions stays inside it: one workgroup runs the
// whole forward and backward of its tile.  The BF16 activations (or
// pre-activation gradients) a product reads sit in LDS; every FP32 activation
// stays in the registers of the lane that produced it, because the data
// gradient puts a layer's pre-activation gradient at the same (position,
// channel) places of the result tiles as the forward put the activation, so
// each tanh derivative is where it is needed.
//  layers 2..4 and their data gradients are implicit GEMMs on the matrix
//  cores (BF16 operands, FP32 accumulation), K = 5 taps x 64 channels in the
//  order t*C + c; a row's A operand is the row at the tap offset inside its
//  block, or an all-zero LDS row where the tap leaves the block (so operand
//  reads never branch):
//    forward, rows p, columns c:        pre[p][c] = sum_t sum_c' h[p + off(t)][c'] W_t[c'][c]
//    data gradient, rows q, columns c': dh[q][c'] = sum_t sum_c d[q - off(t)][c] W_t[c'][c]
//  each wave a 32 x 32 quarter of the 64 x 64 result (2 x 2 MFMA 16x16x32
//  tiles); half of the next product's B operands load while the current one
//  finishes.
// A tile writes the BF16 operands of the weight gradient (inputs and
// pre-activation gradients of layers 2..4), its logits, and one row of
// partial sums: layer-1, bias and head gradients and the loss (nn.hpp).
// ---------------------------------------------------------------------------
constexpr int ACT_ROW = C + 8;  // padded LDS row (bf16 elements; rows stay 16-byte aligned)

// v + the value of the lane selected by a DPP control (in-register cross-lane
// read; out-of-row sources read 0)
template <int CTRL>
__device__ __forceinline__ float add_dpp(float v)
{
    return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}

// this lane's B operands of a product, K slices Q0..Q1-1: output column
// n0 + 16 b + r, K indices q*32 + kq .. q*32 + kq + 7
template <int Q0, int Q1>
__device__ __forceinline__ void load_b(const uint16_t *__restrict__ Bt, int n0, int r, int kq, bf16x8 (&bv)[10][2])
{
#pragma unroll
    for (int q = Q0; q < Q1; ++q)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            bv[q][b] = load_bf16x8(Bt + (size_t)(n0 + b * 16 + r) * KB + q * 32 + kq);
}

// rows arow[a] (this lane's A rows, at (ai, aj) of their block) times the
// columns n0.. of this wave: forward taps (BWD = false) or mirrored taps
// (true); row TILE of src is zero.  The caller loaded K slices 0..4 of the B
// operands in advance; slices 5..9 load here, under the first products.
template <bool BWD>
__device__ __forceinline__ void tile_conv(const uint16_t (*src)[ACT_ROW], const uint16_t *__restrict__ Bt,
                                          bf16x8 (&bv)[10][2], const int (&arow)[2], const int (&ai)[2],
                                          const int (&aj)[2], const bool (&alive)[2], int Bs, int n0, int r,
                                          int kq, floatx4 (&acc)[2][2])
{
    load_b<5, 10>(Bt, n0, r, kq, bv);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        const int t = q >> 1, half = q & 1;
        const int di = BWD ? -tap_di(t) : tap_di(t), dj = BWD ? -tap_dj(t) : tap_dj(t);
        bf16x8 av[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int ii = ai[a] + di, jj = aj[a] + dj;
            const bool ok = alive[a] & (ii >= 0) & (ii < Bs) & (jj >= 0) & (jj < Bs);
            av[a] = load_bf16x8(&src[ok ? arow[a] + di * Bs + dj : TILE][half * 32 + kq]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[q][b], acc[a][b], 0, 0, 0);
    }
}

// the tile's 64 LDS rows to a [64][C] BF16 array in global memory (32 bytes a thread)
__device__ __forceinline__ void store_tile(const uint16_t (*src)[ACT_ROW], uint16_t *__restrict__ dst, int tid)
{
    const int row = tid >> 2, col = (tid & 3) * 16;
    const uint4 *s = reinterpret_cast<const uint4 *>(&src[row][col]);
    uint4 *d = reinterpret_cast<uint4 *>(dst + (size_t)row * C + col);
    d[0] = s[0];
    d[1] = s[1];
}

// Where a tile's blocks come from: block i of the batch is row i of (x, bnd,
// kc), or, with a step counter, row floor(u * n_rows / 2^32) with u the first
// word of Philox(ctr = (i, step, 0, 6), key = seed): a minibatch drawn on the
// device.
struct BatchSrc {
    const int8_t *x, *bnd;
    const float *kc;
    const uint32_t *step;  // null: rows in order
    uint32_t n_rows, seed_lo, seed_hi;
};

// per-lane column sums of one partial-sum row q, written for the fixed-order
// sum over the eight row groups at the end of the tile
__device__ __forceinline__ void put_cols(float (*colpart)[14][C], int grp, int q, const int (&cb)[2], float t0,
                                         float t1)
{
    colpart[grp][q][cb[0]] = t0;
    colpart[grp][q][cb[1]] = t1;
}

template <int BS>
__global__ __launch_bounds__(256, 2) void k_train_tile(NetDev net, TrainWs ws, BatchSrc src, int nblk)
{
    constexpr int Bs = BS;
    constexpr int BND_ZERO = 128;  // index of the zero entry of bs
    __shared__ __attribute__((aligned(16))) uint16_t act[2][TILE + 1][ACT_ROW];  // row TILE: zeros
    __shared__ float colpart[8][14][C];  // [row group][partial-sum row q][channel]
    __shared__ float h1s[TILE][C];        // FP32 layer-1 activations (needed last)
    __shared__ float rowred[2][TILE];
    __shared__ float dls[TILE];
    __shared__ float lrow[TILE];
    __shared__ float ks[16];
    __shared__ uint32_t rows[16];
    __shared__ int8_t xs[TILE + 1];      // entry TILE: 0
    __shared__ int8_t bs[BND_ZERO + 1];  // entry BND_ZERO: 0
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = (wave >> 1) * 32, n0 = (wave & 1) * 32;
    const int r = lane & 15, g4 = lane >> 4, kq = g4 * 8, grp = (wave >> 1) * 4 + g4;
    const int BB = Bs * Bs, NB = 4 * Bs, Pvalid = nblk * BB;
    const int p0 = blockIdx.x * TILE, nb0 = p0 / BB;
    const int nbl = min(TILE / BB, nblk - nb0);
    const float *P = net.params;

    bf16x8 bv[10][2];
    load_b<0, 5>(net.wt, n0, r, kq, bv);  // layer 2's first half, in flight during the set-up and layer 1

    if (tid < nbl) {
        uint32_t row = (uint32_t)(nb0 + tid);
        if (src.step) {
            uint32_t o[4];
            philox4x32_10(row, *src.step, 0u, 6u, src.seed_lo, src.seed_hi, o);
            row = (uint32_t)(((uint64_t)o[0] * src.n_rows) >> 32);
        }
        rows[tid] = row;
        ks[tid] = src.kc[row];
    }
    if (tid < 18) {  // the two zero rows, 9 x 16 bytes each
        uint4 *z = reinterpret_cast<uint4 *>(&act[tid / 9][TILE][0]);
        z[tid % 9] = make_uint4(0u, 0u, 0u, 0u);
    }
    if (tid == 0) {
        xs[TILE] = 0;
        bs[BND_ZERO] = 0;
    }
    __syncthreads();
    if (tid < TILE) {
        const int nl = tid / BB;
        xs[tid] = p0 + tid < Pvalid ? src.x[(size_t)rows[nl] * BB + tid - nl * BB] : (int8_t)0;
    }
    for (int e = tid; e < nbl * NB; e += 256) {
        const int nl = e / NB;
        bs[e] = src.bnd[(size_t)rows[nl] * NB + e - nl * NB];
    }
    int arow[2], ai[2], aj[2];
    bool alive[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        arow[a] = m0 + a * 16 + r;
        alive[a] = p0 + arow[a] < Pvalid;
        const int k = arow[a] % BB;
        ai[a] = k / Bs;
        aj[a] = k - ai[a] * Bs;
    }
    const int cb[2] = {n0 + r, n0 + 16 + r};
    __syncthreads();

    // result place (a, b, i): row m0 + 16 a + 4 g4 + i, column cb[b]; the FP32
    // activations of layers 2..4 stay in registers, layer 1's in LDS
    float h[4][2][2][4];
    // layer 1 (FP32 on the vector units): taps, boundary features, K and bias
    {
        float w1[4][2], u1[4][2], v1[2], b1[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                w1[t][b] = P[OFF_W1 + t * C + cb[b]];
                u1[t][b] = P[OFF_U1 + t * C + cb[b]];
            }
            v1[b] = P[OFF_V1 + cb[b]];
            b1[b] = P[OFF_B1 + cb[b]];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = m0 + a * 16 + 4 * g4 + i;
                const int nl = p / BB, k = p - nl * BB, pi = k / Bs, pj = k - pi * Bs;
                float xt[4], bf[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int ii = pi + tap_di(t), jj = pj + tap_dj(t);
                    xt[t] = (float)xs[(ii >= 0 && jj >= 0 && jj < Bs) ? nl * BB + ii * Bs + jj : TILE];
                }
                const int nbase = nl * NB;
                bf[0] = (float)bs[pi == 0 ? nbase + pj : BND_ZERO];
                bf[1] = (float)bs[pi == Bs - 1 ? nbase + Bs + pj : BND_ZERO];
                bf[2] = (float)bs[pj == 0 ? nbase + 2 * Bs + pi : BND_ZERO];
                bf[3] = (float)bs[pj == Bs - 1 ? nbase + 3 * Bs + pi : BND_ZERO];
                const bool valid = p0 + p < Pvalid;
                const float kv = ks[nl];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    float pre = kv * v1[b] + b1[b];
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        pre += xt[t] * w1[t][b];
                    float f = 0.f;
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        f += bf[t] * u1[t][b];
                    pre += f;
                    const float v = valid ? net_tanh(pre) : 0.f;
                    h1s[p][cb[b]] = v;
                    act[0][p][cb[b]] = f2bf(v);
                }
            }
    }
    __syncthreads();
    store_tile(act[0], ws.hb[0] + (size_t)p0 * C, tid);

    // layers 2..4: act[(l - 2) & 1] holds the BF16 input
#pragma unroll
    for (int l = 2; l <= 4; ++l) {
        const int cur = (l - 2) & 1;
        floatx4 acc[2][2];
        tile_conv<false>(act[cur], net.wt + (size_t)(l - 2) * C * KB, bv, arow, ai, aj, alive, Bs, n0, r, kq, acc);
        // the next product's first B slices: layer l + 1, or the first data gradient (layer 4's)
        load_b<0, 5>(l < 4 ? net.wt + (size_t)(l - 1) * C * KB : net.wtd + (size_t)2 * C * KB, n0, r, kq, bv);
        const float sbias[2] = {tanh_bias(P[off_b(l) + cb[0]]), tanh_bias(P[off_b(l) + cb[1]])};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int p = m0 + a * 16 + 4 * g4 + i;
                    // rows past the batch read only zero rows: a finite tanh(bias), masked
                    h[l - 1][a][b][i] = net_tanh(acc[a][b][i], sbias[b]) * (p0 + p < Pvalid ? 1.f : 0.f);
                }
                if (l < 4)
                    store_col4<ACT_ROW>(&act[cur ^ 1][m0 + a * 16 + 4 * g4][cb[b]], h[l - 1][a][b][0],
                                        h[l - 1][a][b][1], h[l - 1][a][b][2], h[l - 1][a][b][3]);
            }
        if (l < 4) {
            __syncthreads();
            store_tile(act[cur ^ 1], ws.hb[l - 1] + (size_t)p0 * C, tid);
        }
    }

    // head: logit[p] = bo + sum_c h4[p][c] wo[c] (a fixed DPP tree over the 16
    // lanes of a row, then the two column halves), the loss softplus(-x logit)
    // and dlogit = -x sigmoid(-x logit) / P
    const float wo[2] = {P[OFF_WO + cb[0]], P[OFF_WO + cb[1]]};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float s = h[3][a][0][i] * wo[0] + h[3][a][1][i] * wo[1];
            s = add_dpp<0xb1>(s);   // lane ^ 1
            s = add_dpp<0x4e>(s);   // lane ^ 2
            s = add_dpp<0x104>(s);  // lane + 4
            s = add_dpp<0x108>(s);  // lane + 8
            if (r == 0)
                rowred[wave & 1][m0 + a * 16 + 4 * g4 + i] = s;
        }
    __syncthreads();
    if (tid < TILE) {
        float l = 0.f, d = 0.f;
        if (p0 + tid < Pvalid) {
            const float logit = (P[OFF_BO] + rowred[0][tid]) + rowred[1][tid];
            ws.logits[p0 + tid] = logit;
            const float xv = (float)xs[tid];
            const float z = -xv * logit;
            l = z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z));
            d = -xv / (1.f + expf(-z)) / (float)Pvalid;
        }
        dls[tid] = d;
        lrow[tid] = l;
    }
    __syncthreads();

    // head backward: dpre4 = dlogit wo (1 - h4^2); wo and b4 gradient partials
    float d[2][2][4];
    {
        float swo[2] = {0.f, 0.f}, sb4[2] = {0.f, 0.f};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = m0 + a * 16 + 4 * g4 + i;
                const float dl = dls[p];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const float hv = h[3][a][b][i];
                    const float dv = dl * wo[b] * (1.f - hv * hv);
                    d[a][b][i] = dv;
                    act[1][p][cb[b]] = f2bf(dv);
                    swo[b] += hv * dl;
                    sb4[b] += dv;
                }
            }
        put_cols(colpart, grp, 13, cb, swo[0], swo[1]);
        put_cols(colpart, grp, 12, cb, sb4[0], sb4[1]);
    }
    __syncthreads();
    store_tile(act[1], ws.db[2] + (size_t)p0 * C, tid);

    // data gradients: layer l's BF16 pre-activation gradient in act[(l + 1) & 1]
    // -> layer l-1's, times its tanh derivative
#pragma unroll
    for (int l = 4; l >= 2; --l) {
        const int srcb = (l + 1) & 1;
        floatx4 acc[2][2];
        tile_conv<true>(act[srcb], net.wtd + (size_t)(l - 2) * C * KB, bv, arow, ai, aj, alive, Bs, n0, r, kq,
                        acc);
        if (l > 2)
            load_b<0, 5>(net.wtd + (size_t)(l - 3) * C * KB, n0, r, kq, bv);
        float sb[2] = {0.f, 0.f};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float hv = l > 2 ? h[l - 2][a][b][i] : h1s[m0 + a * 16 + 4 * g4 + i][cb[b]];
                    const float v = acc[a][b][i] * (1.f - hv * hv);
                    d[a][b][i] = v;
                    if (l > 2) {
                        act[srcb ^ 1][m0 + a * 16 + 4 * g4 + i][cb[b]] = f2bf(v);
                        sb[b] += v;
                    }
                }
        if (l > 2) {
            put_cols(colpart, grp, 10 + (l - 3), cb, sb[0], sb[1]);
            __syncthreads();
            store_tile(act[srcb ^ 1], ws.db[l - 3] + (size_t)p0 * C, tid);
        }
    }

    // layer-1 gradients from dpre1: taps (W1), boundary features (U1), K (v1), 1 (b1)
    {
        float g1[10][2];
#pragma unroll
        for (int q = 0; q < 10; ++q)
            g1[q][0] = g1[q][1] = 0.f;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = m0 + a * 16 + 4 * g4 + i;
                const int nl = p / BB, k = p - nl * BB, pi = k / Bs, pj = k - pi * Bs;
                const int nbase = nl * NB;
                float in[10];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int ii = pi + tap_di(t), jj = pj + tap_dj(t);
                    in[t] = (float)xs[(ii >= 0 && jj >= 0 && jj < Bs) ? nl * BB + ii * Bs + jj : TILE];
                }
                in[4] = (float)bs[pi == 0 ? nbase + pj : BND_ZERO];
                in[5] = (float)bs[pi == Bs - 1 ? nbase + Bs + pj : BND_ZERO];
                in[6] = (float)bs[pj == 0 ? nbase + 2 * Bs + pi : BND_ZERO];
                in[7] = (float)bs[pj == Bs - 1 ? nbase + 3 * Bs + pi : BND_ZERO];
                in[8] = ks[nl];
                in[9] = 1.f;
                const bool valid = p0 + p < Pvalid;  // d is 0 past the batch; ks there is unset
#pragma unroll
                for (int q = 0; q < 10; ++q)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        g1[q][b] += valid ? in[q] * d[a][b][i] : 0.f;
            }
#pragma unroll
        for (int q = 0; q < 10; ++q)
            put_cols(colpart, grp, q, cb, g1[q][0], g1[q][1]);
    }
    __syncthreads();
    float *part = ws.partial + (size_t)blockIdx.x * PART_ROW;
    for (int e = tid; e < 14 * C; e += 256) {
        const int q = e / C, c = e - q * C;
        float s = 0.f;
#pragma unroll
        for (int g = 0; g < 8; ++g)
            s += colpart[g][q][c];
        part[e] = s;
    }
    if (tid >= 254) {  // the loss and the head-bias gradient over the tile's rows
        const float *v = tid == 254 ? lrow : dls;
        float s = 0.f;
        for (int p = 0; p < TILE; ++p)
            s += v[p];
        part[tid == 254 ? PART_LOSS : PART_BO] = s;
    }
}

// ---------------------------------------------------------------------------
// Weight gradients of layers 2..4, split over positions (the K of the product):
//   wpart[z][s][t*C + c'][c] = sum over the positions p of split s of
//                              in_z[p + off(t)][c'] d_z[p][c]
// (in_z: BF16 input of layer z + 2, d_z: its BF16 pre-activation gradient; 0
// where the tap leaves the block), so a split's rows t*C + c' are laid out
// like the parameter vector.  Each step stages 64 positions of both operands
// in LDS transposed, a channel's positions pairwise in 32-bit words whose
// index is XOR-swizzled by the channel's group of 8 (the staging writes of a
// wave then hit 64 distinct banks); a matrix-core operand (8 consecutive
// positions of one channel) stays one 16-byte read.  Grid: 5 taps x splits x
// 3 layers; each wave a 32 x 32 quarter of the 64 x 64 tile.  advance (if not
// null): the training-step counter, counted here because no other workgroup
// of this kernel reads it (the tile kernel before it drew its minibatch with
// the old count, the Adam update after it uses the new one).
// ---------------------------------------------------------------------------
template <int BS>
__global__ __launch_bounds__(256) void k_wgrad(TrainWs ws, int Pvalid, int splits, uint32_t *advance)
{
    constexpr int Bs = BS;
    constexpr int WROW = 36;  // words per staged channel row: 32 used, rows 16-byte aligned
    __shared__ __attribute__((aligned(16))) uint32_t sd[C][WROW];  // pre-activation gradient
    __shared__ __attribute__((aligned(16))) uint32_t si[C][WROW];  // tap-shifted input
    const int t = blockIdx.x, s = blockIdx.y, z = blockIdx.z;
    if (advance && t == 0 && s == 0 && z == 0 && threadIdx.x == 0)
        *advance += 1u;
    const uint16_t *__restrict__ dpre = ws.db[z];
    const uint16_t *__restrict__ in = ws.hb[z];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = (wave >> 1) * 32, n0 = (wave & 1) * 32;
    const int r = lane & 15, g4 = lane >> 4;
    const int pp = tid >> 3, cg = tid & 7;  // staging: position pair, group of 8 channels
    const int BB = Bs * Bs;
    floatx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int p_begin = s * WGRAD_CHUNK, p_end = min(p_begin + WGRAD_CHUNK, Pvalid);
    // channels 8 cg .. 8 cg + 7 of position p of both operands (0 past the split or outside the block)
    auto fetch = [&](int p, uint4 &vd, uint4 &vi) {
        vd = make_uint4(0u, 0u, 0u, 0u);
        vi = vd;
        if (p < p_end) {
            vd = *reinterpret_cast<const uint4 *>(dpre + (size_t)p * C + 8 * cg);
            const int n = p / BB, k = p - n * BB, i = k / Bs, j = k - i * Bs;
            const int ii = i + tap_di(t), jj = j + tap_dj(t);
            if (ii >= 0 && jj >= 0 && jj < Bs)
                vi = *reinterpret_cast<const uint4 *>(in + (size_t)(n * BB + ii * Bs + jj) * C + 8 * cg);
        }
    };
    uint4 d0, d1, i0, i1;
    fetch(p_begin + 2 * pp, d0, i0);
    fetch(p_begin + 2 * pp + 1, d1, i1);
    for (int p0 = p_begin; p0 < p_end; p0 += 64) {
        const uint16_t *ed0 = reinterpret_cast<const uint16_t *>(&d0), *ed1 = reinterpret_cast<const uint16_t *>(&d1);
        const uint16_t *ei0 = reinterpret_cast<const uint16_t *>(&i0), *ei1 = reinterpret_cast<const uint16_t *>(&i1);
        const int w = pp ^ (cg << 2);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            sd[8 * cg + q][w] = (uint32_t)ed0[q] | ((uint32_t)ed1[q] << 16);
            si[8 * cg + q][w] = (uint32_t)ei0[q] | ((uint32_t)ei1[q] << 16);
        }
        __syncthreads();
        fetch(p0 + 64 + 2 * pp, d0, i0);  // the next step's operands load while this one multiplies
        fetch(p0 + 64 + 2 * pp + 1, d1, i1);
#pragma unroll
        for (int kst = 0; kst < 2; ++kst) {
            bf16x8 av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int row = m0 + a * 16 + r;
                av[a] = load_bf16x8(reinterpret_cast<const uint16_t *>(
                    &si[row][(16 * kst + 4 * g4) ^ (((row >> 3) & 7) << 2)]));
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int row = n0 + b * 16 + r;
                bv[b] = load_bf16x8(reinterpret_cast<const uint16_t *>(
                    &sd[row][(16 * kst + 4 * g4) ^ (((row >> 3) & 7) << 2)]));
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    float *__restrict__ part = ws.wpart + ((size_t)z * splits + s) * KB * C;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = t * C + m0 + a * 16 + 4 * g4 + i, c = n0 + b * 16 + r;
                part[(size_t)k * C + c] = acc[a][b][i];
            }
}

// ---------------------------------------------------------------------------
// End of a training step: the gradient from the partial sums (weight entries
// over the position splits in 4 groups, the other entries over the tiles in
// 16 groups, each combined in a fixed order), the loss, and with ADAM the Adam
// update (the step number t is the device counter, already advanced by the
// weight-gradient kernel; the bias corrections 1 - beta^t are formed in FP64 from the
// exact decimal betas) and the BF16 copies of the updated weights.
// Workgroups [0, FIN_W_BLOCKS) take 64 weight entries each, the rest 16
// partial-sum columns each.
// ---------------------------------------------------------------------------
constexpr int FIN_W_BLOCKS = 3 * C * KB / 64;
constexpr int FIN_S_BLOCKS = (PART_USED + 15) / 16;

__device__ __forceinline__ float adam_update(const NetDev &net, int i, float g, float lr, float c1, float c2)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mi = b1 * net.adam_m[i] + (1.f - b1) * g;
    const float vi = b2 * net.adam_v[i] + (1.f - b2) * g * g;
    net.adam_m[i] = mi;
    net.adam_v[i] = vi;
    const float w = net.params[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    net.params[i] = w;
    return w;
}

// parameter index of partial-sum column j (j != PART_LOSS)
__device__ __forceinline__ int part_param(int j)
{
    if (j < PART_B2)
        return OFF_W1 + j;
    if (j < PART_B3)
        return off_b(2) + j - PART_B2;
    if (j < PART_B4)
        return off_b(3) + j - PART_B3;
    if (j < PART_WO)
        return off_b(4) + j - PART_B4;
    if (j < PART_BO)
        return OFF_WO + j - PART_WO;
    return OFF_BO;
}

template <bool ADAM>
__global__ __launch_bounds__(256) void k_finish(NetDev net, TrainWs ws, int n_tiles, int splits, int Pvalid, float lr,
                                                float *loss_out)
{
    __shared__ float red[16][64];
    const int tid = threadIdx.x;
    float c1 = 1.f, c2 = 1.f;
    if (ADAM) {
        const double t = (double)*net.step;
        c1 = (float)(1.0 - pow(0.9, t));
        c2 = (float)(1.0 - pow(0.999, t));
    }
    if (blockIdx.x < FIN_W_BLOCKS) {
        const int z = blockIdx.x / (C * KB / 64), el = tid & 63, g = tid >> 6;
        const int e = (blockIdx.x - z * (C * KB / 64)) * 64 + el;  // k * C + c, k = t*C + c'
        const float *wp = ws.wpart + (size_t)z * splits * KB * C + e;
        float v = 0.f;
#pragma unroll 8
        for (int s = g; s < splits; s += 4)
            v += wp[(size_t)s * KB * C];
        red[g][el] = v;
        __syncthreads();
        if (g == 0) {
            const float gr = ((red[0][el] + red[1][el]) + red[2][el]) + red[3][el];
            const int i = off_w(z + 2) + e;
            net.grad[i] = gr;
            if (ADAM) {
                const uint16_t wb = f2bf(adam_update(net, i, gr, lr, c1, c2));
                const int k = e / C, c = e - k * C, t = k / C, ci = k - t * C;
                net.wt[((size_t)z * C + c) * KB + k] = wb;
                net.wtd[((size_t)z * C + ci) * KB + t * C + c] = wb;
            }
        }
    } else {
        const int jl = tid & 15, g = tid >> 4;
        const int j = (blockIdx.x - FIN_W_BLOCKS) * 16 + jl;
        float v = 0.f;
        if (j < PART_USED)
#pragma unroll 8
            for (int b = g; b < n_tiles; b += 16)
                v += ws.partial[(size_t)b * PART_ROW + j];
        red[g][jl] = v;
        __syncthreads();
        if (g == 0 && j < PART_USED) {
            float gr = 0.f;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                gr += red[k][jl];
            if (j == PART_LOSS) {
                const float loss = gr * (1.f / (float)Pvalid);
                ws.loss[0] = loss;
                if (loss_out)
                    *loss_out = loss;
            } else {
                const int i = part_param(j);
                net.grad[i] = gr;
                if (ADAM)
                    (void)adam_update(net, i, gr, lr, c1, c2);
            }
        }
    }
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

// A block round's sequences: number b (< count) is block first + b of the
// round's colour, counted replica by replica (per_rep blocks of that colour
// each).  The scorer reads the current blocks from the packed lattice, the
// sampler draws the proposals and applies the Metropolis-Hastings decision.
struct RoundArgs {
    const RepDev *reps;
    const double *kcoup;           // K = beta*J per replica (FP64)
    unsigned long long *accepts;   // accepted blocks per replica
    uint32_t colour, round, first, count, per_rep;
};

// replica r, block position (bx, by) and blocks per row nbx of round sequence b
template <int BS>
__device__ __forceinline__ void round_block(const RoundArgs &ra, uint32_t b, uint32_t &r, uint32_t &bx, uint32_t &by,
                                            uint32_t &nbx)
{
    const uint32_t g = ra.first + b;
    r = g / ra.per_rep;
    nbx = ra.reps[r].Lx / BS;
    block_coords(g - r * ra.per_rep, nbx, ra.colour, &bx, &by);
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

// the FP32 parameters a lane of the incremental passes uses (output channel cw)
struct ArScalars {
    float sbias[3], wo_c, bo;  // sbias: tanh_bias of the layer 2..4 biases
    float l1w[3];  // layer 1: this lane's B operands (channel cw, input k = lane >> 4 of each group)
};

struct ArWeights : ArScalars {
    bf16x8 w[3][10];  // layers 2..4: this lane's B-operand slices (output channel cw)
};

__device__ __forceinline__ void load_ar_scalars(const NetDev &net, int wave, int lane, ArScalars &p)
{
    const float *P = net.params;
    const int cw = 16 * wave + (lane & 15);
#pragma unroll
    for (int l = 0; l < 3; ++l)
        p.sbias[l] = tanh_bias(P[off_b(l + 2) + cw]);
    p.wo_c = P[OFF_WO + cw];
    p.bo = P[OFF_BO];
    const int k = lane >> 4;
    p.l1w[0] = P[OFF_W1 + k * C + cw];
    p.l1w[1] = P[OFF_U1 + k * C + cw];
    p.l1w[2] = k == 0 ? P[OFF_V1 + cw] : (k == 1 ? P[OFF_B1 + cw] : 0.f);
}

// this lane's B-operand slices of layer l + 2 (output channel cw)
__device__ __forceinline__ void load_ar_layer(const NetDev &net, int l, int wave, int lane, bf16x8 (&w)[10])
{
    const int cw = 16 * wave + (lane & 15);
#pragma unroll
    for (int q = 0; q < 10; ++q)
        w[q] = load_bf16x8(net.wt + ((size_t)l * C + cw) * KB + q * 32 + 8 * (lane >> 4));
}

__device__ __forceinline__ void load_ar_weights(const NetDev &net, int wave, int lane, ArWeights &p)
{
#pragma unroll
    for (int l = 0; l < 3; ++l)
        load_ar_layer(net, l, wave, lane, p.w[l]);
    load_ar_scalars(net, wave, lane, p);
}

// Layer 1 of a tile of 16 rows on the matrix cores (FP32 operands,
// v_mfma_f32_16x16x4_f32, three K groups of 4): a row's inputs are its four
// spin taps (0 outside the block), its four boundary features (the boundary
// spin beside the site on that edge: top, bottom, left, right; else 0), then
// K and 1; the B operands are W1, U1 and (v1, b1) of this wave's 16 channels.
// Lane (row lane & 15, input k = lane >> 4) passes its three inputs; the
// result holds pre1 of rows 4 (lane >> 4) + r, channel cw.
__device__ __forceinline__ floatx4 layer1_tile(float in_tap, float in_bnd, float in_k, const ArScalars &p)
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

// Sum of the logit head over this wave's 16 channels for the 4 rows this
// lane holds: within each row of 16 lanes, pairs, then quads (quad
// permutations), then lane + 4 and lane + 8 (row shifts), so lane 0 of the
// row holds ((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7)) + (the same
// for lanes 8..15), a fixed order; it writes out[row].
__device__ __forceinline__ void head_rows(const floatx4 &acc, const ArScalars &p, int lane, float *out)
{
    // the product is rounded before the sums in every kernel that inlines
    // this (no contraction into fused multiply-adds)
#pragma clang fp contract(off)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float v = net_tanh(acc[r], p.sbias[2]) * p.wo_c;
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
// log of the probability (times 2^32) that a site with threshold thr took spin x
__device__ __forceinline__ double site_log(int8_t x, uint32_t thr)
{
    const double t = (double)thr;
    return log(x > 0 ? t : 4294967296.0 - t);
}

template <int XS, int TS>
__device__ __forceinline__ void logq_parts(const int8_t (*xs)[XS], const uint32_t (*thr)[TS], int BB, int tid,
                                           double (*part)[16])
{
    const int s = tid >> 4, pt = tid & 15;
    double acc = 0.0;
    for (int k = pt * 4; k < pt * 4 + 4 && k < BB; ++k)
        acc += site_log(xs[s][k], thr[s][k]);
    part[s][pt] = acc;
}

__device__ __forceinline__ double logq_total(const double *part, int BB)
{
    double sum = 0.0;
    for (int pt = 0; pt < 16; ++pt)
        sum += part[pt];
    return sum - (double)BB * 32.0 * 0.69314718055994530942;
}

// Layers 2..4 of the sampler at site k, for one class of sites: whether the
// site is in the block's first row (TOP) or first or last column (LEFT,
// RIGHT) fixes at compile time which of the five taps fall outside the block
// (an all-zero A slice), so the ten A slices of a layer are all loaded from
// the ring before its chain of products starts.  Every lane of the
// workgroup is at the same site, so the class is the same for all of them.
template <bool TOP, bool LEFT, bool RIGHT>
__device__ constexpr bool tap_inside(int t)
{
    return t == 0 ? !TOP && !LEFT : t == 1 ? !TOP : t == 2 ? !TOP && !RIGHT : t == 3 ? !LEFT : true;
}

template <int BS, bool TOP, bool LEFT, bool RIGHT>
__device__ __forceinline__ void sample_layers(uint16_t (*ring)[RING][SEQ_PER_WG][RING_ROW], const ArWeights &p, int k,
                                              int lane, int cw, float *head_part)
{
    const int slot = k % RING;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        bf16x8 a[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            const int t = q >> 1, half = q & 1;
            if (tap_inside<TOP, LEFT, RIGHT>(t)) {
                const int pslot = (k + tap_di(t) * BS + tap_dj(t) + RING) % RING;
                a[q] = load_bf16x8(&ring[l][pslot][lane & 15][half * 32 + 8 * (lane >> 4)]);
            } else {
                a[q] = zero_bf16x8();
            }
        }
        __builtin_amdgcn_sched_barrier(0);  // every load issued before the first product
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 10; ++q)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[q], p.w[l][q], acc, 0, 0, 0);
        if (l < 2) {
            const float sb = p.sbias[l];
            store_col4<RING_ROW>(&ring[l + 1][slot][4 * (lane >> 4)][cw], net_tanh(acc[0], sb), net_tanh(acc[1], sb),
                                 net_tanh(acc[2], sb), net_tanh(acc[3], sb));
        } else {
            head_rows(acc, p, lane, head_part);
        }
        __syncthreads();
    }
}

// ROUND: the sequences are a block round's proposals (sequence first + b for
// round block b): the scorer of the round has gathered each block's current
// spins (seq.x[b]) and boundary (seq.bnd[first + b]) from the lattice and
// written log q of the current block (seq.logq[b]); K and the Philox key come
// from the replica descriptors, and after the draw the workgroup applies the
// Metropolis-Hastings decision to its 16 blocks (the scorer has written
// log q of the current blocks to seq.logq[b]): lanes 16 s .. 16 s + 15 add
// the change dB of the bonds of four sites each (the site's right and lower
// neighbours inside the block and its boundary neighbours), log A =
// K dB + log q(s) - log q(s') in FP64 against the 53-bit uniform of
// Philox(counter (block id, round, replica, 4)), and an accepted proposal is
// XORed into the packed planes (same-colour blocks share no bond, so the
// workgroups of a round do not interact).
template <int BS, bool ROUND>
__global__ __launch_bounds__(256) void k_nn_sample(NetDev net, SeqDev seq, int first, int n_seq, RoundArgs ra)
{
    constexpr int BB = BS * BS;
    __shared__ __attribute__((aligned(16))) uint16_t ring[3][RING][SEQ_PER_WG][RING_ROW];
    __shared__ float head_part[4][SEQ_PER_WG];
    // per-sequence rows padded so the 16 rows of a tile fall in different LDS banks
    __shared__ int8_t xs[SEQ_PER_WG][68];
    __shared__ int8_t bs[SEQ_PER_WG][36];
    __shared__ uint32_t ut[SEQ_PER_WG][65];  // site uniform; replaced by the site's threshold once drawn
    __shared__ float ks[SEQ_PER_WG];
    __shared__ double lq_part[SEQ_PER_WG][16];
    // ROUND: each sequence's replica, block position and blocks per row; the
    // current spins of its block; the proposal's log q
    __shared__ uint32_t sref[ROUND ? SEQ_PER_WG : 1][4];
    __shared__ int8_t cs[ROUND ? SEQ_PER_WG : 1][68];
    // ROUND: the proposal's log q, the current block's, K in FP64 and the MH uniform
    __shared__ double lqs[ROUND ? SEQ_PER_WG : 1][4];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int s0 = first + blockIdx.x * SEQ_PER_WG, end = first + n_seq;

    ArWeights p;
    load_ar_weights(net, wave & 3, lane, p);  // in flight during the set-up
    for (int i = tid; i < SEQ_PER_WG * 64; i += 256)
        xs[i >> 6][i & 63] = 0;
    if (ROUND) {
        if (tid < SEQ_PER_WG) {
            float kc = 0.f;
            if (s0 + tid < end) {
                const uint32_t b = (uint32_t)(s0 + tid - first);
                uint32_t r, bx, by, nbx;
                round_block<BS>(ra, b, r, bx, by, nbx);
                sref[tid][0] = r;
                sref[tid][1] = bx;
                sref[tid][2] = by;
                sref[tid][3] = nbx;
                const double K = ra.kcoup[r];
                kc = (float)K;
                const RepDev &d = ra.reps[r];
                uint32_t o[4];
                philox4x32_10(by * nbx + bx, ra.round, d.replica, 4u, d.seed_lo, d.seed_hi, o);
                lqs[tid][1] = seq.logq[b];  // the scorer's log q of the current block
                lqs[tid][2] = K;
                lqs[tid][3] = (double)(((uint64_t)o[0] << 21) | (o[1] >> 11)) * 1.1102230246251565404e-16;  // 2^-53
            }
            ks[tid] = kc;
        }
        // the current spins and the boundary, gathered from the lattice by the scorer
        for (int i = tid; i < SEQ_PER_WG * 64; i += 256) {
            const int s = i >> 6, k = i & 63;
            const bool live = s0 + s < end;
            if (live && k < BB)
                cs[s][k] = seq.x[(size_t)(s0 + s - first) * BB + k];
            if (k < 32)
                bs[s][k] = (live && k < 4 * BS) ? seq.bnd[(size_t)(s0 + s) * 4 * BS + k] : (int8_t)0;
        }
        __syncthreads();  // sref, read by the uniforms below
    } else {
        for (int i = tid; i < SEQ_PER_WG * 32; i += 256) {
            const int s = i >> 5, k = i & 31;
            bs[s][k] = (s0 + s < end && k < 4 * BS) ? seq.bnd[(size_t)(s0 + s) * 4 * BS + k] : (int8_t)0;
        }
        if (tid < SEQ_PER_WG)
            ks[tid] = s0 + tid < end ? seq.coupling[s0 + tid] : 0.f;
    }
    // site uniforms: word site & 3 of Philox(ctr = (site >> 2, round, replica, 3)),
    // site = blk * BB + k; BB is a multiple of 4, so one call serves sites 4m..4m+3
    for (int i = tid; i < SEQ_PER_WG * 16; i += 256) {
        const int s = i >> 4, m = i & 15;
        if (s0 + s < end && 4 * m < BB) {
            uint32_t key_lo, key_hi, replica, round, blk;
            if (ROUND) {
                const RepDev &d = ra.reps[sref[s][0]];
                key_lo = d.seed_lo;
                key_hi = d.seed_hi;
                replica = d.replica;
                round = ra.round;
                blk = sref[s][2] * sref[s][3] + sref[s][1];
            } else {
                const uint32_t *kk = seq.key + 4 * (size_t)(s0 + s);
                key_lo = kk[0];
                key_hi = kk[1];
                replica = kk[2];
                round = kk[3];
                blk = seq.blk[s0 + s];
            }
            const uint32_t site0 = blk * (uint32_t)BB + 4u * m;
            uint32_t o[4];
            philox4x32_10(site0 >> 2, round, replica, 3u, key_lo, key_hi, o);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                ut[s][4 * m + r] = o[r];
        }
    }
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
            store_col4<RING_ROW>(&ring[0][slot][4 * kin][cw], net_tanh(pre[0]), net_tanh(pre[1]),
                                               net_tanh(pre[2]), net_tanh(pre[3]));
        }
        __syncthreads();
        if (k == BB)
            break;
        // layers 2..4 on the matrix cores; layer 4 feeds the logit head directly
        float *hp = head_part[wave];
        if (i == 0) {
            if (j == 0)
                sample_layers<BS, true, true, false>(ring, p, k, lane, cw, hp);
            else if (j == BS - 1)
                sample_layers<BS, true, false, true>(ring, p, k, lane, cw, hp);
            else
                sample_layers<BS, true, false, false>(ring, p, k, lane, cw, hp);
        } else {
            if (j == 0)
                sample_layers<BS, false, true, false>(ring, p, k, lane, cw, hp);
            else if (j == BS - 1)
                sample_layers<BS, false, false, true>(ring, p, k, lane, cw, hp);
            else
                sample_layers<BS, false, false, false>(ring, p, k, lane, cw, hp);
        }
    }
    if (wave == 0 && kin == 0)
        ut[srow][BB - 1] = thr_prev;
    __syncthreads();
    logq_parts(xs, ut, BB, tid, lq_part);
    __syncthreads();
    if (!ROUND) {
        for (int i = tid; i < SEQ_PER_WG * 64; i += 256) {
            const int s = i >> 6, k = i & 63;
            if (s0 + s < end && k < BB)
                seq.x[(size_t)(s0 + s) * BB + k] = xs[s][k];
        }
        if (tid < SEQ_PER_WG && s0 + tid < end)
            seq.logq[s0 + tid] = logq_total(lq_part[tid], BB);
        return;
    }
    if (tid < SEQ_PER_WG)
        lqs[tid][0] = logq_total(lq_part[tid], BB);
    __syncthreads();
    // Metropolis-Hastings: 16 lanes per block, four sites a lane
    const int sl = tid >> 4, part = tid & 15;
    const bool live = s0 + sl < end;  // the same for the 16 lanes of a block
    int dB = 0;
    uint32_t changed = 0u;
    if (live) {
        const int8_t *bn = bs[sl];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * part + e;
            if (k < BB) {
                const int i = k / BS, j = k - i * BS;
                const int a = cs[sl][k], ap = xs[sl][k];
                changed |= (uint32_t)(a != ap) << e;
                if (j + 1 < BS)
                    dB += ap * xs[sl][k + 1] - a * cs[sl][k + 1];
                if (i + 1 < BS)
                    dB += ap * xs[sl][k + BS] - a * cs[sl][k + BS];
                if (i == 0)
                    dB += (ap - a) * bn[j];
                if (i == BS - 1)
                    dB += (ap - a) * bn[BS + j];
                if (j == 0)
                    dB += (ap - a) * bn[2 * BS + i];
                if (j == BS - 1)
                    dB += (ap - a) * bn[3 * BS + i];
            }
        }
    }
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1)
        dB += __shfl_xor(dB, m, 16);
    if (!live)
        return;
    const uint32_t r = sref[sl][0], bx = sref[sl][1], by = sref[sl][2];
    const RepDev &d = ra.reps[r];
    // log of pi(s') q(s) / (pi(s) q(s')), pi ~ exp(K B)
    const double logA = lqs[sl][2] * (double)dB + lqs[sl][1] - lqs[sl][0];
    if (!(logA >= 0.0 || lqs[sl][3] < exp(logA)))
        return;
    if (part == 0)
        atomicAdd(&ra.accepts[r], 1ull);
    // a lane's four sites lie in one block row (BS >= 4) or two (BS = 2) and
    // their bits of one colour in one plane word: one XOR per (row, colour)
    uint32_t mask[2][2] = {{0u, 0u}, {0u, 0u}};  // [row of the lane's sites][colour]
    uint32_t word[2][2] = {{0u, 0u}, {0u, 0u}};
    const int k0 = 4 * part, i0 = k0 / BS;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if ((changed >> e) & 1u) {
            const int k = k0 + e, i = k / BS, j = k - i * BS;
            const uint32_t x = bx * BS + j, y = by * BS + i, c = (x + y) & 1u, kk = x >> 1;
            mask[i - i0][c] |= 1u << (kk & 31);
            word[i - i0][c] = c * d.Ly * d.W + y * d.W + (kk >> 5);
        }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int c = 0; c < 2; ++c)
            if (mask[q][c])
                atomicXor(&d.plane0[word[q][c]], mask[q][c]);
}

// Scoring has no site-to-site dependency (every spin is given), so a
// workgroup holds all SCORE_POS positions of its blocks in LDS and runs the
// network one layer at a time: layer 1 for every position, then for layers
// 2..4 wave w (output channels 16w .. 16w+15) walks the position tiles of 16
// rows, two independent MFMA chains at a time, the A slices of the next K
// step loaded before the products of the current one.  A row of a tile is one
// (block, site) pair; its A row is the previous layer at the site's five taps
// (an all-zero LDS row outside the block, so the reads never branch), its B
// operands and K order are the sampler's, and a matrix-core product row
// depends only on its own A row, so every site gets the sampler's logit and
// threshold bit for bit.  A wave holds one layer's weights at a time (the
// next layer's load during the barrier), which with 128 positions per
// workgroup leaves room for four workgroups per CU.  The FP64 logarithms of
// log q are taken one position per thread and then summed in the sampler's
// order.
constexpr int SCORE_POS = 128;  // positions per workgroup (a multiple of 64)
constexpr int SCORE_TILES = 2;  // MFMA chains a wave runs together

// ROUND: the sequences are a block round's current blocks, read from the
// packed lattice with their boundaries and K; the spins go to seq.x[b] and
// the boundary to seq.bnd[n_seq + b] for the round's sampler.
template <int BS, bool ROUND>
__global__ __launch_bounds__(256) void k_nn_score(NetDev net, SeqDev seq, int n_seq, RoundArgs ra)
{
    constexpr int BB = BS * BS;
    constexpr int G = SCORE_POS / BB < 16 ? SCORE_POS / BB : 16;  // blocks per workgroup
    constexpr int P = G * BB;                                      // positions (a multiple of 64)
    constexpr int MT = P / 16;                                     // tiles of 16 positions
    static_assert(P % 64 == 0 && MT % SCORE_TILES == 0, "whole tile groups");
    // activations of the layer being read and the layer being written
    // (ping-pong; row P of each is zero); after layer 4 the first holds the
    // thresholds and the log-q parts, the second the head partials and the
    // per-position logarithms
    __shared__ __attribute__((aligned(16))) uint16_t hbuf[2][P + 1][RING_ROW];
    __shared__ int8_t xs[G][64];
    __shared__ int8_t bs[G][32];
    __shared__ float ks[G];
    float(*head_part)[P] = reinterpret_cast<float(*)[P]>(&hbuf[1][0][0]);              // [4][P]
    uint32_t(*thr_s)[64] = reinterpret_cast<uint32_t(*)[64]>(&hbuf[0][0][0]);         // [G][64]
    double(*lq_part)[16] = reinterpret_cast<double(*)[16]>(&hbuf[0][0][0] + G * 64 * 2);  // [G][16]
    double *lg = reinterpret_cast<double *>(&hbuf[1][0][0]) + 2 * P;  // [P], after the head partials

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int s0 = blockIdx.x * G;

    bf16x8 w[10];
    load_ar_layer(net, 0, wave, lane, w);  // layer 2's, in flight under the set-up and layer 1
    if (ROUND) {
        __shared__ uint32_t sref[G][3];  // replica, bx, by of each block
        if (tid < G) {
            float kc = 0.f;
            if (s0 + tid < n_seq) {
                uint32_t r, bx, by, nbx;
                round_block<BS>(ra, (uint32_t)(s0 + tid), r, bx, by, nbx);
                sref[tid][0] = r;
                sref[tid][1] = bx;
                sref[tid][2] = by;
                kc = (float)ra.kcoup[r];
            }
            ks[tid] = kc;
        }
        __syncthreads();
        for (int i = tid; i < G * 64; i += 256) {
            const int s = i >> 6, k = i & 63;
            const bool live = s0 + s < n_seq;
            int8_t v = 0, bv = 0;
            if (live) {
                const RepDev &d = ra.reps[sref[s][0]];
                const uint32_t bx = sref[s][1], by = sref[s][2];
                if (k < BB)
                    v = (int8_t)spin_at(d, bx * BS + k % BS, by * BS + k / BS);
                if (k < 4 * BS)
                    bv = boundary_spin(d, BS, bx, by, k);
            }
            xs[s][k] = v;
            if (k < 32)
                bs[s][k] = bv;
            // for the sampler of this round: the current spins (its MH) and the
            // boundary of the proposal, sequence n_seq + b
            if (live && k < BB)
                seq.x[(size_t)(s0 + s) * BB + k] = v;
            if (live && k < 4 * BS)
                seq.bnd[(size_t)(n_seq + s0 + s) * 4 * BS + k] = bv;
        }
    } else {
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
    }
    if (tid < 18) {  // the two zero rows, 9 x 16 bytes each
        uint4 *z = reinterpret_cast<uint4 *>(&hbuf[tid / 9][P][0]);
        z[tid % 9] = make_uint4(0u, 0u, 0u, 0u);
    }
    ArScalars p;
    load_ar_scalars(net, wave, lane, p);
    const int cw = 16 * wave + (lane & 15);
    __syncthreads();

    // layer 1: this wave's 16 channels for every tile of 16 positions
    for (int m = 0; m < MT; ++m) {
        const int pos = 16 * m + (lane & 15);  // this lane's row
        const int s = pos / BB, k = pos - s * BB, i = k / BS, j = k - i * BS;
        float in_tap, in_bnd, in_k;
        layer1_inputs<BS>(&xs[s][0], -1, 0.f, &bs[s][0], ks[s], i, j, lane >> 4, &in_tap, &in_bnd, &in_k);
        const floatx4 pre = layer1_tile(in_tap, in_bnd, in_k, p);
        store_col4<RING_ROW>(&hbuf[0][16 * m + 4 * (lane >> 4)][cw], net_tanh(pre[0]), net_tanh(pre[1]),
                             net_tanh(pre[2]), net_tanh(pre[3]));
    }
    __syncthreads();

    // layers 2..4: this wave's 16 output channels for every position; a lane's
    // A row sits at the same place (site k, column j) of every tile whose
    // block row is the same, so the column taps' validity is fixed per lane
    const int r16 = lane & 15, kq = 8 * (lane >> 4);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const uint16_t(*hin)[RING_ROW] = hbuf[l & 1];
        uint16_t(*hout)[RING_ROW] = hbuf[(l + 1) & 1];
        for (int m0 = 0; m0 < MT; m0 += SCORE_TILES) {
            floatx4 acc[SCORE_TILES];
            int si[SCORE_TILES], sj[SCORE_TILES], row[SCORE_TILES];
#pragma unroll
            for (int u = 0; u < SCORE_TILES; ++u) {
                acc[u] = floatx4{0.f, 0.f, 0.f, 0.f};
                row[u] = 16 * (m0 + u) + r16;  // this lane's A row
                const int k = row[u] % BB;
                si[u] = k / BS;
                sj[u] = k - si[u] * BS;
            }
            // the A slices of K step q (tap q >> 1, channel half q & 1); those of
            // step q + 1 are loaded before the products of step q
            bf16x8 a_cur[SCORE_TILES], a_nxt[SCORE_TILES];
            auto load_step = [&](int q, bf16x8 *a) {
                const int t = q >> 1, half = q & 1;
#pragma unroll
                for (int u = 0; u < SCORE_TILES; ++u) {
                    const int ii = si[u] + tap_di(t), jj = sj[u] + tap_dj(t);
                    const bool ok = (ii >= 0) & (jj >= 0) & (jj < BS);
                    a[u] = load_bf16x8(&hin[ok ? row[u] + tap_di(t) * BS + tap_dj(t) : P][half * 32 + kq]);
                }
            };
            load_step(0, a_cur);
#pragma unroll
            for (int q = 0; q < 10; ++q) {
                if (q < 9)
                    load_step(q + 1, a_nxt);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < SCORE_TILES; ++u)
                    acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_cur[u], w[q], acc[u], 0, 0, 0);
#pragma unroll
                for (int u = 0; u < SCORE_TILES; ++u)
                    a_cur[u] = a_nxt[u];
            }
#pragma unroll
            for (int u = 0; u < SCORE_TILES; ++u) {
                const int row0 = 16 * (m0 + u) + 4 * (lane >> 4);
                if (l < 2) {
                    const float sb = p.sbias[l];
                    store_col4<RING_ROW>(&hout[row0][cw], net_tanh(acc[u][0], sb), net_tanh(acc[u][1], sb),
                                         net_tanh(acc[u][2], sb), net_tanh(acc[u][3], sb));
                } else {
                    // hout is the other buffer, free now: head partials of this wave
                    head_rows(acc[u], p, lane, &head_part[wave][16 * (m0 + u)]);
                }
            }
        }
        if (l < 2)
            load_ar_layer(net, l + 1, wave, lane, w);
        __syncthreads();
    }

    // thresholds (position pos = s * BB + k) and log q, in the sampler's order
    for (int pos = tid; pos < P; pos += 256) {
        const int s = pos / BB, k = pos - s * BB;
        thr_s[s][k] = site_threshold(head_logit(head_part[0], head_part[1], head_part[2], head_part[3], pos, p.bo));
    }
    __syncthreads();
    // the FP64 logarithm of every position on a thread of its own, then the
    // sampler's parts (four consecutive sites each, summed in order)
    for (int pos = tid; pos < P; pos += 256) {
        const int s = pos / BB, k = pos - s * BB;
        lg[pos] = site_log(xs[s][k], thr_s[s][k]);
    }
    __syncthreads();
    for (int idx = tid; idx < G * 16; idx += 256) {
        const int s = idx >> 4, pt = idx & 15;
        double acc = 0.0;
        for (int k = pt * 4; k < pt * 4 + 4 && k < BB; ++k)
            acc += lg[s * BB + k];
        lq_part[s][pt] = acc;
    }
    __syncthreads();
    if (tid < G && s0 + tid < n_seq)
        seq.logq[s0 + tid] = logq_total(lq_part[tid], BB);
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

hipError_t train_tiles(const NetDev &net, const TrainWs &ws, const int8_t *x, const int8_t *bnd, const float *kc,
                       int nblk, int Bs, bool sampled, uint32_t n_rows, uint64_t seed, bool advance, hipStream_t st)
{
    const int Pv = nblk * Bs * Bs, n_tiles = (Pv + TILE - 1) / TILE;
    const int splits = (Pv + WGRAD_CHUNK - 1) / WGRAD_CHUNK;
    const BatchSrc srcb{x, bnd, kc, sampled ? (const uint32_t *)net.step : nullptr, n_rows, (uint32_t)seed,
                        (uint32_t)(seed >> 32)};
    uint32_t *adv = advance ? net.step : (uint32_t *)nullptr;
    const dim3 tg(n_tiles), wg(5, splits, 3), blk(256);
    switch (Bs) {
    case 2:
        hipLaunchKernelGGL(k_train_tile<2>, tg, blk, 0, st, net, ws, srcb, nblk);
        hipLaunchKernelGGL(k_wgrad<2>, wg, blk, 0, st, ws, Pv, splits, adv);
        break;
    case 4:
        hipLaunchKernelGGL(k_train_tile<4>, tg, blk, 0, st, net, ws, srcb, nblk);
        hipLaunchKernelGGL(k_wgrad<4>, wg, blk, 0, st, ws, Pv, splits, adv);
        break;
    case 8:
        hipLaunchKernelGGL(k_train_tile<8>, tg, blk, 0, st, net, ws, srcb, nblk);
        hipLaunchKernelGGL(k_wgrad<8>, wg, blk, 0, st, ws, Pv, splits, adv);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t finish_step(const NetDev &net, const TrainWs &ws, int nblk, int Bs, bool adam, float lr,
                       float *loss_out, hipStream_t st)
{
    const int Pv = nblk * Bs * Bs, n_tiles = (Pv + TILE - 1) / TILE;
    const int splits = (Pv + WGRAD_CHUNK - 1) / WGRAD_CHUNK;
    const dim3 grid(FIN_W_BLOCKS + FIN_S_BLOCKS);
    if (adam)
        hipLaunchKernelGGL(k_finish<true>, grid, dim3(256), 0, st, net, ws, n_tiles, splits, Pv, lr, loss_out);
    else
        hipLaunchKernelGGL(k_finish<false>, grid, dim3(256), 0, st, net, ws, n_tiles, splits, Pv, lr, loss_out);
    return hipGetLastError();
}

template <int BS, bool ROUND>
static hipError_t ar_pass_bs(const NetDev &net, const SeqDev &seq, int n_score, int n_sample, const RoundArgs &ra,
                             hipStream_t st)
{
    if (n_score > 0) {
        constexpr int G = SCORE_POS / (BS * BS) < 16 ? SCORE_POS / (BS * BS) : 16;
        hipLaunchKernelGGL((k_nn_score<BS, ROUND>), dim3(blocks_for(n_score, G)), dim3(256), 0, st, net, seq,
                           n_score, ra);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (n_sample > 0) {
        hipLaunchKernelGGL((k_nn_sample<BS, ROUND>), dim3(blocks_for(n_sample, SEQ_PER_WG)), dim3(256), 0, st, net,
                           seq, n_score, n_sample, ra);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t ar_pass(const NetDev &net, const SeqDev &seq, int n_score, int n_sample, int Bs, hipStream_t st)
{
    const RoundArgs none{};
    switch (Bs) {
    case 2: return ar_pass_bs<2, false>(net, seq, n_score, n_sample, none, st);
    case 4: return ar_pass_bs<4, false>(net, seq, n_score, n_sample, none, st);
    case 8: return ar_pass_bs<8, false>(net, seq, n_score, n_sample, none, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t block_round_pass(const NetDev &net, const SeqDev &seq, const RepDev *reps, const double *kcoup, int Bs,
                            uint32_t colour, uint32_t round, uint32_t first, uint32_t count, uint32_t per_rep,
                            int64_t *accepts, hipStream_t st)
{
    const RoundArgs ra{reps, kcoup, reinterpret_cast<unsigned long long *>(accepts), colour, round, first, count,
                       per_rep};
    switch (Bs) {
    case 2: return ar_pass_bs<2, true>(net, seq, (int)count, (int)count, ra, st);
    case 4: return ar_pass_bs<4, true>(net, seq, (int)count, (int)count, ra, st);
    case 8: return ar_pass_bs<8, true>(net, seq, (int)count, (int)count, ra, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t seq_setup(const SeqDev &seq, int n, uint64_t seed, uint32_t replica, uint32_t round, uint32_t blk0,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_seq_setup, dim3(blocks_for(n, 256)), dim3(256), 0, st, seq, n,
                       (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), replica, round, blk0);
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
