// Block-proposal network: shared definitions of the device kernels (nn.hip)
// and the host runtime (nn_api.cpp).
//
// The network proposes a joint update of one Bs x Bs block given its 4*Bs
// boundary spins and K = beta*J, site by site in raster order, so its
// proposal probability is a product of tractable conditionals:
//   layer 1, spin taps A = {(-1,-1), (-1,0), (-1,1), (0,-1)} (row, column):
//     pre1[p,c] = sum_t x[p+t] W1[t,c] + sum_f bnd[p,f] U1[f,c] + K v1[c] + b1[c]
//   layers 2..4, taps B = A + {(0,0)} over the previous layer's activations:
//     pre_l[p,c] = sum_t sum_c' h_{l-1}[p+t,c'] W_l[t,c',c] + b_l[c]
//   h_l = tanh(pre_l);  logit[p] = sum_c h4[p,c] wo[c] + bo;
//   P(x_p = +1 | x_<p, boundary, K) = sigmoid(logit[p]).
// Outside the block the spin field and activations are zero; bnd[p] holds
// the boundary spins next to site p (up, down, left, right), 0 elsewhere.
// Layers 2..4 run on BF16 matrix cores with FP32 accumulation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {
namespace nn {

constexpr int C = 64;       // channels
constexpr int KB = 5 * C;   // K of a type-B layer as a GEMM (5 taps x C)
constexpr int RING = 10;    // ring of positions kept per layer by the incremental pass (>= Bs + 2)

// Offsets into the flat float parameter vector.
constexpr int OFF_W1 = 0, OFF_U1 = 4 * C, OFF_V1 = 8 * C, OFF_B1 = 9 * C;
__host__ __device__ constexpr int off_w(int l) { return 10 * C + (l - 2) * (5 * C * C + C); }
__host__ __device__ constexpr int off_b(int l) { return off_w(l) + 5 * C * C; }
constexpr int OFF_WO = 10 * C + 3 * (5 * C * C + C);
constexpr int OFF_BO = OFF_WO + C;
constexpr int N_PARAMS = OFF_BO + 1;

// tap offsets (row, column); taps 0..3 are A, tap 4 is the centre
__host__ __device__ constexpr int tap_di(int t) { return t < 3 ? -1 : 0; }
__host__ __device__ constexpr int tap_dj(int t) { return t < 3 ? t - 1 : (t == 3 ? -1 : 0); }

// Device pointers of one network: parameters, Adam moments, BF16 copies.
struct NetDev {
    float *params, *adam_m, *adam_v, *grad;
    uint16_t *wt;   // [3][C][KB]  wt[l][c][t*C + c'] = W_l[t][c'][c]   (bf16, forward B operand)
    uint16_t *wtd;  // [3][C][KB]  wtd[l][c'][t*C + c] = W_l[t][c'][c]  (bf16, data-gradient B operand)
    uint32_t *step; // training steps taken since the parameters were set (device counter)
};

// Sequences for the incremental (autoregressive) pass.
struct SeqDev {
    int8_t *x;        // [n][Bs*Bs]: given block (score) or output (sample)
    int8_t *bnd;      // [n][4*Bs]: top row, bottom row, left column, right column
    float *coupling;  // [n]: K = beta*J
    uint32_t *key;    // [n][4]: seed_lo, seed_hi, replica, round
    uint32_t *blk;    // [n]: block id (Philox counter for the site uniforms)
    double *logq;     // [n]
};

// Positions per split of the weight-gradient product (its K; a multiple of 64).
constexpr int WGRAD_CHUNK = 512;

// Positions per training tile: whole blocks of every supported size (2, 4, 8).
constexpr int TILE = 64;

// A tile's row of partial sums (PART_ROW floats): the layer-1 gradients (W1,
// U1, v1, b1: 10 C, in parameter order), the bias gradients of layers 2, 3, 4
// and the head weights (C each), the head bias, the loss.
constexpr int PART_L1 = 0, PART_B2 = 10 * C, PART_B3 = 11 * C, PART_B4 = 12 * C, PART_WO = 13 * C;
constexpr int PART_BO = 14 * C, PART_LOSS = 14 * C + 1, PART_USED = 14 * C + 2, PART_ROW = 15 * C;

// Training workspace (positions padded to a multiple of TILE).
struct TrainWs {
    uint16_t *hb[3];    // [P][C] bf16 inputs of layers 2..4 (activations of layers 1..3)
    uint16_t *db[3];    // [P][C] bf16 pre-activation gradients of layers 2..4
    float *logits;      // [P]
    float *partial;     // [tiles][PART_ROW]
    float *wpart;       // [3][splits][KB][C] weight-gradient partials
    float *loss;        // [1]
};

}  // namespace nn
}  // namespace ising
