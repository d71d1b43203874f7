// Host-side launchers of the block-proposal network kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "nn.hpp"

namespace ising {
namespace nn {

hipError_t cast_weights(const NetDev &net, hipStream_t st);
// Forward and backward of a batch of nblk blocks: rows 0..nblk-1 of (x, bnd,
// kc), or with sampled a minibatch of nblk rows drawn from the n_rows rows
// with the step counter and seed; writes the logits, the tile partial sums and
// the weight-gradient partials; advance: count one training step on the device.
hipError_t train_tiles(const NetDev &net, const TrainWs &ws, const int8_t *x, const int8_t *bnd, const float *kc,
                       int nblk, int Bs, bool sampled, uint32_t n_rows, uint64_t seed, bool advance, hipStream_t st);
// Gradient and loss from the partials (loss also to loss_out if not null);
// adam: the Adam update with the step number of the device counter.
hipError_t finish_step(const NetDev &net, const TrainWs &ws, int nblk, int Bs, bool adam, float lr,
                       float *loss_out, hipStream_t st);
// sequences [0, n_score) are scored, [n_score, n_score + n_sample) sampled
hipError_t ar_pass(const NetDev &net, const SeqDev &seq, int n_score, int n_sample, int Bs, hipStream_t st);
// One colour of a block round for round blocks [first, first + count):
// scores the current blocks (read from the lattice), samples the proposals
// and applies the Metropolis-Hastings decisions to the packed planes.
hipError_t block_round_pass(const NetDev &net, const SeqDev &seq, const RepDev *reps, const double *kcoup, int Bs,
                            uint32_t colour, uint32_t round, uint32_t first, uint32_t count, uint32_t per_rep,
                            int64_t *accepts, hipStream_t st);
hipError_t seq_setup(const SeqDev &seq, int n, uint64_t seed, uint32_t replica, uint32_t round, uint32_t blk0,
                     hipStream_t st);
hipError_t extract(const RepDev *reps, const double *kcoup, int Bs, uint32_t per_rep, uint32_t count,
                   uint32_t draw, int8_t *x, int8_t *bnd, float *kout, hipStream_t st);

}  // namespace nn
}  // namespace ising
