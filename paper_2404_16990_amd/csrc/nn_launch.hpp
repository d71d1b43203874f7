// Host-side launchers of the block-proposal network kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "nn.hpp"

namespace ising {
namespace nn {

hipError_t cast_weights(const NetDev &net, hipStream_t st);
hipError_t forward(const NetDev &net, const TrainWs &ws, const int8_t *x, const int8_t *bnd, const float *kc,
                   int nblk, int Bs, hipStream_t st);
hipError_t backward(const NetDev &net, const TrainWs &ws, const int8_t *x, const int8_t *bnd, const float *kc,
                    int nblk, int Bs, hipStream_t st);
// Adam update with the step number from the device counter, then the counter advanced.
hipError_t adam(const NetDev &net, float lr, hipStream_t st);
// minibatch rows of the training step numbered by the device counter
hipError_t gather_rows(const NetDev &net, const TrainWs &ws, const int8_t *x, const int8_t *bnd, const float *kc,
                       uint32_t n_rows, int batch, int Bs, uint64_t seed, hipStream_t st);
// sequences [0, n_score) are scored, [n_score, n_score + n_sample) sampled
hipError_t ar_pass(const NetDev &net, const SeqDev &seq, int n_score, int n_sample, int Bs, hipStream_t st);
hipError_t block_gather(const RepDev *reps, const double *kcoup, int Bs, uint32_t colour, uint32_t round,
                        uint32_t first, uint32_t count, uint32_t per_rep, const SeqDev &seq, hipStream_t st);
hipError_t block_mh(const RepDev *reps, const double *kcoup, int Bs, uint32_t colour, uint32_t round,
                    uint32_t first, uint32_t count, uint32_t per_rep, const SeqDev &seq, int64_t *accepts,
                    hipStream_t st);
hipError_t seq_setup(const SeqDev &seq, int n, uint64_t seed, uint32_t replica, uint32_t round, uint32_t blk0,
                     hipStream_t st);
hipError_t extract(const RepDev *reps, const double *kcoup, int Bs, uint32_t per_rep, uint32_t count,
                   uint32_t draw, int8_t *x, int8_t *bnd, float *kout, hipStream_t st);

}  // namespace nn
}  // namespace ising
