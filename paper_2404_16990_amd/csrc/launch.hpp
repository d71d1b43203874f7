// Host-side launchers of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device.hpp"

namespace ising {

// Replicas swept in streaming mode: workgroup g of a launch serves list entry
// e with prefix[e] <= g < prefix[e+1] (prefix has n + 1 entries, device memory).
struct StreamList {
    const RepDev *reps;
    const uint32_t *list;
    const uint32_t *prefix;
    uint32_t n;
    uint32_t n_wg;
    uint32_t words_per_wg;
};

// Replicas swept in LDS-resident mode: one workgroup per entry.
struct ResidentList {
    const RepDev *reps;
    const uint32_t *list;
    uint32_t n;
    uint32_t lds_bytes;  // dynamic LDS per workgroup (largest replica of the list)
};

hipError_t launch_init(const RepDev *reps, const int32_t *modes, uint32_t n, uint32_t max_words,
                       hipStream_t st);
// Adds replica r's (B, M) to bond[r * stride], mag[r * stride].
hipError_t launch_observables(const RepDev *reps, uint32_t n, uint32_t max_words, int64_t *bond,
                              int64_t *mag, hipStream_t st, uint32_t stride = 1);
// Adds replica r's (B, M) after step t + step to its trace slot if the step
// is a recorded one (slot from the device counters t, t0; see RecArgs).  The
// recording arguments are read from device memory (rec), where
// launch_begin_run put the current run's, so captured graphs stay valid.
hipError_t launch_observables_rec(const RepDev *reps, uint32_t n, uint32_t max_words, const RecArgs *rec,
                                  uint32_t step, hipStream_t st);
hipError_t launch_fill_i64(int64_t *p, uint64_t n, int64_t v, hipStream_t st);
// Start of a run in one launch: t0 = t for every replica, the recording
// arguments v to dst, and v's trace slots (n x v.n_rec each, if v.bond) zeroed.
hipError_t launch_begin_run(RepDev *reps, uint32_t n, RecArgs *dst, const RecArgs &v, hipStream_t st);
hipError_t launch_advance(RepDev *reps, uint32_t n, uint32_t delta, hipStream_t st);
hipError_t launch_sweep_stream(const StreamList &L, int word_bits, int threads, uint32_t colour,
                               uint32_t sweep_off, const RecArgs *rec, hipStream_t st);
hipError_t launch_sweep_resident(const ResidentList &L, int word_bits, int threads, uint32_t n_sweeps,
                                 const RecArgs *rec, hipStream_t st);
// Raise the dynamic-LDS limit of every resident-kernel instantiation.
hipError_t prepare_resident_kernels(int max_dynamic_lds);
// Largest static LDS of the resident kernels in bytes, as the runtime reports it.
uint32_t resident_static_lds(int threads);

}  // namespace ising
