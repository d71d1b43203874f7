// 3D (simple cubic) sweeps: device descriptor and launchers shared by the host
// runtime (ising3d_api.cpp) and the kernels (ising3d.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

enum : uint32_t { k3Always = 1u, k3Bitsliced = 2u };

// Per-replica device descriptor (64 bytes); t is advanced on the device.
struct Rep3Dev {
    uint32_t *plane0;          // colour-0 plane; colour-1 plane = plane0 + Lz * Ly * W
    uint32_t Lx, Ly, Lz, W;    // W = 32-bit words per colour row = Lx / 64
    uint32_t seed_lo, seed_hi, replica;
    uint32_t flags;            // bit 0: beta*J == 0 (every proposal accepted); bit 1: bit-sliced contract
    uint32_t thr4, thr8, thr12;
    uint32_t t;                // sweeps completed
    uint64_t N;                // Lx * Ly * Lz
};
static_assert(sizeof(Rep3Dev) == 64, "3D descriptor must stay 64 bytes");

// Words of one colour handled by one 256-thread workgroup.
constexpr uint32_t k3WordsPerBlock = 1024;

// Words per group of the sweep for rows of W words: a thread updates groups
// of 4, 2 or 1 consecutive words of a row.
__host__ __device__ inline uint32_t group_width(uint32_t W)
{
    return (W & 3u) == 0 ? 4u : (W & 1u) == 0 ? 2u : 1u;
}

// Workgroup b of a launch serves replica r with prefix[r] <= b < prefix[r+1]
// (prefix: n + 1 entries in device memory).  widths: bit k set when some
// replica's group width is 2^k (one sweep kernel per width present).
struct Sweep3Args {
    const Rep3Dev *reps;
    const uint32_t *prefix;
    uint32_t n, blocks;
    uint32_t widths;
};

hipError_t launch3_init(const Sweep3Args &a, const int32_t *modes, hipStream_t st);
hipError_t launch3_sweep(const Sweep3Args &a, uint32_t colour, uint32_t sweep_off, hipStream_t st);
// Adds replica r's (B, M) to bond[r * stride], mag[r * stride].
hipError_t launch3_observables(const Sweep3Args &a, int64_t *bond, int64_t *mag, uint32_t stride, hipStream_t st);
hipError_t launch3_advance(Rep3Dev *reps, uint32_t n, uint32_t delta, hipStream_t st);

}  // namespace ising
