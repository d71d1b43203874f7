// Swendsen-Wang and Wolff cluster steps on the packed batch state: definitions
// shared by the host runtime (cluster_api.cpp) and the kernels (cluster.hip).
//
// A replica is cut into tiles of 64 columns (one 32-bit word of each colour
// plane per row) by kClRows rows (fewer in the last tile row when Ly is not a
// multiple).  One step is four launches over all tiles of the batch:
//   local     bonds of the tile drawn, clusters inside the tile labelled in LDS
//             (horizontal runs from bit masks, vertical bonds by union-find),
//             every site's label (the global index of its tile-local root)
//             written to the workspace, the occupied bonds that leave the tile
//             (right column, bottom row) kept as two masks;
//   merge     the crossing bonds united in the workspace by lock-free
//             union-find (a root is linked to a smaller index by atomic min);
//   compress  every path from a crossing-bond endpoint to its root rewritten
//             to point at the root, so that each tile-local root of a merged
//             cluster points straight at the cluster's root;
//   flip      root = label of the label; Swendsen-Wang flips the site if its
//             root's bit says so, Wolff if its root is the seed's root.
// The root of every cluster is its smallest site index, whatever the order in
// which the union-find ran, so the result is a function of the random words
// alone.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace ising {

constexpr uint32_t kClRows = 64;
static_assert(kClRows % 8 == 0 && kClRows <= 64, "4 waves of an even number of rows; crossing masks are 64-bit");
// Tiles per kernel launch: keeps every grid far below the 2^32 work-item
// limit of a dispatch (a phase over more tiles is split into launches).
constexpr uint32_t kClTilesPerLaunch = 1u << 22;

// Per-replica cluster descriptor (32 bytes) in the batch's device buffer.
struct ClRep {
    uint64_t g_off;    // byte offset of the replica's label array (Lx*Ly uint32) in the workspace
    uint32_t tile0;    // first tile of the replica in the batch-wide tile numbering
    uint32_t tiles_y;  // tile rows: ceil(Ly / kClRows)
    uint32_t thr2;     // a bond between aligned spins is occupied iff its word >= thr2
    uint32_t none;     // 1 when beta*J == 0: no bond is occupied
    uint32_t pad[2];
};
static_assert(sizeof(ClRep) == 32, "cluster descriptor must stay 32 bytes");

struct ClArgs {
    const RepDev *reps;
    const ClRep *cl;
    const uint32_t *tile_prefix;  // n + 1 entries: each replica's tile0, then the total
    uint32_t n;                   // replicas
    uint32_t tiles;               // tiles of the whole batch (< 2^31)
    char *ws;                     // workspace base (256-byte aligned)
    uint4 *tb;                    // crossing-bond masks, one entry per tile
};

enum { kClSwendsenWang = 0, kClWolff = 1 };

// Enqueue one cluster step (counter t + step for every replica) on st.
hipError_t launch_cluster_step(const ClArgs &a, int algorithm, uint32_t step, hipStream_t st);

// Bytes of the library's own cluster workspace (one copy per device, part of
// the loaded code object, held until the process ends).
constexpr size_t kClStaticWsBytes = size_t(64) << 20;
// Device address of that workspace on `device`, which must be the current
// device; looked up once per device and kept.
hipError_t static_cluster_ws(int device, char **ptr);

}  // namespace ising
