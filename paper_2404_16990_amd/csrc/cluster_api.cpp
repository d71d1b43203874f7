// Host runtime of the cluster steps (Swendsen-Wang, Wolff): descriptors,
// workspace layout, validation and the step loop.  Every device computation
// is a kernel in cluster.hip or kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ising.h"
#include "batch.hpp"
#include "cluster.hpp"
#include "launch.hpp"

using namespace ising;

#define CL_HIP(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(ISING_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Fortuin-Kasteleyn occupation: P(occupied | aligned) = 1 - exp(-2K), i.e.
// occupied iff the bond's word >= floor(exp(-2K) 2^32) (clamped to 2^32 - 1).
void set_bond_threshold(ClRep &c, double J, double beta)
{
    const double K = beta * J;
    c.none = K == 0.0 ? 1u : 0u;
    c.thr2 = prob_threshold(std::exp(-2.0 * K));
}

}  // namespace

int ising::cluster_setup(ising_batch *b, hipStream_t st)
{
    const int32_t n = b->n;
    b->cl.assign(n, ClRep{});
    b->tile_prefix.assign(n + 1, 0u);
    uint64_t tiles = 0;
    size_t off = 0;
    for (int32_t r = 0; r < n; ++r) {
        ClRep &c = b->cl[r];
        const RepDev &d = b->rep[r];
        c.g_off = off;
        off += align256((size_t)d.N * sizeof(uint32_t));
        c.tiles_y = (d.Ly + kClRows - 1) / kClRows;
        c.tile0 = (uint32_t)tiles;
        b->tile_prefix[r] = (uint32_t)tiles;
        set_bond_threshold(c, b->desc[r].J, b->desc[r].beta);
        tiles += (uint64_t)d.W * c.tiles_y;
        if (tiles >= (1ull << 31))
            return fail(ISING_E_UNSUPPORTED, "a batch may hold at most 2^31 - 1 cluster tiles (about 4.4e12 sites)");
    }
    b->tile_prefix[n] = (uint32_t)tiles;
    b->cl_tiles = tiles;
    b->cl_tb_off = off;
    b->cl_ws_bytes = off + (size_t)tiles * sizeof(uint4);
    b->d_cl = reinterpret_cast<ClRep *>(b->buf + b->layout.cl);
    b->d_tile_prefix = reinterpret_cast<uint32_t *>(b->buf + b->layout.clprefix);
    CL_HIP(hipMemcpyAsync(b->d_cl, b->cl.data(), (size_t)n * sizeof(ClRep), hipMemcpyHostToDevice, st));
    CL_HIP(hipMemcpyAsync(b->d_tile_prefix, b->tile_prefix.data(), (size_t)(n + 1) * sizeof(uint32_t),
                          hipMemcpyHostToDevice, st));
    return ISING_OK;
}

int ising::cluster_set_beta(ising_batch *b, int32_t r, hipStream_t st)
{
    set_bond_threshold(b->cl[r], b->desc[r].J, b->desc[r].beta);
    CL_HIP(hipMemcpyAsync(&b->d_cl[r], &b->cl[r], sizeof(ClRep), hipMemcpyHostToDevice, st));
    return ISING_OK;
}

extern "C" {

int ising_cluster_ws_bytes(ising_batch *b, size_t *bytes)
{
    clear_error();
    if (!b || !bytes)
        return fail(ISING_E_INVALID, "handle and bytes must not be NULL");
    *bytes = b->cl_ws_bytes;
    return ISING_OK;
}

int ising_batch_cluster(ising_batch *b, int32_t algorithm, uint64_t n_steps, uint32_t record_every, void *dev_ws,
                        size_t ws_bytes, int64_t *dev_bond_trace, int64_t *dev_mag_trace, void *stream)
{
    clear_error();
    if (!b)
        return fail(ISING_E_INVALID, "NULL batch handle");
    if (algorithm != ISING_CLUSTER_SWENDSEN_WANG && algorithm != ISING_CLUSTER_WOLFF)
        return fail(ISING_E_INVALID, "unknown cluster algorithm");
    if (!dev_ws)
        return fail(ISING_E_INVALID, "dev_ws must not be NULL");
    if ((reinterpret_cast<uintptr_t>(dev_ws) & 255) != 0)
        return fail(ISING_E_INVALID, "dev_ws must be 256-byte aligned");
    if (ws_bytes < b->cl_ws_bytes)
        return fail(ISING_E_NOMEM, "dev_ws is smaller than ising_cluster_ws_bytes()");
    if (n_steps == 0)
        return ISING_OK;
    for (int32_t r = 0; r < b->n; ++r)
        if ((uint64_t)b->rep[r].t + n_steps > 0xffffffffull)
            return fail(ISING_E_INVALID, "step counter would reach 2^32");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    uint32_t n_rec = 0;
    if (record_every > 0 && dev_bond_trace && dev_mag_trace && n_steps / record_every > 0) {
        n_rec = (uint32_t)(n_steps / record_every);
        const uint64_t slots = (uint64_t)b->n * n_rec;
        CL_HIP(launch_fill_i64(dev_bond_trace, slots, 0, hs));
        CL_HIP(launch_fill_i64(dev_mag_trace, slots, 0, hs));
    }
    char *ws = static_cast<char *>(dev_ws);
    ClArgs a;
    a.reps = b->d_rep;
    a.cl = b->d_cl;
    a.tile_prefix = b->d_tile_prefix;
    a.n = (uint32_t)b->n;
    a.ws = ws;
    a.tb = reinterpret_cast<uint4 *>(ws + b->cl_tb_off);
    a.tiles = (uint32_t)b->cl_tiles;
    for (uint64_t i = 0; i < n_steps; ++i) {
        CL_HIP(launch_cluster_step(a, algorithm, (uint32_t)i, hs));
        if (n_rec && (i + 1) % record_every == 0) {
            const uint64_t j = (i + 1) / record_every - 1;
            CL_HIP(launch_observables(b->d_rep, (uint32_t)b->n, b->max_words, dev_bond_trace + j, dev_mag_trace + j,
                                      hs, n_rec));
        }
    }
    CL_HIP(launch_advance(b->d_rep, (uint32_t)b->n, (uint32_t)n_steps, hs));
    for (int32_t r = 0; r < b->n; ++r)
        b->rep[r].t += (uint32_t)n_steps;
    return ISING_OK;
}

}  // extern "C"
