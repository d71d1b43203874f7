// Host runtime of the cluster steps (Swendsen-Wang, Wolff): descriptors,
// workspace layout, validation and the step loop.  Every device computation
// is a kernel in cluster.hip or kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
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

// Steps per captured chunk: enough to amortise the launches of a step (four
// cluster kernels and a recording kernel), few enough to keep capture cheap.
constexpr uint32_t kClChunk = 16;

// n steps (run-local offsets 0 .. n-1 from the device counters), the
// recording of each, and the counter advance, enqueued on st.
// The recording kernels read the run's arguments from the batch's device slot.
int enqueue_cluster_chunk(ising_batch *b, const ClArgs &a, int algorithm, uint32_t n, bool recording,
                          hipStream_t st)
{
    for (uint32_t j = 0; j < n; ++j) {
        CL_HIP(launch_cluster_step(a, algorithm, j, st));
        if (recording)
            CL_HIP(launch_observables_rec(b->d_rep, (uint32_t)b->n, b->max_words, b->d_rec, j, st));
    }
    CL_HIP(launch_advance(b->d_rep, (uint32_t)b->n, n, st));
    return ISING_OK;
}

int cluster_graph(ising_batch *b, const ClArgs &a, int algorithm, uint32_t n, bool recording,
                  hipGraphExec_t *out)
{
    const ClGraphKey key{algorithm, n, a.ws, recording};
    auto it = b->cl_graphs.find(key);
    if (it != b->cl_graphs.end()) {
        *out = it->second;
        return ISING_OK;
    }
    if (b->cl_graphs.size() >= 16)
        drop_cluster_graphs(b);
    CL_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const int st = enqueue_cluster_chunk(b, a, algorithm, n, recording, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (st != ISING_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess)
        return fail(ISING_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess)
        return fail(ISING_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    b->cl_graphs[key] = ex;
    b->n_captures += 1;
    *out = ex;
    return ISING_OK;
}

}  // namespace

void ising::drop_cluster_graphs(ising_batch *b)
{
    if (b->cl_graphs.empty())
        return;
    (void)wait_graph_replays(b);
    for (auto &kv : b->cl_graphs)
        (void)hipGraphExecDestroy(kv.second);
    b->cl_graphs.clear();
}

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

}  // extern "C"

namespace {

// The body of both cluster entry points once the workspace is known.  With
// graphs, whole chunks replay one captured graph and the rest is launched
// directly; without, every step is launched directly (nothing is allocated).
int run_cluster(ising_batch *b, int32_t algorithm, uint64_t n_steps, uint32_t record_every, char *ws,
                int64_t *dev_bond_trace, int64_t *dev_mag_trace, hipStream_t hs, bool graphs)
{
    if (n_steps == 0)
        return ISING_OK;
    for (int32_t r = 0; r < b->n; ++r)
        if ((uint64_t)b->rep[r].t + n_steps > 0xffffffffull)
            return fail(ISING_E_INVALID, "step counter would reach 2^32");
    RecArgs rec{nullptr, nullptr, 0u, 0u};
    if (record_every > 0 && dev_bond_trace && dev_mag_trace && n_steps / record_every > 0) {
        rec.bond = dev_bond_trace;
        rec.mag = dev_mag_trace;
        rec.every = record_every;
        rec.n_rec = (uint32_t)(n_steps / record_every);
    }
    CL_HIP(launch_begin_run(b->d_rep, (uint32_t)b->n, b->d_rec, rec, hs));
    const bool recording = rec.every != 0;
    ClArgs a;
    a.reps = b->d_rep;
    a.cl = b->d_cl;
    a.tile_prefix = b->d_tile_prefix;
    a.n = (uint32_t)b->n;
    a.ws = ws;
    a.tb = reinterpret_cast<uint4 *>(a.ws + b->cl_tb_off);
    a.tiles = (uint32_t)b->cl_tiles;
    const uint64_t full = graphs ? n_steps / kClChunk : 0, rem = n_steps - full * kClChunk;
    if (full > 0) {
        hipGraphExec_t ex = nullptr;
        const int st = cluster_graph(b, a, algorithm, kClChunk, recording, &ex);
        if (st != ISING_OK)
            return st;
        for (uint64_t i = 0; i < full; ++i)
            CL_HIP(hipGraphLaunch(ex, hs));
        CL_HIP(hipEventRecord(b->ev_replay, hs));
        b->replay_pending = true;
    }
    for (uint64_t done = 0; done < rem;) {
        const uint32_t n = (uint32_t)std::min<uint64_t>(rem - done, 1u << 20);
        const int st = enqueue_cluster_chunk(b, a, algorithm, n, recording, hs);
        if (st != ISING_OK)
            return st;
        done += n;
    }
    for (int32_t r = 0; r < b->n; ++r)
        b->rep[r].t += (uint32_t)n_steps;
    return ISING_OK;
}

int check_cluster_args(ising_batch *b, int32_t algorithm)
{
    if (!b)
        return fail(ISING_E_INVALID, "NULL batch handle");
    if (algorithm != ISING_CLUSTER_SWENDSEN_WANG && algorithm != ISING_CLUSTER_WOLFF)
        return fail(ISING_E_INVALID, "unknown cluster algorithm");
    return ISING_OK;
}

}  // namespace

extern "C" {

int ising_batch_cluster(ising_batch *b, int32_t algorithm, uint64_t n_steps, uint32_t record_every, void *dev_ws,
                        size_t ws_bytes, int64_t *dev_bond_trace, int64_t *dev_mag_trace, void *stream)
{
    clear_error();
    int st = check_cluster_args(b, algorithm);
    if (st != ISING_OK)
        return st;
    if (!dev_ws)
        return fail(ISING_E_INVALID, "dev_ws must not be NULL");
    if ((reinterpret_cast<uintptr_t>(dev_ws) & 255) != 0)
        return fail(ISING_E_INVALID, "dev_ws must be 256-byte aligned");
    if (ws_bytes < b->cl_ws_bytes)
        return fail(ISING_E_NOMEM, "dev_ws is smaller than ising_cluster_ws_bytes()");
    return run_cluster(b, algorithm, n_steps, record_every, static_cast<char *>(dev_ws), dev_bond_trace,
                       dev_mag_trace, reinterpret_cast<hipStream_t>(stream), true);
}

int ising_batch_cluster_static(ising_batch *b, int32_t algorithm, uint64_t n_steps, uint32_t record_every,
                               int64_t *dev_bond_trace, int64_t *dev_mag_trace, void *stream)
{
    clear_error();
    int st = check_cluster_args(b, algorithm);
    if (st != ISING_OK)
        return st;
    if (b->cl_ws_bytes > kClStaticWsBytes)
        return fail(ISING_E_NOMEM, "the batch needs " + std::to_string(b->cl_ws_bytes) +
                                       " bytes of cluster workspace; the static workspace holds " +
                                       std::to_string(kClStaticWsBytes) + " (use ising_batch_cluster)");
    int cur = -1;
    CL_HIP(hipGetDevice(&cur));
    if (cur != b->device)
        return fail(ISING_E_INVALID, "the current device is not the batch's device");
    char *ws = nullptr;
    CL_HIP(static_cluster_ws(cur, &ws));
    return run_cluster(b, algorithm, n_steps, record_every, ws, dev_bond_trace, dev_mag_trace,
                       reinterpret_cast<hipStream_t>(stream), false);
}

}  // extern "C"
