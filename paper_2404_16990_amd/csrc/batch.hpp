// Internal definition of a replica batch, shared by the sweep runtime
// (api.cpp) and the block-proposal runtime (nn_api.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ising.h"
#include "cluster.hpp"
#include "device.hpp"
#include "launch.hpp"

namespace ising {

struct Layout {
    size_t reps = 0, lists = 0, obs = 0, rec = 0, modes = 0, kcoup = 0, cl = 0, clprefix = 0;
    std::vector<size_t> planes;
    size_t total = 0;
};

// A captured chunk of cluster steps.  The trace pointers and cadence are not
// part of the key (the kernels read them from the batch's device slot); only
// whether the chunk contains recording kernels at all.
struct ClGraphKey {
    int32_t algorithm;
    uint32_t steps;
    char *ws;
    bool recording;
    bool operator<(const ClGraphKey &o) const
    {
        return std::tie(algorithm, steps, ws, recording) < std::tie(o.algorithm, o.steps, o.ws, o.recording);
    }
};


// Record a failure for ising_last_error() and return its code.
int fail(int code, const std::string &msg);
// Clear the calling thread's error detail (at the start of every ABI call).
void clear_error();
// floor(p 2^32) clamped to 2^32 - 1: the integer threshold of a probability.
uint32_t prob_threshold(double p);
// Cluster-step descriptors of a new batch (cluster_api.cpp): filled on the host
// and uploaded on st (the caller synchronises).
int cluster_setup(ising_batch *b, hipStream_t st);
// Bond threshold of replica r after its beta changed (upload on st).
int cluster_set_beta(ising_batch *b, int32_t r, hipStream_t st);
// Destroy the batch's captured cluster-step chunks (after the last replay
// enqueued on the batch's streams has finished).
void drop_cluster_graphs(ising_batch *b);
// Wait until every graph replay enqueued so far has finished (no-op when
// none was launched since the last wait).
int wait_graph_replays(ising_batch *b);

}  // namespace ising

struct ising_batch {
    int32_t n = 0;
    std::vector<ising_desc> desc;
    std::vector<ising::RepDev> rep;  // host mirror; t advanced when work is enqueued
    char *buf = nullptr;
    size_t bytes = 0;
    ising::Layout layout;
    ising::RepDev *d_rep = nullptr;
    double *d_kcoup = nullptr;  // K = beta*J per replica (device)
    uint32_t *d_lists = nullptr;
    int64_t *d_obs = nullptr;
    ising::RecArgs *d_rec = nullptr;  // recording arguments of the run being enqueued
    int device = 0;
    int lds_max = 0;        // LDS per workgroup the device allows (bytes)
    ising_schedule sched{};
    // derived schedule
    ising::ResidentList res[2]{};  // [0] 32-bit words, [1] 64-bit words
    ising::StreamList str[2]{};
    uint32_t max_words = 0;
    hipStream_t aux = nullptr, cap = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // Captured sweep chunks by sweep count.  ev_replay is recorded after each
    // call's replays; executable graphs are destroyed only after it completed.
    std::map<uint32_t, hipGraphExec_t> graphs;
    hipEvent_t ev_replay = nullptr;
    bool replay_pending = false;
    int64_t n_captures = 0;            // sweep and cluster chunks captured so far
    // cluster steps
    std::vector<ising::ClRep> cl;      // host mirror of the cluster descriptors
    std::vector<uint32_t> tile_prefix; // host mirror of the tile prefix (n + 1 entries)
    ising::ClRep *d_cl = nullptr;
    uint32_t *d_tile_prefix = nullptr;
    uint64_t cl_tiles = 0;             // tiles of the whole batch
    size_t cl_tb_off = 0;              // workspace offset of the crossing-bond masks
    size_t cl_ws_bytes = 0;            // workspace a cluster step needs
    std::map<ising::ClGraphKey, hipGraphExec_t> cl_graphs;
};

