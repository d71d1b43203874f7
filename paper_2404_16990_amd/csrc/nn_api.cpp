// Host runtime and C ABI of the learned block proposals: network state in the
// caller's device buffer, training steps, standalone scoring/sampling, block
// extraction and Metropolis-Hastings block rounds on a replica batch.  Every
// device computation is a kernel in nn.hip.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ising.h"
#include "batch.hpp"
#include "nn.hpp"
#include "nn_launch.hpp"

using namespace ising;
using namespace ising::nn;

#define NN_HIP(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(ISING_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct NNLayout {
    size_t params, adam_m, adam_v, grad, wt, wtd, step;
    size_t hb[3], db[3], logits, partial, wpart, loss;
    size_t sx, sbnd, scoup, skey, sblk, slogq;
    size_t total;
    int Pp;
};

int check_dims(int32_t block, int32_t channels, int32_t max_batch, int32_t max_seq)
{
    if (channels != C)
        return fail(ISING_E_UNSUPPORTED, "the network has 64 channels");
    if (block != 2 && block != 4 && block != 8)
        return fail(ISING_E_UNSUPPORTED, "block size must be 2, 4 or 8");
    if (max_batch < 1 || max_seq < 2)
        return fail(ISING_E_INVALID, "max_batch >= 1 and max_seq >= 2 required");
    if ((int64_t)max_batch * block * block > (1 << 24))
        return fail(ISING_E_UNSUPPORTED, "max_batch too large");
    return ISING_OK;
}

NNLayout make_nn_layout(int32_t block, int32_t max_batch, int32_t max_seq)
{
    NNLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    const int Pp = (max_batch * block * block + TILE - 1) / TILE * TILE;
    L.Pp = Pp;
    L.params = take(N_PARAMS * 4);
    L.adam_m = take(N_PARAMS * 4);
    L.adam_v = take(N_PARAMS * 4);
    L.grad = take(N_PARAMS * 4);
    L.wt = take((size_t)3 * C * KB * 2);
    L.wtd = take((size_t)3 * C * KB * 2);
    L.step = take(4);
    for (int l = 0; l < 3; ++l) {
        L.hb[l] = take((size_t)Pp * C * 2);
        L.db[l] = take((size_t)Pp * C * 2);
    }
    L.logits = take((size_t)Pp * 4);
    L.partial = take((size_t)(Pp / TILE) * PART_ROW * 4);
    L.wpart = take((size_t)3 * ((Pp + WGRAD_CHUNK - 1) / WGRAD_CHUNK) * KB * C * 4);
    L.loss = take(4);
    L.sx = take((size_t)max_seq * block * block);
    L.sbnd = take((size_t)max_seq * 4 * block);
    L.scoup = take((size_t)max_seq * 4);
    L.skey = take((size_t)max_seq * 16);
    L.sblk = take((size_t)max_seq * 4);
    L.slogq = take((size_t)max_seq * 8);
    L.total = off;
    return L;
}

}  // namespace

// A captured training step: everything its kernels take as arguments (the
// step number is read from the device counter).
struct TrainKey {
    bool sampled;
    const void *blocks, *bnd, *coupling;
    int64_t n_rows;
    int32_t batch;
    uint32_t lr_bits;
    uint64_t seed;
    float *loss;
    int32_t steps;  // training steps in one graph
    bool operator<(const TrainKey &o) const
    {
        return std::tie(sampled, blocks, bnd, coupling, n_rows, batch, lr_bits, seed, loss, steps) <
               std::tie(o.sampled, o.blocks, o.bnd, o.coupling, o.n_rows, o.batch, o.lr_bits, o.seed, o.loss,
                        o.steps);
    }
};

struct ising_nn {
    int32_t Bs = 0, max_batch = 0, max_seq = 0;
    char *buf = nullptr;
    NNLayout L{};
    NetDev net{};
    TrainWs ws{};
    SeqDev seq{};
    // captured training steps, replayed on the caller's stream; ev_replay is
    // recorded after each call's replay, and executable graphs are destroyed
    // only after it completed
    hipStream_t cap = nullptr;
    hipEvent_t ev_replay = nullptr;
    bool replay_pending = false;
    std::map<TrainKey, hipGraphExec_t> graphs;
    int64_t captures = 0;
};

namespace {

int check_nn(ising_nn *m)
{
    if (!m)
        return fail(ISING_E_INVALID, "null network handle");
    return ISING_OK;
}

int upload_params(ising_nn *m, const float *host, hipStream_t st)
{
    NN_HIP(hipMemcpyAsync(m->net.params, host, N_PARAMS * sizeof(float), hipMemcpyHostToDevice, st));
    NN_HIP(hipMemsetAsync(m->net.adam_m, 0, N_PARAMS * sizeof(float), st));
    NN_HIP(hipMemsetAsync(m->net.adam_v, 0, N_PARAMS * sizeof(float), st));
    NN_HIP(hipMemsetAsync(m->net.step, 0, sizeof(uint32_t), st));
    NN_HIP(cast_weights(m->net, st));
    NN_HIP(hipStreamSynchronize(st));
    return ISING_OK;
}

int wait_replays(ising_nn *m)
{
    if (m->replay_pending) {
        NN_HIP(hipEventSynchronize(m->ev_replay));
        m->replay_pending = false;
    }
    return ISING_OK;
}

void drop_graphs(ising_nn *m)
{
    (void)wait_replays(m);
    for (auto &kv : m->graphs)
        (void)hipGraphExecDestroy(kv.second);
    m->graphs.clear();
}

// k.steps training steps enqueued on st, each the fused forward and backward
// of every tile (drawing its minibatch rows if sampled), the weight-gradient
// products (which count the step on the device), and the gradient reduction
// with the Adam update, the BF16 weight copies and the loss.
int enqueue_train(ising_nn *m, const TrainKey &k, float lr, hipStream_t st)
{
    const int8_t *x = static_cast<const int8_t *>(k.blocks), *bnd = static_cast<const int8_t *>(k.bnd);
    const float *kc = static_cast<const float *>(k.coupling);
    for (int32_t i = 0; i < k.steps; ++i) {
        NN_HIP(train_tiles(m->net, m->ws, x, bnd, kc, k.batch, m->Bs, k.sampled, (uint32_t)k.n_rows, k.seed, true,
                           st));
        NN_HIP(finish_step(m->net, m->ws, k.batch, m->Bs, true, lr, k.loss, st));
    }
    return ISING_OK;
}

// Replay the captured steps for these arguments `replays` times (capturing
// them on first use).
int train(ising_nn *m, const TrainKey &k, float lr, hipStream_t st, int64_t replays = 1)
{
    auto it = m->graphs.find(k);
    hipGraphExec_t ex = nullptr;
    if (it != m->graphs.end()) {
        ex = it->second;
    } else {
        if (m->graphs.size() >= 8)
            drop_graphs(m);
        NN_HIP(hipStreamBeginCapture(m->cap, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_train(m, k, lr, m->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(m->cap, &g);
        if (rc != ISING_OK) {
            if (g)
                (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess)
            return fail(ISING_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess)
            return fail(ISING_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
        m->graphs[k] = ex;
        m->captures += 1;
    }
    for (int64_t i = 0; i < replays; ++i)
        NN_HIP(hipGraphLaunch(ex, st));
    NN_HIP(hipEventRecord(m->ev_replay, st));
    m->replay_pending = true;
    return ISING_OK;
}

// replicas of one shape with Lx, Ly multiples of 2*Bs; blocks of one colour per replica
int uniform_blocks(ising_batch *b, int Bs, uint32_t *per_rep)
{
    const int32_t Lx = b->desc[0].Lx, Ly = b->desc[0].Ly;
    for (int32_t r = 1; r < b->n; ++r)
        if (b->desc[r].Lx != Lx || b->desc[r].Ly != Ly)
            return fail(ISING_E_UNSUPPORTED, "block moves need every replica of the batch to have one shape");
    if (Lx % (2 * Bs) != 0 || Ly % (2 * Bs) != 0)
        return fail(ISING_E_UNSUPPORTED, "Lx and Ly must be multiples of twice the block size");
    *per_rep = (uint32_t)((Lx / Bs) * (Ly / Bs) / 2);
    return ISING_OK;
}

}  // namespace

extern "C" {

int ising_nn_param_count(int32_t channels, int32_t *count)
{
    clear_error();
    if (!count)
        return fail(ISING_E_INVALID, "count must not be NULL");
    if (channels != C)
        return fail(ISING_E_UNSUPPORTED, "the network has 64 channels");
    *count = N_PARAMS;
    return ISING_OK;
}

int ising_nn_state_bytes(int32_t block, int32_t channels, int32_t max_batch, int32_t max_seq, size_t *bytes)
{
    clear_error();
    if (!bytes)
        return fail(ISING_E_INVALID, "bytes must not be NULL");
    int st = check_dims(block, channels, max_batch, max_seq);
    if (st != ISING_OK)
        return st;
    *bytes = make_nn_layout(block, max_batch, max_seq).total;
    return ISING_OK;
}

int ising_nn_create(int32_t block, int32_t channels, int32_t max_batch, int32_t max_seq, const float *host_params,
                    void *dev_buf, size_t bytes, void *stream, ising_nn **out)
{
    clear_error();
    if (!out)
        return fail(ISING_E_INVALID, "out must not be NULL");
    *out = nullptr;
    int st = check_dims(block, channels, max_batch, max_seq);
    if (st != ISING_OK)
        return st;
    if (!host_params || !dev_buf)
        return fail(ISING_E_INVALID, "parameters and device buffer must not be NULL");
    if ((reinterpret_cast<uintptr_t>(dev_buf) & 255) != 0)
        return fail(ISING_E_INVALID, "dev_buf must be 256-byte aligned");
    const NNLayout L = make_nn_layout(block, max_batch, max_seq);
    if (bytes < L.total)
        return fail(ISING_E_NOMEM, "dev_buf is smaller than ising_nn_state_bytes()");
    ising_nn *m = new (std::nothrow) ising_nn();
    if (!m)
        return fail(ISING_E_NOMEM, "host allocation failed");
    m->Bs = block;
    m->max_batch = max_batch;
    m->max_seq = max_seq;
    m->buf = static_cast<char *>(dev_buf);
    m->L = L;
    char *B = m->buf;
    m->net.params = reinterpret_cast<float *>(B + L.params);
    m->net.adam_m = reinterpret_cast<float *>(B + L.adam_m);
    m->net.adam_v = reinterpret_cast<float *>(B + L.adam_v);
    m->net.grad = reinterpret_cast<float *>(B + L.grad);
    m->net.wt = reinterpret_cast<uint16_t *>(B + L.wt);
    m->net.wtd = reinterpret_cast<uint16_t *>(B + L.wtd);
    m->net.step = reinterpret_cast<uint32_t *>(B + L.step);
    for (int l = 0; l < 3; ++l) {
        m->ws.hb[l] = reinterpret_cast<uint16_t *>(B + L.hb[l]);
        m->ws.db[l] = reinterpret_cast<uint16_t *>(B + L.db[l]);
    }
    m->ws.logits = reinterpret_cast<float *>(B + L.logits);
    m->ws.partial = reinterpret_cast<float *>(B + L.partial);
    m->ws.wpart = reinterpret_cast<float *>(B + L.wpart);
    m->ws.loss = reinterpret_cast<float *>(B + L.loss);
    m->seq.x = reinterpret_cast<int8_t *>(B + L.sx);
    m->seq.bnd = reinterpret_cast<int8_t *>(B + L.sbnd);
    m->seq.coupling = reinterpret_cast<float *>(B + L.scoup);
    m->seq.key = reinterpret_cast<uint32_t *>(B + L.skey);
    m->seq.blk = reinterpret_cast<uint32_t *>(B + L.sblk);
    m->seq.logq = reinterpret_cast<double *>(B + L.slogq);
    st = upload_params(m, host_params, reinterpret_cast<hipStream_t>(stream));
    if (st == ISING_OK) {
        const hipError_t e1 = hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking);
        const hipError_t e2 = e1 == hipSuccess ? hipEventCreateWithFlags(&m->ev_replay, hipEventDisableTiming) : e1;
        if (e2 != hipSuccess)
            st = fail(ISING_E_HIP, std::string("stream/event creation: ") + hipGetErrorString(e2));
    }
    if (st != ISING_OK) {
        if (m->cap)
            (void)hipStreamDestroy(m->cap);
        delete m;
        return st;
    }
    *out = m;
    return ISING_OK;
}

int ising_nn_get_params(ising_nn *m, float *host_params, void *stream)
{
    clear_error();
    int st = check_nn(m);
    if (st != ISING_OK)
        return st;
    if (!host_params)
        return fail(ISING_E_INVALID, "host_params must not be NULL");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    NN_HIP(hipMemcpyAsync(host_params, m->net.params, N_PARAMS * sizeof(float), hipMemcpyDeviceToHost, hs));
    NN_HIP(hipStreamSynchronize(hs));
    return ISING_OK;
}

int ising_nn_set_params(ising_nn *m, const float *host_params, void *stream)
{
    clear_error();
    int st = check_nn(m);
    if (st != ISING_OK)
        return st;
    if (!host_params)
        return fail(ISING_E_INVALID, "host_params must not be NULL");
    return upload_params(m, host_params, reinterpret_cast<hipStream_t>(stream));
}

int ising_nn_graph_stats(ising_nn *m, int32_t *n_cached, int64_t *n_captured)
{
    clear_error();
    int st = check_nn(m);
    if (st != ISING_OK)
        return st;
    if (n_cached)
        *n_cached = (int32_t)m->graphs.size();
    if (n_captured)
        *n_captured = m->captures;
    return ISING_OK;
}

int ising_nn_forward_backward(ising_nn *m, const int8_t *dev_blocks, const int8_t *dev_bnd,
                              const float *dev_coupling, int32_t batch, float *dev_logits, float *dev_grad,
                              float *dev_loss, void *stream)
{
    clear_error();
    int st = check_nn(m);
    if (st != ISING_OK)
        return st;
    if (batch < 1 || batch > m->max_batch)
        return fail(ISING_E_INVALID, "batch must be in [1, max_batch]");
    if (!dev_blocks || !dev_bnd || !dev_coupling)
        return fail(ISING_E_INVALID, "block arrays must not be NULL");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    NN_HIP(train_tiles(m->net, m->ws, dev_blocks, dev_bnd, dev_coupling, batch, m->Bs, false, 0u, 0u, false, hs));
    NN_HIP(finish_step(m->net, m->ws, batch, m->Bs, false, 0.f, nullptr, hs));
    const size_t P = (size_t)batch * m->Bs * m->Bs;
    if (dev_logits)
        NN_HIP(hipMemcpyAsync(dev_logits, m->ws.logits, P * 4, hipMemcpyDeviceToDevice, hs));
    if (dev_grad)
        NN_HIP(hipMemcpyAsync(dev_grad, m->net.grad, N_PARAMS * 4, hipMemcpyDeviceToDevice, hs));
    if (dev_loss)
        NN_HIP(hipMemcpyAsync(dev_loss, m->ws.loss, 4, hipMemcpyDeviceToDevice, hs));
    return ISING_OK;
}

int ising_nn_train_step(ising_nn *m, const int8_t *dev_blocks, const int8_t *dev_bnd, const float *dev_coupling,
                        int32_t batch, float lr, float *dev_loss, void *stream)
{
    clear_error();
    int st = check_nn(m);
    if (st != ISING_OK)
        return st;
    if (batch < 1 || batch > m->max_batch)
        return fail(ISING_E_INVALID, "batch must be in [1, max_batch]");
    if (!dev_blocks || !dev_bnd || !dev_coupling)
        return fail(ISING_E_INVALID, "block arrays must not be NULL");
    if (!(lr > 0.0f))
        return fail(ISING_E_INVALID, "lr must be > 0");
    uint32_t lr_bits;
    std::memcpy(&lr_bits, &lr, 4);
    const TrainKey k{false, dev_blocks, dev_bnd, dev_coupling, 0, batch, lr_bits, 0, dev_loss, 1};
    return train(m, k, lr, reinterpret_cast<hipStream_t>(stream));
}

int ising_nn_train_step_sampled(ising_nn *m, const int8_t *dev_blocks, const int8_t *dev_bnd,
                                const float *dev_coupling, int64_t n_rows, int32_t batch, float lr, uint64_t seed,
                                float *dev_loss, void *stream)
{
    return ising_nn_train_steps_sampled(m, dev_blocks, dev_bnd, dev_coupling, n_rows, batch, lr, seed, 1, dev_loss,
                                        stream);
}

int ising_nn_train_steps_sampled(ising_nn *m, const int8_t *dev_blocks, const int8_t *dev_bnd,
                                 const float *dev_coupling, int64_t n_rows, int32_t batch, float lr, uint64_t seed,
                                 int64_t n_steps, float *dev_loss, void *stream)
{
    clear_error();
    int st = check_nn(m);
    if (st != ISING_OK)
        return st;
    if (batch < 1 || batch > m->max_batch)
        return fail(ISING_E_INVALID, "batch must be in [1, max_batch]");
    if (n_rows < 1 || n_rows > (int64_t)UINT32_MAX)
        return fail(ISING_E_INVALID, "n_rows must be in [1, 2^32 - 1]");
    if (!dev_blocks || !dev_bnd || !dev_coupling)
        return fail(ISING_E_INVALID, "block arrays must not be NULL");
    if (!(lr > 0.0f))
        return fail(ISING_E_INVALID, "lr must be > 0");
    uint32_t lr_bits;
    std::memcpy(&lr_bits, &lr, 4);
    if (n_steps < 1)
        return fail(ISING_E_INVALID, "n_steps must be >= 1");
    // graphs of up to 16 steps: back-to-back steps without a launch between them
    constexpr int32_t G = 16;
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const int64_t full = n_steps / G;
    const int32_t rest = (int32_t)(n_steps % G);
    if (full > 0) {
        const TrainKey k{true, dev_blocks, dev_bnd, dev_coupling, n_rows, batch, lr_bits, seed, dev_loss, G};
        st = train(m, k, lr, hs, full);
        if (st != ISING_OK)
            return st;
    }
    if (rest > 0) {
        const TrainKey k{true, dev_blocks, dev_bnd, dev_coupling, n_rows, batch, lr_bits, seed, dev_loss, rest};
        return train(m, k, lr, hs);
    }
    return ISING_OK;
}

int ising_nn_score(ising_nn *m, int32_t n, const int8_t *dev_blocks, const int8_t *dev_bnd,
                   const float *dev_coupling, double *dev_logq, void *stream)
{
    clear_error();
    int st = check_nn(m);
    if (st != ISING_OK)
        return st;
    if (n < 1 || n > m->max_seq)
        return fail(ISING_E_INVALID, "n must be in [1, max_seq]");
    if (!dev_blocks || !dev_bnd || !dev_coupling || !dev_logq)
        return fail(ISING_E_INVALID, "arrays must not be NULL");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const int BB = m->Bs * m->Bs;
    NN_HIP(hipMemcpyAsync(m->seq.x, dev_blocks, (size_t)n * BB, hipMemcpyDeviceToDevice, hs));
    NN_HIP(hipMemcpyAsync(m->seq.bnd, dev_bnd, (size_t)n * 4 * m->Bs, hipMemcpyDeviceToDevice, hs));
    NN_HIP(hipMemcpyAsync(m->seq.coupling, dev_coupling, (size_t)n * 4, hipMemcpyDeviceToDevice, hs));
    NN_HIP(ar_pass(m->net, m->seq, n, 0, m->Bs, hs));
    NN_HIP(hipMemcpyAsync(dev_logq, m->seq.logq, (size_t)n * 8, hipMemcpyDeviceToDevice, hs));
    return ISING_OK;
}

int ising_nn_sample(ising_nn *m, int32_t n, const int8_t *dev_bnd, const float *dev_coupling, uint64_t seed,
                    uint32_t replica, uint32_t round, uint32_t blk0, int8_t *dev_blocks_out, double *dev_logq,
                    void *stream)
{
    clear_error();
    int st = check_nn(m);
    if (st != ISING_OK)
        return st;
    if (n < 1 || n > m->max_seq)
        return fail(ISING_E_INVALID, "n must be in [1, max_seq]");
    if (!dev_bnd || !dev_coupling || !dev_blocks_out || !dev_logq)
        return fail(ISING_E_INVALID, "arrays must not be NULL");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const int BB = m->Bs * m->Bs;
    NN_HIP(hipMemcpyAsync(m->seq.bnd, dev_bnd, (size_t)n * 4 * m->Bs, hipMemcpyDeviceToDevice, hs));
    NN_HIP(hipMemcpyAsync(m->seq.coupling, dev_coupling, (size_t)n * 4, hipMemcpyDeviceToDevice, hs));
    NN_HIP(seq_setup(m->seq, n, seed, replica, round, blk0, hs));
    NN_HIP(ar_pass(m->net, m->seq, 0, n, m->Bs, hs));
    NN_HIP(hipMemcpyAsync(dev_blocks_out, m->seq.x, (size_t)n * BB, hipMemcpyDeviceToDevice, hs));
    NN_HIP(hipMemcpyAsync(dev_logq, m->seq.logq, (size_t)n * 8, hipMemcpyDeviceToDevice, hs));
    return ISING_OK;
}

int ising_batch_extract_blocks(ising_batch *b, int32_t block, int32_t per_replica, uint32_t draw, int8_t *dev_blocks,
                               int8_t *dev_bnd, float *dev_coupling, void *stream)
{
    clear_error();
    if (!b)
        return fail(ISING_E_INVALID, "null batch handle");
    if (block != 2 && block != 4 && block != 8)
        return fail(ISING_E_UNSUPPORTED, "block size must be 2, 4 or 8");
    if (per_replica < 1)
        return fail(ISING_E_INVALID, "per_replica must be >= 1");
    if (!dev_blocks || !dev_bnd || !dev_coupling)
        return fail(ISING_E_INVALID, "output arrays must not be NULL");
    uint32_t per_rep_blocks = 0;
    int st = uniform_blocks(b, block, &per_rep_blocks);
    if (st != ISING_OK)
        return st;
    const uint64_t count = (uint64_t)b->n * (uint64_t)per_replica;
    if (count > (1u << 30))
        return fail(ISING_E_INVALID, "too many samples");
    NN_HIP(extract(b->d_rep, b->d_kcoup, block, (uint32_t)per_replica, (uint32_t)count, draw, dev_blocks, dev_bnd,
                   dev_coupling, reinterpret_cast<hipStream_t>(stream)));
    return ISING_OK;
}

int ising_batch_block_round(ising_batch *b, ising_nn *m, uint32_t round, int64_t *dev_accepts, void *stream)
{
    clear_error();
    if (!b)
        return fail(ISING_E_INVALID, "null batch handle");
    int st = check_nn(m);
    if (st != ISING_OK)
        return st;
    uint32_t per_rep = 0;
    st = uniform_blocks(b, m->Bs, &per_rep);
    if (st != ISING_OK)
        return st;
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    int64_t *acc = dev_accepts ? dev_accepts : b->d_obs;  // scratch counters when the caller wants none
    const uint32_t total = (uint32_t)b->n * per_rep;
    const uint32_t chunk = (uint32_t)(m->max_seq / 2);
    for (uint32_t colour = 0; colour < 2; ++colour)
        for (uint32_t first = 0; first < total; first += chunk) {
            const uint32_t count = std::min(chunk, total - first);
            NN_HIP(block_round_pass(m->net, m->seq, b->d_rep, b->d_kcoup, m->Bs, colour, round, first, count,
                                    per_rep, acc, hs));
        }
    return ISING_OK;
}

int ising_nn_destroy(ising_nn *m)
{
    if (m) {
        drop_graphs(m);
        if (m->ev_replay)
            (void)hipEventDestroy(m->ev_replay);
        if (m->cap)
            (void)hipStreamDestroy(m->cap);
    }
    delete m;
    return ISING_OK;
}

}  // extern "C"
