// Host runtime and C ABI of the 3D sweeps: validation, thresholds, device
// descriptors and layout, the sweep loop, spin copies.  Every device
// computation is a kernel in ising3d.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ising.h"
#include "../../include/ising3d.h"
#include "batch.hpp"
#include "ising3d.hpp"

using namespace ising;

struct ising3d_batch {
    int32_t n = 0;
    std::vector<ising3d_desc> desc;
    std::vector<Rep3Dev> rep;        // host mirror; t advanced when work is enqueued
    std::vector<uint32_t> prefix;    // workgroup prefix over replicas (n + 1)
    char *buf = nullptr;
    Rep3Dev *d_rep = nullptr;
    uint32_t *d_prefix = nullptr;
    int64_t *d_obs = nullptr;
    uint32_t blocks = 0;
    uint32_t widths = 0;  // bit k: some replica's sweep groups are 2^k words
};

#define H3_HIP(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(ISING_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

namespace {

constexpr int32_t kMaxReplicas3 = 65535;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int check3(const ising3d_desc &d, int32_t i)
{
    const std::string at = " (replica index " + std::to_string(i) + ")";
    if (!(d.J > 0.0) || std::isinf(d.J))
        return fail(ISING_E_INVALID, "J must be finite and > 0" + at);
    if (std::isnan(d.beta) || d.beta < 0.0)
        return fail(ISING_E_INVALID, "beta must be >= 0 (or +inf)" + at);
    if (d.init != ISING_INIT_RANDOM && d.init != ISING_INIT_UP && d.init != ISING_INIT_DOWN)
        return fail(ISING_E_INVALID, "unknown init mode" + at);
    if (d.rng != ISING_RNG_SITE && d.rng != ISING_RNG_BITSLICED)
        return fail(ISING_E_INVALID, "unknown random-number contract (rng)" + at);
    if (d.Lx <= 0 || d.Lx % 64 != 0)
        return fail(ISING_E_UNSUPPORTED, "Lx must be a positive multiple of 64" + at);
    if (d.Ly < 2 || d.Ly % 2 != 0 || d.Lz < 2 || d.Lz % 2 != 0)
        return fail(ISING_E_UNSUPPORTED, "Ly and Lz must be even and >= 2" + at);
    if ((uint64_t)d.Lx * (uint64_t)d.Ly * (uint64_t)d.Lz >= (1ull << 32))
        return fail(ISING_E_UNSUPPORTED, "Lx*Ly*Lz must be below 2^32" + at);
    return ISING_OK;
}

size_t words3(const ising3d_desc &d) { return (size_t)d.Lz * d.Ly * (d.Lx / 64); }

// Device buffer: [descriptors | workgroup prefix | observable scratch | init modes | planes...]
struct Layout3 {
    size_t reps, prefix, obs, modes, total;
    std::vector<size_t> planes;
};

int layout3(int32_t n, const ising3d_desc *d, Layout3 *L)
{
    if (n <= 0 || !d)
        return fail(ISING_E_INVALID, "need n > 0 replicas and a descriptor array");
    if (n > kMaxReplicas3)
        return fail(ISING_E_UNSUPPORTED, "at most 65535 replicas per batch");
    for (int32_t i = 0; i < n; ++i) {
        const int st = check3(d[i], i);
        if (st != ISING_OK)
            return st;
    }
    size_t off = 0;
    L->reps = off;
    off += align256((size_t)n * sizeof(Rep3Dev));
    L->prefix = off;
    off += align256((size_t)(n + 1) * sizeof(uint32_t));
    L->obs = off;
    off += align256((size_t)2 * n * sizeof(int64_t));
    L->modes = off;
    off += align256((size_t)n * sizeof(int32_t));
    L->planes.resize(n);
    for (int32_t i = 0; i < n; ++i) {
        L->planes[i] = off;
        off += align256(2 * words3(d[i]) * sizeof(uint32_t));
    }
    L->total = off;
    return ISING_OK;
}

Sweep3Args args_of(const ising3d_batch *b)
{
    Sweep3Args a;
    a.reps = b->d_rep;
    a.prefix = b->d_prefix;
    a.n = (uint32_t)b->n;
    a.blocks = b->blocks;
    a.widths = b->widths;
    return a;
}

int check_replica3(ising3d_batch *b, int32_t r)
{
    if (!b)
        return fail(ISING_E_INVALID, "NULL batch handle");
    if (r < 0 || r >= b->n)
        return fail(ISING_E_INVALID, "replica index out of range");
    return ISING_OK;
}

}  // namespace

extern "C" {

int ising3d_state_bytes(int32_t n, const ising3d_desc *d, size_t *bytes)
{
    clear_error();
    if (!bytes)
        return fail(ISING_E_INVALID, "bytes must not be NULL");
    Layout3 L;
    const int st = layout3(n, d, &L);
    if (st != ISING_OK)
        return st;
    *bytes = L.total;
    return ISING_OK;
}

int ising3d_batch_create(int32_t n, const ising3d_desc *d, void *dev_buf, size_t bytes, void *stream,
                         ising3d_batch **out)
{
    clear_error();
    if (!out)
        return fail(ISING_E_INVALID, "out must not be NULL");
    *out = nullptr;
    Layout3 L;
    int st = layout3(n, d, &L);
    if (st != ISING_OK)
        return st;
    if (!dev_buf)
        return fail(ISING_E_INVALID, "dev_buf must not be NULL");
    if ((reinterpret_cast<uintptr_t>(dev_buf) & 255) != 0)
        return fail(ISING_E_INVALID, "dev_buf must be 256-byte aligned");
    if (bytes < L.total)
        return fail(ISING_E_NOMEM, "dev_buf is smaller than ising3d_state_bytes()");
    ising3d_batch *b = new (std::nothrow) ising3d_batch();
    if (!b)
        return fail(ISING_E_NOMEM, "host allocation failed");
    b->n = n;
    b->desc.assign(d, d + n);
    b->buf = static_cast<char *>(dev_buf);
    b->d_rep = reinterpret_cast<Rep3Dev *>(b->buf + L.reps);
    b->d_prefix = reinterpret_cast<uint32_t *>(b->buf + L.prefix);
    b->d_obs = reinterpret_cast<int64_t *>(b->buf + L.obs);
    b->rep.resize(n);
    b->prefix.assign(n + 1, 0u);
    std::vector<int32_t> modes(n);
    uint64_t blocks = 0;
    for (int32_t i = 0; i < n; ++i) {
        Rep3Dev &r = b->rep[i];
        std::memset(&r, 0, sizeof(r));
        r.plane0 = reinterpret_cast<uint32_t *>(b->buf + L.planes[i]);
        r.Lx = (uint32_t)d[i].Lx;
        r.Ly = (uint32_t)d[i].Ly;
        r.Lz = (uint32_t)d[i].Lz;
        r.W = r.Lx / 64u;
        r.seed_lo = (uint32_t)(d[i].seed & 0xffffffffu);
        r.seed_hi = (uint32_t)(d[i].seed >> 32);
        r.replica = d[i].replica;
        const double K = d[i].beta * d[i].J;
        r.flags = (K == 0.0 ? k3Always : 0u) | (d[i].rng == ISING_RNG_BITSLICED ? k3Bitsliced : 0u);
        r.thr4 = prob_threshold(std::exp(-4.0 * K));
        r.thr8 = prob_threshold(std::exp(-8.0 * K));
        r.thr12 = prob_threshold(std::exp(-12.0 * K));
        r.N = (uint64_t)r.Lx * r.Ly * r.Lz;
        modes[i] = d[i].init;
        b->prefix[i] = (uint32_t)blocks;
        blocks += (words3(d[i]) + k3WordsPerBlock - 1) / k3WordsPerBlock;
        b->widths |= group_width(r.W);
    }
    if (blocks >= (1ull << 31)) {
        delete b;
        return fail(ISING_E_UNSUPPORTED, "batch too large for one launch");
    }
    b->prefix[n] = (uint32_t)blocks;
    b->blocks = (uint32_t)blocks;
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    auto cleanup = [&](int code) {
        delete b;
        return code;
    };
    hipError_t e;
#define C3_HIP(expr)                                                                            \
    do {                                                                                        \
        e = (expr);                                                                             \
        if (e != hipSuccess)                                                                    \
            return cleanup(fail(ISING_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e))); \
    } while (0)
    int32_t *d_modes = reinterpret_cast<int32_t *>(b->buf + L.modes);
    C3_HIP(hipMemcpyAsync(b->d_rep, b->rep.data(), (size_t)n * sizeof(Rep3Dev), hipMemcpyHostToDevice, hs));
    C3_HIP(hipMemcpyAsync(b->d_prefix, b->prefix.data(), (size_t)(n + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, hs));
    C3_HIP(hipMemcpyAsync(d_modes, modes.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, hs));
    C3_HIP(launch3_init(args_of(b), d_modes, hs));
    C3_HIP(hipStreamSynchronize(hs));
#undef C3_HIP
    *out = b;
    return ISING_OK;
}

int ising3d_batch_run(ising3d_batch *b, uint64_t n_sweeps, uint32_t record_every, int64_t *dev_bond_trace,
                      int64_t *dev_mag_trace, void *stream)
{
    clear_error();
    if (!b)
        return fail(ISING_E_INVALID, "NULL batch handle");
    if (n_sweeps == 0)
        return ISING_OK;
    for (int32_t r = 0; r < b->n; ++r)
        if ((uint64_t)b->rep[r].t + n_sweeps > 0xffffffffull)
            return fail(ISING_E_INVALID, "sweep counter would reach 2^32");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    uint32_t n_rec = 0;
    if (record_every > 0 && dev_bond_trace && dev_mag_trace && n_sweeps / record_every > 0) {
        n_rec = (uint32_t)(n_sweeps / record_every);
        H3_HIP(launch_fill_i64(dev_bond_trace, (uint64_t)b->n * n_rec, 0, hs));
        H3_HIP(launch_fill_i64(dev_mag_trace, (uint64_t)b->n * n_rec, 0, hs));
    }
    const Sweep3Args a = args_of(b);
    for (uint64_t i = 0; i < n_sweeps; ++i) {
        H3_HIP(launch3_sweep(a, 0u, (uint32_t)i, hs));
        H3_HIP(launch3_sweep(a, 1u, (uint32_t)i, hs));
        if (n_rec && (i + 1) % record_every == 0) {
            const uint64_t j = (i + 1) / record_every - 1;
            H3_HIP(launch3_observables(a, dev_bond_trace + j, dev_mag_trace + j, n_rec, hs));
        }
    }
    H3_HIP(launch3_advance(b->d_rep, (uint32_t)b->n, (uint32_t)n_sweeps, hs));
    for (int32_t r = 0; r < b->n; ++r)
        b->rep[r].t += (uint32_t)n_sweeps;
    return ISING_OK;
}

int ising3d_batch_observables(ising3d_batch *b, int64_t *host_bond, int64_t *host_mag, void *stream)
{
    clear_error();
    if (!b)
        return fail(ISING_E_INVALID, "NULL batch handle");
    if (!host_bond || !host_mag)
        return fail(ISING_E_INVALID, "output arrays must not be NULL");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    H3_HIP(launch_fill_i64(b->d_obs, 2 * (uint64_t)b->n, 0, hs));
    H3_HIP(launch3_observables(args_of(b), b->d_obs, b->d_obs + b->n, 1u, hs));
    H3_HIP(hipMemcpyAsync(host_bond, b->d_obs, (size_t)b->n * sizeof(int64_t), hipMemcpyDeviceToHost, hs));
    H3_HIP(hipMemcpyAsync(host_mag, b->d_obs + b->n, (size_t)b->n * sizeof(int64_t), hipMemcpyDeviceToHost, hs));
    H3_HIP(hipStreamSynchronize(hs));
    return ISING_OK;
}

int ising3d_batch_get_spins(ising3d_batch *b, int32_t r, int8_t *host_pm1, void *stream)
{
    clear_error();
    int st = check_replica3(b, r);
    if (st != ISING_OK)
        return st;
    if (!host_pm1)
        return fail(ISING_E_INVALID, "host_pm1 must not be NULL");
    const Rep3Dev &d = b->rep[r];
    const size_t words = (size_t)d.Lz * d.Ly * d.W;
    std::vector<uint32_t> planes(2 * words);
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    H3_HIP(hipMemcpyAsync(planes.data(), d.plane0, planes.size() * 4, hipMemcpyDeviceToHost, hs));
    H3_HIP(hipStreamSynchronize(hs));
    for (uint32_t z = 0; z < d.Lz; ++z)
        for (uint32_t y = 0; y < d.Ly; ++y) {
            const size_t row = (size_t)z * d.Ly + y;
            for (uint32_t x = 0; x < d.Lx; ++x) {
                const uint32_t c = (x + y + z) & 1u, k = x >> 1;
                const uint32_t word = planes[c * words + row * d.W + (k >> 5)];
                host_pm1[row * d.Lx + x] = ((word >> (k & 31)) & 1u) ? 1 : -1;
            }
        }
    return ISING_OK;
}

int ising3d_batch_set_spins(ising3d_batch *b, int32_t r, const int8_t *host_pm1, void *stream)
{
    clear_error();
    int st = check_replica3(b, r);
    if (st != ISING_OK)
        return st;
    if (!host_pm1)
        return fail(ISING_E_INVALID, "host_pm1 must not be NULL");
    const Rep3Dev &d = b->rep[r];
    const size_t words = (size_t)d.Lz * d.Ly * d.W;
    std::vector<uint32_t> planes(2 * words, 0u);
    for (uint32_t z = 0; z < d.Lz; ++z)
        for (uint32_t y = 0; y < d.Ly; ++y) {
            const size_t row = (size_t)z * d.Ly + y;
            for (uint32_t x = 0; x < d.Lx; ++x) {
                const int8_t v = host_pm1[row * d.Lx + x];
                if (v != 1 && v != -1)
                    return fail(ISING_E_INVALID, "spins must be +1 or -1");
                if (v == 1) {
                    const uint32_t c = (x + y + z) & 1u, k = x >> 1;
                    planes[c * words + row * d.W + (k >> 5)] |= 1u << (k & 31);
                }
            }
        }
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    H3_HIP(hipMemcpyAsync(d.plane0, planes.data(), planes.size() * 4, hipMemcpyHostToDevice, hs));
    H3_HIP(hipStreamSynchronize(hs));
    return ISING_OK;
}

int ising3d_batch_get_sweep(ising3d_batch *b, int32_t r, uint64_t *t, void *stream)
{
    clear_error();
    (void)stream;
    int st = check_replica3(b, r);
    if (st != ISING_OK)
        return st;
    if (!t)
        return fail(ISING_E_INVALID, "t must not be NULL");
    *t = b->rep[r].t;
    return ISING_OK;
}

int ising3d_batch_destroy(ising3d_batch *b)
{
    delete b;
    return ISING_OK;
}

}  // extern "C"
