// HIP kernels for gfx950: initial state, checkerboard sweeps (streaming and
// LDS-resident), observables, and small bookkeeping kernels.
//
// The sweep follows the checkerboard algorithm (paper section 2 and the
// Supplementary checkerboard multi-spin algorithm): every colour-0 site, then
// every colour-1 site reading the updated colour 0.  One thread updates one
// 32- or 64-bit word of same-colour spins; neighbour words come from the other
// colour's plane (up, down, same position, and a funnel-shifted horizontal
// word), so a colour phase reads only the other plane and its own word.
#include "device.hpp"
#include "launch.hpp"

namespace ising {

// ---------------------------------------------------------------------------
// initial state: one thread per 32-bit word of one plane
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init(const RepDev *__restrict__ reps,
                                              const int32_t *__restrict__ modes)
{
    const uint32_t r = blockIdx.y;
    const RepDev d = reps[r];
    const int32_t mode = modes[r];
    const uint32_t words = 2u * d.Ly * d.W;  // both planes
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x) {
        uint32_t v;
        if (mode == 1) {
            v = 0xffffffffu;
        } else if (mode == 2) {
            v = 0u;
        } else {
            const uint32_t c = i >= d.Ly * d.W ? 1u : 0u;
            const uint32_t j = i - c * d.Ly * d.W;
            const uint32_t y = j / d.W, w = j - y * d.W;
            const uint32_t p = (c + y) & 1u;
            // site b of this word: x = 64 w + 2 b + p, g = y Lx + x; the
            // Philox call g >> 2 = (y Lx + 64 w) / 4 + b / 2 serves bits 2m, 2m+1
            const uint32_t qbase = (y * d.Lx + 64u * w) >> 2;
            v = 0;
#pragma unroll 4
            for (uint32_t m = 0; m < 16; ++m) {
                uint32_t o[4];
                philox4x32_10(qbase + m, 0u, d.replica, 2u, d.seed_lo, d.seed_hi, o);
                v |= (uint32_t)(o[p] >= 0x80000000u) << (2 * m);
                v |= (uint32_t)(o[p + 2] >= 0x80000000u) << (2 * m + 1);
            }
        }
        d.plane0[i] = v;
    }
}

// ---------------------------------------------------------------------------
// one thread's share of one colour phase: words idx = first, first + THREADS,
// ... < end of a plane of Ly rows x Wn words.  Indices advance incrementally:
// the vertical neighbours wrap with an unsigned min (u or u + total, whichever
// is in range), and the word's first Philox counter is idx * BITS / 4 because
// a colour row holds Wn * BITS = Lx / 2 sites.  FIXED_W: Wn divides THREADS,
// so the thread's column w and its horizontal neighbours never change.
// ---------------------------------------------------------------------------
template <typename Word, int THREADS, bool FIXED_W, bool BITSLICED>
__device__ __forceinline__ void update_words(const Word *__restrict__ src, Word *__restrict__ dst,
                                             uint32_t first, uint32_t end, uint32_t Ly, uint32_t Wn,
                                             const SweepKey &K, bool rec, uint32_t &anti, uint32_t &pop)
{
    constexpr uint32_t QW = WordTraits<Word>::BITS / 4;
    const uint32_t total = Ly * Wn;
    const uint32_t dy = THREADS / Wn, dw = THREADS - dy * Wn;
    uint32_t y = first / Wn, w = first - y * Wn;
    uint32_t wp = w + 1 == Wn ? 0 : w + 1, wm = w == 0 ? Wn - 1 : w - 1;
    for (uint32_t idx = first; idx < end; idx += THREADS) {
        const uint32_t p = (K.colour ^ y) & 1u;
        const uint32_t u = idx - Wn, v = idx + Wn;
        const Word same = src[idx];
        const Word up = src[min(u, u + total)];
        const Word dn = src[min(v, v - total)];
        const Word nb = src[idx - w + (p ? wp : wm)];
        const Word s = dst[idx];
        const Word side = side_word<Word>(same, nb, p);
        const Word ns = update_word<Word, BITSLICED>(s, up, dn, same, side, idx * QW, K);
        dst[idx] = ns;
        if (rec) {
            anti += anti_bonds<Word>(ns, up, dn, same, side);
            pop += (uint32_t)(__popcll((uint64_t)ns) + __popcll((uint64_t)same));
        }
        y += dy;
        if (!FIXED_W) {
            w += dw;
            if (w >= Wn) {
                w -= Wn;
                ++y;
            }
            wp = w + 1 == Wn ? 0 : w + 1;
            wm = w == 0 ? Wn - 1 : w - 1;
        }
    }
}

// One thread's share of a colour phase with the column and contract
// specialisations chosen once (both are uniform over the workgroup).
template <typename Word, int THREADS>
__device__ __forceinline__ void update_words_any(const Word *__restrict__ src, Word *__restrict__ dst,
                                                 uint32_t first, uint32_t end, uint32_t Ly, uint32_t Wn,
                                                 const SweepKey &K, bool rec, uint32_t &anti, uint32_t &pop)
{
    const bool fixed_w = THREADS % Wn == 0;
    if (K.rng) {
        if (fixed_w)
            update_words<Word, THREADS, true, true>(src, dst, first, end, Ly, Wn, K, rec, anti, pop);
        else
            update_words<Word, THREADS, false, true>(src, dst, first, end, Ly, Wn, K, rec, anti, pop);
    } else {
        if (fixed_w)
            update_words<Word, THREADS, true, false>(src, dst, first, end, Ly, Wn, K, rec, anti, pop);
        else
            update_words<Word, THREADS, false, false>(src, dst, first, end, Ly, Wn, K, rec, anti, pop);
    }
}

// ---------------------------------------------------------------------------
// streaming sweep: one colour of one sweep for a list of replicas; each
// workgroup takes a contiguous run of words_per_wg words of one replica
// ---------------------------------------------------------------------------
template <typename Word, int THREADS>
__global__ __launch_bounds__(THREADS) void k_sweep_stream(const RepDev *__restrict__ reps,
                                                          const uint32_t *__restrict__ list,
                                                          const uint32_t *__restrict__ prefix,
                                                          uint32_t nlist, uint32_t words_per_wg,
                                                          uint32_t colour, uint32_t sweep_off,
                                                          const RecArgs *__restrict__ recp)
{
    constexpr int PER32 = WordTraits<Word>::PER32;
    const RecArgs rec = *recp;
    // workgroup -> list entry: largest e with prefix[e] <= blockIdx.x
    uint32_t lo = 0, hi = nlist;
    const uint32_t bid = blockIdx.x;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= bid)
            lo = mid;
        else
            hi = mid;
    }
    const uint32_t tile = bid - prefix[lo];
    const uint32_t r = list[lo];
    const RepDev d = reps[r];
    const uint32_t Wn = d.W / PER32;
    const uint32_t Ly = d.Ly;
    const uint32_t total = Ly * Wn;
    const uint32_t t = d.t + sweep_off;
    const Word *__restrict__ src = reinterpret_cast<const Word *>(d.plane0 + (colour ^ 1u) * Ly * d.W);
    Word *__restrict__ dst = reinterpret_cast<Word *>(d.plane0 + colour * Ly * d.W);
    const SweepKey K = make_key(d, t, colour);

    // recording decision (uniform): after the blue phase of run-local sweep i
    const uint32_t i_run = t - d.t0;
    const bool record = colour == 1u && rec.every != 0u && ((i_run + 1u) % rec.every) == 0u &&
                        ((i_run + 1u) / rec.every - 1u) < rec.n_rec;

    const uint32_t begin = tile * words_per_wg;
    const uint32_t end = min(begin + words_per_wg, total);
    uint32_t anti = 0, pop = 0;
    update_words_any<Word, THREADS>(src, dst, begin + threadIdx.x, end, Ly, Wn, K, record, anti, pop);
    if (record) {
        __shared__ int64_t red[2][THREADS / 64];
        const int64_t a = wave_sum((int64_t)anti);
        const int64_t m = wave_sum((int64_t)pop);
        const int wid = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[0][wid] = a;
            red[1][wid] = m;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t A = 0, Mp = 0;
#pragma unroll
            for (int k = 0; k < THREADS / 64; ++k) {
                A += red[0][k];
                Mp += red[1][k];
            }
            // B = 2N - 2 anti, M = 2 pop - N; the first tile adds the constants
            int64_t db = -2 * A, dm = 2 * Mp;
            if (tile == 0) {
                db += 2 * (int64_t)d.N;
                dm -= (int64_t)d.N;
            }
            const uint32_t slot = (i_run + 1u) / rec.every - 1u;
            atomicAdd(reinterpret_cast<unsigned long long *>(&rec.bond[(uint64_t)r * rec.n_rec + slot]),
                      (unsigned long long)db);
            atomicAdd(reinterpret_cast<unsigned long long *>(&rec.mag[(uint64_t)r * rec.n_rec + slot]),
                      (unsigned long long)dm);
        }
    }
}

// ---------------------------------------------------------------------------
// LDS-resident sweeps: one workgroup owns one replica for n_sweeps sweeps
// ---------------------------------------------------------------------------
// A resident workgroup owns its replica's LDS; for the 1024^2 lattices that is
// the whole CU, so the compiler is told to schedule for THREADS/256 waves per
// SIMD (more registers for interleaving independent Philox calls).
template <typename Word, int THREADS>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(1, THREADS / 256 > 0 ? THREADS / 256 : 1)))
void k_sweep_resident(const RepDev *__restrict__ reps,
                                                            const uint32_t *__restrict__ list,
                                                            uint32_t n_sweeps, const RecArgs *__restrict__ recp)
{
    constexpr int PER32 = WordTraits<Word>::PER32;
    const RecArgs rec = *recp;
    extern __shared__ uint4 lds4[];
    const uint32_t r = list[blockIdx.x];
    const RepDev d = reps[r];
    const uint32_t Ly = d.Ly;
    const uint32_t words32 = Ly * d.W;  // per plane
    const uint32_t Wn = d.W / PER32;
    const uint32_t total = Ly * Wn;
    // both planes: 2 Ly W words; Ly even => a multiple of 4 words (16 bytes)
    const uint32_t n4 = (2u * words32) >> 2;
    const uint4 *__restrict__ g4 = reinterpret_cast<const uint4 *>(d.plane0);
    for (uint32_t i = threadIdx.x; i < n4; i += THREADS)
        lds4[i] = g4[i];
    __syncthreads();
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);

    __shared__ int64_t red[2][THREADS / 64];

    for (uint32_t s_i = 0; s_i < n_sweeps; ++s_i) {
        const uint32_t t = d.t + s_i;
        const uint32_t i_run = t - d.t0;
        const bool record = rec.every != 0u && ((i_run + 1u) % rec.every) == 0u &&
                            ((i_run + 1u) / rec.every - 1u) < rec.n_rec;
#pragma unroll 1
        for (uint32_t colour = 0; colour < 2; ++colour) {
            const Word *src = reinterpret_cast<const Word *>(lds + (colour ^ 1u) * words32);
            Word *dst = reinterpret_cast<Word *>(lds + colour * words32);
            const SweepKey K = make_key(d, t, colour);
            const bool rec_here = record && colour == 1u;
            uint32_t anti = 0, pop = 0;
            update_words_any<Word, THREADS>(src, dst, threadIdx.x, total, Ly, Wn, K, rec_here, anti, pop);
            if (rec_here) {
                const int64_t a = wave_sum((int64_t)anti);
                const int64_t m = wave_sum((int64_t)pop);
                if ((threadIdx.x & 63) == 0) {
                    red[0][threadIdx.x >> 6] = a;
                    red[1][threadIdx.x >> 6] = m;
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    int64_t A = 0, Mp = 0;
                    for (int k = 0; k < THREADS / 64; ++k) {
                        A += red[0][k];
                        Mp += red[1][k];
                    }
                    const uint32_t slot = (i_run + 1u) / rec.every - 1u;
                    rec.bond[(uint64_t)r * rec.n_rec + slot] = 2 * (int64_t)d.N - 2 * A;
                    rec.mag[(uint64_t)r * rec.n_rec + slot] = 2 * Mp - (int64_t)d.N;
                }
            }
            __syncthreads();
        }
    }
    uint4 *__restrict__ o4 = reinterpret_cast<uint4 *>(d.plane0);
    for (uint32_t i = threadIdx.x; i < n4; i += THREADS)
        o4[i] = lds4[i];
}

// ---------------------------------------------------------------------------
// observables of the current state: grid (x: tiles, y: replica); replica r's
// sums are added to bond[r * stride] and mag[r * stride]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_observables(const RepDev *__restrict__ reps,
                                                     int64_t *__restrict__ bond,
                                                     int64_t *__restrict__ mag, uint32_t stride)
{
    const uint32_t r = blockIdx.y;
    const RepDev d = reps[r];
    const uint32_t W = d.W, Ly = d.Ly;
    const uint32_t *src = d.plane0;              // colour 0
    const uint32_t *tgt = d.plane0 + Ly * W;     // colour 1
    uint32_t anti = 0, pop = 0;
    for (uint32_t idx = blockIdx.x * 256 + threadIdx.x; idx < Ly * W; idx += gridDim.x * 256) {
        const uint32_t y = idx / W, w = idx - y * W;
        const NeighIdx n = neigh_idx(y, w, Ly, W, 1u);
        const uint32_t same = src[n.same];
        const uint32_t side = side_word<uint32_t>(same, src[n.nb], n.p);
        const uint32_t s = tgt[idx];
        anti += anti_bonds<uint32_t>(s, src[n.up], src[n.dn], same, side);
        pop += (uint32_t)(__popc(s) + __popc(same));
    }
    __shared__ int64_t red[2][4];
    const int64_t a = wave_sum((int64_t)anti), m = wave_sum((int64_t)pop);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t A = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        int64_t Mp = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        int64_t db = -2 * A, dm = 2 * Mp;
        if (blockIdx.x == 0) {
            db += 2 * (int64_t)d.N;
            dm -= (int64_t)d.N;
        }
        atomicAdd(reinterpret_cast<unsigned long long *>(&bond[(size_t)r * stride]), (unsigned long long)db);
        atomicAdd(reinterpret_cast<unsigned long long *>(&mag[(size_t)r * stride]), (unsigned long long)dm);
    }
}

// Observables of the state after the run-local step i_run = t + step - t0 of
// every replica, added to the trace slot (i_run + 1) / every - 1 when
// (i_run + 1) % every == 0 (the slot is computed on the device, so a captured
// chunk of steps records correctly on every replay).
__global__ __launch_bounds__(256) void k_observables_rec(const RepDev *__restrict__ reps,
                                                         const RecArgs *__restrict__ recp, uint32_t step)
{
    const RecArgs rec = *recp;
    const uint32_t r = blockIdx.y;
    const RepDev d = reps[r];
    const uint32_t i_run = d.t + step - d.t0;
    if (rec.every == 0u || ((i_run + 1u) % rec.every) != 0u || (i_run + 1u) / rec.every - 1u >= rec.n_rec)
        return;
    const uint64_t slot = (uint64_t)r * rec.n_rec + (i_run + 1u) / rec.every - 1u;
    const uint32_t W = d.W, Ly = d.Ly;
    const uint32_t *src = d.plane0;
    const uint32_t *tgt = d.plane0 + Ly * W;
    uint32_t anti = 0, pop = 0;
    for (uint32_t idx = blockIdx.x * 256 + threadIdx.x; idx < Ly * W; idx += gridDim.x * 256) {
        const uint32_t y = idx / W, w = idx - y * W;
        const NeighIdx n = neigh_idx(y, w, Ly, W, 1u);
        const uint32_t same = src[n.same];
        const uint32_t side = side_word<uint32_t>(same, src[n.nb], n.p);
        const uint32_t s = tgt[idx];
        anti += anti_bonds<uint32_t>(s, src[n.up], src[n.dn], same, side);
        pop += (uint32_t)(__popc(s) + __popc(same));
    }
    __shared__ int64_t red[2][4];
    const int64_t a = wave_sum((int64_t)anti), m = wave_sum((int64_t)pop);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t db = -2 * (red[0][0] + red[0][1] + red[0][2] + red[0][3]);
        int64_t dm = 2 * (red[1][0] + red[1][1] + red[1][2] + red[1][3]);
        if (blockIdx.x == 0) {
            db += 2 * (int64_t)d.N;
            dm -= (int64_t)d.N;
        }
        atomicAdd(reinterpret_cast<unsigned long long *>(&rec.bond[slot]), (unsigned long long)db);
        atomicAdd(reinterpret_cast<unsigned long long *>(&rec.mag[slot]), (unsigned long long)dm);
    }
}

// ---------------------------------------------------------------------------
// bookkeeping (graph-safe: plain kernels, no memset nodes)
// ---------------------------------------------------------------------------
__global__ void k_fill_i64(int64_t *__restrict__ p, uint64_t n, int64_t v)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Start of a run, one launch: every replica's t0 = t, the recording
// arguments of the run written to dst (on the stream in order, so a captured
// chunk reads the current run's traces on every replay), and the run's trace
// slots (if any) zeroed for the recording kernels' atomic sums.
__global__ void k_begin_run(RepDev *__restrict__ reps, uint32_t n, RecArgs *__restrict__ dst, RecArgs v)
{
    const uint64_t i0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x, stride = (uint64_t)gridDim.x * blockDim.x;
    if (i0 < n)
        reps[i0].t0 = reps[i0].t;
    if (i0 == 0)
        *dst = v;
    const uint64_t slots = v.bond ? (uint64_t)n * v.n_rec : 0;
    for (uint64_t i = i0; i < slots; i += stride) {
        v.bond[i] = 0;
        v.mag[i] = 0;
    }
}

__global__ void k_advance(RepDev *__restrict__ reps, uint32_t n, uint32_t delta)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n)
        reps[r].t += delta;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_init(const RepDev *reps, const int32_t *modes, uint32_t n, uint32_t max_words,
                       hipStream_t st)
{
    const uint32_t blocks = std::min<uint32_t>((2u * max_words + 255u) / 256u, 4096u);
    hipLaunchKernelGGL(k_init, dim3(blocks, n), dim3(256), 0, st, reps, modes);
    return hipGetLastError();
}

hipError_t launch_observables(const RepDev *reps, uint32_t n, uint32_t max_words, int64_t *bond,
                              int64_t *mag, hipStream_t st, uint32_t stride)
{
    const uint32_t blocks = std::min<uint32_t>((max_words + 255u) / 256u, 2048u);
    hipLaunchKernelGGL(k_observables, dim3(blocks, n), dim3(256), 0, st, reps, bond, mag, stride);
    return hipGetLastError();
}

hipError_t launch_observables_rec(const RepDev *reps, uint32_t n, uint32_t max_words, const RecArgs *rec,
                                  uint32_t step, hipStream_t st)
{
    const uint32_t blocks = std::min<uint32_t>((max_words + 255u) / 256u, 2048u);
    hipLaunchKernelGGL(k_observables_rec, dim3(blocks, n), dim3(256), 0, st, reps, rec, step);
    return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t *p, uint64_t n, int64_t v, hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_i64, dim3((uint32_t)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_begin_run(RepDev *reps, uint32_t n, RecArgs *dst, const RecArgs &v, hipStream_t st)
{
    const uint64_t slots = v.bond ? (uint64_t)n * v.n_rec : 0;
    const uint64_t blocks = std::max<uint64_t>((n + 255) / 256, std::min<uint64_t>((slots + 255) / 256, 1024));
    hipLaunchKernelGGL(k_begin_run, dim3((uint32_t)blocks), dim3(256), 0, st, reps, n, dst, v);
    return hipGetLastError();
}

hipError_t launch_advance(RepDev *reps, uint32_t n, uint32_t delta, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance, dim3((n + 255) / 256), dim3(256), 0, st, reps, n, delta);
    return hipGetLastError();
}

template <typename Word, int T>
static hipError_t stream_t(const StreamList &L, uint32_t colour, uint32_t sweep_off, const RecArgs *rec,
                           hipStream_t st)
{
    hipLaunchKernelGGL((k_sweep_stream<Word, T>), dim3(L.n_wg), dim3(T), 0, st, L.reps, L.list,
                       L.prefix, L.n, L.words_per_wg, colour, sweep_off, rec);
    return hipGetLastError();
}

hipError_t launch_sweep_stream(const StreamList &L, int word_bits, int threads, uint32_t colour,
                               uint32_t sweep_off, const RecArgs *rec, hipStream_t st)
{
    if (L.n == 0)
        return hipSuccess;
    if (word_bits == 64) {
        switch (threads) {
        case 64: return stream_t<uint64_t, 64>(L, colour, sweep_off, rec, st);
        case 128: return stream_t<uint64_t, 128>(L, colour, sweep_off, rec, st);
        case 256: return stream_t<uint64_t, 256>(L, colour, sweep_off, rec, st);
        case 512: return stream_t<uint64_t, 512>(L, colour, sweep_off, rec, st);
        case 1024: return stream_t<uint64_t, 1024>(L, colour, sweep_off, rec, st);
        }
    } else {
        switch (threads) {
        case 64: return stream_t<uint32_t, 64>(L, colour, sweep_off, rec, st);
        case 128: return stream_t<uint32_t, 128>(L, colour, sweep_off, rec, st);
        case 256: return stream_t<uint32_t, 256>(L, colour, sweep_off, rec, st);
        case 512: return stream_t<uint32_t, 512>(L, colour, sweep_off, rec, st);
        case 1024: return stream_t<uint32_t, 1024>(L, colour, sweep_off, rec, st);
        }
    }
    return hipErrorInvalidValue;
}

template <typename Word, int T>
static hipError_t resident_t(const ResidentList &L, uint32_t n_sweeps, const RecArgs *rec, hipStream_t st)
{
    hipLaunchKernelGGL((k_sweep_resident<Word, T>), dim3(L.n), dim3(T), L.lds_bytes, st, L.reps, L.list,
                       n_sweeps, rec);
    return hipGetLastError();
}

template <typename Word, int T>
static hipError_t raise_lds(int bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sweep_resident<Word, T>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t prepare_resident_kernels(int max_dynamic_lds)
{
    hipError_t e = hipSuccess;
#define ISING_RAISE(W, T)                                  \
    if (e == hipSuccess)                                   \
        e = raise_lds<W, T>(max_dynamic_lds);
    ISING_RAISE(uint32_t, 64) ISING_RAISE(uint32_t, 128) ISING_RAISE(uint32_t, 256)
    ISING_RAISE(uint32_t, 512) ISING_RAISE(uint32_t, 1024) ISING_RAISE(uint64_t, 64)
    ISING_RAISE(uint64_t, 128) ISING_RAISE(uint64_t, 256) ISING_RAISE(uint64_t, 512)
    ISING_RAISE(uint64_t, 1024)
#undef ISING_RAISE
    return e;
}

template <typename Word, int T>
static uint32_t static_lds_of()
{
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, reinterpret_cast<const void *>(&k_sweep_resident<Word, T>)) != hipSuccess)
        return 4096u;  // generous fallback: the kernels declare far less
    return (uint32_t)a.sharedSizeBytes;
}

// Largest static LDS of the resident kernels (reported by the runtime), so
// that static + dynamic LDS never exceeds the device limit.
uint32_t resident_static_lds(int /*threads*/)
{
    static uint32_t cached = 0;
    if (cached == 0) {
        uint32_t m = 0;
        const uint32_t v[] = {static_lds_of<uint32_t, 64>(),  static_lds_of<uint32_t, 128>(),
                              static_lds_of<uint32_t, 256>(), static_lds_of<uint32_t, 512>(),
                              static_lds_of<uint32_t, 1024>(), static_lds_of<uint64_t, 64>(),
                              static_lds_of<uint64_t, 128>(), static_lds_of<uint64_t, 256>(),
                              static_lds_of<uint64_t, 512>(), static_lds_of<uint64_t, 1024>()};
        for (uint32_t x : v)
            m = x > m ? x : m;
        cached = m;
    }
    return cached;
}

hipError_t launch_sweep_resident(const ResidentList &L, int word_bits, int threads, uint32_t n_sweeps,
                                 const RecArgs *rec, hipStream_t st)
{
    if (L.n == 0)
        return hipSuccess;
    if (word_bits == 64) {
        switch (threads) {
        case 64: return resident_t<uint64_t, 64>(L, n_sweeps, rec, st);
        case 128: return resident_t<uint64_t, 128>(L, n_sweeps, rec, st);
        case 256: return resident_t<uint64_t, 256>(L, n_sweeps, rec, st);
        case 512: return resident_t<uint64_t, 512>(L, n_sweeps, rec, st);
        case 1024: return resident_t<uint64_t, 1024>(L, n_sweeps, rec, st);
        }
    } else {
        switch (threads) {
        case 64: return resident_t<uint32_t, 64>(L, n_sweeps, rec, st);
        case 128: return resident_t<uint32_t, 128>(L, n_sweeps, rec, st);
        case 256: return resident_t<uint32_t, 256>(L, n_sweeps, rec, st);
        case 512: return resident_t<uint32_t, 512>(L, n_sweeps, rec, st);
        case 1024: return resident_t<uint32_t, 1024>(L, n_sweeps, rec, st);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace ising
