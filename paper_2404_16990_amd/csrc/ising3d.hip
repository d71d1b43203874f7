// 3D sweep kernels: checkerboard Metropolis on the periodic simple-cubic
// lattice (six neighbours; paper section 1), on packed colour planes whose
// rows are indexed by z*Ly + y.
//
// For a colour-c word of row (y, z), the other colour's word with the same
// index in each of the rows (y +- 1, z) and (y, z +- 1) holds the word's four
// neighbours along y and z (a colour's column parity flips with y and with z,
// so the compact positions line up); the other colour's word of the same row
// holds one x neighbour of every site and, funnel-shifted with the word before
// or after it, the other (as in 2D).
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "device3.hpp"
#include "ising3d.hpp"

namespace ising {

namespace {

__device__ __forceinline__ uint32_t block_owner(const uint32_t *__restrict__ prefix, uint32_t n, uint32_t b)
{
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Word indices of the six neighbours of word (row, w) of colour c.
struct Neigh3 {
    uint32_t ym, yp, zm, zp, same, nb, p;
};

__device__ __forceinline__ Neigh3 neigh3(const Rep3Dev &d, uint32_t idx, uint32_t colour)
{
    const uint32_t W = d.W, Ly = d.Ly, Lz = d.Lz;
    const uint32_t row = idx / W, w = idx - row * W;
    const uint32_t z = row / Ly, y = row - z * Ly;
    const uint32_t ym = y == 0 ? Ly - 1 : y - 1, yp = y + 1 == Ly ? 0 : y + 1;
    const uint32_t zm = z == 0 ? Lz - 1 : z - 1, zp = z + 1 == Lz ? 0 : z + 1;
    Neigh3 n;
    n.p = (colour + y + z) & 1u;
    n.same = idx;
    n.ym = (z * Ly + ym) * W + w;
    n.yp = (z * Ly + yp) * W + w;
    n.zm = (zm * Ly + y) * W + w;
    n.zp = (zp * Ly + y) * W + w;
    n.nb = row * W + (n.p ? (w + 1 == W ? 0 : w + 1) : (w == 0 ? W - 1 : w - 1));
    return n;
}

// Update NW words idx0, idx0 + 256, ... of colour c: every neighbour word of
// all NW words is loaded before the first update (the planes do not alias),
// so the loads of a thread are in flight together.
template <int NW, bool BITSLICED>
__device__ __forceinline__ void sweep_words(const uint32_t *__restrict__ src, uint32_t *__restrict__ tgt,
                                            uint32_t idx0, uint32_t colour, uint32_t t, const Rep3Dev &d)
{
    uint32_t s[NW], n[NW][6], q0[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const uint32_t idx = idx0 + 256u * k;
        const Neigh3 nb = neigh3(d, idx, colour);
        const uint32_t same = src[nb.same];
        n[k][0] = src[nb.ym];
        n[k][1] = src[nb.yp];
        n[k][2] = src[nb.zm];
        n[k][3] = src[nb.zp];
        n[k][4] = same;
        n[k][5] = side_word<uint32_t>(same, src[nb.nb], nb.p);
        s[k] = tgt[idx];
        const uint32_t row = idx / d.W, w = idx - row * d.W;
        q0[k] = row * (d.Lx >> 3) + 8u * w;  // (row * Lx / 2 + 32 w) / 4
    }
    const Key3 K = key3(d, t, colour);
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const uint32_t idx = idx0 + 256u * k;
        if constexpr (BITSLICED)
            tgt[idx] = s[k] ^ flip_mask32_3d_bitsliced(s[k], n[k], 8u * idx, K);
        else
            tgt[idx] = s[k] ^ flip_mask32_3d(s[k], n[k], q0[k], K);
    }
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) char gchar;
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) u32x4 gu32x4;

// Global-memory loads and stores at a 32-bit byte offset from a
// workgroup-uniform base, so the address is the base register pair plus one
// offset register.
__device__ __forceinline__ u32x4 load4(const uint32_t *base, uint32_t byte_off)
{
    return *(const gu32x4 *)((const gchar *)base + byte_off);
}

__device__ __forceinline__ uint32_t load1(const uint32_t *base, uint32_t byte_off)
{
    return *(const gu32 *)((const gchar *)base + byte_off);
}

__device__ __forceinline__ void store4(uint32_t *base, uint32_t byte_off, u32x4 v)
{
    *(gu32x4 *)((gchar *)base + byte_off) = v;
}

// Update the four words idx .. idx + 3 of a colour-c row (W a multiple of 4,
// idx a multiple of 4, so the four words share their row and their y and z
// neighbour rows): one 16-byte load from each of the five other-colour rows
// and from the target row, plus the one other-colour word beyond the quad on
// the side its x neighbours reach out to.  Offsets are in bytes and stay below
// 2^32 (a plane of N < 2^32 sites holds N / 16 bytes).
template <bool BITSLICED>
__device__ __forceinline__ void sweep_quad(const uint32_t *__restrict__ src, uint32_t *__restrict__ tgt, uint32_t idx,
                                           uint32_t colour, uint32_t t, const Rep3Dev &d)
{
    const uint32_t W = d.W, Ly = d.Ly, Lz = d.Lz;
    const uint32_t row = idx / W, w = idx - row * W;
    const uint32_t z = row / Ly, y = row - z * Ly;
    const uint32_t p = (colour + y + z) & 1u;
    const uint32_t row_b = 4u * W, slab_b = Ly * row_b, off = 4u * idx;
    const uint32_t off_ym = y == 0 ? off + (Ly - 1) * row_b : off - row_b;
    const uint32_t off_yp = y + 1 == Ly ? off - (Ly - 1) * row_b : off + row_b;
    const uint32_t off_zm = z == 0 ? off + (Lz - 1) * slab_b : off - slab_b;
    const uint32_t off_zp = z + 1 == Lz ? off - (Lz - 1) * slab_b : off + slab_b;
    // p = 1: the word after the quad (the row's first word after its last);
    // p = 0: the word before it (the row's last word before its first)
    const uint32_t off_x = p ? (w + 4 == W ? off + 16u - row_b : off + 16u) : (w == 0 ? off + row_b - 4u : off - 4u);
    const u32x4 ym = load4(src, off_ym), yp = load4(src, off_yp), zm = load4(src, off_zm), zp = load4(src, off_zp);
    const u32x4 same = load4(src, off), s = load4(tgt, off);
    const uint32_t beyond = load1(src, off_x);
    const Key3 K = key3(d, t, colour);
    // word k's other x word: same[k + 1] (or beyond) for p = 1, same[k - 1] (or beyond) for p = 0
    auto update = [&](uint32_t sk, uint32_t ymk, uint32_t ypk, uint32_t zmk, uint32_t zpk, uint32_t samek,
                      uint32_t otherk, uint32_t k) {
        const uint32_t n[6] = {ymk, ypk, zmk, zpk, samek, side_word<uint32_t>(samek, otherk, p)};
        if constexpr (BITSLICED)
            return sk ^ flip_mask32_3d_bitsliced(sk, n, 8u * (idx + k), K);
        else
            return sk ^ flip_mask32_3d(sk, n, 8u * (idx + k), K);
    };
    u32x4 out;
    out.x = update(s.x, ym.x, yp.x, zm.x, zp.x, same.x, p ? same.y : beyond, 0);
    out.y = update(s.y, ym.y, yp.y, zm.y, zp.y, same.y, p ? same.z : same.x, 1);
    out.z = update(s.z, ym.z, yp.z, zm.z, zp.z, same.z, p ? same.w : same.y, 2);
    out.w = update(s.w, ym.w, yp.w, zm.w, zp.w, same.w, p ? beyond : same.z, 3);
    store4(tgt, off, out);
}

// ---------------------------------------------------------------------------
// one colour of one sweep of every replica: grid = blocks of all replicas;
// workgroup b handles k3WordsPerBlock consecutive words of its replica's
// colour-c plane, thread i the words i, i + 256, ...
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k3_sweep(Sweep3Args a, uint32_t colour, uint32_t sweep_off)
{
    constexpr int NW = k3WordsPerBlock / 256;
    const uint32_t r = block_owner(a.prefix, a.n, blockIdx.x);
    const Rep3Dev d = a.reps[r];
    const uint32_t words = d.Lz * d.Ly * d.W;
    const uint32_t first = (blockIdx.x - a.prefix[r]) * k3WordsPerBlock;
    uint32_t *tgt = d.plane0 + (colour ? (size_t)words : 0);
    const uint32_t *src = d.plane0 + (colour ? 0 : (size_t)words);
    const uint32_t t = d.t + sweep_off;
    // the contract is uniform per replica, hence per workgroup
    const bool bitsliced = (d.flags & k3Bitsliced) != 0;
    if ((d.W & 3u) == 0) {
        // rows of a multiple of four words: thread i takes the quad at
        // first + 4 i (words is a multiple of 4, so a quad is whole or absent)
        static_assert(k3WordsPerBlock == 4 * 256, "one quad per thread");
        const uint32_t idx = first + 4u * threadIdx.x;
        if (idx < words) {
            if (bitsliced)
                sweep_quad<true>(src, tgt, idx, colour, t, d);
            else
                sweep_quad<false>(src, tgt, idx, colour, t, d);
        }
        return;
    }
    if (first + k3WordsPerBlock <= words) {
        if (bitsliced)
            sweep_words<NW, true>(src, tgt, first + threadIdx.x, colour, t, d);
        else
            sweep_words<NW, false>(src, tgt, first + threadIdx.x, colour, t, d);
        return;
    }
    for (uint32_t idx = first + threadIdx.x; idx < words; idx += 256) {  // the last, partial block
        if (bitsliced)
            sweep_words<1, true>(src, tgt, idx, colour, t, d);
        else
            sweep_words<1, false>(src, tgt, idx, colour, t, d);
    }
}

// initial states: both colour planes, same block mapping
__global__ __launch_bounds__(256) void k3_init(Sweep3Args a, const int32_t *__restrict__ modes)
{
    const uint32_t r = block_owner(a.prefix, a.n, blockIdx.x);
    const Rep3Dev d = a.reps[r];
    const int32_t mode = modes[r];
    const uint32_t words = d.Lz * d.Ly * d.W;
    const uint32_t first = (blockIdx.x - a.prefix[r]) * k3WordsPerBlock;
    for (uint32_t i = threadIdx.x; i < k3WordsPerBlock; i += 256) {
        const uint32_t idx = first + i;
        if (idx >= words)
            break;
        const uint32_t row = idx / d.W, w = idx - row * d.W;
        const uint32_t z = row / d.Ly, y = row - z * d.Ly;
        for (uint32_t c = 0; c < 2; ++c) {
            uint32_t v = mode == 1 ? ~0u : 0u;
            if (mode == 0) {
                // sites 2b + p of the word's 64 columns: g = base + 2b + p, so
                // call (g >> 2) = base / 4 + (b >> 1) gives bit b from word
                // 2 (b & 1) + p
                const uint32_t p = (c + y + z) & 1u;
                const uint32_t base = row * d.Lx + 64u * w;
                for (uint32_t j = 0; j < 16; ++j) {
                    uint32_t o[4];
                    philox4x32_10((base >> 2) + j, 0u, d.replica, 2u, d.seed_lo, d.seed_hi, o);
                    v |= (uint32_t)(o[p] >= 0x80000000u) << (2 * j);
                    v |= (uint32_t)(o[2 + p] >= 0x80000000u) << (2 * j + 1);
                }
            }
            d.plane0[(size_t)c * words + idx] = v;
        }
    }
}

// (B, M): every bond joins a colour-0 and a colour-1 site, so summing the six
// bonds of every colour-1 site counts each bond once: B = 6 N/2 - 2 A with A
// the anti-aligned pairs; M = 2 (up spins) - N.
__global__ __launch_bounds__(256) void k3_observables(Sweep3Args a, int64_t *__restrict__ bond,
                                                      int64_t *__restrict__ mag, uint32_t stride)
{
    const uint32_t r = block_owner(a.prefix, a.n, blockIdx.x);
    const Rep3Dev d = a.reps[r];
    const uint32_t words = d.Lz * d.Ly * d.W;
    const uint32_t first = (blockIdx.x - a.prefix[r]) * k3WordsPerBlock;
    const uint32_t *src = d.plane0, *tgt = d.plane0 + (size_t)words;
    uint32_t anti = 0, pop = 0;
    for (uint32_t i = threadIdx.x; i < k3WordsPerBlock; i += 256) {
        const uint32_t idx = first + i;
        if (idx >= words)
            break;
        const Neigh3 nb = neigh3(d, idx, 1u);
        const uint32_t same = src[nb.same], s = tgt[idx];
        const uint32_t side = side_word<uint32_t>(same, src[nb.nb], nb.p);
        anti += __popc(s ^ src[nb.ym]) + __popc(s ^ src[nb.yp]) + __popc(s ^ src[nb.zm]) + __popc(s ^ src[nb.zp]) +
                __popc(s ^ same) + __popc(s ^ side);
        pop += __popc(s) + __popc(same);
    }
    __shared__ int64_t red[2][4];
    const int64_t A = wave_sum((int64_t)anti), U = wave_sum((int64_t)pop);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = A;
        red[1][threadIdx.x >> 6] = U;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t db = -2 * (red[0][0] + red[0][1] + red[0][2] + red[0][3]);
        int64_t dm = 2 * (red[1][0] + red[1][1] + red[1][2] + red[1][3]);
        if (blockIdx.x == a.prefix[r]) {
            db += 3 * (int64_t)d.N;
            dm -= (int64_t)d.N;
        }
        atomicAdd(reinterpret_cast<unsigned long long *>(&bond[(size_t)r * stride]), (unsigned long long)db);
        atomicAdd(reinterpret_cast<unsigned long long *>(&mag[(size_t)r * stride]), (unsigned long long)dm);
    }
}

__global__ void k3_advance(Rep3Dev *__restrict__ reps, uint32_t n, uint32_t delta)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n)
        reps[r].t += delta;
}

}  // namespace

hipError_t launch3_init(const Sweep3Args &a, const int32_t *modes, hipStream_t st)
{
    hipLaunchKernelGGL(k3_init, dim3(a.blocks), dim3(256), 0, st, a, modes);
    return hipGetLastError();
}

hipError_t launch3_sweep(const Sweep3Args &a, uint32_t colour, uint32_t sweep_off, hipStream_t st)
{
    hipLaunchKernelGGL(k3_sweep, dim3(a.blocks), dim3(256), 0, st, a, colour, sweep_off);
    return hipGetLastError();
}

hipError_t launch3_observables(const Sweep3Args &a, int64_t *bond, int64_t *mag, uint32_t stride, hipStream_t st)
{
    hipLaunchKernelGGL(k3_observables, dim3(a.blocks), dim3(256), 0, st, a, bond, mag, stride);
    return hipGetLastError();
}

hipError_t launch3_advance(Rep3Dev *reps, uint32_t n, uint32_t delta, hipStream_t st)
{
    hipLaunchKernelGGL(k3_advance, dim3((n + 255) / 256), dim3(256), 0, st, reps, n, delta);
    return hipGetLastError();
}

}  // namespace ising
