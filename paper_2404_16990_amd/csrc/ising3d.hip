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

typedef __attribute__((address_space(1))) char gchar;

template <int NQ>
struct VecOf;
template <>
struct VecOf<1> {
    typedef uint32_t type;
};
template <>
struct VecOf<2> {
    typedef uint32_t type __attribute__((ext_vector_type(2)));
};
template <>
struct VecOf<4> {
    typedef uint32_t type __attribute__((ext_vector_type(4)));
};

// NQ consecutive words loaded / stored as one access at a 32-bit byte offset
// from a workgroup-uniform base, so the address is the base register pair
// plus one offset register.
template <int NQ>
__device__ __forceinline__ void load_words(const uint32_t *base, uint32_t byte_off, uint32_t (&v)[NQ])
{
    typedef typename VecOf<NQ>::type V;
    typedef __attribute__((address_space(1))) V GV;
    const V x = *(const GV *)((const gchar *)base + byte_off);
    if constexpr (NQ == 1) {
        v[0] = x;
    } else {
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            v[k] = x[k];
    }
}

template <int NQ>
__device__ __forceinline__ void store_words(uint32_t *base, uint32_t byte_off, const uint32_t (&v)[NQ])
{
    typedef typename VecOf<NQ>::type V;
    typedef __attribute__((address_space(1))) V GV;
    V x;
    if constexpr (NQ == 1) {
        x = v[0];
    } else {
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            x[k] = v[k];
    }
    *(GV *)((gchar *)base + byte_off) = x;
}

// The NQ words idx .. idx + NQ - 1 of a colour-c row (W a multiple of NQ, idx
// a multiple of NQ, so the words share their row and their y and z neighbour
// rows) and their neighbours: one NQ-word load from each of the five
// other-colour rows and from the target row, plus the one other-colour word
// beyond the group on the side its x neighbours reach out to.  Offsets are in
// bytes and stay below 2^32 (a plane of N < 2^32 sites holds N / 16 bytes).
template <int NQ>
struct Group {
    uint32_t ym[NQ], yp[NQ], zm[NQ], zp[NQ], same[NQ], s[NQ];
    uint32_t beyond, p;
};

template <int NQ>
__device__ __forceinline__ Group<NQ> load_group(const uint32_t *__restrict__ src, const uint32_t *__restrict__ tgt,
                                                uint32_t idx, uint32_t colour, const Rep3Dev &d)
{
    const uint32_t W = d.W, Ly = d.Ly, Lz = d.Lz;
    const uint32_t row = idx / W, w = idx - row * W;
    const uint32_t z = row / Ly, y = row - z * Ly;
    Group<NQ> g;
    g.p = (colour + y + z) & 1u;
    const uint32_t row_b = 4u * W, slab_b = Ly * row_b, off = 4u * idx;
    const uint32_t off_ym = y == 0 ? off + (Ly - 1) * row_b : off - row_b;
    const uint32_t off_yp = y + 1 == Ly ? off - (Ly - 1) * row_b : off + row_b;
    const uint32_t off_zm = z == 0 ? off + (Lz - 1) * slab_b : off - slab_b;
    const uint32_t off_zp = z + 1 == Lz ? off - (Lz - 1) * slab_b : off + slab_b;
    // p = 1: the word after the group (the row's first word after its last);
    // p = 0: the word before it (the row's last word before its first)
    const uint32_t off_x = g.p ? (w + NQ == W ? off + 4u * NQ - row_b : off + 4u * NQ)
                               : (w == 0 ? off + row_b - 4u : off - 4u);
    load_words<NQ>(src, off_ym, g.ym);
    load_words<NQ>(src, off_yp, g.yp);
    load_words<NQ>(src, off_zm, g.zm);
    load_words<NQ>(src, off_zp, g.zp);
    load_words<NQ>(src, off, g.same);
    load_words<NQ>(tgt, off, g.s);
    uint32_t b[1];
    load_words<1>(src, off_x, b);
    g.beyond = b[0];
    return g;
}

template <int NQ, bool BITSLICED>
__device__ __forceinline__ void update_group(const Group<NQ> &g, uint32_t *__restrict__ tgt, uint32_t idx,
                                             const Key3 &K)
{
    uint32_t out[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        // word k's other x word: same[k + 1] (or beyond) for p = 1, same[k - 1] (or beyond) for p = 0
        const uint32_t after = k + 1 < NQ ? g.same[k + 1 < NQ ? k + 1 : k] : g.beyond;
        const uint32_t before = k > 0 ? g.same[k > 0 ? k - 1 : 0] : g.beyond;
        const uint32_t n[6] = {g.ym[k], g.yp[k], g.zm[k], g.zp[k], g.same[k],
                               side_word<uint32_t>(g.same[k], g.p ? after : before, g.p)};
        if constexpr (BITSLICED)
            out[k] = g.s[k] ^ flip_mask32_3d_bitsliced(g.s[k], n, 8u * (idx + k), K);
        else
            out[k] = g.s[k] ^ flip_mask32_3d(g.s[k], n, 8u * (idx + k), K);
    }
    store_words<NQ>(tgt, 4u * idx, out);
}

// Thread i of a workgroup updates the 4 / NQ groups of NQ words at
// first + NQ i + 256 NQ j that lie below words (words is a multiple of NQ, so
// a group is whole or absent): every group's loads are issued before the first
// update (a group past the plane loads group 0 instead and is not updated).
template <int NQ, bool BITSLICED>
__device__ __forceinline__ void sweep_groups(const uint32_t *__restrict__ src, uint32_t *__restrict__ tgt,
                                             uint32_t first, uint32_t words, uint32_t colour, uint32_t t,
                                             const Rep3Dev &d)
{
    constexpr int NG = 4 / NQ;
    static_assert(k3WordsPerBlock == 4 * 256, "four words per thread");
    if constexpr (NG == 1) {
        const uint32_t idx = first + NQ * threadIdx.x;
        if (idx < words) {
            const Group<NQ> g = load_group<NQ>(src, tgt, idx, colour, d);
            update_group<NQ, BITSLICED>(g, tgt, idx, key3(d, t, colour));
        }
        return;
    }
    Group<NQ> g[NG];
#pragma unroll
    for (int j = 0; j < NG; ++j) {
        const uint32_t idx = first + NQ * threadIdx.x + 256u * NQ * j;
        g[j] = load_group<NQ>(src, tgt, idx < words ? idx : 0u, colour, d);
    }
    const Key3 K = key3(d, t, colour);
#pragma unroll
    for (int j = 0; j < NG; ++j) {
        const uint32_t idx = first + NQ * threadIdx.x + 256u * NQ * j;
        if (idx < words)
            update_group<NQ, BITSLICED>(g[j], tgt, idx, K);
    }
}

// ---------------------------------------------------------------------------
// one colour of one sweep of every replica with group width NQ: grid =
// blocks of all replicas; workgroup b handles k3WordsPerBlock consecutive
// words of its replica's colour-c plane, each thread four of them in groups of
// NQ consecutive words
// ---------------------------------------------------------------------------
template <int NQ>
__global__ __launch_bounds__(256) void k3_sweep(Sweep3Args a, uint32_t colour, uint32_t sweep_off)
{
    const uint32_t r = block_owner(a.prefix, a.n, blockIdx.x);
    const Rep3Dev d = a.reps[r];
    // one kernel per group width (each with its own register budget): the
    // workgroups of replicas with another width leave at once
    if (group_width(d.W) != NQ)
        return;
    const uint32_t words = d.Lz * d.Ly * d.W;
    const uint32_t first = (blockIdx.x - a.prefix[r]) * k3WordsPerBlock;
    uint32_t *tgt = d.plane0 + (colour ? (size_t)words : 0);
    const uint32_t *src = d.plane0 + (colour ? 0 : (size_t)words);
    const uint32_t t = d.t + sweep_off;
    // the contract is uniform per replica, hence per workgroup
    if ((d.flags & k3Bitsliced) != 0)
        sweep_groups<NQ, true>(src, tgt, first, words, colour, t, d);
    else
        sweep_groups<NQ, false>(src, tgt, first, words, colour, t, d);
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
    if (a.widths & 4u)
        hipLaunchKernelGGL(k3_sweep<4>, dim3(a.blocks), dim3(256), 0, st, a, colour, sweep_off);
    if (a.widths & 2u)
        hipLaunchKernelGGL(k3_sweep<2>, dim3(a.blocks), dim3(256), 0, st, a, colour, sweep_off);
    if (a.widths & 1u)
        hipLaunchKernelGGL(k3_sweep<1>, dim3(a.blocks), dim3(256), 0, st, a, colour, sweep_off);
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
