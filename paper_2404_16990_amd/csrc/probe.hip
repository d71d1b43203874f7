// Micro-benchmarks that measure the issue cost of the instructions the sweep
// is built from, and a plain copy kernel of known size used to calibrate HBM
// traffic counters.  Built into libising_probe.so (not part of the sweep
// library); the roofline of the sweep kernel is derived from these costs.
//
// Each probe thread runs 8 independent dependency chains of one instruction
// so that issue rate, not latency, bounds it.  Only ALU instructions appear in
// the inline assembly; the chains' results are stored with ordinary stores.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "device3.hpp"

namespace {

constexpr int kChains = 8;

enum Which { MAD_U64_U32 = 0, MUL_HI_U32 = 1, MUL_LO_U32 = 2, BITOP3 = 3, XOR = 4, ADD = 5, PHILOX = 6,
             LSHL_ADD_U64 = 7, ADDC = 8, CMP = 9, BFE = 10, ALIGNBIT = 11, CNDMASK = 12 };

template <int W>
__global__ __launch_bounds__(256) void k_alu(uint32_t *out, uint32_t seed, int iters)
{
    uint32_t a[kChains], b[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        a[c] = seed ^ (threadIdx.x * 0x9E3779B9u + c);
        b[c] = seed + blockIdx.x * 77u + c;
    }
    const uint32_t m = 0xD2511F53u ^ seed;
    const uint64_t mm = ((uint64_t)m << 32) | (m ^ 0x5bd1e995u);
    uint64_t lm[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        lm[c] = __builtin_amdgcn_uicmp(a[c], b[c], 36);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (W == MAD_U64_U32) {
                uint64_t acc = ((uint64_t)b[c] << 32) | a[c];
                asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(acc) : "v"(a[c]), "v"(m) : "vcc");
                a[c] = (uint32_t)acc;
                b[c] = (uint32_t)(acc >> 32);
            } else if constexpr (W == MUL_HI_U32) {
                asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[c]) : "v"(m));
            } else if constexpr (W == MUL_LO_U32) {
                asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[c]) : "v"(m));
            } else if constexpr (W == BITOP3) {
                asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[c]) : "v"(b[c]), "v"(m));
            } else if constexpr (W == XOR) {
                asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[c]) : "v"(b[c]));
            } else if constexpr (W == ADD) {
                asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[c]) : "v"(b[c]));
            } else if constexpr (W == LSHL_ADD_U64) {
                uint64_t acc = ((uint64_t)b[c] << 32) | a[c];
                asm volatile("v_lshl_add_u64 %0, %0, 0, %1" : "+v"(acc) : "v"(mm));
                a[c] = (uint32_t)acc;
                b[c] = (uint32_t)(acc >> 32);
            } else if constexpr (W == ADDC) {
                asm volatile("v_addc_co_u32_e64 %0, %1, %0, %0, %1" : "+v"(a[c]), "+s"(lm[c]));
            } else if constexpr (W == CMP) {
                asm volatile("v_cmp_lt_u32_e64 %0, %1, %2" : "=s"(lm[c]) : "v"(a[c]), "v"(b[c]));
                a[c] += (uint32_t)lm[c];
            } else if constexpr (W == BFE) {
                asm volatile("v_bfe_i32 %0, %0, 7, 1" : "+v"(a[c]));
            } else if constexpr (W == ALIGNBIT) {
                asm volatile("v_alignbit_b32 %0, %0, %1, 31" : "+v"(a[c]) : "v"(b[c]));
            } else if constexpr (W == CNDMASK) {
                asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(a[c]) : "v"(b[c]), "s"(lm[c]));
            }
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        r ^= a[c] ^ b[c] ^ (uint32_t)lm[c] ^ (uint32_t)(lm[c] >> 32);
    out[blockIdx.x * 256 + threadIdx.x] = r;
}

// Philox4x32-10 throughput: calls per second (each thread: 4 independent calls per iteration)
__global__ __launch_bounds__(256) void k_philox(uint32_t *out, uint32_t seed, int iters)
{
    uint32_t acc = 0;
    const uint32_t base = blockIdx.x * 256u + threadIdx.x;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            uint32_t x0 = base * 4u + c, x1 = (uint32_t)i, x2 = 7u, x3 = 0u;
            uint32_t k0 = seed, k1 = seed * 3u;
#pragma unroll
            for (int rnd = 0; rnd < 10; ++rnd) {
                const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
                const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
                const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), x1, k0, 0x96);
                const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), x3, k1, 0x96);
                x1 = (uint32_t)p1;
                x3 = (uint32_t)p0;
                x0 = n0;
                x2 = n2;
                k0 += 0x9E3779B9u;
                k1 += 0xBB67AE85u;
            }
            acc += x0 ^ x1 ^ x2 ^ x3;
        }
    }
    out[base] = acc;
}

// Shader-clock and real-time stamps around a chain of v_xor_b32 (lane 0 of each
// wave records both), to measure the shader clock and the per-SIMD issue rate.
__global__ __launch_bounds__(256) void k_clock(uint64_t *stamps, uint32_t *out, int iters)
{
    uint32_t a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        a[c] = threadIdx.x * 3u + c;
    const uint32_t b = blockIdx.x ^ 0x5bd1e995u;
    const uint64_t c0 = clock64();
    const uint64_t w0 = wall_clock64();
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c)
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[c]) : "v"(b));
    }
    const uint64_t c1 = clock64();
    const uint64_t w1 = wall_clock64();
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        r ^= a[c];
    out[blockIdx.x * 256 + threadIdx.x] = r;
    if ((threadIdx.x & 63) == 0) {
        const uint32_t wave = blockIdx.x * 4 + (threadIdx.x >> 6);
        stamps[4 * wave + 0] = c1 - c0;
        stamps[4 * wave + 1] = w1 - w0;
        stamps[4 * wave + 2] = c0;
        stamps[4 * wave + 3] = w0;
    }
}

// The sweep's per-word arithmetic with no memory traffic: every thread
// updates two register-resident words per iteration with ising::update_word
// (classification, Philox, acceptance) from synthetic neighbour words and a
// fresh counter per word and iteration; the results are XOR-accumulated, so no
// update waits for the previous one.  THREADS and the occupancy hint match the
// sweep kernels (256 threads as the streaming kernel; 1024 threads with at most
// four waves per SIMD as the LDS-resident kernel).  Sites per second of the
// faster shape is the measured ALU ceiling of the sweep's instruction mix
// (thresholds of T_c).  With `bonds` 0 the neighbour words are unrelated to
// the spin word, so half of the bonds are anti-aligned; with 1 each neighbour
// word differs from the spin word in about 1/8 of its bits (the AND of three
// hashed words), close to the 0.146 of the 2D model at T_c.  The site
// contract's cost does not depend on the bonds; the bit-sliced contract's
// lazy comparison runs until the wave's last undecided site is decided, and
// far more sites are undecided (at most one anti-aligned neighbour) in an
// ordered lattice than in random words.
__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    // the finaliser of Steele, Lea and Flood's SplitMix64 (OOPSLA 2014)
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

template <typename Word, bool BITSLICED, int THREADS>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(1, THREADS >= 1024 ? 4 : 8)))
void k_mix(uint32_t *out, uint32_t seed, int iters, uint32_t thr4, uint32_t thr8, int bonds)
{
    using ising::SweepKey;
    const uint32_t tid = blockIdx.x * (uint32_t)THREADS + threadIdx.x;
    SweepKey K;
    K.k0 = seed;
    K.k1 = seed * 3u + 1u;
    K.t = 0;
    K.replica = blockIdx.x;
    K.colour = 1u;
    K.thr4 = thr4;
    K.thr8 = thr8;
    K.always = 0u;
    K.rng = BITSLICED ? 1u : 0u;
    const Word s0 = (Word)(tid * 0x9E3779B97F4A7C15ull), s1 = (Word)(tid * 0xD6E8FEB86659FD93ull);
    const Word up = (Word)(tid * 0xC2B2AE3D27D4EB4Full), dn = (Word)(tid * 0x165667B19E3779F9ull);
    const Word same = (Word)(tid * 0x27D4EB2F165667C5ull);
    const Word side = same ^ up;
    // anti-aligned bits of the four neighbours when bonds = 1
    Word m[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t h = 4u * (uint64_t)tid + (uint64_t)k;
        m[k] = (Word)(mix64(3 * h + 1) & mix64(3 * h + 2) & mix64(3 * h + 3));
    }
    constexpr uint32_t QW = ising::WordTraits<Word>::BITS / 4;
    Word acc = 0;
    for (int i = 0; i < iters; ++i) {
        K.t = (uint32_t)i;
        const Word v = (Word)(uint32_t)i * (Word)0x9E3779B9u;
        const uint32_t q = (2u * tid + (uint32_t)i * 0x200000u) * QW;
        const Word a = s0 ^ v, b = s1 ^ v;
        if (bonds) {
            Word na[4], nb[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                na[k] = a ^ m[k];
                nb[k] = b ^ m[k ^ 1];
            }
            // opaque to the compiler (an empty statement, no instruction):
            // otherwise it folds s ^ (s ^ m) to m and hoists the
            // classification out of the loop, work the sweep cannot skip
            asm volatile("" : "+v"(na[0]), "+v"(na[1]), "+v"(na[2]), "+v"(na[3]));
            asm volatile("" : "+v"(nb[0]), "+v"(nb[1]), "+v"(nb[2]), "+v"(nb[3]));
            acc ^= ising::update_word<Word, BITSLICED>(a, na[0], na[1], na[2], na[3], q, K);
            acc ^= ising::update_word<Word, BITSLICED>(b, nb[0], nb[1], nb[2], nb[3], q + QW, K);
        } else {
            acc ^= ising::update_word<Word, BITSLICED>(a, up, dn, same, side, q, K);
            acc ^= ising::update_word<Word, BITSLICED>(b, dn, up, side, same, q + QW, K);
        }
    }
    out[tid] = (uint32_t)acc ^ (uint32_t)((uint64_t)acc >> 32);
}

// The 3D sweep's per-word arithmetic (six-input classification, Philox,
// three-threshold acceptance) on register-resident words.
template <bool BITSLICED, bool BONDS>
__global__ __launch_bounds__(256) void k_mix3(uint32_t *out, uint32_t seed, int iters, uint32_t thr4, uint32_t thr8,
                                              uint32_t thr12)
{
    const uint32_t tid = blockIdx.x * 256u + threadIdx.x;
    ising::Key3 K;
    K.k0 = seed;
    K.k1 = seed * 3u + 1u;
    K.t = 0;
    K.replica = blockIdx.x;
    K.colour = 1u;
    K.thr4 = thr4;
    K.thr8 = thr8;
    K.thr12 = thr12;
    K.always = 0u;
    uint32_t s = tid * 0x9E3779B9u;
    uint32_t n[6] = {tid * 0xC2B2AE3Du, tid * 0x165667B1u, tid * 0x27D4EB2Fu, tid * 0x85EBCA77u, tid * 0x7FEB352Du,
                     tid * 0x846CA68Bu};
    // BONDS: neighbour k differs from the spin word where m[k] is set, in
    // about 11/32 of the bits ((h1 & h2) | (h3 & h4 & h5)), close to the 0.33
    // of the 3D model near its T_c
    uint32_t m[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const uint64_t h = 8u * (uint64_t)(6u * tid + (uint32_t)k);
        m[k] = (uint32_t)((mix64(h + 1) & mix64(h + 2)) | (mix64(h + 3) & mix64(h + 4) & mix64(h + 5)));
    }
    for (int i = 0; i < iters; ++i) {
        K.t = (uint32_t)i;
        const uint32_t c = (tid + (uint32_t)i * 0x100000u) * 8u;
        if constexpr (BONDS) {
            uint32_t nn[6];
#pragma unroll
            for (int k = 0; k < 6; ++k)
                nn[k] = s ^ m[k];
            // opaque (no instruction): keeps s ^ (s ^ m) from folding to m
            asm volatile("" : "+v"(nn[0]), "+v"(nn[1]), "+v"(nn[2]), "+v"(nn[3]), "+v"(nn[4]), "+v"(nn[5]));
            s ^= BITSLICED ? ising::flip_mask32_3d_bitsliced(s, nn, c, K) : ising::flip_mask32_3d(s, nn, c, K);
        } else {
            s ^= BITSLICED ? ising::flip_mask32_3d_bitsliced(s, n, c, K) : ising::flip_mask32_3d(s, n, c, K);
        }
    }
    out[tid] = s;
}

__global__ __launch_bounds__(256) void k_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src, size_t n16)
{
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256)
        dst[i] = src[i];
}

// One v_mfma_f32_16x16x32_bf16 with per-lane operands exactly as given
// (a, b: 64 lanes x 8 bf16 bit patterns; out: 64 lanes x 4 floats), to check
// the builtin's lane layout against a host matrix product.
typedef __bf16 probe_bf16x8 __attribute__((ext_vector_type(8)));
typedef float probe_floatx4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(64) void k_mfma_layout(const uint16_t *a, const uint16_t *b, float *out)
{
    const int l = threadIdx.x;
    probe_bf16x8 va, vb;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        va[i] = __builtin_bit_cast(__bf16, a[l * 8 + i]);
        vb[i] = __builtin_bit_cast(__bf16, b[l * 8 + i]);
    }
    probe_floatx4 c = {0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, c, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        out[l * 4 + i] = c[i];
}

// One v_mfma_f32_16x16x4_f32 with per-lane operands as given (a, b: one float
// per lane; out: 64 lanes x 4 floats).
__global__ __launch_bounds__(64) void k_mfma_layout_f32(const float *a, const float *b, float *out)
{
    const int l = threadIdx.x;
    probe_floatx4 c = {0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[l], b[l], c, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        out[l * 4 + i] = c[i];
}

template <int W>
hipError_t run_alu(uint32_t *out, int blocks, int iters, hipStream_t st)
{
    hipLaunchKernelGGL(k_alu<W>, dim3(blocks), dim3(256), 0, st, out, 12345u, iters);
    return hipGetLastError();
}

// Shortest of `reps` timed k_mix launches (after one warm-up launch) in each
// of the two launch shapes.
template <typename Word, bool BITSLICED>
hipError_t mix_best(uint32_t *o, int blocks, int iters, unsigned thr4, unsigned thr8, int bonds, int reps,
                    hipEvent_t e0, hipEvent_t e1, float *best)
{
    hipError_t err = hipSuccess;
    for (int shape = 0; shape < 2 && err == hipSuccess; ++shape) {
        for (int rep = 0; rep <= reps && err == hipSuccess; ++rep) {
            err = hipEventRecord(e0, nullptr);
            if (err != hipSuccess)
                break;
            if (shape == 0)
                hipLaunchKernelGGL((k_mix<Word, BITSLICED, 256>), dim3(blocks), dim3(256), 0, nullptr, o, 12345u,
                                   iters, thr4, thr8, bonds);
            else
                hipLaunchKernelGGL((k_mix<Word, BITSLICED, 1024>), dim3(blocks / 4), dim3(1024), 0, nullptr, o,
                                   12345u, iters, thr4, thr8, bonds);
            err = hipGetLastError();
            if (err == hipSuccess)
                err = hipEventRecord(e1, nullptr);
            if (err == hipSuccess)
                err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess)
                err = hipEventElapsedTime(&ms, e0, e1);
            if (err == hipSuccess && rep > 0 && (*best <= 0.f || ms < *best))
                *best = ms;
        }
    }
    return err;
}

}  // namespace

extern "C" {

/* Measured ALU ceiling of the 3D sweep's per-word arithmetic: k_mix3 over
 * blocks x 256 threads x iters words of 32 sites under contract rng (0 site,
 * 1 bit-sliced), with random neighbour words (bonds 0) or neighbours that
 * differ from the spin word in about 11/32 of the bits (bonds 1); *ms =
 * kernel time. */
int ising_probe_mix3(void *out, int blocks, int iters, unsigned thr4, unsigned thr8, unsigned thr12, int rng,
                     int bonds, float *ms)
{
    if (!out || !ms || blocks <= 0 || iters <= 0 || (rng != 0 && rng != 1) || (bonds != 0 && bonds != 1))
        return -1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return -4;
    uint32_t *o = static_cast<uint32_t *>(out);
    auto launch = [&](uint32_t seed) {
        if (rng && bonds)
            hipLaunchKernelGGL((k_mix3<true, true>), dim3(blocks), dim3(256), 0, nullptr, o, seed, iters, thr4, thr8,
                               thr12);
        else if (rng)
            hipLaunchKernelGGL((k_mix3<true, false>), dim3(blocks), dim3(256), 0, nullptr, o, seed, iters, thr4, thr8,
                               thr12);
        else if (bonds)
            hipLaunchKernelGGL((k_mix3<false, true>), dim3(blocks), dim3(256), 0, nullptr, o, seed, iters, thr4, thr8,
                               thr12);
        else
            hipLaunchKernelGGL((k_mix3<false, false>), dim3(blocks), dim3(256), 0, nullptr, o, seed, iters, thr4,
                               thr8, thr12);
    };
    launch(777u);
    hipError_t st = hipEventRecord(e0, nullptr);
    launch(12345u);
    if (st == hipSuccess)
        st = hipEventRecord(e1, nullptr);
    if (st == hipSuccess)
        st = hipEventSynchronize(e1);
    if (st == hipSuccess)
        st = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st == hipSuccess ? 0 : -4;
}

/* Measured ALU ceiling of the sweep's per-word arithmetic: k_mix with 32- or
 * 64-bit words under the site (rng 0) or bit-sliced (rng 1) random-number
 * contract, in two launch shapes with the same total thread count: blocks x
 * 256 threads, and blocks / 4 x 1024 threads (blocks must be a multiple of 4).
 * Each shape runs one warm-up launch, then `reps` timed launches; *ms receives
 * the shortest timed launch over both shapes.  bonds: 0 neighbour words
 * unrelated to the spin word, 1 neighbour words that differ from it in about
 * 1/8 of the bits (see k_mix).  Sites counted per launch:
 * blocks * 256 * iters * 2 * word_bits.  Returns 0, or <0 on error. */
int ising_probe_mix(int word_bits, void *out, int blocks, int iters, unsigned thr4, unsigned thr8, int rng,
                    int bonds, int reps, float *ms)
{
    if (!out || blocks <= 0 || blocks % 4 != 0 || iters <= 0 || reps <= 0 || !ms ||
        (word_bits != 32 && word_bits != 64) || (rng != 0 && rng != 1) || (bonds != 0 && bonds != 1))
        return -1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return -4;
    uint32_t *o = static_cast<uint32_t *>(out);
    *ms = 0.f;
    hipError_t err;
    if (word_bits == 32 && rng == 0)
        err = mix_best<uint32_t, false>(o, blocks, iters, thr4, thr8, bonds, reps, e0, e1, ms);
    else if (word_bits == 32)
        err = mix_best<uint32_t, true>(o, blocks, iters, thr4, thr8, bonds, reps, e0, e1, ms);
    else if (rng == 0)
        err = mix_best<uint64_t, false>(o, blocks, iters, thr4, thr8, bonds, reps, e0, e1, ms);
    else
        err = mix_best<uint64_t, true>(o, blocks, iters, thr4, thr8, bonds, reps, e0, e1, ms);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return err == hipSuccess ? 0 : -4;
}

/*
 * Time one probe on the null stream.  which: 0 v_mad_u64_u32, 1 v_mul_hi_u32,
 * 2 v_mul_lo_u32, 3 v_bitop3_b32, 4 v_xor_b32, 5 v_add_u32, 6 full Philox4x32-10.
 * out: device buffer of blocks*256 uint32.  Returns 0 and the elapsed
 * milliseconds of the timed launch (after one warm-up launch), <0 on error.
 * Operations counted: blocks*256*iters*8 instructions (which 0..5, 7..12) or
 * blocks*256*iters*4 Philox calls (which 6).  The compare probe (9) also
 * issues one v_add_u32 per compare to keep its chains dependent.
 */
int ising_probe_alu(int which, void *out, int blocks, int iters, float *ms)
{
    if (!out || blocks <= 0 || iters <= 0 || !ms)
        return -1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return -4;
    uint32_t *o = static_cast<uint32_t *>(out);
    hipError_t err = hipSuccess;
    for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
        if (rep == 1)
            err = hipEventRecord(e0, nullptr);
        if (err != hipSuccess)
            break;
        switch (which) {
        case MAD_U64_U32: err = run_alu<MAD_U64_U32>(o, blocks, iters, nullptr); break;
        case MUL_HI_U32: err = run_alu<MUL_HI_U32>(o, blocks, iters, nullptr); break;
        case MUL_LO_U32: err = run_alu<MUL_LO_U32>(o, blocks, iters, nullptr); break;
        case BITOP3: err = run_alu<BITOP3>(o, blocks, iters, nullptr); break;
        case XOR: err = run_alu<XOR>(o, blocks, iters, nullptr); break;
        case ADD: err = run_alu<ADD>(o, blocks, iters, nullptr); break;
        case LSHL_ADD_U64: err = run_alu<LSHL_ADD_U64>(o, blocks, iters, nullptr); break;
        case ADDC: err = run_alu<ADDC>(o, blocks, iters, nullptr); break;
        case CMP: err = run_alu<CMP>(o, blocks, iters, nullptr); break;
        case BFE: err = run_alu<BFE>(o, blocks, iters, nullptr); break;
        case ALIGNBIT: err = run_alu<ALIGNBIT>(o, blocks, iters, nullptr); break;
        case CNDMASK: err = run_alu<CNDMASK>(o, blocks, iters, nullptr); break;
        case PHILOX:
            hipLaunchKernelGGL(k_philox, dim3(blocks), dim3(256), 0, nullptr, o, 12345u, iters);
            err = hipGetLastError();
            break;
        default: err = hipErrorInvalidValue;
        }
    }
    if (err == hipSuccess)
        err = hipEventRecord(e1, nullptr);
    if (err == hipSuccess)
        err = hipEventSynchronize(e1);
    if (err == hipSuccess)
        err = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return err == hipSuccess ? 0 : -4;
}

/*
 * Clock probe: blocks*4 waves each run iters*8 dependent-free v_xor_b32; for
 * every wave, stamps[4w..4w+3] = {shader cycles, wall ticks, start cycle,
 * start wall tick} (wall ticks from the constant-rate real-time counter).
 * stamps: device buffer of blocks*4*4 uint64; out: blocks*256 uint32.
 * *ms: event-timed duration of the launch; *wall_khz: the real-time
 * counter's rate reported by the runtime.
 */
int ising_probe_clock(void *stamps, void *out, int blocks, int iters, float *ms, int *wall_khz)
{
    if (!stamps || !out || blocks <= 0 || iters <= 0 || !ms || !wall_khz)
        return -1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        return -4;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return -4;
    hipError_t err = hipEventRecord(e0, nullptr);
    if (err == hipSuccess) {
        hipLaunchKernelGGL(k_clock, dim3(blocks), dim3(256), 0, nullptr, static_cast<uint64_t *>(stamps),
                           static_cast<uint32_t *>(out), iters);
        err = hipGetLastError();
    }
    if (err == hipSuccess)
        err = hipEventRecord(e1, nullptr);
    if (err == hipSuccess)
        err = hipEventSynchronize(e1);
    if (err == hipSuccess)
        err = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return err == hipSuccess ? 0 : -4;
}

/* One MFMA 16x16x32 bf16 on device buffers a, b (64*8 uint16 each) -> out (64*4 float). */
int ising_probe_mfma_layout(const void *a, const void *b, void *out)
{
    if (!a || !b || !out)
        return -1;
    hipLaunchKernelGGL(k_mfma_layout, dim3(1), dim3(64), 0, nullptr, static_cast<const uint16_t *>(a),
                       static_cast<const uint16_t *>(b), static_cast<float *>(out));
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return -4;
    return 0;
}

int ising_probe_mfma_layout_f32(const void *a, const void *b, void *out)
{
    if (!a || !b || !out)
        return -1;
    hipLaunchKernelGGL(k_mfma_layout_f32, dim3(1), dim3(64), 0, nullptr, static_cast<const float *>(a),
                       static_cast<const float *>(b), static_cast<float *>(out));
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return -4;
    return 0;
}

/* Copy bytes (a multiple of 16) from src to dst `reps` times; elapsed ms of all reps. */
int ising_probe_copy(void *dst, const void *src, size_t bytes, int reps, float *ms)
{
    if (!dst || !src || bytes % 16 != 0 || reps <= 0 || !ms)
        return -1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return -4;
    const size_t n16 = bytes / 16;
    hipError_t err = hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps && err == hipSuccess; ++r) {
        hipLaunchKernelGGL(k_copy, dim3(4096), dim3(256), 0, nullptr, static_cast<uint4 *>(dst),
                           static_cast<const uint4 *>(src), n16);
        err = hipGetLastError();
    }
    if (err == hipSuccess)
        err = hipEventRecord(e1, nullptr);
    if (err == hipSuccess)
        err = hipEventSynchronize(e1);
    if (err == hipSuccess)
        err = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return err == hipSuccess ? 0 : -4;
}

}  // extern "C"
