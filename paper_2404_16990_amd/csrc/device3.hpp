// Per-word arithmetic of the 3D (simple cubic) sweep, shared by the sweep
// kernel (ising3d.hip) and the instruction-mix probe (probe.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "ising3d.hpp"

namespace ising {

// Everything one colour of one sweep of one replica needs besides the spins.
struct Key3 {
    uint32_t k0, k1, t, replica, colour, thr4, thr8, thr12, always;
};

__device__ __forceinline__ Key3 key3(const Rep3Dev &d, uint32_t t, uint32_t colour)
{
    Key3 K;
    K.k0 = d.seed_lo;
    K.k1 = d.seed_hi;
    K.t = t;
    K.replica = d.replica;
    K.colour = colour;
    K.thr4 = d.thr4;
    K.thr8 = d.thr8;
    K.thr12 = d.thr12;
    K.always = d.flags & k3Always;
    return K;
}

// Classes of the 32 sites of a word by the number a of anti-aligned
// neighbours among six, counted by full adders: a >= 3 (dE <= 0), a = 2
// (dE = 4J), a = 1 (dE = 8J); the rest (a = 0) have dE = 12J.
struct Classes3 {
    uint32_t ge3, eq2, eq1;
};

__device__ __forceinline__ Classes3 classify6(uint32_t s, const uint32_t (&n)[6])
{
    const uint32_t a0 = s ^ n[0], a1 = s ^ n[1], a2 = s ^ n[2];
    const uint32_t a3 = s ^ n[3], a4 = s ^ n[4], a5 = s ^ n[5];
    const uint32_t s1 = __builtin_amdgcn_bitop3_b32(a0, a1, a2, 0x96), c1 = __builtin_amdgcn_bitop3_b32(a0, a1, a2, 0xE8);
    const uint32_t s2 = __builtin_amdgcn_bitop3_b32(a3, a4, a5, 0x96), c2 = __builtin_amdgcn_bitop3_b32(a3, a4, a5, 0xE8);
    const uint32_t b0 = s1 ^ s2, k0 = s1 & s2;  // a = b0 + 2 (c1 + c2 + k0)
    const uint32_t b1 = __builtin_amdgcn_bitop3_b32(c1, c2, k0, 0x96), b2 = __builtin_amdgcn_bitop3_b32(c1, c2, k0, 0xE8);
    Classes3 c;
    c.ge3 = b2 | (b1 & b0);
    c.eq2 = ~b2 & b1 & ~b0;
    c.eq1 = ~b2 & ~b1 & b0;
    return c;
}

// Sites to flip in a colour-c word (site contract: site 32 w + b of the row
// draws word (h & 3) of call h >> 2, h = row * Lx / 2 + 32 w + b; q0 is the
// call of bit 0).  The threshold of a site is selected from its class bits
// with two v_bitop3 (eq2 ? thr4 : eq1 ? thr8 : thr12) and compared into a lane
// mask that is shifted into the accumulator as a carry (bits 31 down to 0).
__device__ __forceinline__ uint32_t flip_mask32_3d(uint32_t s, const uint32_t (&n)[6], uint32_t q0, const Key3 &K)
{
    if (K.always)
        return ~0u;
    const Classes3 cl = classify6(s, n);
    const uint32_t thr4 = __builtin_amdgcn_readfirstlane(K.thr4), thr8 = __builtin_amdgcn_readfirstlane(K.thr8);
    const uint32_t thr12 = __builtin_amdgcn_readfirstlane(K.thr12);
    uint32_t acc = 0;
#pragma unroll
    for (int q = 7; q >= 0; --q) {
        uint32_t r[4];
        philox4x32_10(q0 + q, K.t, K.replica, K.colour, K.k0, K.k1, r);
#pragma unroll
        for (int j = 3; j >= 0; --j) {
            const int b = 4 * q + j;
            const uint32_t m2 = (uint32_t)__builtin_amdgcn_sbfe((int32_t)cl.eq2, b, 1);
            const uint32_t m1 = (uint32_t)__builtin_amdgcn_sbfe((int32_t)cl.eq1, b, 1);
            const uint32_t thr = __builtin_amdgcn_bitop3_b32(m2, thr4, __builtin_amdgcn_bitop3_b32(m1, thr8, thr12, 0xCA),
                                                             0xCA);
            acc = shift_in_carry(acc, __builtin_amdgcn_uicmp(r[j], thr, 36 /* unsigned < */));
        }
    }
    return cl.ge3 | acc;
}

// Sites to flip in a colour-c word under the bit-sliced contract: the word's
// 32 sites are one group (counters c0 + m, m = 0..7, c0 = 8 x the word's
// index in its plane), each site's uniform is compared with its threshold
// (eq2: thr4, eq1: thr8, otherwise thr12) from the top bit down, and words are
// drawn four at a time until no lane of the wave has an undecided site, so the
// result equals the full comparison.
__device__ __forceinline__ uint32_t flip_mask32_3d_bitsliced(uint32_t s, const uint32_t (&n)[6], uint32_t c0,
                                                             const Key3 &K)
{
    if (K.always)
        return ~0u;
    const Classes3 cl = classify6(s, n);
    const uint32_t thr4 = __builtin_amdgcn_readfirstlane(K.thr4), thr8 = __builtin_amdgcn_readfirstlane(K.thr8);
    const uint32_t thr12 = __builtin_amdgcn_readfirstlane(K.thr12);
    uint32_t und = ~cl.ge3, acc = 0;
    if (thr4 == 0u)  // thr12 <= thr8 <= thr4 = 0: no proposal with dE > 0 is accepted
        return cl.ge3;
    if (__builtin_amdgcn_ballot_w64(und != 0u) == 0)
        return cl.ge3;
    for (int m = 0; m < 8; ++m) {
        uint32_t w[4];
        philox4x32_10(c0 + m, K.t, K.replica, K.colour, K.k0, K.k1, w);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * m + j;
            const uint32_t m4 = 0u - ((thr4 >> (31 - k)) & 1u), m8 = 0u - ((thr8 >> (31 - k)) & 1u);
            const uint32_t m12 = 0u - ((thr12 >> (31 - k)) & 1u);
            // threshold bit k of every site: eq2 ? thr4 : eq1 ? thr8 : thr12
            const uint32_t q = __builtin_amdgcn_bitop3_b32(cl.eq2, m4, __builtin_amdgcn_bitop3_b32(cl.eq1, m8, m12, 0xCA),
                                                           0xCA);
            acc |= und & ~w[j] & q;
            und &= ~(w[j] ^ q);
        }
        if (__builtin_amdgcn_ballot_w64(und != 0u) == 0)
            break;
    }
    return cl.ge3 | acc;
}

}  // namespace ising
