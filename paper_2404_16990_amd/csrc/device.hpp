// Device-side building blocks shared by the sweep, init and observable kernels.
//
// Layout of one replica in device memory (1 bit per spin, bit 1 <=> s = +1):
//   plane c (c = colour 0 red, 1 blue) holds Ly rows of W = Lx/64 uint32 words;
//   bit b of word w in row y is the site with compact index k = 32 w + b of
//   that colour in that row, i.e. column x = 2 k + ((c + y) & 1).
//   Plane 1 follows plane 0 directly.  A 64-bit word w' is the pair of 32-bit
//   words (2w', 2w'+1), little-endian, so 32- and 64-bit access see the same
//   bytes.
// This replaces the paper's eight int16 arrays with domain folding (section 2,
// Eq. 1 and Fig. 3), which exist to keep periodic neighbours on adjacent
// processing elements; global memory and LDS need no such adjacency.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

// Per-replica device descriptor (64 bytes), written by the host at create and
// by set_* calls; t and t0 are advanced on the device by the run kernels.
struct RepDev {
    uint32_t *plane0;   // colour-0 plane; colour-1 plane = plane0 + Ly * W
    uint32_t Lx, Ly, W; // W = 32-bit words per colour row = Lx / 64
    uint32_t seed_lo, seed_hi, replica;
    uint32_t always;    // 1 when beta*J == 0: every proposal is accepted
    uint32_t thr4, thr8;  // acceptance thresholds for dE = 4J and 8J
    uint32_t t;         // sweeps completed
    uint32_t t0;        // value of t when the current run started
    uint32_t rng;       // random-number contract: 0 one word per site, 1 bit-sliced groups
    uint64_t N;         // Lx * Ly
};
static_assert(sizeof(RepDev) == 64, "descriptor must stay 64 bytes");

// Where fused observables of recorded sweeps go.
struct RecArgs {
    int64_t *bond;   // [n_replicas * n_rec] or null
    int64_t *mag;
    uint32_t every;  // 0 = no recording
    uint32_t n_rec;
};

template <typename Word> struct WordTraits;
template <> struct WordTraits<uint32_t> { static constexpr int BITS = 32; static constexpr int PER32 = 1; };
template <> struct WordTraits<uint64_t> { static constexpr int BITS = 64; static constexpr int PER32 = 2; };

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ---------------------
// Each round: two 32x32->64-bit products (v_mad_u64_u32), the high halves
// XORed with the other two counter words and the round key in one 3-input
// bitwise op (v_bitop3_b32 with truth table 0x96 = a ^ b ^ c).  Key words are
// wave-uniform and stay in scalar registers.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Everything the update of one colour of one sweep of one replica needs
// besides the spins (all wave-uniform).
struct SweepKey {
    uint32_t k0, k1, t, replica, colour, thr4, thr8, always, rng;
};

__device__ __forceinline__ SweepKey make_key(const RepDev &d, uint32_t t, uint32_t colour)
{
    SweepKey k;
    k.k0 = d.seed_lo;
    k.k1 = d.seed_hi;
    k.t = t;
    k.replica = d.replica;
    k.colour = colour;
    k.thr4 = d.thr4;
    k.thr8 = d.thr8;
    k.always = d.always;
    k.rng = d.rng;
    return k;
}

// acc * 2 + (bit of this lane in the lane mask): the carry-in form of
// v_addc_co_u32 reads a compare result directly.  Written as one instruction
// because the compiler otherwise rewrites the shift-and-add chain into
// v_cndmask / shift / or sequences that cost more issue slots.
__device__ __forceinline__ uint32_t shift_in_carry(uint32_t acc, uint64_t lanemask)
{
    uint32_t out;
    uint64_t carry_out;
    asm("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(out), "=s"(carry_out) : "v"(acc), "s"(lanemask));
    return out;
}

// Classes of the 32 sites of a word by the number of anti-aligned neighbours
// (a_k = s ^ n_k), counted with two half adders: ge2 (two or more: dE <= 0)
// and eq1 (exactly one: dE = 4J); the rest have none (dE = 8J).
struct Classes {
    uint32_t ge2, eq1;
};

__device__ __forceinline__ Classes classify(uint32_t s, uint32_t up, uint32_t dn, uint32_t same, uint32_t side)
{
    const uint32_t a1 = s ^ up, a2 = s ^ dn, a3 = s ^ same, a4 = s ^ side;
    const uint32_t s1 = a1 ^ a2, c1 = a1 & a2;
    const uint32_t s2 = a3 ^ a4, c2 = a3 & a4;
    Classes c;
    c.ge2 = c1 | c2 | (s1 & s2);
    c.eq1 = (s1 ^ s2) & ~(c1 | c2);
    return c;
}

// Neighbour classification and Metropolis acceptance for one 32-bit word of
// same-colour spins (the multi-spin idea of the paper's Algorithm 2,
// flipQuarter, restated for 1-bit words):
//   a_k = s ^ n_k marks spins anti-aligned with neighbour k;
//   two half adders give per-bit partial sums (s1, c1), (s2, c2);
//   >= 2 anti-aligned neighbours  <=> dE <= 0   -> flip unconditionally;
//   exactly one                   <=> dE = 4J   -> flip iff r < thr4;
//   none                          <=> dE = 8J   -> flip iff r < thr8.
// q0 = Philox counter word of the word's first four sites (sites 4j..4j+3 of
// the word use call q0 + j).  Returns the mask of spins to flip.
__device__ __forceinline__ uint32_t flip_mask32(uint32_t s, uint32_t up, uint32_t dn, uint32_t same,
                                                uint32_t side, uint32_t q0, const SweepKey &K)
{
    const Classes cl = classify(s, up, dn, same, side);
    const uint32_t ge2 = cl.ge2, eq1 = cl.eq1;
    // Acceptance in four instructions per site: broadcast the site's class bit
    // (v_bfe_i32), select its threshold (v_bitop3, table 0xCA = m ? thr4 :
    // thr8), compare r < thr into a lane mask (v_cmp_lt_u32), and shift that
    // lane's bit of the mask into the accumulator as a carry (acc + acc + c,
    // v_addc_co_u32).  Sites are visited from bit 31 down so each lands at its
    // own position.
    const uint32_t thr4 = __builtin_amdgcn_readfirstlane(K.thr4);
    uint32_t acc = 0;
#pragma unroll
    for (int q = 7; q >= 0; --q) {
        uint32_t r[4];
        philox4x32_10(q0 + q, K.t, K.replica, K.colour, K.k0, K.k1, r);
#pragma unroll
        for (int j = 3; j >= 0; --j) {
            const int b = 4 * q + j;
            const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int32_t)eq1, b, 1);
            const uint32_t t = __builtin_amdgcn_bitop3_b32(m, thr4, K.thr8, 0xCA);
            acc = shift_in_carry(acc, __builtin_amdgcn_uicmp(r[j], t, 36 /* unsigned < */));
        }
    }
    return ge2 | acc;
}

// Acceptance under the bit-sliced random-number contract for NH groups of 32
// sites (the 32-bit halves of one word; group h uses Philox counters
// c0 + 8h + m, m = 0..7, whose four words are W_4m .. W_4m+3).  A site's
// uniform has bit 31 - k equal to its bit of W_k, so it is compared with its
// threshold (thr4 for eq1 sites, thr8 for the others) from the top bit down:
// at level k an undecided site whose uniform bit is 0 where the threshold bit
// is 1 is accepted, and every site whose two bits differ is decided.  Words
// are drawn four at a time and drawing stops once no lane of the wave has an
// undecided site, so the result equals the full comparison.
template <int NH>
__device__ __forceinline__ void bitsliced_accept(const uint32_t (&undecided)[NH], const uint32_t (&eq1)[NH],
                                                 uint32_t c0, const SweepKey &K, uint32_t (&acc)[NH])
{
    uint32_t und[NH], any = 0;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        und[h] = undecided[h];
        acc[h] = 0;
        any |= und[h];
    }
    const uint32_t thr4 = __builtin_amdgcn_readfirstlane(K.thr4), thr8 = __builtin_amdgcn_readfirstlane(K.thr8);
    if (thr4 == 0u)  // thr8 <= thr4 = 0: no proposal with dE > 0 is accepted
        return;
    if (__builtin_amdgcn_ballot_w64(any != 0u) == 0)
        return;
    for (int m = 0; m < 8; ++m) {
        uint32_t w[NH][4];
#pragma unroll
        for (int h = 0; h < NH; ++h)
            philox4x32_10(c0 + 8u * h + m, K.t, K.replica, K.colour, K.k0, K.k1, w[h]);
        any = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * m + j;
            const uint32_t m4 = 0u - ((thr4 >> (31 - k)) & 1u), m8 = 0u - ((thr8 >> (31 - k)) & 1u);
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                const uint32_t q = __builtin_amdgcn_bitop3_b32(eq1[h], m4, m8, 0xCA);  // threshold bit k
                acc[h] |= und[h] & ~w[h][j] & q;
                und[h] &= ~(w[h][j] ^ q);
            }
        }
#pragma unroll
        for (int h = 0; h < NH; ++h)
            any |= und[h];
        if (__builtin_amdgcn_ballot_w64(any != 0u) == 0)
            break;
    }
}

// Horizontal neighbour word of the other colour (the paper's Algorithm 1,
// getBitAbove / getBitBelow, as a funnel shift).  For a target word in a row
// whose colour-c sites sit at odd columns (p = 1) the second horizontal
// neighbour of bit k is bit k + 1 of the other plane, taken from the next word
// nb at the top; for p = 0 it is bit k - 1, taken from the previous word nb.
// Each 32-bit half is one funnel shift (v_alignbit_b32) of two 32-bit words.
template <typename Word>
__device__ __forceinline__ Word side_word(Word same, Word nb, uint32_t p)
{
    if constexpr (WordTraits<Word>::BITS == 32) {
        const uint32_t from_next = __builtin_amdgcn_alignbit(nb, same, 1);   // same >> 1 | nb << 31
        const uint32_t from_prev = __builtin_amdgcn_alignbit(same, nb, 31);  // same << 1 | nb >> 31
        return p ? from_next : from_prev;
    } else {
        const uint32_t sl = (uint32_t)same, sh = (uint32_t)(same >> 32);
        const uint32_t nl = (uint32_t)nb, nh = (uint32_t)(nb >> 32);
        const uint32_t next_lo = __builtin_amdgcn_alignbit(sh, sl, 1), next_hi = __builtin_amdgcn_alignbit(nl, sh, 1);
        const uint32_t prev_lo = __builtin_amdgcn_alignbit(sl, nh, 31), prev_hi = __builtin_amdgcn_alignbit(sh, sl, 31);
        const uint32_t lo = p ? next_lo : prev_lo, hi = p ? next_hi : prev_hi;
        return ((uint64_t)hi << 32) | lo;
    }
}

// Update of one Word (32 or 64 spins) given its neighbour words; a 64-bit
// word is two independent 32-bit halves (sites 0..31 and 32..63).
// BITSLICED selects the random-number contract at compile time (the kernels
// branch once per workgroup on the replica's contract), so each contract's
// loop is compiled on its own.
template <typename Word, bool BITSLICED = false>
__device__ __forceinline__ Word update_word(Word s, Word up, Word dn, Word same, Word side, uint32_t q0,
                                            const SweepKey &K)
{
    if (K.always)
        return ~s;
    if constexpr (BITSLICED) {
        constexpr int NH = WordTraits<Word>::BITS / 32;
        uint32_t und[NH], eq1[NH], ge2[NH], acc[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const Classes c = classify((uint32_t)(s >> (32 * h)), (uint32_t)(up >> (32 * h)),
                                       (uint32_t)(dn >> (32 * h)), (uint32_t)(same >> (32 * h)),
                                       (uint32_t)(side >> (32 * h)));
            ge2[h] = c.ge2;
            eq1[h] = c.eq1;
            und[h] = ~c.ge2;
        }
        bitsliced_accept<NH>(und, eq1, q0, K, acc);
        Word flip = 0;
#pragma unroll
        for (int h = 0; h < NH; ++h)
            flip |= (Word)(ge2[h] | acc[h]) << (32 * h);
        return s ^ flip;
    }
    if constexpr (WordTraits<Word>::BITS == 32) {
        return s ^ flip_mask32(s, up, dn, same, side, q0, K);
    } else {
        const uint32_t lo = flip_mask32((uint32_t)s, (uint32_t)up, (uint32_t)dn, (uint32_t)same,
                                        (uint32_t)side, q0, K);
        const uint32_t hi = flip_mask32((uint32_t)(s >> 32), (uint32_t)(up >> 32), (uint32_t)(dn >> 32),
                                        (uint32_t)(same >> 32), (uint32_t)(side >> 32), q0 + 8, K);
        return s ^ (((uint64_t)hi << 32) | lo);
    }
}

// Number of anti-aligned bonds touching the (already updated) word s.
template <typename Word>
__device__ __forceinline__ uint32_t anti_bonds(Word s, Word up, Word dn, Word same, Word side)
{
    return (uint32_t)(__popcll((uint64_t)(s ^ up)) + __popcll((uint64_t)(s ^ dn)) +
                      __popcll((uint64_t)(s ^ same)) + __popcll((uint64_t)(s ^ side)));
}

// Indices of the neighbour words of word (y, w) in a plane of Ly rows x Wn
// words, periodic in both directions, without branches.
struct NeighIdx {
    uint32_t same, up, dn, nb, p;
};

__device__ __forceinline__ NeighIdx neigh_idx(uint32_t y, uint32_t w, uint32_t Ly, uint32_t Wn, uint32_t colour)
{
    NeighIdx n;
    const uint32_t yu = y == 0 ? Ly - 1 : y - 1;
    const uint32_t yd = y + 1 == Ly ? 0 : y + 1;
    const uint32_t wp = w + 1 == Wn ? 0 : w + 1;
    const uint32_t wm = w == 0 ? Wn - 1 : w - 1;
    n.p = (colour + y) & 1u;
    n.same = y * Wn + w;
    n.up = yu * Wn + w;
    n.dn = yd * Wn + w;
    n.nb = y * Wn + (n.p ? wp : wm);
    return n;
}

__device__ __forceinline__ int64_t wave_sum(int64_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        v += __shfl_xor(v, m, 64);
    return v;
}

}  // namespace ising
