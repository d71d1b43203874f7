// Cluster-step kernels: Swendsen-Wang and Wolff updates (named in paper
// section 1 as the cure for critical slowing down; Swendsen and Wang, PRL 58,
// 86 (1987); Wolff, PRL 62, 361 (1989)) on the packed colour planes of a
// replica batch.  Bonds between aligned neighbours are occupied with
// probability 1 - exp(-2 beta J) (the Fortuin-Kasteleyn representation).
//
// Random words (counter-based, Philox4x32-10 keyed by the replica's seed):
//   bond  right / down bond owned by site g = y*Lx + x: words 2(g&1) and
//         2(g&1)+1 of ctr {g >> 1, t, replica, 7};
//   flip  Swendsen-Wang flips the cluster with root R iff bit R & 31 of word
//         (R >> 5) & 3 of ctr {R >> 7, t, replica, 8} is set;
//   seed  Wolff's seed is ((w0 << 32) | w1) mod (Lx*Ly), w = ctr {0, t, replica, 9}.
// The root of a cluster is its smallest site index.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cluster.hpp"

namespace ising {

namespace {

constexpr uint32_t kRowsPerWave = kClRows / 4;  // 4 waves per 256-thread workgroup

// Global-memory views of pointers that reach the kernels inside descriptors:
// loads through them compile to global (or, when uniform, scalar) loads that
// the compiler can issue back to back instead of flat loads.
typedef __attribute__((address_space(1))) uint32_t gu32;

__device__ __forceinline__ gu32 *global_view(uint32_t *p) { return (gu32 *)p; }
__device__ __forceinline__ const gu32 *global_view(const uint32_t *p) { return (const gu32 *)p; }

// Index of the calling thread's wave in its workgroup, as a wave-uniform value.
__device__ __forceinline__ uint32_t wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// The replica that owns batch-wide tile b: the largest r with prefix[r] <= b
// (wave-uniform; prefix[0] = 0 <= b < prefix[n]).
__device__ __forceinline__ uint32_t tile_owner(const uint32_t *__restrict__ prefix, uint32_t n, uint32_t b)
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

struct Tile {
    uint32_t r;              // replica
    uint32_t lt;             // tile index inside the replica
    uint32_t tx, x0, y0;     // tile column (= word index in a colour row), first column, first row
    uint32_t rows;           // rows in this tile
    uint32_t txn;            // tile column to the right (periodic)
};

__device__ __forceinline__ Tile locate(const ClArgs &a, const RepDev &d, uint32_t r, uint32_t b)
{
    Tile T;
    T.r = r;
    T.lt = b - a.tile_prefix[r];
    const uint32_t ty = T.lt / d.W;
    T.tx = T.lt - ty * d.W;
    T.x0 = 64u * T.tx;
    T.y0 = kClRows * ty;
    T.rows = min(kClRows, d.Ly - T.y0);
    T.txn = T.tx + 1 == d.W ? 0u : T.tx + 1;
    return T;
}

// Position after the last break below column j of a row whose occupied
// right-bond mask is H: the first column of j's horizontal run.
__device__ __forceinline__ uint32_t run_start(uint64_t H, uint32_t j)
{
    const uint64_t breaks = ~H & ((1ull << j) - 1ull);
    return breaks ? 64u - (uint32_t)__clzll(breaks) : 0u;
}

// ---- union-find in LDS (tile-local indices r*64 + j) -----------------------
// Parents only decrease (a root is linked to a smaller index by atomic min),
// so every path is strictly decreasing and every loop below ends.  The label
// array is addressed through an LDS-typed pointer and read with relaxed
// workgroup-scope atomic loads: ds_read, never cached in a register, never the
// flat path.
typedef __attribute__((address_space(3))) uint32_t lu32;

__device__ __forceinline__ uint32_t lds_load(lu32 *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t lds_find(lu32 *L, uint32_t a)
{
    uint32_t p = lds_load(L + a);
    while (p != a) {
        a = p;
        p = lds_load(L + a);
    }
    return a;
}

__device__ __forceinline__ void lds_union(lu32 *L, uint32_t a, uint32_t b)
{
    for (;;) {
        a = lds_find(L, a);
        b = lds_find(L, b);
        if (a == b)
            return;
        if (a > b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        const uint32_t old = __hip_atomic_fetch_min(L + b, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == b)
            return;
        b = old;  // b was linked meanwhile: unite a with its new parent
    }
}

// ---- union-find in the workspace (site indices of one replica) ------------
__device__ __forceinline__ uint32_t ws_load(gu32 *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Union-find in the workspace, up to two unions or four path compressions per
// lane stepped together: each step loads the next node of every walk at once,
// so a lane waits for its longest walk instead of for the sum of them.
// Inactive walks load a valid node (index 0 of the replica) and ignore it.
//
// ws_union2: unite A[k] and B[k] for every k with act[k]: find both roots,
// link the larger to the smaller by atomic min; if the larger was linked
// meanwhile, unite the smaller with its new parent.
__device__ __forceinline__ void ws_union2(gu32 *G, uint32_t (&A)[2], uint32_t (&B)[2], bool (&act)[2])
{
    while (act[0] || act[1]) {
        for (;;) {
            uint32_t qa[2], qb[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                qa[k] = ws_load(G + A[k]);
                qb[k] = ws_load(G + B[k]);
            }
            bool more = false;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (act[k] && qa[k] != A[k]) {
                    A[k] = qa[k];
                    more = true;
                }
                if (act[k] && qb[k] != B[k]) {
                    B[k] = qb[k];
                    more = true;
                }
            }
            if (!more)
                break;
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (!act[k])
                continue;
            if (A[k] == B[k]) {
                act[k] = false;
                continue;
            }
            const uint32_t lo = min(A[k], B[k]), hi = max(A[k], B[k]);
            const uint32_t old = __hip_atomic_fetch_min(G + hi, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (old == hi) {
                act[k] = false;
            } else {  // hi was linked meanwhile: unite lo with its new parent
                A[k] = lo;
                B[k] = old;
            }
        }
    }
}

// ws_compress4: point every node on the path from p[w] to its root at the root,
// for every w with (mask >> w) & 1.  Runs when no link changes any more;
// concurrent walkers only write the same root.
__device__ __forceinline__ void ws_compress4(gu32 *G, uint32_t (&p)[4], uint32_t mask)
{
    uint32_t R[4];
    bool go[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        R[w] = p[w];
        go[w] = (mask >> w) & 1u;
    }
    while (go[0] || go[1] || go[2] || go[3]) {
        uint32_t q[4];
#pragma unroll
        for (int w = 0; w < 4; ++w)
            q[w] = G[R[w]];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            if (go[w] && q[w] == R[w])
                go[w] = false;
            else if (go[w])
                R[w] = q[w];
        }
    }
#pragma unroll
    for (int w = 0; w < 4; ++w)
        go[w] = ((mask >> w) & 1u) && p[w] != R[w];
    while (go[0] || go[1] || go[2] || go[3]) {
        uint32_t q[4];
#pragma unroll
        for (int w = 0; w < 4; ++w)
            q[w] = G[p[w]];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            if (go[w]) {
                G[p[w]] = R[w];
                p[w] = q[w];
                go[w] = p[w] != R[w];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// local: bonds, in-tile labels, crossing masks.  Grid: one 256-thread
// workgroup per tile; wave w owns rows w*R .. w*R + R - 1 of the tile
// (R = kRowsPerWave).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cl_local(ClArgs a, uint32_t step, uint32_t base)
{
    __shared__ uint32_t L[kClRows * 64];
    __shared__ uint64_t Hm[kClRows], Dm[kClRows];
    const uint32_t tile = base + blockIdx.x;
    const uint32_t r = tile_owner(a.tile_prefix, a.n, tile);
    const RepDev d = a.reps[r];
    const ClRep c = a.cl[r];
    const Tile T = locate(a, d, r, tile);
    const uint32_t lane = threadIdx.x & 63u, wv = wave_id();
    const uint32_t W = d.W, Lx = d.Lx, Ly = d.Ly, t = d.t + step;
    const gu32 *P0 = global_view(d.plane0), *P1 = P0 + (size_t)Ly * W;
    gu32 *G = global_view(reinterpret_cast<uint32_t *>(a.ws + c.g_off));
    const uint32_t first = wv * kRowsPerWave;
    // rows of this wave (even, possibly 0)
    const uint32_t nr = T.rows > first ? min(kRowsPerWave, T.rows - first) : 0u;
    // One vector load brings all the words the wave needs (with R rows per
    // wave: lane k <= R the colour-0 word of row k, R < k <= 2R + 1 the
    // colour-1 word of row k - R - 1, 2R + 1 < k <= 3R + 1 the word of row
    // k - 2R - 2 that holds column 0 of the next tile; row R is the row below
    // the wave's rows).  They are broadcast with readlane after the bond
    // draws, so the load latency overlaps them.
    constexpr uint32_t R1 = kRowsPerWave + 1, R2 = 2 * kRowsPerWave + 2, R3 = 3 * kRowsPerWave + 2;
    static_assert(R3 <= 64, "one load per lane");
    uint32_t word;
    {
        const uint32_t k = lane < R1 ? lane : lane < R2 ? lane - R1 : lane < R3 ? lane - R2 : 0u;
        uint32_t y = T.y0 + min(first + k, lane < R2 ? T.rows : T.rows - 1);
        y = y == Ly ? 0u : y;
        const bool plane1 = lane < R1 ? false : lane < R2 ? true : lane < R3 ? (y & 1u) != 0 : false;
        const uint32_t col = lane >= R2 && lane < R3 ? T.txn : T.tx;
        word = (plane1 ? P1 : P0)[(size_t)y * W + col];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the load ahead of the bond draws
    // column order from a compact pair (odd << 32 | even): column j is bit
    // (j & 1) * 32 + (j >> 1)
    const uint32_t csh = ((lane & 1u) << 5) | (lane >> 1);
    auto column_order = [&](uint32_t even, uint32_t odd) {
        const uint64_t x = ((uint64_t)odd << 32) | even;
        return __ballot((x >> csh) & 1u);
    };
    // Lane j draws the call of column pair j & 31 (columns 2(j & 31) and
    // 2(j & 31) + 1) in row 2i + (j >> 5) of the wave; its four words are the
    // right and down bonds of the even and of the odd column.  Each of the four
    // comparisons' ballots is then, in its low and high halves, the two rows'
    // masks of that kind in compact order (bit k: column 2k, or 2k + 1).
    // Two halves of four row pairs: all bond draws of a half first (straight
    // line; rows past the tile draw for its last rows and are masked, and the
    // first half keeps the load above in flight), then its pairs, each reading
    // the spin words it needs from the loaded lanes; a half's 16 ballots and a
    // pair's words stay within the scalar registers (all 32 ballots plus all
    // 50 words at once spill).
    constexpr uint32_t HP = kRowsPerWave / 4;
#pragma unroll
    for (uint32_t h = 0; h < 2; ++h) {
        uint64_t bre[HP], bde[HP], bro[HP], bdo[HP];
#pragma unroll
        for (uint32_t ii = 0; ii < HP; ++ii) {
            const uint32_t i = h * HP + ii;
            const uint32_t row = T.y0 + min(first + 2 * i, T.rows - 2) + (lane >> 5);
            const uint32_t g = row * Lx + T.x0 + 2u * (lane & 31u);
            uint32_t w[4];
            philox4x32_10(g >> 1, t, d.replica, 7u, d.seed_lo, d.seed_hi, w);
            const bool on = 2 * i < nr && !c.none;
            bre[ii] = __ballot(on && w[0] >= c.thr2);
            bde[ii] = __ballot(on && w[1] >= c.thr2);
            bro[ii] = __ballot(on && w[2] >= c.thr2);
            bdo[ii] = __ballot(on && w[3] >= c.thr2);
        }
        __builtin_amdgcn_sched_barrier(0);  // and the first use of the loaded words after them
#pragma unroll
        for (uint32_t ii = 0; ii < HP; ++ii) {
            const uint32_t i = h * HP + ii;
            if (2 * i >= nr)
                break;
            // colour-0 / colour-1 words of rows 2i, 2i + 1, 2i + 2 of the wave
            // and the column-0 bits of the next tile in rows 2i, 2i + 1
            const uint32_t p0a = __builtin_amdgcn_readlane(word, 2 * i), p1a = __builtin_amdgcn_readlane(word, R1 + 2 * i);
            const uint32_t p0b = __builtin_amdgcn_readlane(word, 2 * i + 1);
            const uint32_t p1b = __builtin_amdgcn_readlane(word, R1 + 2 * i + 1);
            const uint32_t p0c = __builtin_amdgcn_readlane(word, 2 * i + 2);
            const uint32_t p1c = __builtin_amdgcn_readlane(word, R1 + 2 * i + 2);
            const uint32_t nxa = __builtin_amdgcn_readlane(word, R2 + 2 * i) & 1u;
            const uint32_t nxb = __builtin_amdgcn_readlane(word, R2 + 2 * i + 1) & 1u;
            const uint32_t rl = first + 2 * i, ya = T.y0 + rl;
            const uint32_t yb = ya + 1;
            // a row's even columns have colour y & 1, its odd columns the other
            const uint32_t ea = (ya & 1u) ? p1a : p0a, oa = (ya & 1u) ? p0a : p1a;
            const uint32_t eb = (yb & 1u) ? p1b : p0b, ob = (yb & 1u) ? p0b : p1b;
            // the row below b has the parity of yb + 1 (Ly is even, so also after wrapping)
            const uint32_t ec = (yb & 1u) ? p0c : p1c, oc = (yb & 1u) ? p1c : p0c;
            // aligned bonds in compact order: the right neighbour of column 2k is
            // column 2k + 1 (odd bit k), that of column 2k + 1 is column 2k + 2
            // (even bit k + 1, the next tile's column 0 for k = 31); the down
            // neighbour of a column is the same column of the next row
            const uint32_t hea = ~(ea ^ oa) & (uint32_t)bre[ii], hoa = ~(oa ^ ((ea >> 1) | (nxa << 31))) & (uint32_t)bro[ii];
            const uint32_t dea = ~(ea ^ eb) & (uint32_t)bde[ii], doa = ~(oa ^ ob) & (uint32_t)bdo[ii];
            const uint32_t heb = ~(eb ^ ob) & (uint32_t)(bre[ii] >> 32);
            const uint32_t hob = ~(ob ^ ((eb >> 1) | (nxb << 31))) & (uint32_t)(bro[ii] >> 32);
            const uint32_t deb = ~(eb ^ ec) & (uint32_t)(bde[ii] >> 32), dob = ~(ob ^ oc) & (uint32_t)(bdo[ii] >> 32);
            const uint64_t HA = column_order(hea, hoa), DA = column_order(dea, doa);
            const uint64_t HB = column_order(heb, hob), DB = column_order(deb, dob);
            if (lane == 0) {
                Hm[rl] = HA;
                Dm[rl] = DA;
                Hm[rl + 1] = HB;
                Dm[rl + 1] = DB;
            }
            L[rl * 64 + lane] = rl * 64 + run_start(HA, lane);
            L[(rl + 1) * 64 + lane] = (rl + 1) * 64 + run_start(HB, lane);
        }
    }
    __syncthreads();
    // vertical bonds inside the tile; a bond is skipped when its left
    // neighbour's bond already joins the same two runs
    for (uint32_t rl = first; rl < first + kRowsPerWave && rl + 1 < T.rows; ++rl) {
        const uint64_t D = Dm[rl], implied = D & Hm[rl] & Hm[rl + 1];
        if (((D >> lane) & 1u) && !(lane > 0 && ((implied >> (lane - 1)) & 1u)))
            lds_union((lu32 *)L, rl * 64 + lane, (rl + 1) * 64 + lane);
    }
    __syncthreads();
    // roots of the wave's rows, the finds of all rows stepped together (no
    // link changes any more; rows past the tile repeat its last row)
    uint32_t X[kRowsPerWave];
#pragma unroll
    for (uint32_t k = 0; k < kRowsPerWave; ++k)
        X[k] = (first + min(k, nr > 0 ? nr - 1 : 0u)) * 64 + lane;
    for (bool more = nr > 0; more;) {
        uint32_t q[kRowsPerWave];
#pragma unroll
        for (uint32_t k = 0; k < kRowsPerWave; ++k)
            q[k] = L[X[k]];
        more = false;
#pragma unroll
        for (uint32_t k = 0; k < kRowsPerWave; ++k) {
            more |= q[k] != X[k];
            X[k] = q[k];
        }
    }
#pragma unroll
    for (uint32_t k = 0; k < kRowsPerWave; ++k)
        if (k < nr)
            G[(size_t)(T.y0 + first + k) * Lx + T.x0 + lane] = (T.y0 + (X[k] >> 6)) * Lx + T.x0 + (X[k] & 63u);
    if (wv == 0) {
        // right-edge crossing bonds: bit 63 of each row's horizontal mask
        const uint64_t xr = __ballot(lane < T.rows && (Hm[lane] >> 63) != 0);
        if (lane == 0) {
            const uint64_t xd = Dm[T.rows - 1];
            a.tb[tile] = make_uint4((uint32_t)xd, (uint32_t)(xd >> 32), (uint32_t)xr, (uint32_t)(xr >> 32));
        }
    }
}

// Endpoints of the crossing bond k of a tile: k < 64 is the down bond of
// column k of the tile's last row, 64 <= k < 64 + rows the right bond of row
// k - 64's last column.
struct Crossing {
    uint32_t a, b;
};

__device__ __forceinline__ Crossing crossing(const RepDev &d, const Tile &T, uint32_t k)
{
    Crossing e;
    if (k < 64u) {
        const uint32_t y = T.y0 + T.rows - 1, yn = y + 1 == d.Ly ? 0u : y + 1;
        e.a = y * d.Lx + T.x0 + k;
        e.b = yn * d.Lx + T.x0 + k;
    } else {
        const uint32_t y = T.y0 + (k - 64u);
        e.a = y * d.Lx + T.x0 + 63u;
        e.b = y * d.Lx + 64u * T.txn;
    }
    return e;
}

// ---------------------------------------------------------------------------
// merge / compress: one wave per tile; lane j takes down bond j and right
// bond j (j < rows).
// ---------------------------------------------------------------------------
template <bool COMPRESS>
__global__ __launch_bounds__(256) void k_cl_cross(ClArgs a, uint32_t base)
{
    const uint32_t b = base + blockIdx.x * 4u + (threadIdx.x >> 6);
    if (b >= a.tiles)
        return;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t r = tile_owner(a.tile_prefix, a.n, b);
    const RepDev d = a.reps[r];
    const Tile T = locate(a, d, r, b);
    gu32 *G = global_view(reinterpret_cast<uint32_t *>(a.ws + a.cl[r].g_off));
    const uint4 tb = a.tb[b];
    const uint64_t xd = tb.x | ((uint64_t)tb.y << 32);
    const uint64_t xr = tb.z | ((uint64_t)tb.w << 32);
    // lane j: down bond j (edge 0) and right bond j of row j (edge 1)
    const bool on0 = ((xd >> lane) & 1u) != 0, on1 = lane < T.rows && ((xr >> lane) & 1u);
    const Crossing e0 = crossing(d, T, lane), e1 = crossing(d, T, 64u + min(lane, T.rows - 1));
    if (COMPRESS) {
        uint32_t p[4] = {on0 ? e0.a : 0u, on0 ? e0.b : 0u, on1 ? e1.a : 0u, on1 ? e1.b : 0u};
        ws_compress4(G, p, (on0 ? 3u : 0u) | (on1 ? 12u : 0u));
        return;
    }
    // Uniting the endpoints' current labels unites the endpoints.  Runs of
    // crossing bonds usually join the same two tile-local clusters, so a bond
    // whose label pair equals the previous lane's bond on the same edge is
    // already covered by that lane's union.
    uint32_t A[2], B[2];
    bool act[2];
#pragma unroll
    for (int edge = 0; edge < 2; ++edge) {
        const bool on = edge == 0 ? on0 : on1;
        const Crossing &e = edge == 0 ? e0 : e1;
        uint32_t la = 0xffffffffu, lb = 0xffffffffu;
        if (on) {
            la = ws_load(G + e.a);
            lb = ws_load(G + e.b);
        }
        const uint32_t pa = (uint32_t)__shfl_up((int)la, 1, 64), pb = (uint32_t)__shfl_up((int)lb, 1, 64);
        const bool dup = lane > 0 && pa == la && pb == lb;
        act[edge] = on && !dup;
        A[edge] = act[edge] ? la : 0u;
        B[edge] = act[edge] ? lb : 0u;
    }
    ws_union2(G, A, B, act);
}

// ---------------------------------------------------------------------------
// flip: one 256-thread workgroup per tile, rows as in k_cl_local.
// ---------------------------------------------------------------------------
template <int ALGO>
__global__ __launch_bounds__(256) void k_cl_flip(ClArgs a, uint32_t step, uint32_t base)
{
    const uint32_t tile = base + blockIdx.x;
    const uint32_t r = tile_owner(a.tile_prefix, a.n, tile);
    const RepDev d = a.reps[r];
    const ClRep c = a.cl[r];
    const Tile T = locate(a, d, r, tile);
    const uint32_t lane = threadIdx.x & 63u, wv = wave_id();
    const uint32_t W = d.W, Lx = d.Lx, Ly = d.Ly, t = d.t + step;
    gu32 *P0 = global_view(d.plane0), *P1 = P0 + (size_t)Ly * W;
    const gu32 *G = global_view(reinterpret_cast<const uint32_t *>(a.ws + c.g_off));
    const uint32_t first = wv * kRowsPerWave;
    const uint32_t nr = T.rows > first ? min(kRowsPerWave, T.rows - first) : 0u;
    if (nr == 0)
        return;
    uint32_t seed_root = 0;
    if (ALGO == kClWolff) {
        uint32_t w[4];
        philox4x32_10(0u, t, d.replica, 9u, d.seed_lo, d.seed_hi, w);
        const uint32_t S = (uint32_t)((((uint64_t)w[0] << 32) | w[1]) % d.N);
        seed_root = G[G[S]];
    }
    // Lane j takes column 2 (j & 31) + (j >> 5): a ballot over the wave is
    // then the row's even columns (bits 0..31) and odd columns (bits 32..63)
    // in compact order, i.e. the flip masks of its two colour words.
    const uint32_t col = ((lane & 31u) << 1) | (lane >> 5);
    // root of every site of the wave's rows: all label loads first, then all
    // second-level loads (rows past the tile repeat its last row)
    uint32_t R[kRowsPerWave];
#pragma unroll
    for (uint32_t k = 0; k < kRowsPerWave; ++k)
        R[k] = G[(size_t)(T.y0 + first + min(k, nr - 1)) * Lx + T.x0 + col];
#pragma unroll
    for (uint32_t k = 0; k < kRowsPerWave; ++k)
        R[k] = G[R[k]];
    // Lane 2k + e (k < nr) owns row k's word of the colour its even (e = 0)
    // or odd (e = 1) columns hold: colour y & 1 for the even columns.  Only
    // this workgroup touches these words in this launch, so each is read once
    // here and written once at the end with its row's flips.
    const uint32_t my_row = lane >> 1, my_y = T.y0 + first + min(my_row, nr - 1);
    gu32 *my_word = ((((my_y ^ lane) & 1u) != 0) ? P1 : P0) + (size_t)my_y * W + T.tx;
    const uint32_t spins = lane < 2 * nr ? *my_word : 0u;
    uint32_t my_flip = 0;
#pragma unroll
    for (uint32_t k = 0; k < kRowsPerWave; ++k) {
        bool flip;
        if (ALGO == kClWolff) {
            flip = R[k] == seed_root;
        } else {
            uint32_t w[4];
            philox4x32_10(R[k] >> 7, t, d.replica, 8u, d.seed_lo, d.seed_hi, w);
            const uint32_t q = (R[k] >> 5) & 3u;
            const uint32_t word = q == 0 ? w[0] : q == 1 ? w[1] : q == 2 ? w[2] : w[3];
            flip = (word >> (R[k] & 31u)) & 1u;
        }
        const uint64_t F = __ballot(flip);
        if (my_row == k)
            my_flip = (lane & 1u) ? (uint32_t)(F >> 32) : (uint32_t)F;
    }
    if (lane < 2 * nr && my_flip != 0u)
        *my_word = spins ^ my_flip;
}

}  // namespace

hipError_t launch_cluster_step(const ClArgs &a, int algorithm, uint32_t step, hipStream_t st)
{
    // Each phase covers every tile before the next starts; a phase is split
    // into launches of at most kClTilesPerLaunch tiles.
    for (uint32_t base = 0; base < a.tiles; base += kClTilesPerLaunch) {
        const uint32_t cnt = min(kClTilesPerLaunch, a.tiles - base);
        hipLaunchKernelGGL(k_cl_local, dim3(cnt), dim3(256), 0, st, a, step, base);
    }
    for (int phase = 0; phase < 2; ++phase)
        for (uint32_t base = 0; base < a.tiles; base += kClTilesPerLaunch) {
            const uint32_t cnt = min(kClTilesPerLaunch, a.tiles - base);
            if (phase == 0)
                hipLaunchKernelGGL(k_cl_cross<false>, dim3((cnt + 3u) / 4u), dim3(256), 0, st, a, base);
            else
                hipLaunchKernelGGL(k_cl_cross<true>, dim3((cnt + 3u) / 4u), dim3(256), 0, st, a, base);
        }
    for (uint32_t base = 0; base < a.tiles; base += kClTilesPerLaunch) {
        const uint32_t cnt = min(kClTilesPerLaunch, a.tiles - base);
        if (algorithm == kClWolff)
            hipLaunchKernelGGL(k_cl_flip<kClWolff>, dim3(cnt), dim3(256), 0, st, a, step, base);
        else
            hipLaunchKernelGGL(k_cl_flip<kClSwendsenWang>, dim3(cnt), dim3(256), 0, st, a, step, base);
    }
    return hipGetLastError();
}

// Workspace of the allocation-free cluster entry point.  In host code this
// name only stands for the symbol; its device address comes from
// hipGetSymbolAddress, separately for every device.
static __device__ __align__(256) unsigned char scratch[kClStaticWsBytes];

hipError_t static_cluster_ws(int device, char **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex lock;
    static char *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(lock);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        addr[device] = static_cast<char *>(p);
    }
    *ptr = addr[device];
    return hipSuccess;
}

}  // namespace ising
