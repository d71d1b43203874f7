/*
 * Plain CPU oracle for checkerboard Metropolis sweeps of the periodic 3D
 * nearest-neighbour Ising model (simple cubic lattice, six neighbours).
 *
 * TEST INFRASTRUCTURE ONLY, like ising_oracle.c (linked into the same
 * liboracle.so, from which it takes only the Philox function).  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; it shares
 * nothing with the GPU library.
 *
 * What it follows: paper section 1 states the Hamiltonian H = -J sum s_i s_j
 * and that each spin has 6 neighbours in 3D; the Metropolis rule (accept a
 * flip when ran() < exp(-beta dE)) and the red/black order of section 2 and
 * Supplementary S2 carry over unchanged, a site's colour now being the parity
 * of x + y + z so that all six neighbours have the other colour.
 *
 * Fixed conventions (the contract shared with the GPU library only as prose):
 *  - state s[g], g = (z*Ly + y)*Lx + x, int8 +-1; Lx, Ly, Lz even.
 *  - colour c = (x + y + z) & 1; colour 0 is updated first in every sweep.
 *  - dE = 2 J s (sum of the six neighbours) in {-12, ..., 12} J; dE <= 0 and
 *    K = beta*J == 0 accept without a draw; otherwise dE = 4J, 8J, 12J accept
 *    iff r < thr_k = min(floor(exp(-4kK) 2^32), 2^32 - 1), k = 1, 2, 3.
 *  - r for the colour-c site g in sweep t, h = g >> 1: with rng = 0, word
 *    (h & 3) of Philox(ctr = {h >> 2, t, replica, c}); with rng = 1 (the
 *    bit-sliced contract of the 2D library, unchanged but for the 3D index),
 *    the colour-c sites h = 32q .. 32q + 31 form group q with words W_k = word
 *    (k & 3) of Philox(ctr = {8q + (k >> 2), t, replica, c}), k = 0..31, and
 *    bit 31 - k of site 32q + b's uniform is bit b of W_k.
 *  - random initial state: s = +1 iff word (g & 3) of Philox(ctr = {g >> 2,
 *    0, replica, 2}) >= 2^31.
 *  - observables: B = sum s(x,y,z) (s(x+1,y,z) + s(x,y+1,z) + s(x,y,z+1)),
 *    every bond once (E = -J B); M = sum s.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

#define O3_OK 0
#define O3_EINVAL (-1)
#define O3_ENOMEM (-3)

enum { O3_INIT_RANDOM = 0, O3_INIT_UP = 1, O3_INIT_DOWN = 2 };

typedef struct {
    int32_t Lx, Ly, Lz;
    int32_t init;
    double J, beta;
    uint64_t seed;
    uint32_t replica;
    int32_t rng; /* 0: one Philox word per site; 1: bit-sliced group words */
} oracle3_desc;

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

static uint32_t word_of(const oracle3_desc *d, uint64_t index, uint32_t t, uint32_t tag)
{
    uint32_t ctr[4], key[2], out[4];
    ctr[0] = (uint32_t)(index >> 2);
    ctr[1] = t;
    ctr[2] = d->replica;
    ctr[3] = tag;
    key[0] = (uint32_t)(d->seed & 0xffffffffu);
    key[1] = (uint32_t)(d->seed >> 32);
    oracle_philox4x32_10(ctr, key, out);
    return out[index & 3];
}

/* Uniform of colour-c site h under the bit-sliced contract; the 32 words of
 * the last group used are cached (sites are visited in increasing h). */
typedef struct {
    int valid;
    uint64_t q;
    uint32_t t, colour;
    uint32_t w[32];
} group3;

static uint32_t bitsliced_uniform3(const oracle3_desc *d, uint32_t colour, uint32_t t, uint64_t h, group3 *cache)
{
    const uint64_t q = h >> 5;
    const uint32_t b = (uint32_t)(h & 31u);
    uint32_t u = 0, k;
    if (!cache->valid || cache->q != q || cache->t != t || cache->colour != colour) {
        /* word k of the group is the site-stream word at index 32q + k */
        for (k = 0; k < 32; ++k)
            cache->w[k] = word_of(d, 32u * q + k, t, colour);
        cache->valid = 1;
        cache->q = q;
        cache->t = t;
        cache->colour = colour;
    }
    for (k = 0; k < 32; ++k)
        u |= ((cache->w[k] >> b) & 1u) << (31u - k);
    return u;
}

static uint32_t threshold_of(double p)
{
    double scaled = ldexp(p, 32);
    return scaled >= 4294967295.0 ? 0xffffffffu : (uint32_t)floor(scaled);
}

int oracle3_thresholds(double J, double beta, uint32_t thr[3], int32_t *always)
{
    double K;
    int k;
    if (!(J > 0.0) || isinf(J) || isnan(beta) || beta < 0.0)
        return O3_EINVAL;
    K = beta * J;
    *always = K == 0.0 ? 1 : 0;
    for (k = 1; k <= 3; ++k)
        thr[k - 1] = threshold_of(exp(-4.0 * k * K));
    return O3_OK;
}

static int desc_ok(const oracle3_desc *d)
{
    uint32_t thr[3];
    int32_t always;
    if (d->Lx < 2 || d->Ly < 2 || d->Lz < 2 || (d->Lx & 1) || (d->Ly & 1) || (d->Lz & 1))
        return 0;
    if ((uint64_t)d->Lx * (uint64_t)d->Ly * (uint64_t)d->Lz > 0xffffffffull)
        return 0;
    if (oracle3_thresholds(d->J, d->beta, thr, &always) != O3_OK)
        return 0;
    if (d->rng != 0 && d->rng != 1)
        return 0;
    return d->init == O3_INIT_RANDOM || d->init == O3_INIT_UP || d->init == O3_INIT_DOWN;
}

int oracle3_init(const oracle3_desc *d, int8_t *s)
{
    uint64_t g, N;
    if (!desc_ok(d))
        return O3_EINVAL;
    N = (uint64_t)d->Lx * d->Ly * d->Lz;
    for (g = 0; g < N; ++g) {
        if (d->init == O3_INIT_UP)
            s[g] = 1;
        else if (d->init == O3_INIT_DOWN)
            s[g] = -1;
        else
            s[g] = word_of(d, g, 0u, 2u) >= 0x80000000u ? 1 : -1;
    }
    return O3_OK;
}

void oracle3_observables(int32_t Lx, int32_t Ly, int32_t Lz, const int8_t *s, int64_t *bond, int64_t *mag)
{
    int64_t B = 0, M = 0;
    int32_t x, y, z;
    for (z = 0; z < Lz; ++z)
        for (y = 0; y < Ly; ++y)
            for (x = 0; x < Lx; ++x) {
                const int64_t g = ((int64_t)z * Ly + y) * Lx + x;
                const int32_t here = s[g];
                const int32_t xp = s[((int64_t)z * Ly + y) * Lx + (x + 1) % Lx];
                const int32_t yp = s[((int64_t)z * Ly + (y + 1) % Ly) * Lx + x];
                const int32_t zp = s[((int64_t)((z + 1) % Lz) * Ly + y) * Lx + x];
                B += here * (xp + yp + zp);
                M += here;
            }
    *bond = B;
    *mag = M;
}

static void flip_colour(const oracle3_desc *d, int8_t *s, uint32_t t, int colour, const uint32_t thr[3],
                        int32_t always)
{
    const int32_t Lx = d->Lx, Ly = d->Ly, Lz = d->Lz;
    int32_t x, y, z;
    group3 cache;
    cache.valid = 0;
    for (z = 0; z < Lz; ++z)
        for (y = 0; y < Ly; ++y)
            for (x = 0; x < Lx; ++x) {
                const int64_t g = ((int64_t)z * Ly + y) * Lx + x;
                int32_t sum, dE;
                uint32_t r;
                if (((x + y + z) & 1) != colour)
                    continue;
                sum = s[((int64_t)z * Ly + y) * Lx + (x + 1) % Lx] + s[((int64_t)z * Ly + y) * Lx + (x + Lx - 1) % Lx] +
                      s[((int64_t)z * Ly + (y + 1) % Ly) * Lx + x] + s[((int64_t)z * Ly + (y + Ly - 1) % Ly) * Lx + x] +
                      s[((int64_t)((z + 1) % Lz) * Ly + y) * Lx + x] + s[((int64_t)((z + Lz - 1) % Lz) * Ly + y) * Lx + x];
                dE = 2 * s[g] * sum; /* units of J: -12 .. 12 in steps of 4 */
                if (dE <= 0 || always) {
                    s[g] = (int8_t)(-s[g]);
                    continue;
                }
                r = d->rng == 1 ? bitsliced_uniform3(d, (uint32_t)colour, t, (uint64_t)g >> 1, &cache)
                                : word_of(d, (uint64_t)g >> 1, t, (uint32_t)colour);
                if (r < thr[dE / 4 - 1])
                    s[g] = (int8_t)(-s[g]);
            }
}

/* n sweeps from counter t0; recording as oracle_sweeps (2D). */
int oracle3_sweeps(const oracle3_desc *d, int8_t *s, uint64_t t0, uint64_t n, uint32_t record_every, int64_t *bond,
                   int64_t *mag)
{
    uint32_t thr[3];
    int32_t always;
    uint64_t i;
    if (!desc_ok(d) || t0 + n > 0x100000000ull)
        return O3_EINVAL;
    oracle3_thresholds(d->J, d->beta, thr, &always);
    for (i = 0; i < n; ++i) {
        const uint32_t t = (uint32_t)(t0 + i);
        flip_colour(d, s, t, 0, thr, always);
        flip_colour(d, s, t, 1, thr, always);
        if (record_every && bond && mag && (i + 1) % record_every == 0) {
            const uint64_t j = (i + 1) / record_every - 1;
            oracle3_observables(d->Lx, d->Ly, d->Lz, s, &bond[j], &mag[j]);
        }
    }
    return O3_OK;
}

typedef struct {
    int32_t n, stride, first;
    const oracle3_desc *d;
    int8_t *const *states;
    const uint64_t *t0;
    uint64_t n_sweeps;
    uint32_t record_every;
    int64_t *bond, *mag;
    uint64_t n_rec;
    int status;
} job3;

static void *worker3(void *arg)
{
    job3 *j = (job3 *)arg;
    int32_t r;
    for (r = j->first; r < j->n; r += j->stride) {
        int64_t *b = j->bond ? j->bond + (uint64_t)r * j->n_rec : NULL;
        int64_t *m = j->mag ? j->mag + (uint64_t)r * j->n_rec : NULL;
        const int st = oracle3_sweeps(&j->d[r], j->states[r], j->t0 ? j->t0[r] : 0, j->n_sweeps, j->record_every, b, m);
        if (st != O3_OK)
            j->status = st;
    }
    return NULL;
}

/* Replica r runs on thread r % n_threads; results do not depend on n_threads. */
int oracle3_run_batch(int32_t n, const oracle3_desc *d, int8_t *const *states, const uint64_t *t0, uint64_t n_sweeps,
                      uint32_t record_every, int64_t *bond, int64_t *mag, int32_t n_threads)
{
    job3 *jobs;
    pthread_t *tids;
    int32_t k, started = 0;
    int status = O3_OK;
    if (n <= 0)
        return O3_EINVAL;
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > n)
        n_threads = n;
    jobs = (job3 *)calloc((size_t)n_threads, sizeof(job3));
    tids = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return O3_ENOMEM;
    }
    for (k = 0; k < n_threads; ++k) {
        jobs[k].n = n;
        jobs[k].stride = n_threads;
        jobs[k].first = k;
        jobs[k].d = d;
        jobs[k].states = states;
        jobs[k].t0 = t0;
        jobs[k].n_sweeps = n_sweeps;
        jobs[k].record_every = record_every;
        jobs[k].bond = bond;
        jobs[k].mag = mag;
        jobs[k].n_rec = record_every ? n_sweeps / record_every : 0;
        jobs[k].status = O3_OK;
    }
    for (k = 1; k < n_threads; ++k) {
        if (pthread_create(&tids[k], NULL, worker3, &jobs[k]) != 0)
            break;
        started = k;
    }
    worker3(&jobs[0]);
    for (k = started + 1; k < n_threads; ++k)
        worker3(&jobs[k]);
    for (k = 1; k <= started; ++k)
        pthread_join(tids[k], NULL);
    for (k = 0; k < n_threads; ++k)
        if (jobs[k].status != O3_OK)
            status = jobs[k].status;
    free(jobs);
    free(tids);
    return status;
}
