/*
 * Plain CPU oracle for checkerboard Metropolis sweeps of the periodic 2D
 * nearest-neighbour Ising model.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what the GPU library computes.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or helper with the GPU library, and the GPU library
 * never calls it.
 *
 * What it follows:
 *  - Hamiltonian H = -J sum_<ij> s_i s_j, s = +-1, four neighbours in 2D,
 *    J > 0, no field (paper section 1, Introduction).
 *  - Metropolis rule: a proposed single-spin flip is accepted when ran() <
 *    exp(-beta dE), ran() uniform on [0,1) (paper section 1).
 *  - Checkerboard order: every "red" site (x+y even) is visited, then every
 *    "blue" site (x+y odd); sites of one colour only see the other colour
 *    (paper section 2; Supplementary algorithm S2, the checkerboard
 *    multi-spin algorithm, and its FlipSpin function).  Its neighbour sum is
 *    printed over three terms; the adjacency list it sums over has four
 *    entries and section 1 says each 2D spin has four neighbours, so all four
 *    are summed here.
 *  - Random numbers: the paper's hardware generator is not published
 *    (Supplementary S.4), so uniforms come from Philox4x32-10 (Salmon,
 *    Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 *    SC'11), written here from that paper's definition.
 *
 * Fixed conventions (the "contract" shared with the GPU library only as
 * prose, never as code):
 *  - state s[y*Lx + x], int8, +1 or -1; x = column (0..Lx-1), y = row.
 *  - colour c = (x + y) & 1; colour 0 (red) is updated first in every sweep.
 *  - compact index of a site inside its colour: h = (y*Lx + x) >> 1.
 *  - uniform for site (x,y) in sweep t, colour c:
 *      r = Philox(ctr = {h >> 2, t, replica, c}, key = {seed_lo, seed_hi})[h & 3]
 *    a 32-bit integer; ran() = r / 2^32.
 *  - bit-sliced variant (rng = 1, an alternative random-number contract):
 *    the colour-c sites with compact indices 32g .. 32g+31 form group g; its
 *    words are W_k = Philox(ctr = {8g + (k >> 2), t, replica, c}, key)[k & 3]
 *    for k = 0..31, and site h = 32g + b takes the 32-bit uniform whose bit
 *    31 - k is bit b of W_k (the group's words, transposed).  Comparing that
 *    uniform with a threshold most significant bit first needs, per site,
 *    only the words up to the first bit where the two differ.
 *  - thresholds: K = beta*J (one rounding), p1 = exp(-4K), p2 = exp(-8K),
 *    thr_k = min(floor(p_k * 2^32), 2^32 - 1); dE = 4J accepts iff r < thr_1,
 *    dE = 8J iff r < thr_2; dE <= 0 always accepts and draws nothing;
 *    K == 0 accepts every proposal.
 *  - random initial state: g = y*Lx + x;
 *      s = +1 iff Philox(ctr = {g >> 2, 0, replica, 2}, key)[g & 3] >= 2^31.
 *  - observables: B = sum_{x,y} s(x,y) (s(x+1,y) + s(x,y+1)) (every bond
 *    once), M = sum s, E = -J B.
 */
#define _POSIX_C_SOURCE 200112L /* pthread barriers */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-3)

enum { OR_INIT_RANDOM = 0, OR_INIT_UP = 1, OR_INIT_DOWN = 2 };

typedef struct {
    int32_t Lx, Ly;
    double J, beta;
    uint64_t seed;
    uint32_t replica;
    int32_t init;
    int32_t rng; /* 0: one Philox word per site; 1: bit-sliced group words */
} oracle_desc;

/* ---- Philox4x32-10 (Salmon et al., SC'11) ------------------------------ */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    /* Multipliers and Weyl key increments from the Philox definition. */
    const uint32_t mul0 = 0xD2511F53u, mul1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t prod0, prod1;
        uint32_t n0, n1, n2, n3;
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        prod0 = (uint64_t)mul0 * (uint64_t)x0;
        prod1 = (uint64_t)mul1 * (uint64_t)x2;
        n0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
        n1 = (uint32_t)prod1;
        n2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
        n3 = (uint32_t)prod0;
        x0 = n0;
        x1 = n1;
        x2 = n2;
        x3 = n3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

static uint32_t site_uniform(uint64_t seed, uint32_t tag_or_colour, uint32_t t,
                             uint32_t replica, uint64_t index)
{
    uint32_t ctr[4], key[2], out[4];
    ctr[0] = (uint32_t)(index >> 2);
    ctr[1] = t;
    ctr[2] = replica;
    ctr[3] = tag_or_colour;
    key[0] = (uint32_t)(seed & 0xffffffffu);
    key[1] = (uint32_t)(seed >> 32);
    oracle_philox4x32_10(ctr, key, out);
    return out[index & 3];
}

/* ---- acceptance thresholds (Metropolis rule, section 1) ----------------- */

static uint32_t prob_to_threshold(double p)
{
    double scaled = ldexp(p, 32);
    if (scaled >= 4294967295.0)
        return 0xffffffffu;
    return (uint32_t)floor(scaled);
}

int oracle_thresholds(double J, double beta, uint32_t *thr4, uint32_t *thr8, int32_t *always)
{
    double K;
    if (!(J > 0.0) || isinf(J) || isnan(beta) || beta < 0.0)
        return OR_EINVAL;
    K = beta * J;
    *always = (K == 0.0) ? 1 : 0;
    *thr4 = prob_to_threshold(exp(-4.0 * K));
    *thr8 = prob_to_threshold(exp(-8.0 * K));
    return OR_OK;
}

/* ---- state set-up ------------------------------------------------------- */

/* Uniform of site h (compact index within its colour) under the bit-sliced
 * contract: bit 31 - k of the result is bit (h & 31) of word k of group h >> 5.
 * The 32 words of the last group used are kept in *cache, since the sites of
 * one colour are visited in increasing h. */
typedef struct {
    int valid;
    uint64_t g;
    uint32_t t, colour;
    uint32_t w[32];
} group_words;

static uint32_t bitsliced_uniform(const oracle_desc *d, uint32_t colour, uint32_t t, uint64_t h,
                                  group_words *cache)
{
    const uint64_t g = h >> 5;
    const uint32_t b = (uint32_t)(h & 31u);
    uint32_t u = 0, k;
    if (!cache->valid || cache->g != g || cache->t != t || cache->colour != colour) {
        /* word k of the group is word (k & 3) of call 8g + (k >> 2), i.e. the
           site-uniform stream at index 32g + k */
        for (k = 0; k < 32; ++k)
            cache->w[k] = site_uniform(d->seed, colour, t, d->replica, 32u * g + k);
        cache->valid = 1;
        cache->g = g;
        cache->t = t;
        cache->colour = colour;
    }
    for (k = 0; k < 32; ++k)
        u |= ((cache->w[k] >> b) & 1u) << (31u - k);
    return u;
}

static int desc_ok(const oracle_desc *d)
{
    uint32_t a, b;
    int32_t c;
    if (d->Lx < 2 || d->Ly < 2 || (d->Lx & 1) || (d->Ly & 1))
        return 0;
    if ((uint64_t)d->Lx * (uint64_t)d->Ly > 0xffffffffull)
        return 0;
    if (oracle_thresholds(d->J, d->beta, &a, &b, &c) != OR_OK)
        return 0;
    if (d->rng != 0 && d->rng != 1)
        return 0;
    return d->init == OR_INIT_RANDOM || d->init == OR_INIT_UP || d->init == OR_INIT_DOWN;
}

int oracle_init(const oracle_desc *d, int8_t *s)
{
    int32_t x, y;
    if (!desc_ok(d))
        return OR_EINVAL;
    for (y = 0; y < d->Ly; ++y) {
        for (x = 0; x < d->Lx; ++x) {
            uint64_t g = (uint64_t)y * (uint64_t)d->Lx + (uint64_t)x;
            int8_t v;
            if (d->init == OR_INIT_UP)
                v = 1;
            else if (d->init == OR_INIT_DOWN)
                v = -1;
            else
                v = site_uniform(d->seed, 2u, 0u, d->replica, g) >= 0x80000000u ? 1 : -1;
            s[g] = v;
        }
    }
    return OR_OK;
}

/* ---- observables (Hamiltonian, section 1; |M| of section 3.1) ----------- */

void oracle_observables(int32_t Lx, int32_t Ly, const int8_t *s, int64_t *bond, int64_t *mag)
{
    int64_t B = 0, M = 0;
    int32_t x, y;
    for (y = 0; y < Ly; ++y) {
        for (x = 0; x < Lx; ++x) {
            int32_t right = s[(int64_t)y * Lx + (x + 1) % Lx];
            int32_t below = s[(int64_t)((y + 1) % Ly) * Lx + x];
            int32_t here = s[(int64_t)y * Lx + x];
            B += here * (right + below);
            M += here;
        }
    }
    *bond = B;
    *mag = M;
}

/* ---- one sweep: red sites, then blue sites (Supplementary algorithm S2) -- */

/* Update the colour-`colour` sites of rows y_begin .. y_end - 1.  They read
 * only sites of the other colour, so any split of the rows gives the same
 * result. */
static void flip_colour_rows(const oracle_desc *d, int8_t *s, uint32_t t, int colour,
                             uint32_t thr4, uint32_t thr8, int32_t always, int32_t y_begin, int32_t y_end)
{
    const int32_t Lx = d->Lx, Ly = d->Ly;
    int32_t x, y;
    group_words cache;
    cache.valid = 0;
    for (y = y_begin; y < y_end; ++y) {
        for (x = 0; x < Lx; ++x) {
            int64_t i = (int64_t)y * Lx + x;
            int32_t sum, dE;
            int accept;
            if (((x + y) & 1) != colour)
                continue;
            sum = s[(int64_t)y * Lx + (x + 1) % Lx] + s[(int64_t)y * Lx + (x + Lx - 1) % Lx] +
                  s[(int64_t)((y + 1) % Ly) * Lx + x] + s[(int64_t)((y + Ly - 1) % Ly) * Lx + x];
            dE = 2 * s[i] * sum; /* energy change of the flip, in units of J */
            if (dE <= 0 || always) {
                accept = 1;
            } else {
                uint64_t h = (uint64_t)i >> 1;
                uint32_t r = d->rng == 1 ? bitsliced_uniform(d, (uint32_t)colour, t, h, &cache)
                                         : site_uniform(d->seed, (uint32_t)colour, t, d->replica, h);
                accept = r < (dE == 4 ? thr4 : thr8);
            }
            if (accept)
                s[i] = (int8_t)(-s[i]);
        }
    }
}

static void flip_colour(const oracle_desc *d, int8_t *s, uint32_t t, int colour,
                        uint32_t thr4, uint32_t thr8, int32_t always)
{
    flip_colour_rows(d, s, t, colour, thr4, thr8, always, 0, d->Ly);
}

/*
 * Run n sweeps of one replica starting at sweep counter t0.  After the sweep
 * with run-local index i, if (i + 1) % record_every == 0, (B, M) go to
 * bond[j], mag[j] with j = (i + 1) / record_every - 1.
 */
int oracle_sweeps(const oracle_desc *d, int8_t *s, uint64_t t0, uint64_t n,
                  uint32_t record_every, int64_t *bond, int64_t *mag)
{
    uint32_t thr4, thr8;
    int32_t always;
    uint64_t i;
    if (!desc_ok(d) || t0 + n > 0x100000000ull)
        return OR_EINVAL;
    oracle_thresholds(d->J, d->beta, &thr4, &thr8, &always);
    for (i = 0; i < n; ++i) {
        uint32_t t = (uint32_t)(t0 + i);
        flip_colour(d, s, t, 0, thr4, thr8, always);
        flip_colour(d, s, t, 1, thr4, thr8, always);
        if (record_every && bond && mag && (i + 1) % record_every == 0) {
            uint64_t j = (i + 1) / record_every - 1;
            oracle_observables(d->Lx, d->Ly, s, &bond[j], &mag[j]);
        }
    }
    return OR_OK;
}

/* ---- many independent replicas on host threads -------------------------- */

typedef struct {
    int32_t n;
    int32_t *next; /* shared: the next replica not yet taken */
    const oracle_desc *d;
    int8_t *const *states;
    const uint64_t *t0;
    uint64_t n_sweeps;
    uint32_t record_every;
    int64_t *bond, *mag;
    uint64_t n_rec;
    int status;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *job = (batch_job *)arg;
    int32_t r;
    while ((r = __atomic_fetch_add(job->next, 1, __ATOMIC_RELAXED)) < job->n) {
        int64_t *b = job->bond ? job->bond + (uint64_t)r * job->n_rec : NULL;
        int64_t *m = job->mag ? job->mag + (uint64_t)r * job->n_rec : NULL;
        int st = oracle_sweeps(&job->d[r], job->states[r], job->t0 ? job->t0[r] : 0,
                               job->n_sweeps, job->record_every, b, m);
        if (st != OR_OK)
            job->status = st;
    }
    return NULL;
}

/* Threads take replicas one at a time in index order until none is left;
 * replicas are independent, so results do not depend on n_threads. */
int oracle_run_batch(int32_t n, const oracle_desc *d, int8_t *const *states, const uint64_t *t0,
                     uint64_t n_sweeps, uint32_t record_every, int64_t *bond, int64_t *mag,
                     int32_t n_threads)
{
    batch_job *jobs;
    pthread_t *tids;
    int32_t k, started = 0, next = 0;
    int status = OR_OK;
    if (n <= 0)
        return OR_EINVAL;
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > n)
        n_threads = n;
    jobs = (batch_job *)calloc((size_t)n_threads, sizeof(batch_job));
    tids = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return OR_ENOMEM;
    }
    for (k = 0; k < n_threads; ++k) {
        jobs[k].n = n;
        jobs[k].next = &next;
        jobs[k].d = d;
        jobs[k].states = states;
        jobs[k].t0 = t0;
        jobs[k].n_sweeps = n_sweeps;
        jobs[k].record_every = record_every;
        jobs[k].bond = bond;
        jobs[k].mag = mag;
        jobs[k].n_rec = record_every ? n_sweeps / record_every : 0;
        jobs[k].status = OR_OK;
    }
    for (k = 1; k < n_threads; ++k) {
        if (pthread_create(&tids[k], NULL, batch_worker, &jobs[k]) != 0)
            break;
        started = k;
    }
    batch_worker(&jobs[0]); /* threads that failed to start leave their replicas to the others */
    for (k = 1; k <= started; ++k)
        pthread_join(tids[k], NULL);
    for (k = 0; k < n_threads; ++k)
        if (jobs[k].status != OR_OK)
            status = jobs[k].status;
    free(jobs);
    free(tids);
    return status;
}

/* ---- one lattice on host threads: the rows of a colour split between them -- */

typedef struct {
    const oracle_desc *d;
    int8_t *s;
    uint64_t t0, n;
    uint32_t record_every;
    int64_t *bond, *mag;
    uint32_t thr4, thr8;
    int32_t always;
    int32_t index;
    /* shared */
    pthread_mutex_t *lock;
    pthread_cond_t *gate;
    int32_t *n_workers; /* -1 until every thread that will take part has started */
    pthread_barrier_t *bar;
} rows_job;

static void *rows_worker(void *arg)
{
    rows_job *j = (rows_job *)arg;
    int32_t nw, y0, y1;
    uint64_t i;
    pthread_mutex_lock(j->lock);
    while (*j->n_workers < 0)
        pthread_cond_wait(j->gate, j->lock);
    nw = *j->n_workers;
    pthread_mutex_unlock(j->lock);
    y0 = (int32_t)((int64_t)j->index * j->d->Ly / nw);
    y1 = (int32_t)((int64_t)(j->index + 1) * j->d->Ly / nw);
    for (i = 0; i < j->n; ++i) {
        uint32_t t = (uint32_t)(j->t0 + i);
        int colour;
        for (colour = 0; colour < 2; ++colour) {
            flip_colour_rows(j->d, j->s, t, colour, j->thr4, j->thr8, j->always, y0, y1);
            pthread_barrier_wait(j->bar);
        }
        if (j->record_every && j->bond && j->mag && (i + 1) % j->record_every == 0) {
            if (j->index == 0) {
                uint64_t k = (i + 1) / j->record_every - 1;
                oracle_observables(j->d->Lx, j->d->Ly, j->s, &j->bond[k], &j->mag[k]);
            }
            pthread_barrier_wait(j->bar);
        }
    }
    return NULL;
}

/*
 * oracle_sweeps for one lattice on up to n_threads host threads (at most one
 * per row): in each colour phase thread k updates rows Ly*k/m .. Ly*(k+1)/m - 1
 * of the m threads that started, then all wait for each other.  Sites of one
 * colour only read the other colour and every uniform is a function of
 * (seed, replica, sweep, colour, site), so the result equals oracle_sweeps
 * for every thread count.
 */
int oracle_sweeps_rows(const oracle_desc *d, int8_t *s, uint64_t t0, uint64_t n, uint32_t record_every,
                       int64_t *bond, int64_t *mag, int32_t n_threads)
{
    uint32_t thr4, thr8;
    int32_t always, k, started = 0, n_workers = -1;
    rows_job *jobs;
    pthread_t *tids;
    pthread_mutex_t lock = PTHREAD_MUTEX_INITIALIZER;
    pthread_cond_t gate = PTHREAD_COND_INITIALIZER;
    pthread_barrier_t bar;
    if (!desc_ok(d) || t0 + n > 0x100000000ull)
        return OR_EINVAL;
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > d->Ly)
        n_threads = d->Ly;
    if (n_threads == 1)
        return oracle_sweeps(d, s, t0, n, record_every, bond, mag);
    oracle_thresholds(d->J, d->beta, &thr4, &thr8, &always);
    jobs = (rows_job *)calloc((size_t)n_threads, sizeof(rows_job));
    tids = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return OR_ENOMEM;
    }
    for (k = 0; k < n_threads; ++k) {
        jobs[k].d = d;
        jobs[k].s = s;
        jobs[k].t0 = t0;
        jobs[k].n = n;
        jobs[k].record_every = record_every;
        jobs[k].bond = bond;
        jobs[k].mag = mag;
        jobs[k].thr4 = thr4;
        jobs[k].thr8 = thr8;
        jobs[k].always = always;
        jobs[k].index = k;
        jobs[k].lock = &lock;
        jobs[k].gate = &gate;
        jobs[k].n_workers = &n_workers;
        jobs[k].bar = &bar;
    }
    /* threads 1.. wait at the gate until the number of participants is known */
    for (k = 1; k < n_threads; ++k) {
        if (pthread_create(&tids[k], NULL, rows_worker, &jobs[k]) != 0)
            break;
        started = k;
    }
    pthread_barrier_init(&bar, NULL, (unsigned)(started + 1));
    pthread_mutex_lock(&lock);
    n_workers = started + 1;
    pthread_cond_broadcast(&gate);
    pthread_mutex_unlock(&lock);
    rows_worker(&jobs[0]);
    for (k = 1; k <= started; ++k)
        pthread_join(tids[k], NULL);
    pthread_barrier_destroy(&bar);
    free(jobs);
    free(tids);
    return OR_OK;
}
