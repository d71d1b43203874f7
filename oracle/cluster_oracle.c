/*
 * Plain CPU oracle for Swendsen-Wang and Wolff cluster steps of the periodic
 * 2D nearest-neighbour Ising model.
 *
 * TEST INFRASTRUCTURE ONLY, like ising_oracle.c (linked into the same
 * liboracle.so, from which it takes only the Philox function).  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; it
 * shares nothing with the GPU library.
 *
 * What it follows.  Paper section 1 names the Swendsen-Wang and Wolff cluster
 * algorithms as the cure for the critical slowing down of single-spin
 * Metropolis near T_c; the algorithms themselves are taken from their
 * original papers:
 *  - Swendsen and Wang, PRL 58, 86 (1987): with H = -J sum s_i s_j, every bond
 *    between two aligned neighbours is occupied with probability
 *    p = 1 - exp(-2 beta J) (the Fortuin-Kasteleyn representation), bonds
 *    between anti-aligned neighbours never; the clusters are the connected
 *    components of the occupied bonds; every cluster is flipped with
 *    probability 1/2, independently.
 *  - Wolff, PRL 62, 361 (1989): a seed site is chosen uniformly; the cluster
 *    grows from it by adding, over every bond from a cluster site to an
 *    aligned neighbour not yet in it, that neighbour with probability p; the
 *    whole cluster is flipped.  Each bond is tested once, so the grown cluster
 *    is the component of the seed in a configuration of independently
 *    occupied bonds; the growth below draws each bond's occupancy from that
 *    bond's own counter, the same draw the Swendsen-Wang labelling sees.
 *
 * Fixed conventions (the contract shared with the GPU library only as prose):
 *  - state s[g], g = y*Lx + x, int8 +-1.
 *  - site g owns two bonds: "right" to ((x+1) mod Lx, y) and "down" to
 *    (x, (y+1) mod Ly).  With Lx = 2 or Ly = 2 two distinct bonds join the
 *    same pair of sites (the periodic lattice's double bonds), each drawn on
 *    its own.
 *  - K = beta*J; thr = min(floor(exp(-2K) 2^32), 2^32 - 1).  A bond is
 *    occupied iff its two spins are equal, K > 0 and its word u >= thr (so
 *    P(occupied) = 1 - thr/2^32).  The word of the right bond of g is word
 *    2(g & 1) of Philox(ctr = {g >> 1, t, replica, 7}), of the down bond word
 *    2(g & 1) + 1.
 *  - the root of a cluster is its smallest site index.
 *  - Swendsen-Wang: the cluster with root R flips iff bit (R & 31) of word
 *    (R >> 5) & 3 of Philox(ctr = {R >> 7, t, replica, 8}) is 1.
 *  - Wolff: with w = Philox(ctr = {0, t, replica, 9}), the seed is
 *    S = ((w0 << 32) | w1) mod (Lx Ly); the cluster of S flips.
 *  - a step uses counter t; the next step (or sweep) uses t + 1.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

#define CL_OK 0
#define CL_EINVAL (-1)
#define CL_ENOMEM (-3)

enum { CL_SWENDSEN_WANG = 0, CL_WOLFF = 1 };

/* Same layout as oracle_desc in ising_oracle.c. */
typedef struct {
    int32_t Lx, Ly;
    double J, beta;
    uint64_t seed;
    uint32_t replica;
    int32_t init;
    int32_t rng;
} cl_desc;

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void oracle_observables(int32_t Lx, int32_t Ly, const int8_t *s, int64_t *bond, int64_t *mag);

static void draw(const cl_desc *d, uint32_t c0, uint32_t t, uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = c0;
    ctr[1] = t;
    ctr[2] = d->replica;
    ctr[3] = tag;
    key[0] = (uint32_t)(d->seed & 0xffffffffu);
    key[1] = (uint32_t)(d->seed >> 32);
    oracle_philox4x32_10(ctr, key, out);
}

/* Occupation threshold of the Fortuin-Kasteleyn bond probability. */
int oracle_bond_threshold(double J, double beta, uint32_t *thr, int32_t *none)
{
    double K, scaled;
    if (!(J > 0.0) || isinf(J) || isnan(beta) || beta < 0.0)
        return CL_EINVAL;
    K = beta * J;
    *none = (K == 0.0) ? 1 : 0;
    scaled = ldexp(exp(-2.0 * K), 32);
    *thr = scaled >= 4294967295.0 ? 0xffffffffu : (uint32_t)floor(scaled);
    return CL_OK;
}

static int cl_desc_ok(const cl_desc *d)
{
    uint32_t thr;
    int32_t none;
    if (d->Lx < 2 || d->Ly < 2 || (d->Lx & 1) || (d->Ly & 1))
        return 0;
    if ((uint64_t)d->Lx * (uint64_t)d->Ly > 0xffffffffull)
        return 0;
    return oracle_bond_threshold(d->J, d->beta, &thr, &none) == CL_OK;
}

typedef struct {
    const cl_desc *d;
    const int8_t *s;
    uint32_t t, thr;
    int32_t none;
} bond_ctx;

/* Is the bond that site g owns in direction dir (0 right, 1 down) occupied? */
static int occupied(const bond_ctx *b, uint64_t g, int dir)
{
    const cl_desc *d = b->d;
    const uint64_t x = g % (uint64_t)d->Lx, y = g / (uint64_t)d->Lx;
    const uint64_t h = dir == 0 ? y * d->Lx + (x + 1) % d->Lx : ((y + 1) % d->Ly) * d->Lx + x;
    uint32_t w[4];
    if (b->none || b->s[g] != b->s[h])
        return 0;
    draw(d, (uint32_t)(g >> 1), b->t, 7u, w);
    return w[2 * (g & 1) + dir] >= b->thr;
}

/* Push onto the queue every neighbour of v joined to it by an occupied bond
 * and not yet labelled, labelling it with lab. */
static void visit_neighbours(const bond_ctx *b, uint64_t v, uint32_t *label, uint32_t lab,
                             uint32_t *queue, uint64_t *tail)
{
    const cl_desc *d = b->d;
    const uint64_t Lx = (uint64_t)d->Lx, Ly = (uint64_t)d->Ly;
    const uint64_t x = v % Lx, y = v / Lx;
    /* the four bonds of v: its own right and down bonds, the right bond of its
       left neighbour and the down bond of its upper neighbour */
    const uint64_t right = y * Lx + (x + 1) % Lx, down = ((y + 1) % Ly) * Lx + x;
    const uint64_t left = y * Lx + (x + Lx - 1) % Lx, up = ((y + Ly - 1) % Ly) * Lx + x;
    const uint64_t other[4] = {right, down, left, up};
    const uint64_t owner[4] = {v, v, left, up};
    const int dir[4] = {0, 1, 0, 1};
    int k;
    for (k = 0; k < 4; ++k) {
        if (label[other[k]] != 0xffffffffu || !occupied(b, owner[k], dir[k]))
            continue;
        label[other[k]] = lab;
        queue[(*tail)++] = (uint32_t)other[k];
    }
}

/*
 * Cluster roots of the bond configuration of step t: label[g] = smallest site
 * index of the cluster of g.  Breadth-first search started from every
 * unlabelled site in increasing order, so each search starts at its cluster's
 * smallest index.
 */
int oracle_cluster_labels(const cl_desc *d, const int8_t *s, uint32_t t, uint32_t *label)
{
    bond_ctx b;
    uint64_t N, g;
    uint32_t *queue;
    if (!cl_desc_ok(d))
        return CL_EINVAL;
    N = (uint64_t)d->Lx * (uint64_t)d->Ly;
    queue = (uint32_t *)malloc(N * sizeof(uint32_t));
    if (!queue)
        return CL_ENOMEM;
    b.d = d;
    b.s = s;
    b.t = t;
    oracle_bond_threshold(d->J, d->beta, &b.thr, &b.none);
    for (g = 0; g < N; ++g)
        label[g] = 0xffffffffu;
    for (g = 0; g < N; ++g) {
        uint64_t head = 0, tail = 0;
        if (label[g] != 0xffffffffu)
            continue;
        label[g] = (uint32_t)g;
        queue[tail++] = (uint32_t)g;
        while (head < tail)
            visit_neighbours(&b, queue[head++], label, (uint32_t)g, queue, &tail);
    }
    free(queue);
    return CL_OK;
}

static int sw_flips(const cl_desc *d, uint32_t root, uint32_t t)
{
    uint32_t w[4];
    draw(d, root >> 7, t, 8u, w);
    return (w[(root >> 5) & 3u] >> (root & 31u)) & 1u;
}

uint32_t oracle_wolff_seed(const cl_desc *d, uint32_t t)
{
    uint32_t w[4];
    const uint64_t N = (uint64_t)d->Lx * (uint64_t)d->Ly;
    draw(d, 0u, t, 9u, w);
    return (uint32_t)((((uint64_t)w[0] << 32) | w[1]) % N);
}

static int sw_step(const cl_desc *d, int8_t *s, uint32_t t, uint32_t *label)
{
    const uint64_t N = (uint64_t)d->Lx * (uint64_t)d->Ly;
    uint64_t g;
    int st = oracle_cluster_labels(d, s, t, label);
    if (st != CL_OK)
        return st;
    for (g = 0; g < N; ++g)
        if (sw_flips(d, label[g], t))
            s[g] = (int8_t)(-s[g]);
    return CL_OK;
}

/* Wolff growth from the seed: a stack of cluster sites whose bonds are still
 * to be tested; in[] marks membership. */
static int wolff_step(const cl_desc *d, int8_t *s, uint32_t t, uint32_t *in)
{
    const uint64_t N = (uint64_t)d->Lx * (uint64_t)d->Ly;
    uint32_t *stack;
    uint64_t top = 0, g, k;
    bond_ctx b;
    uint32_t seed;
    stack = (uint32_t *)malloc(N * sizeof(uint32_t));
    if (!stack)
        return CL_ENOMEM;
    b.d = d;
    b.s = s;
    b.t = t;
    oracle_bond_threshold(d->J, d->beta, &b.thr, &b.none);
    for (g = 0; g < N; ++g)
        in[g] = 0xffffffffu;
    seed = oracle_wolff_seed(d, t);
    in[seed] = 1;
    stack[top++] = seed;
    while (top > 0) {
        const uint32_t v = stack[--top];
        visit_neighbours(&b, v, in, 1u, stack, &top);
    }
    for (k = 0; k < N; ++k)
        if (in[k] == 1u)
            s[k] = (int8_t)(-s[k]);
    free(stack);
    return CL_OK;
}

/*
 * n cluster steps of one replica from counter t0 (algorithm CL_SWENDSEN_WANG
 * or CL_WOLFF).  After the step with run-local index i, if
 * (i + 1) % record_every == 0, (B, M) go to bond[j], mag[j] with
 * j = (i + 1) / record_every - 1.
 */
int oracle_cluster_steps(const cl_desc *d, int8_t *s, int32_t algorithm, uint64_t t0, uint64_t n,
                         uint32_t record_every, int64_t *bond, int64_t *mag)
{
    uint32_t *work;
    uint64_t i;
    int st = CL_OK;
    if (!cl_desc_ok(d) || t0 + n > 0x100000000ull ||
        (algorithm != CL_SWENDSEN_WANG && algorithm != CL_WOLFF))
        return CL_EINVAL;
    work = (uint32_t *)malloc((uint64_t)d->Lx * (uint64_t)d->Ly * sizeof(uint32_t));
    if (!work)
        return CL_ENOMEM;
    for (i = 0; i < n && st == CL_OK; ++i) {
        const uint32_t t = (uint32_t)(t0 + i);
        st = algorithm == CL_SWENDSEN_WANG ? sw_step(d, s, t, work) : wolff_step(d, s, t, work);
        if (st == CL_OK && record_every && bond && mag && (i + 1) % record_every == 0) {
            uint64_t j = (i + 1) / record_every - 1;
            oracle_observables(d->Lx, d->Ly, s, &bond[j], &mag[j]);
        }
    }
    free(work);
    return st;
}

/* ---- many independent replicas on host threads -------------------------- */

typedef struct {
    int32_t n, stride, first, algorithm;
    const cl_desc *d;
    int8_t *const *states;
    const uint64_t *t0;
    uint64_t n_steps;
    uint32_t record_every;
    int64_t *bond, *mag;
    uint64_t n_rec;
    int status;
} cl_job;

static void *cl_worker(void *arg)
{
    cl_job *job = (cl_job *)arg;
    int32_t r;
    for (r = job->first; r < job->n; r += job->stride) {
        int64_t *b = job->bond ? job->bond + (uint64_t)r * job->n_rec : NULL;
        int64_t *m = job->mag ? job->mag + (uint64_t)r * job->n_rec : NULL;
        int st = oracle_cluster_steps(&job->d[r], job->states[r], job->algorithm, job->t0 ? job->t0[r] : 0,
                                      job->n_steps, job->record_every, b, m);
        if (st != CL_OK)
            job->status = st;
    }
    return NULL;
}

/* Replica r runs on thread r % n_threads; results do not depend on n_threads. */
int oracle_run_cluster_batch(int32_t n, const cl_desc *d, int8_t *const *states, int32_t algorithm,
                             const uint64_t *t0, uint64_t n_steps, uint32_t record_every, int64_t *bond,
                             int64_t *mag, int32_t n_threads)
{
    cl_job *jobs;
    pthread_t *tids;
    int32_t k, started = 0;
    int status = CL_OK;
    if (n <= 0)
        return CL_EINVAL;
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > n)
        n_threads = n;
    jobs = (cl_job *)calloc((size_t)n_threads, sizeof(cl_job));
    tids = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return CL_ENOMEM;
    }
    for (k = 0; k < n_threads; ++k) {
        jobs[k].n = n;
        jobs[k].stride = n_threads;
        jobs[k].first = k;
        jobs[k].algorithm = algorithm;
        jobs[k].d = d;
        jobs[k].states = states;
        jobs[k].t0 = t0;
        jobs[k].n_steps = n_steps;
        jobs[k].record_every = record_every;
        jobs[k].bond = bond;
        jobs[k].mag = mag;
        jobs[k].n_rec = record_every ? n_steps / record_every : 0;
        jobs[k].status = CL_OK;
    }
    for (k = 1; k < n_threads; ++k) {
        if (pthread_create(&tids[k], NULL, cl_worker, &jobs[k]) != 0)
            break;
        started = k;
    }
    cl_worker(&jobs[0]);
    for (k = started + 1; k < n_threads; ++k)
        cl_worker(&jobs[k]);
    for (k = 1; k <= started; ++k)
        pthread_join(tids[k], NULL);
    for (k = 0; k < n_threads; ++k)
        if (jobs[k].status != CL_OK)
            status = jobs[k].status;
    free(jobs);
    free(tids);
    return status;
}
