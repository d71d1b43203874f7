/*
 * The C ABI of libising.so used from plain C with the HIP runtime API only (no
 * Python, no torch): a batch of three replicas in caller-owned device memory,
 * checked against properties that hold exactly.
 *  - beta = 0: every proposal is accepted, so each sweep negates the lattice:
 *    after 3 sweeps the spins are the negated start, the bond sum is that of
 *    the start after every sweep and the magnetisation alternates in sign;
 *  - beta = infinity from a cold start: nothing ever flips;
 *  - the recorded traces end at the values ising_batch_observables returns,
 *    the sweep counter reads 3, and a NULL handle is rejected with detail.
 * Exit status 0 and "ok" on success.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ising.h"

#define CHECK(expr)                                                                                    \
    do {                                                                                               \
        int rc_ = (expr);                                                                              \
        if (rc_ != ISING_OK) {                                                                         \
            fprintf(stderr, "%s:%d %s -> %s (%s)\n", __FILE__, __LINE__, #expr, ising_strerror(rc_),  \
                    ising_last_error());                                                               \
            return 1;                                                                                  \
        }                                                                                              \
    } while (0)
#define HIPCHECK(expr)                                                                                 \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) {                                                                        \
            fprintf(stderr, "%s:%d %s -> %s\n", __FILE__, __LINE__, #expr, hipGetErrorString(e_));     \
            return 1;                                                                                  \
        }                                                                                              \
    } while (0)
#define EXPECT(cond)                                                                                   \
    do {                                                                                               \
        if (!(cond)) {                                                                                 \
            fprintf(stderr, "%s:%d expected %s\n", __FILE__, __LINE__, #cond);                         \
            return 1;                                                                                  \
        }                                                                                              \
    } while (0)

/* bond sum (each bond once) and magnetisation of a periodic Lx x Ly lattice of +-1 */
static void observe(const int8_t *s, int Lx, int Ly, long long *B, long long *M)
{
    long long b = 0, m = 0;
    for (int y = 0; y < Ly; ++y)
        for (int x = 0; x < Lx; ++x) {
            const int v = s[y * Lx + x];
            b += v * (s[y * Lx + (x + 1) % Lx] + s[((y + 1) % Ly) * Lx + x]);
            m += v;
        }
    *B = b;
    *M = m;
}

int main(void)
{
    enum { N = 3, SWEEPS = 3 };
    const ising_desc d[N] = {
        {128, 66, 1.0, 0.0, 12345u, 0u, ISING_INIT_RANDOM, ISING_RNG_SITE},
        {64, 64, 1.0, INFINITY, 777u, 1u, ISING_INIT_UP, ISING_RNG_SITE},
        {192, 34, 1.0, 0.4, 4242u, 2u, ISING_INIT_RANDOM, ISING_RNG_BITSLICED},
    };
    size_t bytes = 0;
    CHECK(ising_state_bytes(N, d, &bytes));
    void *buf = NULL;
    int64_t *bond = NULL, *mag = NULL;
    hipStream_t st;
    HIPCHECK(hipStreamCreate(&st));
    HIPCHECK(hipMalloc(&buf, bytes));
    HIPCHECK(hipMalloc((void **)&bond, sizeof(int64_t) * N * SWEEPS));
    HIPCHECK(hipMalloc((void **)&mag, sizeof(int64_t) * N * SWEEPS));
    ising_batch *b = NULL;
    CHECK(ising_batch_create(N, d, buf, bytes, st, &b));

    int8_t *s0 = malloc((size_t)d[0].Lx * d[0].Ly), *s1 = malloc((size_t)d[0].Lx * d[0].Ly);
    int8_t *c = malloc((size_t)d[1].Lx * d[1].Ly);
    CHECK(ising_batch_get_spins(b, 0, s0, st));
    long long B0, M0;
    observe(s0, d[0].Lx, d[0].Ly, &B0, &M0);

    CHECK(ising_batch_run(b, SWEEPS, 1, bond, mag, st));
    int64_t hb[N * SWEEPS], hm[N * SWEEPS], ob[N], om[N];
    HIPCHECK(hipMemcpyAsync(hb, bond, sizeof hb, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(hm, mag, sizeof hm, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    CHECK(ising_batch_observables(b, ob, om, st));

    /* beta = 0: negated after an odd number of sweeps; B constant, M alternating */
    CHECK(ising_batch_get_spins(b, 0, s1, st));
    for (int i = 0; i < d[0].Lx * d[0].Ly; ++i)
        EXPECT(s1[i] == -s0[i]);
    for (int k = 0; k < SWEEPS; ++k) {
        EXPECT(hb[0 * SWEEPS + k] == B0);
        EXPECT(hm[0 * SWEEPS + k] == ((k % 2 == 0) ? -M0 : M0));
    }
    /* beta = infinity from all +1: frozen at B = 2N, M = N */
    CHECK(ising_batch_get_spins(b, 1, c, st));
    for (int i = 0; i < d[1].Lx * d[1].Ly; ++i)
        EXPECT(c[i] == 1);
    EXPECT(hb[1 * SWEEPS + SWEEPS - 1] == 2LL * d[1].Lx * d[1].Ly && hm[1 * SWEEPS + SWEEPS - 1] == (long long)d[1].Lx * d[1].Ly);
    /* the traces end where the observables call is */
    for (int r = 0; r < N; ++r)
        EXPECT(hb[r * SWEEPS + SWEEPS - 1] == ob[r] && hm[r * SWEEPS + SWEEPS - 1] == om[r]);
    uint64_t t = 0;
    CHECK(ising_batch_get_sweep(b, 2, &t, st));
    EXPECT(t == SWEEPS);
    /* a NULL handle is an error with detail, not a crash */
    EXPECT(ising_batch_run(NULL, 1, 0, NULL, NULL, st) == ISING_E_INVALID);
    EXPECT(strlen(ising_last_error()) > 0);

    CHECK(ising_batch_destroy(b));
    HIPCHECK(hipFree(buf));
    HIPCHECK(hipFree(bond));
    HIPCHECK(hipFree(mag));
    HIPCHECK(hipStreamDestroy(st));
    free(s0);
    free(s1);
    free(c);
    printf("ok\n");
    return 0;
}
