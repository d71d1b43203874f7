/*
 * ising3d.h — C ABI of the 3D part of libising.so: red/black Metropolis sweeps
 * of the periodic simple-cubic Ising model, H = -J sum_<ij> s_i s_j with six
 * neighbours per spin (paper section 1 names 3D, with 6 neighbours, as the
 * generalisation of the 2D model it simulates), for a batch of independent
 * replicas on one GPU.
 *
 * Conventions are those of ising.h (status codes ISING_*, caller-owned device
 * memory, streams passed as void*, one host thread per handle,
 * ising_last_error() for detail), with these definitions:
 *  - site (x, y, z), 0 <= x < Lx, 0 <= y < Ly, 0 <= z < Lz; linear index
 *    g = (z*Ly + y)*Lx + x; colour c = (x + y + z) & 1, so that the six
 *    neighbours of a site have the other colour.  A sweep updates every
 *    colour-0 site, then every colour-1 site.
 *  - dE = 2 J s (sum of the six neighbours); dE <= 0 and beta*J == 0 accept
 *    without a draw; dE = 4J, 8J, 12J accept iff r < thr_k =
 *    min(floor(exp(-4 k beta J) 2^32), 2^32 - 1), k = 1, 2, 3.
 *  - r of the colour-c site g in sweep t, h = g >> 1: under ISING_RNG_SITE
 *    word (h & 3) of Philox4x32-10(ctr = {h >> 2, t, replica, c}, key = seed);
 *    under ISING_RNG_BITSLICED the colour-c sites h = 32q .. 32q + 31 form
 *    group q with words W_k = word (k & 3) of Philox(ctr = {8q + (k >> 2), t,
 *    replica, c}), k = 0..31, and site 32q + b's uniform has bit 31 - k equal
 *    to bit b of W_k (the 2D definition of ising.h on the 3D index).
 *  - init ISING_INIT_RANDOM: s = +1 iff word (g & 3) of Philox(ctr = {g >> 2,
 *    0, replica, 2}) >= 2^31; ISING_INIT_UP / ISING_INIT_DOWN: all +1 / -1.
 *  - observables: B = sum s(x,y,z) (s(x+1,y,z) + s(x,y+1,z) + s(x,y,z+1)),
 *    every bond once (E = -J B); M = sum s.
 * Layout in device memory: per replica two colour planes of Lz*Ly rows
 * (row index z*Ly + y) of Lx/64 uint32 words; bit k of word w of a row holds
 * the site of that colour with compact index 32 w + k, at column
 * x = 2 (32 w + k) + ((c + y + z) & 1).
 */
#ifndef ISING3D_H
#define ISING3D_H

#include <stddef.h>
#include <stdint.h>

#include "ising.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * One 3D replica.  Lx a positive multiple of 64, Ly and Lz even and >= 2,
 * Lx*Ly*Lz < 2^32 (ISING_E_UNSUPPORTED otherwise); J finite and > 0, beta >= 0
 * or +infinity, init one of ISING_INIT_*, rng ISING_RNG_SITE or
 * ISING_RNG_BITSLICED (ISING_E_INVALID otherwise).
 */
typedef struct {
    int32_t Lx, Ly, Lz;
    int32_t init;
    double J, beta;
    uint64_t seed;
    uint32_t replica;
    int32_t rng;
} ising3d_desc;

typedef struct ising3d_batch ising3d_batch;

/* Bytes of device memory a batch of n 3D replicas needs (host-only). */
int ising3d_state_bytes(int32_t n, const ising3d_desc *d, size_t *bytes);

/* Create a batch in dev_buf (>= ising3d_state_bytes bytes, 256-byte aligned)
 * and initialise every replica on stream.  Blocking.  Sweep counters start
 * at 0. */
int ising3d_batch_create(int32_t n, const ising3d_desc *d, void *dev_buf, size_t bytes, void *stream,
                         ising3d_batch **out);

/* n_sweeps sweeps of every replica, asynchronous on stream; recording as in
 * ising_batch_run: after the sweep with run-local index i, if
 * (i + 1) % record_every == 0, (B, M) go to dev_bond_trace[r * n_rec + j],
 * dev_mag_trace[r * n_rec + j], j = (i + 1) / record_every - 1.  Counters
 * must stay below 2^32 (ISING_E_INVALID). */
int ising3d_batch_run(ising3d_batch *b, uint64_t n_sweeps, uint32_t record_every, int64_t *dev_bond_trace,
                      int64_t *dev_mag_trace, void *stream);

/* Current (B, M) of every replica into host arrays of n int64 (blocking). */
int ising3d_batch_observables(ising3d_batch *b, int64_t *host_bond, int64_t *host_mag, void *stream);

/* Replica r's spins to / from a host int8 array of Lx*Ly*Lz values +-1 at
 * index g (blocking); set_spins rejects other values (ISING_E_INVALID). */
int ising3d_batch_get_spins(ising3d_batch *b, int32_t r, int8_t *host_pm1, void *stream);
int ising3d_batch_set_spins(ising3d_batch *b, int32_t r, const int8_t *host_pm1, void *stream);

/* Replica r's sweep counter (value after all enqueued work). */
int ising3d_batch_get_sweep(ising3d_batch *b, int32_t r, uint64_t *t, void *stream);

int ising3d_batch_destroy(ising3d_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* ISING3D_H */
