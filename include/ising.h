/*
 * ising.h — C ABI of the MI355X checkerboard Metropolis library (libising.so).
 *
 * The library runs red/black Metropolis sweeps of the periodic 2D
 * nearest-neighbour Ising model, H = -J sum_<ij> s_i s_j with s = +-1 and
 * J > 0 (paper section 1), for a batch of independent replicas, each with its
 * own size, coupling, temperature, seed and replica id.  A sweep updates every
 * red site ((x+y) even) and then every blue site, each proposal accepted by the
 * Metropolis rule ran() < exp(-beta dE) (section 1; section 2 and the
 * checkerboard multi-spin algorithm of the Supplementary Information, S.1).
 *
 * Conventions shared by every call:
 *  - Plain C; every function returns an int status: ISING_OK (0) or a
 *    negative ISING_E_* code.  ising_last_error() gives detail for the
 *    calling thread.
 *  - All device memory belongs to the caller.  ising_state_bytes() says how
 *    many bytes of device memory a batch needs; the caller allocates them
 *    (any allocator) and keeps them alive, unmoved, until
 *    ising_batch_destroy().  The library allocates no device memory; it owns
 *    only host-side metadata.
 *  - "stream" arguments are hipStream_t values passed as void* (NULL = the
 *    null stream).  Calls documented as asynchronous only enqueue work on that
 *    stream; device faults surface at the next blocking call.
 *  - A handle must not be used from two host threads at once.
 *  - Spin encoding inside the library: 1 bit per spin, bit 1 <=> s = +1.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the
 *    replica's 64-bit seed; the uniform of site (x, y) in sweep t is word
 *    (h & 3) of Philox(ctr = {h >> 2, t, replica, colour}), h = (y*Lx + x) >> 1,
 *    colour = (x + y) & 1.  Results therefore do not depend on word width,
 *    launch shape or how replicas are batched.
 *  - Acceptance: dE <= 0 always; dE = 4J iff r < floor(exp(-4 beta J) 2^32);
 *    dE = 8J iff r < floor(exp(-8 beta J) 2^32) (thresholds clamped to
 *    2^32 - 1; beta*J == 0 accepts everything).
 *  - Observables: bond sum B = sum_{x,y} s(x,y) (s(x+1,y) + s(x,y+1)), every
 *    bond once, so E = -J B; magnetisation M = sum s (|M| is the observable of
 *    paper section 3.1).
 */
#ifndef ISING_H
#define ISING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ISING_OK = 0,
    ISING_E_INVALID = -1,     /* an argument is out of range or inconsistent */
    ISING_E_UNSUPPORTED = -2, /* valid physics, but a shape this library does not run */
    ISING_E_NOMEM = -3,       /* host allocation failed or a caller buffer is too small */
    ISING_E_HIP = -4,         /* a HIP runtime call failed; detail in ising_last_error() */
    ISING_E_STATE = -5        /* the call is not valid in the handle's current state */
};

enum { ISING_INIT_RANDOM = 0, ISING_INIT_UP = 1, ISING_INIT_DOWN = 2 };

/*
 * One replica (one simulation; the paper runs one per PE column, section 2).
 *  Lx, Ly   columns and rows; Lx must be a positive multiple of 64 and Ly even
 *           and >= 2 (ISING_E_UNSUPPORTED otherwise); Lx*Ly < 2^32.
 *  J        coupling, finite and > 0 (ISING_E_INVALID otherwise).
 *  beta     inverse temperature 1/T (k_B = 1), >= 0; +infinity means T = 0.
 *  seed     64-bit Philox key of this replica.
 *  replica  32-bit replica id (third Philox counter word); replicas that share
 *           a seed must differ here to draw independent numbers.
 *  init     ISING_INIT_RANDOM: s = +1 iff word (g & 3) of
 *           Philox(ctr = {g >> 2, 0, replica, 2}) >= 2^31 with g = y*Lx + x
 *           (the paper starts from a completely random configuration,
 *           section 3.1); ISING_INIT_UP / ISING_INIT_DOWN: all +1 / all -1.
 *  rng      which uniform a proposal with dE > 0 is compared with (section 1's
 *           ran(); the paper's generator is unpublished, Supplementary S.4):
 *           ISING_RNG_SITE: for the colour-c site with compact index
 *             h = (y*Lx + x) >> 1 in sweep t, word (h & 3) of
 *             Philox4x32-10(ctr = {h >> 2, t, replica, c}, key = seed);
 *           ISING_RNG_BITSLICED: the colour-c sites h = 32g .. 32g+31 form
 *             group g with words W_k = word (k & 3) of Philox(ctr =
 *             {8g + (k >> 2), t, replica, c}), k = 0..31, and site 32g + b
 *             takes the uniform whose bit 31 - k is bit b of W_k.  Compared
 *             with the threshold from the top bit down, most sites are decided
 *             after a few words, so the library draws only the words needed.
 *           Both give exact Metropolis acceptance; they give different
 *           trajectories (ISING_E_INVALID for other values).
 */
enum { ISING_RNG_SITE = 0, ISING_RNG_BITSLICED = 1 };

typedef struct {
    int32_t Lx, Ly;
    double J, beta;
    uint64_t seed;
    uint32_t replica;
    int32_t init;
    int32_t rng;
} ising_desc;

typedef struct ising_batch ising_batch;

/* Static text for a status code. */
const char *ising_strerror(int code);

/* Detail of the last failure on the calling thread ("" if none); valid until
 * the next library call on this thread. */
const char *ising_last_error(void);

/*
 * Bytes of device memory needed for a batch of n replicas described by d[0..n).
 * Pure host computation (no device call).  Errors: ISING_E_INVALID (n <= 0,
 * NULL pointers, bad J/beta/init), ISING_E_UNSUPPORTED (bad shape).
 */
int ising_state_bytes(int32_t n, const ising_desc *d, size_t *bytes);

/*
 * Create a batch in the caller's device buffer dev_buf (bytes >= the value
 * from ising_state_bytes, 256-byte aligned) and initialise every replica on
 * stream.  Sweep counters start at 0.  Blocking: returns once the
 * descriptors are uploaded and the initial states written.
 * On success *out holds the handle.  Errors: as ising_state_bytes, plus
 * ISING_E_NOMEM (buffer too small or host allocation failure), ISING_E_HIP.
 */
int ising_batch_create(int32_t n, const ising_desc *d, void *dev_buf, size_t bytes,
                       void *stream, ising_batch **out);

/*
 * Run n_sweeps full sweeps (red then blue, Supplementary algorithm S2) of
 * every replica.  Asynchronous on stream.  Replica r's sweep counter t_r
 * advances by n_sweeps and must stay below 2^32 (ISING_E_INVALID otherwise).
 * Running a then b sweeps gives exactly the state of running a + b.
 *
 * If record_every > 0 and both trace pointers are non-NULL, after the sweep
 * with run-local index i (0-based) such that (i + 1) % record_every == 0 the
 * replica's (B, M) are written to dev_bond_trace[r * n_rec + j] and
 * dev_mag_trace[r * n_rec + j], j = (i + 1) / record_every - 1,
 * n_rec = n_sweeps / record_every.  Both traces are device arrays of at least
 * n * n_rec int64 values owned by the caller; every slot is written.
 * record_every == 0 or NULL traces record nothing.
 */
int ising_batch_run(ising_batch *b, uint64_t n_sweeps, uint32_t record_every,
                    int64_t *dev_bond_trace, int64_t *dev_mag_trace, void *stream);

/*
 * Current (B, M) of every replica into host arrays of n int64 each.
 * Blocking: enqueues a popcount reduction on stream and waits for it.
 */
int ising_batch_observables(ising_batch *b, int64_t *host_bond, int64_t *host_mag,
                            void *stream);

/*
 * Copy replica r's spins to / from a host int8 array of Lx*Ly values +-1 in
 * row-major order (index y*Lx + x).  Blocking on stream.  set_spins rejects
 * values other than +-1 with ISING_E_INVALID and leaves the state unchanged.
 */
int ising_batch_get_spins(ising_batch *b, int32_t r, int8_t *host_pm1, void *stream);
int ising_batch_set_spins(ising_batch *b, int32_t r, const int8_t *host_pm1, void *stream);

/* Read / set replica r's sweep counter (for checkpoint and resume).  The
 * counter read is the value after all work enqueued so far; set_sweep blocks
 * until the new value is on the device. */
int ising_batch_get_sweep(ising_batch *b, int32_t r, uint64_t *t, void *stream);
int ising_batch_set_sweep(ising_batch *b, int32_t r, uint64_t t, void *stream);

/* Change replica r's inverse temperature (same validity rules as in
 * ising_desc); thresholds are recomputed.  Blocking; applies to sweeps
 * enqueued afterwards. */
int ising_batch_set_beta(ising_batch *b, int32_t r, double beta, void *stream);

/*
 * Cluster steps: Swendsen-Wang and Wolff, the non-local updates that paper
 * section 1 names as the cure for the critical slowing down of single-spin
 * Metropolis near T_c (algorithms from Swendsen and Wang, PRL 58, 86 (1987),
 * and Wolff, PRL 62, 361 (1989)).  A step acts on the batch's packed state
 * and uses the replica's counter t like a sweep, so sweeps and steps can be
 * interleaved in any order.
 *  bonds     site g = y*Lx + x owns a "right" bond to ((x+1) mod Lx, y) and a
 *            "down" bond to (x, (y+1) mod Ly) (with Ly = 2 each vertical pair
 *            has two bonds).  In step t a bond is occupied iff its two spins
 *            are equal, beta*J > 0 and its word is >= thr2 =
 *            min(floor(exp(-2 beta J) 2^32), 2^32 - 1) (the Fortuin-Kasteleyn
 *            probability 1 - exp(-2 beta J)); the right bond's word is word
 *            2(g & 1), the down bond's word 2(g & 1) + 1 of
 *            Philox(ctr = {g >> 1, t, replica, 7}).
 *  clusters  connected components of the occupied bonds; a cluster's root is
 *            its smallest site index.
 *  ISING_CLUSTER_SWENDSEN_WANG  the cluster with root R flips iff bit R & 31
 *            of word (R >> 5) & 3 of Philox(ctr = {R >> 7, t, replica, 8}) is 1.
 *  ISING_CLUSTER_WOLFF  with w = Philox(ctr = {0, t, replica, 9}) the cluster
 *            of site S = ((w0 << 32) | w1) mod (Lx*Ly) flips.
 */
enum { ISING_CLUSTER_SWENDSEN_WANG = 0, ISING_CLUSTER_WOLFF = 1 };

/* Bytes of device workspace ising_batch_cluster needs for batch b: a 32-bit
 * label per site of every replica (each replica's labels 256-byte aligned)
 * plus 16 bytes per tile of 64 x 64 sites.  Host-only.
 * Errors: ISING_E_INVALID (NULL argument). */
int ising_cluster_ws_bytes(ising_batch *b, size_t *bytes);

/*
 * n_steps cluster steps of every replica with the given algorithm.
 * Asynchronous on stream.  Each step uses counter t_r and advances it by one;
 * t_r + n_steps must stay below 2^32.
 *  dev_ws     caller-owned device scratch of ws_bytes >= ising_cluster_ws_bytes()
 *             bytes, 256-byte aligned.  It holds nothing between calls, and no
 *             other work may use it while the call's kernels run.
 *  record_every, dev_bond_trace, dev_mag_trace  as in ising_batch_run, with
 *             steps in place of sweeps.
 * Whole chunks of 16 steps are captured once per (algorithm, workspace,
 * traces) in a hipGraph and replayed; the trace slot of a step is computed on
 * the device, so results do not depend on how a run is split into calls.
 * Errors: ISING_E_INVALID (NULL handle or workspace, misaligned workspace,
 * unknown algorithm, counter overflow), ISING_E_NOMEM (ws_bytes too small),
 * ISING_E_HIP.
 */
int ising_batch_cluster(ising_batch *b, int32_t algorithm, uint64_t n_steps, uint32_t record_every,
                        void *dev_ws, size_t ws_bytes, int64_t *dev_bond_trace, int64_t *dev_mag_trace,
                        void *stream);

/*
 * ising_batch_cluster without a caller workspace, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is the library's own:
 * ISING_CLUSTER_STATIC_WS_BYTES bytes of device memory in the loaded code
 * object, one copy per device, held until the process ends; its address on a
 * device is looked up on the first call with that device current.  Steps are
 * launched directly (no graph is captured), and nothing is allocated.  Every
 * call on one device shares that workspace: calls whose work overlaps on one
 * device (other streams, other threads) race and must be serialised by the
 * caller.  The workspace holds nothing between calls (each step rewrites all
 * of it that it reads), so results equal ising_batch_cluster's bit for bit.
 * The current device must be the batch's device.
 * Errors: ISING_E_INVALID (as ising_batch_cluster; current device is not the
 * batch's), ISING_E_NOMEM (ising_cluster_ws_bytes() of the batch exceeds
 * ISING_CLUSTER_STATIC_WS_BYTES; the detail gives both sizes), ISING_E_HIP.
 */
#define ISING_CLUSTER_STATIC_WS_BYTES ((size_t)64 << 20)
int ising_batch_cluster_static(ising_batch *b, int32_t algorithm, uint64_t n_steps, uint32_t record_every,
                               int64_t *dev_bond_trace, int64_t *dev_mag_trace, void *stream);

/*
 * Execution schedule (what the autotuner chooses; every schedule gives
 * bit-identical results).
 *  word_bits        32 or 64: bits per machine word a thread updates
 *                   (64 needs Lx % 128 == 0; such replicas fall back to 32).
 *  resident_max_bytes  replicas whose two colour planes fit in this many
 *                   bytes of LDS run whole sweeps inside one workgroup;
 *                   0 disables that mode, larger than the device's LDS per
 *                   workgroup is clamped.
 *  resident_threads workgroup size of the LDS-resident mode (64..1024, a
 *                   multiple of 64).
 *  stream_threads   workgroup size of the streaming mode (64..1024).
 *  stream_words     words per streaming workgroup (a multiple of stream_threads).
 *  sweeps_per_launch  sweeps per graph launch / resident launch (>= 1).
 *  use_graph        1: capture sweeps_per_launch sweeps into a hipGraph and
 *                   replay it; 0: launch kernels directly.
 */
typedef struct {
    int32_t word_bits;
    int32_t resident_max_bytes;
    int32_t resident_threads;
    int32_t stream_threads;
    int32_t stream_words;
    int32_t sweeps_per_launch;
    int32_t use_graph;
} ising_schedule;

int ising_batch_get_schedule(ising_batch *b, ising_schedule *s);
/* Validates s (ISING_E_INVALID) and installs it; cached graphs are dropped. */
int ising_batch_set_schedule(ising_batch *b, const ising_schedule *s);

/*
 * Choose the execution schedule by measurement (the project's autotuner) and
 * install it.  Blocking.  The batch's planes are saved to host memory; each
 * candidate schedule then runs trial_sweeps sweeps (>= 1) from that same saved
 * state, timed with HIP events after one untimed warm-up pass, and its final
 * planes must equal the first candidate's bit for bit (ISING_E_STATE
 * otherwise: that would be a kernel bug, and the detail names the candidate).
 * Candidates are searched one schedule field at a time (word width, resident
 * threshold and workgroup size, streaming workgroup shape, sweeps per launch);
 * a candidate replaces the current best only when it is at least 2 % faster.
 * Every candidate runs the same number of sweeps: trial_sweeps rounded up to
 * a multiple of 100 (so every sweeps_per_launch candidate, 10, 25, 50 and
 * 100, runs whole chunks and the graph replays a timed run uses are the ones
 * timed and checked); its warm-up pass is one chunk (which also captures the
 * chunk's graph).
 * Afterwards the saved planes and sweep counters are restored, so tuning
 * leaves the simulation unchanged.  If the environment variable
 * ISING_AUTOTUNE_CACHE names a file, a schedule stored there for the same
 * device and the same multiset of (lattice shape, random-number contract) is
 * installed without
 * measuring, and new results are appended to it.  *chosen (optional) receives
 * the installed schedule; *n_tried (optional) the number of candidates timed
 * (0 on a cache hit).
 */
int ising_batch_autotune(ising_batch *b, int32_t trial_sweeps, ising_schedule *chosen,
                         int32_t *n_tried, void *stream);

/* Number of replicas in each execution mode under the current schedule. */
int ising_batch_mode_counts(ising_batch *b, int32_t *n_resident, int32_t *n_streamed);

/*
 * Captured-graph bookkeeping of batch b (host-only, no device call).
 * ising_batch_run and ising_batch_cluster replay one captured hipGraph per
 * chunk length (sweeps_per_launch sweeps, or 16 cluster steps per algorithm,
 * workspace and recording on/off); the trace pointers and record cadence of a
 * call are written to device memory before its replays, so calls with other
 * trace buffers reuse the same graph.  *n_cached (optional) receives the
 * number of executable graphs held now, *n_captured (optional) the number of
 * captures since the batch was created.  Executable graphs are destroyed
 * (schedule change, destroy) only after the replays enqueued by the last
 * call that launched any have finished.  Errors: ISING_E_INVALID (NULL handle).
 */
int ising_batch_graph_stats(ising_batch *b, int32_t *n_cached, int64_t *n_captured);

/* ==========================================================================
 * Learned block proposals.
 *
 * A small autoregressive network proposes a joint update of one Bs x Bs
 * block (Bs = 2, 4 or 8) given the block's 4*Bs boundary spins and the
 * coupling K = beta*J, one site at a time in raster order (k = i*Bs + j):
 * four masked 3x3 convolution layers of 64 channels (the first sees only
 * earlier sites, the others also the current position of the previous layer),
 * tanh activations, per-site boundary features and K as inputs, and a 1x1
 * logit head; layers 2..4 run on BF16 matrix cores with FP32 accumulation.
 * Site k is proposed +1 with probability thr_k / 2^32,
 * thr_k = clamp(floor(sigmoid(logit_k) 2^32), 1, 2^32 - 1), using the uniform
 * word (s & 3) of Philox(ctr = {s >> 2, round, replica, 3}), s = blk*Bs*Bs + k,
 * so log q of a block is an exact sum of logs of thresholds (FP64).  A
 * proposal is accepted with the Metropolis-Hastings probability
 * min(1, pi(s') q(s) / (pi(s) q(s'))), pi ~ exp(K * bond sum), using the 53-bit
 * uniform ((w0 << 21) | (w1 >> 11)) 2^-53 of Philox(ctr = {blk, round, replica, 4});
 * q(s) of the current block is scored by the same kernel code that samples,
 * so the stationary distribution stays the Boltzmann distribution of the
 * paper's section 1 whatever the network has learned.
 *
 * Flat float parameter vector (C = 64 channels): W1[4][C] (spin taps
 * (-1,-1), (-1,0), (-1,1), (0,-1)), U1[4][C] (boundary up, down, left, right),
 * v1[C] (K), b1[C], then for layers 2..4 W[5][C][C] (the four taps and the
 * centre; index [tap][in][out]) and b[C], then wo[C], bo[1].
 * Block data layout: spins int8 [n][Bs*Bs] row-major; boundary int8
 * [n][4*Bs] = top row, bottom row, left column, right column (values +-1);
 * coupling float [n].
 * ========================================================================== */
typedef struct ising_nn ising_nn;

/* Number of floats in the parameter vector for `channels` channels (64 only). */
int ising_nn_param_count(int32_t channels, int32_t *count);

/* Device bytes for a network with training batches of up to max_batch blocks
 * and incremental passes of up to max_seq sequences per launch. */
int ising_nn_state_bytes(int32_t block, int32_t channels, int32_t max_batch, int32_t max_seq, size_t *bytes);

/* Create a network in the caller's device buffer (256-byte aligned) from host
 * parameters (param_count floats).  Adam moments start at zero.  Blocking. */
int ising_nn_create(int32_t block, int32_t channels, int32_t max_batch, int32_t max_seq,
                    const float *host_params, void *dev_buf, size_t bytes, void *stream, ising_nn **out);
int ising_nn_get_params(ising_nn *m, float *host_params, void *stream);  /* blocking */
int ising_nn_set_params(ising_nn *m, const float *host_params, void *stream);  /* blocking; resets Adam */

/* Teacher-forced forward and backward on `batch` blocks (device arrays):
 * per-site logits (float [batch*Bs*Bs], may be NULL), the gradient of the
 * mean per-site negative log-likelihood (float [param_count], may be NULL)
 * and the loss (float [1]).  Asynchronous. */
int ising_nn_forward_backward(ising_nn *m, const int8_t *dev_blocks, const int8_t *dev_bnd,
                              const float *dev_coupling, int32_t batch, float *dev_logits, float *dev_grad,
                              float *dev_loss, void *stream);

/* One Adam step (Kingma and Ba's Algorithm 1: beta1 0.9, beta2 0.999, eps
 * 1e-8, bias corrections 1 - beta^t with t the step number since the
 * parameters were last set, kept on the device) on `batch` blocks; the loss
 * before the step goes to dev_loss.  The whole step (forward, backward,
 * Adam, BF16 weight copies) is captured into a hipGraph the first time it is
 * called with a given set of arguments and replayed afterwards; at most 8
 * argument sets are kept (the oldest are destroyed once their replays have
 * finished).  Asynchronous. */
int ising_nn_train_step(ising_nn *m, const int8_t *dev_blocks, const int8_t *dev_bnd, const float *dev_coupling,
                        int32_t batch, float lr, float *dev_loss, void *stream);

/* ising_nn_train_step on a minibatch the library draws from a training set of
 * n_rows blocks (dev_blocks [n_rows][Bs*Bs], dev_bnd [n_rows][4 Bs],
 * dev_coupling [n_rows], same layouts as above): row i of the k-th training
 * step since the parameters were last set is floor(u * n_rows / 2^32), u the
 * first word of Philox4x32-10(counter (i, k, 0, 6), key seed), i < batch.
 * The training kernels read the drawn rows straight from the training set,
 * so it stays where it is and the host takes no part in sampling.
 * Errors: ISING_E_INVALID for batch outside [1, max_batch], n_rows outside
 * [1, 2^32 - 1], NULL arrays or lr <= 0.  Asynchronous. */
int ising_nn_train_step_sampled(ising_nn *m, const int8_t *dev_blocks, const int8_t *dev_bnd,
                                const float *dev_coupling, int64_t n_rows, int32_t batch, float lr, uint64_t seed,
                                float *dev_loss, void *stream);

/* n_steps >= 1 consecutive ising_nn_train_step_sampled steps in one call
 * (the same rows, parameters and results as n_steps single calls; dev_loss,
 * if not NULL, holds the last step's loss).  The steps run as replays of
 * graphs of up to 16 captured steps each, so consecutive steps follow each
 * other on the GPU without a launch between them.  Errors: those of
 * ising_nn_train_step_sampled, and ISING_E_INVALID for n_steps < 1.
 * Asynchronous. */
int ising_nn_train_steps_sampled(ising_nn *m, const int8_t *dev_blocks, const int8_t *dev_bnd,
                                 const float *dev_coupling, int64_t n_rows, int32_t batch, float lr, uint64_t seed,
                                 int64_t n_steps, float *dev_loss, void *stream);

/* Autoregressive passes on n <= max_seq sequences.  Site k = i*Bs + j of a
 * block has P(x_k = +1 | x_<k, boundary, K) = sigmoid(logit_k) and the uint32
 * threshold thr_k = clamp(floor(sigmoid(logit_k) * 2^32), 1, 2^32 - 1);
 * log q = sum_k log(x_k > 0 ? thr_k : 2^32 - thr_k) - Bs*Bs*32*ln 2 in FP64.
 * sample: x_k = +1 iff u_k < thr_k, u_k = word (s & 3) of
 * Philox4x32-10(counter (s >> 2, round, replica, 3), key seed) with
 * s = (blk0 + i) * Bs*Bs + k for sequence i; returns the blocks and log q.
 * score: log q of the given blocks, evaluated row by row with the sampler's
 * per-site arithmetic, so a sampled block scores to the same log q bit for
 * bit.  Errors: ISING_E_INVALID for n outside [1, max_seq] or NULL arrays.
 * Asynchronous. */
int ising_nn_score(ising_nn *m, int32_t n, const int8_t *dev_blocks, const int8_t *dev_bnd,
                   const float *dev_coupling, double *dev_logq, void *stream);
int ising_nn_sample(ising_nn *m, int32_t n, const int8_t *dev_bnd, const float *dev_coupling, uint64_t seed,
                    uint32_t replica, uint32_t round, uint32_t blk0, int8_t *dev_blocks_out, double *dev_logq,
                    void *stream);

/* Training data from a batch (all replicas the same shape, Lx and Ly
 * multiples of 2*Bs): per_replica blocks of each replica at positions drawn
 * from Philox(ctr = {i, draw, replica, 5}) (bx = w0 mod Lx/Bs,
 * by = w1 mod Ly/Bs); writes [n*per_replica] blocks, boundaries and K.
 * Asynchronous. */
int ising_batch_extract_blocks(ising_batch *b, int32_t block, int32_t per_replica, uint32_t draw,
                               int8_t *dev_blocks, int8_t *dev_bnd, float *dev_coupling, void *stream);

/* One block round of every replica: all blocks with (bx + by) even, then all
 * with (bx + by) odd.  For each block the network scores the current spins s
 * and samples a proposal s' (block id by*(Lx/Bs) + bx, the round as Philox
 * counter word) given the block's boundary; with dB the change of the bond
 * sum, log A = K dB + log q(s) - log q(s') in FP64 and the proposal replaces
 * the block iff log A >= 0 or u < exp(log A), u = ((w0 << 21) | (w1 >> 11))
 * * 2^-53 from Philox4x32-10(counter (block id, round, replica, 4), key seed).
 * Blocks of one colour share no bond, so the order within a colour does not
 * matter.  dev_accepts (int64 [n], may be NULL) accumulates accepted blocks
 * per replica.  Errors: ISING_E_UNSUPPORTED unless every replica has one shape
 * with Lx and Ly multiples of 2*Bs.  Asynchronous. */
int ising_batch_block_round(ising_batch *b, ising_nn *m, uint32_t round, int64_t *dev_accepts, void *stream);

/* Captured training steps held now (*n_cached) and captured since creation
 * (*n_captured); either may be NULL.  Host-only. */
int ising_nn_graph_stats(ising_nn *m, int32_t *n_cached, int64_t *n_captured);

/* Free host metadata and captured graphs (after their replays finished). */
int ising_nn_destroy(ising_nn *m);

/* Free host metadata and cached graphs.  Waits only for the graph replays
 * enqueued by the batch's last call that launched any (so their executable
 * graphs outlive them); the caller must not free dev_buf while work on it is
 * still queued. */
int ising_batch_destroy(ising_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* ISING_H */
