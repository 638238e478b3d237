/*
 * aco.h -- C ABI of the MI355X (gfx950) tensorized Ant Colony Optimization
 * library for the symmetric Euclidean TSP (Yang, Jiang & Cheng, "Tensorized
 * Ant Colony Optimization for GPU Acceleration", GECCO'24 Companion).
 *
 * One iteration of the method on one GPU:
 *   transition  P = RowNormalized(tau^alpha * eta^beta)^(1/gamma)   Sec. 2.1 Eq. (1), Eq. (4)
 *   construct   every ant builds a tour by Adaptive Independent
 *               Roulette: next = argmax over unvisited j of P[c,j]*r_j  Sec. 2.2, Sec. 2.4
 *   lengths     f(s) = closed tour length                           Sec. 2.3 (Eq. 3)
 *   update      top-k elite, index-mapped deposit dTau = sum of A,
 *               evaporation, then the next P                         Sec. 2.3 Eq. (2), Eq. (3)
 *
 * Conventions
 *   - n cities, m ants.  Every matrix the library keeps is FP32, row-major,
 *     n rows with a padded leading dimension ld = aco_leading_dim(n) (a multiple
 *     of 64 floats); columns n..ld-1 are zero and never candidates.
 *   - Device memory: the caller owns all of it.  The library carves every
 *     buffer from one caller-provided workspace (aco_workspace_bytes) and calls
 *     no device allocator.  The context object itself is a small host struct.
 *   - Asynchrony: calls enqueue work on the HIP stream bound at creation and
 *     return.  Exceptions that block the host: aco_create (validates the
 *     distance matrix), aco_set_eta (validates eta), aco_run (final copy),
 *     aco_best and aco_sync.
 *   - Errors: every call returns an aco_status; nothing aborts or throws across
 *     the ABI.  aco_last_error() gives a thread-local message for the last
 *     failure.  Device faults surface as ACO_EDEVICE at the next blocking call.
 *   - Random numbers: a counter-based Philox4x32-10 (Salmon, Moraes, Dror &
 *     Shaw, SC'11) with key = (seed mod 2^32, seed >> 32).  The deviate r_j that
 *     ant a draws for city j at step s of iteration t is word (j mod 4) of
 *     counter (j/4, s, a, t), mapped to (2*(w>>9)+1) * 2^-24.  The start city
 *     of ant a is (w0 * n) >> 32 with w0 word 0 of counter (0, 0, a, t).
 *     Results therefore do not depend on launch shape or scheduling.
 */
#ifndef ACO_H
#define ACO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aco_ctx aco_ctx;

typedef enum {
    ACO_OK = 0,
    ACO_EINVAL = -1,  /* bad argument, shape or input matrix            */
    ACO_ENOMEM = -2,  /* workspace too small                             */
    ACO_EDEVICE = -3, /* HIP runtime error or device fault               */
    ACO_ESTATE = -4   /* call out of order (e.g. construct before any P) */
} aco_status;

/* Parameters beyond the four fixed at creation.  Defaults: tau0 = 1,
 * elite_k = 0 (every ant deposits), gamma_max = 1.5, gamma_min = 1.0. */
typedef struct {
    float tau0;      /* initial pheromone on every edge, > 0                      */
    int32_t elite_k; /* 0: all ants deposit; 0 < k <= m: the k shortest (Sec. 2.3) */
    float gamma_max; /* AdaIR exponent at the first iteration (Sec. 2.4), > 0      */
    float gamma_min; /* AdaIR exponent at the last iteration, > 0                  */
} aco_params;

/* Largest supported city count (the update keeps one FP64 row in LDS). */
#define ACO_MAX_CITIES 16384

/* Leading dimension (in elements) of every n-column matrix the library keeps:
 * n rounded up to a multiple of 64.  Pure function. */
int32_t aco_leading_dim(int32_t n);

/* Bytes of device workspace needed for n cities and up to m_max ants per
 * iteration, 256-byte aligned.  Pure function; 0 for invalid sizes. */
size_t aco_workspace_bytes(int32_t n, int32_t m_max);

/* Create a context for one TSP instance.
 *   dist_dev   device pointer, n x n FP32 row-major (dense, leading dim n): the
 *              distance matrix.  Must be symmetric (bitwise), zero on the
 *              diagonal, finite and > 0 elsewhere.  Copied; the caller may free
 *              it after the call returns.
 *   n          3 <= n <= ACO_MAX_CITIES
 *   alpha,beta >= 0, exponents of tau and eta in Eq. (1)
 *   rho        evaporation rate in (0, 1]
 *   Q          deposit numerator (Q / tour length), > 0
 *   m_max      largest number of ants any later aco_construct may use, >= 1
 *   workspace_dev, workspace_bytes   caller-owned device memory, at least
 *              aco_workspace_bytes(n, m_max) bytes, 256-byte aligned; must stay
 *              valid until aco_destroy.
 *   hip_stream the hipStream_t every later call enqueues on (NULL: the null stream)
 *   out        receives the context
 * Initialises tau to tau0 and eta to 1/d (the plain heuristic of Eq. (1)).
 * Blocks: validates dist and computes the deposit quantisation exponent.
 * Errors: ACO_EINVAL for bad sizes, parameters or dist; ACO_ENOMEM for a small
 * workspace; ACO_EDEVICE for HIP errors.  On error *out is NULL. */
aco_status aco_create(const float* dist_dev, int32_t n, float alpha, float beta, float rho,
                      float Q, int32_t m_max, void* workspace_dev, size_t workspace_bytes,
                      void* hip_stream, aco_ctx** out);

/* Re-bind the stream later calls enqueue on. */
aco_status aco_set_stream(aco_ctx* ctx, void* hip_stream);

/* Set tau0, elite_k and the gamma schedule; resets tau to tau0, clears the
 * best-so-far and invalidates P (call aco_transition next).
 * Errors: ACO_EINVAL for tau0 <= 0, elite_k < 0 or > m_max, gamma <= 0. */
aco_status aco_set_params(aco_ctx* ctx, const aco_params* params);

/* MAX-MIN pheromone bounds (the MAX-MIN Ant System of Stuetzle and Hoos; not
 * in the paper): from the next aco_update on, every off-diagonal tau is clamped
 * into [tau_min, tau_max] right after evaporation and deposit (on the rounded
 * FP32 value), and P is built from the clamped tau.  tau0 is not clamped.
 * Defaults 0 and +INFINITY: no bounds.  Single-instance contexts only.
 * Errors: ACO_EINVAL unless 0 <= tau_min <= tau_max, tau_min finite, tau_max > 0
 * (tau_max may be +INFINITY). */
aco_status aco_set_tau_bounds(aco_ctx* ctx, float tau_min, float tau_max);

/* Replace the heuristic eta of Eq. (1) (default 1/d) by a caller matrix.
 *   eta_dev  device pointer, n x n FP32 dense (leading dim n), or NULL to
 *            return to 1/d.
 * Blocks to validate: if any off-diagonal entry is not finite or not > 0 the
 * context falls back to 1/d (aco_eta_active() then reports 0) and the call
 * still returns ACO_OK.  Invalidates P. */
aco_status aco_set_eta(aco_ctx* ctx, const float* eta_dev);

/* 1 if a caller eta is in use, 0 if eta = 1/d. */
int32_t aco_eta_active(const aco_ctx* ctx);

/* Preprocessing, Sec. 2.1 Eq. (1), with the AdaIR exponent of Eq. (4) folded
 * in: P_ij = (W_ij / sum_k W_ik)^(1/gamma), W_ij = tau_ij^alpha * eta_ij^beta,
 * P_ii = 0; computed in FP64, stored FP32.  tau is not changed.
 * Errors: ACO_EINVAL for gamma <= 0 or not finite. */
aco_status aco_transition(aco_ctx* ctx, float gamma);

/* Ant-system tensorization and AdaIR selection, Sec. 2.2 and Sec. 2.4: m ants
 * (1 <= m <= m_max), each on its own wavefront, start at their random city and
 * take n-1 steps; at each step the next city is the argmax over unvisited j of
 * fl32(P[c,j] * r_j), ties to the smallest j.  Also computes each ant's closed
 * tour length (FP64 sum in tour order, rounded to FP32) and the successor and
 * predecessor maps the index-mapped deposit reads.
 * Outputs (device views below): tours m x n int32, lengths m FP32.
 * Errors: ACO_EINVAL for m out of range; ACO_ESTATE if no P is current. */
aco_status aco_construct(aco_ctx* ctx, int32_t m, uint64_t seed, uint32_t iter);

/* Ant-path tensorization and pheromone update, Sec. 2.3 Eq. (2), Eq. (3),
 * applied to the tours of the last aco_construct:
 *   1. elite set: the elite_k shortest tours (length, then ant index), or all;
 *   2. index-mapped deposit: every elite ant adds Q/L (quantised to an integer
 *      multiple of 2^-S, aco_deposit_scale) on both orientations of each of its
 *      tour edges, summed exactly in 64-bit integers (order-free);
 *   3. evaporation: tau_ij <- fl32(fma(1-rho, tau_ij, dTau_ij)) in FP64;
 *   4. P from the new tau with gamma_next (as aco_transition);
 * and keeps the best-so-far tour (shortest; ties keep the earlier iteration,
 * then the smaller ant).
 * Errors: ACO_EINVAL for bad gamma_next; ACO_ESTATE without a construct since
 * the last update. */
aco_status aco_update(aco_ctx* ctx, float gamma_next);

/* A whole run of `iters` iterations with m ants: P with gamma_0, then per
 * iteration t construct (iteration counter = the context's running counter)
 * and update with gamma_{t+1}, gamma following the cosine annealing schedule
 * of Sec. 2.4 from gamma_max to gamma_min (aco_gamma_schedule).  Clears the
 * best-so-far first; tau continues from its current state.  Blocks at the end
 * and copies the best tour (n int32) and its length to host memory (either
 * pointer may be NULL). */
aco_status aco_run(aco_ctx* ctx, int32_t m, uint64_t seed, int32_t iters,
                   int32_t* best_tour_host, float* best_len_host);

/* Cosine annealing of gamma over T iterations (Sec. 2.4):
 * gamma_t = gmin + (gmax - gmin) * (1 + cos(pi * t / (T-1))) / 2, computed in
 * FP64 and rounded to FP32; t is clamped to T-1; T <= 1 gives gmax. */
float aco_gamma_schedule(int32_t t, int32_t T, float gamma_max, float gamma_min);

/* Borrowed device views into the workspace, valid until the next call that
 * writes them or aco_destroy.  tau and P are n x ld; tours m_max x n (rows of
 * the last construct); lengths m_max. */
const float* aco_pheromone(const aco_ctx* ctx);
const float* aco_transition_matrix(const aco_ctx* ctx);
const int32_t* aco_tours(const aco_ctx* ctx);
const float* aco_lengths(const aco_ctx* ctx);
/* The rows of P as last sorted for ACO_SELECT_ADAIR_SORTED: each row keeps its
 * first K entries (the walk never reads further), values (FP32, descending,
 * ties by ascending city) and their cities (uint16), row r at offset r * K of
 * each device array.  K = aco_sorted_prefix(ctx).  The context owns both
 * arrays (valid until aco_destroy); NULL for a NULL context. */
const float* aco_sorted_rows(const aco_ctx* ctx);
const uint16_t* aco_sorted_cities(const aco_ctx* ctx);
/* K, the entries each sorted row keeps at the current walk: 64 * walk rounded
 * up to a power of two, at most n; 0 at a walk of 0 (the walk then reads no
 * sorted entry and no row is sorted) and for a NULL context. */
int32_t aco_sorted_prefix(const aco_ctx* ctx);

/* What the ACO_SELECT_ADAIR_SORTED constructs since the previous call (or
 * since aco_create) read, then resets the counts (blocks): out3[0] the sorted
 * entries read (whole batches of the group width), summed over ants and steps;
 * out3[1] the steps the walk left to the scan; out3[2] the 4-city blocks those
 * scans read.
 * Errors: ACO_EINVAL for a NULL pointer. */
aco_status aco_sorted_walk_stats(aco_ctx* ctx, uint64_t* out3);

/* Exponent S of the deposit quantisation: the largest S with
 * m_max * Q / L_lb * 2^S < 2^62, L_lb = sum over cities of the nearest
 * neighbour distance (FP64, ascending city order).  -1 for NULL. */
int32_t aco_deposit_scale(const aco_ctx* ctx);

/* Best-so-far tour, its length and its iteration (blocks).  Any pointer may be
 * NULL.  Length is +inf and iteration -1 before any update. */
aco_status aco_best(aco_ctx* ctx, int32_t* tour_host, float* len_host, int32_t* iter_host);

/* Checkpoint and resume: copy tau (n x ld FP32, device) and the iteration
 * counter out of / into the context.  aco_set_state invalidates P.  The
 * generator is stateless, so a resumed run repeats an uninterrupted one. */
aco_status aco_get_state(const aco_ctx* ctx, float* tau_dev_out, uint32_t* iter_out);
aco_status aco_set_state(aco_ctx* ctx, const float* tau_dev, uint32_t iter);

/* Construct schedules: how many lanes of a 64-lane wavefront build one ant
 * (Sec. 2.2's function mapping over ants), and whether each ant keeps the
 * sorted list of 4-city blocks that still hold an unvisited city (a step then
 * scans only those).  Every schedule gives bit-identical results: the
 * generator is keyed by city block, not by lane.  ACO_SCHED_AUTO picks by
 * size: 16 lanes up to 64 cities, 32 up to 128, 64 up to 256, then 64 with
 * the list. */
#define ACO_SCHED_AUTO (-1)
#define ACO_SCHED_G16 0      /* 16 lanes per ant, 4 ants per wavefront */
#define ACO_SCHED_G32 1      /* 32 lanes per ant, 2 ants per wavefront */
#define ACO_SCHED_G32_LIVE 2 /* 32 lanes per ant, live-block list      */
#define ACO_SCHED_G64 3      /* one ant per wavefront                  */
#define ACO_SCHED_G64_LIVE 4 /* one ant per wavefront, live-block list */

/* Select the construct schedule of this context (ACO_SCHED_*).
 * Errors: ACO_EINVAL for an unknown code. */
aco_status aco_set_schedule(aco_ctx* ctx, int32_t schedule);

/* Per-step selection rule of aco_construct (and so of aco_run).
 *   ACO_SELECT_ADAIR     Sec. 2.4: argmax over the unvisited j of fl32(P[c,j] * r_j),
 *                        r_j the deviate of counter (j/4, s, ant, iter), word j mod 4
 *                        (the default).
 *   ACO_SELECT_ROULETTE  the Roulette Wheel that Sec. 2.4's Independent Roulette
 *                        replaces (the baseline of the ablation in Sec. 3): city j
 *                        with probability P[c,j] / sum of P[c,k] over the unvisited
 *                        k.  One deviate per step, v = word 0 of counter
 *                        (0, s, ant, iter); x = v * total; the first city in
 *                        ascending order of positive weight whose running sum
 *                        exceeds x.  Sums in FP64, associated per chunk of
 *                        4 * lanes cities, so the city can differ from a strictly
 *                        sequential sum's only when x lies within rounding of a
 *                        boundary.  No positive weight left: the smallest unvisited
 *                        city.  The paper's RW samples from M_p of Eq. (1), i.e.
 *                        P built with gamma = 1 (aco_set_params with gamma_max =
 *                        gamma_min = 1 for aco_run).  The row's chunk totals are
 *                        kept one per lane, so a forced schedule of G lanes needs
 *                        ceil(ceil(n/4)/G) <= G (16 lanes: n <= 1024; 32: n <= 4096);
 *                        ACO_SCHED_AUTO always fits.
 * Errors: ACO_EINVAL for an unknown code; aco_construct returns ACO_EINVAL when
 * the schedule does not fit the roulette wheel at this n. */
#define ACO_SELECT_ADAIR 0
#define ACO_SELECT_ROULETTE 1
#define ACO_SELECT_ADAIR_SORTED 2
aco_status aco_set_selection(aco_ctx* ctx, int32_t selection);

/* ACO_SELECT_ADAIR_SORTED: the same selection as ACO_SELECT_ADAIR, bit for bit,
 * found with less work.  Every deviate of Sec. 2.4 is below 1, so a city's
 * score fl32(P[c,j] * r_j) never exceeds P[c,j].  While this selection is set,
 * aco_transition and aco_update also sort every row of the P they build (value
 * descending, city ascending; into workspace buffers), and aco_construct sorts
 * first if P has not been sorted yet.
 * A step then reads the row's entries in that order, one per lane of the
 * ant's group (G lanes: 16, 32 or 64 by schedule) at a time, scoring the
 * unvisited ones.  It stops as soon as the smallest P of a batch is below the
 * best score found: no later city can reach that score.  If 64 * walk entries
 * (aco_set_sorted_walk) have not decided the step, it scans the row's blocks
 * (only the live ones under a *_LIVE schedule) as ACO_SELECT_ADAIR does.  Any
 * schedule runs it.  ACO_SCHED_AUTO takes no live list.  It takes the
 * narrowest group that still leaves two wavefronts of ants per SIMD:
 * 16 lanes from 8192 ants, 32 lanes from 4096 ants, else 64. */
#define ACO_SORTED_WALK_MAX 256

/* A step of ACO_SELECT_ADAIR_SORTED reads at most 64 * batches sorted entries
 * before it falls back to the scan (default 8; 0 always scans).
 * Errors: ACO_EINVAL outside [0, ACO_SORTED_WALK_MAX]. */
aco_status aco_set_sorted_walk(aco_ctx* ctx, int32_t batches);

/* ------------------------------------------------------------------------ */
/* Batched engine: many independent instances of uneven size advanced        */
/* together, one persistent construct launch and one row-update launch per  */
/* iteration (optionally replayed from a captured hipGraph).  Instance i      */
/* evolves exactly -- bit for bit -- as aco_create(dist_i, n_i, alpha, beta, */
/* rho, Q, m_max = m_i) + aco_set_params(params) + aco_run(m_i, seed_i, ...)  */
/* would alone.                                                              */
/* ------------------------------------------------------------------------ */
typedef struct aco_batch aco_batch;

/* One row of a schedule table: instances with n <= n_max (the first row that
 * matches, rows sorted by n_max) use `schedule`. */
typedef struct {
    int32_t n_max;
    int32_t schedule;
} aco_schedule_entry;

/* Batch schedule flag: OR'd into ACO_SCHED_G16, ACO_SCHED_G32 or ACO_SCHED_G64,
 * the instances of that row construct with AdaIR's sorted walk (as
 * ACO_SELECT_ADAIR_SORTED at the default walk of 8 batches) instead of the
 * full scan, and every iteration also sorts their rows of P, whole (Sec. 2.4;
 * the same tours bit for bit).  Only rows with n_max <= ACO_BATCH_SORTED_MAX_N
 * may carry it. */
#define ACO_SCHED_SORTED 16
#define ACO_BATCH_SORTED_MAX_N 1024

/* Device views of one member of a batch (borrowed; valid until destroy). */
typedef struct {
    int32_t n, ld, m, deposit_scale, schedule;
    const float* tau;        /* n x ld */
    const float* P;          /* n x ld */
    const int32_t* tours;    /* m x n (last iteration) */
    const float* lengths;    /* m */
    const int32_t* best_tour;/* n */
} aco_batch_view;

/* Bytes of device workspace for `count` instances of n_host[i] cities and
 * m_host[i] ants (host arrays).  0 for invalid sizes. */
size_t aco_batch_workspace_bytes(const int32_t* n_host, const int32_t* m_host, int32_t count);

/* Create a batch.
 *   dists_dev          one device buffer; instance i's dense n_i x n_i FP32
 *                      distance matrix starts at element dist_offsets_host[i]
 *                      (same requirements as aco_create's dist; copied)
 *   n_host, m_host     cities and ants of each instance (host, count entries)
 *   seeds_host         generator seed of each instance (host)
 *   alpha..Q, params   shared by all instances (params NULL: defaults;
 *                      elite_k >= m_i means all ants for instance i)
 *   workspace          caller-owned device memory, 256-byte aligned, at least
 *                      aco_batch_workspace_bytes(); valid until destroy
 *   hip_stream         the stream every call enqueues on; a non-null stream
 *                      is needed for graph replay
 * Blocks to validate the instances.  Errors as aco_create. */
aco_status aco_batch_create(const float* dists_dev, const int64_t* dist_offsets_host,
                            const int32_t* n_host, const int32_t* m_host,
                            const uint64_t* seeds_host, int32_t count, float alpha, float beta,
                            float rho, float Q, const aco_params* params, void* workspace_dev,
                            size_t workspace_bytes, void* hip_stream, aco_batch** out);

/* Install a schedule table (host array, copied) and the number of persistent
 * construct wavefronts (0: 4096).  Instances no row covers use ACO_SCHED_AUTO.
 * Blocks (uploads the task queue).  Errors: ACO_EINVAL for unknown codes, and
 * for ACO_SCHED_SORTED on a live-list schedule or a row with n_max above
 * ACO_BATCH_SORTED_MAX_N. */
aco_status aco_batch_set_schedules(aco_batch* b, const aco_schedule_entry* table,
                                   int32_t entries, int32_t persistent_waves);

/* Flags of aco_batch_run. */
#define ACO_BATCH_GRAPH 1          /* capture one iteration once, replay it      */
#define ACO_BATCH_TIME_CONSTRUCT 2 /* launch directly and time every construct   */

/* Run `iters` iterations on every instance, from its current pheromone state
 * and the batch's running iteration counter, with the cosine gamma schedule
 * over `iters` (as aco_run).  Clears the best-so-far records first.  Enqueues
 * and returns.  flags: ACO_BATCH_GRAPH (needs a non-null stream) captures one
 * iteration once and replays it; ACO_BATCH_TIME_CONSTRUCT launches directly
 * and records a HIP event pair around each persistent construct launch (read
 * with aco_batch_construct_time).  Errors: ACO_EINVAL for iters outside
 * [0, 65535]. */
aco_status aco_batch_run(aco_batch* b, int32_t iters, int32_t flags);

/* Total and count of the construct launches timed by the last run with
 * ACO_BATCH_TIME_CONSTRUCT (milliseconds, HIP events on the batch's stream).
 * Blocks. */
aco_status aco_batch_construct_time(aco_batch* b, double* ms_total, int32_t* launches);

/* Best-so-far length and iteration of every instance (host arrays of count
 * entries) and the best tours concatenated in instance order (sum of n_i
 * entries); any pointer may be NULL.  Blocks. */
aco_status aco_batch_best(aco_batch* b, float* lens_host, int32_t* iters_host,
                          int32_t* tours_host);

/* Device views of instance i.  Errors: ACO_EINVAL for i out of range. */
aco_status aco_batch_instance(const aco_batch* b, int32_t i, aco_batch_view* view);

/* What the sorted walks of the members with ACO_SCHED_SORTED read since the
 * previous call (or since aco_batch_create), summed over those members, then
 * resets the counts: out3 as aco_sorted_walk_stats.  Blocks.
 * Errors: ACO_EINVAL for a NULL pointer. */
aco_status aco_batch_sorted_walk_stats(aco_batch* b, uint64_t* out3);

/* Block until the batch's enqueued work is done; reports device errors. */
aco_status aco_batch_sync(aco_batch* b);

/* Free the host object (the workspace stays the caller's). NULL is a no-op. */
void aco_batch_destroy(aco_batch* b);

/* ------------------------------------------------------------------------ */
/* Learned heuristic: an edge MLP whose output replaces eta = 1/d in Eq. (1) */
/* (Sec. 2.1) through aco_set_eta.  Not part of the paper.                   */
/*   features  f1 = d_ij / dNN (dNN = mean nearest-neighbour distance),      */
/*             f2 = log2(1 + rank_i(j)), f3 = log2(1 + rank_j(i)), where      */
/*             rank_i(j) is j's 1-based position among i's neighbours by     */
/*             distance, ties to the smaller index; each FP64, rounded once  */
/*             to FP32                                                       */
/*   network   3 -> 64 -> 64 -> 1, ReLU; parameters and the first hidden     */
/*             layer in BF16, FP32 accumulation (MFMA for the 64 x 64 layer)  */
/*   heuristic eta = sigmoid(z)^kappa / f1^lambda, in FP64: the network's     */
/*             edge probability times a power of the plain 1/d (dNN is a     */
/*             constant factor, which the row normalisation of Eq. (1)       */
/*             removes)                                                      */
/*   params    ACO_MLP_PARAMS FP32 values in this order: W1[64][3], b1[64],  */
/*             W2[64][64] (row = output unit), b2[64], W3[64], b3; a "BF16   */
/*             parameter" array holds their BF16 roundings as FP32 values    */
/*   training  mean BCE-with-logits against targets y in [0, 1]; gradient    */
/*             passes the rounding points through as the identity; Adam      */
/*             (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master parameters, */
/*             re-rounded to BF16 after each step.                            */
/* All pointers are device pointers unless named _host; every call enqueues  */
/* on hip_stream.                                                            */
/* ------------------------------------------------------------------------ */
#define ACO_MLP_PARAMS 4481

/* kNN ranks of every city pair (rank_dev: n x n int32, rank_i(i) = 0), each
 * city's nearest-neighbour distance (nn_dist_dev: n FP32) and their mean
 * (mean_nn_dev: one FP64, summed in city order).  dist as aco_create's. */
aco_status aco_edge_ranks(const float* dist_dev, int32_t n, int32_t* rank_dev, float* nn_dist_dev,
                          double* mean_nn_dev, void* hip_stream);

/* eta for every edge (eta_dev: n x n dense FP32; diagonal 0) from BF16
 * parameters; kappa, lambda >= 0.  Adds the number of non-finite or zero
 * outputs to *nonfinite_dev (the caller zeroes it first; aco_set_eta falls
 * back to 1/d on them). */
aco_status aco_mlp_eta(const float* bf16_params_dev, const float* dist_dev,
                       const int32_t* rank_dev, const double* mean_nn_dev, int32_t n,
                       float kappa, float lambda, float* eta_dev, uint32_t* nonfinite_dev,
                       void* hip_stream);

/* Features of the n (n - 1) off-diagonal edges, row by row with the diagonal
 * skipped (feats_dev: n (n - 1) x 3 FP32). */
aco_status aco_mlp_features(const float* dist_dev, const int32_t* rank_dev,
                            const double* mean_nn_dev, int32_t n, float* feats_dev,
                            void* hip_stream);

/* Training targets y_ij = tau_ij / max_{k != i} tau_ik in the same edge order
 * (tau_dev: n x ld FP32, e.g. aco_pheromone; y_dev: n (n - 1) FP32). */
aco_status aco_mlp_targets(const float* tau_dev, int32_t n, int32_t ld, float* y_dev,
                           void* hip_stream);

/* BF16 rounding (nearest, ties to even) of ACO_MLP_PARAMS values. */
aco_status aco_mlp_round(const float* params_dev, float* bf16_params_dev, void* hip_stream);

typedef struct aco_mlp_trainer aco_mlp_trainer;

/* Device workspace for a trainer with minibatches of `batch` edges (0 if
 * batch < 1). */
size_t aco_mlp_trainer_workspace_bytes(int32_t batch);

/* Create a trainer from ACO_MLP_PARAMS FP32 initial parameters (copied).
 * The caller's workspace (256-byte aligned) must stay valid until destroy. */
aco_status aco_mlp_trainer_create(const float* init_params_dev, int32_t batch,
                                  void* workspace_dev, size_t workspace_bytes, void* hip_stream,
                                  aco_mlp_trainer** out);

/* Gradient of the mean loss over `count` given edges (1 <= count <= batch;
 * feats count x 3, y count) at the current BF16 parameters, into grad_dev
 * (ACO_MLP_PARAMS FP32; may be NULL).  Updates nothing. */
aco_status aco_mlp_trainer_gradient(aco_mlp_trainer* t, const float* feats_dev,
                                    const float* y_dev, int32_t count, float* grad_dev);

/* One Adam step with the last gradient (learning rate lr > 0).
 * Errors: ACO_ESTATE before any gradient. */
aco_status aco_mlp_trainer_apply(aco_mlp_trainer* t, float lr);

/* One training step: a minibatch of `batch` edges drawn with replacement from
 * the `count` edges of (feats_dev, y_dev) by the counter-based generator
 * (key = seed, counter = (b / 4, step, 0xFFFFFFFE, 0)), its gradient, and one
 * Adam step. */
aco_status aco_mlp_trainer_step(aco_mlp_trainer* t, const float* feats_dev, const float* y_dev,
                                int64_t count, uint64_t seed, float lr);

/* Copy the FP32 master and/or the BF16 parameters out (either may be NULL). */
aco_status aco_mlp_trainer_params(const aco_mlp_trainer* t, float* master_dev,
                                  float* bf16_params_dev);

/* Mean loss of the last gradient (blocks). */
aco_status aco_mlp_trainer_loss(aco_mlp_trainer* t, double* loss_host);

/* Free the host object.  NULL is a no-op. */
void aco_mlp_trainer_destroy(aco_mlp_trainer* t);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid it): the
 * gradient of aco_mlp_trainer_gradient, computed by the same kernels, at the
 * given BF16 parameters, with no trainer, no workspace and no allocation.
 * Its scratch (per-edge activations and per-chunk partial gradients, about
 * 12.7 MB for the maximum) is a fixed array in device memory that each GPU
 * holds from the first call on it until the process ends.
 *   bf16_params_dev  ACO_MLP_PARAMS FP32 values that are BF16 roundings
 *   feats_dev, y_dev count x 3 features and count targets (as the trainer's)
 *   count            1 <= count <= ACO_MLP_NOALLOC_MAX_EDGES
 *   grad_dev         out: ACO_MLP_PARAMS FP32, the mean-loss gradient
 *   loss_dev         out: one FP64 mean loss, or NULL
 *   hip_stream       enqueues here; it must belong to the current device
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one
 * GPU (on different streams or threads without ordering) race and give wrong
 * results.  Calls on one stream are ordered and safe.
 * Errors: ACO_EINVAL for a NULL input or output, count out of range, or a
 * stream of another device; ACO_EDEVICE for HIP errors. */
#define ACO_MLP_NOALLOC_MAX_EDGES 16384
aco_status aco_mlp_gradient_noalloc(const float* bf16_params_dev, const float* feats_dev,
                                    const float* y_dev, int32_t count, float* grad_dev,
                                    double* loss_dev, void* hip_stream);

/* Diagnostic: write the deviates r_j, j = 0..count-1, that ant a draws at step
 * s of iteration t (see the header comment) to out_dev (device, count FP32),
 * on hip_stream.  Errors: ACO_EINVAL for count < 0. */
aco_status aco_uniforms(uint64_t seed, uint32_t iter, uint32_t ant, uint32_t step,
                        int32_t count, float* out_dev, void* hip_stream);

/* Block until all work enqueued by this context has finished; reports device
 * errors as ACO_EDEVICE. */
aco_status aco_sync(aco_ctx* ctx);

/* Free the host context (the workspace stays the caller's). NULL is a no-op. */
void aco_destroy(aco_ctx* ctx);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char* aco_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ACO_H */
