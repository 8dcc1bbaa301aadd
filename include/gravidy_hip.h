/*
 * gravidy_hip.h — C ABI of the MI355X (gfx950) Hermite-4 block-time-step
 * direct-summation N-body library with Plummer softening, after GraviDy
 * (arXiv:1702.00440).
 *
 * The library evaluates, on one GPU, the steps of the paper's integration
 * scheme (Sec. 2.4, the numbered step list): the O(N^2) initial force and
 * energy, the search for the active particles of a block step, the
 * prediction of all particles, the O(N_act * N) force (acceleration, Eq. (3),
 * and its time derivative, the jerk), and the Hermite correction with the new
 * block time step. Every step runs on the device; the host only sequences
 * launches.
 *
 * Conventions shared by every call:
 *   - Return value: gd_status, 0 (GD_OK) on success, negative on error. No call
 *     throws or aborts. gd_last_error() gives a message for the last failure.
 *   - Units: G = 1 (N-body units, Sec. 3.1).
 *   - Array arguments are DEVICE pointers (memory on the GPU the context runs
 *     on) unless marked "host". Vectors are row-major (n, 3) arrays of
 *     double: element (i, d) at index 3 * i + d. The caller owns every array;
 *     the library reads or writes it during the call (in stream order) and
 *     keeps no reference after the call's work has run.
 *   - Device memory: the library never allocates device memory. The caller
 *     provides one workspace of at least gd_workspace_bytes() bytes, aligned
 *     to 256 bytes, which the context owns until gd_destroy.
 *   - Streams: all device work is enqueued on the stream given to gd_init
 *     (a hipStream_t; NULL means the default stream). Calls that return host
 *     values synchronise that stream; the others return once work is queued.
 *   - Threads: one context is driven by one host thread at a time. Distinct
 *     contexts may be used concurrently.
 *   - Time: block time steps are dt_max / 2^k (k >= 0), clamped at dt_min;
 *     both must be powers of two. Times are kept exactly as integer multiples
 *     of dt_min; log2(dt_max / dt_min) must be at most 40.
 */
#ifndef GRAVIDY_HIP_H
#define GRAVIDY_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gd_ctx gd_ctx; /* opaque; host-side state owned by the library */

typedef enum {
  GD_OK = 0,
  GD_EINVAL = -1,     /* an argument is out of its documented range */
  GD_ENOMEM = -2,     /* the workspace is smaller than gd_workspace_bytes() */
  GD_EHIP = -3,       /* a HIP runtime call failed; see gd_last_error() */
  GD_ESTATE = -4,     /* the call is not valid in the context's current phase */
  GD_ENONFINITE = -5  /* a non-finite acceleration or jerk was produced */
} gd_status;

typedef struct {
  double eta;        /* time-step accuracy parameter (Sec. 3.2; paper default 0.01), > 0 */
  double eps;        /* Plummer softening length (Eq. (3); paper default 1e-4); 0 or >= 1e-30
                        (>= 1e-10 with GD_FLAG_MIXED) */
  double eps_bh;     /* softening of every pair that involves the central particle */
  double dt_max;     /* largest block step, a power of two (e.g. 0.125) */
  double dt_min;     /* smallest block step, a power of two <= dt_max (e.g. 2^-22) */
  int64_t bh_index;  /* central massive particle (Sec. 6, planned extension), -1 for none;
                        with one, eps and eps_bh must both be >= 1e-30 */
  int32_t flags;     /* 0 or GD_FLAG_MIXED; other bits must be 0 */
} gd_params;

/* gd_params.flags: mixed-precision pair arithmetic (the alternative to FP64
 * that Sec. 2.3 names) in every force evaluation of the context or pool
 * (initial force, block steps, gd_force). Per pair, the scalar factors
 * (differences, r.r + eps^2, r.w, the inverse square root, m q^3 and
 * 3 (r.w) q^2) are FP64. The acceleration terms of Eq. (3) are formed in FP32
 * from m q^3 and the differences rounded to FP32, and summed in FP32 over
 * each j tile (at most 256 / LJ terms per lane) before they are added into
 * FP64 accumulators. The jerk terms stay FP64: jerk sums that cancel strongly
 * defeat FP32 terms. The pair with a central particle, the predictor, the
 * corrector, the time steps, the schedule and the energy stay FP64. The
 * acceleration then differs from the FP64 path's by a relative error of
 * order 1e-7 (at most 1.7e-6 on the tested workloads), the jerk by rounding
 * (about 1e-13). */
#define GD_FLAG_MIXED 1

typedef struct {
  double t;                   /* current block time of the context */
  int64_t block_steps;        /* block steps taken since gd_init / gd_set_state */
  int64_t particle_steps;     /* sum of N_act over those steps */
  int64_t pair_interactions;  /* sum of N_act * N over those steps (self pair counted) */
  int64_t dtmin_clamps;       /* times a step was clamped at dt_min */
  double e0;                  /* energy at gd_init (kinetic + softened potential) */
  double e;                   /* energy at the last synchronised time gd_step_to reached */
  double wall_s;              /* host wall-clock seconds spent in gd_step_to since gd_init /
                                 gd_reinit / gd_set_state (pools: from gd_pool_admit to the
                                 replay that finished the cluster) */
} gd_stats;

/*
 * Bytes of device workspace a context for n particles with parameters p
 * needs (n >= 2). Host-only; no device work. p may be NULL: the size is then
 * the largest that any parameters need (it depends on n and, for large n,
 * on whether eps > 0).
 */
gd_status gd_workspace_bytes(int64_t n, const gd_params* p, size_t* bytes);

/*
 * Create a context and compute the initial state (Sec. 2.4, steps 1-3):
 * masses m[n], positions x[n][3] and velocities v[n][3] (device arrays, copied
 * in) at t = 0; the O(N^2) initial acceleration and jerk of every particle;
 * the initial block step of each particle from dt* = eta |a| / |jerk| (the
 * largest dt_max / 2^k <= dt*, clamped at dt_min); the initial energy (read
 * by gd_stats as e0). Synchronises the stream.
 * Errors: GD_EINVAL for n < 2, a NULL pointer, eta <= 0, eps outside
 * {0} U [1e-30, inf) (with GD_FLAG_MIXED: {0} U [1e-10, inf), since the
 * self pair's m / eps^3 is rounded to FP32), dt_max/dt_min not powers of two
 * or dt_min > dt_max, log2(dt_max/dt_min) > 40, flags other than 0 or
 * GD_FLAG_MIXED, a bad central-particle setting, or non-finite m/x/v or
 * m < 0 (checked on the device); GD_ENOMEM if ws_bytes is too small; GD_EHIP
 * on HIP failure. On error *ctx is NULL.
 */
gd_status gd_init(gd_ctx** ctx, const gd_params* p, int64_t n, const double* m, const double* x,
                  const double* v, void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * Restart an existing context from new masses, positions and velocities of
 * the same n (device arrays as in gd_init), at t = 0: the same steps as
 * gd_init (initial force, block steps, energy) without creating host
 * resources; captured graphs are kept. Statistics restart from zero.
 * Synchronises. Errors as gd_init (GD_EINVAL, GD_ENONFINITE, GD_EHIP).
 */
gd_status gd_reinit(gd_ctx* c, const double* m, const double* x, const double* v);

/*
 * Force-kernel timing. With enable != 0, gd_step_to runs its block steps as
 * direct launches on the context's stream instead of graph replays, and
 * every force launch issued by gd_reinit, gd_step_to and gd_force with an
 * index list records its own start and end in HIP events
 * (hipExtLaunchKernelGGL); the elapsed times of
 * the launches that did work are summed. Counters restart at zero on every
 * call. gd_profile_get reports the summed milliseconds, the number of such
 * launches, and their pair interactions (N_act * N each). Host outputs; any
 * may be NULL. Results are identical with and without timing.
 * Errors: GD_EINVAL for a NULL context; GD_EHIP (event creation).
 */
gd_status gd_profile_force(gd_ctx* c, int enable);
gd_status gd_profile_get(gd_ctx* c, double* force_ms, int64_t* launches, int64_t* pairs);

/*
 * The same force-launch timing split by block size: bucket b holds the
 * launches with n_act_min[b] <= N_act < n_act_min[b + 1] (the last bucket is
 * open), with N_act recorded on the device after each timed step. Host
 * outputs of GD_PROFILE_BUCKETS entries each (any may be NULL): the lower
 * edges (1, 2, 8, 64, 1024, 4096), the summed milliseconds, the number of
 * launches and their pair interactions. Counters restart with
 * gd_profile_force.
 * Errors: GD_EINVAL for a NULL context.
 */
#define GD_PROFILE_BUCKETS 6
gd_status gd_profile_buckets(gd_ctx* c, int64_t* n_act_min, double* force_ms, int64_t* launches,
                             int64_t* pairs);

/*
 * Prediction of all particles (Sec. 2.4, steps 5 and 7(a)).
 * t == NULL: find the next block time t_next (the earliest t_i + dt_i),
 * mark the active particles (t_i + dt_i == t_next), and predict every particle
 * to t_next with the third-order Taylor series (x, v, a, jerk at its own t_i).
 * t != NULL (host): predict every particle to the time *t, with no active set
 * (for diagnostics; gd_force then needs an explicit index list).
 * Queues work only. Errors: GD_ESTATE if nothing is left to do (never in
 * practice: some particle is always due), GD_EHIP.
 */
gd_status gd_predict(gd_ctx* c, const double* t);

/*
 * Softened acceleration (Eq. (3)) and jerk (its time derivative) of a set of
 * particles from all n particles, on the predicted state of the last
 * gd_predict (Sec. 2.4 step 7(c); Sec. 2.5). The self pair is excluded.
 * idx == NULL: the active set of the last gd_predict(NULL); n_act is ignored
 * and acc/jerk, if given, must hold n rows (the first N_act rows are written,
 * in the order of gd_active).
 * idx != NULL: n_act device int32 indices in [0, n) (repeats allowed); the
 * call synchronises to check them. n_act = 0 is an empty list: nothing is
 * computed or written (idx is not read, but must not be NULL).
 * acc, jerk: device (n_act, 3) outputs, or NULL to keep the result internal
 * (as gd_correct needs it). Queues work only when idx == NULL.
 * Errors: GD_ESTATE before any gd_predict, or idx == NULL after gd_predict(t);
 * GD_EINVAL for n_act < 0 or > n; GD_EHIP.
 */
gd_status gd_force(gd_ctx* c, const int32_t* idx, int64_t n_act, double* acc, double* jerk);

/*
 * gd_force for an index list with a chosen decomposition of the force kernel
 * (its split of the j sum; Sec. 2.5 describes the paper's): lanes_per_i lanes
 * of a wave share each listed particle (16, 32 or 64), and the n particles
 * are cut into at most `slices` j slices of whole 256-particle tiles (as many
 * as keep each slice's tile count, none empty), whose partial sums are then
 * added in slice order. Every decomposition sums the same terms in another
 * order, so results agree to rounding; gd_force picks one from n_act and n.
 * For tests of every kernel variant and for timing them (with
 * gd_profile_force). Arguments and errors as gd_force with idx != NULL, plus
 * GD_EINVAL for lanes_per_i outside {16, 32, 64}, slices outside
 * [1, ceil(n / 256)], or a decomposition whose partial sums (slices times
 * n_act) exceed the workspace's partial-force buffer. Synchronises.
 */
gd_status gd_force_plan(gd_ctx* c, const int32_t* idx, int64_t n_act, int32_t lanes_per_i, int32_t slices,
                        double* acc, double* jerk);

/*
 * Active set of the last gd_predict(NULL): writes N_act device int32 indices
 * to idx (capacity n; may be NULL) and N_act to *n_act (host). Synchronises.
 * The order of the list is unspecified; results never depend on it.
 */
gd_status gd_active(gd_ctx* c, int32_t* idx, int64_t* n_act);

/*
 * Correction of the active set (Sec. 2.4 step 7(d)): fourth-order Hermite
 * corrector from the old and new acceleration and jerk, new block step from
 * the Aarseth criterion with eta (Sec. 3.2), and the move of the active
 * particles to t_next. Queues work only.
 * Errors: GD_ESTATE unless the last calls were gd_predict(NULL) then
 * gd_force(NULL, ...); GD_EHIP.
 */
gd_status gd_correct(gd_ctx* c);

/*
 * Integrate from the current time to t_end (host value, a multiple of dt_max
 * not before the current time) by repeated block steps (predict, force,
 * correct). At every multiple of dt_max all particles are synchronised; the
 * energy is computed there (kept as stats.e). st (host, may be NULL)
 * receives the statistics. Synchronises.
 * Errors: GD_EINVAL for a bad t_end; GD_ESTATE after a gd_predict not
 * followed by gd_correct; GD_ENONFINITE; GD_EHIP.
 */
gd_status gd_step_to(gd_ctx* c, double t_end, gd_stats* st);

/*
 * Progress report for long integrations: with interval_s > 0, gd_step_to
 * writes a line to stderr (current time, t_end, block and particle steps so
 * far, seconds since the call began) whenever it reads the device schedule
 * after a batch of block steps and interval_s seconds have passed since its
 * last line. 0 (the default) turns it off. Host-only; results are unchanged.
 * Errors: GD_EINVAL for a NULL context or a negative or non-finite interval.
 */
gd_status gd_progress(gd_ctx* c, double interval_s);

/*
 * Energy of the synchronised state, Eq. (2) with G = 1: ekin = 1/2 sum m v^2;
 * epot = -sum_{i<j} m_i m_j / sqrt(|r_ij|^2 + eps^2) (softened; the quantity
 * the softened dynamics conserve); epot_unsoft (may be NULL) the same with
 * eps = 0 as printed in Eq. (2). Host outputs. Synchronises.
 * Errors: GD_ESTATE if the particles are not all at the same time (only
 * after gd_init, gd_set_state or gd_step_to they are); GD_EHIP.
 */
gd_status gd_energy(gd_ctx* c, double* ekin, double* epot, double* epot_unsoft);

/*
 * Diagnostics of the synchronised state (Sec. 4.2):
 *   - Lagrange radii: for each fraction f in fractions[0..n_frac) (host, in
 *     (0, 1], at most 32), the distance from the centre of mass of the first
 *     particle, in ascending distance (ties by index), at which the
 *     cumulative mass reaches f times the total mass; written to radii
 *     (host) in the same order;
 *   - *t_rh (host, may be NULL): half-mass relaxation time, Eq. (5) with G = 1,
 *     0.138 (N r_h^3 / m)^(1/2) / ln(0.1 N), m the mean mass, r_h the radius
 *     at f = 1/2 (also returned in *r_half, may be NULL);
 *   - level_counts (host, may be NULL): particles per block-step level,
 *     level k meaning dt = dt_max / 2^k, for k < n_levels (zero beyond
 *     log2(dt_max / dt_min)).
 * Synchronises. Errors: GD_ESTATE unless synchronised (as gd_energy),
 * GD_EINVAL for bad fractions or buffers, GD_EHIP.
 */
gd_status gd_diagnostics(gd_ctx* c, const double* fractions, int32_t n_frac, double* radii,
                         double* t_rh, double* r_half, int64_t* level_counts, int32_t n_levels);

/*
 * Copy the particle state out: x, v, a (acceleration), jerk as device
 * (n, 3) arrays at each particle's own time; t_i and dt_i as device double[n];
 * *t_now (host) the current block time. Any pointer may be NULL.
 * Synchronises.
 */
gd_status gd_get_state(gd_ctx* c, double* x, double* v, double* a, double* jerk, double* t_i,
                       double* dt_i, double* t_now);

/*
 * Replace the particle state (same layout as gd_get_state; all pointers
 * required, t_now host). Valid states: dt_i a power of two in
 * [dt_min, dt_max], t_i a multiple of dt_i, t_i <= t_now < t_i + dt_i, every
 * value finite. Masses are kept. Statistics restart from zero. Synchronises.
 * Errors: GD_EINVAL for an invalid state (checked on the device); GD_EHIP.
 */
gd_status gd_set_state(gd_ctx* c, const double* x, const double* v, const double* a,
                       const double* jerk, const double* t_i, const double* dt_i, double t_now);

/*
 * Pools: continuous batching of independent clusters.
 *
 * A pool integrates many independent clusters (each its own N, initial
 * conditions and end time) that arrive over time. Each cluster follows the
 * same method as a context (Sec. 2.4 steps 2-7). One pool step advances every
 * resident cluster by one of its own block steps, with one launch per phase
 * (predict, force, correct) for all of them together, so small clusters
 * share the GPU instead of queueing for it. A cluster's decomposition depends
 * only on its own (N_act, N): its results are bitwise the same whether it
 * runs alone (in a pool or a context) or packed with others. Pools take
 * softened clusters (eps > 0) without a central particle.
 *
 * Memory: the caller provides one device arena (256-byte aligned). It holds
 * the pool tables and, first-fit, the workspace of every admitted cluster
 * (gd_workspace_bytes(n) each) until it is released: admission is by device
 * footprint.
 */
typedef struct gd_pool gd_pool;

/* Largest max_clusters of a pool. */
#define GD_POOL_MAX_CLUSTERS 256

/* Arena bytes for max_clusters slots plus the workspaces of `count` clusters
 * of sizes n[0..count) resident at once (host-only). max_clusters <=
 * GD_POOL_MAX_CLUSTERS. */
gd_status gd_pool_arena_bytes(int32_t max_clusters, const int64_t* n, int32_t count, size_t* bytes);

/* Create an empty pool. p: parameters shared by every cluster (bh_index -1,
 * eps > 0). Errors: GD_EINVAL, GD_ENOMEM (arena too small for the tables),
 * GD_EHIP. Synchronises. */
gd_status gd_pool_create(gd_pool** pool, const gd_params* p, int32_t max_clusters, void* arena,
                         size_t arena_bytes, void* hip_stream);

/* Admit one cluster: masses m[n], positions x[n][3], velocities v[n][3]
 * (device arrays, copied in) at t = 0, to be integrated to t_end (host
 * value, a positive multiple of dt_max). Runs the cluster's initialisation
 * (initial force, steps, energy) and makes it resident; *slot receives its
 * slot. Returns GD_ENOMEM, with nothing changed, when no slot or no arena gap
 * of gd_workspace_bytes(n) is free (retry after a release). Synchronises. */
gd_status gd_pool_admit(gd_pool* pool, int64_t n, const double* m, const double* x, const double* v,
                        double t_end, int32_t* slot);

/* Advance every resident cluster by up to 32 of its own block steps (one
 * graph replay). Clusters that reached their end time (or produced a
 * non-finite force) stop being resident; their slots are written to
 * finished (host, room for the pool's max_clusters entries, may be NULL)
 * and counted in *n_finished.
 * Synchronises. */
gd_status gd_pool_run(gd_pool* pool, int32_t* finished, int32_t* n_finished);

/* Final state of a finished cluster: x, v device (n, 3) outputs (either may
 * be NULL); st (host, may be NULL) its statistics, with e0 and e the energy
 * at t = 0 and t_end. Errors: GD_ESTATE while it runs, GD_ENONFINITE if it
 * failed. Synchronises. */
gd_status gd_pool_result(gd_pool* pool, int32_t slot, double* x, double* v, gd_stats* st);

/* Free a slot and its arena block (a running cluster is dropped). */
gd_status gd_pool_release(gd_pool* pool, int32_t slot);

/* Number of resident (running) clusters (host output). */
gd_status gd_pool_resident(gd_pool* pool, int32_t* count);

/* Free the host side of the pool (not the arena). NULL is a no-op. */
void gd_pool_destroy(gd_pool* pool);

/* Message of the last failing call on pool (NULL: last gd_pool_create failure). */
const char* gd_pool_last_error(const gd_pool* pool);

/* Statistics (host output). Synchronises. */
gd_status gd_stats_get(gd_ctx* c, gd_stats* st);

/*
 * Histogram of the active-block sizes (the block time steps of Sec. 2.4): counts[b]
 * (host, GD_NACT_BINS entries) receives the number of block steps taken with
 * 2^b <= N_act < 2^(b+1) since gd_init, gd_reinit or gd_set_state. The counts
 * sum to gd_stats.block_steps. Synchronises.
 * Errors: GD_EINVAL for NULL arguments; GD_EHIP.
 */
#define GD_NACT_BINS 32
gd_status gd_nact_histogram(gd_ctx* c, int64_t* counts);

/*
 * gd_step_to replays block steps of two kernels each: the force (with the
 * active set of the step) and the corrector, which also predicts every
 * particle to the next block time it expects (the next multiple of the
 * current smallest step) and lists the particles active then. When a
 * corrected particle's new step changes the smallest one, the expectation
 * fails, and the next replayed step predicts and lists anew instead of
 * stepping (a refill; results are the same either way). *refills (host)
 * receives the number of such steps since gd_init, gd_reinit or
 * gd_set_state. Synchronises. Errors: GD_EINVAL for NULL arguments; GD_EHIP.
 */
gd_status gd_refills(gd_ctx* c, int64_t* refills);

/* Free the host-side context (not the workspace, which the caller owns). NULL is a no-op. */
void gd_destroy(gd_ctx* c);

/* Message for the last failing call on c (c may be NULL: then the last
 * failure of gd_init or gd_force_noalloc on this thread). */
const char* gd_last_error(const gd_ctx* c);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * acceleration and jerk that gd_force computes for an index list, from the
 * caller's arrays, with no context and no workspace. The call allocates
 * nothing. Its intermediate arrays (the j stream, the listed particles'
 * state, the slice partials and the schedule record) live in one scratch
 * array of the library per GPU, about 11.3 MiB, held from the library's
 * first use on that GPU until the process ends; the first call on a device
 * looks up that device's copy.
 *   p          parameters, validated as in gd_init; eps, eps_bh, bh_index and
 *              GD_FLAG_MIXED select the pair arithmetic
 *   n          particles, 2 <= n <= GD_NOALLOC_MAX_N
 *   m          device, n masses
 *   x, v       device, (n, 3) positions and velocities, all at one time
 *   idx        device, n_act int32 indices (repeats allowed); an index outside
 *              [0, n) gives NaN output rows
 *   n_act      0 <= n_act <= n; 0 queues nothing
 *   acc, jerk  device, (n_act, 3) outputs in list order; either may be NULL
 *   hip_stream the stream (on the current device) that the work is queued on;
 *              the call does not synchronise, so it may be captured
 * Results are bitwise those of gd_force(c, idx, n_act, acc, jerk) on a context
 * of the same n and parameters whose predicted state is (x, v).
 * Calls on one GPU share its scratch array and every call rewrites it: calls
 * whose work is not ordered (different streams with no dependency between
 * them) race and give wrong results. Calls on one stream are ordered.
 * Errors (message in gd_last_error(NULL)): GD_EINVAL for invalid parameters,
 * n or n_act out of range, or a NULL array when n_act > 0; GD_EHIP.
 */
#define GD_NOALLOC_MAX_N 65536
gd_status gd_force_noalloc(const gd_params* p, int64_t n, const double* m, const double* x,
                           const double* v, const int32_t* idx, int64_t n_act, double* acc,
                           double* jerk, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* GRAVIDY_HIP_H */
