/*
 * mgp.h -- C ABI of libmgp, Metropolis-family parallel resampling on AMD
 * Instinct MI355X (gfx950).
 *
 * The method is that of "The Megopolis Resampler: Memory Coalesced Resampling
 * on GPUs" (Chesser, Nguyen, Ranasinghe; arXiv 2109.13504): every particle i
 * runs B accept/reject steps against candidate ancestors and the output is
 * one ancestor index per particle (Section 3: "a list containing an ancestor
 * for each particle"). Weights need not be normalised (Section 7 removes the
 * normalisation stage for exactly this reason).
 *
 * Conventions for every entry point:
 *   - Pointers named *_dev are device pointers (HBM of the current device);
 *     everything else is host memory. The caller owns every buffer it passes;
 *     the library allocates only inside batch-plan, server and SIR-filter
 *     objects and frees that memory when the object is destroyed.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on that stream, like HIP's own: a return of
 *     MGP_OK means the work was enqueued.
 *   - Argument errors are reported synchronously with a negative MGP_E* code
 *     and a thread-local message (mgp_last_error). Nothing is enqueued then.
 *   - Data errors found on the device (a weight that is NaN, infinite or
 *     negative, or all weights zero) are reported in mgp_stats.status as
 *     MGP_EWEIGHTS; every ancestor is then written as -1.
 *   - Results are pure functions of (weights, variant, B, seed, stream_id,
 *     partition_bytes, segment): identical across calls, launch shapes and
 *     batches.
 */
#ifndef MGP_H
#define MGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define MGP_OK 0
#define MGP_EINVAL (-1)   /* bad argument (null pointer, n < 1, bad variant, eps out of range, ...) */
#define MGP_ERANGE (-2)   /* B above b_max, workspace too small, size out of range */
#define MGP_ENOMEM (-3)   /* device memory or HBM budget exhausted */
#define MGP_EHIP (-4)     /* a HIP runtime call or kernel launch failed */
#define MGP_EBUSY (-5)    /* object in use / request not finished */
#define MGP_EWEIGHTS (-6) /* device-side status: invalid weights */

/* ---- resamplers --------------------------------------------------------- */
typedef enum mgp_variant {
    MGP_METROPOLIS = 0, /* Algorithm 2: j ~ U{0, N-1} per particle and step */
    MGP_C1 = 1,         /* Algorithm 3: one partition per 32-particle group for all steps */
    MGP_C2 = 2,         /* Algorithm 4: a new partition per group at every step */
    MGP_MEGOPOLIS = 3   /* Algorithm 5: B offsets shared by every particle, wrapped segments (32 wide) */
} mgp_variant;

typedef struct mgp_params {
    int32_t variant;          /* mgp_variant */
    uint32_t B;               /* > 0: run exactly B steps; 0: derive B from epsilon */
    double epsilon;           /* bias bound in (0, 1] of eq. (proposition); used when B == 0 */
    uint64_t seed;            /* Philox4x32-10 key */
    uint32_t stream_id;       /* Philox counter word 2: 0 for a single filter, filter / request id otherwise */
    uint32_t partition_bytes; /* C1/C2 partition size P_size in bytes, multiple of 4; 0 means 128 */
    uint32_t b_max;           /* upper clamp for a derived B, and the limit for an explicit B; 0 means 65536 */
    uint32_t segment;         /* Megopolis segment width: 32 (the paper's warp; 0 means 32) or 64 (the gfx950
                                 wavefront); single-filter entry points only */
} mgp_params;

/* Written on the device by mgp_resample / mgp_compute_B (48 bytes). */
typedef struct mgp_stats {
    double w_sum;     /* sum of the weights, fp64 */
    double ratio;     /* E(w) / max(w), fp64 */
    double b_raw;     /* log(eps) / log(1 - ratio) before ceil / clamp; 0 when B was given */
    float w_max;      /* max(w), fp32 */
    uint32_t B;       /* iterations used (0 when status != MGP_OK) */
    uint32_t clamped; /* 1 if the derived B was clamped to b_max */
    int32_t status;   /* MGP_OK or MGP_EWEIGHTS */
    uint32_t n;       /* number of particles */
    uint32_t tag;     /* hash of (n, variant, seed, stream_id) of the call that wrote it */
} mgp_stats;

/* Bytes of device workspace mgp_resample / mgp_compute_B need for n
 * particles with these params (it grows with b_max, for the Megopolis
 * offsets). Host-only; touches no device. */
int mgp_workspace_size(int32_t n, const mgp_params* params, size_t* bytes);

/* RESAMPLE(x, w) -> ancestors (Algorithms 2-5; Section 3 for the problem
 * statement). Steps, all on `stream`:
 *   1. reduce the weights: fp32 max, fp64 sum, validation;
 *   2. B = params->B, or ceil(log eps / log(1 - E(w)/max w)) from eq.
 *      (proposition) (Section 4.1), clamped to [1, b_max]; Megopolis offsets
 *      o_0..o_{B-1} (Algorithm 5) are generated here;
 *   3. the accept loop: ancestors_dev[i] = k_i for i in [0, n).
 * For n <= 8192 (MGP_MEGOPOLIS) or n <= 4096 (the other variants) the three
 * steps run as one launch that keeps the weights in LDS, and for MGP_MEGOPOLIS
 * up to 32768 as two (step 2 inside the accept loop); the results, stats
 * included, are the same. These leave nothing in the workspace for a
 * following mgp_resample_prepared, which only mgp_compute_B prepares.
 * w_dev          : n fp32 weights, device, contiguous, >= 0 and finite.
 * ancestors_dev  : n int32, device, written.
 * stats_dev      : device mgp_stats written by step 2, or NULL.
 * workspace_dev  : >= mgp_workspace_size bytes of device memory, 256-byte
 *                  aligned, owned by the caller; no initialisation needed. Its
 *                  contents are scratch between calls; calls that share a
 *                  workspace must be ordered (same stream or synchronised). */
int mgp_resample(const float* w_dev, int32_t n, const mgp_params* params, int32_t* ancestors_dev,
                 mgp_stats* stats_dev, void* workspace_dev, size_t workspace_bytes, void* stream);

/* Bytes of the static scratch that mgp_resample_noalloc uses as its
 * workspace (64 MiB per device). */
#define MGP_NOALLOC_SCRATCH_BYTES (64u << 20)

/* mgp_resample without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). Same steps, kernels and results as
 * mgp_resample; the workspace is a fixed array of MGP_NOALLOC_SCRATCH_BYTES
 * in the library's device memory, one per device, held until the process
 * ends. The call allocates nothing: on its first call on a device it looks up
 * that device's copy of the array (hipGetSymbolAddress), with the stream's
 * device current.
 * Sizes: mgp_workspace_size(n, params) must fit the scratch, else MGP_ERANGE
 * and nothing is enqueued. With the default b_max that is n up to about
 * 8.3 million for MGP_MEGOPOLIS (whose workspace holds the 8n-byte mirror)
 * and any n for the other variants.
 * Every call on a device shares that device's scratch and leaves its
 * contents there: calls that overlap on one device (different streams
 * without synchronisation) race and must not be issued. The scratch needs
 * no initialisation. w_dev, ancestors_dev, stats_dev, stream: as
 * mgp_resample. */
int mgp_resample_noalloc(const float* w_dev, int32_t n, const mgp_params* params, int32_t* ancestors_dev,
                         mgp_stats* stats_dev, void* stream);

/* RESAMPLE with M != N: m ancestors drawn from n weighted inputs, as the
 * paper's closing discussion (Section 8) proposes for D-PMC-style samplers,
 * with the Megopolis offsets ranging over the input count. Output i in
 * [0, m) starts its chain at input i mod n and runs the B steps of
 * mgp_resample with its own random draws (Philox counter index i; C1/C2
 * group floor(i / 32)); candidates and offsets range over [0, n). With
 * m == n the result equals mgp_resample's.
 * w_dev: n fp32 weights; ancestors_dev: m int32, each in [0, n); workspace:
 * mgp_workspace_size(n, params) bytes; stats_dev, stream: as mgp_resample.
 * Megopolis with m <= n runs the mirrored kernel; m > n the generic one. */
int mgp_resample_m(const float* w_dev, int32_t n, int32_t m, const mgp_params* params, int32_t* ancestors_dev,
                   mgp_stats* stats_dev, void* workspace_dev, size_t workspace_bytes, void* stream);

/* Steps 1 and 2 of mgp_resample only: the reduction, B, and (for
 * MGP_MEGOPOLIS) the offsets, kept in the workspace for a following
 * mgp_resample_prepared. The paper leaves B to be pre-estimated when its
 * cost matters (Section 3); this split lets a caller time or reuse it.
 * stats_dev: device mgp_stats, written (may be NULL). */
int mgp_compute_B(const float* w_dev, int32_t n, const mgp_params* params, mgp_stats* stats_dev,
                  void* workspace_dev, size_t workspace_bytes, void* stream);

/* Step 3 of mgp_resample only: the accept loop, using the B, status and
 * offsets that the preceding mgp_compute_B on this workspace left there.
 * params and n must equal that call's; the kernel checks a tag of
 * (n, variant, seed, stream_id) written by mgp_compute_B, and on a mismatch
 * (or invalid weights) writes -1 to every ancestor. w_dev must hold the same
 * weights as in that call: with MGP_MEGOPOLIS (n <= 2^29 - 4096) the loop
 * reads the mirrored copy of them that mgp_compute_B left in the workspace,
 * not w_dev, so weights changed in between are not seen. */
int mgp_resample_prepared(const float* w_dev, int32_t n, const mgp_params* params, int32_t* ancestors_dev,
                          void* workspace_dev, size_t workspace_bytes, void* stream);

/* Particle copy x_bar_i = x_{k_i} (last statement of Algorithms 2-5):
 * out_dev[i][c] = states_dev[ancestors_dev[i]][c] for i < n_out, c < d.
 * states_dev : n_states x d fp32, row-major (array of structures), device.
 * out_dev    : n_out x d fp32, device, written; must not overlap states_dev.
 * An ancestor outside [0, n_states) (e.g. the -1 of a failed resample)
 * yields a row of NaN, never an out-of-bounds read. */
int mgp_gather(const float* states_dev, int32_t n_states, int32_t d, const int32_t* ancestors_dev,
               int32_t n_out, float* out_dev, void* stream);

/* RESAMPLE(x, w) -> x_bar in one pass: mgp_resample with the particle copy
 * x_bar_i = x_{k_i} that ends Algorithms 2-5 done by the accept loop itself,
 * while each ancestor k_i is still in a register (no second launch, no
 * re-read of the ancestor array).
 * states_dev    : n x d fp32, row-major, device (the particles x).
 * d             : floats per row, >= 1 (d % 4 == 0 with 16-byte aligned
 *                 states_dev and out_dev moves float4s).
 * out_dev       : n x d fp32, device, written (x_bar); must not overlap
 *                 states_dev.
 * ancestors_dev : n int32, device, written; NULL when only x_bar is wanted.
 * w_dev, params, stats_dev, workspace: as mgp_resample (same steps, same
 * launch counts). The result equals mgp_resample followed by mgp_gather on
 * the same arguments, bit for bit; invalid weights give -1 ancestors and NaN
 * rows. */
int mgp_resample_gather(const float* w_dev, int32_t n, const mgp_params* params, const float* states_dev, int32_t d,
                        int32_t* ancestors_dev, float* out_dev, mgp_stats* stats_dev, void* workspace_dev,
                        size_t workspace_bytes, void* stream);

/* Step 3 of mgp_resample_gather only (the accept loop with the particle
 * copy), after mgp_compute_B on this workspace: as mgp_resample_prepared,
 * with states_dev, d, ancestors_dev and out_dev as in mgp_resample_gather. */
int mgp_resample_gather_prepared(const float* w_dev, int32_t n, const mgp_params* params, const float* states_dev,
                                 int32_t d, int32_t* ancestors_dev, float* out_dev, void* workspace_dev,
                                 size_t workspace_bytes, void* stream);

/* ---- batched filters ----------------------------------------------------
 * Many independent filters of uneven size resampled by one graph launch.
 * Each filter's result is exactly that of mgp_resample (+ mgp_gather) with
 * the same weights, B / epsilon, seed and stream_id: the batch changes the
 * schedule, never the numbers. The paper's kernels resample one filter per
 * launch and note that launch overhead dominates small N (Section 6.2);
 * this mode removes it for many small filters. */
typedef struct mgp_filter_desc {
    const float* w_dev;          /* n fp32 weights (device) */
    int32_t n;                   /* particles, 1 <= n <= 2^29 - 4096 */
    uint32_t B;                  /* > 0: iterations; 0: from epsilon */
    double epsilon;              /* bias bound in (0, 1] when B == 0 */
    uint64_t seed;               /* Philox key of this filter */
    uint32_t stream_id;          /* Philox stream of this filter */
    uint32_t reserved;           /* must be 0 */
    int32_t* ancestors_dev;      /* n int32 (device), written */
    const float* states_dev;     /* n x d fp32 (device) or NULL: no gather for this filter */
    float* out_states_dev;       /* n x d fp32 (device), written when states_dev is set */
    mgp_stats* stats_dev;        /* device stats of this filter, or NULL */
} mgp_filter_desc;

typedef struct mgp_batch_config {
    int32_t variant;             /* mgp_variant, shared by every filter */
    int32_t d;                   /* state dimension of the fused gather (0: no gather) */
    uint32_t partition_bytes;    /* C1/C2; 0 means 128 */
    uint32_t b_max;              /* per-filter clamp / limit of B; 0 means 65536 */
    int32_t block_threads;       /* 64, 128 or 256; 0: autotune */
    int32_t particles_per_thread;/* Megopolis: 1, 2, 4 or 8 (8 with 64 or 128 threads); others: 1; 0: autotune */
    int32_t schedule;            /* 1: one block per tile; 2: persistent blocks on per-XCD queues; 0: autotune */
    int32_t use_graph;           /* 1: one hipGraph launch per run; 0: three plain launches */
    const char* tune_cache;      /* autotuner cache file (read and updated), or NULL */
} mgp_batch_config;

typedef struct mgp_batch_info {
    int32_t filters;
    int32_t block_threads;
    int32_t particles_per_thread;
    int32_t schedule;
    int32_t from_cache;          /* 1 if the tuning came from tune_cache */
    int32_t xcds;                /* XCDs the tile order was balanced over */
    int64_t particles;           /* sum of n */
    int64_t tiles;               /* accept-loop tiles */
    int64_t device_bytes;        /* device memory owned by the plan */
    double est_particle_steps;   /* sum of n * B from the plan-time reduction */
    int64_t grid;                /* workgroups of the accept-loop launch */
} mgp_batch_info;

typedef struct mgp_batch_plan mgp_batch_plan;

/* Builds a plan: validates the descriptors, allocates the plan's device
 * memory (per-filter stats, partials, offsets, mirrors, tile tables), runs
 * the reduction once on `stream` to estimate each filter's B (for load
 * balance only), picks the launch shape (autotuning when asked) and captures
 * the run into a hipGraph. Synchronises `stream`. Caller keeps the filters'
 * buffers alive for the plan's lifetime. */
int mgp_batch_plan_create(const mgp_filter_desc* filters, int32_t count, const mgp_batch_config* config,
                          void* stream, mgp_batch_plan** plan);

/* Replaces every filter's seed (count entries, host) for the following runs;
 * the copy is enqueued on `stream`. */
int mgp_batch_set_seeds(mgp_batch_plan* plan, const uint64_t* seeds, void* stream);

/* Runs the batch: reduction, B and offsets for every filter, then the accept
 * loops and fused gathers, as one graph launch on `stream`. */
int mgp_batch_run(mgp_batch_plan* plan, void* stream);

/* The comparison path: the same filters as one mgp_resample (+ mgp_gather)
 * launch sequence per filter, on `stream`, into the same outputs. */
int mgp_batch_run_separate(mgp_batch_plan* plan, void* stream);

int mgp_batch_plan_info(const mgp_batch_plan* plan, mgp_batch_info* info);

/* Frees the plan's device memory and graph. The plan must be idle. */
int mgp_batch_plan_destroy(mgp_batch_plan* plan);

/* ---- serving ------------------------------------------------------------
 * A resample server: requests of mixed size arrive at any time, are
 * admitted while earlier ones run, and are executed in micro-batches on
 * several HIP streams (continuous batching). Inputs (weights, states) stay
 * where the caller keeps them in device memory; the server allocates every
 * request's outputs and workspace from one device pool of hbm_budget bytes,
 * so admission is exactly "the request's footprint fits the pool now".
 * Requests are admitted in arrival order. A request's result is a pure
 * function of its own (weights, B / epsilon, seed, stream_id): identical
 * alone and in any mix. */
typedef struct mgp_server_config {
    int32_t variant;             /* mgp_variant of every request */
    int32_t d;                   /* state dimension of the fused gather (0: none) */
    uint32_t partition_bytes;    /* C1/C2; 0 means 128 */
    uint32_t b_max;              /* per-request clamp / limit of B; 0 means 65536 */
    uint64_t hbm_budget;         /* bytes of the device pool for outputs + workspaces */
    int32_t streams;             /* HIP streams running micro-batches concurrently (>= 1) */
    int32_t max_batch;           /* requests per micro-batch (>= 1) */
    int64_t max_batch_particles; /* particles per micro-batch; 0 means 2^24 */
    int32_t max_n;               /* largest request size accepted; 0 means 2^22 */
    int32_t simulate;            /* 1: no device work; completions are simulated (host tests) */
    double sim_us_fixed;         /* simulated executor: time per micro-batch, microseconds */
    double sim_ns_per_particle;  /* simulated executor: time per particle of a micro-batch */
    int32_t sim_fail_every;      /* simulated executor: fail every k-th micro-batch (0: never) */
    int32_t reserved;
} mgp_server_config;

typedef struct mgp_request {
    const float* w_dev;          /* n fp32 weights (device), kept valid until the request completes */
    int32_t n;
    uint32_t B;                  /* > 0: iterations; 0: from epsilon */
    double epsilon;
    uint64_t seed;
    uint32_t stream_id;
    uint32_t reserved;           /* must be 0 */
    const float* states_dev;     /* n x d fp32 (device), or NULL for ancestors only */
} mgp_request;

enum { MGP_REQ_QUEUED = 0, MGP_REQ_RUNNING = 1, MGP_REQ_DONE = 2, MGP_REQ_FAILED = 3, MGP_REQ_CANCELLED = 4 };

typedef struct mgp_request_result {
    int32_t state;               /* MGP_REQ_* */
    int32_t status;              /* mgp_stats.status of the request (MGP_EWEIGHTS for invalid weights) */
    uint32_t B;                  /* iterations used */
    int32_t n;
    const int32_t* ancestors_dev;/* server-owned, valid until mgp_server_release */
    const float* out_states_dev; /* server-owned (NULL without states), valid until mgp_server_release */
    double t_submit, t_admit, t_dispatch, t_done; /* seconds since the server started */
} mgp_request_result;

typedef struct mgp_server_stats {
    int64_t submitted, admitted, completed, failed, cancelled, released;
    int64_t micro_batches;
    int64_t queued;              /* waiting for admission now */
    int64_t in_flight;           /* admitted, not completed */
    uint64_t pool_bytes;         /* size of the device pool */
    uint64_t pool_in_use;        /* bytes allocated now */
    uint64_t pool_peak;          /* high-water mark of pool_in_use */
    int64_t max_concurrent_batches; /* most micro-batches on the device at once */
} mgp_server_stats;

typedef struct mgp_server mgp_server;

/* Starts the server: allocates the pool and per-stream tables, starts the
 * scheduler thread. */
int mgp_server_create(const mgp_server_config* config, mgp_server** server);

/* Queues a request (thread-safe, non-blocking). MGP_ENOMEM if its footprint
 * can never fit the pool; MGP_EINVAL / MGP_ERANGE for bad arguments. */
int mgp_server_submit(mgp_server* server, const mgp_request* request, uint64_t* ticket);

/* Current state of a request (thread-safe). */
int mgp_server_poll(mgp_server* server, uint64_t ticket, mgp_request_result* result);

/* Waits until the request is done, failed or cancelled, or timeout_ms passes
 * (MGP_EBUSY then; a negative timeout waits forever). */
int mgp_server_wait(mgp_server* server, uint64_t ticket, double timeout_ms, mgp_request_result* result);

/* Copies a finished request's outputs into caller buffers on `stream`:
 * ancestors_dev (n int32) and, if the request had states and out_states_dev
 * is not NULL, out_states_dev (n x d fp32). MGP_EBUSY if not finished. The
 * copy reads server memory: release the ticket only after `stream` has
 * finished it. */
int mgp_server_copy_outputs(mgp_server* server, uint64_t ticket, int32_t* ancestors_dev, float* out_states_dev,
                            void* stream);

/* Cancels a request that is still queued; MGP_EBUSY once it was admitted. */
int mgp_server_cancel(mgp_server* server, uint64_t ticket);

/* Returns a finished request's outputs to the pool and forgets the ticket. */
int mgp_server_release(mgp_server* server, uint64_t ticket);

int mgp_server_get_stats(mgp_server* server, mgp_server_stats* stats);

/* Stops accepting requests, cancels those still queued, lets admitted ones
 * finish, frees everything. Outputs not yet released become invalid. */
int mgp_server_destroy(mgp_server* server);

/* ---- SIR particle filter ------------------------------------------------
 * The modified SIR filter of Section 7 (Algorithm 6) on the model of eqs.
 * (predict-end2end) and (update-end2end):
 *   x_t = x_{t-1}/2 + 25 x_{t-1}/(1 + x_{t-1}^2) + 8 cos(1.2 t) + v,  v ~ N(0, 10)
 *   z_t = x_t^2/20 + n,  n ~ N(0, 1)
 * for R independent runs of n particles each, all runs advanced together:
 *   stage 1  predict and update: x_t^(i) from x_bar_{t-1}^(i) and the noise,
 *            w_t^(i) = exp(-(z_t - (x_t^(i))^2/20)^2 / 2) (the likelihood
 *            without its constant factor; no normalisation);
 *   stage 2  RESAMPLE: one batched resample of the R runs (mgp_batch_*
 *            semantics, one filter per run, stream_id = run index), with the
 *            fused gather x_bar_t^(i) = x_t^(k_i);
 *   stage 3  the estimate x_hat_t = (sum_i x_bar_t^(i)) / n, in fp64.
 * Arithmetic of stage 1 is fp64; x and w are stored as fp32. The noise of
 * particle i, run r, step t is sqrt(10) times Box-Muller in its two-output
 * form on Philox4x32-10 at counter (t, 5, r, floor(i / 4)), key = seed:
 * words (x0, x1) serve particles 4m, 4m+1 and (x2, x3) particles 4m+2, 4m+3;
 * for a pair (a, b), u1 = (a + 1) 2^-32, u2 = b 2^-32, and the even particle
 * takes sqrt(-2 ln u1) cos(2 pi u2), the odd one sqrt(-2 ln u1) sin(2 pi u2).
 * The resample of step t uses key seed + t * 2^32 and stream r. A run whose
 * weights all underflow to 0 at a step (status MGP_EWEIGHTS; its ancestors
 * are -1) keeps its predicted particles for that step: stage 3 writes
 * x_bar_t = x_t and its estimate is their mean. Results are pure functions of (x_bar_0, z, config): identical for
 * every launch shape and for graph or stage-by-stage execution, up to the
 * ~1e-16 relative rounding order of the fp64 mean. */
/* Stage 2 by a prefix-sum method (the unbiased comparison rows of Table 2):
 * values of mgp_sir_config.variant beside the mgp_variant ones. B, epsilon,
 * partition_bytes, block_threads and particles_per_thread are then unused
 * (the B history records 1). */
#define MGP_SIR_MULTINOMIAL 4 /* Algorithm 7 */
#define MGP_SIR_SYSTEMATIC 5  /* Algorithm 8 */

typedef struct mgp_sir_config {
    int32_t variant;              /* mgp_variant of stage 2, or MGP_SIR_MULTINOMIAL / MGP_SIR_SYSTEMATIC */
    int32_t runs;                 /* R, 1 <= R <= 65535 (e.g. trajectories x Monte Carlo runs) */
    int32_t n;                    /* particles per run, 1 <= n <= 2^29 - 4096, R * n <= 2^32 */
    int32_t steps;                /* T >= 1: the filter runs steps t = 1..T */
    uint32_t B;                   /* > 0: iterations of every resample; 0: from epsilon at every step */
    uint32_t partition_bytes;     /* C1/C2 partition size; 0 means 128 */
    double epsilon;               /* bias bound in (0, 1], used when B == 0 (Section 7 uses 0.1) */
    uint64_t seed;                /* Philox key of the noise; the resample of step t uses seed + t * 2^32 */
    uint32_t b_max;               /* clamp / limit of B; 0 means 65536 */
    int32_t use_graph;            /* 1: mgp_sir_run is one hipGraph launch of all T steps */
    int32_t block_threads;        /* accept-loop block size (64, 128, 256); 0: 256 */
    int32_t particles_per_thread; /* accept-loop particles per thread; 0: 4 for Megopolis, else 1 */
    int32_t reserved;             /* must be 0 */
    int32_t reserved2;            /* must be 0 */
} mgp_sir_config;

/* Device buffers of a filter, for inspection. Row r of each buffer starts at
 * element r * ld; elements [0, n) of a row are used. */
typedef struct mgp_sir_buffers {
    float* x_dev;                 /* x_t: predicted particles of the last stage 1 */
    float* w_dev;                 /* w_t: weights of the last stage 1 */
    float* xbar_dev;              /* x_bar_t: particles after the last stage 2 */
    int32_t* ancestors_dev;       /* ancestors of the last stage 2 */
    int64_t ld;                   /* row stride in elements (n rounded up to 64) */
    int64_t device_bytes;         /* device memory owned by the filter */
    int64_t accept_grid;          /* workgroups of the stage-2 accept loop */
    int32_t block_threads;
    int32_t particles_per_thread;
} mgp_sir_buffers;

typedef struct mgp_sir_filter mgp_sir_filter;

/* A filter holds one set of buffers: its calls must be ordered (issued on one
 * stream, or synchronised between streams). Calls on different filters are
 * independent. */

/* Allocates the filter's device memory (particles, weights, the per-run
 * resampler tables, the estimate history) and, with use_graph, captures the T
 * steps into one hipGraph. Measurements start as 0 (set them with
 * mgp_sir_set_measurements); there are no particles until mgp_sir_reset.
 * Synchronises `stream`. */
int mgp_sir_create(const mgp_sir_config* config, void* stream, mgp_sir_filter** filter);

/* z_host: R x (T + 1) fp64, row-major, host; z_host[r * (T + 1) + t] is the
 * measurement of run r at step t (column 0 is unused). Copied before return. */
int mgp_sir_set_measurements(mgp_sir_filter* filter, const double* z_host, void* stream);

/* Starts over at step 1 from the initial particles x_bar_0: x0_dev is R x n
 * fp32, row-major, device, copied on `stream`. Clears the history. */
int mgp_sir_reset(mgp_sir_filter* filter, const float* x0_dev, void* stream);

/* The three stages of step t (Algorithm 6), enqueued on `stream`. They must
 * be called in the order stage 1, 2, 3 of step 1, then of step 2, ...;
 * a call out of that order returns MGP_EINVAL and enqueues nothing. */
int mgp_sir_predict_update(mgp_sir_filter* filter, int32_t t, void* stream);
int mgp_sir_resample(mgp_sir_filter* filter, int32_t t, void* stream);
int mgp_sir_estimate(mgp_sir_filter* filter, int32_t t, void* stream);

/* Steps 1..T, right after mgp_sir_reset: one graph launch with use_graph,
 * else 5 T plain launches (stage 1; finalize and accept loop; two for the
 * mean). */
int mgp_sir_run(mgp_sir_filter* filter, void* stream);

/* Copies the history of the steps run so far (R x T each, row-major, host;
 * entry [r * T + t - 1] is step t of run r; any pointer may be NULL):
 * est_host the estimates x_hat_t, B_host the iterations of each resample,
 * status_host MGP_OK or MGP_EWEIGHTS. Synchronises `stream`. */
int mgp_sir_results(mgp_sir_filter* filter, double* est_host, uint32_t* B_host, int32_t* status_host, void* stream);

int mgp_sir_get_buffers(const mgp_sir_filter* filter, mgp_sir_buffers* buffers);

enum { MGP_SIR_X = 0, MGP_SIR_W = 1, MGP_SIR_XBAR = 2, MGP_SIR_ANCESTORS = 3 };

/* Copies one buffer (MGP_SIR_X, _W, _XBAR: fp32; MGP_SIR_ANCESTORS: int32) as
 * a dense R x n row-major array into dst_dev (device, caller-owned), on
 * `stream`. */
int mgp_sir_copy_buffer(const mgp_sir_filter* filter, int32_t which, void* dst_dev, void* stream);

/* Frees the filter's device memory and graph. The filter must be idle. */
int mgp_sir_destroy(mgp_sir_filter* filter);

/* Thread-local description of the last error of this thread ("" if none). */
const char* mgp_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int mgp_version(void);

/* ---- prefix-sum resamplers (the unbiased comparison methods) ------------
 * Multinomial (Algorithm 7) and systematic (Algorithm 8) resampling, the
 * methods Section 6.5 and Table 2 compare Megopolis with. Each output i gets
 * the first input j whose inclusive prefix sum of weights exceeds a threshold
 * t_i in [0, S):
 *   MGP_MULTINOMIAL: t_i = floor(r_i S / 2^64), r_i an independent 64-bit
 *                    draw per output (Philox counter (0, 6, stream_id, i));
 *   MGP_SYSTEMATIC:  t_i = floor((i + u) S / N) in fp64, one draw u in [0, 1)
 *                    per call (Philox counter (0, 7, stream_id, 0)).
 * The prefix sum runs on 64-bit fixed-point weights q_j = floor(w_j 2^K),
 * K = 62 - ceil(log2 N) - E where max w = m 2^E, m in [0.5, 1): exact in any
 * summation order, S < 2^62. Weights below 2^-(62 - ceil(log2 N)) of the
 * largest become 0 and are never chosen. */
typedef enum mgp_prefix_method {
    MGP_MULTINOMIAL = 0, /* Algorithm 7 */
    MGP_SYSTEMATIC = 1   /* Algorithm 8 */
} mgp_prefix_method;

/* Bytes of device workspace mgp_resample_prefix needs for n particles
 * (about 8n: the prefix sums). Host-only. */
int mgp_prefix_workspace_size(int32_t n, size_t* bytes);

/* Ancestors by multinomial or systematic resampling, all on `stream`: the
 * reduction and validation of mgp_resample (stats_dev as there, with B = 1),
 * the fixed-point prefix sum, then one threshold and bisection per output.
 * w_dev: n fp32 weights (device), >= 0, finite, not all zero (else stats
 * status MGP_EWEIGHTS and every ancestor -1). ancestors_dev: n int32
 * (device), written. method: mgp_prefix_method. seed, stream_id: the Philox
 * key and counter word 2. workspace_dev: mgp_prefix_workspace_size bytes,
 * 256-byte aligned, caller-owned scratch. */
int mgp_resample_prefix(const float* w_dev, int32_t n, int32_t method, uint64_t seed, uint32_t stream_id,
                        int32_t* ancestors_dev, mgp_stats* stats_dev, void* workspace_dev, size_t workspace_bytes,
                        void* stream);

/* ---- memory-system probes ------------------------------------------------
 * The streaming-read rate of the device at one buffer size: the benchmark
 * reports it as the memory ceiling beside the accept loop's achieved rate
 * (the loop streams its mirrored weights from whichever level holds them).
 * One launch of `blocks` blocks of 256 threads reads every 16-byte vector of
 * buf_dev[0, bytes) `passes` times (grid-stride, four loads in flight per
 * thread; each pass starts its sweep about 38% of the buffer further on, so
 * a block's reads are not served by the L2 its previous pass filled) and
 * writes one float per block to sink_dev (blocks floats, device), so no load
 * is elided. bytes: a positive multiple of 16, below 16 GiB (MGP_ERANGE);
 * buf_dev 16-byte aligned; contents are read, never written. Time it with
 * events on `stream`: rate = passes * bytes / time. */
int mgp_probe_stream_read(const void* buf_dev, size_t bytes, int32_t passes, int32_t blocks, float* sink_dev,
                          void* stream);

/* The Megopolis accept loop's read pattern without its arithmetic: the
 * ceiling the loop's own access pattern sets. n particles, four per thread in
 * blocks of 256 threads (n / 1024 blocks), read at each of `steps` steps the
 * candidate that Algorithm 5's segment arithmetic gives for the step's offset
 * offsets_dev[b] (steps uint32 values, device; values >= n are clamped to
 * n - 1), from mirror_dev, a mirrored array of at least 2n + 1024 floats
 * (mirror_bytes), in rounds of five steps whose loads are issued together.
 * No random draws and no accept steps. Rate = 4 n steps bytes / time.
 * sink_dev: n / 1024 floats, written only if a block's sum of what it read
 * is negative (never, for non-negative contents). n: a multiple of 1024, at
 * most 2^29 (MGP_ERANGE above); steps: a positive multiple of 5. */
int mgp_probe_pattern_read(const float* mirror_dev, size_t mirror_bytes, uint32_t n, const uint32_t* offsets_dev,
                           int32_t steps, float* sink_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MGP_H */
