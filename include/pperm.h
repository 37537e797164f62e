/*
 * pperm.h -- C ABI of the MI355X parallel flatPERM library (libpperm.so).
 *
 * The library grows many interacting flatPERM sequences of self-avoiding walks
 * on the square (d = 2) or cubic (d = 3) lattice and estimates c_n, the number
 * of n-step walks from the origin (Campbell & Janse van Rensburg, "Parallel
 * PERM": Sec. 1 for Rosenbluth growth and eqns (1)-(4), Sec. 2 for flatPERM and
 * eqn (6), Sec. 3 and Fig. 1 for Algorithms 1 and 2).
 *
 * Conventions for every call:
 *   - return 0 on success, a negative PPERM_E* code on failure; no exception
 *     ever crosses this boundary;
 *   - device pointers are HIP device memory on the device current at
 *     pperm_create; host pointers are ordinary host memory owned by the caller;
 *   - all device work is enqueued on the hipStream_t given to pperm_create and
 *     is asynchronous unless the call says it synchronises;
 *   - a context is not thread-safe; distinct contexts on distinct streams may
 *     be used concurrently.
 *
 * Determinism: the results are a function of (dim, n_max, n_sequences, seed,
 * stream, mode) and of the sequence of pperm_run_tours / pperm_merge_epoch calls
 * only.  hash_slots and walks_per_wave change speed, never a bit of a result.
 */
#ifndef PPERM_H
#define PPERM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define PPERM_OK          0
#define PPERM_EINVAL     -1   /* bad argument, bad configuration, buffer too small   */
#define PPERM_ENOMEM     -2   /* host allocation failed                               */
#define PPERM_EDEVICE    -3   /* a HIP call failed; pperm_last_device_error() has it */
#define PPERM_ESTATE     -4   /* call out of order (e.g. estimates before any merge)  */
#define PPERM_ERANGE     -5   /* a scaled weight left the normal FP64 range           */
#define PPERM_EOVERFLOW  -6   /* step cap hit, or a tour/copy counter would overflow  */
#define PPERM_EINCOMPLETE -7  /* a chained launch ended before all of its epochs ran  */

/* ---- modes ------------------------------------------------------------------ */
/* PPERM_SHARED: Algorithm 2 (Sec. 3, Fig. 1 right).  All sequences compare their
 *   weights with one pooled running average; M is the total number of passes of
 *   all sequences through the empty walk.
 * PPERM_INDEPENDENT: Algorithm 1 (Sec. 3, Fig. 1 left).  Each sequence keeps its
 *   own running averages; the estimate is their mean over sequences (eqn (7)).
 * PPERM_ROSENBLUTH: plain Rosenbluth sampling (Sec. 1): no pruning, no enrichment. */
#define PPERM_SHARED       0u
#define PPERM_INDEPENDENT  1u
#define PPERM_ROSENBLUTH   2u

/* ---- configuration ------------------------------------------------------------ */
typedef struct pperm_config {
    uint32_t struct_size;     /* sizeof(pperm_config); guards the ABI version            */
    uint32_t dim;             /* 2 or 3                                                   */
    uint32_t n_max;           /* maximum walk length, 1 .. 32766                          */
    uint32_t n_sequences;     /* N >= 1 flatPERM sequences                                */
    uint64_t seed;            /* Philox4x32-10 key                                        */
    uint32_t mode;            /* PPERM_SHARED / PPERM_INDEPENDENT / PPERM_ROSENBLUTH      */
    uint32_t stream_id;       /* xored into the key's high word; distinct problems of one
                                 batch use distinct ids                                   */
    uint32_t hash_slots;      /* per-walk occupancy table size, 0 = auto: a power of two,
                                 or (one walk per wave) 3 * 2^k; at least 2 (n_max + 1),
                                 or 1.5 (n_max + 1) where the sums stay in global memory */
    uint32_t walks_per_wave;  /* walks sharing one 64-lane wavefront, 0 = auto            */
    uint32_t step_cap;        /* growth steps per sequence per pperm_run_tours call after
                                 which the sequence stops with PPERM_EOVERFLOW; 0 = the
                                 watchdog default min(2^31, 4096 * tours * (n_max + 1))  */
    uint32_t flags;           /* PPERM_FLAG_GROUP_STATS | _OBSERVABLES | _SUMS_GLOBAL, or 0 */
} pperm_config;

/* Keep 16 group sums of the weights recorded at n_max (sequence s in group
 * s mod 16), cumulative over merged epochs, for pperm_error_estimate.  Adds one
 * small kernel to every merge; never changes any other result. */
#define PPERM_FLAG_GROUP_STATS  1u
#define PPERM_GROUPS            16u

/* Keep, beside every weight sum, the sum of W * R^2 over the same samples
 * (R^2: squared end-to-end distance of the walk), merged like the weights, for
 * the ratio estimator of eqn (5) (pperm_observable_r2).  Needs one walk per
 * wavefront and PPERM_SHARED or PPERM_ROSENBLUTH mode; such contexts run
 * through pperm_run_tours / pperm_merge_epoch (and their graphs) only.  The
 * walks themselves, and every other result, are unchanged. */
#define PPERM_FLAG_OBSERVABLES  2u

/* Launch tuning: keep each sequence's per-length sums in its global row even
 * where they would fit in LDS beside the occupancy table.  Less LDS per walk
 * lets more walks share a compute unit, at the cost of a global read per
 * step; results never change.  Needs one walk per wavefront; such contexts
 * run through pperm_run_tours / pperm_merge_epoch (and their graphs) only. */
#define PPERM_FLAG_SUMS_GLOBAL  4u

/* Per-sequence counters, cumulative over the context's life (10 x uint64 each). */
typedef struct pperm_seq_stats {
    uint64_t steps;       /* growth steps (walk-steps)                                */
    uint64_t events;      /* random blocks drawn (one per growth event)              */
    uint64_t enrich;      /* decisions with c > 1 copies                             */
    uint64_t copies;      /* sum of (c - 1) over those decisions                     */
    uint64_t prunes;      /* walks removed by pruning                                */
    uint64_t traps;       /* arrivals at a walk with a_+ = 0                         */
    uint64_t tours;       /* passes through the empty walk                           */
    uint64_t max_depth;   /* deepest pending-copy stack                              */
    uint64_t digest;      /* FNV-1a 32 over one byte per step, dir | a_+ << 3,
                             zero-extended (instrumentation: compares walks)   */
    uint64_t capped;      /* 1 once the step cap stopped this sequence               */
} pperm_seq_stats;

/* Byte offsets of the state inside the caller's workspace (for inspection).
 * Weight sums are extended-range numbers: value = m * 2^e with an FP64
 * mantissa m in [0.5, 1) (m = 0, e = 0 for zero) and an int32 exponent, so
 * that walk weights of any size are carried without underflow or overflow.
 * They are stored as 16-byte records { double m; int32_t e; uint32_t h; }
 * where h is the sample count (per-sequence sums) or 0 (pooled sums). */
typedef struct pperm_layout {
    uint64_t G;          /* records, pooled weight sums G_n: [n1p] or [N][n1p]          */
    uint64_t HG;         /* u64, pooled sample counts: same shape as G                    */
    uint64_t MG;         /* u64, pooled tour counts: [1] or [N]                           */
    uint64_t L;          /* records [N][n1p]: per-sequence sums and counts of the epoch   */
    uint64_t m;          /* u32 [N], per-sequence tours of the open epoch                 */
    uint64_t t;          /* u64 [N], per-sequence global tour counter                     */
    uint64_t stats;      /* pperm_seq_stats [N]                                           */
    uint64_t stack;      /* 32-byte pending-copy entries, private to the kernels          */
    uint64_t scratch;    /* merge partial sums, private                                   */
    uint64_t ctrl;       /* work-queue head and error flags, private                      */
    uint64_t total;      /* bytes used                                                    */
    uint32_t row;        /* n1p: records per row of G/HG/L (>= n_max + 1)                */
    uint32_t stack_slots;/* walks that can be in flight at once                           */
    uint64_t groups;     /* 16 records (group sums at n_max) then 16 u64 (group tours)  */
    uint64_t obs_L;      /* records [N][n1p]: epoch sums of W * R^2 (0: no observables)  */
    uint64_t obs_G;      /* records [n1p]: pooled sums of W * R^2 (0: no observables)     */
} pperm_layout;

typedef struct pperm_ctx pperm_ctx;

/* Device bytes the caller must provide to pperm_create for this configuration
 * (used for admission by memory footprint).  *bytes receives the size. */
int pperm_workspace_bytes(const pperm_config* cfg, size_t* bytes);

/* Create a context: one instance of the problem the paper poses -- estimate
 * c_n for n <= n_max on the d-dimensional hypercubic lattice (Sec. 1) with N
 * flatPERM sequences sharing their running averages (Algorithm 2, Sec. 3 and
 * Fig. 1), or kept apart (Algorithm 1) -- with every sum zero and no tour run.
 * cfg is copied.  d_workspace (>= pperm_workspace_bytes,
 * 256-byte aligned) is caller-owned device memory that must outlive the
 * context; the library zero-initialises its state on `hip_stream` (a
 * hipStream_t, or NULL for the default stream).  *out receives the
 * library-owned context.  Errors: EINVAL for a bad config or a short/misaligned
 * workspace, ENOMEM, EDEVICE. */
int pperm_create(const pperm_config* cfg, void* d_workspace, size_t bytes,
                 void* hip_stream, pperm_ctx** out);

/* Every sequence runs `tours_per_sequence` more tours (passes through the empty
 * walk, Sec. 1) against the pooled sums frozen at the last merge plus its own
 * sums of the open epoch (Algorithm 2, Sec. 3; the epoch-synchronous reading of
 * its sharing).  Repeated calls before a merge extend the same epoch.
 * Asynchronous.  Errors: EINVAL (0 tours), EOVERFLOW (total tours would exceed
 * 2^32 - 1), EDEVICE. */
int pperm_run_tours(pperm_ctx* ctx, uint32_t tours_per_sequence);

/* Close the epoch: the pooling of Algorithm 2 (Sec. 3, Fig. 1 right), in
 * which all sequences' weight sums and tour counts form one running average.
 * Every sequence's sums of the epoch are added into the pooled sums G_n with
 * an aligned pairwise tree over sequences (deterministic; padded with zeros
 * to a power of two), its sample counts into HG_n and its tours into M, and
 * then zeroed.  In PPERM_INDEPENDENT mode (Algorithm 1, Fig. 1 left) each
 * sequence's sums go into its own pooled sums instead.  Asynchronous.
 * Errors: EINVAL (null context), EDEVICE. */
int pperm_merge_epoch(pperm_ctx* ctx);

/* Device bytes of the scratch a batched launch of `count` problems needs. */
int pperm_batch_workspace_bytes(size_t count, size_t* bytes);

/* Batched epoch step: every context ctxs[i] runs tours_each[i] more tours (0 =
 * none), exactly as pperm_run_tours would, in persistent launches that share the
 * GPU between all of them; each context's results are bit-identical to running
 * it alone (a single problem is itself run as a batch of one).  Problems are
 * grouped by the LDS their walks need; each group runs on its own stream, forked
 * from and joined back into `hip_stream` (NULL: the default stream), which must
 * be ordered after all earlier work of the contexts (simplest: create every
 * context on `hip_stream`).  d_workspace: caller-owned device memory of at least
 * pperm_batch_workspace_bytes(count), 256-byte aligned, not in use by another
 * batch in flight.  Contexts whose per-length sums stay in global memory (long
 * walks, PPERM_FLAG_SUMS_GLOBAL) run in classes of their own.  Not thread-safe
 * per device.  Errors: EINVAL (bad arguments, a context twice, contexts on
 * another device, a context with observables), EOVERFLOW, EDEVICE. */
int pperm_run_batch(pperm_ctx* const* ctxs, size_t count, const uint32_t* tours_each,
                    void* d_workspace, size_t bytes, void* hip_stream);

/* pperm_run_batch for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same launches, the same bits, with the launch entries and queue words
 * in a fixed scratch array of the library (one per device, about 96 KiB, held
 * until the process ends) instead of a caller workspace.  At most
 * PPERM_NOALLOC_MAX_PROBLEMS contexts per call (EINVAL beyond).  The problem
 * classes run one after another on hip_stream (NULL: the default stream) with
 * no library streams.  Every call on a device shares that device's scratch, so
 * calls that overlap on one device (other streams, other threads) race; calls
 * in order on one stream do not.  Allocates no device memory.  Errors: as
 * pperm_run_batch. */
#define PPERM_NOALLOC_MAX_PROBLEMS 4096u
int pperm_run_batch_noalloc(pperm_ctx* const* ctxs, size_t count, const uint32_t* tours_each,
                            void* hip_stream);

/* One epoch -- pperm_run_tours(tours) then pperm_merge_epoch -- captured once
 * as a HIP graph and replayed: each pperm_epoch_graph_launch enqueues the
 * whole epoch on the context's stream with one launch, with exactly the
 * effect of the two calls.  Capture runs on a private stream; the context
 * must have no unmerged tours (ESTATE), at creation and at each launch.  The
 * graph belongs to its context and must be destroyed before it. */
typedef struct pperm_graph pperm_graph;
int pperm_epoch_graph_create(pperm_ctx* ctx, uint32_t tours, pperm_graph** out);
int pperm_epoch_graph_launch(pperm_graph* graph);
int pperm_epoch_graph_destroy(pperm_graph* graph);

/* Device bytes of the scratch pperm_run_job needs for these contexts and
 * epoch counts. */
int pperm_job_workspace_bytes(pperm_ctx* const* ctxs, const uint32_t* epochs, size_t count,
                              size_t* bytes);

/* Whole epoch schedules in persistent launches: context ctxs[i] runs epochs[i]
 * epochs, epoch e being schedules[i][e] tours per sequence followed by the
 * merge, exactly as the calls pperm_run_tours(schedules[i][e]) and
 * pperm_merge_epoch would (Algorithm 2, Sec. 3; same bits).  Each problem
 * moves to its next epoch as soon as its own merge is done: sequences merge
 * into the aligned pairwise tree as they finish, on the device.  A problem
 * one of whose sequences hits its step cap stops after that epoch (its context
 * then reports EOVERFLOW); the other problems run on.  After the launch every
 * context whose epochs did not all run for another reason is flagged
 * (pperm_estimates / pperm_sync then return EINCOMPLETE).  Problems run
 * in up to four LDS classes, one persistent launch each on library streams
 * forked from and joined into hip_stream (NULL: the default stream), which
 * must be ordered after all earlier work of the contexts.  d_workspace:
 * caller-owned device memory of pperm_job_workspace_bytes, 256-byte aligned.
 * Errors: EINVAL (bad arguments, a zero entry in a schedule, a context twice,
 * another device, PPERM_INDEPENDENT mode, several walks per wave, observables,
 * per-length sums in global memory), ESTATE (a context with unmerged tours),
 * EOVERFLOW, EDEVICE. */
int pperm_run_job(pperm_ctx* const* ctxs, const uint32_t* const* schedules, const uint32_t* epochs,
                  size_t count, void* d_workspace, size_t bytes, void* hip_stream);

/* Stop rule of a chained problem: stop at the first merge where
 * pperm_error_estimate is at most target_rel_err (> 0 needs
 * PPERM_FLAG_GROUP_STATS), or where the pooled tours M reach tour_cap (0:
 * no cap); target checked first. */
typedef struct pperm_job_limits {
    double target_rel_err;
    uint64_t tour_cap;
} pperm_job_limits;

/* What a chained launch (pperm_run_job or pperm_run_job_sliced) reported,
 * read from its workspace after it ran (synchronises hip_stream). */
typedef struct pperm_job_report_t {
    uint32_t problems_finished;   /* problems that ran or stopped their whole schedule  */
    uint32_t items_run;           /* (problem, epoch, sequence) items completed          */
    uint32_t problems_failed;     /* problems stopped by a sequence's step cap           */
    uint32_t waves_left_idle;     /* waves that left after 120 s without any progress    */
    uint32_t problems_incomplete; /* problems whose epochs did not all run (pperm_run_job) */
} pperm_job_report_t;
int pperm_job_report(const void* d_workspace, size_t bytes, void* hip_stream, pperm_job_report_t* out);

/* pperm_run_job with, per problem, the stop rule of limits[i] (NULL: none)
 * evaluated on the device after every merge, and a time slice: after slice_us
 * microseconds (0: none) no epoch starts, the epochs under way finish.  The
 * call synchronises and writes epochs_done[i] (epochs run and merged), stop[i]
 * (0, 1 target, 2 tour cap, 3 step cap; may be NULL) and rel_err[i] (the estimate after the
 * last merge, +inf when undefined or with no stop rule; may be NULL).  A
 * problem's result is the same however its epochs are split over calls. */
int pperm_run_job_sliced(pperm_ctx* const* ctxs, const uint32_t* const* schedules, const uint32_t* epochs,
                         size_t count, void* d_workspace, size_t bytes, void* hip_stream,
                         const pperm_job_limits* limits, uint32_t slice_us, uint32_t* epochs_done,
                         uint32_t* stop, double* rel_err);

/* Synchronise the stream and read the merged state into caller-owned host
 * buffers of `len` >= n_max + 1 entries:
 *   log_cn[n] = log of the estimate of c_n (eqn (4); the mean of eqn (7) in
 *               PPERM_INDEPENDENT mode), -inf where no sample reached n;
 *   hist[n]   = pooled number of samples at length n (may be NULL);
 *   *tours    = pooled number of tours M (may be NULL).
 * Reflects merged epochs only.  Errors: EINVAL, ESTATE (no merged tour yet),
 * ERANGE / EOVERFLOW (raised by a kernel since the last check), EDEVICE. */
int pperm_estimates(pperm_ctx* ctx, double* log_cn, uint64_t* hist, uint64_t* tours, size_t len);

/* Algorithm 1 only (PPERM_INDEPENDENT): synchronise and write each sequence's
 * own estimate -- eqn (4) for that sequence alone, its pooled weight sum over
 * its own tours -- as log_cn[s * (n_max + 1) + n] (-inf where the sequence has
 * no sample at n), the inputs of eqn (7) and of the geometric combination.
 * log_cn: caller-owned host buffer of len >= N * (n_max + 1) entries.
 * Errors: EINVAL (other modes, short buffer), ESTATE (a sequence with no
 * merged tour), ERANGE / EOVERFLOW / EINCOMPLETE, EDEVICE. */
int pperm_sequence_estimates(pperm_ctx* ctx, double* log_cn, size_t len);

/* Synchronise and estimate the relative error of the estimate of c_{n_max}
 * from the 16 sequence groups (needs PPERM_FLAG_GROUP_STATS).  Each group k has
 * the cumulative sum A_k of the weights its sequences recorded at n_max (added
 * in increasing s within an epoch, then to the running total) and its tour
 * count C_k; its estimate is g_k = A_k / C_k (eqn (4) restricted to the group).
 * *rel_err = sd(g) / (4 mean(g)), the standard error of the mean of 16 groups
 * relative to that mean (sample standard deviation, 15 degrees of freedom);
 * +inf while a group has no tour or no weight at n_max.  log_groups (16 entries,
 * may be NULL) receives log g_k.  Errors: EINVAL (flag not set), EDEVICE. */
int pperm_error_estimate(pperm_ctx* ctx, double* rel_err, double* log_groups);

/* Synchronise and read the ratio estimator of eqn (5) for O = R^2, the mean
 * squared end-to-end distance of walks of length n under the uniform
 * distribution: out[n] = (pooled sum of W * R^2) / (pooled sum of W), from the
 * merged epochs, NaN where no sample reached n (out[0] = 0).  out: caller-owned
 * host buffer of len >= n_max + 1 entries.  Errors: EINVAL (no
 * PPERM_FLAG_OBSERVABLES, short buffer), ESTATE (no merged tour yet), ERANGE /
 * EOVERFLOW (raised by a kernel since the last check), EDEVICE. */
int pperm_observable_r2(pperm_ctx* ctx, double* out, size_t len);

/* Synchronise and copy the per-sequence counters into `out` (N entries). */
int pperm_sequence_stats(pperm_ctx* ctx, pperm_seq_stats* out, size_t count);

/* Synchronise and sum the per-sequence counters over all sequences. */
int pperm_stats(pperm_ctx* ctx, pperm_seq_stats* total);

/* Synchronise and return the first error a kernel raised (0 if none). */
int pperm_sync(pperm_ctx* ctx);

/* Checkpoint and resume between epochs.  Between a merge and the next run the
 * whole future of a context is fixed by its configuration and its merged state
 * (pooled sums, counts and tours, every sequence's tour counter and counters,
 * group sums, observable sums), because the random numbers are counter-based.
 * pperm_checkpoint_bytes gives the size of that state (O(n_max + N));
 * pperm_checkpoint_save synchronises and copies it into a caller-owned host
 * buffer; pperm_checkpoint_load writes it into a context created with the same
 * problem (dim, n_max, N, seed, mode, stream_id and the result flags; the
 * launch tuning fields may differ), after which every further call gives the
 * same bits as on the saved context.  Errors: EINVAL (null pointers, short
 * buffer, not a checkpoint, another problem), ESTATE (unmerged tours on the
 * context), ERANGE / EOVERFLOW (a kernel error on the saved context), EDEVICE. */
int pperm_checkpoint_bytes(const pperm_ctx* ctx, size_t* bytes);
int pperm_checkpoint_save(pperm_ctx* ctx, void* host_buf, size_t bytes);
int pperm_checkpoint_load(pperm_ctx* ctx, const void* host_buf, size_t bytes);

/* Workspace layout and the launch shape the library chose. */
int pperm_layout_of(const pperm_ctx* ctx, pperm_layout* out);
int pperm_launch_shape(const pperm_ctx* ctx, uint32_t* walks_per_wave, uint32_t* hash_slots,
                       uint32_t* workgroups);

/* Destroy a context (does not free the caller's workspace). */
int pperm_destroy(pperm_ctx* ctx);

/* ---- serving: continuous batching of sampling jobs ---------------------------
 * A server owns a device memory pool (caller-owned, carved by a first-fit
 * allocator; an eighth of it is kept for the launches) and a FIFO of submitted
 * jobs.  Each pperm_server_step admits queued jobs in arrival order while their
 * workspace (pperm_workspace_bytes) fits in the pool and the active sequences
 * stay within max_active_sequences, then runs one time slice of chained epochs
 * (pperm_run_job_sliced) in which every active job advances at its own pace and
 * stops at the first merge where its stop rule holds; stopped jobs retire.  A job's results
 * depend only on its own description, never on what else is served with it.
 * Not thread-safe. */
typedef struct pperm_server pperm_server;

typedef struct pperm_job {
    uint32_t struct_size;      /* sizeof(pperm_job)                                       */
    uint32_t dim;              /* 2 or 3                                                  */
    uint32_t n_max;
    uint32_t n_sequences;      /* N >= 16 for the relative-error stop rule                */
    uint64_t seed;
    uint32_t mode;             /* PPERM_SHARED or PPERM_ROSENBLUTH                        */
    uint32_t stream_id;
    uint32_t tours_per_epoch;  /* T >= 1                                                  */
    uint32_t warmup;           /* 1: first epochs of 1, 1, 2, 4, ... tours (doubling while
                                  the total stays within T) and the remainder, then T      */
    double target_rel_err;     /* stop at the first merge with pperm_error_estimate <= this
                                  (0: no such stop)                                       */
    uint64_t tour_cap;         /* stop at the first merge where the pooled tours M reach
                                  this                                                    */
} pperm_job;

#define PPERM_JOB_QUEUED  0u
#define PPERM_JOB_ACTIVE  1u
#define PPERM_JOB_DONE    2u
#define PPERM_JOB_FAILED  3u

typedef struct pperm_job_info {
    uint32_t state;            /* PPERM_JOB_*                                             */
    int32_t error;             /* the error that failed the job (PPERM_JOB_FAILED)        */
    uint32_t epochs;           /* epochs run                                              */
    uint32_t stop;             /* 1 stopped by the error target, 2 by the tour cap        */
    uint64_t tours;            /* pooled tours M                                          */
    uint64_t steps;            /* walk-steps                                              */
    double rel_err;            /* the last error estimate                                 */
    uint64_t workspace_bytes;  /* its share of the pool while active                      */
} pperm_job_info;

/* Create a server on the current device.  d_pool: caller-owned device memory,
 * 256-byte aligned, pool_bytes long, outliving the server; all device work goes
 * to hip_stream.  Errors: EINVAL (pool too small for the batch scratch). */
int pperm_server_create(void* d_pool, size_t pool_bytes, uint32_t max_active_sequences,
                        void* hip_stream, pperm_server** out);

/* Queue a job; *id receives its id (1, 2, ...).  The job is validated here
 * (EINVAL for a bad description, PPERM_INDEPENDENT mode, a length whose sums no
 * longer fit in LDS beside the occupancy table, or a job that can never fit
 * the pool; EOVERFLOW when tour_cap + N * T would pass 2^32 - 1). */
int pperm_server_submit(pperm_server* srv, const pperm_job* job, uint64_t* id);

/* One scheduling step (admit, one time slice of chained epochs with the stop
 * rules evaluated on the device, retire); writes
 * the ids of the jobs retired by this step into finished[0 .. cap) and their
 * number into *n_finished (may exceed cap; the rest are still retired).
 * Synchronises.  A job whose own calls fail is retired as PPERM_JOB_FAILED;
 * the step itself fails only for device errors (EDEVICE). */
int pperm_server_step(pperm_server* srv, uint64_t* finished, size_t cap, size_t* n_finished);

/* State and counters of a job (EINVAL for an unknown or released id). */
int pperm_server_info(pperm_server* srv, uint64_t id, pperm_job_info* info);

/* The estimates of a retired job, as pperm_estimates (len >= n_max + 1; hist
 * may be NULL).  ESTATE if the job is not done. */
int pperm_server_result(pperm_server* srv, uint64_t id, double* log_cn, uint64_t* hist,
                        size_t len);

/* Forget a retired job's results. */
int pperm_server_release(pperm_server* srv, uint64_t id);

/* Length of a step's time slice in microseconds (default 100000): after it no
 * job starts another epoch in that step (results never depend on it). */
int pperm_server_set_slice(pperm_server* srv, uint32_t slice_us);

/* Jobs waiting and active, and the pool bytes in use. */
int pperm_server_counts(pperm_server* srv, uint32_t* queued, uint32_t* active, uint64_t* pool_used);

/* Destroy the server and every job it still holds (does not free the pool). */
int pperm_server_destroy(pperm_server* srv);

/* The server's pool allocator run on a script, host only (for checking it):
 * ops[i] > 0 allocates ops[i] bytes, ops[i] < 0 frees the block returned by
 * operation -ops[i] - 1.  offsets[i] receives the offset of each allocation
 * (-1 when it does not fit, 0 for a free).  Returns the bytes still in use. */
int64_t pperm_pool_script(uint64_t pool_bytes, const int64_t* ops, size_t count, int64_t* offsets);

/* Static description of an error code, and the text of the last HIP error. */
const char* pperm_strerror(int code);
const char* pperm_last_device_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PPERM_H */
