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
    uint32_t hash_slots;      /* per-walk occupancy table size (power of two), 0 = auto   */
    uint32_t walks_per_wave;  /* walks sharing one 64-lane wavefront, 0 = auto            */
    uint32_t step_cap;        /* growth steps per sequence per pperm_run_tours call after
                                 which the sequence stops with PPERM_EOVERFLOW; 0 = the
                                 watchdog default min(2^31, 4096 * tours * (n_max + 1))  */
    uint32_t flags;           /* reserved, must be 0                                      */
} pperm_config;

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
    uint64_t digest;      /* FNV-1a 64 over one byte per step: dir | a_+ << 3        */
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
} pperm_layout;

typedef struct pperm_ctx pperm_ctx;

/* Device bytes the caller must provide to pperm_create for this configuration
 * (used for admission by memory footprint).  *bytes receives the size. */
int pperm_workspace_bytes(const pperm_config* cfg, size_t* bytes);

/* Create a context.  cfg is copied.  d_workspace (>= pperm_workspace_bytes,
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

/* Close the epoch: fold every sequence's sums into the pooled sums with an
 * aligned pairwise tree over sequences (deterministic), then zero them.
 * Asynchronous. */
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
 * batch in flight.  Not thread-safe per device.  Errors: EINVAL (bad arguments,
 * a context twice, contexts on another device), EOVERFLOW, EDEVICE. */
int pperm_run_batch(pperm_ctx* const* ctxs, size_t count, const uint32_t* tours_each,
                    void* d_workspace, size_t bytes, void* hip_stream);

/* Synchronise the stream and read the merged state into caller-owned host
 * buffers of `len` >= n_max + 1 entries:
 *   log_cn[n] = log of the estimate of c_n (eqn (4); the mean of eqn (7) in
 *               PPERM_INDEPENDENT mode), -inf where no sample reached n;
 *   hist[n]   = pooled number of samples at length n (may be NULL);
 *   *tours    = pooled number of tours M (may be NULL).
 * Reflects merged epochs only.  Errors: EINVAL, ESTATE (no merged tour yet),
 * ERANGE / EOVERFLOW (raised by a kernel since the last check), EDEVICE. */
int pperm_estimates(pperm_ctx* ctx, double* log_cn, uint64_t* hist, uint64_t* tours, size_t len);

/* Synchronise and copy the per-sequence counters into `out` (N entries). */
int pperm_sequence_stats(pperm_ctx* ctx, pperm_seq_stats* out, size_t count);

/* Synchronise and sum the per-sequence counters over all sequences. */
int pperm_stats(pperm_ctx* ctx, pperm_seq_stats* total);

/* Synchronise and return the first error a kernel raised (0 if none). */
int pperm_sync(pperm_ctx* ctx);

/* Workspace layout and the launch shape the library chose. */
int pperm_layout_of(const pperm_ctx* ctx, pperm_layout* out);
int pperm_launch_shape(const pperm_ctx* ctx, uint32_t* walks_per_wave, uint32_t* hash_slots,
                       uint32_t* workgroups);

/* Destroy a context (does not free the caller's workspace). */
int pperm_destroy(pperm_ctx* ctx);

/* Static description of an error code, and the text of the last HIP error. */
const char* pperm_strerror(int code);
const char* pperm_last_device_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PPERM_H */
