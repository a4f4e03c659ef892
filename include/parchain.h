/*
 * parchain.h - C ABI of libparchain.so: round-based parallel
 * nearest-neighbour-chain hierarchical agglomerative clustering (HAC) on one
 * AMD Instinct MI355X (gfx950).
 *
 * Problem (ParChain paper, Sec. 2 opening paragraph and Alg. 1): the input is
 * a set of n points in R^d and a linkage criterion; the output is a
 * dendrogram, here the n-1 merges (child a, child b, height, size), where the
 * height of a merge is the linkage distance between the two clusters it
 * joins (Table 1).
 *
 * Method (Alg. 1-4): every round finds the nearest active cluster of every
 * chain tail ("terminal") with a range query whose radius comes from an upper
 * bound on that distance (Sec. 4, Table 1 radii), then merges every pair of
 * reciprocal nearest neighbours at once. Nearest-neighbour ties are broken by
 * the cluster ID, the lowest point index in the cluster (Sec. 1 footnote).
 *
 * All functions are safe to call from C and C++ and never throw. Functions
 * returning pc_status return PC_OK (0) or a negative error code; on error,
 * pc_last_error() describes the failure and output buffers are unspecified.
 */
#ifndef PARCHAIN_H
#define PARCHAIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PC_OK = 0,
    PC_ERR_INVALID_ARG = -1,     /* NULL pointer, n < 1, d outside [1, 2048], n > 2^31-2, bad enum */
    PC_ERR_NONFINITE_INPUT = -2, /* a coordinate is NaN or +-Inf */
    PC_ERR_OUT_OF_MEMORY = -3,   /* device workspace does not fit */
    PC_ERR_DEVICE = -4,          /* a HIP runtime call failed */
    PC_ERR_UNSUPPORTED = -5,     /* a valid request the library does not serve */
    PC_ERR_BUSY = -6,            /* context in use by another thread */
    PC_ERR_CANCELLED = -7
} pc_status;

/* Linkage criteria of Table 1. */
typedef enum {
    PC_LINK_COMPLETE = 0,  /* max over x in A, y in B of ||x-y|| */
    PC_LINK_AVERAGE = 1,   /* "avg-1": mean over x in A, y in B of ||x-y|| */
    PC_LINK_WARD = 2,      /* sqrt(2|A||B|/(|A|+|B|)) * ||mean(A)-mean(B)|| */
    PC_LINK_AVERAGE_SQ = 3 /* "avg-2": mean over x in A, y in B of ||x-y||^2
                              = ||mean(A)-mean(B)||^2 + Var(A)/|A| + Var(B)/|B|
                              with Var the sum of squared deviations from the
                              mean; heights are in squared units */
} pc_linkage;

/*
 * Precision of the screening tiles (Table 1 distances are what they bound).
 * At 4 <= d <= 128 a round first compares every chain tail with every active
 * cluster through matrix-core Gram tiles of rounded centroids, and large
 * complete / average candidate pairs are bracketed by tiles over their point
 * pairs; every candidate those tiles cannot rule out (by rigorous rounding
 * bounds) is then evaluated in FP64. So in every mode every decision and
 * every height comes from FP64 arithmetic on the float32 inputs, and the rows
 * are the same; the modes differ in the tiles' element type, hence in speed
 * and in how many candidates need the FP64 evaluation (pc_stats.refined).
 * Below d = 4 (and above 128) no tiles are used and the modes coincide.
 */
typedef enum {
    PC_PREC_FP16_REFINE = 0, /* FP16 operands, FP32 accumulate (default) */
    PC_PREC_BF16_REFINE = 1, /* BF16 operands, FP32 accumulate */
    PC_PREC_FP32 = 2,        /* FP32 operands and accumulate (the FP32
                                matrix-core instruction) */
    PC_PREC_EXACT = PC_PREC_FP16_REFINE
} pc_precision;

/* One dendrogram row, scipy linkage-matrix convention: leaves are 0..n-1,
 * row r creates cluster n+r, a < b. Rows are sorted by (height, size, lowest
 * point index of the new cluster); "height" in that key is the largest
 * height in the row's subtree (equal to the row's own height when the
 * dendrogram is monotone). 32 bytes. */
typedef struct {
    int64_t a, b;
    double height;
    int64_t size;
} pc_merge;

/* pc_options.timing bits */
#define PC_TIME_KERNELS 1
#define PC_TIME_PHASES 2

/* Options; pass NULL for defaults. struct_size must be sizeof(pc_options). */
typedef struct {
    uint32_t struct_size;
    int32_t precision; /* pc_precision, default PC_PREC_FP16_REFINE */
    int32_t prune;     /* 1 (default): range-query pruning (Sec. 4);
                          0: every terminal scans every active cluster
                          (same result, for ablations and tests) */
    int32_t timing;    /* bit 0 (PC_TIME_KERNELS): time the search and tile
                          kernels with HIP events on the call's stream (fills
                          the kernel_* stats); bit 1 (PC_TIME_PHASES): also
                          the rounds by phase (ms_nn, ms_merge, ms_update; 4
                          more events and 3 host reads per round). 0: none */
    int32_t cache_slots; /* cluster-pair distance cache (Alg. 4, Sec. 5):
                          capacity ~ cache_slots * n entries; -1 = default
                          (64 for average, 0 = off for complete, the paper's
                          settings; Ward and avg-2 values are O(1) from
                          centroids and never use it) */
    int32_t reserved;
} pc_options;

/* Counters of one pc_hac call; struct_size must be sizeof(pc_stats). */
typedef struct {
    uint32_t struct_size;
    int32_t reserved;
    int64_t rounds;           /* rounds of Alg. 1 */
    int64_t terminals;        /* sum over rounds of |Z| (terminal clusters) */
    int64_t cluster_evals;    /* cluster-pair linkage distances computed */
    int64_t point_pair_evals; /* point-pair distances computed ("D") */
    int64_t overflow_queries; /* terminals served by the full-scan kernel */
    double ms_total;          /* device time of the call (HIP events) */
    double ms_init;           /* layout + first grid */
    double ms_rounds;         /* all rounds */
    double ms_finalize;       /* sort rows + relabel */
    /* with PC_TIME_KERNELS: summed device time and launch count of the
     * search/evaluation kernels (HIP events around each launch) */
    double kernel_ms[4];      /* [0] search: ring search (bound pass), box-tree
                                 search or Gram pass 0; [1] block ring search,
                                 full scan or interval tiles; [2] exact pair
                                 tiles; [3] ring search (pair emission pass) or
                                 Gram pass 1 with exact candidate values */
    int64_t kernel_launches[4];
    int64_t candidate_visits[4]; /* candidate clusters examined, per kernel above */
    int64_t cache_hits;       /* pair distances reused from the cache */
    int64_t cache_inserts;    /* cache slots taken (claims and stores) */
    int64_t cache_fail;       /* stores dropped because the probe window was full */
    int64_t cache_derived;    /* pair values combined from cached parts
                                 (Lance-Williams rules, Table 2 / Sec. 5) */
    int64_t refined;          /* candidates the screening tiles could not rule
                                 out, then given their exact FP64 value */
    int64_t fp64_fallbacks;   /* of those, the ones beyond one per screened
                                 chain tail: FP64 work owed to the tiles'
                                 error bounds */
    /* with PC_TIME_PHASES: device time of the rounds by phase */
    double ms_nn;             /* terminals, spatial index, nearest-neighbour
                                 search and candidate evaluation */
    double ms_merge;          /* chain update, reciprocal pairs, merges */
    double ms_update;         /* active set and point-range compaction */
} pc_stats;

typedef struct pc_context pc_context;

/*
 * Create a context on HIP device `device` (the caller's current device if
 * device < 0). The context owns the device workspace, grown on demand and
 * reused across calls; it is not thread-safe (concurrent calls on one
 * context return PC_ERR_BUSY). hbm_budget_bytes > 0 caps the device bytes
 * the context may hold: a call whose workspace would exceed it runs the Gram
 * search's chain tails in smaller batches where it can, and otherwise fails
 * with PC_ERR_OUT_OF_MEMORY (the context keeps what it held). 0: no cap.
 */
pc_status pc_context_create(int device, size_t hbm_budget_bytes, pc_context **out);
void pc_context_destroy(pc_context *ctx);

/* Device bytes pc_hac needs for (n, d, linkage); 0 on bad arguments. */
size_t pc_hac_workspace_bytes(int64_t n, int32_t d, int32_t linkage, const pc_options *opt);

/*
 * Cluster n points (float32, row-major n x d) under `linkage`.
 *   points           device pointer if points_on_device != 0, else host
 *   out              n-1 rows (pc_merge); device pointer if out_on_device
 *   stream           hipStream_t to order the work on, or NULL (legacy
 *                    default stream); the call returns when the rows are
 *                    written (it synchronises the stream)
 *   stats            optional counters
 * n == 1 returns PC_OK and writes nothing. Inputs are validated before any
 * clustering work: NULL pointers, n < 1, d outside [1, 2048], n > 2^31-2 and unknown enums
 * give PC_ERR_INVALID_ARG; NaN/Inf coordinates give PC_ERR_NONFINITE_INPUT.
 * The caller keeps ownership of `points` and `out`; the library keeps no
 * reference to them after the call returns.
 */
pc_status pc_hac(pc_context *ctx, const float *points, int64_t n, int32_t d, int points_on_device,
                 int32_t linkage, const pc_options *opt, pc_merge *out, int out_on_device,
                 void *stream, pc_stats *stats);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): pc_hac on
 * device pointers that allocates nothing. Every buffer of the call is a
 * window of one static device array of PC_NOALLOC_SCRATCH_BYTES per GPU (held
 * by each GPU the library runs on until the process ends; its device address
 * is taken once per device by pc_context_create). No hipMalloc, hipFree or
 * other allocating routine is called.
 *   points, out      device pointers (n x d float32 row-major; n-1 rows)
 *   ctx, linkage, opt, stream, stats   as for pc_hac
 * Records cannot grow here: the Gram search runs its chain tails in smaller
 * batches instead, the ring search re-walks its rings, and a round that needs
 * more pair-list, tile or filter space than the scratch holds fails with
 * PC_ERR_OUT_OF_MEMORY, as does an input whose workspace does not fit (the
 * limit depends on n, d and the linkage: Ward and avg-2 at d = 2 reach about
 * 600K points, complete and average fewer). The cluster-pair cache is
 * smaller or off; the rows are pc_hac's (average linkage: heights within
 * 1e-12 relative, as with any cache size). The scratch keeps the last call's
 * contents, and the call clears what must start empty. Calls on one GPU share
 * its array: calls that overlap in time on one GPU (any context, any stream)
 * race and give wrong results.
 */
#define PC_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
pc_status pc_hac_noalloc(pc_context *ctx, const float *points, int64_t n, int32_t d, int32_t linkage,
                         const pc_options *opt, pc_merge *out, void *stream, pc_stats *stats);

/*
 * ---- Serving: many requests on one device --------------------------------
 * A server keeps up to `slots` requests on the GPU at once, each on its own
 * context and HIP stream, so the rounds of different requests overlap on the
 * device; requests that arrive while others run are admitted as slots and
 * memory free up (continuous batching of whole requests). Admission: device
 * bytes are accounted per slot, an idle slot counting what its context kept
 * from earlier requests and a busy one its request's reservation (at least
 * that). A request's reservation starts at pc_hac_workspace_bytes(n, d,
 * linkage, opt); it starts when a slot is free and the bytes it adds fit in
 * the budget. While it runs, its context may not hold more than the
 * reservation; a request that needs more (its candidate records grow with
 * the data) goes back to the head of the queue with twice the reservation
 * (counted in pc_server_stats.requeued) and fails with PC_ERR_OUT_OF_MEMORY
 * once that would exceed the whole budget. So the bytes in use never exceed
 * the budget. Waiting requests are taken in arrival order; a later request
 * that fits may start before an earlier one that does not (first fit), until
 * the earlier one has been passed over 16 times. A request whose footprint
 * exceeds the whole budget is refused at submission with
 * PC_ERR_OUT_OF_MEMORY. A request's rows are those pc_hac computes for the
 * same input, whatever else runs. All server functions are thread-safe.
 */
typedef struct pc_server pc_server;

typedef struct {
    uint32_t struct_size;       /* sizeof(pc_server_options) */
    int32_t slots;              /* requests on the device at once, 1..64; <= 0 selects 4 */
    uint64_t hbm_budget_bytes;  /* admission budget; 0 selects 80% of the device's free memory */
    double fake_us_per_kpoint;  /* test hook: > 0 runs no device work at all; a request then
                                   occupies its slot for this many microseconds per 1000
                                   points and its rows are zero (host-only tests of admission) */
    double fake_growth;         /* test hook (with fake_us_per_kpoint): a request needs its
                                   footprint times this many bytes (<= 0 selects 1) */
} pc_server_options;

typedef struct {
    uint32_t struct_size;     /* sizeof(pc_request_info), set by the caller */
    int32_t status;           /* pc_status of the request (PC_ERR_CANCELLED if cancelled) */
    int32_t state;            /* 0 waiting, 1 running, 2 done, 3 cancelled */
    int32_t slot;             /* slot that ran it, -1 before */
    uint64_t footprint_bytes; /* admission footprint */
    double t_submit_ms, t_start_ms, t_done_ms; /* server clock: ms since pc_server_create */
    pc_stats stats;           /* pc_hac's counters for the request (struct_size set) */
    char error[120];          /* pc_last_error() text of a failed request */
} pc_request_info;

typedef struct {
    uint32_t struct_size;     /* sizeof(pc_server_stats), set by the caller */
    int32_t slots;
    int64_t submitted, completed, rejected, cancelled, failed;
    int32_t running, queued, peak_running, reserved;
    uint64_t budget_bytes, bytes_in_use, peak_bytes_in_use;
    int64_t requeued;         /* requests sent back to the queue with a larger reservation */
} pc_server_stats;

/* Create a server on the device of `ctx` (the caller's current device if ctx
 * is NULL); opt may be NULL. The server does not use ctx itself, which stays
 * the caller's: each slot holds a context and a non-blocking stream of its
 * own on that device. In the no-device test mode (fake_us_per_kpoint > 0)
 * ctx is ignored. */
pc_status pc_server_create(pc_context *ctx, const pc_server_options *opt, pc_server **out);

/* Queue a request. `points` (host, float32, n x d row-major) and `out` (host,
 * n-1 rows) stay owned by the caller and must stay valid until the request
 * is done or cancelled; the server reads and writes them from its worker
 * threads. *ticket identifies the request. Bad arguments give
 * PC_ERR_INVALID_ARG; a footprint above the budget PC_ERR_OUT_OF_MEMORY;
 * non-finite coordinates are reported as the request's status. */
pc_status pc_server_submit(pc_server *srv, const float *points, int64_t n, int32_t d, int32_t linkage,
                           const pc_options *opt, pc_merge *out, uint64_t *ticket);

/* Whether a request has finished: *done = 1 once it is done or cancelled,
 * then *result is its status (PC_OK, PC_ERR_CANCELLED or the error of pc_hac)
 * and *stats (struct_size set by the caller) its counters; while it waits or
 * runs, *done = 0 and *result = PC_ERR_BUSY. Any pointer may be NULL.
 * Unknown tickets: PC_ERR_INVALID_ARG. */
pc_status pc_server_poll(pc_server *srv, uint64_t ticket, int *done, pc_status *result, pc_stats *stats);

/* The full record of a request: state, slot, reserved bytes, times, counters
 * and error text (info may be NULL). Unknown tickets: PC_ERR_INVALID_ARG. */
pc_status pc_server_query(pc_server *srv, uint64_t ticket, pc_request_info *info);

/* Wait until the request is done or cancelled; timeout_ms < 0 waits without
 * limit. PC_ERR_BUSY when the time runs out (info then shows the state). */
pc_status pc_server_wait(pc_server *srv, uint64_t ticket, double timeout_ms, pc_request_info *info);

/* Cancel a waiting request (its status becomes PC_ERR_CANCELLED). A running
 * request cannot be cancelled: PC_ERR_BUSY. Finished requests: no effect. */
pc_status pc_server_cancel(pc_server *srv, uint64_t ticket);

/* Forget a finished or cancelled request (its ticket becomes unknown). */
pc_status pc_server_release(pc_server *srv, uint64_t ticket);

pc_status pc_server_get_stats(pc_server *srv, pc_server_stats *stats);

/* Cancel every waiting request, let the running ones finish, free all. */
void pc_server_destroy(pc_server *srv);

/* Thread-local description of the last error on this thread ("" if none). */
const char *pc_last_error(void);

/* Library version string. */
const char *pc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PARCHAIN_H */
