/*
 * bp.h -- C ABI of libbp, the MI355X (gfx950) feasibility check of the
 * bin_packing constraint by lower bounds.
 *
 * Method: Tardivo, Michel, Pontelli, "Constraint Propagation on GPU: A Case
 * Study for the Bin Packing Constraint" (arXiv 2402.14821).
 *   - the constraint bin_packing(X, W, L) with k bins of capacity c: Sec. 3;
 *   - the feasibility check "fail when a lower bound exceeds k": Alg. 1;
 *   - the reduction of a partial packing to a plain instance with one virtual
 *     item per loaded bin: Sec. 3 ("Feasibility check") and Fig. 3;
 *   - the bounds L1, L2 and the dual feasible functions MT, RAD2, FS1, CCM1,
 *     VB2, BJ1 with their parameter ranges: Sec. 3.1;
 *   - the bound of a function: max over its parameters of
 *     ceil(sum f(w) / f(c)), and the early return once lb > k: Alg. 2.
 *
 * Conventions shared by every entry point:
 *   - Sizes and capacities are int32: 1 <= C <= 2^31 - 1, 0 <= w <= C,
 *     0 <= residual <= C.  Reduced instances hold at most BP_MAX_ITEMS items.
 *   - All arithmetic is exact integer arithmetic; results are deterministic.
 *   - The caller owns every buffer it passes.  Synchronous calls do not keep
 *     pointers after they return.  *_dev calls take device pointers and a
 *     hipStream_t passed as void* (NULL is HIP's null stream); their inputs
 *     must stay alive and unchanged until the work queued on that stream has
 *     completed.
 *   - The library owns contexts, queues and their device workspaces and frees
 *     them on destroy.  No exception crosses this interface.
 *   - A context may be used by one host thread at a time.  The device work of
 *     a context's calls runs in call order, whatever streams it is queued on:
 *     each launch waits for the previous launch of the same context (the
 *     context reuses one set of device workspaces), so a *_dev call followed
 *     by any other call needs no synchronisation by the caller.
 *   - On error a negative bp_status is returned and bp_last_error() gives a
 *     message for the calling thread.  Output buffers are then unspecified.
 */
#ifndef BP_H_
#define BP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bp_status;
#define BP_OK 0
#define BP_ERR_ARG (-1)    /* NULL pointer, negative count, C < 1, bad flags */
#define BP_ERR_RANGE (-2)  /* size or residual outside [0, C], bin index out of range, bin overfull, sweep outside the paper's range */
#define BP_ERR_NOMEM (-3)  /* host or device allocation failed */
#define BP_ERR_DEVICE (-4) /* a HIP call failed */
#define BP_ERR_AGAIN (-5)  /* queue full or HBM budget exhausted (non-blocking submit) */
#define BP_ERR_STATE (-6)  /* destroyed handle, unknown ticket, queue shut down */
#define BP_ERR_LIMIT (-7)  /* input larger than the library's limits */

/* Largest instance a check takes: n + m (residual form) or r (items form)
 * at most 16 384 (one workgroup sorts such an instance in its LDS), or at
 * most BP_MAX_ITEMS when c <= 2^21 and c <= 16 (n + m) (the instance is then
 * prepared from tables of c + 2 entries by kernels over the whole GPU);
 * larger ones are BP_ERR_LIMIT.  The standalone reductions take up to
 * BP_MAX_REDUCE_ITEMS. */
#define BP_MAX_ITEMS (1 << 20)
#define BP_MAX_REDUCE_ITEMS (1 << 30)
#define BP_MAX_BATCH (1 << 20) /* most instances in one batched call */

/* The bound collection, in the order used for results and tie-breaks: L1 and
 * L2 (Sec. 3.1), then the six functions in the order Alg. 2 visits them. */
enum { BP_L1 = 0, BP_L2, BP_MT, BP_RAD2, BP_FS1, BP_CCM1, BP_VB2, BP_BJ1, BP_NB };

/* Parameter ranges of the bounds.  lo[b] > hi[b] is an empty range (bound 0).
 * lo/hi of BP_L1 are ignored.  A caller-given range must lie inside the
 * paper's range of that bound (Sec. 3.1), else BP_ERR_RANGE:
 *   L2, MT [0, C/2]; RAD2 [C/4 + 1, C/3]; FS1 [1, 100]; CCM1 [1, C/2];
 *   VB2 [2, C]; BJ1 [1, C]   (all divisions floor). */
typedef struct bp_sweep {
  int64_t lo[BP_NB];
  int64_t hi[BP_NB];
  uint32_t flags;
  uint32_t reserved;
} bp_sweep;

/* flags of bp_sweep: cut the top of the VB2 range to
 * floor((2^32 - 1) / (r * max w)) as the paper does to stay inside 32-bit
 * sums (Sec. 4, "Implementation details").  Off by default: the library
 * accumulates in 64 bits and needs no cut. */
#define BP_SWEEP_PAPER_VB2_CLAMP 1u

/* flags of bp_sweep: compute the MT and BJ1 sums over most of their
 * parameters from threshold sums of the sorted sizes instead of one
 * evaluation per (item, parameter).  With U(t) = sum_w max(0, w - t) over
 * the sizes 0 < w < c and K = floor(c / lambda), the BJ1 sum of Sec. 3.1 is
 * exactly sum_{m=1..K} U(c - m lambda) - sum_{j=1..K} U(j lambda); the MT sum
 * is a sum of the sizes on either side of lambda (small sizes) or of
 * c - lambda (big sizes).  The results are the same integers as without the
 * flag; only the work per parameter changes (about 2K threshold sums
 * instead of r evaluations; parameters with large K stay dense).  bp_bounds
 * .evals still counts r * (sum of range sizes). */
#define BP_SWEEP_SEGMENTS 2u

/* Result of one check.  value[b] is the bound, argmax_lambda[b] the smallest
 * parameter attaining it (-1 for L1 and for an empty range).  lb is the
 * maximum over the collection, lb_arg the first bound attaining it, verdict
 * 1 = PASS (lb <= k, not refuted) and 0 = FAIL (lb > k, Alg. 1).  A PASS does
 * not prove that a packing exists.  r is the reduced item count, evals the
 * number of (item, parameter) evaluations of the six functions,
 * r * sum of range sizes.  status is BP_OK or the error found on the device
 * for this instance (device-side inputs are validated there). */
typedef struct bp_bounds {
  int64_t value[BP_NB];
  int64_t argmax_lambda[BP_NB];
  int64_t lb;
  int32_t lb_arg;
  int32_t verdict;
  int64_t k;
  int64_t r;
  int64_t evals;
  int32_t status;
  int32_t early_exit; /* 1 when an early-exit call stopped once lb > k (values then partial) */
  int64_t evals_done; /* (item, parameter) evaluations of the work that ran: evals, less what an
                         early exit skipped; for a served request computed from another node's
                         sums, (changed items) x (sum of range sizes) */
} bp_bounds;

/* Library version string (static storage). */
const char *bp_version(void);

/* Message of the last error on the calling thread ("" if none). */
const char *bp_last_error(void);

/* Fill *out with the paper's parameter ranges for capacity C (Sec. 3.1).
 * r and max_w are only read with BP_SWEEP_PAPER_VB2_CLAMP.  Host only. */
bp_status bp_default_sweep(int32_t C, int64_t r, int32_t max_w, uint32_t flags, bp_sweep *out);

/* A context binds one GPU, one HIP stream of default priority, device
 * workspaces that grow on demand, pinned staging buffers and the captured
 * HIP graphs of the pipeline.  device is a HIP ordinal. */
typedef struct bp_ctx bp_ctx;
bp_status bp_ctx_create(int device, bp_ctx **out);
bp_status bp_ctx_destroy(bp_ctx *ctx);

/* Launch shape of the parameter sweep, held per context.  Results do not
 * depend on it; only the speed does.
 *   lanes_params   parameters per lane in a sweep tile: 1, 2 or 4 (a tile is
 *                  64 x lanes_params consecutive parameters of one bound);
 *   waves_per_cu   resident waves of the persistent sweep kernel per compute
 *                  unit: 4 .. 32;
 *   tasks_per_wave tasks per resident wave the planner aims at; tiles dearer
 *                  than a task are split into item chunks: 1 .. 64;
 *   min_chunk      fewest items in one chunk of a split tile: 64 .. 65536.
 * A new context starts with {2, 32, 32, 2048}. */
typedef struct bp_tuning {
  int32_t lanes_params;
  int32_t waves_per_cu;
  int32_t tasks_per_wave;
  int32_t min_chunk;
} bp_tuning;
bp_status bp_ctx_get_tuning(bp_ctx *ctx, bp_tuning *out);
bp_status bp_ctx_set_tuning(bp_ctx *ctx, const bp_tuning *tuning);


/* Stage timing for diagnostics and measurement.  With enable = 1 the context
 * launches the pipeline kernels one by one instead of replaying its graph and
 * records HIP events around each on the call's stream; every check takes the
 * pipeline then, also one small enough for the one-launch path.  bp_ctx_stage_times
 * waits for every call made since timing was last switched on (set_timing
 * restarts the count) and returns the mean durations in milliseconds:
 * ms[0] reduction + sort + prefix (prep), ms[1] sweeps, ms[2] combine of
 * split tiles + finalize;
 * *runs (optional) receives the number of calls averaged.  BP_ERR_STATE if
 * timing is off or no call was timed.  Every 64th timed call waits for the
 * oldest pending one, so long timed runs stay bounded in memory. */
bp_status bp_ctx_set_timing(bp_ctx *ctx, int32_t enable);
bp_status bp_ctx_stage_times(bp_ctx *ctx, double ms[3], int64_t *runs);

/* Reduction of a partial packing (Sec. 3, Fig. 3), run on the device.
 * residual[m] are the remaining capacities of the k = m bins, unpacked[n] the
 * sizes of the items not yet packed.  out_items (capacity n + m) receives the
 * unpacked sizes in order, then the load C - residual[j] of every bin with
 * residual[j] < C in bin order; *out_r their count.  Host pointers. */
bp_status bp_residual_reduce(bp_ctx *ctx, int32_t C, int32_t m, const int32_t *residual,
                             const int32_t *unpacked, int64_t n, int32_t *out_items, int64_t *out_r);

/* The same reduction from the constraint's variables: size[n] and bin_of[n]
 * (bin index in [0, m), or -1 for an unpacked item).  out_residual[m]
 * (optional) receives C minus each bin's load.  Loads above C: BP_ERR_RANGE. */
bp_status bp_assignment_reduce(bp_ctx *ctx, int32_t C, int32_t m, const int32_t *size,
                               const int32_t *bin_of, int64_t n, int32_t *out_items, int64_t *out_r,
                               int32_t *out_residual);

/* All bounds of one reduced instance items[r] (host pointer) with k bins.
 * sweep = NULL uses the paper's ranges.  Never exits early. */
bp_status bp_lower_bounds(bp_ctx *ctx, int32_t C, int32_t k, const int32_t *items, int64_t r,
                          const bp_sweep *sweep, bp_bounds *out);

/* As bp_lower_bounds with device pointers: d_items[r] on the device, the
 * result written to d_out (device) in stream order.  Validation of the sizes
 * happens on the device and is reported in d_out->status. */
bp_status bp_lower_bounds_dev(bp_ctx *ctx, int32_t C, int32_t k, const int32_t *d_items, int64_t r,
                              const bp_sweep *sweep, bp_bounds *d_out, void *stream);

/* The feasibility check of Alg. 1 on a partial packing: reduce (residual[m],
 * unpacked[n]) on the device, compute the bounds and FAIL iff lb > m.
 * flags: BP_NO_EARLY_EXIT evaluates every bound; without it the device stops
 * scheduling work once lb > m is known (the verdict is the same; lb is then
 * some value > m).  verdict and lb may be NULL; bounds (optional) receives
 * the full record. */
#define BP_NO_EARLY_EXIT 1u
/* flags of bp_feasible, bp_feasible_dev and bp_request: the sums as with
 * BP_SWEEP_SEGMENTS (same results, less work). */
#define BP_SEGMENTS 2u
bp_status bp_feasible(bp_ctx *ctx, int32_t C, int32_t m, const int32_t *residual, const int32_t *unpacked,
                      int64_t n, uint32_t flags, int32_t *verdict, int64_t *lb, bp_bounds *bounds);

/* As bp_feasible with device pointers d_residual[m] and d_unpacked[n]; the
 * full record goes to d_out (device) in stream order.  Sizes are validated
 * on the device (d_out->status). */
bp_status bp_feasible_dev(bp_ctx *ctx, int32_t C, int32_t m, const int32_t *d_residual, const int32_t *d_unpacked,
                          int64_t n, uint32_t flags, bp_bounds *d_out, void *stream);

/* Batches in CSR form: instance i has items[off[i] .. off[i+1]), capacity
 * C[i] and k[i] bins.  off has count + 1 entries, off[0] = 0. */
typedef struct bp_batch {
  int32_t count;
  int32_t reserved;
  const int64_t *off;
  const int32_t *items;
  const int32_t *C;
  const int32_t *k;
} bp_batch;

/* All instances of a batch in one persistent launch; host pointers.
 * per_inst (optional) gives one bp_sweep per instance.  out[count]. */
bp_status bp_lower_bounds_batch(bp_ctx *ctx, const bp_batch *batch, const bp_sweep *per_inst, bp_bounds *out);

/* Batched with the items on the device: batch->off, C, k are host arrays
 * (they size the launch), d_items the device item array, d_out[count] a
 * device array.  Queued on stream; nothing is copied back. */
bp_status bp_lower_bounds_batch_dev(bp_ctx *ctx, const bp_batch *batch, const int32_t *d_items,
                                    const bp_sweep *per_inst, bp_bounds *d_out, void *stream);

/* Batched feasibility check of reduced instances with k[i] bins each;
 * flags as in bp_feasible.  verdict[count], lb[count] and bounds[count]
 * (the records, with early_exit and evals_done) may each be NULL. */
bp_status bp_feasible_batch(bp_ctx *ctx, const bp_batch *batch, uint32_t flags, int32_t *verdict, int64_t *lb,
                            bp_bounds *bounds);

/* Autotuner: times the sweep of this batch (host pointers, as
 * bp_lower_bounds_batch) under candidate shapes, one knob at a time starting
 * from the context's current shape, reps runs each (best of), and leaves the
 * fastest shape set on the context.  *best and *best_ms (sweep milliseconds)
 * may be NULL. */
bp_status bp_autotune_batch(bp_ctx *ctx, const bp_batch *batch, const bp_sweep *per_inst, int32_t reps,
                            bp_tuning *best, double *best_ms);

/* Order in which a launch schedules the six functions' tiles (L2's tiles
 * always go first): order[0..5] is a permutation of BP_MT .. BP_BJ1, tiles of
 * earlier functions first, longest first within a function.  NULL restores
 * the default, longest tile first over all functions.  Results do not
 * depend on it; with early exit (Alg. 2 returns after the first function
 * whose bound exceeds k; Alg. 4 skips work once lb > k) the work done
 * before a refutation does.  BP_ERR_ARG if order is not a permutation. */
bp_status bp_ctx_set_order(bp_ctx *ctx, const int32_t *order);

/* The autotuner with a cache on disk.  The batch's shape is summarised as a
 * key: the count of instances and of items (each rounded up to a power of
 * two), the distinct capacities (rounded up to powers of two, at most eight)
 * and the sweep flags of per_inst.  A line of cache_path (a text file, one
 * "key lanes_params waves_per_cu tasks_per_wave min_chunk sweep_ms" per
 * line) with this key sets that shape on the context without timing
 * anything (*from_cache = 1); otherwise bp_autotune_batch runs and its
 * result is appended (*from_cache = 0).  cache_path NULL: no cache.  An
 * unreadable or malformed file is treated as empty; a failed append is
 * BP_ERR_ARG after the shape is set.  *best, *best_ms, *from_cache may be
 * NULL. */
bp_status bp_autotune_batch_cached(bp_ctx *ctx, const bp_batch *batch, const bp_sweep *per_inst, int32_t reps,
                                   const char *cache_path, bp_tuning *best, double *best_ms, int32_t *from_cache);

/* Allocation-free variant of bp_feasible_dev, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The same check and record as
 * bp_feasible_dev, without a context, on the calling thread's current HIP
 * device; d_residual[m], d_unpacked[n] and d_out are device pointers owned
 * by the caller, and the work is queued on stream.  The launch tables and
 * every workspace live in one static device array of
 * BP_NOALLOC_SCRATCH_BYTES per GPU, held by the process until it ends and
 * shared by every call on that GPU, which keeps the last call's contents:
 * calls that overlap on one GPU (other streams, other host threads) race
 * and must be serialised by the caller.  The kernels clear what has to start
 * at zero.  No hipMalloc, hipFree, pinned-host allocation, memory copy or
 * graph is used.  flags: BP_NO_EARLY_EXIT only (the sweeps run dense;
 * BP_SEGMENTS is BP_ERR_ARG).  n + m > BP_NOALLOC_MAX_ITEMS: BP_ERR_LIMIT. */
#define BP_NOALLOC_MAX_ITEMS (1 << 14)
#define BP_NOALLOC_SCRATCH_BYTES (32u << 20)
bp_status bp_feasible_dev_noalloc(int32_t C, int32_t m, const int32_t *d_residual, const int32_t *d_unpacked,
                                  int64_t n, uint32_t flags, bp_bounds *d_out, void *stream);

/* ---- served checks (continuous batching) -------------------------------- */

/* One item committed to a bin by the search (Sec. 5: decreasing best fit
 * assigns an unpacked item to a bin), relative to a parent node. */
typedef struct bp_commit {
  int32_t size; /* the item's size: one of the parent's unpacked items */
  int32_t bin;  /* 0 .. m - 1; the bin's load plus size must not exceed C */
} bp_commit;

/* One request: a node of the search.  Either a partial packing in residual
 * form, as bp_feasible takes it (parent = 0), or the node reached from an
 * earlier request of the same queue (parent = its ticket) by committing
 * ncommit items: the unpacked items lose those sizes and each commit's bin
 * gains its size.  A child request is checked from the parent's per-
 * parameter sums kept on the device when they are still there (the reduced
 * instance changes by the committed items and by the changed bins' virtual
 * items, Fig. 3), else from the parent's instance kept on the host; its
 * residual and unpacked may then be NULL (n is ignored).  C and m of a child
 * are its parent's. */
typedef struct bp_request {
  int32_t C;
  int32_t m;
  int64_t n;
  const int32_t *residual; /* m entries */
  const int32_t *unpacked; /* n entries */
  uint64_t tag;            /* caller's value, returned in the result */
  uint32_t flags;          /* BP_NO_EARLY_EXIT | BP_SEGMENTS */
  uint32_t reserved;
  uint64_t parent;           /* 0, or the ticket of an earlier request of this queue */
  const bp_commit *commits;  /* ncommit items (parent != 0) */
  int32_t ncommit;           /* 0 .. BP_MAX_COMMIT */
  int32_t reserved2;
} bp_request;
#define BP_MAX_COMMIT 1024

typedef struct bp_result {
  uint64_t ticket;
  uint64_t tag;
  bp_status status;
  int32_t verdict;
  int64_t lb;
  double submit_us; /* host clock at submit, microseconds */
  double start_us;  /* host clock when the request's batch was launched */
  double done_us;   /* host clock when the result became visible */
  bp_bounds bounds;
  int32_t from_parent; /* 1: computed from another node's per-parameter sums; 0: full sweeps */
  int32_t reserved;
} bp_result;

typedef struct bp_queue_stats {
  uint64_t submitted, completed, rejected, batches, in_flight;
  uint64_t bytes_in_use, bytes_peak, budget;
  double busy_us;
  uint64_t from_parent;  /* completed from another node's sums */
  uint64_t full_sweeps;  /* completed by the full sweeps */
  uint64_t nodes_kept;   /* node states on the device now */
  uint64_t node_evictions;
  uint64_t node_bytes;   /* device bytes of the node-state arena */
} bp_queue_stats;

/* A queue owns a serving thread that admits requests into free slots while
 * earlier batches run, launches them as batches on its own streams and
 * publishes results.  hbm_budget_bytes is allocated at creation: three
 * quarters hold the node states of finished requests (least recently used
 * evicted first), one quarter bounds the device memory charged to admitted
 * requests (inputs and workspaces); max_slots bounds the requests admitted
 * at once.  A request that does not fit waits (blocking submit) or is
 * rejected with BP_ERR_AGAIN. */
typedef struct bp_queue bp_queue;
bp_status bp_queue_create(bp_ctx *ctx, size_t hbm_budget_bytes, int32_t max_slots, bp_queue **out);

/* Copy the request (the caller may free its arrays on return) and return a
 * ticket.  blocking = 0: BP_ERR_AGAIN when no slot or budget is free;
 * blocking = 1: wait for one.  A request larger than the admission share of
 * the budget is BP_ERR_LIMIT.  A child request whose parent the queue no
 * longer knows (the queue keeps the most recent BP_QUEUE_HISTORY nodes) and
 * that carries no instance is BP_ERR_STATE; a commit outside [0, m) or past
 * its bin's capacity is BP_ERR_RANGE. */
#define BP_QUEUE_HISTORY 65536
bp_status bp_queue_submit(bp_queue *q, const bp_request *req, int32_t blocking, uint64_t *ticket);

/* Up to max finished results; waits up to timeout_us (0 = do not wait) for
 * the first one.  *got receives the count. */
bp_status bp_queue_poll(bp_queue *q, bp_result *out, int32_t max, int32_t *got, int32_t timeout_us);

bp_status bp_queue_stats_get(bp_queue *q, bp_queue_stats *out);

/* Open-loop replay of a request stream, for load tests: request i is
 * submitted (non-blocking) once arrival_s[i] seconds have passed since the
 * call began (arrival_s non-decreasing).  parent_index[i] >= 0 names an
 * earlier request of the stream: the request is submitted as that one's
 * child (its parent field is set to that request's ticket); if that request
 * was not admitted, this one is not submitted either (status[i] =
 * BP_ERR_STATE), as a search cannot go on from a node it never checked.
 * tickets[n] receives the tickets (0 when not admitted), status[n] each
 * submit's status (BP_ERR_AGAIN when rejected), *lateness_s the largest
 * delay between an arrival time and its submit.  The requests' arrays must
 * stay valid during the call; reqs[i].parent is overwritten. */
bp_status bp_queue_replay(bp_queue *q, bp_request *reqs, const double *arrival_s, const int64_t *parent_index,
                          int64_t n, uint64_t *tickets, int32_t *status, double *lateness_s);

/* Stop admitting, finish the batches on the device, complete still-queued
 * requests with BP_ERR_STATE, join the thread and free everything. */
bp_status bp_queue_destroy(bp_queue *q);

/* ---- the propagator and the search around the check ---------------------- */

/* A caller's feasibility check for bp_solve: the lower bound *lb of the
 * partial packing (residual[m] of the k = m bins, unpacked[n]).  Return
 * BP_OK, or an error that stops the search. */
typedef bp_status (*bp_check_fn)(void *user, int32_t C, int32_t m, const int32_t *residual,
                                 const int32_t *unpacked, int64_t n, int64_t *lb);

enum { BP_SOLVE_DFFS = 0, BP_SOLVE_L2 = 1, BP_SOLVE_NO_CHECK = 2 };
enum { BP_SOLVE_OPTIMAL = 1, BP_SOLVE_LIMIT = 0 };
/* bp_solve_opts.disable: rules switched off (all on by default) */
enum {
  BP_SOLVE_OFF_KNAPSACK = 1u << 0,  /* the knapsack filtering of Alg. 1 */
  BP_SOLVE_OFF_FILL = 1u << 1,      /* dominance: an item that fills a bin exactly goes there */
  BP_SOLVE_OFF_SINGLE = 1u << 2,    /* dominance: a bin into which no two items fit takes the heaviest */
  BP_SOLVE_OFF_SYMMETRY = 1u << 3   /* on backtracking, bins of the same load leave same-size items */
};

typedef struct bp_solve_opts {
  int32_t mode;          /* the check at every node: BP_SOLVE_DFFS (the whole collection, bp_feasible),
                            BP_SOLVE_L2 (L1 and L2 only), BP_SOLVE_NO_CHECK (filtering alone) */
  uint32_t check_flags;  /* flags of bp_feasible for BP_SOLVE_DFFS (BP_SEGMENTS, BP_NO_EARLY_EXIT) */
  int64_t max_nodes;     /* search nodes per attempt (0: no limit) */
  double time_limit_s;   /* for the whole solve (0: no limit) */
  bp_check_fn check;     /* non-NULL: this check replaces the library's (ctx may then be NULL) */
  void *user;
  uint32_t disable;      /* BP_SOLVE_OFF_* bits */
  int32_t reserved;
} bp_solve_opts;

typedef struct bp_solve_result {
  int32_t status;        /* BP_SOLVE_OPTIMAL: bins is the optimum; BP_SOLVE_LIMIT: a limit stopped an attempt */
  int32_t bins;          /* bins of the packing returned */
  int32_t lower;         /* the root's lower bound (the first k tried) */
  int32_t upper;         /* first fit decreasing's bins */
  int32_t attempts;      /* values of k tried */
  int32_t limit_reached;
  int64_t nodes;         /* search nodes over all attempts */
  int64_t fails;         /* nodes whose subtree held no packing */
  int64_t checks;        /* feasibility checks (Alg. 1) */
  int64_t check_fails;   /* checks with lb > k */
  double seconds;
  double check_seconds;  /* time inside the checks */
  int64_t filter_fails;  /* nodes the filtering rules failed before the check */
} bp_solve_result;

/* Bin packing by the paper's resolution procedure (Sec. 5): k starts at the
 * root's lower bound and grows until an attempt packs the n items into k
 * bins; first fit decreasing bounds it from above.  An attempt is a
 * depth-first search with decreasing best fit, the two symmetry-breaking
 * rules on backtracking and the two dominance rules of Sec. 5 (exact fill;
 * the heaviest item into a bin that takes at most one more).  Every node
 * runs the filtering of Alg. 1 (load coherence, basic load tightening, item
 * elimination and commitment, then the same through the knapsack test of
 * bp_subset_sum_gap) to a fixpoint and then the feasibility check of Alg. 1.
 * The reductions and the symmetry constraint the paper's solvers add from
 * other work are not built.  bin_of[n] (optional) receives the packing, in
 * the caller's item order.  Sizes in [0, C], n <= 16 384.  Errors:
 * BP_ERR_ARG (NULL, C < 1, unknown mode, the library's check without a
 * context), BP_ERR_RANGE (a size outside [0, C]), BP_ERR_LIMIT, or the
 * check's own error, which stops the search. */
bp_status bp_solve(bp_ctx *ctx, int32_t C, int64_t n, const int32_t *sizes, const bp_solve_opts *opts,
                   int32_t *bin_of, bp_solve_result *out);

/* The knapsack test of the propagator (the bin packability, load tightening
 * and item reasoning of Alg. 1 rest on it): an approximate subset-sum test
 * over x[n], sorted non-increasing, host memory.  Returns 1 when it proves
 * that no subset of x sums into [alpha, beta]; then every subset sum is
 * <= *below or >= *above (*above is 2^61 - 1 when no sum exceeds beta).
 * Returns 0 when it proves nothing (alpha <= 0 <= beta is always 0: the
 * empty set).  BP_ERR_ARG for NULL pointers, n < 0, or x not sorted. */
int32_t bp_subset_sum_gap(const int32_t *x, int32_t n, int64_t alpha, int64_t beta, int64_t *below,
                          int64_t *above);

/* ---- self test of the host-side division constants ----------------------- */

/* Checks, on the host, the multiply-shift constants the kernels use against
 * plain integer division: every divisor d in [d_lo, d_hi] with numerators
 * n in [0, n_hi] (and the extreme numerators).  mode 0: floor(n / d) for
 * n < 2^31; mode 1: ceil(a lam / c) - 1 (f_VB2's quotient), d taken as c;
 * mode 2: the divisibility test d | n; mode 3: floor(n / d) through an fp64
 * reciprocal and one correction step; mode 4: floor((a lam - 1) / c) the
 * same way, d taken as c; mode 5: floor(n / d) by one high multiply where
 * n d <= 2^32 (d >= 2); mode 6: ceil(a lam / c) - 1 by one high multiply
 * where a c <= 2^32, d taken as c.  d_lo >= 1, d_hi < 2^31, n_hi < 2^31, else
 * BP_ERR_ARG (also for any other mode).  Returns the number of mismatches
 * found (0 = all exact) or a negative status. */
int64_t bp_selftest_division(uint32_t d_lo, uint32_t d_hi, uint32_t n_hi, uint32_t mode);

#ifdef __cplusplus
}
#endif
#endif /* BP_H_ */
