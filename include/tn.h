/*
 * tn.h - C ABI of the MI355X (gfx950) temporal component-matrix library.
 *
 * The library computes, for a temporal network of n nodes and m events
 * (u, v, t), the component matrix of Sec. 3 of "Temporal network compression
 * via network hashing": bit (u, w) is 1 iff node w is reachable from node u by
 * a time-respecting path (Sec. 2.1).  The matrix is built by streaming the
 * events in reverse chronological order (Sec. 3.4), each event OR-ing one
 * bit-packed row into another (Algorithm 1's update), so that row u is the
 * maximum out-component of u and column w the in-component of w.  On top of
 * it sit the hashing framework of Sec. 4 (H hashed proxy networks of K
 * super-nodes, built in one batched launch, Sec. 4.1 and 4.3) and the fusion
 * estimator of Sec. 4.2, plus a learned combiner (a small MLP) that maps the
 * H per-hash lifted sizes to a size estimate.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: tn_status, 0 on success, a negative code otherwise; the
 *   thread-local message of the last failure is tn_last_error().  Arguments
 *   are validated on the host before any device work is enqueued; on error
 *   nothing is enqueued and no output is touched.
 * - Memory: pointers documented HOST are ordinary host memory, borrowed for
 *   the duration of the call.  Pointers documented DEVICE are device memory
 *   on the context's device, owned by the caller and never freed by the
 *   library.  The context owns all scratch memory it allocates (device
 *   scratch, and pinned host staging for device-to-host copies); it serves
 *   one call at a time.
 * - Ordering: device work is enqueued on the context's stream (tn_create /
 *   tn_set_stream) and is asynchronous unless stated otherwise;
 *   tn_sync() waits for it and reports a device-side error.
 * - Bit layout: a bit matrix of R rows is R rows of ld uint64 words,
 *   row-major; node w is bit (w & 63) of word (w >> 6); ld >= ceil(n/64);
 *   every bit at a column >= n, and every word beyond ceil(n/64), is 0 in
 *   every output.
 * - Events: src/dst uint32 node ids < n; t int64 integer time steps
 *   (Sec. 2.1), non-decreasing (the time-ordered list of Algorithm 1).
 *   Unless TN_TIES_SEQUENTIAL is set, events at the same time step are not
 *   adjacent (Sec. 2.1): information crosses at most one event per time
 *   step.  Self-loops are no-ops; repeated events are idempotent.
 * - Determinism: every integer output is bit-exact and independent of launch
 *   configuration; MLP outputs are deterministic for a given input.
 */
#ifndef TN_H
#define TN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tn_status;
enum {
    TN_OK = 0,
    TN_E_ARG = -1,         /* bad size, null pointer, ld too small, ...      */
    TN_E_RANGE = -2,       /* a node id >= n                                 */
    TN_E_ORDER = -3,       /* event times decrease                           */
    TN_E_NOMEM = -4,       /* host or device allocation failed               */
    TN_E_HIP = -5,         /* a HIP runtime call failed                      */
    TN_E_UNSUPPORTED = -6  /* outside the supported sizes                    */
};

/* Event flags. */
enum {
    TN_DIRECTED = 1u,        /* event (u, v, t) carries information u -> v only
                                (the non-mutual sharing of the footnote in Sec. 3) */
    TN_TIES_SEQUENTIAL = 2u, /* list order is strict time order: Algorithm 1 read
                                literally, events at one time step chain          */
    TN_FORWARD = 4u,         /* Algorithm 1 in time order (Sec. 3.1): row x of the
                                result is x's in-component (the nodes that can
                                reach x) instead of its out-component; the result
                                is the transpose of the reverse-time one
                                (Sec. 3.4).  Not valid for hashing.            */
    TN_HLL = 8u              /* tn_plan_create only: plan for tn_hll_execute
                                (the time-step schedule its register stream
                                runs level by level); tn_plan_execute rejects
                                such a plan                                    */
};

typedef struct tn_ctx tn_ctx;     /* device, stream, scratch, autotune cache   */
typedef struct tn_plan tn_plan;   /* one network's device-resident schedule    */
typedef struct tn_batch tn_batch; /* many networks' schedules, one launch      */

/* ---- context ---------------------------------------------------------- */

/* Thread-local text of the last error (never NULL). */
const char *tn_last_error(void);

/* The row stride (in uint64 words) this library suggests for a bit matrix of
 * n columns: ceil(n/64) rounded up to 16 words (one 128-byte line) once a
 * row spans 16 words or more, so that every row starts on a line and the
 * column slices of the row-OR kernels never straddle two lines; ceil(n/64)
 * below that.  Any ld >= ceil(n/64) is accepted everywhere; this one is
 * faster (the padding words are written as 0).  Host only. */
int64_t tn_recommended_ld(uint32_t n);

/* Creates a context on HIP device `device`, enqueuing on `stream` (a
 * hipStream_t; NULL = the null stream).  *out receives the context. */
tn_status tn_create(int device, void *stream, tn_ctx **out);

/* Changes the stream subsequent calls enqueue on. */
tn_status tn_set_stream(tn_ctx *ctx, void *stream);

/* Waits for the context's stream; reports a device error as TN_E_HIP. */
tn_status tn_sync(tn_ctx *ctx);

/* Frees the context's scratch memory (device and pinned host).  Plans and
 * batches must be destroyed first.  NULL is ignored. */
void tn_destroy(tn_ctx *ctx);

/* Kernel timing on the context's stream.  While enabled, every kernel the
 * context launches is bracketed by two HIP events recorded on its stream.
 * tn_profile_take waits for the stream, writes up to `cap` records (kernel
 * id, milliseconds) in launch order to HOST arrays ids / ms, clears all
 * records and returns how many it wrote (or a negative tn_status). */
enum {
    TN_K_IDENTITY = 1,     /* C <- I                                        */
    TN_K_ROWOR = 2,        /* the level-by-level row-OR stream              */
    TN_K_OUT_SIZES = 3,    /* row popcounts                                 */
    TN_K_IN_SIZES = 4,     /* column popcounts                              */
    TN_K_BATCH = 5,        /* persistent multi-network row-OR               */
    TN_K_HASH = 6,         /* bucket map and bucket counts                  */
    TN_K_RECOMBINE = 7,    /* fusion of the hashed proxies                  */
    TN_K_MLP_FORWARD = 8,
    TN_K_MLP_BACKWARD = 9,
    TN_K_MLP_ADAM = 10,
    TN_K_AUX = 11          /* small fills, features, reductions             */
};
tn_status tn_profile_enable(tn_ctx *ctx, int enable);
int32_t tn_profile_take(tn_ctx *ctx, int32_t *ids, float *ms, int32_t cap);

/* ---- exact component matrix (Sec. 3, Algorithm 1, reverse time Sec. 3.4) */

/* Plans the reverse-time stream of one network on the host: groups the events
 * of each time step into independent items (two-node pairs, or compound
 * groups where a node meets several others at one time step, which must read
 * every old row before writing any), turns them into binary row-OR ops
 * (compound groups fold through scratch rows), and places each op on the
 * earliest level after the last write of every row it reads and the last
 * access of every row it writes, so the ops of one level are independent;
 * levels hold at most 1024 ops.  The schedule is copied to the device
 * (synchronously) and kept in the plan.
 * src, dst, t: HOST, m entries.  flags: TN_DIRECTED | TN_TIES_SEQUENTIAL |
 * TN_FORWARD (the stream then runs in time order) | TN_HLL (a plan of pair
 * and compound items by level, for tn_hll_execute only).
 * Errors: TN_E_ARG (n == 0, null arrays with m > 0, bad flags),
 * TN_E_RANGE, TN_E_ORDER, TN_E_UNSUPPORTED (m >= 2^32 or n >= 2^31). */
tn_status tn_plan_create(tn_ctx *ctx, uint32_t n, int64_t m,
                         const uint32_t *src, const uint32_t *dst,
                         const int64_t *t, uint32_t flags, tn_plan **out);

typedef struct tn_plan_stats {
    uint32_t n;
    int64_t m;
    int64_t levels;          /* dependency levels of the schedule          */
    int64_t pairs;           /* two-node items                             */
    int64_t gathers;         /* rows written by compound items             */
    int64_t gather_sources;  /* rows read by compound items                */
    int64_t compound_items;  /* time-step groups of >= 3 nodes             */
    int64_t max_level_items; /* widest level (pairs + gathers)             */
    int64_t max_level_gathers;
    int64_t device_bytes;    /* size of the device-resident schedule       */
    double host_seconds;     /* planning time on the host                  */
    int64_t directed_pairs;  /* pairs that update one row only             */
    int64_t ops;             /* binary ops of the device schedule          */
    int64_t op_levels;       /* levels of the binary-op schedule           */
    int64_t scratch_rows;    /* scratch rows compound time steps fold into */
} tn_plan_stats;

tn_status tn_plan_get_stats(const tn_plan *plan, tn_plan_stats *out);

/* Host-only form of the planning step (no device needed): builds the same
 * level schedule tn_plan_create uploads and exposes it for inspection.
 * Level l (0-based, l < levels) owns pair items [lvl_pair[l], lvl_pair[l+1])
 * of `pairs` (2 uint32 each: u, then v with bit 31 set for a one-way
 * directed pair that only updates row u) and gathers [lvl_gat[l],
 * lvl_gat[l+1]); gather g writes row gat_tgt[g] with the OR of rows
 * gat_src[gat_ptr[g] .. gat_ptr[g+1]) as they were before the level.
 * The arrays are owned by the schedule and valid until its destruction. */
typedef struct tn_host_schedule tn_host_schedule;
tn_status tn_schedule_build(uint32_t n, int64_t m, const uint32_t *src,
                            const uint32_t *dst, const int64_t *t,
                            uint32_t flags, tn_host_schedule **out);
tn_status tn_schedule_arrays(const tn_host_schedule *s, tn_plan_stats *stats,
                             const uint32_t **lvl_pair, const uint32_t **lvl_gat,
                             const uint32_t **pairs, const uint32_t **gat_tgt,
                             const uint32_t **gat_ptr, const uint32_t **gat_src);
/* The binary-op form of the same schedule, the one tn_plan_create uploads:
 * level l (l < stats.op_levels) owns ops [lvl_op[l], lvl_op[l+1]) of `ops`,
 * 4 uint32 each {a, b, d1, d2}: r = row a | row b, then rows d1 and d2 get r
 * (d2 = 0xffffffff: none).  A row id with bit 31 set is scratch row
 * (id & 0x7fffffff); an undirected pair is (u, v, u, v), a one-way pair
 * (u, v, u, none), and a compound time step folds each target's old row and
 * its partners' old rows into a scratch row, then copies it back.  Ops of
 * one level read rows no op of that level writes. */
tn_status tn_schedule_op_arrays(const tn_host_schedule *s,
                                const uint32_t **lvl_op, const uint32_t **ops);
/* The forwarded form of the binary-op schedule that the plain row-OR kernel
 * runs (host only, for inspection and tests): levels of at most level_cap
 * ops (0 or more than 768: 768, the form the kernel runs; smaller caps
 * split more levels), *levels of them, level l owning ops [lvl[l], lvl[l+1]),
 * 4 uint32 each {a, b, d1, d2} as in the op form, except that an operand
 * with bit 30 set is the result r of op (operand & 0x3ff) of level l - 1,
 * and a destination with bit 30 set is not written to memory (level l + 1
 * overwrites that row, reading it, if at all, through the same
 * forwarding).  Within a level, an op with exactly one operand read from
 * memory has it as b, and the ops with both read from memory come first.
 * The arrays live until tn_schedule_destroy or the next call with another
 * level_cap. */
tn_status tn_schedule_fwd_arrays(tn_host_schedule *s, uint32_t level_cap, uint32_t *levels,
                                 const uint32_t **lvl, const uint32_t **ops);
void tn_schedule_destroy(tn_host_schedule *s);

/* Destroys a plan (frees its device schedule).  NULL is ignored. */
void tn_plan_destroy(tn_plan *plan);

/* Runs a plan: C <- I_n, then every level of row ORs in order.
 * C: DEVICE, n x ld uint64, written entirely (including padding words).
 * slice_words: words of every row one workgroup owns (0 = tuned default);
 * any value gives the same bits.  Errors: TN_E_ARG (ld < ceil(n/64)). */
tn_status tn_plan_execute(tn_ctx *ctx, const tn_plan *plan, uint64_t *C,
                          int64_t ld, uint32_t slice_words);

/* Saturated rows (Sec. 3.4: rows of the reverse-time matrix only gain bits,
 * and an OR with a row that already holds every column of a slice gives that
 * full slice).  Enabled by default: tn_plan_execute and tn_batch_execute then
 * skip the row loads such an operand makes redundant and the stores of full
 * results into rows already full, and a workgroup stops once every row of its
 * column slice is full; the matrices they write are identical either way.
 * enable = 0 makes every op load and store its rows (a batch re-plans its
 * launch shape at its next execution).  Errors: TN_E_ARG (ctx NULL). */
tn_status tn_set_saturation(tn_ctx *ctx, int enable);

/* Row traffic of the last tn_plan_execute on this context: words[0] = uint64
 * row words its row-OR kernel loaded, words[1] = row words it stored (words
 * of the padding columns past ceil(n/64) are not counted).  words: HOST
 * uint64[2], zeros before the first execute.  Waits for the context's
 * stream.  Errors: TN_E_ARG, TN_E_HIP. */
tn_status tn_plan_last_traffic(tn_ctx *ctx, uint64_t *words);

/* One call (Sec. 3.1 Algorithm 1 in reverse time, Sec. 3.4).  Inputs HOST,
 * C DEVICE as above; the call returns once C is complete.  It runs the
 * streamed build below with its default chunk size. */
tn_status tn_build_component_matrix(tn_ctx *ctx, uint32_t n, int64_t m,
                                    const uint32_t *src, const uint32_t *dst,
                                    const int64_t *t, uint32_t flags,
                                    uint64_t *C, int64_t ld);

/* Streamed one-shot build (Sec. 3.4: the reverse-time recurrence consumes
 * the event list from its end).  The list is cut into chunks of about
 * chunk_events events on time-step boundaries; 0 selects chunks of
 * max(2^18, m/64) events after a first chunk of a quarter of that (at least
 * 2^14) that doubles up to it, so that a stream that saturates early plans
 * little before its first launch; host
 * threads plan chunks concurrently while the device applies them in
 * reverse-time order to C.  Rows only gain bits, so once every row is all
 * ones within a column slice nothing earlier in time can change it: such
 * slices stop, and once all slices have, the remaining (earlier) chunks are
 * neither planned further nor run.  The result equals tn_plan_execute's.
 * Inputs HOST, borrowed for the call; C DEVICE, n x ld, written entirely.
 * stats (HOST, may be NULL) reports what ran.  Errors as tn_plan_create,
 * plus TN_E_ARG for ld < ceil(n/64) or chunk_events < 0; nothing is
 * enqueued when validation fails. */
typedef struct {
    int64_t chunks;       /* chunks the list was cut into                   */
    int64_t chunks_run;   /* chunks launched on the device                  */
    int64_t events_run;   /* events in the launched chunks                  */
    int64_t levels_run;   /* op levels in the launched chunks               */
    int32_t saturated;    /* 1: every row ended all ones, and it was seen   */
    int32_t slice_words;  /* words per row each workgroup owned             */
    double seconds;       /* wall time of the call                          */
} tn_stream_stats;
tn_status tn_build_component_matrix_streamed(tn_ctx *ctx, uint32_t n, int64_t m,
                                             const uint32_t *src, const uint32_t *dst,
                                             const int64_t *t, uint32_t flags,
                                             uint64_t *C, int64_t ld,
                                             int64_t chunk_events,
                                             tn_stream_stats *stats);

/* Online insertion (Sec. 3.5: the matrix algorithm takes new events, and new
 * nodes as new identity rows, without recomputation).  tn_online_create
 * writes C <- I (n rows; a node joins with its first event) and keeps the
 * stream state of C: its column slices' saturation bits and a launch ring.
 * Each tn_online_insert applies a batch of events to C as the next part of
 * one stream, chunked and planned as in tn_build_component_matrix_streamed.
 * With TN_FORWARD the stream runs in time order: every batch must be later
 * than all events applied so far, and C's rows are in-components (Algorithm
 * 1 as printed).  Without it the stream runs in reverse time: every batch
 * must be earlier than all applied, and rows are out-components.  Events of
 * one time step form one snapshot and must come in one batch (with
 * TN_TIES_SEQUENTIAL a batch may continue the last time step).  Once every
 * row is all ones, further batches change nothing and are skipped.
 * C: DEVICE, n x ld, caller-owned, must outlive the state; it is complete
 * once the context's stream reaches the work an insert enqueued (tn_sync).
 * Event arrays: HOST, read during the call only.  stats (HOST, may be NULL)
 * describe the batch.  Errors: TN_E_ARG (bad sizes, flags, ld, or a state
 * of another context), TN_E_RANGE, TN_E_ORDER (times within the batch, or
 * against those applied); nothing is enqueued when a check fails. */
typedef struct tn_online tn_online;
tn_status tn_online_create(tn_ctx *ctx, uint32_t n, uint32_t flags,
                           uint64_t *C, int64_t ld, tn_online **out);
tn_status tn_online_insert(tn_ctx *ctx, tn_online *online, int64_t m,
                           const uint32_t *src, const uint32_t *dst,
                           const int64_t *t, int64_t chunk_events,
                           tn_stream_stats *stats);
/* Waits for the context's stream and frees the state (not C).  NULL is
 * ignored. */
void tn_online_destroy(tn_online *online);

/* HyperLogLog variant of the stream (Sec. 3.4, last paragraph; HLL in
 * Sec. 2.2): every node starts with the HLL structure of {node} and each
 * time step merges the structures its events join (register-wise maximum,
 * the same level schedule and snapshot ties as the matrix), so row u ends as
 * the HLL structure of u's out-component (in-component with TN_FORWARD) in
 * s = 2^log2s one-byte registers instead of n bits.  Registers follow
 * Flajolet et al. (2007): the top log2s bits of an element's 64-bit hash pick
 * the register, which keeps the largest 1-based position of the leftmost 1
 * in the remaining bits (64 - log2s + 1 for all zeros).  est[u] is the HLL
 * estimate alpha_s s^2 / sum_j 2^-M[j], or s ln(s / V) when that is at most
 * 5s/2 and V > 0 registers are zero (alpha_16 = 0.673, alpha_32 = 0.697,
 * alpha_64 = 0.709, else 0.7213 / (1 + 1.079 / s)).
 * node_hash: DEVICE uint64[n], one uniform hash per node (an input: the
 * library draws no random numbers).  M: DEVICE n x s uint8, row-major,
 * written entirely, starting on 16 bytes (rows move in 16-byte words).  est: DEVICE float64[n] or NULL.  log2s in [4, 16].
 * tn_hll_execute runs on a plan's schedule (asynchronous): on a TN_HLL
 * plan one launch per level (two for a level with compound items) spreads
 * the level's items over the whole device, one group of lanes per item and
 * row; on another plan the row-OR kernel's level loop runs with byte-wise
 * maximum, one workgroup per word column.  tn_hll_build plans (TN_HLL), runs
 * and waits.  Errors: TN_E_ARG, plus those of tn_plan_create. */
tn_status tn_hll_execute(tn_ctx *ctx, const tn_plan *plan, uint32_t log2s,
                         const uint64_t *node_hash, uint8_t *M, double *est);
tn_status tn_hll_build(tn_ctx *ctx, uint32_t n, int64_t m, const uint32_t *src,
                       const uint32_t *dst, const int64_t *t, uint32_t flags,
                       uint32_t log2s, const uint64_t *node_hash, uint8_t *M,
                       double *est);

/* tn_plan_execute, then the component sizes of the matrix it wrote (as
 * tn_component_sizes; Sec. 3.1, Eq. 1).  A saturating execution leaves a
 * per-slice state in which a slice whose every row ended all ones is marked
 * (Sec. 3.4: rows only gain bits); its columns then count in every row's
 * out-size and have in-size n without a read of the matrix, so a saturated
 * network's sizes cost no second pass over C.  Other slices, and executions
 * that keep no state (saturation off, small networks on one wavefront per
 * word column), are counted from C.  Arguments and errors as
 * tn_plan_execute and tn_component_sizes; out_sizes, in_sizes: DEVICE
 * int32[n], either may be NULL. */
tn_status tn_plan_execute_sizes(tn_ctx *ctx, const tn_plan *plan, uint64_t *C, int64_t ld,
                                uint32_t slice_words, int32_t *out_sizes, int32_t *in_sizes);

/* Component sizes (Sec. 3.1, Eq. 1): out_sizes[u] = ones in row u (the
 * maximum out-component size of u), in_sizes[w] = ones in column w (the
 * in-component size of w).  C: DEVICE n x ld.  out_sizes, in_sizes: DEVICE
 * int32[n], either may be NULL.  Padding bits of C must be 0. */
tn_status tn_component_sizes(tn_ctx *ctx, uint32_t n, const uint64_t *C,
                             int64_t ld, int32_t *out_sizes, int32_t *in_sizes);

/* ---- many networks in one persistent launch ---------------------------- */

/* Plans B networks (host threads) and uploads their schedules.  Arrays of B
 * entries: n[b], m[b], and HOST pointers src[b], dst[b], t[b] as in
 * tn_plan_create.  Errors as tn_plan_create, for the first failing b. */
tn_status tn_batch_create(tn_ctx *ctx, int32_t B, const uint32_t *n,
                          const int64_t *m, const uint32_t *const *src,
                          const uint32_t *const *dst, const int64_t *const *t,
                          uint32_t flags, tn_batch **out);

/* Builds all B component matrices in one persistent launch: workgroups take
 * (network, column slice) tiles from a device work queue, largest first,
 * keep the slice in LDS when it fits, and write it back to C[b].  The first
 * call tunes the tile shape on the device and captures the launch in a HIP
 * graph; later calls with the same C / ld replay it.  C: HOST array of B
 * DEVICE pointers, ld: HOST array of B leading dimensions. */
tn_status tn_batch_execute(tn_ctx *ctx, tn_batch *batch, uint64_t *const *C,
                           const int64_t *ld);

/* Per-batch statistics: total levels, pairs, tiles and the chosen shape.
 * stats: HOST array of B entries, or NULL.  tiles, lds_tiles may be NULL. */
tn_status tn_batch_get_stats(const tn_batch *batch, tn_plan_stats *stats,
                             int64_t *tiles, int64_t *lds_tiles);

/* The launch shape the batch runs with (the tuned one once it has been
 * executed): shape[0] threads per workgroup, [1] dynamic LDS bytes per
 * workgroup, [2] workgroups resident per compute unit, [3] grid size,
 * [4] slice halvings below the widest slice that fits, [5] slice width of
 * global-memory tiles in words.  shape: HOST int64[6].  Errors: TN_E_ARG. */
tn_status tn_batch_get_shape(const tn_batch *batch, int64_t *shape);

void tn_batch_destroy(tn_batch *batch);

/* One call: batch create, execute, destroy. */
tn_status tn_build_component_matrix_batched(tn_ctx *ctx, int32_t B,
                                            const uint32_t *n, const int64_t *m,
                                            const uint32_t *const *src,
                                            const uint32_t *const *dst,
                                            const int64_t *const *t,
                                            uint32_t flags, uint64_t *const *C,
                                            const int64_t *ld);

/* ---- hashing framework (Sec. 4) ----------------------------------------- */

/* Network hashing (Sec. 4.1): H independent hash functions map the n nodes
 * to K super-nodes, h_j(u) = (acc_0(x0) ^ acc_1(x1) ^ acc_2(x2)) mod K with
 * x0 / x1 the low / high 32 bits of u, x2 = x0 + x1, and acc_i a polynomial
 * of `order` coefficients evaluated by repeated (x * acc + a) mod (2^61 - 1).
 * coeffs: HOST, H x 3 x order uint64, each < 2^61 - 1 (the random table A).
 * Writes bucket[j*n + u] = h_j(u) (DEVICE uint32[H*n]) and
 * count[j*K + r] = |h_j^{-1}(r)| (DEVICE int32[H*K]), then plans the H
 * hashed networks (super-events (h_j(u), h_j(v), t)) as one batch, returned
 * in *proxies; build them with tn_batch_execute into H matrices of K rows.
 * src, dst, t: HOST events as in tn_plan_create.
 * Errors: TN_E_ARG (H == 0, K == 0, order < 1), TN_E_UNSUPPORTED
 * (K > 65536), TN_E_RANGE, TN_E_ORDER. */
tn_status tn_hash_compress(tn_ctx *ctx, uint32_t n, int64_t m,
                           const uint32_t *src, const uint32_t *dst,
                           const int64_t *t, uint32_t flags, uint32_t H,
                           uint32_t K, const uint64_t *coeffs, int32_t order,
                           uint32_t *bucket, int32_t *count,
                           tn_batch **proxies);

/* Hash and build all H proxies in one call, streamed (Sec. 4.1 hashing,
 * Sec. 4.3 independent proxies, Sec. 3.4 reverse time).  bucket and count as
 * in tn_hash_compress; P: DEVICE, H consecutive K x ldK uint64 matrices
 * (proxy j at P + j*K*ldK), written entirely.  The event list is cut into
 * chunks of whole time steps from its end (chunk_events as in
 * tn_build_component_matrix_streamed, except that the default first chunk
 * is a sixteenth of the others: proxies of few super-nodes saturate within
 * few events); each chunk's H mapped sub-streams are
 * planned on host threads and applied in one launch that resumes from the
 * proxies (K <= 4096: one wavefront per word column of every proxy, the
 * column in LDS; larger K: batched tiles).  Once every column or tile of
 * every proxy is all ones the earlier chunks are skipped.  The proxies
 * equal those of tn_hash_compress + tn_batch_execute.  stats (HOST, may be
 * NULL) as for the streamed build.  The bucket maps come down into pinned
 * host memory that the context keeps for later calls (4*H*n bytes).
 * Errors as tn_hash_compress, plus TN_E_ARG for ldK < ceil(K/64). */
tn_status tn_hash_build_proxies(tn_ctx *ctx, uint32_t n, int64_t m,
                                const uint32_t *src, const uint32_t *dst,
                                const int64_t *t, uint32_t flags, uint32_t H,
                                uint32_t K, const uint64_t *coeffs, int32_t order,
                                uint32_t *bucket, int32_t *count, uint64_t *P,
                                int64_t ldK, int64_t chunk_events,
                                tn_stream_stats *stats);

/* Fusion (Sec. 4.2, Eqs. DefInvHComp and DefEstOCMerge):
 * est[u] = |{w < n : P_j[h_j(u)][h_j(w)] = 1 for every j < H}|, the size of
 * the estimated out-component (a superset of the true one), and, if lifted
 * is not NULL, lifted[j*n + u] = |h_j^{-1}(OC_j(h_j(u)))| =
 * sum of count[j][r] over the super-nodes r in row h_j(u) of P_j.
 * P: DEVICE, H matrices of K rows x ldK words, matrix j at P + j*K*ldK.
 * bucket, count: DEVICE as written by tn_hash_compress.
 * est: DEVICE int32[n].  lifted: DEVICE int32[H*n] or NULL.
 * A node whose proxy row is full in every hash keeps every node (est = n)
 * and skips the AND over the chunks; the call waits for the context's
 * stream once, to size that work. */
tn_status tn_recombine(tn_ctx *ctx, uint32_t n, uint32_t H, uint32_t K,
                       const uint64_t *P, int64_t ldK, const uint32_t *bucket,
                       const int32_t *count, int32_t *est, int32_t *lifted);

/* ---- learned combiner (a 16 -> 64 -> 64 -> 1 ReLU MLP, FP32) ------------ */

/* Number of float parameters: per layer W (out x in, row-major) then b. */
int32_t tn_mlp_param_count(void);

/* Seeded initial parameters on the device: every weight of layer i is
 * (2u - 1) * sqrt(6 / fan_in_i) (He-uniform), every bias 0.  For weight p
 * of the packed vector, u is the top 24 bits of the p-th output of a
 * SplitMix64 generator seeded with `seed` (Steele, Lea and Flood, 2014),
 * times 2^-24; the product is formed in fp64 and rounded to float once.
 * Equal seeds give bit-equal parameters on any device.  params: DEVICE
 * float[tn_mlp_param_count()], caller-owned, overwritten; asynchronous on the
 * context's stream.  Errors: TN_E_ARG for a NULL ctx or params. */
tn_status tn_mlp_init(tn_ctx *ctx, uint64_t seed, float *params);

/* Features x[u*H + j] = ln(lifted[j*n + u] / n) as float.  lifted: DEVICE
 * int32[H*n]; x: DEVICE float[n*H].  H must be 16. */
tn_status tn_mlp_features(tn_ctx *ctx, uint32_t n, uint32_t H,
                          const int32_t *lifted, float *x);

/* yhat[i] = MLP(x[i*16 .. i*16+15]).  params, x, yhat: DEVICE. */
tn_status tn_mlp_forward(tn_ctx *ctx, const float *params, const float *x,
                         int64_t N, float *yhat);

/* Size estimates from the network's output: sizes[i] = n_nodes * exp(yhat)
 * where yhat = MLP(x[i]), clamped to [1, est[i]] when est is not NULL (the
 * fusion estimate is an upper bound of the true size) and to [1, n_nodes]
 * otherwise.  params, x: DEVICE; est: DEVICE int32[N] or NULL; sizes:
 * DEVICE float[N]. */
tn_status tn_mlp_predict(tn_ctx *ctx, const float *params, const float *x,
                         int64_t N, uint32_t n_nodes, const int32_t *est,
                         float *sizes);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, 1-based
 * step) on the mean squared error over N samples.  Sample s is row idx[s] of
 * x / entry idx[s] of y when idx is not NULL (a minibatch drawn from a
 * resident dataset; every idx[s] must index a row of x), else row s.
 * params, adam_m, adam_v: DEVICE
 * float[tn_mlp_param_count()], updated in place.  x: DEVICE float rows of
 * 16; y: DEVICE float; idx: DEVICE int32[N] or NULL.  loss: DEVICE float[1]
 * or NULL, receives the loss before the step.  grad: DEVICE float[param
 * count] or NULL, receives the gradient.  The gradient is summed in a fixed
 * order, so equal inputs give bit-equal results. */
tn_status tn_mlp_train_step(tn_ctx *ctx, float *params, float *adam_m,
                            float *adam_v, int64_t step, const float *x,
                            const float *y, const int32_t *idx, int64_t N,
                            float lr, float *loss, float *grad);

/* tn_mlp_train_step for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same step, bit for bit, with its partial gradients in a
 * static device array of the library instead of the context's scratch.  The
 * call allocates nothing.  N must be <= 16384 (TN_E_UNSUPPORTED otherwise;
 * nothing is enqueued); the array takes 5.4 MB on each GPU the library runs
 * on, held until the process ends, and is bound at tn_create.  Every call on
 * a GPU shares that GPU's array, so calls that overlap on one GPU (several
 * streams or threads) race; calls in stream order do not.  Arguments,
 * ownership and the other errors as tn_mlp_train_step. */
tn_status tn_mlp_train_step_noalloc(tn_ctx *ctx, float *params, float *adam_m,
                                    float *adam_v, int64_t step, const float *x,
                                    const float *y, const int32_t *idx, int64_t N,
                                    float lr, float *loss, float *grad);

#ifdef __cplusplus
}
#endif

#endif /* TN_H */
