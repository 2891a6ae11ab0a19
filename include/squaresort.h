/*
 * squaresort.h -- C ABI of libsquaresort, an MI355X (gfx950) implementation
 * of SquareSort (M. Koucky, J. Matejka, "SquareSort: a cache-oblivious
 * sorting algorithm", arXiv 2407.14801).
 *
 * Problem statement followed (Section 2.1, and the memory model of Section
 * 1.2): sort the n items of array A into a distinct array D of n cells; A may
 * be permuted on the way; arrays are passed as a pointer to their first
 * element.  Here A is the `in` buffer (clobbered) and D the `out` buffer.
 *
 * Ownership: every buffer pointer is a DEVICE pointer owned by the caller,
 * except the offsets and seeds arrays of the batched calls (HOST arrays, read
 * before the call returns).  No call allocates memory: scratch comes from the
 * caller's workspace (squaresort_u32_noalloc: from a static array the library
 * holds per GPU).  Calls are re-entrant when they use distinct workspaces.
 *
 * Streams: every call enqueues its work on `stream` (a hipStream_t, or null
 * for the default stream).  A sort with n above the cut-off synchronises
 * `stream` once per recursion step inside the call (the host learns which
 * buckets of the step need another step), and returns after the last launch
 * was enqueued; a base-case sort (n <= cut-off) does not wait, except that
 * an array of more than 16384 keys synchronises once at its end (to report a
 * device failure word).
 *
 * Order: unsigned ascending.  Key/value sorts are stable: the output is
 * ordered by (key, original index).
 *
 * Errors are returned as sqs_status codes; nothing is thrown across the ABI.
 * On any error the contents of `out` (and of `in`) are unspecified.
 */
#ifndef SQUARESORT_H
#define SQUARESORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SQS_OK = 0,
    SQS_ERR_ARG = -1,          /* null pointer with n > 0, bad cut-off, bad kind, a flag
                                  the entry point does not take                        */
    SQS_ERR_ALIAS = -2,        /* in and out (or value / bucket arrays) overlap        */
    SQS_ERR_WORKSPACE = -3,    /* workspace missing or smaller than needed; the
                                  analogue of the paper's C code failing when its
                                  pre-carved buffers run out (Appendix)              */
    SQS_ERR_DEVICE = -4,       /* a HIP launch or copy failed, a device-side bounded
                                  wait ran out, or a SQS_FLAG_VALIDATE check of the
                                  library's own result failed                         */
    SQS_ERR_PRECOND = -5,      /* a precondition of the input failed: under
                                  SQS_FLAG_ALG1_PIVOTS some node found no sample of
                                  distinct pivots in 64 draws (the input lacks
                                  distinct keys); under SQS_FLAG_COLS_SORTED with
                                  SQS_FLAG_VALIDATE a column of `in` is not sorted  */
    SQS_ERR_DEPTH = -6,        /* recursion deeper than SQS_MAX_DEPTH levels (the
                                  depth is at most n, Section 3, space bound)         */
    SQS_ERR_UNSUPPORTED = -7   /* n beyond the supported range (see sqs_max_n)        */
} sqs_status;

enum { SQS_KIND_U32 = 0, SQS_KIND_U64 = 1, SQS_KIND_KV = 2 };

enum {
    SQS_FLAG_DIGEST = 1u,      /* accumulate the recursion-tree digest into *digest    */
    /* Pivot rule of Alg. 1 as a mode, for inputs of distinct keys: each
     * node's m-1 pivots are pairwise distinct and differ from the node's
     * smallest key; a sample that is not is drawn again whole (attempt a,
     * draw t at position floor(sm64(K ^ sm64(3*2^62 | a*2^32 | t)) * n /
     * 2^64), up to 64 attempts, else SQS_ERR_PRECOND); buckets are
     * [p_{j-1}, p_j).  Without the flag pivots are drawn with replacement
     * and a run of equal pivots yields a single-value bucket (Section 2.1,
     * last paragraph). */
    SQS_FLAG_ALG1_PIVOTS = 2u,
    /* Checks, at the cost of one synchronisation at the end of the call:
     * single-instance sorts verify that the output is in key order;
     * skew_transpose_u32 verifies the bucket bounds it wrote (bs[0] = 0,
     * bs[m] = n, non-decreasing) and that every key of bucket j lies between
     * the bucket's inclusive bounds.  A failed check is SQS_ERR_DEVICE (the
     * library's result is wrong).  With SQS_FLAG_COLS_SORTED it also checks
     * that every column of `in` is sorted (SQS_ERR_PRECOND if not).  Needs a
     * workspace (>= 256 bytes) even for small n.  Not taken by the batched
     * calls (SQS_ERR_ARG). */
    SQS_FLAG_VALIDATE = 4u,
    /* skew_transpose_u32 only: the caller's columns are already sorted (the
     * state Alg. 1 reaches before SkewTranspose), so they are counted but not
     * sorted again.  Other entry points reject it (SQS_ERR_ARG). */
    SQS_FLAG_COLS_SORTED = 8u,
    /* squaresort_u32/u64/kv only: in, out (and the value arrays) are PINNED
     * HOST memory (hipHostMalloc'd: mapped into the device's address space),
     * not device memory -- the analogue of the paper's external-memory
     * experiment (Section 4.3), with host memory in the place of the file and
     * HBM holding only the per-level metadata (the workspace stays device
     * memory).  Every pass reads and writes the arrays over the host link in
     * contiguous runs; nothing of the arrays is staged in HBM.  A pointer
     * that is not pinned host memory is SQS_ERR_ARG.  Other entry points
     * reject the flag (SQS_ERR_ARG). */
    SQS_FLAG_HOST_ARRAYS = 16u
};

#define SQS_MAX_DEPTH 64

/* Tile word of sqs_params (fields of two bits; value 3 is invalid in each):
 *   SQS_TILE_COLW(v)  waves per work-group of the wave-level column kernel
 *                     (nodes of at most 1024 columns, one column per wave):
 *                     v = 0: 4, 1: 2, 2: 8 (template instances);
 *   SQS_TILE_WCAP(v)  largest bucket (or base-case segment) sorted by one
 *                     wave: 1024 >> v keys; larger ones go to the 4-wave
 *                     work-group kernel;
 *   SQS_TILE_M4CAP(v) largest bucket sorted by one 4-wave work-group:
 *                     4096 >> v keys; larger ones go to the 16-wave kernel
 *                     (up to 16384 keys). */
#define SQS_TILE_COLW(v)  ((uint32_t)(v) & 3u)
#define SQS_TILE_WCAP(v)  (((uint32_t)(v) & 3u) << 2)
#define SQS_TILE_M4CAP(v) (((uint32_t)(v) & 3u) << 4)
#define SQS_TILE_MASK     0x3Fu

/* Parameters shared by every entry point.
 *   cutoff          in/out.  Base case iff a (sub)array has n <= cutoff keys
 *                   (Alg. 1 first step; the paper's cut-off experiment,
 *                   Section 4.2, varies it).  0 selects the automatic value
 *                   (the largest array one work-group sorts) and is replaced
 *                   by it on return.  Must be 4 <= cutoff <=
 *                   sqs_max_cutoff(kind) otherwise; SQS_ERR_ARG if not.  (4
 *                   keeps every bucket that is not single-valued smaller than
 *                   its node, so the recursion ends.)
 *   flags           SQS_FLAG_* above.
 *   tile            tile shapes (0 = the library's defaults), SQS_TILE_*
 *                   below; any value gives the same output and recursion
 *                   tree, only the time changes (an autotuner picks it with
 *                   the cut-off, as the paper's cut-off experiment of
 *                   Section 4.2 picks C).  Unknown bits or values: SQS_ERR_ARG.
 *   workspace       device scratch of workspace_bytes bytes, at least
 *                   squaresort_workspace_bytes(n, kind, cutoff) (or the
 *                   batched query): the per-level arrays the paper allocates
 *                   on its call stack (Section 1.2), O(n) in total (Section 3,
 *                   space bound).  Its contents need not be initialised and
 *                   are unspecified afterwards.
 *   digest          device pointer to one uint64; with SQS_FLAG_DIGEST the
 *                   call ADDS (mod 2^64) the digest of its recursion tree:
 *                   the sum over internal nodes of sm64(K ^ H), where K is the
 *                   node's generator key and H = sum_r sm64(x_r ^ sm64(r)) over
 *                   the node's array right after its SkewTranspose (x_r is the
 *                   key, or key ^ sm64(value) for key/value sorts; sm64 is the
 *                   first SplitMix64 output from a given state).  The caller
 *                   zeroes it first.
 */
typedef struct sqs_params {
    uint64_t cutoff;
    uint32_t flags;
    uint32_t tile;
    void *workspace;
    uint64_t workspace_bytes;
    uint64_t *digest;
} sqs_params;

/* Largest automatic / allowed cut-off and largest n for a kind (0 for an
 * unknown kind). */
uint64_t sqs_max_cutoff(int kind);
uint64_t sqs_max_n(int kind);

/* Bytes of workspace an n-element sort of `kind` at `cutoff` (0 = auto)
 * needs: the O(n) scratch of the space bound (Section 3), which the paper's
 * C code passes as pre-carved buffers (Appendix).  Returns 0 for an unknown
 * kind.  (It takes the cut-off rather than a whole sqs_params block: nothing
 * else in the block changes the size.) */
uint64_t squaresort_workspace_bytes(uint64_t n, int kind, uint64_t cutoff);

/* SquareSort (Alg. 1, Section 2.1) of n uint32 keys: in (n keys, clobbered)
 * -> out (n keys, sorted).  in and out must not overlap.  seed selects the
 * pivot draws (the root generator key is sm64(seed)); the output does not
 * depend on it, the recursion tree does.  Errors: SQS_ERR_ARG,
 * SQS_ERR_ALIAS, SQS_ERR_WORKSPACE (n > 16384 without enough workspace),
 * SQS_ERR_UNSUPPORTED (n > sqs_max_n), SQS_ERR_DEVICE, SQS_ERR_DEPTH. */
int squaresort_u32(uint64_t n, uint32_t *in, uint32_t *out, uint64_t seed,
                   sqs_params *params, void *stream);

/* SquareSort (Alg. 1) of n uint64 keys; same contract as squaresort_u32. */
int squaresort_u64(uint64_t n, uint64_t *in, uint64_t *out, uint64_t seed,
                   sqs_params *params, void *stream);

/* Key/value SquareSort (Alg. 1): keys_in/vals_in (both clobbered, n each) ->
 * keys_out/vals_out, ordered by (key, original index).  The paper assumes
 * distinct keys (Section 2.1); equal keys keep their input order because
 * every base-case sort and every SkewTranspose is stable.  n < 2^32; no two
 * of the four arrays may overlap.  Errors as squaresort_u32. */
int squaresort_kv(uint64_t n, uint64_t *keys_in, uint32_t *vals_in,
                  uint64_t *keys_out, uint32_t *vals_out, uint64_t seed,
                  sqs_params *params, void *stream);

/* The root step of SquareSort up to and including SkewTranspose (Alg. 1
 * with Alg. 2, Section 2.2): views in as m = ceil(sqrt(n)) columns, sorts
 * each column in place (so `in` is clobbered; skipped under
 * SQS_FLAG_COLS_SORTED), draws the m-1 pivots from the ORIGINAL input at the
 * root generator key of `seed`, and writes the skew-transposed array to out:
 * bucket j occupies [bucket_start[j], bucket_start[j+1]) and holds, column
 * by column, the keys of that column that fall in bucket j, in sorted order.
 * bucket_start (device, m+1 uint64, nullable) receives the bucket bounds.
 * out equals SquareSort's array A right after the root's SkewTranspose at
 * the same seed, so this call is also the root dump of a sort.  Requires
 * 2 <= n <= 2^28 (n < 2: SQS_ERR_ARG; above: SQS_ERR_UNSUPPORTED).  cutoff
 * only sizes the column sorts (columns are always sorted completely).
 * Synchronises `stream` once. */
int skew_transpose_u32(uint64_t n, uint32_t *in, uint32_t *out, uint64_t *bucket_start,
                       uint64_t seed, sqs_params *params, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sort as squaresort_u32, with its scratch in a library-owned static device
 * array of SQS_STATIC_SCRATCH_BYTES bytes on each GPU (held until the
 * process ends) instead of the caller's workspace.  The call itself
 * allocates nothing.  params may be null; its workspace fields are ignored;
 * cutoff, SQS_FLAG_DIGEST (with digest), SQS_FLAG_ALG1_PIVOTS and
 * SQS_FLAG_VALIDATE work as in squaresort_u32.  The scratch of the CURRENT
 * device is used and a non-null stream must belong to that device
 * (SQS_ERR_ARG otherwise).  A size whose scratch need,
 * squaresort_workspace_bytes(n, SQS_KIND_U32, cutoff), exceeds
 * SQS_STATIC_SCRATCH_BYTES returns SQS_ERR_WORKSPACE before any work (at the
 * automatic cut-off every n <= 2^24 fits).  All calls on one GPU share its
 * array and every call rewrites what it needs, so calls that overlap on one
 * GPU (two host threads, or two streams without ordering between them)
 * race: the caller must order them.  Other errors as squaresort_u32. */
#define SQS_STATIC_SCRATCH_BYTES (32ull << 20)
int squaresort_u32_noalloc(uint64_t n, uint32_t *in, uint32_t *out, uint64_t seed,
                           sqs_params *params, void *stream);

/* Batched form: many independent SquareSorts (Alg. 1 on each instance) in
 * one launch sequence.  `count` independent uint32 instances packed back to
 * back in in/out: instance i is [offsets[i], offsets[i+1]) (offsets: HOST
 * array of count+1 entries, offsets[0] = 0, non-decreasing; total
 * offsets[count] < 2^32; each instance <= sqs_max_n(SQS_KIND_U32)).  seeds:
 * HOST array of count seeds.  Instance i ends exactly as squaresort_u32
 * would leave it on that range alone with seeds[i] and the same cut-off
 * (same output, same recursion tree); with SQS_FLAG_DIGEST the call adds the
 * sum of the instances' digests.  All instances share one launch sequence:
 * base-case instances go straight to the base-case kernels, the others are
 * the root nodes of one shared first recursion step.  Errors: SQS_ERR_ARG
 * for bad offsets/seeds/pointers or single-instance flags,
 * SQS_ERR_UNSUPPORTED for sizes past the limits, SQS_ERR_ALIAS,
 * SQS_ERR_WORKSPACE below squaresort_batched_workspace_bytes. */
uint64_t squaresort_batched_workspace_bytes(uint32_t count, const uint64_t *offsets, int kind,
                                            uint64_t cutoff);
int squaresort_batched_u32(uint32_t count, const uint64_t *offsets, uint32_t *in, uint32_t *out,
                           const uint64_t *seeds, sqs_params *params, void *stream);

/* Batched key/value form: the same contract as squaresort_batched_u32 for
 * (uint64 key, uint32 value) instances, each ordered by (key, original index
 * within its instance) exactly as squaresort_kv leaves it.  kind for the
 * workspace query: SQS_KIND_KV. */
int squaresort_batched_kv(uint32_t count, const uint64_t *offsets, uint64_t *keys_in, uint32_t *vals_in,
                          uint64_t *keys_out, uint32_t *vals_out, const uint64_t *seeds,
                          sqs_params *params, void *stream);

/* Batched form as a planned graph (the batched form of the survey's build
 * plan: many instances in one launch sequence, captured once and replayed;
 * the cut-off experiment of Section 4.2 is the precedent for choosing the
 * cut-off ahead of the data).  Planning takes the arguments of
 * squaresort_batched_u32 plus a device status word, does the host-side work
 * of the call once (the plan of every recursion step that depends only on
 * the instance sizes, uploaded synchronously into the workspace), and
 * captures the call's launches into a HIP graph; sqs_plan_launch replays
 * that graph on `stream` (asynchronously, no host work, no allocation),
 * sorting whatever the instances of `in` hold at that time into `out` -- the
 * buffers, sizes, seeds, cut-off, workspace, digest and status pointers are
 * bound at planning time.  A replay never waits for the device: the
 * internal buckets of every recursion step are finished on chip with their
 * subtrees (buckets of at most 4096 keys whose columns are base cases); a
 * bucket beyond that sets bit 1 of *status (SQS_STATUS_UNFINISHED: `out`
 * is then incomplete, the call that does so needs squaresort_batched_u32),
 * a device failure sets bit 2 (SQS_STATUS_DEVICE).  Every replay clears
 * *status first; with SQS_FLAG_DIGEST (the only flag taken) every replay
 * ADDS its digest.  The workspace (at least
 * squaresort_batched_graph_workspace_bytes) belongs to the plan until it is
 * destroyed.  Instances up to 2^28 keys.  Replays of one plan must not
 * overlap.  Planning allocates host-side objects (a stream, the graph);
 * errors as squaresort_batched_u32, plus SQS_ERR_ARG for a null status or
 * plan pointer. */
typedef struct sqs_plan sqs_plan;
enum { SQS_STATUS_UNFINISHED = 1u, SQS_STATUS_DEVICE = 2u };
uint64_t squaresort_batched_graph_workspace_bytes(uint32_t count, const uint64_t *offsets, uint64_t cutoff);
int squaresort_batched_graph_u32(uint32_t count, const uint64_t *offsets, uint32_t *in, uint32_t *out,
                                 const uint64_t *seeds, sqs_params *params, uint32_t *status, sqs_plan **plan);
int sqs_plan_launch(sqs_plan *plan, void *stream);
int sqs_plan_destroy(sqs_plan *plan);

/* Measurement support (not part of the sort): while enabled, every launch is
 * bracketed by HIP events on its stream and the elapsed times are summed per
 * kernel.  sqs_timing_enable clears the table.  sqs_timing_report writes a
 * JSON object {"kernel": [total_ms, launches, units], ...} into buf
 * (truncated to len-1 bytes, NUL-terminated) and returns the full length;
 * units counts the keys the launches processed (pivots for the pivot
 * kernels, buckets for the scans). */
int sqs_timing_enable(int on);
int64_t sqs_timing_report(char *buf, uint64_t len);

/* Human-readable name of a status code (a static string). */
const char *sqs_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif
