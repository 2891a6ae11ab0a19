/*
 * squaresort.h -- C ABI of libsquaresort, an MI355X (gfx950) implementation
 * of SquareSort (M. Koucky, J. Matejka, "SquareSort: a cache-oblivious
 * sorting algorithm", arXiv 2407.14801).
 *
 * Problem statement followed (Section 2.1): sort the n items of array A into
 * a distinct array D of n cells; A may be permuted on the way.  Here A is the
 * `in` buffer (clobbered) and D the `out` buffer.
 *
 * All buffer pointers are DEVICE pointers owned by the caller.  Every call is
 * asynchronous on `stream` except where the recursion needs the bucket sizes
 * of a level on the host (the call then synchronises `stream` internally and
 * returns after the last launch was enqueued).  Calls are re-entrant when
 * they use distinct workspaces.  No call allocates memory.
 *
 * Order: unsigned ascending.  Key/value sorts are stable: the output is
 * ordered by (key, original index).
 *
 * Errors are returned as sqs_status codes; nothing is thrown across the ABI.
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
    SQS_ERR_ARG = -1,          /* null pointer with n > 0, bad cut-off, bad kind      */
    SQS_ERR_ALIAS = -2,        /* in and out overlap                                   */
    SQS_ERR_WORKSPACE = -3,    /* workspace missing or smaller than needed            */
    SQS_ERR_DEVICE = -4,       /* a HIP launch or copy failed                         */
    SQS_ERR_PRECOND = -5,      /* SQS_FLAG_ALG1_PIVOTS: some node found no sample of
                                  distinct pivots in 64 draws (the input lacks
                                  distinct keys); the output is undefined          */
    SQS_ERR_DEPTH = -6,        /* recursion deeper than SQS_MAX_DEPTH levels          */
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
     * and a run of equal pivots yields a single-value bucket. */
    SQS_FLAG_ALG1_PIVOTS = 2u
};

#define SQS_MAX_DEPTH 64

/* Parameters shared by every entry point.
 *   cutoff          in/out.  Base case iff a (sub)array has n <= cutoff keys
 *                   (Alg. 1 first step).  0 selects the automatic value (the
 *                   largest array one work-group sorts in LDS) and is
 *                   replaced by it on return.  Must be 4 <= cutoff <=
 *                   sqs_max_cutoff(kind) otherwise; SQS_ERR_ARG if not.
 *   flags           SQS_FLAG_DIGEST.
 *   workspace       device scratch of workspace_bytes bytes, at least
 *                   squaresort_workspace_bytes(n, kind, cutoff).
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
    uint32_t reserved;
    void *workspace;
    uint64_t workspace_bytes;
    uint64_t *digest;
} sqs_params;

/* Largest automatic / allowed cut-off and largest n for a kind. */
uint64_t sqs_max_cutoff(int kind);
uint64_t sqs_max_n(int kind);

/* Bytes of workspace an n-element sort of `kind` at `cutoff` (0 = auto) needs. */
uint64_t squaresort_workspace_bytes(uint64_t n, int kind, uint64_t cutoff);

/* SquareSort (Alg. 1) of n uint32 keys: in (n keys, clobbered) -> out (n keys,
 * sorted).  seed selects the pivot draws; the output does not depend on it. */
int squaresort_u32(uint64_t n, uint32_t *in, uint32_t *out, uint64_t seed,
                   sqs_params *params, void *stream);

/* SquareSort of n uint64 keys; same contract as squaresort_u32. */
int squaresort_u64(uint64_t n, uint64_t *in, uint64_t *out, uint64_t seed,
                   sqs_params *params, void *stream);

/* Key/value SquareSort: keys_in/vals_in (both clobbered) -> keys_out/vals_out,
 * ordered by (key, original index).  n < 2^32. */
int squaresort_kv(uint64_t n, uint64_t *keys_in, uint32_t *vals_in,
                  uint64_t *keys_out, uint32_t *vals_out, uint64_t seed,
                  sqs_params *params, void *stream);

/* The root step of SquareSort up to and including SkewTranspose (Alg. 1 with
 * Alg. 2): views in as m = ceil(sqrt(n)) columns, sorts each column (in place,
 * so `in` is clobbered), draws the m-1 pivots from the ORIGINAL input at the
 * root generator key of `seed`, and writes the skew-transposed array to out:
 * bucket j occupies [bucket_start[j], bucket_start[j+1]) and holds, column by
 * column, the keys of that column that fall in bucket j, in sorted order.
 * bucket_start (device, m+1 uint64, nullable) receives the bucket bounds.
 * out equals SquareSort's array A right after the root's SkewTranspose at the
 * same seed.  Requires n >= 2 (n < 2: SQS_ERR_ARG).  cutoff only sizes the
 * column sorts (columns are always sorted completely). */
int skew_transpose_u32(uint64_t n, uint32_t *in, uint32_t *out, uint64_t *bucket_start,
                       uint64_t seed, sqs_params *params, void *stream);

/* Batched form: many independent instances in one launch sequence.
 * `count` independent uint32 instances packed back to back in
 * in/out: instance i is [offsets[i], offsets[i+1]) (offsets: HOST array of
 * count+1 entries, offsets[0] = 0, non-decreasing; total offsets[count] <
 * 2^32; each instance <= sqs_max_n(SQS_KIND_U32)).  seeds: HOST array of
 * count seeds.  Instance i ends exactly as squaresort_u32 would leave it on
 * that range alone with seeds[i] and the same cut-off (same output, same
 * recursion tree); with SQS_FLAG_DIGEST the call adds the sum of the
 * instances' digests.  All instances share one launch sequence: base-case
 * instances go straight to the base-case kernels, the others are the root
 * nodes of one shared first recursion step.  Errors: SQS_ERR_ARG for bad
 * offsets/seeds/pointers, SQS_ERR_UNSUPPORTED for sizes past the limits,
 * SQS_ERR_ALIAS, SQS_ERR_WORKSPACE below squaresort_batched_workspace_bytes. */
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

/* Measurement support (not part of the sort): while enabled, every launch is
 * bracketed by HIP events on its stream and the elapsed times are summed per
 * kernel.  sqs_timing_enable clears the table.  sqs_timing_report writes a
 * JSON object {"kernel": [total_ms, launches, units], ...} into buf
 * (truncated to len-1 bytes, NUL-terminated) and returns the full length;
 * units counts the keys the launches processed (pivots for the pivot
 * kernels, buckets for the scans). */
int sqs_timing_enable(int on);
int64_t sqs_timing_report(char *buf, uint64_t len);

/* Human-readable name of a status code. */
const char *sqs_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif
