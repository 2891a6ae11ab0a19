/*
 * squaresort_oracle.h -- plain, slow, single-threaded CPU oracle of SquareSort
 * (Koucky & Matejka, "SquareSort: a cache-oblivious sorting algorithm",
 * arXiv 2407.14801).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path
 * (libsquaresort) never calls it, shares no code with it, and includes no
 * header from this directory.
 *
 * Elements are held as structure-of-arrays: a 64-bit key array and an
 * optional 32-bit value array.  u32 keys are widened to u64 by the wrappers
 * (an order-preserving embedding).  Order is unsigned ascending by key;
 * every leaf sort is stable, so key/value output is ordered by
 * (key, original index).
 *
 * Conventions where the paper leaves a choice (each is listed, with the
 * passage it reads, in the design notes of the repository):
 *   - m = ceil(sqrt(n)) by exact integer square root (Alg. 1).
 *   - column i = [min(i*m,n), min((i+1)*m,n)), i = 0..m-1 (Alg. 1).
 *   - m-1 pivot samples drawn with replacement from the node INPUT, at
 *     positions given by a counter-based generator built on SplitMix64
 *     (Section 2.1 allows repeated samples in its C code; Alg. 1 samples
 *     the same multiset after the column sort).
 *   - bucket j holds the keys x with bucket(x) = j, where
 *       bucket(x) = #{t : s_t < x} + #{t : s_t = x and strict_t},
 *     strict_t = (t <= m-3 and s_t = s_{t+1}).  For distinct pivots this is
 *     the "<= pivot" rule of Alg. 3; a run of equal pivots yields a single
 *     value bucket at the end of the run (Section 2.1, last paragraph).
 *   - a non-empty bucket that admits exactly one key value is copied, not
 *     recursed into (Section 2.1, last paragraph).
 *   - base case: n <= C (cut-off C >= 4) sorts directly (Alg. 1 first step).
 *
 * A second pivot rule follows Alg. 1 literally (for inputs of distinct
 * keys): m-1 pivots that are pairwise distinct and differ from the node's
 * minimum, a failing sample redrawn whole, buckets [p_{j-1}, p_j).  Its
 * draws use their own counter range (orc_draw_pos_alg1).
 *
 * Status codes: 0 ok, -1 bad argument (C < 4, null pointer with n > 0),
 * -2 out of memory, -4 the Alg. 1 rule found no valid sample in
 * ORC_ALG1_ATTEMPTS draws (the input lacks distinct keys).
 */
#ifndef SQUARESORT_ORACLE_H
#define SQUARESORT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- counter-based generator (SplitMix64, Steele/Lea/Flood 2014) ---- */
uint64_t orc_sm64(uint64_t state);                 /* first SplitMix64 output from `state` */
uint64_t orc_root_key(uint64_t seed);              /* sm64(seed)                           */
uint64_t orc_child_key(uint64_t K, uint32_t phase, uint64_t i); /* phase 0 column, 1 bucket */
uint64_t orc_draw_pos(uint64_t K, uint64_t t, uint64_t n);      /* floor(draw * n / 2^64)   */
/* draw t of attempt a under the Alg. 1 rule: counter 3*2^62 | a*2^32 | t   */
uint64_t orc_draw_pos_alg1(uint64_t K, uint64_t a, uint64_t t, uint64_t n);

enum { ORC_RULE_REPLACEMENT = 0, ORC_RULE_ALG1 = 1 };
#define ORC_ALG1_ATTEMPTS 64
uint64_t orc_ceil_isqrt(uint64_t n);

/* ---- full SquareSort (Alg. 1).  A is clobbered; D receives the sorted
 * output.  vals_a / vals_d may be NULL (keys only).  digest (nullable)
 * receives the order-independent tree digest:  sum over internal nodes of
 * sm64(K_node ^ H_node), H_node = sum_r sm64(x_r ^ sm64(r)) over the node's
 * array right after its SkewTranspose, x_r = key_r (keys only) or
 * key_r ^ sm64(val_r) (key/value).  nodes (nullable) receives the number of
 * internal nodes. */
int orc_squaresort(uint64_t n, uint64_t *keys_a, uint32_t *vals_a,
                   uint64_t *keys_d, uint32_t *vals_d,
                   uint64_t seed, uint64_t cutoff,
                   uint64_t *digest, uint64_t *nodes);

int orc_squaresort_u32(uint64_t n, const uint32_t *in, uint32_t *out,
                       uint64_t seed, uint64_t cutoff, uint64_t *digest, uint64_t *nodes);
int orc_squaresort_u64(uint64_t n, const uint64_t *in, uint64_t *out,
                       uint64_t seed, uint64_t cutoff, uint64_t *digest, uint64_t *nodes);
int orc_squaresort_kv(uint64_t n, const uint64_t *keys_in, const uint32_t *vals_in,
                      uint64_t *keys_out, uint32_t *vals_out,
                      uint64_t seed, uint64_t cutoff, uint64_t *digest, uint64_t *nodes);

/* SquareSort under either pivot rule; key_max is the largest key of the key
 * type (UINT32_MAX or UINT64_MAX), used by the single-value bucket test. */
int orc_squaresort_rule(uint64_t n, uint64_t *keys_a, uint32_t *vals_a,
                        uint64_t *keys_d, uint32_t *vals_d, uint64_t seed, uint64_t cutoff,
                        uint64_t key_max, int rule, uint64_t *digest, uint64_t *nodes);

/* ---- the root node's pivots: m-1 sorted samples and strict flags ---- */
int orc_root_pivots(uint64_t n, const uint64_t *keys_in, uint64_t seed,
                    uint64_t *pivots /* m-1 */, uint8_t *strict /* m-1 */);
/* the same under the Alg. 1 rule; attempts (nullable) receives the number
 * of samples drawn (1 = the first was valid) */
int orc_root_pivots_alg1(uint64_t n, const uint64_t *keys_in, uint64_t seed,
                         uint64_t *pivots, uint8_t *strict, uint64_t *attempts);

/* bucket index of key x against sorted pivots s[0..npiv) with strict flags */
uint64_t orc_bucket_of(uint64_t x, const uint64_t *s, const uint8_t *strict, uint64_t npiv);

/* ---- SkewTranspose with explicit pivots (Section 2.2).
 * src holds m columns of the node (column i = [min(i*m,n), min((i+1)*m,n)),
 * each sorted); pivots s[0..m-1) with strict flags; +inf closes the last
 * bucket.  Writes dst and bucket_start[0..m] (bucket j = [bs[j], bs[j+1])).
 * threshold = 0 writes the layout out from its definition (what SquareSort
 * uses); threshold >= 2 runs the recursive quarter schedule of Alg. 2 (its
 * blocks below `threshold` columns or buckets moved directly) as a
 * cross-check (threshold 1 is rejected: halving one column never ends). */
int orc_skew_transpose_explicit(uint64_t n,
                                const uint64_t *src_keys, const uint32_t *src_vals,
                                uint64_t *dst_keys, uint32_t *dst_vals,
                                const uint64_t *pivots, const uint8_t *strict,
                                uint64_t *bucket_start, uint32_t threshold);

/* ---- the root intermediate: columns of `in` sorted, pivots sampled from
 * `in` at the root key of `seed`, SkewTranspose into out; bucket_start
 * (nullable) gets m+1 entries.  Equal to SquareSort's array A right after
 * the root's SkewTranspose. */
int orc_root_intermediate(uint64_t n, const uint64_t *keys_in, const uint32_t *vals_in,
                          uint64_t *keys_out, uint32_t *vals_out,
                          uint64_t *bucket_start, uint64_t seed);

/* ---- selected buckets of the root intermediate, for sizes where the
 * whole intermediate is too slow to build: for each j = sel[s], the bounds
 * [bucket_start[j], bucket_start[j+1]) into sel_bounds[2s], sel_bounds[2s+1]
 * and, if sel_keys_out is not NULL, the bucket's keys back to back in the
 * SkewTranspose layout (column by column, sorted within a column). */
int orc_root_buckets(uint64_t n, const uint64_t *keys_in, uint64_t seed,
                     uint64_t nsel, const uint64_t *sel, uint64_t *sel_bounds,
                     uint64_t *sel_keys_out);

/* ---- recursion-tree statistics (for the tree-shape checks): for each
 * depth d < max_depth, the number of internal nodes and the sum of their
 * sizes; returns the depth reached via *depth. */
int orc_tree_stats(uint64_t n, const uint64_t *keys_in, uint64_t seed, uint64_t cutoff,
                   uint64_t max_depth, uint64_t *node_count, uint64_t *size_sum,
                   uint64_t *depth);
int orc_tree_stats_rule(uint64_t n, const uint64_t *keys_in, uint64_t seed, uint64_t cutoff,
                        int rule, uint64_t max_depth, uint64_t *node_count, uint64_t *size_sum,
                        uint64_t *depth);

/* ---- threads for the children of a root node (SquareSort, tree
 * statistics) and for the column sorts of orc_root_intermediate; 1 (the
 * default) runs everything on the calling thread.  The output and the
 * digest do not depend on it. */
void orc_set_threads(uint32_t threads);

/* ---- a plain stable merge sort by key (the base case "simple_sort") ---- */
int orc_stable_sort(uint64_t n, uint64_t *keys, uint32_t *vals);

#ifdef __cplusplus
}
#endif
#endif
