/*
 * squaresort_oracle.c -- plain CPU oracle of SquareSort (arXiv 2407.14801).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  Written for
 * readability, not speed: SquareSort takes the steps of Alg. 1 in the
 * paper's order; SkewTranspose is written out from the layout it defines
 * (Section 2.2), with the recursive schedule of Alg. 2 kept as a separate
 * cross-check; the conventions are stated in squaresort_oracle.h.  No
 * blocking, no fusion.  The children of a root node may run on several
 * threads (orc_set_threads); they share no memory and draw from their own
 * generator keys, so the bytes are the same as on one thread.
 */
#include "squaresort_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Counter-based generator.  SplitMix64 (Steele, Lea, Flood, OOPSLA 2014):
 * the state advances by the golden gamma and the output is the variant-13
 * finaliser.  orc_sm64(x) is the first output of a generator whose state
 * is x.  The paper draws pivots with the C library's rand() (appendix);
 * a counter-based draw keyed by the node gives the same distribution and
 * does not depend on the order in which nodes run.                       */
uint64_t orc_sm64(uint64_t state)
{
    uint64_t z = state + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t orc_root_key(uint64_t seed) { return orc_sm64(seed); }

uint64_t orc_child_key(uint64_t K, uint32_t phase, uint64_t i)
{
    return orc_sm64(K ^ orc_sm64(2 * i + phase));
}

uint64_t orc_draw_pos(uint64_t K, uint64_t t, uint64_t n)
{
    uint64_t u = orc_sm64(K ^ orc_sm64((1ull << 63) | t));
    return (uint64_t)(((unsigned __int128)u * n) >> 64);
}

/* Draw t of attempt a under the Alg. 1 pivot rule: its own counter range
 * (bits 63 and 62 set, attempt in bits 32..61), so attempts never reuse a
 * draw of the other rule or of another attempt. */
uint64_t orc_draw_pos_alg1(uint64_t K, uint64_t a, uint64_t t, uint64_t n)
{
    uint64_t c = (3ull << 62) | ((a & 0x3FFFFFFFull) << 32) | (t & 0xFFFFFFFFull);
    uint64_t u = orc_sm64(K ^ orc_sm64(c));
    return (uint64_t)(((unsigned __int128)u * n) >> 64);
}

/* m = ceil(sqrt(n)) exactly (Alg. 1, "m = ceil(sqrt n)").  Bit-by-bit
 * integer square root: no floating point decides m. */
uint64_t orc_ceil_isqrt(uint64_t n)
{
    uint64_t r = 0;
    for (int b = 31; b >= 0; --b) {
        uint64_t c = r | (1ull << b);
        if (c * c <= n) r = c;           /* c < 2^32, so c*c fits in 64 bits */
    }
    return r + (r * r < n ? 1 : 0);
}

/* ------------------------------------------------------------------ */
/* simple_sort: a stable top-down merge sort by key (the paper's base case
 * sorts small arrays directly; MergeSort is the sort it names for pivots). */
static void merge_rec(uint64_t *k, uint32_t *v, uint64_t *tk, uint32_t *tv,
                      uint64_t lo, uint64_t hi)
{
    if (hi - lo < 2) return;
    uint64_t mid = lo + (hi - lo) / 2;
    merge_rec(k, v, tk, tv, lo, mid);
    merge_rec(k, v, tk, tv, mid, hi);
    uint64_t a = lo, b = mid, o = lo;
    while (a < mid && b < hi) {
        if (k[b] < k[a]) { tk[o] = k[b]; if (v) tv[o] = v[b]; ++b; }
        else             { tk[o] = k[a]; if (v) tv[o] = v[a]; ++a; }   /* ties: left first */
        ++o;
    }
    while (a < mid) { tk[o] = k[a]; if (v) tv[o] = v[a]; ++a; ++o; }
    while (b < hi)  { tk[o] = k[b]; if (v) tv[o] = v[b]; ++b; ++o; }
    memcpy(k + lo, tk + lo, (hi - lo) * sizeof *k);
    if (v) memcpy(v + lo, tv + lo, (hi - lo) * sizeof *v);
}

int orc_stable_sort(uint64_t n, uint64_t *keys, uint32_t *vals)
{
    if (n < 2) return 0;
    uint64_t *tk = malloc(n * sizeof *tk);
    uint32_t *tv = vals ? malloc(n * sizeof *tv) : NULL;
    if (!tk || (vals && !tv)) { free(tk); free(tv); return -2; }
    merge_rec(keys, vals, tk, tv, 0, n);
    free(tk);
    free(tv);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Bucket rule.  "x goes to bucket t or earlier" is x <= s_t for a plain
 * pivot and x < s_t for a strict one (a pivot followed by an equal pivot).
 * bucket(x) counts the pivots x is NOT at-or-below. */
static int le_pivot(uint64_t x, uint64_t s, uint8_t strict)
{
    return strict ? (x < s) : (x <= s);
}

uint64_t orc_bucket_of(uint64_t x, const uint64_t *s, const uint8_t *strict, uint64_t npiv)
{
    uint64_t b = 0;
    for (uint64_t t = 0; t < npiv; ++t)          /* plain count, no search */
        if (!le_pivot(x, s[t], strict[t])) ++b;
    return b;
}

/* ------------------------------------------------------------------ */
/* SkewTranspose (Section 2.2).  Its output is fixed by the layout it
 * produces: bucket j occupies [bs[j], bs[j+1]) and holds the keys of bucket
 * j of column 0, then those of column 1, and so on, each column's keys in
 * their (sorted) column order.  Since the columns are contiguous and sorted,
 * that is the stable partition of the node array by bucket index, written
 * out here as: bucket starts from the bucket sizes, then every key of every
 * column, in order, to the next free slot of its bucket.                  */

/* bucket index of x: the number of pivots x is not at-or-below.  The
 * predicate "x at-or-below pivot t" is monotone in t for sorted pivots with
 * strict runs, so a binary search finds the first pivot x is at-or-below. */
static uint64_t bucket_search(uint64_t x, const uint64_t *piv, const uint8_t *strict, uint64_t npiv)
{
    uint64_t lo = 0, hi = npiv;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (le_pivot(x, piv[mid], strict[mid])) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* bucket sizes, then bucket starts: an exclusive prefix sum (the bucket
 * positions of Section 2.2).  bs has m+1 entries, bs[m] = n.              */
static void bucket_positions(uint64_t n, const uint64_t *keys, const uint64_t *piv,
                             const uint8_t *strict, uint64_t m, uint64_t *bs)
{
    memset(bs, 0, (m + 1) * sizeof *bs);
    for (uint64_t r = 0; r < n; ++r) bs[bucket_search(keys[r], piv, strict, m - 1) + 1]++;
    for (uint64_t j = 1; j <= m; ++j) bs[j] += bs[j - 1];
}

/* The bucket of every key of the node array, column by column.  A column
 * is sorted and so are the pivots, so one merge-like scan of the column
 * against the pivots gives its keys' buckets in order (the counting scan of
 * Section 2.1): the bucket index only moves forward.                      */
static void column_buckets(uint64_t n, uint64_t m, const uint64_t *keys, const uint64_t *piv,
                           const uint8_t *strict, uint32_t *bk)
{
    for (uint64_t i = 0; i < m; ++i) {
        uint64_t lo = (i * m < n) ? i * m : n;
        uint64_t hi = ((i + 1) * m < n) ? (i + 1) * m : n;
        uint64_t b = 0;
        for (uint64_t r = lo; r < hi; ++r) {
            while (b < m - 1 && !le_pivot(keys[r], piv[b], strict[b])) ++b;
            bk[r] = (uint32_t)b;
        }
    }
}

static int skew_layout(uint64_t n, uint64_t m, const uint64_t *sk, const uint32_t *sv,
                       uint64_t *dk, uint32_t *dv, const uint64_t *piv, const uint8_t *strict,
                       uint64_t *bs)
{
    uint64_t *fill = malloc(m * sizeof *fill);
    uint32_t *bk = malloc(n * sizeof *bk);
    if (!fill || !bk) { free(fill); free(bk); return -2; }
    column_buckets(n, m, sk, piv, strict, bk);
    memset(bs, 0, (m + 1) * sizeof *bs);                 /* bucket sizes, then starts */
    for (uint64_t r = 0; r < n; ++r) bs[bk[r] + 1]++;
    for (uint64_t j = 1; j <= m; ++j) bs[j] += bs[j - 1];
    memcpy(fill, bs, m * sizeof *fill);
    for (uint64_t r = 0; r < n; ++r) {                   /* columns in order, keys in column order */
        dk[fill[bk[r]]] = sk[r];
        if (dv) dv[fill[bk[r]]] = sv[r];
        fill[bk[r]]++;
    }
    int ok = 1;                                          /* every bucket filled exactly */
    for (uint64_t j = 0; j < m; ++j) ok &= (fill[j] == bs[j + 1]);
    free(fill);
    free(bk);
    return ok ? 0 : -3;
}

/* Cross-check: the recursive schedule of Section 2.2.  The grid of
 * (column, bucket) cells is cut into quarters, visited as: first half of the
 * columns with the first half of the buckets, second half of the columns
 * with the first half of the buckets, then the same two for the second half
 * of the buckets.  So every column gives up its cells in bucket order and
 * every bucket receives its cells in column order, which is all the layout
 * needs.  A block with fewer than `threshold` columns or buckets moves its
 * cells directly, bucket by bucket, column by column.  Each column keeps a
 * read position, each bucket a write position; a cell of column c and
 * bucket b is the run of column c's remaining keys whose bucket is b (the
 * keys' buckets are precomputed once).                                    */
typedef struct {
    const uint64_t *sk; const uint32_t *sv;
    uint64_t *dk; uint32_t *dv;
    const uint64_t *bk;           /* bucket of every source key */
    uint64_t *rd, *rd_end, *wr;   /* per column read position / end, per bucket write position */
    uint64_t threshold;
} quad_ctx;

static void quad_leaf(quad_ctx *q, uint64_t c0, uint64_t c1, uint64_t b0, uint64_t b1)
{
    for (uint64_t b = b0; b < b1; ++b)
        for (uint64_t c = c0; c < c1; ++c) {
            uint64_t p = q->rd[c];
            while (p < q->rd_end[c] && q->bk[p] == b) {
                q->dk[q->wr[b]] = q->sk[p];
                if (q->dv) q->dv[q->wr[b]] = q->sv[p];
                q->wr[b]++;
                p++;
            }
            q->rd[c] = p;
        }
}

static void quad_split(quad_ctx *q, uint64_t c0, uint64_t c1, uint64_t b0, uint64_t b1)
{
    if (c1 - c0 < q->threshold || b1 - b0 < q->threshold) { quad_leaf(q, c0, c1, b0, b1); return; }
    uint64_t cm = c0 + (c1 - c0) / 2, bm = b0 + (b1 - b0) / 2;
    quad_split(q, c0, cm, b0, bm);
    quad_split(q, cm, c1, b0, bm);
    quad_split(q, c0, cm, bm, b1);
    quad_split(q, cm, c1, bm, b1);
}

static int skew_quadrants(uint64_t n, uint64_t m, const uint64_t *sk, const uint32_t *sv,
                          uint64_t *dk, uint32_t *dv, const uint64_t *piv, const uint8_t *strict,
                          uint64_t *bs, uint64_t threshold)
{
    uint64_t *bk = malloc(n * sizeof *bk), *rd = malloc(m * sizeof *rd);
    uint64_t *rd_end = malloc(m * sizeof *rd_end), *wr = malloc(m * sizeof *wr);
    int rc = -2;
    if (!bk || !rd || !rd_end || !wr) goto out;
    bucket_positions(n, sk, piv, strict, m, bs);
    for (uint64_t r = 0; r < n; ++r) bk[r] = bucket_search(sk[r], piv, strict, m - 1);
    for (uint64_t i = 0; i < m; ++i) {
        rd[i] = (i * m < n) ? i * m : n;
        rd_end[i] = ((i + 1) * m < n) ? (i + 1) * m : n;
    }
    memcpy(wr, bs, m * sizeof *wr);
    quad_ctx q = { sk, sv, dk, dv, bk, rd, rd_end, wr, threshold };
    quad_split(&q, 0, m, 0, m);
    rc = 0;                                              /* every cell moved exactly once */
    for (uint64_t j = 0; j < m; ++j) if (wr[j] != bs[j + 1]) rc = -3;
    for (uint64_t i = 0; i < m; ++i) if (rd[i] != rd_end[i]) rc = -3;
out:
    free(bk); free(rd); free(rd_end); free(wr);
    return rc;
}

static int skew_transpose_node(uint64_t n, uint64_t m,
                               const uint64_t *sk, const uint32_t *sv,
                               uint64_t *dk, uint32_t *dv,
                               const uint64_t *piv, const uint8_t *strict,
                               uint64_t *bs, uint32_t threshold)
{
    if (threshold == 0) return skew_layout(n, m, sk, sv, dk, dv, piv, strict, bs);
    return skew_quadrants(n, m, sk, sv, dk, dv, piv, strict, bs, threshold);
}

int orc_skew_transpose_explicit(uint64_t n,
                                const uint64_t *src_keys, const uint32_t *src_vals,
                                uint64_t *dst_keys, uint32_t *dst_vals,
                                const uint64_t *pivots, const uint8_t *strict,
                                uint64_t *bucket_start, uint32_t threshold)
{
    if (n < 2 || !src_keys || !dst_keys || !pivots || !strict || !bucket_start) return -1;
    if (threshold == 1) return -1;   /* halving a single column never ends */
    uint64_t m = orc_ceil_isqrt(n);
    return skew_transpose_node(n, m, src_keys, src_vals, dst_keys, dst_vals,
                               pivots, strict, bucket_start, threshold);
}

/* ------------------------------------------------------------------ */
/* Pivot selection: m-1 samples with replacement from the node input A,
 * sorted (MergeSort), strict flags on every pivot followed by an equal one.
 * The paper's Alg. 1 samples distinct pivots from D and resamples on a
 * repeat; its C code samples independently and tolerates repeats.  The
 * multiset of D equals that of A, so positions drawn uniformly from A give
 * the same distribution.                                                  */
static int choose_pivots(uint64_t K, uint64_t n, uint64_t m, const uint64_t *a_keys,
                         uint64_t *piv, uint8_t *strict)
{
    for (uint64_t t = 0; t + 1 < m; ++t) piv[t] = a_keys[orc_draw_pos(K, t, n)];
    int rc = orc_stable_sort(m - 1, piv, NULL);
    if (rc) return rc;
    for (uint64_t t = 0; t + 1 < m; ++t)
        strict[t] = (t + 2 < m && piv[t] == piv[t + 1]) ? 1 : 0;
    return 0;
}

/* The pivot rule of Alg. 1: m-1 pivots, pairwise distinct and none equal
 * to the node's minimum; a sample that breaks either condition is thrown
 * away whole and drawn again.  Buckets are [p_{j-1}, p_j): with every
 * pivot marked strict the bucket rule above counts the pivots <= x, which
 * is exactly that half-open rule (keys equal to a pivot go right).  Inputs
 * with too few distinct keys never yield such a sample; after
 * ORC_ALG1_ATTEMPTS draws the oracle gives up with -4.                    */
static int choose_pivots_alg1(uint64_t K, uint64_t n, uint64_t m, const uint64_t *a_keys,
                              uint64_t *piv, uint8_t *strict, uint64_t *attempts)
{
    uint64_t lo = a_keys[0];
    for (uint64_t r = 1; r < n; ++r) if (a_keys[r] < lo) lo = a_keys[r];
    for (uint64_t a = 0; a < ORC_ALG1_ATTEMPTS; ++a) {
        for (uint64_t t = 0; t + 1 < m; ++t) piv[t] = a_keys[orc_draw_pos_alg1(K, a, t, n)];
        int rc = orc_stable_sort(m - 1, piv, NULL);
        if (rc) return rc;
        int ok = m < 2 || piv[0] != lo;
        for (uint64_t t = 0; ok && t + 2 < m; ++t) ok = piv[t] != piv[t + 1];
        if (ok) {
            for (uint64_t t = 0; t + 1 < m; ++t) strict[t] = 1;
            if (attempts) *attempts = a + 1;
            return 0;
        }
    }
    return -4;
}

static int choose_pivots_rule(int rule, uint64_t K, uint64_t n, uint64_t m, const uint64_t *a_keys,
                              uint64_t *piv, uint8_t *strict)
{
    if (rule == ORC_RULE_ALG1) return choose_pivots_alg1(K, n, m, a_keys, piv, strict, NULL);
    return choose_pivots(K, n, m, a_keys, piv, strict);
}

int orc_root_pivots(uint64_t n, const uint64_t *keys_in, uint64_t seed,
                    uint64_t *pivots, uint8_t *strict)
{
    if (n < 2 || !keys_in || !pivots || !strict) return -1;
    uint64_t m = orc_ceil_isqrt(n);
    return choose_pivots(orc_root_key(seed), n, m, keys_in, pivots, strict);
}

int orc_root_pivots_alg1(uint64_t n, const uint64_t *keys_in, uint64_t seed,
                         uint64_t *pivots, uint8_t *strict, uint64_t *attempts)
{
    if (n < 2 || !keys_in || !pivots || !strict) return -1;
    uint64_t m = orc_ceil_isqrt(n);
    return choose_pivots_alg1(orc_root_key(seed), n, m, keys_in, pivots, strict, attempts);
}

/* A non-empty bucket j admits exactly one key value.  Inclusive bounds:
 *   upper U_j = s_j (plain) or s_j - 1 (strict); U_{m-1} = +inf;
 *   lower L_j = s_{j-1} + 1 (plain) or s_{j-1} (strict); L_0 = -inf.
 * For a non-empty bucket neither adjustment can wrap around.              */
static int single_value_bucket(uint64_t j, uint64_t m, const uint64_t *piv, const uint8_t *strict)
{
    if (j == 0 || j == m - 1) {
        /* an unbounded side admits more than one value unless pinned at
         * the type's end: L_0 = 0 so bucket 0 is single-valued iff U_0 = 0;
         * U_{m-1} = max so bucket m-1 is single-valued iff L_{m-1} = max.
         * Keys are held as u64; for u32 inputs max is 2^32-1, handled by
         * the caller through `key_max`.                                   */
        return -1;
    }
    uint64_t lo = strict[j - 1] ? piv[j - 1] : piv[j - 1] + 1;
    uint64_t hi = strict[j] ? piv[j] - 1 : piv[j];
    return lo == hi;
}

static int is_single_value(uint64_t j, uint64_t m, const uint64_t *piv, const uint8_t *strict,
                           uint64_t key_max)
{
    int r = single_value_bucket(j, m, piv, strict);
    if (r >= 0) return r;
    if (m == 1) return 0;
    if (j == 0) {                       /* [0, U_0] */
        uint64_t hi = strict[0] ? piv[0] - 1 : piv[0];
        return hi == 0;
    }
    /* j == m-1: [L_{m-1}, key_max] */
    uint64_t lo = strict[m - 2] ? piv[m - 2] : piv[m - 2] + 1;
    return lo == key_max;
}

/* ------------------------------------------------------------------ */
/* Alg. 1 SquareSort(A, D, n).                                            */
typedef struct {
    uint64_t cutoff, key_max;
    uint64_t digest, nodes;
    /* tree statistics (optional) */
    uint64_t max_depth, *node_count, *size_sum, depth_reached;
    int err;
    int rule;          /* ORC_RULE_REPLACEMENT or ORC_RULE_ALG1 */
} sqs_ctx;

/* Threads for the children of a root node (1 = everything on the calling
 * thread).  Nodes never share memory and every node's draws depend on its
 * own key only, so running the root's children concurrently yields the same
 * bytes and the same digest (a sum mod 2^64) as running them in order.    */
static unsigned orc_threads = 1;

void orc_set_threads(uint32_t threads) { orc_threads = threads ? threads : 1; }

static uint64_t elem_hash_x(uint64_t key, const uint32_t *vals, uint64_t r)
{
    return vals ? (key ^ orc_sm64(vals[r])) : key;
}

static void squaresort_rec(sqs_ctx *g, uint64_t K, uint64_t n,
                           uint64_t *ak, uint32_t *av, uint64_t *dk, uint32_t *dv,
                           uint64_t depth);

/* one child of a node: its generator key and its range [lo, lo+len) */
typedef struct { uint64_t K, lo, len; } child_task;

typedef struct {
    sqs_ctx g;                      /* this worker's own counters */
    const child_task *tasks;
    uint64_t ntasks, *next;         /* shared claim counter */
    uint64_t *ak, *dk;
    uint32_t *av, *dv;
    uint64_t depth;
} child_worker;

static void *child_worker_run(void *arg)
{
    child_worker *w = arg;
    for (;;) {
        uint64_t t = __atomic_fetch_add(w->next, 1, __ATOMIC_RELAXED);
        if (t >= w->ntasks || w->g.err) break;
        const child_task *c = &w->tasks[t];
        squaresort_rec(&w->g, c->K, c->len, w->ak + c->lo, w->av ? w->av + c->lo : NULL,
                       w->dk + c->lo, w->dv ? w->dv + c->lo : NULL, w->depth);
    }
    return NULL;
}

/* Sorts every child range A -> D: in order on this thread, or (at the
 * root, with orc_threads > 1) claimed one at a time by the threads. */
static void run_children(sqs_ctx *g, const child_task *tasks, uint64_t ntasks,
                         uint64_t *ak, uint32_t *av, uint64_t *dk, uint32_t *dv, uint64_t depth)
{
    unsigned P = (depth == 1 && orc_threads > 1 && ntasks > 1) ? orc_threads : 1;
    if (P > ntasks) P = (unsigned)ntasks;
    if (P <= 1) {
        for (uint64_t t = 0; t < ntasks && !g->err; ++t)
            squaresort_rec(g, tasks[t].K, tasks[t].len, ak + tasks[t].lo, av ? av + tasks[t].lo : NULL,
                           dk + tasks[t].lo, dv ? dv + tasks[t].lo : NULL, depth);
        return;
    }
    child_worker *w = calloc(P, sizeof *w);
    pthread_t *th = calloc(P, sizeof *th);
    uint64_t *stats = g->node_count ? calloc(2 * P * g->max_depth, sizeof *stats) : NULL;
    if (!w || !th || (g->node_count && !stats)) { free(w); free(th); free(stats); g->err = -2; return; }
    uint64_t next = 0;
    unsigned started = 0;
    for (unsigned p = 0; p < P; ++p) {
        w[p].g = *g;
        w[p].g.digest = 0; w[p].g.nodes = 0; w[p].g.depth_reached = 0; w[p].g.err = 0;
        if (stats) {
            w[p].g.node_count = stats + 2 * p * g->max_depth;
            w[p].g.size_sum = stats + (2 * p + 1) * g->max_depth;
        }
        w[p].tasks = tasks; w[p].ntasks = ntasks; w[p].next = &next;
        w[p].ak = ak; w[p].av = av; w[p].dk = dk; w[p].dv = dv; w[p].depth = depth;
    }
    for (unsigned p = 1; p < P; ++p) {
        if (pthread_create(&th[p], NULL, child_worker_run, &w[p]) != 0) break;
        started = p;
    }
    child_worker_run(&w[0]);              /* the calling thread works too */
    for (unsigned p = 1; p <= started; ++p) pthread_join(th[p], NULL);
    for (unsigned p = 0; p < P; ++p) {
        g->digest += w[p].g.digest;
        g->nodes += w[p].g.nodes;
        if (w[p].g.depth_reached > g->depth_reached) g->depth_reached = w[p].g.depth_reached;
        if (w[p].g.err && !g->err) g->err = w[p].g.err;
        if (stats)
            for (uint64_t d = 0; d < g->max_depth; ++d) {
                g->node_count[d] += w[p].g.node_count[d];
                g->size_sum[d] += w[p].g.size_sum[d];
            }
    }
    free(w); free(th); free(stats);
}

static void squaresort_rec(sqs_ctx *g, uint64_t K, uint64_t n,
                           uint64_t *ak, uint32_t *av, uint64_t *dk, uint32_t *dv,
                           uint64_t depth)
{
    if (g->err) return;
    if (n <= g->cutoff) {                       /* base case: sort small arrays directly */
        memcpy(dk, ak, n * sizeof *dk);
        if (dv) memcpy(dv, av, n * sizeof *dv);
        int rc = orc_stable_sort(n, dk, dv);
        if (rc) g->err = rc;
        return;
    }
    if (depth + 1 > g->depth_reached) g->depth_reached = depth + 1;
    if (g->node_count && depth < g->max_depth) {
        g->node_count[depth]++;
        g->size_sum[depth] += n;
    }
    uint64_t m = orc_ceil_isqrt(n);
    uint64_t *piv = malloc((m - 1) * sizeof *piv);
    uint8_t *strict = malloc(m - 1);
    uint64_t *bs = malloc((m + 1) * sizeof *bs);
    child_task *tasks = malloc(m * sizeof *tasks);
    uint64_t nt = 0;
    if (!piv || !strict || !bs || !tasks) { g->err = -2; goto out; }

    /* pivots come from the node input before the column children clobber it */
    int rc = choose_pivots_rule(g->rule, K, n, m, ak, piv, strict);
    if (rc) { g->err = rc; goto out; }

    /* sort each column of A into the same position of D */
    for (uint64_t i = 0; i < m; ++i) {
        uint64_t lo = (i * m < n) ? i * m : n;
        uint64_t hi = ((i + 1) * m < n) ? (i + 1) * m : n;
        if (hi > lo) tasks[nt++] = (child_task){ orc_child_key(K, 0, i), lo, hi - lo };
    }
    run_children(g, tasks, nt, ak, av, dk, dv, depth + 1);
    if (g->err) goto out;

    /* bucket positions, then SkewTranspose D -> A */
    rc = skew_transpose_node(n, m, dk, dv, ak, av, piv, strict, bs, 0);
    if (rc) { g->err = rc; goto out; }

    /* digest of this node's post-transpose array */
    {
        uint64_t H = 0;
        for (uint64_t r = 0; r < n; ++r) H += orc_sm64(elem_hash_x(ak[r], av, r) ^ orc_sm64(r));
        g->digest += orc_sm64(K ^ H);
        g->nodes++;
    }

    /* sort each bucket from A into D; single-value buckets are copied */
    nt = 0;
    for (uint64_t j = 0; j < m; ++j) {
        uint64_t lo = bs[j], hi = bs[j + 1];
        if (hi == lo) continue;
        if (is_single_value(j, m, piv, strict, g->key_max)) {
            memcpy(dk + lo, ak + lo, (hi - lo) * sizeof *dk);
            if (dv) memcpy(dv + lo, av + lo, (hi - lo) * sizeof *dv);
        } else {
            tasks[nt++] = (child_task){ orc_child_key(K, 1, j), lo, hi - lo };
        }
    }
    run_children(g, tasks, nt, ak, av, dk, dv, depth + 1);
out:
    free(piv); free(strict); free(bs); free(tasks);
}

static int run_squaresort_rule(uint64_t n, uint64_t *ak, uint32_t *av, uint64_t *dk, uint32_t *dv,
                               uint64_t seed, uint64_t cutoff, uint64_t key_max, int rule,
                               uint64_t *digest, uint64_t *nodes)
{
    if (cutoff < 4 || (rule != ORC_RULE_REPLACEMENT && rule != ORC_RULE_ALG1)) return -1;
    if (n > 0 && (!ak || !dk)) return -1;
    sqs_ctx g = { cutoff, key_max, 0, 0, 0, NULL, NULL, 0, 0, rule };
    squaresort_rec(&g, orc_root_key(seed), n, ak, av, dk, dv, 0);
    if (digest) *digest = g.digest;
    if (nodes) *nodes = g.nodes;
    return g.err;
}

static int run_squaresort(uint64_t n, uint64_t *ak, uint32_t *av, uint64_t *dk, uint32_t *dv,
                          uint64_t seed, uint64_t cutoff, uint64_t key_max,
                          uint64_t *digest, uint64_t *nodes)
{
    if (cutoff < 4) return -1;
    if (n > 0 && (!ak || !dk)) return -1;
    sqs_ctx g = { cutoff, key_max, 0, 0, 0, NULL, NULL, 0, 0, ORC_RULE_REPLACEMENT };
    squaresort_rec(&g, orc_root_key(seed), n, ak, av, dk, dv, 0);
    if (digest) *digest = g.digest;
    if (nodes) *nodes = g.nodes;
    return g.err;
}

int orc_squaresort(uint64_t n, uint64_t *keys_a, uint32_t *vals_a,
                   uint64_t *keys_d, uint32_t *vals_d,
                   uint64_t seed, uint64_t cutoff, uint64_t *digest, uint64_t *nodes)
{
    if ((vals_a == NULL) != (vals_d == NULL)) return -1;
    return run_squaresort(n, keys_a, vals_a, keys_d, vals_d, seed, cutoff, UINT64_MAX,
                          digest, nodes);
}

int orc_squaresort_rule(uint64_t n, uint64_t *keys_a, uint32_t *vals_a,
                        uint64_t *keys_d, uint32_t *vals_d, uint64_t seed, uint64_t cutoff,
                        uint64_t key_max, int rule, uint64_t *digest, uint64_t *nodes)
{
    if ((vals_a == NULL) != (vals_d == NULL)) return -1;
    return run_squaresort_rule(n, keys_a, vals_a, keys_d, vals_d, seed, cutoff, key_max, rule,
                               digest, nodes);
}

int orc_squaresort_u32(uint64_t n, const uint32_t *in, uint32_t *out,
                       uint64_t seed, uint64_t cutoff, uint64_t *digest, uint64_t *nodes)
{
    if (n > 0 && (!in || !out)) return -1;
    uint64_t *a = malloc((n ? n : 1) * sizeof *a), *d = malloc((n ? n : 1) * sizeof *d);
    if (!a || !d) { free(a); free(d); return -2; }
    for (uint64_t r = 0; r < n; ++r) a[r] = in[r];
    int rc = run_squaresort(n, a, NULL, d, NULL, seed, cutoff, UINT32_MAX, digest, nodes);
    for (uint64_t r = 0; r < n && rc == 0; ++r) out[r] = (uint32_t)d[r];
    free(a); free(d);
    return rc;
}

int orc_squaresort_u64(uint64_t n, const uint64_t *in, uint64_t *out,
                       uint64_t seed, uint64_t cutoff, uint64_t *digest, uint64_t *nodes)
{
    if (n > 0 && (!in || !out)) return -1;
    uint64_t *a = malloc((n ? n : 1) * sizeof *a);
    if (!a) return -2;
    if (n) memcpy(a, in, n * sizeof *a);
    int rc = run_squaresort(n, a, NULL, out, NULL, seed, cutoff, UINT64_MAX, digest, nodes);
    free(a);
    return rc;
}

int orc_squaresort_kv(uint64_t n, const uint64_t *keys_in, const uint32_t *vals_in,
                      uint64_t *keys_out, uint32_t *vals_out,
                      uint64_t seed, uint64_t cutoff, uint64_t *digest, uint64_t *nodes)
{
    if (n > 0 && (!keys_in || !vals_in || !keys_out || !vals_out)) return -1;
    uint64_t *ak = malloc((n ? n : 1) * sizeof *ak);
    uint32_t *av = malloc((n ? n : 1) * sizeof *av);
    if (!ak || !av) { free(ak); free(av); return -2; }
    if (n) { memcpy(ak, keys_in, n * sizeof *ak); memcpy(av, vals_in, n * sizeof *av); }
    int rc = run_squaresort(n, ak, av, keys_out, vals_out, seed, cutoff, UINT64_MAX,
                            digest, nodes);
    free(ak); free(av);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Every column of the node array sorted in place (stable): what the column
 * children leave in D.  With orc_threads > 1 the columns are shared out. */
typedef struct {
    uint64_t n, m, *next;
    uint64_t *k;
    uint32_t *v;
    int err;
} colsort_job;

static void *colsort_run(void *arg)
{
    colsort_job *j = arg;
    for (;;) {
        uint64_t i = __atomic_fetch_add(j->next, 1, __ATOMIC_RELAXED);
        if (i >= j->m) break;
        uint64_t lo = (i * j->m < j->n) ? i * j->m : j->n;
        uint64_t hi = ((i + 1) * j->m < j->n) ? (i + 1) * j->m : j->n;
        if (hi > lo) {
            int rc = orc_stable_sort(hi - lo, j->k + lo, j->v ? j->v + lo : NULL);
            if (rc) j->err = rc;
        }
    }
    return NULL;
}

static int sort_columns(uint64_t n, uint64_t m, uint64_t *k, uint32_t *v)
{
    unsigned P = orc_threads > m ? (unsigned)m : orc_threads;
    if (P < 1) P = 1;
    uint64_t next = 0;
    colsort_job *jobs = calloc(P, sizeof *jobs);
    pthread_t *th = calloc(P, sizeof *th);
    if (!jobs || !th) { free(jobs); free(th); return -2; }
    unsigned started = 0;
    for (unsigned p = 0; p < P; ++p) jobs[p] = (colsort_job){ n, m, &next, k, v, 0 };
    for (unsigned p = 1; p < P; ++p) {
        if (pthread_create(&th[p], NULL, colsort_run, &jobs[p]) != 0) break;
        started = p;
    }
    colsort_run(&jobs[0]);
    for (unsigned p = 1; p <= started; ++p) pthread_join(th[p], NULL);
    int rc = 0;
    for (unsigned p = 0; p < P; ++p) if (jobs[p].err) rc = jobs[p].err;
    free(jobs); free(th);
    return rc;
}

int orc_root_intermediate(uint64_t n, const uint64_t *keys_in, const uint32_t *vals_in,
                          uint64_t *keys_out, uint32_t *vals_out,
                          uint64_t *bucket_start, uint64_t seed)
{
    if (n < 2 || !keys_in || !keys_out) return -1;
    if ((vals_in == NULL) != (vals_out == NULL)) return -1;
    uint64_t m = orc_ceil_isqrt(n);
    uint64_t *piv = malloc((m - 1) * sizeof *piv);
    uint8_t *strict = malloc(m - 1);
    uint64_t *bs = malloc((m + 1) * sizeof *bs);
    uint64_t *dk = malloc(n * sizeof *dk);
    uint32_t *dv = vals_in ? malloc(n * sizeof *dv) : NULL;
    int rc = -2;
    if (!piv || !strict || !bs || !dk || (vals_in && !dv)) goto out;
    rc = choose_pivots(orc_root_key(seed), n, m, keys_in, piv, strict);
    if (rc) goto out;
    /* the column children leave every column of D sorted */
    memcpy(dk, keys_in, n * sizeof *dk);
    if (dv) memcpy(dv, vals_in, n * sizeof *dv);
    rc = sort_columns(n, m, dk, dv);
    if (rc) goto out;
    rc = skew_transpose_node(n, m, dk, dv, keys_out, vals_out, piv, strict, bs, 0);
    if (rc == 0 && bucket_start) memcpy(bucket_start, bs, (m + 1) * sizeof *bs);
out:
    free(piv); free(strict); free(bs); free(dk); free(dv);
    return rc;
}

int orc_tree_stats_rule(uint64_t n, const uint64_t *keys_in, uint64_t seed, uint64_t cutoff,
                        int rule, uint64_t max_depth, uint64_t *node_count, uint64_t *size_sum,
                        uint64_t *depth)
{
    if (cutoff < 4 || (n > 0 && !keys_in) || !node_count || !size_sum) return -1;
    if (rule != ORC_RULE_REPLACEMENT && rule != ORC_RULE_ALG1) return -1;
    uint64_t *a = malloc((n ? n : 1) * sizeof *a), *d = malloc((n ? n : 1) * sizeof *d);
    if (!a || !d) { free(a); free(d); return -2; }
    if (n) memcpy(a, keys_in, n * sizeof *a);
    memset(node_count, 0, max_depth * sizeof *node_count);
    memset(size_sum, 0, max_depth * sizeof *size_sum);
    sqs_ctx g = { cutoff, UINT64_MAX, 0, 0, max_depth, node_count, size_sum, 0, 0, rule };
    squaresort_rec(&g, orc_root_key(seed), n, a, NULL, d, NULL, 0);
    if (depth) *depth = g.depth_reached;
    free(a); free(d);
    return g.err;
}

int orc_tree_stats(uint64_t n, const uint64_t *keys_in, uint64_t seed, uint64_t cutoff,
                   uint64_t max_depth, uint64_t *node_count, uint64_t *size_sum,
                   uint64_t *depth)
{
    return orc_tree_stats_rule(n, keys_in, seed, cutoff, ORC_RULE_REPLACEMENT, max_depth,
                               node_count, size_sum, depth);
}

/* ------------------------------------------------------------------ */
/* Selected buckets of the root intermediate, computed one bucket set at a
 * time for sizes where the whole intermediate is too slow to build: every
 * bucket j is, column by column, the column's keys of bucket j in sorted
 * order (the SkewTranspose layout).  Writes all m+1 bucket bounds and, for
 * the nsel requested buckets (ascending), their keys back to back.        */
static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

int orc_root_buckets(uint64_t n, const uint64_t *keys_in, uint64_t seed,
                     uint64_t nsel, const uint64_t *sel, uint64_t *sel_bounds,
                     uint64_t *sel_keys_out)
{
    if (n < 2 || !keys_in || !sel || !sel_bounds) return -1;
    uint64_t m = orc_ceil_isqrt(n);
    for (uint64_t s2 = 0; s2 < nsel; ++s2) if (sel[s2] >= m) return -1;
    uint64_t *piv = malloc((m - 1) * sizeof *piv);
    uint8_t *strict = malloc(m - 1);
    int rc = -2;
    if (!piv || !strict) goto out;
    rc = choose_pivots(orc_root_key(seed), n, m, keys_in, piv, strict);
    if (rc) goto out;
    uint64_t at = 0;
    for (uint64_t s2 = 0; s2 < nsel; ++s2) {
        uint64_t j = sel[s2];
        /* x is in bucket j iff it is at-or-below pivot j (or j is the last
         * bucket) and not at-or-below pivot j-1 (or j is the first) */
        uint64_t below = 0, count = 0;
        for (uint64_t r = 0; r < n; ++r) {
            uint64_t x = keys_in[r];
            int after_prev = (j == 0) || !le_pivot(x, piv[j - 1], strict[j - 1]);
            int upto_this = (j == m - 1) || le_pivot(x, piv[j], strict[j]);
            if (!after_prev) ++below;
            else if (upto_this) ++count;
        }
        sel_bounds[2 * s2] = below;
        sel_bounds[2 * s2 + 1] = below + count;
        if (!sel_keys_out) continue;
        /* the bucket's keys, column by column, sorted within a column */
        for (uint64_t i = 0; i < m; ++i) {
            uint64_t lo = (i * m < n) ? i * m : n, hi = ((i + 1) * m < n) ? (i + 1) * m : n;
            uint64_t first = at;
            for (uint64_t r = lo; r < hi; ++r) {
                uint64_t x = keys_in[r];
                if ((j == 0 || !le_pivot(x, piv[j - 1], strict[j - 1])) &&
                    (j == m - 1 || le_pivot(x, piv[j], strict[j])))
                    sel_keys_out[at++] = x;
            }
            qsort(sel_keys_out + first, at - first, sizeof *sel_keys_out, cmp_u64);
        }
    }
    rc = 0;
out:
    free(piv); free(strict);
    return rc;
}
