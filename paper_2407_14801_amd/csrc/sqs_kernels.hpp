// sqs_kernels.hpp -- the HIP kernels of one SquareSort recursion step,
// batched over every internal node of that step (Alg. 1 of arXiv 2407.14801).
//
// A node owns the range [off, off+n) of both global arrays A (its input,
// clobbered) and D (its output).  For a batch of nodes the step runs:
//   k_sample          m-1 pivot draws per node from its input A
//   k_sort_pivots*    sort them; strict flags (pivot equal to the next one)
//   k_colsort_*       sort each column A -> D (base case) or take it sorted
//                     from deeper recursion, and count: per column i and
//                     bucket block J the keys before J; per column group g
//                     and bucket j the keys of g in j
//   k_colscan         prefix of the group counts over groups, bucket totals
//   k_bucket_start    exclusive scan of totals: bucket j = [bs[j], bs[j+1])
//   k_tile_plan       keys per SkewTranspose tile; heavy tiles' chunks listed
//   k_transpose       SkewTranspose D -> A over (column group x bucket block)
//                     tiles, staged through LDS; k_transpose_heavy takes the
//                     chunks of heavy tiles (decoupled look-back)
//   k_classify        per bucket: empty / single value / small / mid4 / mid /
//                     big / internal, with a resolved span per sorted bucket
//   k_order_lists     largest-first claim order of the mid and big spans
//   k_bucket_*        copy single-value buckets, sort small (one wave), mid4
//                     and mid (one work-group) and big (MSD splits) buckets
//                     A -> D; internal buckets form the next batch
// Columns and buckets of at most WCAP keys are sorted by one wave each; the
// block kernels handle up to their LDS capacity.  Also here: the grid-wide
// split of large base-case segments (k_base_*), the HBM count of columns
// longer than one LDS sort (k_blockoff, k_tilecount), the Alg. 1 node minima
// (k_node_min) and the tree digest (k_digest*).
#pragma once

#include "sqs_device.hpp"

namespace sqs {

// ------------------------------------------------------------ configuration
constexpr int SORT_NW = 16;                  // waves of the block-sort work-groups
constexpr int SORT_IPT = 16;                 // keys per thread
constexpr int SORT_NT = SORT_NW * WAVE;      // 1024 threads
constexpr int SORT_CAP = SORT_NT * SORT_IPT; // 16384 keys per block sort
constexpr int WR = 16;                       // rows of a wave sort
constexpr int WCAP = WR * WAVE;              // 1024 keys per wave sort
constexpr int SM_NW = 4;                     // waves of the small-segment work-groups
constexpr int M4_NW = 4;                     // waves of the mid4 bucket work-groups
constexpr uint32_t M4_CAP = M4_NW * WAVE * SORT_IPT;  // 4096 keys per mid4 sort
constexpr int TG = 64;                       // columns per column group
constexpr int TB = 64;                       // buckets per bucket block
constexpr int TR_NW = 4;                     // waves of the transpose work-group
constexpr int TR_IPT = 10;                   // keys per thread per chunk
constexpr int TR_CH = TR_NW * WAVE * TR_IPT; // 2560 keys per transpose chunk
constexpr int CL_NT = 1024;                  // threads of the classify work-group

using SortSm = SortSmem<SORT_NW, SORT_IPT>;

// ------------------------------------------------------------ batch layout
struct NodeDesc {
    uint64_t off;      // first slot of the node in A and D
    uint64_t key;      // generator key of the node
    uint32_t n, m;     // size, columns (= buckets) = ceil(sqrt(n))
    uint32_t groups;   // ceil(m / TG)
    uint32_t nJ;       // ceil(m / TB)
    uint32_t piv;      // first pivot slot (m-1 slots)
    uint32_t bkt;      // first bucket slot (m+1 slots in bs, m in tot)
    uint64_t src;      // first slot of the column/bucket-block offsets ((nJ+1)*m)
    uint64_t blk;      // first slot of the group/bucket counts (groups*m)
    uint32_t flags;    // NODE_COLS_RECURSED: columns > cut-off come sorted in D
    uint32_t sub;      // work-groups per column group (a power of two <= TG): each takes TG/sub
                       // columns; with sub > 1 they add their bucket counts into the group's
};
constexpr uint32_t NODE_COLS_RECURSED = 1u;
// m > SORT_CAP: a column does not fit one LDS sort.  Its columns are sorted
// into D before the count (by the base-case kernels or by recursion), and the
// count runs through HBM (k_blockoff, k_tilecount) instead of in LDS.
constexpr uint32_t NODE_HUGE = 2u;
// each node's pivot slot starts at a multiple of PIV_ALIGN keys and is padded
// to one, so a thread can load its PIV_ALIGN pivots with 16-byte loads
constexpr uint32_t PIV_ALIGN = 16;

struct BucketItem {
    uint32_t node, j, lo, size;   // lo: node-local first slot
};
// Bucket classes by size: copy (one key value), small (<= WCAP, a wave),
// mid4 (<= M4_CAP, a 4-wave work-group), mid (<= SORT_CAP, a 16-wave
// work-group), big (<= cut-off, MSD splits), internal (> cut-off).
enum { CLS_COPY = 0, CLS_SMALL = 1, CLS_MID4 = 2, CLS_MID = 3, CLS_BIG = 4, CLS_INTERNAL = 5, NCLS = 6 };
// device counters of a batch: NCLS list sizes, NCLS take counters, NCLS key
// totals, then a flag set when the Alg. 1 pivot rule found no valid sample
constexpr int CTR_FAIL = 3 * NCLS;
// SkewTranspose chunks of heavy tiles: item count, take counter, and a flag
// set when a chunk's wait for its predecessor ran past its bound
constexpr int CTR_TR_ITEMS = 3 * NCLS + 1;
constexpr int CTR_TR_TAKE = 3 * NCLS + 2;
constexpr int CTR_TR_FAIL = 3 * NCLS + 3;
// set when the MSD-split kernel's segment stack would overflow (it cannot:
// see k_bucket_big); the call then returns SQS_ERR_DEVICE
constexpr int CTR_BIG_FAIL = 3 * NCLS + 4;
// validation (SQS_FLAG_VALIDATE): a column given as sorted is not, and a
// bucket of the SkewTranspose output holds a key outside its bounds
constexpr int CTR_PRE_FAIL = 3 * NCLS + 5;
constexpr int CTR_CHECK_FAIL = 3 * NCLS + 6;
// the wide-bucket kernel (k_bucket_wide): its take counter over the MSD-split
// list (from the end), the keys it sorted, and the buckets it may take
constexpr int CTR_WIDE_TAKE = 3 * NCLS + 7;
constexpr int CTR_WIDE_KEYS = 3 * NCLS + 8;
constexpr int CTR_WIDE_ELIG = 3 * NCLS + 9;
constexpr int CTR_WORDS = 3 * NCLS + 10;
// sample attempts of the Alg. 1 pivot rule before a node gives up
constexpr uint32_t ALG1_ATTEMPTS = 64;
constexpr uint32_t COPY_CH = 32768;           // keys per piece of a single-value bucket copy
constexpr uint32_t CP_NT = 1024;              // threads of a copy work-group
constexpr uint32_t BIG_CAP = 16 * SORT_CAP;  // largest automatic cut-off: 262144 keys
// buckets of 32-bit keys without values above SORT_CAP and up to WIDE_CAP
// keys, with a key range of at least WIDE_RANGE values, are sorted whole in
// LDS (k_bucket_wide)
constexpr uint32_t WIDE_CAP = 28672;
constexpr uint32_t WIDE_RANGE = 16;

// A base-case sort item, resolved: its first slot in A and D, its size and
// the inclusive key bounds of its bucket (one load gives a sort kernel all
// it needs, instead of a chain of list entry, node and pivot loads).
template <class K> struct Span {
    uint64_t base;
    uint32_t size, pad;
    K lo, hi;
};

template <class K> struct Batch {
    const NodeDesc *nodes;
    uint32_t N;
    const uint32_t *pivStart;    // N+1 prefix of m-1
    const uint32_t *tileStart;   // N+1 prefix of groups*nJ
    const uint32_t *bucStart;    // N+1 prefix of m
    const uint32_t *digStart;    // N+1 prefix of digest chunks
    // nodes whose columns / pivots are handled by work-groups (m > WCAP) and
    // by waves (m <= WCAP): node index lists and their group prefixes
    const uint32_t *bigIdx, *bigGrp;
    uint32_t NB;
    const uint32_t *smlIdx, *smlGrp;
    uint32_t NS;
    K *piv;
    uint8_t *strict;
    uint32_t *srcOff;   // [J][i] per node: keys of column i in buckets < J*TB
    uint32_t *blk;      // [g][j] per node: keys of group g in bucket j (then prefix over g)
    uint32_t *bs;       // [j] per node, m+1 entries
    uint32_t *tot;      // [j] per node
    BucketItem *list[NCLS];
    uint32_t cap[NCLS];
    Span<K> *span[NCLS];           // mid4, mid, big: the items resolved (same index as the list)
    Span<K> *ord[NCLS];            // mid, big: the spans in claim order (largest first), or null
    uint32_t *ctr;      // NCLS list sizes, NCLS take counters (work-groups claim items), NCLS key totals, fail flag
    K *nmin;            // per node: smallest key of its input (Alg. 1 pivot rule)
    uint32_t alg1;      // 1: Alg. 1 pivot rule (distinct, above the minimum, resampled; [ ) buckets)
    uint32_t bigInD;    // 1: the big-list items start in D (else in A)
    uint32_t *trItem;   // heavy transpose chunks: (tile, chunk) pairs, a tile's chunks adjacent
    unsigned long long *trRec;   // per heavy chunk: TB words (status << 62 | value), see k_transpose
    uint32_t trCap;
    unsigned long long *H;
    uint32_t wcap, m4cap;   // largest bucket of the wave class and of the mid4 class (tile choice)
};

// largest k with prefix[k] <= item (prefix is non-decreasing, prefix[0] = 0)
// Claims the next item of list c for the calling work-group (all threads get
// the same index).  Items of the bucket lists differ widely in cost, so
// work-groups take them one by one instead of in a fixed stride.
__device__ inline uint32_t take_item(uint32_t *ctr, int c, uint32_t *slot)
{
    if (threadIdx.x == 0) *slot = atomicAdd(&ctr[NCLS + c], 1u);
    __syncthreads();
    const uint32_t it = *slot;
    __syncthreads();
    return it;
}

__device__ inline uint32_t find_node(const uint32_t *prefix, uint32_t N, uint32_t item)
{
    uint32_t lo = 0, hi = N - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// bucket of x among npiv sorted pivots (count of pivots x is not at-or-below)
template <class K>
__device__ inline uint32_t bucket_search(K x, const K *piv, const uint8_t *st, uint32_t npiv)
{
    uint32_t a = 0, e = npiv;
    while (a < e) {
        const uint32_t mid = (a + e) >> 1;
        if (le_pivot(x, piv[mid], st[mid] != 0)) e = mid; else a = mid + 1;
    }
    return a;
}

// ------------------------------------------------------------ utility kernels
__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------ pivots
// m-1 draws with replacement from the node's input (Alg. 1 pivot selection;
// the appendix code also draws from the input before the column sorts).
template <class K>
__global__ void k_sample(Batch<K> b, const K *A)
{
    const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= b.pivStart[b.N]) return;
    const uint32_t k = find_node(b.pivStart, b.N, item);
    const NodeDesc nd = b.nodes[k];
    const uint32_t t = item - b.pivStart[k];
    if (t >= nd.m - 1) return;                       // padding of the node's slot
    const uint32_t pos = b.alg1 ? pivot_draw_alg1(nd.key, 0, t, nd.n) : pivot_draw(nd.key, t, nd.n);
    b.piv[nd.piv + t] = A[nd.off + pos];
}

// Smallest key of every node's input (the Alg. 1 rule excludes it as a
// pivot): one block per 16384-key chunk, an atomic min per node.
template <class K>
__global__ void k_node_min(Batch<K> b, const K *A)
{
    constexpr uint32_t CHUNK = 16384;
    __shared__ K wmin[4];
    const uint32_t k = find_node(b.digStart, b.N, blockIdx.x);
    const NodeDesc nd = b.nodes[k];
    const uint32_t r0 = (blockIdx.x - b.digStart[k]) * CHUNK, r1 = min(nd.n, r0 + CHUNK);
    K mn = (K)KeyT<K>::MAXV;
    for (uint32_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) { const K x = A[nd.off + r]; mn = x < mn ? x : mn; }
    mn = wave_min(mn);
    if (lane_id() == 0) wmin[wave_id()] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t w = 1; w < blockDim.x / WAVE; ++w) mn = wmin[w] < mn ? wmin[w] : mn;
        if (sizeof(K) == 4) atomicMin(reinterpret_cast<unsigned int *>(&b.nmin[k]), (unsigned int)mn);
        else atomicMin(reinterpret_cast<unsigned long long *>(&b.nmin[k]), (unsigned long long)mn);
    }
}

// Sort the samples of one node (any correct sort; the paper uses MergeSort):
// one work-group per node with more than WCAP pivots ...
// Under the Alg. 1 rule a sorted sample with a repeated value or the node's
// minimum is drawn again whole (attempt a+1, read from the node input A) up
// to ALG1_ATTEMPTS times; every pivot is then strict ([ ) buckets).
template <class K>
__global__ __launch_bounds__(SORT_NT) void k_sort_pivots_big(Batch<K> b, const K *A)
{
    __shared__ SortSm sm;
    const uint32_t node = b.bigIdx[blockIdx.x];
    const NodeDesc nd = b.nodes[node];
    const uint32_t cnt = nd.m - 1;
    K k[SORT_IPT];
    uint32_t v[SORT_IPT];
    const int R = block_rows<SORT_NW, SORT_IPT>(cnt);
    for (uint32_t a = 0;; ++a) {
        tables_clear<SORT_NW, 256>(sm.s.tab);          // sm.k64 below reuses the tables
#pragma unroll
        for (int r = 0; r < SORT_IPT; ++r) {
            const uint32_t p = bpos(r, R);
            k[r] = (K)0;
            if (r < R && p < cnt) k[r] = a == 0 ? b.piv[nd.piv + p] : A[nd.off + pivot_draw_alg1(nd.key, a, p, nd.n)];
        }
        wait_vmem();
        __syncthreads();
        block_sort<K, false, SORT_NW, SORT_IPT>(k, v, cnt, sm);
#pragma unroll
        for (int r = 0; r < SORT_IPT; ++r) {
            const uint32_t p = bpos(r, R);
            if (r < R && p < cnt) sm.k64[p] = (uint64_t)k[r];
        }
        __syncthreads();
        if (!b.alg1) break;
        bool bad = threadIdx.x == 0 && sm.k64[0] == (uint64_t)b.nmin[node];
        for (uint32_t t = threadIdx.x; t + 1 < cnt; t += SORT_NT) bad |= sm.k64[t] == sm.k64[t + 1];
        if (!__syncthreads_or(bad)) break;
        if (a + 1 == ALG1_ATTEMPTS) {
            if (threadIdx.x == 0) atomicOr(&b.ctr[CTR_FAIL], 1u);
            break;
        }
    }
#pragma unroll
    for (int r = 0; r < SORT_IPT; ++r) {
        const uint32_t p = bpos(r, R);
        if (r < R && p < cnt) b.piv[nd.piv + p] = k[r];
    }
    for (uint32_t t = threadIdx.x; t < cnt; t += SORT_NT)
        b.strict[nd.piv + t] = b.alg1 ? 1 : ((t + 1 < cnt && sm.k64[t] == sm.k64[t + 1]) ? 1 : 0);
}

// ... and one wave per node with at most WCAP pivots.
template <class K>
__global__ __launch_bounds__(SM_NW * WAVE) void k_sort_pivots_small(Batch<K> b, const K *A)
{
    __shared__ WaveSmem<WR> wsm[SM_NW];
    const uint32_t w = wave_id(), l = lane_id();
    wave_table_clear(wsm[w].tab);
    wave_lds_sync();
    const uint32_t slot = blockIdx.x * SM_NW + w;
    if (slot >= b.NS) return;
    const uint32_t node = b.smlIdx[slot];
    const NodeDesc nd = b.nodes[node];
    const uint32_t cnt = nd.m - 1;
    K k[WR], nx[WR];
    uint32_t v[WR];
    for (uint32_t a = 0;; ++a) {
#pragma unroll
        for (int r = 0; r < WR; ++r) {
            const uint32_t p = r * WAVE + l;
            k[r] = (K)0;
            if (p < cnt) k[r] = a == 0 ? b.piv[nd.piv + p] : A[nd.off + pivot_draw_alg1(nd.key, a, p, nd.n)];
        }
        wave_sort<K, false, WR>(k, v, cnt, wsm[w]);
        // the next pivot in order (lane l+1, or lane 0 of the next row)
        bool bad = false;
#pragma unroll
        for (int r = 0; r < WR; ++r) {
            const uint32_t p = r * WAVE + l;
            nx[r] = __shfl_down(k[r], 1, WAVE);
            const K first_next = __shfl(k[r + 1 < WR ? r + 1 : r], 0, WAVE);
            if (l == WAVE - 1) nx[r] = first_next;
            bad |= p + 1 < cnt && nx[r] == k[r];
        }
        if (!b.alg1) break;
        bad |= l == 0 && cnt > 0 && k[0] == b.nmin[node];
        if (__ballot(bad) == 0) break;
        if (a + 1 == ALG1_ATTEMPTS) {
            if (l == 0) atomicOr(&b.ctr[CTR_FAIL], 1u);
            break;
        }
    }
#pragma unroll
    for (int r = 0; r < WR; ++r) {
        const uint32_t p = r * WAVE + l;
        if (p < cnt) {
            b.piv[nd.piv + p] = k[r];
            b.strict[nd.piv + p] = b.alg1 ? 1 : ((p + 1 < cnt && nx[r] == k[r]) ? 1 : 0);
        }
    }
}

// pivot q of a slice held as 16-byte words
template <class K> __device__ inline K piv_of(const uint4 *raw, int q);
template <> __device__ inline uint32_t piv_of<uint32_t>(const uint4 *raw, int q)
{
    const uint4 v = raw[q >> 2];
    return (q & 3) == 0 ? v.x : (q & 3) == 1 ? v.y : (q & 3) == 2 ? v.z : v.w;
}
template <> __device__ inline uint64_t piv_of<uint64_t>(const uint4 *raw, int q)
{
    const uint4 v = raw[q >> 1];
    return (q & 1) == 0 ? ((uint64_t)v.y << 32 | v.x) : ((uint64_t)v.w << 32 | v.z);
}

__device__ inline bool strict_of(const uint4 &raw, int q)
{
    const uint32_t w = q < 4 ? raw.x : q < 8 ? raw.y : q < 12 ? raw.z : raw.w;
    return ((w >> (8 * (q & 3))) & 255u) != 0;
}

// ------------------------------------------------------------ column phase
__device__ inline uint32_t column_len(uint32_t i, uint32_t m, uint32_t n)
{
    const uint64_t lo = (uint64_t)i * m;
    return lo < n ? (uint32_t)min((uint64_t)m, (uint64_t)n - lo) : 0u;
}

// key at position p of a sorted column held in LDS
// ------------------------------------------------------- merge column sort
// Columns of 64-bit keys of at most MergeCap::CAP keys are sorted by a stable
// merge sort in LDS (keys, and values beside them), which leaves the
// registers of the radix passes free: each thread first sorts IPT
// consecutive keys in registers (odd-even transposition: adjacent exchanges
// of strictly greater keys, so equal keys keep their order), then runs of L
// merge into runs of 2L; each thread produces IPT consecutive outputs of its
// run pair, finding where they start on the merge path (a binary search over
// the pair's diagonal) and taking the smaller head IPT times, the left
// run's head on ties (stable).  A thread's run is an odd number of keys, so
// that the lanes' accesses to their own runs (IPT 8-byte words apart) fall
// into different LDS banks.
template <bool HV> struct MergeCap {
    static constexpr int IPT = HV ? 13 : 17;             // keys per thread
    static constexpr int SLOTS = SORT_NT * IPT;
    static constexpr int CAP = SLOTS < SORT_CAP ? SLOTS : SORT_CAP;   // 13312 (with values) or 16384 keys
};
template <bool HV> struct MergeSm {
    uint64_t k[MergeCap<HV>::SLOTS];
    uint32_t v[HV ? MergeCap<HV>::SLOTS : 1];
};
// the column kernel's LDS: the sort layout, or the merge sort's arrays over it
template <bool HV, bool MG> struct ColSm {
    SortSm sort;
};
template <bool HV> struct ColSm<HV, true> {
    union {
        SortSm sort;
        MergeSm<HV> mg;
    };
};
static_assert(sizeof(ColSm<true, true>) <= 160 * 1024, "fits one CU's LDS");

// Stable sort of K[0 .. len) (and V) in place, runs of IPT keys (odd);
// len <= IPT * (threads of the work-group).
// Entry: the keys are in LDS and a barrier has passed; exit: sorted, after
// a barrier.  Positions len .. (a multiple of IPT) are padding, set here to
// the largest key: being last, they stay behind equal real keys.
template <bool HV, int IPT>
__device__ __forceinline__ void lds_merge_sort(uint64_t *K, uint32_t *V, uint32_t len)
{
    const uint32_t t = threadIdx.x;
    const uint32_t nact = (len + IPT - 1) / IPT;         // threads that hold keys
    const uint32_t lenp = nact * IPT;
    if (t < lenp - len) {                                // fewer than IPT pads
        K[len + t] = ~0ull;
        if (HV) V[len + t] = 0u;
    }
    __syncthreads();
    uint64_t k[IPT];
    uint32_t v[IPT];
    const uint32_t pos = t * IPT;
    if (t < nact) {
#pragma unroll
        for (int s = 0; s < IPT; ++s) {
            k[s] = K[pos + s];
            if (HV) v[s] = V[pos + s];
        }
#pragma unroll
        for (int rd = 0; rd < IPT; ++rd) {
#pragma unroll
            for (int s = rd & 1; s + 1 < IPT; s += 2) {
                const bool sw = k[s] > k[s + 1];
                const uint64_t a = k[s], b = k[s + 1];
                k[s] = sw ? b : a;
                k[s + 1] = sw ? a : b;
                if (HV) {
                    const uint32_t x = v[s], y = v[s + 1];
                    v[s] = sw ? y : x;
                    v[s + 1] = sw ? x : y;
                }
            }
        }
#pragma unroll
        for (int s = 0; s < IPT; ++s) {                  // own positions: no other thread reads them yet
            K[pos + s] = k[s];
            if (HV) V[pos + s] = v[s];
        }
    }
    __syncthreads();
    // Runs of at most 32 * IPT keys pair up inside one wave's 64 * IPT keys
    // (every wave's first key is a multiple of 2L), so those rounds need
    // only the wave's own LDS ordering, not a work-group barrier.
    auto sync = [&](bool local) {
        if (local) wave_lds_sync();
        else __syncthreads();
    };
#pragma unroll 1
    for (uint32_t L = IPT; L < len; L *= 2) {            // uniform over the work-group
        if (t < nact) {
            const uint32_t a0 = pos / (2 * L) * (2 * L);
            const uint32_t la = min(L, lenp - a0);
            const uint32_t b0 = a0 + la;
            const uint32_t lb = b0 < lenp ? min(L, lenp - b0) : 0u;
            const uint32_t d = pos - a0;                 // outputs of the pair before this thread's
            // merge path: i = keys of the left run among the first d outputs
            uint32_t lo = d > lb ? d - lb : 0u, hi = min(d, la);
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (K[a0 + mid] <= K[b0 + d - mid - 1]) lo = mid + 1; else hi = mid;
            }
            // the outputs one by one: the smaller head, the left run's on ties
            uint32_t i = lo, j = d - lo;
            uint64_t ka = i < la ? K[a0 + i] : 0ull;
            uint64_t kb = j < lb ? K[b0 + j] : 0ull;
#pragma unroll
            for (int s = 0; s < IPT; ++s) {
                const bool ta = i < la && (j >= lb || ka <= kb);
                k[s] = ta ? ka : kb;
                if (HV) v[s] = V[ta ? a0 + i : b0 + j];
                i += ta ? 1u : 0u;
                j += ta ? 0u : 1u;
                const bool more = ta ? i < la : j < lb;
                const uint32_t nx = min(ta ? a0 + i : b0 + j, lenp - 1u);
                const uint64_t kn = more ? K[nx] : 0ull;
                ka = ta ? kn : ka;
                kb = ta ? kb : kn;
            }
        }
        sync(L <= 32u * IPT);
        if (t < nact) {
#pragma unroll
            for (int s = 0; s < IPT; ++s) {
                K[pos + s] = k[s];
                if (HV) V[pos + s] = v[s];
            }
        }
        sync(2 * L <= 32u * IPT && 2 * L < len);        // the next round's pairs
    }
    __syncthreads();                                     // callers read any position
}

// A segment of 64-bit keys (and values) sorted by the LDS merge sort: loaded
// into LDS (k, v) from `from`, sorted, stored to `to`; size <= NT * IPT.
template <bool HV, int IPT, int NT>
__device__ __forceinline__ void merge_segment(const uint64_t *from, const uint32_t *vfrom, uint64_t *to, uint32_t *vto,
                              uint32_t size, uint64_t *k, uint32_t *v)
{
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));                      // positions recomputed here, not kept live
    uint64_t mk[IPT];
    uint32_t mv[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t p = (uint32_t)r * NT + tid;
        mk[r] = p < size ? from[p] : 0ull;
        if (HV) mv[r] = p < size ? vfrom[p] : 0u;
    }
    wait_vmem();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t p = (uint32_t)r * NT + tid;
        if (p < size) {
            k[p] = mk[r];
            if (HV) v[p] = mv[r];
        }
    }
    __syncthreads();
    lds_merge_sort<HV, IPT>(k, v, size);
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t p = (uint32_t)r * NT + tid;
        if (p < size) {
            to[p] = k[p];
            if (HV) vto[p] = v[p];
        }
    }
}

template <class K> __device__ inline K col_key(const SortSm &sm, uint32_t p)
{
    return sizeof(K) == 4 ? (K)sm.k32[p] : (K)sm.k64[p];
}

// Nodes with m > WCAP: one work-group per (node, column group).  Each column
// is sorted in LDS (base case) unless deeper recursion already sorted it;
// then every pivot finds, by a galloping search in the sorted column, how
// many keys are at-or-below it.  Summed over the group these positions give
// the group's bucket counts.
template <class K, bool HV, bool MG = false>
__global__ __launch_bounds__(SORT_NT) void k_colsort_big(Batch<K> b, const K *src, const uint32_t *vsrc,
                                                          K *dst, uint32_t *vdst, uint32_t cutoff)
{
    static_assert(!MG || sizeof(K) == 8, "the merge column sort takes 64-bit keys");
    __shared__ ColSm<HV, MG> csm;
    SortSm &sm = csm.sort;
    const uint32_t bi = find_node(b.bigGrp, b.NB, blockIdx.x);
    const NodeDesc nd = b.nodes[b.bigIdx[bi]];
    const uint32_t wi = blockIdx.x - b.bigGrp[bi];
    const uint32_t S = nd.sub, g = wi / S, cps = TG / S;
    const uint32_t m = nd.m, n = nd.n, npiv = m - 1;
    const uint32_t i0 = g * TG + (wi % S) * cps;
    if (i0 >= m) return;                                 // a sub-group past the last column
    const uint32_t ncol = min(cps, m - i0);
    const bool recursed = nd.flags & NODE_COLS_RECURSED;
    static_assert(PIV_ALIGN * SORT_NT >= SORT_CAP, "one pivot slice per thread covers a node");
    constexpr int PPT = PIV_ALIGN;                       // pivots t0 .. t0 + PPT - 1 of this thread
    const uint32_t t0 = threadIdx.x * PPT;

    uint32_t P[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) P[q] = 0;

    uint32_t total = 0;
    for (uint32_t c = 0; c < ncol; ++c) {
        const uint32_t i = i0 + c;
        const uint32_t len = column_len(i, m, n);
        total += len;
        if (len == 0) {                                   // uniform over the work-group
            for (uint32_t J = threadIdx.x; J <= nd.nJ; J += SORT_NT) b.srcOff[nd.src + (uint64_t)J * m + i] = 0;
            continue;
        }
        const bool sorted = recursed && len > cutoff;   // sorted by its own recursion
        const uint64_t base = nd.off + (uint64_t)i * m;
        K clo = (K)0;
        int passes = 0;
        int binned = 2;
        int rsh = 0;
        uint32_t rlast = 255u;
        bool fast = false;
        const uint32_t *rtab = nullptr;
        // this thread's pivots and strict flags, as 16-byte loads of its
        // aligned, padded slice (entries past npiv are not used); for 32-bit
        // keys issued here, so that they arrive while the column is stored.
        // 64-bit keys have no registers to spare: they load and search the
        // slice in two halves of 8, each just before its search.
        constexpr int PH = sizeof(K) == 4 ? PPT : PPT / 2;
        constexpr int PV4 = PH * (int)sizeof(K) / 16;
        uint4 praw[PV4];
        uint4 sraw = make_uint4(0u, 0u, 0u, 0u);
        auto load_pivots = [&](uint32_t th) {
            if (th < npiv) {
                const uint4 *p4 = reinterpret_cast<const uint4 *>(b.piv + nd.piv + th);
#pragma unroll
                for (int v4 = 0; v4 < PV4; ++v4) praw[v4] = p4[v4];
                if (PH == 16) {
                    sraw = *reinterpret_cast<const uint4 *>(b.strict + nd.piv + th);
                } else {
                    const uint2 s2 = *reinterpret_cast<const uint2 *>(b.strict + nd.piv + th);
                    sraw = make_uint4(s2.x, s2.y, 0u, 0u);
                }
            }
        };
        if constexpr (MG) {
            // 64-bit keys: stable merge sort in LDS; the sorted column stays
            // there for the count
            constexpr int MI = MergeCap<HV>::IPT;
            uint64_t *Kc = csm.mg.k;
            uint32_t *Vc = csm.mg.v;
            uint64_t mk[MI];
            uint32_t mv[MI];
            // the row positions are recomputed for every column (not kept in
            // registers across the column loop, which would spill)
            uint32_t tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
#pragma unroll
            for (int r = 0; r < MI; ++r) {
                const uint32_t p = (uint32_t)r * SORT_NT + tid;
                const bool ok = p < len;
                mk[r] = ok ? (uint64_t)(sorted ? dst[base + p] : src[base + p]) : 0ull;
                if (HV) mv[r] = ok && !sorted ? vsrc[base + p] : 0u;
            }
            wait_vmem();
#pragma unroll
            for (int r = 0; r < MI; ++r) {
                const uint32_t p = (uint32_t)r * SORT_NT + tid;
                if (p < len) {
                    Kc[p] = mk[r];
                    if (HV) Vc[p] = mv[r];
                }
            }
            __syncthreads();
            if (!sorted) {
                lds_merge_sort<HV, MI>(Kc, Vc, len);
                uint32_t tid2 = threadIdx.x;
                asm volatile("" : "+v"(tid2));
#pragma unroll
                for (int r = 0; r < MI; ++r) {
                    const uint32_t p = (uint32_t)r * SORT_NT + tid2;
                    if (p < len) {
                        dst[base + p] = (K)Kc[p];
                        if (HV) vdst[base + p] = Vc[p];
                    }
                }
            }
        } else {
            K kk[SORT_IPT];
            uint32_t vv[SORT_IPT];
            tables_clear<SORT_NW, 256>(sm.s.tab);           // the previous search reused this LDS
            const int R = block_rows<SORT_NW, SORT_IPT>(len);
#pragma unroll
            for (int r = 0; r < SORT_IPT; ++r) {
                const uint32_t p = bpos(r, R);
                const bool ok = r < R && p < len;
                kk[r] = ok ? (sorted ? dst[base + p] : src[base + p]) : (K)0;
                if (HV) vv[r] = ok && !sorted ? vsrc[base + p] : 0u;
            }
            wait_vmem();
            __syncthreads();
            // 32-bit keys without values sort by bins of the key range; a column
            // with a crowded bin (and every other key type) by LSD radix passes
            if constexpr (sizeof(K) == 4 && !HV) {
                if (!sorted) {
                    uint32_t blo = 0u, nbin = 0u;
                    binned = bin_sort<SORT_NW, SORT_IPT>(kk, len, sm, blo, rsh, nbin);
                    if (binned == 1) { clo = (K)blo; rlast = nbin - 1u; }
                    if (binned == 2) {                     // loaded again: see lds_sort
                        block_load<K, HV, SORT_NW, SORT_IPT>(kk, vv, len, src + base, nullptr);
                        tables_clear<SORT_NW, 256>(sm.s.tab);
                        __syncthreads();
                    }
                }
            }
            if (!sorted && binned == 2) {
                block_sort<K, HV, SORT_NW, SORT_IPT>(kk, vv, len, sm, false, (K)0, (K)0, &clo, &passes);
                rsh = 8 * (passes - 1);
            }
            // 32-bit keys without values: the sorted column (minus clo) is still in
            // the exchange buffer, and the start of every bin (or of every
            // last-pass digit) in the tables' space, so the count searches there
            // and narrows each whole-column search to the keys of the pivot's bin
            // (digit)
            fast = sizeof(K) == 4 && !HV && !sorted && (passes > 0 || binned == 1);
            rtab = binned == 1 ? bin_starts(sm) : sm.s.tab[0].off;
            if (sizeof(K) == 4) load_pivots(t0);
            if (!sorted) {
#pragma unroll
                for (int r = 0; r < SORT_IPT; ++r) {
                    const uint32_t p = bpos(r, R);
                    if (r < R && p < len) {
                        dst[base + p] = kk[r];
                        if (HV) vdst[base + p] = vv[r];
                    }
                }
            }
            if (!fast) {
                __syncthreads();
#pragma unroll
                for (int r = 0; r < SORT_IPT; ++r) {
                    const uint32_t p = bpos(r, R);
                    if (r < R && p < len) { if (sizeof(K) == 4) sm.k32[p] = (uint32_t)kk[r]; else sm.k64[p] = (uint64_t)kk[r]; }
                }
                __syncthreads();
            }
        }
        // key at position q of the sorted column, and a pivot in the same
        // space (below the column minimum: 0 taken as strict, below every key)
        auto ck = [&](uint32_t q) -> K {
            if constexpr (MG) return (K)csm.mg.k[q];
            return fast ? (K)sm.s.buf[q] : col_key<K>(sm, q);
        };
        auto tpiv = [&](K p, bool &st) -> K {
            if (!fast) return p;
            if (p < clo) { st = true; return (K)0; }
            return (K)(p - clo);
        };
        // whole-column search range of a pivot (fast: its bin or last-pass digit)
        auto range = [&](K p, uint32_t &a, uint32_t &e) {
            a = 0;
            e = len;
            if (fast) {
                const K d = (K)(p >> rsh);
                if (d > (K)rlast) { a = len; return; }                // above every key
                a = min(rtab[(uint32_t)d], len);
                e = d < (K)rlast ? min(rtab[(uint32_t)d + 1], len) : len;
            }
        };
        // Each pivot's position in the sorted column (keys at or below it).
        bool counted = false;
        if constexpr (sizeof(K) == 4 && !HV) {
            if (binned == 1) {
                // Sorted by bins: the position is the start of the pivot's bin
                // plus the keys of that bin at or below it.  A bin of a sort
                // that succeeded holds at most BIN_NET = 16 keys (bins of
                // width one: keys of one value only, so their start or end is
                // the position), and every key after the bin is larger than
                // the pivot, so five halving steps over the 16 words from the
                // bin's start (reads clamped to the column's last key, the
                // result to the column's length) find it without the bin's
                // end; the steps of the 16 pivots are independent, so their
                // LDS reads overlap.
                static_assert(BIN_NET <= 16, "five halving steps cover a bin");
                const uint32_t *bst = bin_starts(sm);
                const uint32_t nbin = rlast + 1u, c0 = (uint32_t)clo, last = len - 1u;
                const uint32_t nq = t0 < npiv ? min((uint32_t)PPT, npiv - t0) : 0u;
                uint32_t la[PPT], lx[PPT];
                bool lsr[PPT];
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    const uint32_t p = (uint32_t)piv_of<K>(praw, q);
                    const bool s = strict_of(sraw, q);
                    uint32_t a = 0u, xe = 0u;               // below every key: position 0
                    bool sr = false;
                    if (p > c0 || (p == c0 && !s)) {
                        const uint32_t x = p - c0, d = x >> rsh;
                        if (d >= nbin) a = len;              // above every key
                        else if (rsh == 0) a = s ? bst[d] : (d + 1u < nbin ? bst[d + 1] : len);
                        else {
                            a = bst[d];
                            xe = x - (s ? 1u : 0u);          // keys <= xe are at or below p
                            sr = true;
                        }
                    }
                    la[q] = a;
                    lx[q] = xe;
                    lsr[q] = sr;
                }
                if (rsh > 0) {
#pragma unroll
                    for (int stp = 16; stp >= 1; stp >>= 1) {
#pragma unroll
                        for (int q = 0; q < PPT; ++q) {
                            const uint32_t v = sm.s.buf[min(la[q] + (uint32_t)(stp - 1), last)];
                            if (lsr[q] && v <= lx[q]) la[q] += (uint32_t)stp;
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    if (q < (int)nq) {
                        const uint32_t t = t0 + q;
                        const uint32_t a = min(la[q], len);
                        P[q] += a;
                        if ((t + 1) % TB == 0) b.srcOff[nd.src + (uint64_t)((t + 1) / TB) * m + i] = a;
                    }
                }
                counted = true;
            }
        }
        // Otherwise the slice's first and last pivot are searched over the
        // whole column (or their last-pass digit's range), the others inside
        // that bracket; the searches of one step are independent, so their
        // LDS reads overlap.
        if (!counted) {
#pragma unroll
        for (int h = 0; h < PPT / PH; ++h) {
            const uint32_t th = t0 + h * PH;
            if (sizeof(K) != 4) load_pivots(th);
            const uint32_t nq = th < npiv ? min((uint32_t)PH, npiv - th) : 0u;
            if (nq > 0) {
                K pf = (K)0, pl = (K)0;
                bool sf = false, sl = false;
#pragma unroll
                for (int q = 0; q < PH; ++q) {
                    if (q == 0) { sf = strict_of(sraw, q); pf = tpiv(piv_of<K>(praw, q), sf); }
                    if (q == (int)nq - 1) { sl = strict_of(sraw, q); pl = tpiv(piv_of<K>(praw, q), sl); }
                }
                uint32_t af, ef, al, el;
                range(pf, af, ef);
                range(pl, al, el);
                while (af < ef || al < el) {
                    if (af < ef) {
                        const uint32_t mid = (af + ef) >> 1;
                        if (le_pivot(ck(mid), pf, sf)) af = mid + 1; else ef = mid;
                    }
                    if (al < el) {
                        const uint32_t mid = (al + el) >> 1;
                        if (le_pivot(ck(mid), pl, sl)) al = mid + 1; else el = mid;
                    }
                }
                uint32_t A[PH], E[PH];
#pragma unroll
                for (int q = 0; q < PH; ++q) {
                    const bool inner = q > 0 && q + 1 < (int)nq;
                    A[q] = inner ? af : 0u;
                    E[q] = inner ? al : 0u;
                }
                bool more = true;
                while (more) {
                    more = false;
#pragma unroll
                    for (int q = 1; q + 1 < PH; ++q) {
                        if (A[q] < E[q]) {
                            const uint32_t mid = (A[q] + E[q]) >> 1;
                            bool sq = strict_of(sraw, q);
                            const K pq = tpiv(piv_of<K>(praw, q), sq);
                            if (le_pivot(ck(mid), pq, sq)) A[q] = mid + 1;
                            else E[q] = mid;
                            more |= A[q] < E[q];
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < PH; ++q) {
                    if (q < (int)nq) {
                        const uint32_t t = th + q;
                        const uint32_t a = q == 0 ? af : (q == (int)nq - 1 ? al : A[q]);
                        P[h * PH + q] += a;
                        if ((t + 1) % TB == 0) b.srcOff[nd.src + (uint64_t)((t + 1) / TB) * m + i] = a;
                    }
                }
            }
        }
        }
        if (threadIdx.x == 0) {
            b.srcOff[nd.src + i] = 0;
            b.srcOff[nd.src + (uint64_t)nd.nJ * m + i] = len;
        }
        __syncthreads();
    }
    // per-bucket counts of the group from the accumulated positions
    uint32_t *Pl = sm.k32;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t t = t0 + q;
        if (t < npiv) Pl[t] = P[q];
    }
    __syncthreads();
    uint32_t *blk = b.blk + nd.blk + (uint64_t)g * m;
    if (S == 1) {
        for (uint32_t t = threadIdx.x; t < npiv; t += SORT_NT) blk[t] = Pl[t] - (t > 0 ? Pl[t - 1] : 0u);
        if (threadIdx.x == 0) blk[m - 1] = total - (npiv > 0 ? Pl[npiv - 1] : 0u);
    } else {                                             // the group's counts start at zero
        for (uint32_t t = threadIdx.x; t < npiv; t += SORT_NT) {
            const uint32_t c = Pl[t] - (t > 0 ? Pl[t - 1] : 0u);
            if (c) atomicAdd(&blk[t], c);
        }
        if (threadIdx.x == 0) atomicAdd(&blk[m - 1], total - (npiv > 0 ? Pl[npiv - 1] : 0u));
    }
}

// Nodes with m <= WCAP: one work-group of SM_NW waves per (node, column
// group), one wave per column.  After the wave sort the column is put in the
// wave's LDS and every pivot finds its position in it (keys at or below it)
// as in k_colsort_big: lane l owns pivots 16l .. 16l + 15 (in registers for
// the whole group), searches its first and last over the column and the
// others inside that bracket.  Summed over the group's columns the positions
// give the group's bucket counts; every 64th gives a bucket-block offset.
template <class K, bool HV, int NWS>
__global__ __launch_bounds__(NWS * WAVE) void k_colsort_small(Batch<K> b, const K *src, const uint32_t *vsrc,
                                                               K *dst, uint32_t *vdst, uint32_t cutoff)
{
    static_assert(PIV_ALIGN * WAVE >= WCAP, "one pivot slice per lane covers a node");
    static_assert(NWS >= 1 && TG % NWS == 0, "whole columns per wave");
    __shared__ WaveSmem<WR> wsm[NWS];
    __shared__ uint32_t Pl[WCAP];
    __shared__ uint32_t total_sh;
    const uint32_t si = find_node(b.smlGrp, b.NS, blockIdx.x);
    const NodeDesc nd = b.nodes[b.smlIdx[si]];
    const uint32_t wi = blockIdx.x - b.smlGrp[si];
    const uint32_t S = nd.sub, g = wi / S, cps = TG / S;
    const uint32_t m = nd.m, n = nd.n, npiv = m - 1, nJ = nd.nJ;
    const uint32_t i0 = g * TG + (wi % S) * cps;
    if (i0 >= m) return;                                 // a sub-group past the last column
    const uint32_t ncol = min(cps, m - i0);
    const bool recursed = nd.flags & NODE_COLS_RECURSED;
    const uint32_t w = wave_id(), l = lane_id();
    // the sorted column: the wave's exchange buffer (u32 keys), or its table
    // and buffer together (u64 keys; the table is cleared again after)
    static_assert(sizeof(RankTab<256>) + sizeof(uint32_t) * WR * WAVE >= sizeof(uint64_t) * WCAP, "column fits");
    K *ck = sizeof(K) == 4 ? reinterpret_cast<K *>(wsm[w].buf) : reinterpret_cast<K *>(&wsm[w]);

    for (uint32_t t = threadIdx.x; t < WCAP; t += NWS * WAVE) Pl[t] = 0;
    if (threadIdx.x == 0) total_sh = 0;
    wave_table_clear(wsm[w].tab);
    // this lane's pivots and strict flags (16-byte loads of its aligned, padded slice)
    constexpr int PPT = PIV_ALIGN;
    constexpr int PV4 = PPT * (int)sizeof(K) / 16;
    const uint32_t t0 = l * PPT;
    const uint32_t nq = t0 < npiv ? min((uint32_t)PPT, npiv - t0) : 0u;
    uint4 praw[PV4];
    uint4 sraw = make_uint4(0u, 0u, 0u, 0u);
    if (nq > 0) {
        const uint4 *p4 = reinterpret_cast<const uint4 *>(b.piv + nd.piv + t0);
#pragma unroll
        for (int v4 = 0; v4 < PV4; ++v4) praw[v4] = p4[v4];
        sraw = *reinterpret_cast<const uint4 *>(b.strict + nd.piv + t0);
    }
    uint32_t P[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) P[q] = 0;
    uint32_t total = 0;
    __syncthreads();

    for (uint32_t c = w; c < ncol; c += NWS) {
        const uint32_t i = i0 + c;
        const uint32_t len = __builtin_amdgcn_readfirstlane(column_len(i, m, n));
        uint32_t *so = b.srcOff + nd.src + i;              // so[J*m]
        total += len;
        if (len == 0) {
            for (uint32_t J = l; J <= nJ; J += WAVE) so[(uint64_t)J * m] = 0;
            continue;
        }
        const bool sorted = recursed && len > cutoff;
        const uint64_t base = nd.off + (uint64_t)i * m;
        K kk[WR];
        uint32_t vv[WR];
#pragma unroll
        for (int r = 0; r < WR; ++r) {
            const uint32_t p = r * WAVE + l;
            const bool ok = p < len;
            kk[r] = ok ? (sorted ? dst[base + p] : src[base + p]) : (K)0;
            if (HV) vv[r] = ok && !sorted ? vsrc[base + p] : 0u;
        }
        K clo = (K)0;
        int passes = 0;
        // 32-bit keys without values: bins, then radix passes if a bin is
        // crowded (the bin sort leaves the table to be cleared: at once for
        // the radix passes, after the count when the bin starts serve it)
        int binned = 2;
        int rsh = 0;
        uint32_t rlast = 255u;
        if constexpr (sizeof(K) == 4 && !HV) {
            if (!sorted) {
                uint32_t blo = 0u, nbin = 0u;
                binned = wave_bin_sort<WR>(kk, len, wsm[w], blo, rsh, nbin);
                if (binned == 1) { clo = (K)blo; rlast = nbin - 1u; }
                if (binned == 2) {                     // the radix passes need a clear table
                    wave_table_clear(wsm[w].tab);
                    wave_lds_sync();
                }
            }
        }
        if (!sorted && binned == 2) {
            wave_sort<K, HV, WR>(kk, vv, len, wsm[w], &clo, &passes);
            rsh = 8 * (passes - 1);
        }
        if (!sorted) {
#pragma unroll
            for (int r = 0; r < WR; ++r) {
                const uint32_t p = r * WAVE + l;
                if (p < len) {
                    dst[base + p] = kk[r];
                    if (HV) vdst[base + p] = vv[r];
                }
            }
        }
        // 32-bit keys without values: the sorted column (minus clo) is still
        // in the wave's buffer and the last pass's digit starts in its table;
        // the count searches there, each whole-column search narrowed to the
        // pivot's digit (as in k_colsort_big)
        const bool fast = sizeof(K) == 4 && !HV && !sorted && (passes > 0 || binned == 1);
        const uint32_t *rtab = binned == 1 ? wave_bin_starts(wsm[w]) : wsm[w].tab.off;
        wave_lds_sync();
        if (!fast) {
#pragma unroll
            for (int r = 0; r < WR; ++r) {
                const uint32_t p = r * WAVE + l;
                if (p < len) ck[p] = kk[r];
            }
            wave_lds_sync();
        }
        auto tpiv = [&](K p, bool &st) -> K {
            if (!fast) return p;
            if (p < clo) { st = true; return (K)0; }
            return (K)(p - clo);
        };
        auto range = [&](K p, uint32_t &a, uint32_t &e) {
            a = 0;
            e = len;
            if (fast) {
                const K d = (K)(p >> rsh);
                if (d > (K)rlast) { a = len; return; }
                a = min(rtab[(uint32_t)d], len);
                e = d < (K)rlast ? min(rtab[(uint32_t)d + 1], len) : len;
            }
        };
        // positions of the lane's first and last pivot over the column, the
        // others inside that bracket (independent searches step together)
        if (nq > 0) {
            K pf = (K)0, pl = (K)0;
            bool sf = false, sl = false;
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                if (q == 0) { sf = strict_of(sraw, q); pf = tpiv(piv_of<K>(praw, q), sf); }
                if (q == (int)nq - 1) { sl = strict_of(sraw, q); pl = tpiv(piv_of<K>(praw, q), sl); }
            }
            uint32_t af, ef, al, el;
            range(pf, af, ef);
            range(pl, al, el);
            while (af < ef || al < el) {
                if (af < ef) {
                    const uint32_t mid = (af + ef) >> 1;
                    if (le_pivot(ck[mid], pf, sf)) af = mid + 1; else ef = mid;
                }
                if (al < el) {
                    const uint32_t mid = (al + el) >> 1;
                    if (le_pivot(ck[mid], pl, sl)) al = mid + 1; else el = mid;
                }
            }
            uint32_t A[PPT], E[PPT];
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const bool inner = q > 0 && q + 1 < (int)nq;
                A[q] = inner ? af : 0u;
                E[q] = inner ? al : 0u;
            }
            bool more = true;
            while (more) {
                more = false;
#pragma unroll
                for (int q = 1; q + 1 < PPT; ++q) {
                    if (A[q] < E[q]) {
                        const uint32_t mid = (A[q] + E[q]) >> 1;
                        bool sq = strict_of(sraw, q);
                        const K pq = tpiv(piv_of<K>(praw, q), sq);
                        if (le_pivot(ck[mid], pq, sq)) A[q] = mid + 1;
                        else E[q] = mid;
                        more |= A[q] < E[q];
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                if (q < (int)nq) {
                    const uint32_t t = t0 + q;
                    const uint32_t a = q == 0 ? af : (q == (int)nq - 1 ? al : A[q]);
                    P[q] += a;
                    if ((t + 1) % TB == 0) so[(uint64_t)((t + 1) / TB) * m] = a;
                }
            }
        }
        if (l == 0) { so[0] = 0; so[(uint64_t)nJ * m] = len; }
        wave_lds_sync();
        if (sizeof(K) == 8 || binned == 1) {             // the column or the bins overlaid the table
            wave_table_clear(wsm[w].tab);
            wave_lds_sync();
        }
    }
    // per-bucket counts of the group from the summed positions
#pragma unroll
    for (int q = 0; q < PPT; ++q)
        if (q < (int)nq && P[q]) atomicAdd(&Pl[t0 + q], P[q]);
    if (l == 0 && total) atomicAdd(&total_sh, total);
    __syncthreads();
    const uint32_t tot = total_sh;
    uint32_t *blk = b.blk + nd.blk + (uint64_t)g * m;
    for (uint32_t t = threadIdx.x; t < m; t += NWS * WAVE) {
        const uint32_t hi = t < npiv ? Pl[t] : tot;
        const uint32_t c = hi - (t > 0 ? Pl[t - 1] : 0u);
        if (S == 1) blk[t] = c;
        else if (c) atomicAdd(&blk[t], c);               // the group's counts start at zero
    }
}

// Per node and bucket j: exclusive prefix of the group counts over groups
// (in place) and the bucket total.
template <class K>
__global__ void k_colscan(Batch<K> b)
{
    const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= b.bucStart[b.N]) return;
    const uint32_t k = find_node(b.bucStart, b.N, item);
    const NodeDesc nd = b.nodes[k];
    const uint32_t j = item - b.bucStart[k];
    uint32_t run = 0;
    uint32_t *p = b.blk + nd.blk + j;
    constexpr uint32_t B = 16;                       // loads of B groups in flight together
    for (uint32_t g0 = 0; g0 < nd.groups; g0 += B) {
        uint32_t c[B];
#pragma unroll
        for (uint32_t q = 0; q < B; ++q) c[q] = g0 + q < nd.groups ? p[(uint64_t)(g0 + q) * nd.m] : 0u;
#pragma unroll
        for (uint32_t q = 0; q < B; ++q)
            if (g0 + q < nd.groups) { p[(uint64_t)(g0 + q) * nd.m] = run; run += c[q]; }
    }
    b.tot[nd.bkt + j] = run;
}

// Bucket positions (Section 2.2): exclusive scan of the bucket totals.
template <class K>
__global__ __launch_bounds__(1024) void k_bucket_start(Batch<K> b, unsigned long long *bs64_out)
{
    __shared__ uint32_t wsum[16];
    const NodeDesc nd = b.nodes[blockIdx.x];
    const uint32_t m = nd.m;
    const uint32_t per = (m + 1023) / 1024;
    const uint32_t j0 = threadIdx.x * per;
    uint32_t s = 0;
    for (uint32_t q = 0; q < per; ++q)
        if (j0 + q < m) s += b.tot[nd.bkt + j0 + q];
    const uint32_t incl = wave_incl_scan(s);
    if (lane_id() == WAVE - 1) wsum[wave_id()] = incl;
    __syncthreads();
    uint32_t run = incl - s;
    for (uint32_t w = 0; w < wave_id(); ++w) run += wsum[w];
    constexpr uint32_t B = 16;                       // loads of B totals in flight together
    for (uint32_t q0 = 0; q0 < per; q0 += B) {
        uint32_t t[B];
#pragma unroll
        for (uint32_t q = 0; q < B; ++q) t[q] = q0 + q < per && j0 + q0 + q < m ? b.tot[nd.bkt + j0 + q0 + q] : 0u;
#pragma unroll
        for (uint32_t q = 0; q < B; ++q) {
            if (q0 + q < per && j0 + q0 + q < m) {
                b.bs[nd.bkt + j0 + q0 + q] = run;
                if (bs64_out) bs64_out[j0 + q0 + q] = run;
                run += t[q];
            }
        }
    }
    if (threadIdx.x == 0) {
        b.bs[nd.bkt + m] = nd.n;
        if (bs64_out) bs64_out[m] = nd.n;
    }
}

// ------------------------------------------------------------ SkewTranspose
// Tile (group g, bucket block J): the runs of the TG columns of g that fall
// in the TB buckets of J are read contiguously (column order), partitioned
// stably by bucket in LDS, and written as contiguous runs per bucket.  The
// layout is that of Alg. 2/3: bucket j receives, column by column, the
// column's keys of bucket j in sorted order.  Tiles larger than one chunk
// are processed chunk by chunk in column order, which keeps that order.
//
// Per key, the column is read from a per-position map filled run by run, and
// the bucket from a 512-slot table over the block's key range.  Pivot t is
// passed by the keys at or above its threshold p_t (s_t for a strict pivot,
// s_t + 1 otherwise; thresholds are non-decreasing).  Slot u starts at
// lo + u*2^sh and holds the number of thresholds at or below its start, so a
// key's bucket lies between the entries of its slot and the next, and a
// binary search over the thresholds in between (usually none) finishes it.
// The table is built by one atomic add per pivot at the first slot its
// threshold does not exceed, then a scan.  A non-strict pivot equal to the
// largest key has no threshold: no key passes it and no slot counts it.
constexpr int TR_LUT_BITS = 9;
constexpr int TR_LUT = 1 << TR_LUT_BITS;

template <class K> struct TileSmem {
    RankTab<TB> tab[TR_NW];
    uint32_t wsum[TR_NW];
    uint32_t buf[TR_CH];         // exchange buffer; the slot counts while the table is built
    uint8_t colOf[TR_CH];        // column of each chunk position; then the bucket of each sorted position
    uint32_t relBase[TG];        // node-relative source index of chunk position q is relBase[c] + q (mod 2^32)
    uint32_t cOff[TG + 1];
    uint32_t dstb[TB];           // node-relative destination of the bucket's next key
    uint32_t wbase[TB];          // per chunk: destination of sorted position p is wbase[d] + p
    K pth[TB];                   // pivot thresholds of the block
    uint8_t lut[TR_LUT + 1];
};

// local bucket of x among the npv pivots of the block, given x >= lo
template <class K>
__device__ inline uint32_t tile_bucket(K x, K lo, int sh, const TileSmem<K> &sm)
{
    const K du = (K)((K)(x - lo) >> sh);
    const uint32_t u = du < (K)(TR_LUT - 1) ? (uint32_t)du : (uint32_t)(TR_LUT - 1);
    uint32_t a = sm.lut[u], e = sm.lut[u + 1];
    while (a < e) {                                  // duplicate pivots can share a slot
        const uint32_t mid = (a + e) >> 1;
        if (x >= sm.pth[mid]) a = mid + 1; else e = mid;
    }
    return a;
}

// The block's thresholds and slot table (all threads; two barriers inside;
// wave 0 writes the table after the second, so it is visible after the
// caller's next barrier).  lo: the pivot before the block
// (or 0), which every key of the block is at or above; sh as returned.
template <class K>
__device__ inline int tile_table(const Batch<K> &b, const NodeDesc &nd, uint32_t j0, uint32_t npv, K lo,
                                 TileSmem<K> &sm)
{
    using T = KeyT<K>;
    const uint32_t tid = threadIdx.x;
    const K hi = npv > 0 ? b.piv[nd.piv + j0 + npv - 1] : lo;
    const int sh = max(0, T::bitlen((K)(hi - lo)) - TR_LUT_BITS);
    for (uint32_t u = tid; u <= (uint32_t)TR_LUT; u += TR_NW * WAVE) sm.buf[u] = 0;
    __syncthreads();
    if (tid < npv) {
        const K sv = b.piv[nd.piv + j0 + tid];
        const bool strict = b.strict[nd.piv + j0 + tid] != 0;
        const K p = strict ? sv : (K)(sv + 1);
        sm.pth[tid] = p;
        if (strict || sv != (K)T::MAXV) {            // else no key passes it
            const K d = (K)(p - lo);
            const K q = (K)(d >> sh) + (((d & (K)(((K)1 << sh) - 1)) != 0) ? (K)1 : (K)0);
            atomicAdd(&sm.buf[q < (K)TR_LUT ? (uint32_t)q : (uint32_t)TR_LUT], 1u);
        }
    }
    __syncthreads();
    if (tid < WAVE) {                                // inclusive scan of the TR_LUT + 1 counts
        constexpr int PER = TR_LUT / WAVE;
        uint32_t c[PER], sum = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) { c[q] = sm.buf[tid * PER + q]; sum += c[q]; }
        uint32_t run = wave_incl_scan(sum) - sum;
#pragma unroll
        for (int q = 0; q < PER; ++q) { run += c[q]; sm.lut[tid * PER + q] = (uint8_t)run; }
        if (tid == WAVE - 1) sm.lut[TR_LUT] = (uint8_t)(run + sm.buf[TR_LUT]);
    }
    return sh;
}

// Tiles with more than TR_HEAVY keys (presorted inputs put a column group's
// keys into a few bucket blocks) are not processed by their own work-group:
// each of their chunks is an item for the TR_EXTRA persistent work-groups of
// k_transpose_heavy.  A chunk's destinations depend on the bucket counts of
// the tile's earlier chunks; it publishes its own counts (aggregate), walks
// back over its predecessors' records until one holds an inclusive prefix,
// then publishes its inclusive prefix (decoupled look-back).  Items are taken
// in ticket order, so every predecessor belongs to a running work-group that
// publishes its aggregate before it waits: the walk always ends.  Record
// words pack status and value, and are read and written as device-scope
// atomics (coherent across the chip's L2 caches).
constexpr uint32_t TR_HEAVY = 3 * TR_CH;
constexpr uint32_t TR_EXTRA = 1024;
constexpr unsigned long long TR_AGG = 1ull << 62, TR_INCL = 2ull << 62;
constexpr uint32_t TR_SPIN = 1u << 16;       // bound of one wait (tens of ms: far above a chunk's time)
constexpr uint32_t TR_SEQ = 0xFFFFFFFFu;     // item index of a tile processed whole by its work-group

// Keys of every tile; the heavy ones become chunk items (records cleared).
// One wave per tile.
template <class K>
__global__ __launch_bounds__(TR_NW * WAVE) void k_tile_plan(Batch<K> b, uint32_t tiles)
{
    const uint32_t tile = blockIdx.x * TR_NW + wave_id();
    if (tile >= tiles) return;
    const uint32_t l = lane_id();
    const uint32_t k = find_node(b.tileStart, b.N, tile);
    const NodeDesc nd = b.nodes[k];
    const uint32_t tix = tile - b.tileStart[k];
    const uint32_t g = tix / nd.nJ, J = tix % nd.nJ, m = nd.m;
    const uint32_t i0 = g * TG, ncol = min((uint32_t)TG, m - i0);
    uint32_t len = 0;
    if (l < ncol)
        len = b.srcOff[nd.src + (uint64_t)(J + 1) * m + i0 + l] - b.srcOff[nd.src + (uint64_t)J * m + i0 + l];
    const uint32_t N = __builtin_amdgcn_readlane(wave_incl_scan(len), WAVE - 1);
    if (N <= TR_HEAVY) return;
    const uint32_t nch = (N + TR_CH - 1) / TR_CH;
    uint32_t s0 = 0;
    if (l == 0) s0 = atomicAdd(&b.ctr[CTR_TR_ITEMS], nch);
    s0 = __builtin_amdgcn_readfirstlane(s0);
    if (s0 + nch > b.trCap) {                      // cannot happen: trCap bounds the chunks
        if (l == 0) atomicOr(&b.ctr[CTR_TR_FAIL], 1u);
        return;
    }
    for (uint32_t c = l; c < nch; c += WAVE) { b.trItem[2 * (s0 + c)] = tile; b.trItem[2 * (s0 + c) + 1] = c; }
    for (uint32_t c = 0; c < nch; ++c) b.trRec[(uint64_t)(s0 + c) * TB + l] = 0ull;
}

// Keys of bucket d in the tile's chunks before this one, plus the bucket's
// tile destination: walk back over the records of the earlier items.
template <class K>
__device__ inline uint32_t tr_lookback(const Batch<K> &b, uint32_t item, uint32_t d)
{
    uint32_t run = 0;
    for (uint32_t p = item - 1;; --p) {
        unsigned long long v;
        uint32_t spins = 0;
        while (((v = __hip_atomic_load(&b.trRec[(uint64_t)p * TB + d], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT)) >> 62) == 0) {
            if (++spins > TR_SPIN) {                 // never expected: report instead of waiting on
                atomicOr(&b.ctr[CTR_TR_FAIL], 1u);
                return run;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        run += (uint32_t)v;
        if ((v >> 62) == 2) return run;
    }
}

// One tile (item == TR_SEQ: all its chunks in order, unless it is heavy) or
// one chunk of a heavy tile (item: its index in the chunk list).
template <class K, bool HV>
__device__ void transpose_tile(const Batch<K> &b, const K *src, const uint32_t *vsrc, K *dst, uint32_t *vdst,
                               TileSmem<K> &sm, uint32_t tile, uint32_t item, uint32_t chunk)
{
    using T = KeyT<K>;
    const uint32_t k = find_node(b.tileStart, b.N, tile);
    const NodeDesc nd = b.nodes[k];
    const uint32_t tix = tile - b.tileStart[k];
    const uint32_t g = tix / nd.nJ, J = tix % nd.nJ;
    const uint32_t m = nd.m;
    const uint32_t i0 = g * TG, ncol = min((uint32_t)TG, m - i0);
    const uint32_t j0 = J * TB, nb = min((uint32_t)TB, m - j0);
    const uint32_t npv = (j0 + nb <= m - 1) ? nb : nb - 1;   // real pivots of the block
    const uint32_t tid = threadIdx.x;
    const uint32_t l = lane_id(), w = wave_id();

    if (tid < WAVE) {                      // one wave builds the run table
        uint32_t a = 0, len = 0;
        if (tid < ncol) {
            a = b.srcOff[nd.src + (uint64_t)J * m + i0 + tid];
            len = b.srcOff[nd.src + (uint64_t)(J + 1) * m + i0 + tid] - a;
        }
        const uint32_t incl = wave_incl_scan(len);
        if (tid < ncol) {
            sm.cOff[tid] = incl - len;
            sm.relBase[tid] = (i0 + tid) * m + a - (incl - len);     // mod 2^32; the true value is < n
        }
        if (tid == ncol - 1) sm.cOff[ncol] = incl;
    }
    if (tid < nb) {
        const uint32_t j = j0 + tid;
        sm.dstb[tid] = b.bs[nd.bkt + j] + b.blk[nd.blk + (uint64_t)g * m + j];
    }
    // every key of the block is >= the pivot before it (or 0)
    const K lo = j0 > 0 ? b.piv[nd.piv + j0 - 1] : (K)0;
    const int sh = tile_table(b, nd, j0, npv, lo, sm);
    const uint32_t N = sm.cOff[ncol];
    RankTab<TB> &tab = sm.tab[w];
    const bool seq = item == TR_SEQ;
    if (seq && N > TR_HEAVY) {             // its chunks are items of the persistent work-groups
        __syncthreads();
        return;
    }

    for (uint32_t q0 = seq ? 0u : chunk * TR_CH; q0 < (seq ? N : min(N, (chunk + 1) * TR_CH)); q0 += TR_CH) {
        const uint32_t chN = min((uint32_t)TR_CH, N - q0);
        const int nrows = wave_rows<TR_IPT>(chN);
        // column map of the chunk: wave w fills the runs of columns w, w + TR_NW, ...
        for (uint32_t c = w; c < ncol; c += TR_NW) {
            const uint32_t s0 = max(sm.cOff[c], q0), s1 = min(sm.cOff[c + 1], q0 + chN);
            for (uint32_t q = s0 + l; q < s1; q += WAVE) sm.colOf[q - q0] = (uint8_t)c;
        }
        __syncthreads();
        K kk[TR_IPT];
        uint32_t vv[TR_IPT], dig[TR_IPT], pos[TR_IPT];
        // all loads of the chunk first, so that they are in flight together
#pragma unroll
        for (int r = 0; r < TR_IPT; ++r) {
            kk[r] = (K)0;
            vv[r] = 0;
            const uint32_t p = item_pos<TR_NW, TR_IPT>(r);
            if (r < nrows && p < chN) {
                const uint32_t c = sm.colOf[p];
                const uint32_t rel = sm.relBase[c] + q0 + p;
                const uint64_t at = nd.off + (rel < nd.n ? rel : 0u);  // guard: inside the node
                kk[r] = src[at];
                if (HV) vv[r] = vsrc[at];
            }
        }
#pragma unroll
        for (int r = 0; r < TR_IPT; ++r) {
            dig[r] = TB - 1;
            if (r < nrows) {
                const uint32_t p = item_pos<TR_NW, TR_IPT>(r);
                if (p < chN) dig[r] = tile_bucket(kk[r], lo, sh, sm);
                pos[r] = rank_row(tab, dig[r]);
            }
        }
        __syncthreads();
        scan_tables<TR_NW, TB>(sm.tab, sm.wsum);
#pragma unroll
        for (int r = 0; r < TR_IPT; ++r) if (r < nrows) pos[r] += tab.off[dig[r]];
#pragma unroll
        for (int wd = 0; wd < T::WORDS; ++wd) {
#pragma unroll
            for (int r = 0; r < TR_IPT; ++r) {
                if (r < nrows) {
                    sm.buf[pos[r]] = T::word(kk[r], wd);
                    if (wd == 0) sm.colOf[pos[r]] = (uint8_t)dig[r];
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < TR_IPT; ++r)
                if (r < nrows) kk[r] = T::set_word(kk[r], wd, sm.buf[item_pos<TR_NW, TR_IPT>(r)]);
            __syncthreads();
        }
        if (HV) {
#pragma unroll
            for (int r = 0; r < TR_IPT; ++r) if (r < nrows) sm.buf[pos[r]] = vv[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < TR_IPT; ++r) if (r < nrows) vv[r] = sm.buf[item_pos<TR_NW, TR_IPT>(r)];
            __syncthreads();
        }
        // sorted chunk position p of bucket d goes to wbase[d] + p; positions
        // past chN carry the padding digit TB - 1 and come last
        if (seq) {
            if (tid < nb) {
                const uint32_t s0 = min(sm.tab[0].off[tid], chN);
                const uint32_t e0 = min(tid + 1 < TB ? sm.tab[0].off[tid + 1] : (uint32_t)TR_CH, chN);
                sm.wbase[tid] = sm.dstb[tid] - s0;
                sm.dstb[tid] += e0 - s0;
            }
        } else if (tid < WAVE) {            // wave 0, lane = bucket of the block
            static_assert(TB == WAVE, "one lane per bucket of a tile");
            const uint32_t d = tid;
            const uint32_t s0 = d < nb ? min(sm.tab[0].off[d], chN) : 0u;
            const uint32_t e0 = d < nb ? min(d + 1 < TB ? sm.tab[0].off[d + 1] : (uint32_t)TR_CH, chN) : 0u;
            unsigned long long *rec = b.trRec + (uint64_t)item * TB + d;
            uint32_t base;
            if (chunk == 0) {
                base = d < nb ? sm.dstb[d] : 0u;
            } else {
                __hip_atomic_store(rec, TR_AGG | (e0 - s0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                base = tr_lookback(b, item, d);
            }
            __hip_atomic_store(rec, TR_INCL | (uint32_t)(base + e0 - s0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (d < nb) sm.wbase[d] = base - s0;
        }
        wait_vmem();
        __syncthreads();
#pragma unroll
        for (int r = 0; r < TR_IPT; ++r) {
            if (r < nrows) {
                const uint32_t p = item_pos<TR_NW, TR_IPT>(r);
                if (p < chN) {
                    const uint32_t rel = sm.wbase[sm.colOf[p]] + p;
                    if (rel < nd.n) {                                        // guard: inside the node
                        dst[nd.off + rel] = kk[r];
                        if (HV) vdst[nd.off + rel] = vv[r];
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Every tile that is not heavy, whole, by its own work-group.  Registers are
// held to eight waves per SIMD for 32-bit keys (LDS admits eight work-groups
// per CU) and seven for 64-bit keys; key/value tiles would spill, so stay free.
// (Chunks of 2560 keys: a tile of the 2^28 root holds 4096 +- 512 keys, so
// most take two chunks either way, and smaller chunks raise the occupancy:
// 4096-key chunks 1.04 ms, 3072 1.02 ms, 2560 0.92 ms; 5120 keys 1.14 ms.)
template <class K, bool HV>
__global__ __launch_bounds__(TR_NW * WAVE, HV ? 1 : (sizeof(K) == 4 ? 8 : 7))
void k_transpose(Batch<K> b, const K *src, const uint32_t *vsrc, K *dst, uint32_t *vdst)
{
    __shared__ TileSmem<K> sm;
    tables_clear<TR_NW, TB>(sm.tab);
    transpose_tile<K, HV>(b, src, vsrc, dst, vdst, sm, blockIdx.x, TR_SEQ, 0u);
}

// The chunks of the heavy tiles, taken in ticket order by TR_EXTRA
// persistent work-groups (after k_transpose).
template <class K, bool HV>
__global__ __launch_bounds__(TR_NW * WAVE) void k_transpose_heavy(Batch<K> b, const K *src, const uint32_t *vsrc,
                                                                  K *dst, uint32_t *vdst, uint32_t tiles)
{
    __shared__ TileSmem<K> sm;
    __shared__ uint32_t item_sh;
    const uint32_t cnt = min(b.ctr[CTR_TR_ITEMS], b.trCap);
    if (cnt == 0) return;
    tables_clear<TR_NW, TB>(sm.tab);
    while (true) {
        if (threadIdx.x == 0) item_sh = atomicAdd(&b.ctr[CTR_TR_TAKE], 1u);
        __syncthreads();
        const uint32_t it = item_sh;
        __syncthreads();
        if (it >= cnt) break;
        const uint32_t tile = b.trItem[2 * it];
        if (tile >= tiles) {                       // cannot happen: k_tile_plan writes every item
            if (threadIdx.x == 0) atomicOr(&b.ctr[CTR_TR_FAIL], 1u);
            continue;
        }
        transpose_tile<K, HV>(b, src, vsrc, dst, vdst, sm, tile, it, b.trItem[2 * it + 1]);
    }
}

// ------------------------------------------------------------ nodes with m > SORT_CAP
// Strict flags of sorted pivots (one work-group per listed node).
template <class K>
__global__ void k_strict_flags(Batch<K> b, const uint32_t *nodeList)
{
    const NodeDesc nd = b.nodes[nodeList[blockIdx.x]];
    const uint32_t cnt = nd.m - 1;
    for (uint32_t t = threadIdx.x; t < cnt; t += blockDim.x)
        b.strict[nd.piv + t] = b.alg1 ? 1 : ((t + 1 < cnt && b.piv[nd.piv + t] == b.piv[nd.piv + t + 1]) ? 1 : 0);
}

// Bucket-block offsets of a sorted column in D: srcOff[J][i] = number of keys
// of column i at or below pivot 64J - 1 (binary search in HBM), J = 0..nJ.
// One work-group per (node, column); colStart is the prefix of the listed
// nodes' column counts.
template <class K>
__global__ void k_blockoff(Batch<K> b, const K *D, const uint32_t *nodeList, const uint32_t *colStart,
                           uint32_t nList)
{
    const uint32_t q = find_node(colStart, nList, blockIdx.x);
    const NodeDesc nd = b.nodes[nodeList[q]];
    const uint32_t i = blockIdx.x - colStart[q];
    const uint32_t len = column_len(i, nd.m, nd.n);
    const K *col = D + nd.off + (uint64_t)i * nd.m;
    for (uint32_t J = threadIdx.x; J <= nd.nJ; J += blockDim.x) {
        uint32_t a = 0;
        if (J == nd.nJ) a = len;
        else if (J > 0) {
            const uint32_t t = J * TB - 1;
            const K pv = b.piv[nd.piv + t];
            const bool ps = b.strict[nd.piv + t] != 0;
            uint32_t e = len;
            while (a < e) {
                const uint32_t mid = (a + e) >> 1;
                if (le_pivot(col[mid], pv, ps)) a = mid + 1; else e = mid;
            }
        }
        b.srcOff[nd.src + (uint64_t)J * nd.m + i] = a;
    }
}

// Per (column group, bucket) counts of a node whose columns are sorted in D,
// one work-group per SkewTranspose tile (g, J): the tile's keys are read as
// in k_transpose, each key's bucket found the same way, and the 64 bucket
// counts are LDS atomic adds (commutative: the counts do not depend on
// order).  Tiles of other nodes return at once.
template <class K>
__global__ __launch_bounds__(TR_NW * WAVE) void k_tilecount(Batch<K> b, const K *src)
{
    __shared__ TileSmem<K> sm;
    __shared__ uint32_t hist[TB];
    using T = KeyT<K>;
    const uint32_t k = find_node(b.tileStart, b.N, blockIdx.x);
    const NodeDesc nd = b.nodes[k];
    if (!(nd.flags & NODE_HUGE)) return;
    const uint32_t tix = blockIdx.x - b.tileStart[k];
    const uint32_t g = tix / nd.nJ, J = tix % nd.nJ;
    const uint32_t m = nd.m;
    const uint32_t i0 = g * TG, ncol = min((uint32_t)TG, m - i0);
    const uint32_t j0 = J * TB, nb = min((uint32_t)TB, m - j0);
    const uint32_t npv = (j0 + nb <= m - 1) ? nb : nb - 1;
    const uint32_t tid = threadIdx.x;
    const uint32_t l = lane_id(), w = wave_id();
    if (tid < WAVE) {
        uint32_t a = 0, len = 0;
        if (tid < ncol) {
            a = b.srcOff[nd.src + (uint64_t)J * m + i0 + tid];
            len = b.srcOff[nd.src + (uint64_t)(J + 1) * m + i0 + tid] - a;
        }
        const uint32_t incl = wave_incl_scan(len);
        if (tid < ncol) {
            sm.cOff[tid] = incl - len;
            sm.relBase[tid] = (i0 + tid) * m + a - (incl - len);     // mod 2^32; the true value is < n
        }
        if (tid == ncol - 1) sm.cOff[ncol] = incl;
    }
    if (tid < TB) hist[tid] = 0;
    const K lo = j0 > 0 ? b.piv[nd.piv + j0 - 1] : (K)0;
    const int sh = tile_table(b, nd, j0, npv, lo, sm);
    const uint32_t N = sm.cOff[ncol];
    for (uint32_t q0 = 0; q0 < N; q0 += TR_CH) {
        const uint32_t chN = min((uint32_t)TR_CH, N - q0);
        for (uint32_t c = w; c < ncol; c += TR_NW) {
            const uint32_t s0 = max(sm.cOff[c], q0), s1 = min(sm.cOff[c + 1], q0 + chN);
            for (uint32_t q = s0 + l; q < s1; q += WAVE) sm.colOf[q - q0] = (uint8_t)c;
        }
        __syncthreads();
        for (uint32_t p = tid; p < chN; p += TR_NW * WAVE) {
            const uint32_t c = sm.colOf[p];
            const uint32_t rel = sm.relBase[c] + q0 + p;
            const K x = src[nd.off + (rel < nd.n ? rel : 0u)];     // guard: inside the node
            atomicAdd(&hist[tile_bucket(x, lo, sh, sm)], 1u);
        }
        __syncthreads();
    }
    if (tid < nb) b.blk[nd.blk + (uint64_t)g * m + j0 + tid] = hist[tid];
}

// ------------------------------------------------------------ digest
// H_node = sum_r sm64(x_r ^ sm64(r)) over the node's post-transpose array.
template <class K, bool HV>
__global__ void k_digest(Batch<K> b, const K *A, const uint32_t *VA)
{
    constexpr uint32_t CHUNK = 16384;
    const uint32_t k = find_node(b.digStart, b.N, blockIdx.x);
    const NodeDesc nd = b.nodes[k];
    const uint32_t c = blockIdx.x - b.digStart[k];
    const uint32_t r0 = c * CHUNK, r1 = min(nd.n, r0 + CHUNK);
    unsigned long long s = 0;
    for (uint32_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        uint64_t x = (uint64_t)A[nd.off + r];
        if (HV) x ^= splitmix((uint64_t)VA[nd.off + r]);
        s += splitmix(x ^ splitmix((uint64_t)r));
    }
    s = wave_sum_u64(s);
    if (lane_id() == 0) atomicAdd(&b.H[k], s);
}

template <class K>
__global__ void k_digest_finish(Batch<K> b, unsigned long long *digest)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= b.N) return;
    atomicAdd(digest, (unsigned long long)splitmix(b.nodes[k].key ^ b.H[k]));
}

// ------------------------------------------------------------ bucket phase
// Inclusive key bounds of bucket j: U_j = s_j, or s_j - 1 for a strict
// pivot, U_{m-1} = max; L_j = s_{j-1} + 1, or s_{j-1} after a strict pivot,
// L_0 = 0.  A non-empty bucket with L_j = U_j admits exactly one key value
// (the appendix copies such buckets instead of recursing).
template <class K>
__device__ inline void bucket_bounds(const Batch<K> &b, const NodeDesc &nd, uint32_t j, K &lo, K &hi)
{
    const bool hasLo = j > 0, hasHi = j + 1 < nd.m;
    K sl = (K)0, sh = (K)0;
    uint8_t tl = 1, th = 1;
    if (hasLo) { sl = b.piv[nd.piv + j - 1]; tl = b.strict[nd.piv + j - 1]; }
    if (hasHi) { sh = b.piv[nd.piv + j]; th = b.strict[nd.piv + j]; }
    lo = hasLo ? (tl ? sl : (K)(sl + 1)) : (K)0;
    hi = hasHi ? (th ? (K)(sh - 1) : sh) : (K)KeyT<K>::MAXV;
}

// ---- validation (SQS_FLAG_VALIDATE)
// Sets *flag when some x[p] > x[p+1] with p and p+1 in the same segment of
// seg keys (seg = the column length for columns, n for a whole output).
template <class K>
__global__ void k_check_sorted(const K *x, uint64_t n, uint64_t seg, uint32_t *flag)
{
    bool bad = false;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p + 1 < n; p += (uint64_t)gridDim.x * blockDim.x)
        if ((p + 1) % seg != 0 && x[p] > x[p + 1]) bad = true;
    if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(flag, 1u);
}

// The SkewTranspose output of the batch's only node against its bucket
// bounds: bs[0] = 0, bs[m] = n, bs non-decreasing, and every key of bucket j
// inside [L_j, U_j].  Sets ctr[CTR_CHECK_FAIL] otherwise.
template <class K>
__global__ void k_check_buckets(Batch<K> b, const K *out)
{
    const NodeDesc nd = b.nodes[0];
    const uint32_t *bs = b.bs + nd.bkt;
    bool bad = false;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t j = t0; j < nd.m; j += stride) bad |= bs[j] > bs[j + 1];
    if (t0 == 0) bad |= bs[0] != 0u || bs[nd.m] != nd.n;
    for (uint64_t p = t0; p < nd.n; p += stride) {
        uint32_t lo = 0, hi = nd.m;                       // last j with bs[j] <= p
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (bs[mid] <= p) lo = mid; else hi = mid;
        }
        K L, U;
        bucket_bounds(b, nd, lo, L, U);
        const K x = out[nd.off + p];
        bad |= x < L || x > U;
    }
    if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(&b.ctr[CTR_CHECK_FAIL], 1u);
}

// Classify every bucket and append it to its work list.  Appends are
// counted per wave (ballots), then per work-group in LDS, and take one global
// atomic per class and work-group (list order does not affect any result).
template <class K>
__global__ __launch_bounds__(CL_NT) void k_classify(Batch<K> b, uint32_t cutoff)
{
    __shared__ uint32_t wgCnt[NCLS], wgBase[NCLS];
    __shared__ unsigned long long wgKeys[NCLS];
    const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
    if (threadIdx.x < NCLS) { wgCnt[threadIdx.x] = 0; wgKeys[threadIdx.x] = 0; }
    __syncthreads();
    int cls = -1;
    BucketItem it{0, 0, 0, 0};
    K blo = (K)0, bhi = (K)0;
    uint64_t base = 0;
    if (item < b.bucStart[b.N]) {
        const uint32_t k = find_node(b.bucStart, b.N, item);
        const NodeDesc nd = b.nodes[k];
        const uint32_t j = item - b.bucStart[k];
        const uint32_t lo = b.bs[nd.bkt + j], s = b.bs[nd.bkt + j + 1] - lo;
        it = BucketItem{k, j, lo, s};
        if (s > 0) {
            bucket_bounds(b, nd, j, blo, bhi);
            base = nd.off + lo;
            if (blo == bhi) cls = CLS_COPY;
            else if (s > cutoff) cls = CLS_INTERNAL;
            else if (s <= b.wcap) cls = CLS_SMALL;
            else if (s <= b.m4cap) cls = CLS_MID4;
            else if (s <= (uint32_t)SORT_CAP) cls = CLS_MID;
            else cls = CLS_BIG;
        }
    }
    const uint32_t l = lane_id();
    // single-value buckets are copied in pieces of at most COPY_CH keys
    const uint32_t pieces = cls == CLS_COPY ? (it.size + COPY_CH - 1) / COPY_CH : 0u;
    const uint32_t pincl = wave_incl_scan(pieces);
    const uint32_t ptot = __shfl(pincl, WAVE - 1, WAVE);
    uint32_t woff[NCLS] = {};                             // this wave's first slot in the work-group's run
    if (ptot > 0 && l == 0) woff[CLS_COPY] = atomicAdd(&wgCnt[CLS_COPY], ptot);
    woff[CLS_COPY] = __shfl(woff[CLS_COPY], 0, WAVE);
    unsigned long long mask[NCLS];
#pragma unroll
    for (int c = 0; c < NCLS; ++c) {
        const unsigned long long ks = wave_sum_u64(cls == c ? it.size : 0u);   // keys per class (measurement)
        if (ks && l == 0) atomicAdd(&wgKeys[c], ks);
        mask[c] = __ballot(cls == c);
        if (c == CLS_COPY) continue;
        uint32_t o = 0;
        if (mask[c] && l == 0) o = atomicAdd(&wgCnt[c], (uint32_t)__popcll(mask[c]));
        woff[c] = __shfl(o, 0, WAVE);
    }
    // buckets the wide-bucket kernel may take (counted for every key type)
    const unsigned long long wide = __ballot(cls == CLS_BIG && it.size <= WIDE_CAP &&
                                             (uint64_t)(K)(bhi - blo) >= (uint64_t)WIDE_RANGE);
    if (wide && l == 0) atomicAdd(&b.ctr[CTR_WIDE_ELIG], (uint32_t)__popcll(wide));
    __syncthreads();
    if (threadIdx.x < NCLS) {
        const uint32_t c = threadIdx.x;
        wgBase[c] = wgCnt[c] ? atomicAdd(&b.ctr[c], wgCnt[c]) : 0u;
        if (wgKeys[c]) atomicAdd(&b.ctr[2 * NCLS + c], (uint32_t)wgKeys[c]);
    }
    __syncthreads();
    if (pieces > 0) {
        const uint32_t at0 = wgBase[CLS_COPY] + woff[CLS_COPY] + pincl - pieces;
        for (uint32_t q = 0; q < pieces; ++q) {
            const uint32_t off = q * COPY_CH;
            if (at0 + q < b.cap[CLS_COPY])
                b.list[CLS_COPY][at0 + q] = BucketItem{it.node, it.j, it.lo + off, min(COPY_CH, it.size - off)};
        }
    }
#pragma unroll
    for (int c = 1; c < NCLS; ++c) {
        if (cls == c) {
            const uint32_t at = wgBase[c] + woff[c] + rank_in_mask((uint32_t)mask[c], (uint32_t)(mask[c] >> 32));
            if (at < b.cap[c]) {
                b.list[c][at] = it;
                if (b.span[c]) b.span[c][at] = Span<K>{base, it.size, 0u, blo, bhi};
            }
        }
    }
}

// Single-value buckets: A -> D (one work-group per piece of at most COPY_CH
// keys, persistent); the keys are written from the piece's first key, the
// values copied.
template <class K, bool HV>
__global__ __launch_bounds__(CP_NT) void k_bucket_copy(Batch<K> b, const K *A, const uint32_t *VA, K *D, uint32_t *VD)
{
    const uint32_t cnt = min(b.ctr[CLS_COPY], b.cap[CLS_COPY]);
    constexpr uint32_t U = 8;                        // loads in flight per thread
    for (uint32_t it = blockIdx.x; it < cnt; it += gridDim.x) {
        const BucketItem e = b.list[CLS_COPY][it];
        const uint64_t base = b.nodes[e.node].off + e.lo;
        if (e.size == 0) continue;
        // every key of the piece is the bucket's one value: it is read once,
        // only the values are copied
        const K key = A[base];
        for (uint32_t p0 = 0; p0 < e.size; p0 += CP_NT * U) {
            uint32_t y[U];
            if (HV) {
#pragma unroll
                for (uint32_t u = 0; u < U; ++u) {
                    const uint32_t p = p0 + u * CP_NT + threadIdx.x;
                    if (p < e.size) y[u] = VA[base + p];
                }
                wait_vmem();
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t p = p0 + u * CP_NT + threadIdx.x;
                if (p < e.size) { D[base + p] = key; if (HV) VD[base + p] = y[u]; }
            }
        }
    }
}

// Buckets of at most WCAP keys: one wave per bucket (persistent).
template <class K, bool HV>
__global__ __launch_bounds__(SM_NW * WAVE) void k_bucket_small(Batch<K> b, const K *A, const uint32_t *VA,
                                                               K *D, uint32_t *VD)
{
    __shared__ WaveSmem<WR> wsm[SM_NW];
    const uint32_t w = wave_id(), l = lane_id();
    const uint32_t cnt = min(b.ctr[CLS_SMALL], b.cap[CLS_SMALL]);
    if (blockIdx.x * SM_NW + w >= cnt) return;      // no item for this wave
    wave_table_clear(wsm[w].tab);
    wave_lds_sync();
    for (uint32_t it = blockIdx.x * SM_NW + w; it < cnt; it += gridDim.x * SM_NW) {
        const BucketItem e = b.list[CLS_SMALL][it];
        const uint64_t base = b.nodes[e.node].off + e.lo;
        K kk[WR];
        uint32_t vv[WR];
#pragma unroll
        for (int r = 0; r < WR; ++r) {
            const uint32_t p = r * WAVE + l;
            kk[r] = p < e.size ? A[base + p] : (K)0;
            if (HV) vv[r] = p < e.size ? VA[base + p] : 0u;
        }
        // 32-bit keys without values: bins, radix passes for a crowded bin
        // (after clearing the table the bin sort used)
        bool radix = true;
        if constexpr (sizeof(K) == 4 && !HV) {
            uint32_t blo, nbin;
            int bsh;
            const int res = wave_bin_sort<WR>(kk, e.size, wsm[w], blo, bsh, nbin);
            radix = res == 2;
            if (radix) {
                wave_table_clear(wsm[w].tab);
                wave_lds_sync();
            }
        }
        if (radix) wave_sort<K, HV, WR>(kk, vv, e.size, wsm[w]);
#pragma unroll
        for (int r = 0; r < WR; ++r) {
            const uint32_t p = r * WAVE + l;
            if (p < e.size) {
                D[base + p] = kk[r];
                if (HV) VD[base + p] = vv[r];
            }
        }
    }
}


// Claim order of the mid (block 0) and big (block 1) spans: largest items
// first, written as a permuted copy.  Work-groups take items one at a time, so taking them in
// decreasing size (longest-processing-time order) makes the work-groups that
// take the last items finish close together; in list order a large bucket
// taken late sets the end of the whole kernel.  Sizes are counting-sorted
// into 256 bins of 2^shift keys; the order inside a bin is whatever the
// atomics give, and no output depends on it.
template <class K>
__global__ __launch_bounds__(1024) void k_order_lists(Batch<K> b, uint32_t shiftMid, uint32_t shiftBig)
{
    __shared__ uint32_t at[256];
    const int c = blockIdx.x == 0 ? CLS_MID : CLS_BIG;
    const uint32_t shift = blockIdx.x == 0 ? shiftMid : shiftBig;
    Span<K> *ord = b.ord[c];
    if (!ord) return;
    const uint32_t tid = threadIdx.x;
    const uint32_t cnt = min(b.ctr[c], b.cap[c]);
    const Span<K> *sp = b.span[c];
    if (tid < 256) at[tid] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < cnt; i += blockDim.x)                  // bin 0 holds the largest sizes
        atomicAdd(&at[255u - min((sp[i].size - 1u) >> shift, 255u)], 1u);
    __syncthreads();
    if (tid < WAVE) {                                                  // exclusive scan, 4 bins a lane
        uint32_t v[4], t4 = 0;
        for (int q = 0; q < 4; ++q) { v[q] = at[4 * tid + q]; t4 += v[q]; }
        uint32_t r0 = wave_incl_scan(t4) - t4;
        for (int q = 0; q < 4; ++q) { at[4 * tid + q] = r0; r0 += v[q]; }
    }
    __syncthreads();
    for (uint32_t i = tid; i < cnt; i += blockDim.x) {
        const Span<K> e = sp[i];
        ord[atomicAdd(&at[255u - min((e.size - 1u) >> shift, 255u)], 1u)] = e;
    }
}

// Buckets of one LDS sort: one work-group of NW waves per bucket
// (persistent), of class CLS (mid4: 4 waves, up to M4_CAP keys, several
// work-groups per CU; mid: 16 waves, up to SORT_CAP keys).
// 64-bit keys in the 16-wave class: buckets up to the merge capacity by the
// LDS merge sort (its arrays over the radix sort's LDS), larger ones by radix
// passes.
template <class K, bool HV, int NW> struct MidSmem {
    static constexpr bool MG = false;
    SortSmem<NW, SORT_IPT> sort;
};
template <bool HV> struct MidSmem<uint64_t, HV, SORT_NW> {
    static constexpr bool MG = true;
    union {
        SortSm sort;
        MergeSm<HV> mg;
    };
};

template <class K, bool HV, int NW, int CLS>
__global__ __launch_bounds__(NW * WAVE, 4) void k_bucket_mid(Batch<K> b, const K *A, const uint32_t *VA,
                                                          K *D, uint32_t *VD)
{
    __shared__ MidSmem<K, HV, NW> msm;
    SortSmem<NW, SORT_IPT> &sm = msm.sort;
    __shared__ uint32_t take_sh;
    const uint32_t cnt = min(b.ctr[CLS], b.cap[CLS]);
    uint32_t it = take_item(b.ctr, CLS, &take_sh);
    if (it >= cnt) return;                           // no item left: skip the table clear
    tables_clear<NW, 256>(sm.s.tab);
    __syncthreads();
    bool dirty = false;                              // a merge sort has used the tables' LDS
    for (; it < cnt; it = take_item(b.ctr, CLS, &take_sh)) {
        const Span<K> e = b.ord[CLS] ? b.ord[CLS][it] : b.span[CLS][it];
        const uint64_t base = e.base;
        const K blo = e.lo, bhi = e.hi;
        if constexpr (MidSmem<K, HV, NW>::MG) {
            if (e.size <= (uint32_t)MergeCap<HV>::CAP) {
                merge_segment<HV, MergeCap<HV>::IPT, NW * WAVE>(A + base, HV ? VA + base : nullptr, D + base,
                                                               HV ? VD + base : nullptr, e.size, msm.mg.k,
                                                               msm.mg.v);
                dirty = true;
                __syncthreads();
                continue;
            }
            if (dirty) {
                tables_clear<NW, 256>(sm.s.tab);
                __syncthreads();
                dirty = false;
            }
        }
        K kk[SORT_IPT];
        uint32_t vv[SORT_IPT];
        const int R = block_rows<NW, SORT_IPT>(e.size);
#pragma unroll
        for (int r = 0; r < SORT_IPT; ++r) {
            const uint32_t p = bpos(r, R);
            kk[r] = r < R && p < e.size ? A[base + p] : (K)0;
            if (HV) vv[r] = r < R && p < e.size ? VA[base + p] : 0u;
        }
        wait_vmem();
        lds_sort<K, HV, NW, SORT_IPT>(kk, vv, e.size, sm, blo, bhi, A + base);
#pragma unroll
        for (int r = 0; r < SORT_IPT; ++r) {
            const uint32_t p = bpos(r, R);
            if (r < R && p < e.size) {
                D[base + p] = kk[r];
                if (HV) VD[base + p] = vv[r];
            }
        }
        __syncthreads();
    }
}


// Buckets of CAP+1 .. cutoff keys (a base case larger than one LDS sort):
// one work-group per bucket (persistent) runs an MSD radix split through
// global memory and sorts the parts in LDS.  A split counts the top bits of
// (x - lo) over the segment, then scatters it stably (chunks in order, LDS
// ranking inside a chunk) into the other buffer; parts that fit one LDS sort
// are sorted into D in place, larger ones are split again (A and D alternate
// as source and target), single-value parts are copied.  The result is the
// stable sort of the bucket, as any base-case sort must produce.
struct BigSeg {
    uint32_t off, size;          // bucket-relative
    uint32_t in_d;               // segment currently lives in D (else in A)
    uint32_t pad;
    uint64_t lo, hi;             // inclusive key range of the segment
};
// The MSD-split kernel runs half-size work-groups (8 waves, 8192-key LDS
// sorts, about 76 KB of LDS) so that two share a CU and one's global-memory
// phases overlap the other's LDS work.
constexpr int BK_NW = 8;
constexpr int BK_IPT = 16;
constexpr int BK_NT = BK_NW * WAVE;
constexpr int BK_CAP = BK_NT * BK_IPT;          // 8192 keys per LDS sort
using BigSm = SortSmem<BK_NW, BK_IPT>;
constexpr int BIG_STACK = 256;
constexpr int SPLIT_MAX = 4;                 // at most 16 parts per split
constexpr uint32_t SPLIT_PART = 6144;        // aimed part size (fits one LDS sort with room)

// Radix sort of a part of 32-bit keys without values whose bin sort found a
// crowded bin: from[0 .. size) -> to[0 .. size), keys in [lo, hi].  Not
// inlined, so that its registers are allocated apart from the bin sort's
// (both sorts inlined into one kernel spill).  All threads call it.
__device__ __noinline__ void big_leaf_radix(const uint32_t *from, uint32_t *to, uint32_t size, uint32_t lo,
                                            uint32_t hi, BigSm &sm)
{
    uint32_t kk[BK_IPT], vv[BK_IPT];
    block_load<uint32_t, false, BK_NW, BK_IPT>(kk, vv, size, from, nullptr);
    tables_clear<BK_NW, 256>(sm.s.tab);
    __syncthreads();
    block_sort<uint32_t, false, BK_NW, BK_IPT>(kk, vv, size, sm, true, lo, hi);
    const int R = block_rows<BK_NW, BK_IPT>(size);
#pragma unroll
    for (int r = 0; r < BK_IPT; ++r) {
        const uint32_t p = bpos(r, R);
        if (r < R && p < size) to[p] = kk[r];
    }
}

// Leaves of 64-bit keys: the stable LDS merge sort (runs of IPT keys, BK_NT
// threads) for parts of at most BK_NT * IPT keys (5632 with values, 7680
// without), over the same LDS as the radix sort and small enough for two
// work-groups per CU.
template <bool HV> struct BigMergeSm {
    static constexpr int IPT = HV ? 11 : 15;
    static constexpr int CAP = BK_NT * IPT;
    uint64_t k[CAP];
    uint32_t v[HV ? CAP : 1];
};
template <class K, bool HV> struct BigSmem {
    BigSm sort;
};
template <bool HV> struct BigSmem<uint64_t, HV> {
    union {
        BigSm sort;
        BigMergeSm<HV> mg;
    };
};
static_assert(sizeof(BigSmem<uint64_t, true>) <= 70 * 1024 && sizeof(BigSmem<uint64_t, false>) <= 70 * 1024,
              "two work-groups per CU with the kernel's other shared arrays");

// Leaves of 64-bit keys above the merge capacity: radix passes, in a
// function that is not inlined (its registers apart from the kernel's).
template <bool HV>
__device__ __noinline__ void big_leaf_radix64(const uint64_t *from, const uint32_t *vfrom, uint64_t *to,
                                              uint32_t *vto, uint32_t size, uint64_t lo, uint64_t hi, BigSm &sm)
{
    uint64_t kk[BK_IPT];
    uint32_t vv[BK_IPT];
    block_load<uint64_t, HV, BK_NW, BK_IPT>(kk, vv, size, from, vfrom);
    tables_clear<BK_NW, 256>(sm.s.tab);
    __syncthreads();
    block_sort<uint64_t, HV, BK_NW, BK_IPT>(kk, vv, size, sm, true, lo, hi);
    const int R = block_rows<BK_NW, BK_IPT>(size);
#pragma unroll
    for (int r = 0; r < BK_IPT; ++r) {
        const uint32_t p = bpos(r, R);
        if (r < R && p < size) {
            to[p] = kk[r];
            if (HV) vto[p] = vv[r];
        }
    }
}

// Part statistics of one 64-key row for at most 2^SPLIT_MAX parts, from
// SPLIT_MAX ballots of the part bits (valid lanes only): `mine` = the valid
// lanes whose part equals this lane's part d, `lanes_j` = the valid lanes of
// part j = this lane's index (meaningful for lanes below 2^SPLIT_MAX).
__device__ inline void part_masks(bool ok, uint32_t d, unsigned long long &mine, unsigned long long &lanes_j)
{
    const uint32_t l = lane_id();
    unsigned long long me = __ballot(ok), mj = me;
#pragma unroll
    for (int k = 0; k < SPLIT_MAX; ++k) {
        const unsigned long long bk = __ballot(ok && ((d >> k) & 1u));
        me &= ((d >> k) & 1u) ? bk : ~bk;
        mj &= ((l >> k) & 1u) ? bk : ~bk;
    }
    mine = me;
    lanes_j = mj;
}

// (not inlined either: the split's registers stay apart from the sort's)
template <bool HV>
__device__ __noinline__ void big_leaf_merge(const uint64_t *from, const uint32_t *vfrom, uint64_t *to, uint32_t *vto,
                                            uint32_t size, BigMergeSm<HV> &mg)
{
    merge_segment<HV, BigMergeSm<HV>::IPT, BK_NT>(from, vfrom, to, vto, size, mg.k, mg.v);
}

// Buckets of 32-bit keys without values from one LDS sort up to WIDE_CAP keys
// (base cases, taken from the small end of the MSD-split list before the
// MSD-split kernel runs): the whole bucket sits in LDS (the CU's 160 KB) and
// one bin sort of WBINS bins orders it, so every key is read and written
// once, where the split reads it three times and writes it twice.  The bins
// cut the bucket's key range [lo, hi] into WBINS intervals by a fixed-point
// multiply (bin = (x - lo) * mul / 2^32, non-decreasing in x; for a range of
// fewer than WBINS values, one bin per value, which needs no sort): about 2
// to 3.5 keys a bin for uniform keys.  Every key takes its slot in its bin
// from an LDS atomic add, the bins are laid out by a scan, and every bin of
// at most BIN_NET keys is sorted in place by a sorting network.  A bucket with
// a bin of more keys (clustered keys), or with a key range of fewer than
// WIDE_RANGE values, is left untouched to the MSD-split kernel; a sorted one
// has the size of its list entry set to zero, which that kernel skips.  Items
// are claimed from the end of the list, which is ordered largest first,
// until one exceeds WIDE_CAP.
static_assert(WIDE_RANGE == 1u << SPLIT_MAX, "one MSD split pass separates a smaller range's values");
constexpr int WIDE_IPT = (int)WIDE_CAP / SORT_NT;     // 28 keys per thread
constexpr int WBINS = 8192;
constexpr int WBPT = WBINS / SORT_NT;                 // 8 bins per thread
static_assert(WIDE_IPT * SORT_NT == (int)WIDE_CAP && WBPT * SORT_NT == WBINS, "whole rows and bins per thread");
struct WideSmem {
    uint32_t buf[WIDE_CAP + BIN_NET];   // the keys, then all-ones words under the networks' last reads
    uint32_t st[WBINS + 1];             // bin counts, then bin starts (st[WBINS] = size)
    uint32_t wsum[SORT_NW];
    uint32_t wflag[SORT_NW];
    uint2 bl[SORT_NW][64];              // per wave: bins of 9 .. BIN_NET keys (start, size)
};

__global__ __launch_bounds__(SORT_NT, 1) void k_bucket_wide(Batch<uint32_t> b, const uint32_t *A, uint32_t *D)
{
    __shared__ WideSmem sm;
    __shared__ uint32_t take_sh;
    const uint32_t tid = threadIdx.x, w = wave_id(), l = lane_id();
    const uint32_t cnt = min(b.ctr[CLS_BIG], b.cap[CLS_BIG]);
    Span<uint32_t> *list = b.ord[CLS_BIG];
    if (b.ctr[CTR_WIDE_ELIG] == 0) return;           // no bucket to take (say, few key values)
    while (true) {
        if (tid == 0) take_sh = atomicAdd(&b.ctr[CTR_WIDE_TAKE], 1u);
        __syncthreads();
        const uint32_t k = take_sh;
        __syncthreads();
        if (k >= cnt) break;
        const uint32_t it = cnt - 1u - k;
        const Span<uint32_t> e = list[it];
        if (e.size > WIDE_CAP) break;                 // every later claim is at least as large
        // a range of fewer values: one pass of the MSD split separates the
        // values without sorting (the bins' atomic adds would collide on a
        // few words)
        if (e.size == 0 || e.hi - e.lo < WIDE_RANGE) continue;
        const uint64_t base = e.base;
        const uint32_t size = e.size, lo = e.lo, range = e.hi - e.lo;
        const bool one = range < (uint32_t)WBINS;     // one key value per bin
        const uint32_t mul = one ? 0u : (uint32_t)(((uint64_t)WBINS << 32) / ((uint64_t)range + 1u));
        auto bin = [&](uint32_t x) { return one ? x - lo : __umulhi(x - lo, mul); };
#pragma unroll
        for (int q = 0; q < WBPT; ++q) sm.st[q * SORT_NT + tid] = 0u;
        uint32_t x[WIDE_IPT], rk[WIDE_IPT];
#pragma unroll
        for (int r = 0; r < WIDE_IPT; ++r) {          // the loads first, in flight together
            const uint32_t p = (uint32_t)r * SORT_NT + tid;
            x[r] = p < size ? A[base + p] : 0u;
        }
        wait_vmem();
        __syncthreads();
#pragma unroll
        for (int r = 0; r < WIDE_IPT; ++r)
            if ((uint32_t)r * SORT_NT + tid < size) rk[r] = atomicAdd(&sm.st[bin(x[r])], 1u);
        __syncthreads();
        // bins WBPT*t .. WBPT*t + WBPT - 1: counts, crowding, exclusive starts
        uint32_t c[WBPT], tot = 0u;
        bool crowded = false;
#pragma unroll
        for (int q = 0; q < WBPT; ++q) {
            c[q] = sm.st[WBPT * tid + q];
            tot += c[q];
            crowded |= c[q] > (uint32_t)BIN_NET;
        }
        const uint32_t incl = wave_incl_scan(tot);
        const bool over = !one && __ballot(crowded) != 0ull;
        if (l == WAVE - 1) { sm.wsum[w] = incl; sm.wflag[w] = over ? 1u : 0u; }
        __syncthreads();
        uint32_t run = incl - tot;
        bool any = false;
#pragma unroll
        for (int ww = 0; ww < SORT_NW; ++ww) {
            if ((uint32_t)ww < w) run += sm.wsum[ww];
            any |= sm.wflag[ww] != 0u;
        }
        if (any) {                                    // uniform: left to the MSD split
            __syncthreads();
            continue;
        }
#pragma unroll
        for (int q = 0; q < WBPT; ++q) { sm.st[WBPT * tid + q] = run; run += c[q]; }
        if (tid == 0) sm.st[WBINS] = size;
        if (tid < (uint32_t)BIN_NET) sm.buf[size + tid] = 0xFFFFFFFFu;   // at least every key
        __syncthreads();
#pragma unroll
        for (int r = 0; r < WIDE_IPT; ++r)
            if ((uint32_t)r * SORT_NT + tid < size) sm.buf[sm.st[bin(x[r])] + rk[r]] = x[r];
        __syncthreads();
        if (!one) {
            // bins of at most 8 keys by 4- or 8-key networks (as large as the
            // wave's largest such bin needs), then the wave's larger bins,
            // listed, one per lane by 16-key networks
            uint32_t bigit = 0u;
#pragma unroll 1
            for (int q = 0; q < WBPT; ++q) {
                const uint32_t bb = tid + (uint32_t)q * SORT_NT;
                const uint32_t s = sm.st[bb], cb = sm.st[bb + 1] - s;
                const bool big = cb > 8u;
                bigit |= (big ? 1u : 0u) << q;
                const uint32_t cs = big ? 0u : cb;
                const uint32_t cm = wave_max(cs);
                if (cm <= 1u) continue;
                if (cm <= 4u) bin_net<4>(sm.buf, s, cs);
                else bin_net<8>(sm.buf, s, cs);
            }
            const uint32_t nbig = (uint32_t)__popc(bigit);
            const uint32_t bincl = wave_incl_scan(nbig);
            const uint32_t btot = __shfl(bincl, WAVE - 1, WAVE);
            if (btot > 0u) {
                if (btot <= 64u) {
                    uint2 *bl = sm.bl[w];
                    uint32_t o = bincl - nbig;
#pragma unroll 1
                    for (int q = 0; q < WBPT; ++q)
                        if ((bigit >> q) & 1u) {
                            const uint32_t bb = tid + (uint32_t)q * SORT_NT;
                            bl[o++] = make_uint2(sm.st[bb], sm.st[bb + 1] - sm.st[bb]);
                        }
                    wave_lds_sync();
                    if (l < btot) {
                        const uint2 e2 = bl[l];
                        bin_net<16>(sm.buf, e2.x, e2.y);
                    }
                } else {
#pragma unroll 1
                    for (int q = 0; q < WBPT; ++q) {
                        if (__ballot((bigit >> q) & 1u) == 0ull) continue;
                        const uint32_t bb = tid + (uint32_t)q * SORT_NT;
                        const bool big = (bigit >> q) & 1u;
                        bin_net<16>(sm.buf, big ? sm.st[bb] : 0u, big ? sm.st[bb + 1] - sm.st[bb] : 0u);
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < WIDE_IPT; ++r) {
            const uint32_t p = (uint32_t)r * SORT_NT + tid;
            if (p < size) D[base + p] = sm.buf[p];
        }
        if (tid == 0) {
            list[it].size = 0u;                       // done: the MSD-split kernel skips it
            atomicAdd(&b.ctr[CTR_WIDE_KEYS], size);
        }
        __syncthreads();
    }
}

template <class K, bool HV>
__global__ __launch_bounds__(BK_NT, 4) void k_bucket_big(Batch<K> b, K *A, uint32_t *VA, K *D, uint32_t *VD)
{
    using T = KeyT<K>;
    __shared__ BigSmem<K, HV> bsm;
    BigSm &sm = bsm.sort;
    __shared__ BigSeg stack[BIG_STACK];
    __shared__ uint32_t hist[256], base[256], run[256];
    __shared__ uint32_t whist[BK_NW][1 << SPLIT_MAX];
    __shared__ uint32_t ccnt[1 << SPLIT_MAX], coff[1 << SPLIT_MAX];
    __shared__ uint32_t sp_sh, overflow_sh;
    const uint32_t tid = threadIdx.x;
    __shared__ uint32_t take_sh;
    const uint32_t cnt = min(b.ctr[CLS_BIG], b.cap[CLS_BIG]);
    for (uint32_t it = take_item(b.ctr, CLS_BIG, &take_sh); it < cnt; it = take_item(b.ctr, CLS_BIG, &take_sh)) {
        const Span<K> e = b.ord[CLS_BIG] ? b.ord[CLS_BIG][it] : b.span[CLS_BIG][it];
        if (e.size == 0) continue;                   // sorted by k_bucket_wide
        const uint64_t bbase = e.base;
        if (tid == 0) {
            stack[0] = BigSeg{0u, e.size, b.bigInD, 0u, (uint64_t)e.lo, (uint64_t)e.hi};
            sp_sh = 1;
            overflow_sh = 0;
        }
        __syncthreads();
        while (true) {
            const uint32_t sp = sp_sh;
            if (sp == 0) break;
            const BigSeg sg = stack[sp - 1];
            __syncthreads();
            if (tid == 0) sp_sh = sp - 1;
            K *src = sg.in_d ? D : A;
            uint32_t *vsrc = sg.in_d ? VD : VA;
            const uint64_t sb = bbase + sg.off;
            if (sg.size <= (uint32_t)BK_CAP || sg.lo == sg.hi) {
                if (sg.lo == sg.hi) {                       // one key value: already in order
                    if (!sg.in_d)
                        for (uint32_t p = tid; p < sg.size; p += BK_NT) {
                            D[sb + p] = A[sb + p];
                            if (HV) VD[sb + p] = VA[sb + p];
                        }
                } else if constexpr (sizeof(K) == 8) {
                    if (sg.size <= (uint32_t)BigMergeSm<HV>::CAP)
                        big_leaf_merge<HV>(src + sb, HV ? vsrc + sb : nullptr, D + sb, HV ? VD + sb : nullptr,
                                           sg.size, bsm.mg);
                    else
                        big_leaf_radix64<HV>(src + sb, HV ? vsrc + sb : nullptr, D + sb, HV ? VD + sb : nullptr,
                                             sg.size, (uint64_t)sg.lo, (uint64_t)sg.hi, sm);
                } else {
                    K kk[BK_IPT];
                    uint32_t vv[BK_IPT];
                    tables_clear<BK_NW, 256>(sm.s.tab);
                    const int R = block_rows<BK_NW, BK_IPT>(sg.size);
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r) {
                        const uint32_t p = bpos(r, R);
                        kk[r] = r < R && p < sg.size ? src[sb + p] : (K)0;
                        if (HV) vv[r] = r < R && p < sg.size ? vsrc[sb + p] : 0u;
                    }
                    wait_vmem();
                    __syncthreads();
                    // 32-bit keys without values: bins, and a part with a
                    // crowded bin by the radix passes of big_leaf_radix
                    bool done = true;
                    if constexpr (sizeof(K) == 4 && !HV) {
                        uint32_t blo, nbin;
                        int bsh;
                        if (bin_sort<BK_NW, BK_IPT>(kk, sg.size, sm, blo, bsh, nbin, true, (uint32_t)sg.lo,
                                                    (uint32_t)sg.hi) == 2) {
                            big_leaf_radix(src + sb, D + sb, sg.size, (uint32_t)sg.lo, (uint32_t)sg.hi, sm);
                            done = false;
                        }
                    } else {
                        block_sort<K, HV, BK_NW, BK_IPT>(kk, vv, sg.size, sm, true, (K)sg.lo, (K)sg.hi);
                    }
                    if (done) {
#pragma unroll
                        for (int r = 0; r < BK_IPT; ++r) {
                            const uint32_t p = bpos(r, R);
                            if (r < R && p < sg.size) {
                                D[sb + p] = kk[r];
                                if (HV) VD[sb + p] = vv[r];
                            }
                        }
                    }
                }
                __syncthreads();
                continue;
            }
            // ---- split by the top sbits bits of (x - lo).  A range of at
            // most SPLIT_MAX bits is split into single values (copied, not
            // sorted); otherwise sbits is the fewest bits that give parts of
            // about SPLIT_PART keys (for the merge leaves of 64-bit keys, two
            // thirds of their capacity) and, for 32-bit keys, the fewest
            // 8-bit passes per part that any split of at most SPLIT_MAX bits
            // gives
            K *dstb = sg.in_d ? A : D;
            uint32_t *vdstb = sg.in_d ? VA : VD;
            const K klo = (K)sg.lo;
            const int bits = T::bitlen((K)((K)sg.hi - klo));
            int sbits = bits;
            if (bits > SPLIT_MAX) {
                constexpr uint32_t part = sizeof(K) == 8 ? 2u * BigMergeSm<HV>::CAP / 3u : SPLIT_PART;
                sbits = min(32 - __clz((sg.size - 1) / part), SPLIT_MAX);
                if (sizeof(K) == 4) {
                    const int best = (bits - SPLIT_MAX + 7) / 8;
                    while (sbits < SPLIT_MAX && (bits - sbits + 7) / 8 > best) ++sbits;
                }
            }
            const int shift = bits - sbits;
            const uint32_t nparts = 1u << sbits;
            if (tid < 256) { hist[tid] = 0; run[tid] = 0; }
            if (tid < BK_NW * (1 << SPLIT_MAX)) (&whist[0][0])[tid] = 0;
            __syncthreads();
            {                                                            // count, per-wave histograms
                // 64-bit keys: lane j < 2^SPLIT_MAX counts the wave's keys of
                // part j by row ballots (LDS atomics collide when few parts
                // take most keys, as in duplicate-heavy key sets); 32-bit keys
                // keep the atomics, cheaper when they do not collide
                uint32_t *wh = whist[wave_id()];
                uint32_t wc = 0u;
                for (uint32_t p0 = 0; p0 < sg.size; p0 += BK_CAP) {    // a chunk's loads in flight together
                    K x[BK_IPT];
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r) {
                        const uint32_t p = p0 + r * BK_NT + tid;
                        x[r] = p < sg.size ? src[sb + p] : klo;
                    }
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r) {
                        const bool ok = p0 + r * BK_NT + tid < sg.size;
                        const uint32_t d = min((uint32_t)(((K)(x[r] - klo)) >> shift), nparts - 1);
                        if constexpr (sizeof(K) == 8) {
                            unsigned long long mine, lj;
                            part_masks(ok, d, mine, lj);
                            wc += (uint32_t)__popcll(lj);
                        } else if (ok) {
                            atomicAdd(&wh[d], 1u);
                        }
                    }
                }
                if (sizeof(K) == 8 && lane_id() < (1u << SPLIT_MAX)) wh[lane_id()] = wc;
            }
            __syncthreads();
            if (tid < nparts) {
                uint32_t c = 0;
                for (int w = 0; w < BK_NW; ++w) c += whist[w][tid];
                hist[tid] = c;
            }
            __syncthreads();
            if (tid < WAVE) {                                            // exclusive scan of <= 256 counts
                uint32_t c[4], t4 = 0;
                for (int q = 0; q < 4; ++q) { c[q] = 4 * tid + q < nparts ? hist[4 * tid + q] : 0u; t4 += c[q]; }
                uint32_t r0 = wave_incl_scan(t4) - t4;
                for (int q = 0; q < 4; ++q) { if (4 * tid + q < 256) base[4 * tid + q] = r0; r0 += c[q]; }
            }
            if constexpr (sizeof(K) == 4 && !HV) {
                // keys without values need no stable split: a key's place in
                // its part's run of the chunk comes from an LDS atomic add
                if (tid < (1u << SPLIT_MAX)) ccnt[tid] = 0u;
                __syncthreads();
                for (uint32_t c0 = 0; c0 < sg.size; c0 += BK_CAP) {
                    const uint32_t chN = min((uint32_t)BK_CAP, sg.size - c0);
                    K kk[BK_IPT];
                    uint32_t rk[BK_IPT];
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r) {                  // loads first, in flight together
                        const uint32_t p = item_pos<BK_NW, BK_IPT>(r);
                        kk[r] = p < chN ? src[sb + c0 + p] : (K)0;
                    }
                    wait_vmem();
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r) {
                        const uint32_t p = item_pos<BK_NW, BK_IPT>(r);
                        if (p < chN)
                            rk[r] = atomicAdd(&ccnt[min((uint32_t)(((K)(kk[r] - klo)) >> shift), nparts - 1)], 1u);
                    }
                    __syncthreads();
                    if (tid < WAVE) {                                    // runs of the chunk's parts
                        const uint32_t cc = tid < nparts ? ccnt[tid] : 0u;
                        const uint32_t ex = wave_incl_scan(cc) - cc;
                        if (tid < nparts) coff[tid] = ex;
                    }
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r) {
                        const uint32_t p = item_pos<BK_NW, BK_IPT>(r);
                        if (p < chN) {
                            const uint32_t d = min((uint32_t)(((K)(kk[r] - klo)) >> shift), nparts - 1);
                            sm.s.buf[coff[d] + rk[r]] = (uint32_t)kk[r];
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r) {                  // in chunk order: contiguous runs
                        const uint32_t p = item_pos<BK_NW, BK_IPT>(r);
                        if (p < chN) {
                            const K x = (K)sm.s.buf[p];
                            const uint32_t d = min((uint32_t)(((K)(x - klo)) >> shift), nparts - 1);
                            const uint32_t at = base[d] + run[d] + (p - coff[d]);
                            if (at < sg.size) dstb[sb + at] = x;         // guard: inside the segment
                        }
                    }
                    __syncthreads();
                    if (tid < nparts) { run[tid] += ccnt[tid]; ccnt[tid] = 0u; }
                    __syncthreads();
                }
            } else {
                // stable scatter, chunk by chunk: a key's place among the
                // chunk's keys of its part comes from the wave's row ballots
                // (rows and lanes in input order) and the waves' counts
                for (uint32_t c0 = 0; c0 < sg.size; c0 += BK_CAP) {
                    const uint32_t chN = min((uint32_t)BK_CAP, sg.size - c0);
                    const int nrows = wave_rows<BK_IPT>(chN);
                    const uint32_t w = wave_id(), l = lane_id();
                    K kk[BK_IPT];
                    uint32_t vv[BK_IPT], pos[BK_IPT];
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r) {                      // loads first, in flight together
                        const uint32_t p = item_pos<BK_NW, BK_IPT>(r);
                        kk[r] = r < nrows && p < chN ? src[sb + c0 + p] : (K)0;
                        if (HV) vv[r] = r < nrows && p < chN ? vsrc[sb + c0 + p] : 0u;
                    }
                    wait_vmem();
                    auto part = [&](K x) { return min((uint32_t)(((K)(x - klo)) >> shift), nparts - 1); };
                    uint32_t wc = 0u;                    // lane j: the wave's keys of part j in earlier rows
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r) {
                        if (r < nrows) {
                            const bool ok = item_pos<BK_NW, BK_IPT>(r) < chN;
                            const uint32_t d = part(kk[r]);
                            unsigned long long mine, lj;
                            part_masks(ok, d, mine, lj);
                            pos[r] = __shfl(wc, (int)d, WAVE) + rank_in_mask((uint32_t)mine, (uint32_t)(mine >> 32));
                            wc += (uint32_t)__popcll(lj);
                        }
                    }
                    if (l < (1u << SPLIT_MAX)) whist[w][l] = wc;
                    __syncthreads();
                    // lane j: part j's start in the chunk and this wave's first slot of it
                    uint32_t tot = 0u, pre = 0u;
                    if (l < (1u << SPLIT_MAX)) {
#pragma unroll
                        for (int ww = 0; ww < BK_NW; ++ww) {
                            const uint32_t c = whist[ww][l];
                            tot += c;
                            pre += (uint32_t)ww < w ? c : 0u;
                        }
                    }
                    const uint32_t start = wave_incl_scan(tot) - tot;
                    if (w == 0 && l < (1u << SPLIT_MAX)) { coff[l] = start; ccnt[l] = tot; }
                    const uint32_t first = start + pre;
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r)
                        if (r < nrows) pos[r] += __shfl(first, (int)part(kk[r]), WAVE);
                    // exchange into chunk order by part (valid keys only)
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r)
                        if (r < nrows && item_pos<BK_NW, BK_IPT>(r) < chN) sm.k64[pos[r]] = (uint64_t)kk[r];
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r)
                        if (r < nrows) kk[r] = (K)sm.k64[item_pos<BK_NW, BK_IPT>(r)];
                    __syncthreads();
                    if (HV) {
#pragma unroll
                        for (int r = 0; r < BK_IPT; ++r)
                            if (r < nrows && item_pos<BK_NW, BK_IPT>(r) < chN) sm.s.buf[pos[r]] = vv[r];
                        __syncthreads();
#pragma unroll
                        for (int r = 0; r < BK_IPT; ++r) if (r < nrows) vv[r] = sm.s.buf[item_pos<BK_NW, BK_IPT>(r)];
                        __syncthreads();
                    }
                    // element at chunk position p has part d (recomputed from its key);
                    // it goes to base[d] + run[d] + (p - start of d in this chunk)
#pragma unroll
                    for (int r = 0; r < BK_IPT; ++r) {
                        if (r < nrows) {
                            const uint32_t p = item_pos<BK_NW, BK_IPT>(r);
                            if (p < chN) {
                                const uint32_t d = part(kk[r]);
                                const uint32_t at = base[d] + run[d] + (p - coff[d]);
                                if (at < sg.size) {                                  // guard: inside the segment
                                    dstb[sb + at] = kk[r];
                                    if (HV) vdstb[sb + at] = vv[r];
                                }
                            }
                        }
                    }
                    __syncthreads();
                    if (tid < nparts) run[tid] += ccnt[tid];
                    __syncthreads();
                }
            }
            if (tid == 0) {                                              // push the parts
                uint32_t top = sp_sh;
                for (uint32_t q = nparts; q-- > 0;) {
                    if (hist[q] == 0) continue;
                    if (top >= BIG_STACK) { overflow_sh = 1; break; }
                    const uint64_t plo = sg.lo + ((uint64_t)q << shift);
                    uint64_t phi = plo + (shift >= 64 ? ~0ull : (((uint64_t)1 << shift) - 1));
                    if (phi > sg.hi || phi < plo) phi = sg.hi;
                    stack[top++] = BigSeg{sg.off + base[q], hist[q], sg.in_d ? 0u : 1u, 0u, plo, phi};
                }
                sp_sh = top;
            }
            __syncthreads();
            // Cannot happen: a split of s <= SPLIT_MAX bits pops one segment
            // and pushes at most 2^s, so the stack grows by at most 2^s - 1
            // <= 3.75 s entries, and s summed along a path is at most the key
            // bits (every part spans s bits fewer): at most 241 entries for
            // 64-bit keys.  Reported rather than assumed.
            if (overflow_sh) {
                if (tid == 0) atomicOr(&b.ctr[CTR_BIG_FAIL], 1u);
                break;
            }
        }
        __syncthreads();
    }
}

// ---- Small nodes sorted on chip.  A node of at most SN_CAP 32-bit keys
// whose columns are base cases (ceil(sqrt n) <= cut-off) is processed with
// its whole subtree by one work-group: every bucket of such a node is smaller
// and has the same property, so no recursion step leaves the work-group.  The
// steps are Alg. 1's, on the node's range of A and D in global memory:
//   pivots     m-1 draws from the node input at the node key's positions,
//              sorted, strict flags (as the batch kernels)
//   columns    D[column i] = sort(A[column i]): each column (at most 64 keys)
//              sorted by one wave with a bitonic network across its lanes
//   transpose  SkewTranspose D -> A: a stable pass by bucket index, which is
//              the layout of Section 2.2 (bucket j, then column order)
//   buckets    a base-case bucket of at most 64 keys sorted by one wave
//              (bitonic), a single-value bucket copied, a larger base-case
//              bucket (cut-offs above 64) taken from a stable sort of the
//              node's A' by key (buckets are key ranges in order); every
//              other bucket pushed on a work-group stack as a node of its
//              own (child key of phase 1), processed the same way later
// The pending nodes are disjoint ranges of more than `cutoff` >= 4 keys, so
// the stack never holds more than SN_CAP / 5 of them.
constexpr int SN_NW = 4;
constexpr int SN_IPT = 16;
constexpr int SN_NT = SN_NW * WAVE;
constexpr uint32_t SN_CAP = SN_NW * WAVE * SN_IPT;   // 4096 keys
constexpr uint32_t SN_STACK = SN_CAP / 5 + 1;
constexpr uint32_t SN_MMAX = 64;                      // ceil(sqrt(SN_CAP))
using SnSm = SortSmem<SN_NW, SN_IPT>;

struct SmallNode {
    unsigned long long off;
    uint32_t n, pad;
    unsigned long long key;
};
struct SnFrame {
    uint16_t off, n;          // relative to the work-group's root node
    uint32_t pad;
    unsigned long long key;
};

// ascending bitonic sort of one key per lane within every aligned segment of
// S lanes of a wave (S a power of two, 2 <= S <= 64): the partners of every
// step lie in the same segment, and the last merge runs ascending in all
template <int S> __device__ inline uint32_t seg_bitonic(uint32_t x)
{
    const uint32_t l = lane_id();
#pragma unroll
    for (int k = 2; k <= S; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t y = lane_xor(x, j);
            const bool up = k == S || (l & (uint32_t)k) == 0;
            const bool keep_min = ((l & (uint32_t)j) == 0) == up;
            x = keep_min ? min(x, y) : max(x, y);
        }
    }
    return x;
}
// the same for a wave-uniform segment size S in {4, 8, 16, 32, 64}
__device__ inline uint32_t seg_bitonic_rt(uint32_t x, uint32_t S)
{
    switch (S) {
    case 4: return seg_bitonic<4>(x);
    case 8: return seg_bitonic<8>(x);
    case 16: return seg_bitonic<16>(x);
    case 32: return seg_bitonic<32>(x);
    default: return seg_bitonic<64>(x);
    }
}
// smallest power of two >= x, at least 4 (x <= 64)
__device__ inline uint32_t seg_of(uint32_t x)
{
    uint32_t S = 4;
    while (S < x) S <<= 1;
    return S;
}

// One stable radix pass by the digits dg (< 256; rows past count must hold
// 255): keys move to their ranks, as one pass of block_sort.  The tables must
// be clear; they are clear again on return.  Wave 0's offsets (the first
// position of every digit) stay in sm.s.tab[0].off until the tables are used
// again.
template <int NW, int IPT>
__device__ void digit_pass(uint32_t (&k)[IPT], const uint32_t (&dg)[IPT], uint32_t count, SortSmem<NW, IPT> &sm)
{
    const int R = block_rows<NW, IPT>(count);
    const int nrows = wave_rows_of(count, R);
    RankTab<256> &tab = sm.s.tab[wave_id()];
    uint32_t pos[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (r < nrows) pos[r] = rank_row(tab, dg[r]);
    __syncthreads();
    scan_tables<NW, 256>(sm.s.tab, sm.wsum);
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (r < nrows) pos[r] += tab.off[dg[r]];
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (r < nrows) sm.s.buf[pos[r]] = k[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (r < nrows) k[r] = sm.s.buf[bpos(r, R)];
    __syncthreads();
}

struct SnShared {
    SnSm sm;
    SnFrame stack[SN_STACK];
    uint32_t piv[SN_MMAX], pivs[SN_MMAX];
    uint8_t pst[SN_MMAX], cls[SN_MMAX];
    uint32_t bsl[SN_MMAX + 1];
    unsigned long long hred[SN_NW];
    uint32_t sp_sh, bigbase_sh;
};

// A node of at most WN_CAP keys (m <= 16) processed by one wave, for
// cut-offs of at most 64 (every base-case bucket then fits the wave's bitonic
// segments): the steps of small_subtree with wave-level synchronisation only.
// wb: the wave's LDS scratch (WN_CAP + 16 words).  Buckets above the cut-off
// are pushed on the work-group's stack (slots from an LDS atomic).
constexpr uint32_t WN_CAP = 256;
__device__ __noinline__ void wave_node(SnShared &sh, uint64_t root_off, SnFrame fr, uint32_t *A, uint32_t *D,
                                 uint32_t cutoff, unsigned long long *digest, uint32_t *wbg)
{
    // the scratch is LDS: addressed as such (a called function sees a generic pointer)
    __attribute__((address_space(3))) uint32_t *wb = (__attribute__((address_space(3))) uint32_t *)wbg;
    constexpr int WR4 = WN_CAP / WAVE;
    const uint32_t l = lane_id();
    const uint64_t off = root_off + fr.off;
    const uint32_t n = fr.n;
    const uint64_t K = fr.key;
    uint32_t m = 1;
    while (m * m < n) ++m;                              // ceil(sqrt n) <= 16
    const uint32_t npiv = m - 1;
    __attribute__((address_space(3))) uint32_t *wp = wb + WN_CAP;   // the sorted pivots
    {                                                   // the node into LDS: one round trip
        uint32_t v[WR4];
#pragma unroll
        for (int r = 0; r < WR4; ++r) {
            const uint32_t p = (uint32_t)r * WAVE + l;
            v[r] = p < n ? A[off + p] : 0u;
        }
#pragma unroll
        for (int r = 0; r < WR4; ++r) {
            const uint32_t p = (uint32_t)r * WAVE + l;
            if (p < n) wb[p] = v[r];
        }
        wave_lds_sync();
    }
    // pivots: draw t by lane t, ranked among the draws by shuffles
    const uint32_t x = l < npiv ? wb[pivot_draw(K, l, n)] : 0xFFFFFFFFu;
    uint32_t rk = 0;
    for (uint32_t u = 0; u < npiv; ++u) {
        const uint32_t y = (uint32_t)__builtin_amdgcn_readlane((int)x, (int)u);   // u: the same in every lane
        rk += (y < x || (y == x && u < l)) ? 1u : 0u;
    }
    // columns, in place: 64 / S at a time in segments of S >= m lanes, bitonic
    const uint32_t S = seg_of(m), per = WAVE / S;
    for (uint32_t ib = 0; ib < m; ib += per) {
        const uint32_t i = ib + l / S, e = l % S;
        const uint32_t c0 = i * m, len = (i < m && c0 < n) ? min(m, n - c0) : 0u;
        uint32_t y = e < len ? wb[c0 + e] : 0xFFFFFFFFu;
        y = seg_bitonic_rt(y, S);
        if (e < len) wb[c0 + e] = y;
    }
    if (l < npiv) wp[rk] = x;
    wave_lds_sync();
    // lane j: pivot j and its strict flag (a run of equal pivots: all but the last)
    const uint32_t pj = l < npiv ? wp[l] : 0u;
    const uint32_t sj = l + 1 < npiv && wp[l] == wp[l + 1] ? 1u : 0u;
    uint32_t kk[WR4], dg[WR4], pos[WR4];
#pragma unroll
    for (int r = 0; r < WR4; ++r) {
        const uint32_t p = (uint32_t)r * WAVE + l;
        kk[r] = p < n ? wb[p] : 0u;                     // D, column-major
        // bucket: the first pivot the key lies at or below (four fixed
        // halving steps over at most 15 pivots, every lane in every step,
        // so that the shuffles read active lanes only)
        uint32_t lo = 0;
#pragma unroll
        for (uint32_t stp = 8; stp >= 1; stp >>= 1) {
            const uint32_t t = lo + stp - 1;
            const uint32_t pm = __shfl(pj, (int)min(t, 15u), WAVE), st = __shfl(sj, (int)min(t, 15u), WAVE);
            if (t < npiv && !le_pivot(kk[r], pm, st != 0u)) lo += stp;
        }
        dg[r] = lo;
    }
    // SkewTranspose: a stable pass by bucket (at most 16), ranks from row ballots
    uint32_t wc = 0u;                                   // lane j: keys of bucket j in earlier rows
#pragma unroll
    for (int r = 0; r < WR4; ++r) {
        const bool ok = (uint32_t)r * WAVE + l < n;
        unsigned long long me = __ballot(ok), mj = me;
#pragma unroll
        for (int bit = 0; bit < 4; ++bit) {
            const unsigned long long bk = __ballot(ok && ((dg[r] >> bit) & 1u));
            me &= ((dg[r] >> bit) & 1u) ? bk : ~bk;
            mj &= ((l >> bit) & 1u) ? bk : ~bk;
        }
        pos[r] = __shfl(wc, (int)dg[r], WAVE) + rank_in_mask((uint32_t)me, (uint32_t)(me >> 32));
        wc += (uint32_t)__popcll(mj);
    }
    const uint32_t bst = wave_incl_scan(l < m ? wc : 0u) - (l < m ? wc : 0u);   // lane j: bucket j's start
    const uint32_t nj = l < m ? wc : 0u;
    unsigned long long h = 0;
    wave_lds_sync();                                    // the columns are read
#pragma unroll
    for (int r = 0; r < WR4; ++r) {
        const uint32_t first = __shfl(bst, (int)dg[r], WAVE);      // every lane (a shuffle reads active lanes only)
        if ((uint32_t)r * WAVE + l < n) {
            const uint32_t q = pos[r] + first;
            wb[q] = kk[r];
            A[off + q] = kk[r];                         // A' for the child nodes
            if (digest) h += splitmix((uint64_t)kk[r] ^ splitmix((uint64_t)q));
        }
    }
    if (digest) {
        h = wave_sum_u64(h);
        if (l == 0) atomicAdd(digest, (unsigned long long)splitmix(K ^ h));
    }
    wave_lds_sync();
    // buckets (lane j): single value, base case (at most the cut-off <= 64
    // keys) or a child node
    enum : uint32_t { W_SORT = 0, W_COPY = 1, W_NODE = 2, W_EMPTY = 3 };
    uint32_t c = W_EMPTY;
    // every lane: the previous lane's pivot and flag (lane 0's are not used)
    const uint32_t pl = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)pj, 0x138, 0xF, 0xF, false);   // wave_shr 1
    const uint32_t slo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)sj, 0x138, 0xF, 0xF, false);
    if (l < m && nj > 0) {
        const uint64_t L = l == 0 ? 0ull : (slo ? (uint64_t)pl : (uint64_t)pl + 1);
        const int64_t U = l == npiv ? (int64_t)0xFFFFFFFFu : (sj ? (int64_t)pj - 1 : (int64_t)pj);
        if ((int64_t)L == U) c = W_COPY;
        else if (nj > cutoff) c = W_NODE;
        else c = W_SORT;
    }
    if (c == W_NODE) {
        const uint32_t slot = atomicAdd(&sh.sp_sh, 1u);
        sh.stack[slot] = SnFrame{(uint16_t)(fr.off + bst), (uint16_t)nj, 0u, node_child_key(K, 1, l)};
    }
    // base-case buckets, four consecutive ones at a time (segments of 16
    // lanes when they all fit, else pairs in segments of 32, else singly)
    for (uint32_t jb = 0; jb < m; jb += 4) {
        uint32_t sz[4], b0s[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t j = jb + q;
            const uint32_t cq = (uint32_t)__builtin_amdgcn_readlane((int)c, (int)min(j, 63u));
            const uint32_t nq = (uint32_t)__builtin_amdgcn_readlane((int)nj, (int)min(j, 63u));
            sz[q] = j < m && cq == W_SORT ? nq : 0u;
            b0s[q] = (uint32_t)__builtin_amdgcn_readlane((int)bst, (int)min(j, 63u));
        }
        const uint32_t mx4 = max(max(sz[0], sz[1]), max(sz[2], sz[3]));
        const uint32_t mxa = max(sz[0], sz[1]), mxb = max(sz[2], sz[3]);
        uint32_t jobs = 0, njobs = 0;
        auto add = [&](uint32_t dj, uint32_t g, uint32_t Sg) {
            jobs |= (dj | (g << 2) | ((uint32_t)__builtin_ctz(Sg) << 5)) << (8 * njobs);
            ++njobs;
        };
        if (mx4 == 0) {
        } else if (mx4 <= 16) {
            add(0, 4, 16);
        } else {
            if (mxa > 0) { if (mxa <= 32) add(0, 2, 32); else { add(0, 1, 64); add(1, 1, 64); } }
            if (mxb > 0) { if (mxb <= 32) add(2, 2, 32); else { add(2, 1, 64); add(3, 1, 64); } }
        }
        for (uint32_t t = 0; t < njobs; ++t) {
            const uint32_t jd = (jobs >> (8 * t)) & 255u;
            const uint32_t dj = jd & 3u, g = (jd >> 2) & 7u, Sg = 1u << (jd >> 5);
            const uint32_t q = l / Sg, e = l % Sg;
            uint32_t b0 = 0u, len = 0u;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if ((uint32_t)u == dj + q && q < g) { b0 = b0s[u]; len = sz[u]; }
            uint32_t y = e < len ? wb[b0 + e] : 0xFFFFFFFFu;
            y = seg_bitonic_rt(y, Sg);
            if (e < len) D[off + b0 + e] = y;
        }
    }
    // single-value buckets: copied
    for (uint32_t j = 0; j < m; ++j) {
        if ((uint32_t)__builtin_amdgcn_readlane((int)c, (int)j) != W_COPY) continue;
        const uint32_t b0 = (uint32_t)__builtin_amdgcn_readlane((int)bst, (int)j);
        const uint32_t len = (uint32_t)__builtin_amdgcn_readlane((int)nj, (int)j);
        for (uint32_t e = l; e < len; e += WAVE) D[off + b0 + e] = wb[b0 + e];
    }
}

// The whole subtree of one on-chip node (the caller has cleared sh.sm's
// tables once; they are clear again on return).  Ends with a barrier.
__device__ __forceinline__ void small_subtree(SnShared &sh, const SmallNode root, uint32_t *A, uint32_t *D, uint32_t cutoff,
                              unsigned long long *digest)
{
    SnSm &sm = sh.sm;
    SnFrame *stack = sh.stack;
    uint32_t *piv = sh.piv, *pivs = sh.pivs, *bsl = sh.bsl;
    uint8_t *pst = sh.pst, *cls = sh.cls;
    unsigned long long *hred = sh.hred;
    uint32_t &sp_sh = sh.sp_sh, &bigbase_sh = sh.bigbase_sh;
    enum : uint8_t { B_SORT = 0, B_COPY = 1, B_NODE = 2, B_BIG = 3, B_EMPTY = 4 };
    const uint32_t tid = threadIdx.x, l = lane_id(), w = wave_id();
    {
        if (tid == 0) {
            stack[0] = SnFrame{0, (uint16_t)root.n, 0u, root.key};
            sp_sh = 1;
        }
        __syncthreads();
        while (true) {
            const uint32_t sp = sp_sh;
            if (sp == 0) break;
            const SnFrame fr = stack[sp - 1];
            if (cutoff <= (uint32_t)WAVE && fr.n <= WN_CAP) {
                // up to SN_NW small nodes from the top of the stack, one per wave
                uint32_t nw = 1;
                while (nw < (uint32_t)SN_NW && nw < sp && stack[sp - 1 - nw].n <= WN_CAP) ++nw;
                const SnFrame mine = stack[sp - 1 - min(w, nw - 1)];
                __syncthreads();                        // every frame read before any push
                if (tid == 0) sp_sh = sp - nw;
                __syncthreads();
                if (w < nw) wave_node(sh, root.off, mine, A, D, cutoff, digest, sm.s.buf + w * (WN_CAP + 16));
                __syncthreads();
                continue;
            }
            __syncthreads();
            if (tid == 0) { sp_sh = sp - 1; bigbase_sh = 0u; }
            const uint64_t off = root.off + fr.off;
            const uint32_t n = fr.n;
            const uint64_t K = fr.key;
            uint32_t m = 1;
            while (m * m < n) ++m;                      // ceil(sqrt n), n <= SN_CAP
            const uint32_t npiv = m - 1;
            const int R = block_rows<SN_NW, SN_IPT>(n);
            const int nrows = wave_rows_of(n, R);
            // ---- the node into LDS in one round trip (every load in flight together)
            {
                uint32_t v[SN_IPT];
#pragma unroll
                for (int r = 0; r < SN_IPT; ++r) {
                    const uint32_t p = (uint32_t)r * SN_NT + tid;
                    v[r] = p < n ? A[off + p] : 0u;
                }
#pragma unroll
                for (int r = 0; r < SN_IPT; ++r) {
                    const uint32_t p = (uint32_t)r * SN_NT + tid;
                    if (p < n) sm.s.buf[p] = v[r];
                }
            }
            __syncthreads();
            // ---- pivots: m-1 draws from the node input
            if (tid < npiv) piv[tid] = sm.s.buf[pivot_draw(K, tid, n)];
            __syncthreads();
            // ---- columns (m <= 64 keys each), in place: 64 / S columns per
            // wave at a time, each in a segment of S >= m lanes, bitonic
            {
                const uint32_t S = seg_of(m), per = WAVE / S;
                for (uint32_t ib = w * per; ib < m; ib += SN_NW * per) {
                    const uint32_t i = ib + l / S, e = l % S;
                    const uint32_t c0 = i * m, len = (i < m && c0 < n) ? min(m, n - c0) : 0u;
                    uint32_t x = e < len ? sm.s.buf[c0 + e] : 0xFFFFFFFFu;
                    x = seg_bitonic_rt(x, S);
                    if (e < len) sm.s.buf[c0 + e] = x;
                }
            }
            __syncthreads();
            if (tid < npiv) {                           // rank sort of the draws
                const uint32_t x = piv[tid];
                uint32_t rk = 0;
                for (uint32_t u = 0; u < npiv; ++u) {
                    const uint32_t y = piv[u];
                    rk += (y < x || (y == x && u < tid)) ? 1u : 0u;
                }
                pivs[rk] = x;
            }
            uint32_t kk[SN_IPT], dg[SN_IPT];
#pragma unroll
            for (int r = 0; r < SN_IPT; ++r)
                if (r < nrows) kk[r] = sm.s.buf[bpos(r, R)];          // D, column-major
            __syncthreads();
            if (tid < npiv) pst[tid] = (tid + 1 < npiv && pivs[tid] == pivs[tid + 1]) ? 1 : 0;
            __syncthreads();
            // ---- SkewTranspose: bucket of every key, then a stable pass by bucket
#pragma unroll
            for (int r = 0; r < SN_IPT; ++r) {
                if (r < nrows) {
                    uint32_t lo = 0, hi = npiv;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (le_pivot(kk[r], pivs[mid], pst[mid] != 0)) hi = mid; else lo = mid + 1;
                    }
                    dg[r] = bpos(r, R) < n ? lo : 255u;
                }
            }
            digit_pass<SN_NW, SN_IPT>(kk, dg, n, sm);
            // bucket starts from wave 0's digit offsets (read before the tables are used again)
            if (tid < m) bsl[tid] = sm.s.tab[0].off[tid];
            if (tid == 0) bsl[m] = n;
            unsigned long long h = 0;
#pragma unroll
            for (int r = 0; r < SN_IPT; ++r) {
                const uint32_t p = bpos(r, R);
                if (r < nrows && p < n) {
                    A[off + p] = kk[r];
                    sm.s.buf[p] = kk[r];                // A' for the bucket sorts
                    if (digest) h += splitmix((uint64_t)kk[r] ^ splitmix((uint64_t)p));
                }
            }
            if (digest) {                               // the node's tree-digest term
                h = wave_sum_u64(h);
                if (l == 0) hred[w] = h;
            }
            __syncthreads();
            if (digest && tid == 0) {
                unsigned long long hs = 0;
                for (int q = 0; q < SN_NW; ++q) hs += hred[q];
                atomicAdd(digest, (unsigned long long)splitmix(K ^ hs));
            }
            // ---- buckets: classes, internal ones pushed
            if (tid < m) {
                const uint32_t j = tid, nj = bsl[j + 1] - bsl[j];
                const uint64_t L = j == 0 ? 0ull : (pst[j - 1] ? (uint64_t)pivs[j - 1] : (uint64_t)pivs[j - 1] + 1);
                const int64_t U = j == npiv ? (int64_t)0xFFFFFFFFu
                                            : (pst[j] ? (int64_t)pivs[j] - 1 : (int64_t)pivs[j]);
                const bool mono = nj > 0 && (int64_t)L == U;
                uint8_t c = B_SORT;
                if (nj == 0) c = B_EMPTY;
                else if (mono) c = B_COPY;
                else if (nj > cutoff) c = B_NODE;
                else if (nj > (uint32_t)WAVE) c = B_BIG;
                cls[j] = c;
                if (c == B_BIG) bigbase_sh = 1u;
            }
            __syncthreads();
            if (tid == 0) {
                uint32_t top = sp_sh;
                for (uint32_t j = m; j-- > 0;) {
                    if (cls[j] != B_NODE) continue;
                    stack[top++] = SnFrame{(uint16_t)(fr.off + bsl[j]), (uint16_t)(bsl[j + 1] - bsl[j]), 0u,
                                           node_child_key(K, 1, j)};
                }
                sp_sh = top;
            }
            // base-case buckets (at most 64 keys here): four consecutive ones
            // per wave at a time, in segments of 16 lanes when they all fit,
            // else as two pairs in segments of 32, else one by one
            for (uint32_t jb = 4 * w; jb < m; jb += 4 * SN_NW) {
                uint32_t sz[4];
                uint32_t mx4 = 0, mxa = 0, mxb = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t j = jb + q;
                    sz[q] = j < m && cls[j] == B_SORT ? bsl[j + 1] - bsl[j] : 0u;
                    mx4 = max(mx4, sz[q]);
                }
                mxa = max(sz[0], sz[1]);
                mxb = max(sz[2], sz[3]);
                // jobs: (first bucket offset, buckets, segment lanes), 8 bits each
                uint32_t jobs = 0, njobs = 0;
                auto add = [&](uint32_t dj, uint32_t g, uint32_t S) {
                    jobs |= (dj | (g << 2) | ((uint32_t)__builtin_ctz(S) << 5)) << (8 * njobs);
                    ++njobs;
                };
                if (mx4 == 0) {
                } else if (mx4 <= 16) {
                    add(0, 4, 16);
                } else {
                    if (mxa > 0) { if (mxa <= 32) add(0, 2, 32); else { add(0, 1, 64); add(1, 1, 64); } }
                    if (mxb > 0) { if (mxb <= 32) add(2, 2, 32); else { add(2, 1, 64); add(3, 1, 64); } }
                }
#pragma unroll 1
                for (uint32_t t = 0; t < njobs; ++t) {      // g consecutive buckets in segments of S lanes
                    const uint32_t jd = (jobs >> (8 * t)) & 255u;
                    const uint32_t j0 = jb + (jd & 3u), g = (jd >> 2) & 7u, S = 1u << (jd >> 5);
                    const uint32_t q = l / S, e = l % S, j = j0 + q;
                    const bool mine = q < g && j < m && cls[j] == B_SORT;
                    const uint32_t b0 = mine ? bsl[j] : 0u, nj = mine ? bsl[j + 1] - b0 : 0u;
                    uint32_t x = e < nj ? sm.s.buf[b0 + e] : 0xFFFFFFFFu;
                    x = seg_bitonic_rt(x, S);
                    if (e < nj) D[off + b0 + e] = x;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {                // single-value buckets: copied
                    const uint32_t j = jb + q;
                    if (j < m && cls[j] == B_COPY) {
                        const uint32_t b0 = bsl[j], nj = bsl[j + 1] - b0;
                        for (uint32_t e = l; e < nj; e += WAVE) D[off + b0 + e] = sm.s.buf[b0 + e];
                    }
                }
            }
            if (bigbase_sh) {                           // base cases above 64 keys (cut-offs above 64)
                uint32_t vv[SN_IPT];
                __syncthreads();                        // buf: the bucket waves are done with it
                block_sort<uint32_t, false, SN_NW, SN_IPT>(kk, vv, n, sm);
#pragma unroll
                for (int r = 0; r < SN_IPT; ++r) {
                    const uint32_t p = bpos(r, R);
                    if (r < nrows && p < n) {
                        uint32_t lo = 0, hi = m;        // bucket of position p
                        while (hi - lo > 1) {
                            const uint32_t mid = (lo + hi) >> 1;
                            if (bsl[mid] <= p) lo = mid; else hi = mid;
                        }
                        if (cls[lo] == B_BIG) D[off + p] = kk[r];
                    }
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();                                    // every thread has seen the empty stack
}

__global__ __launch_bounds__(SN_NT, 3) void k_small_nodes(const SmallNode *roots, uint32_t count, uint32_t *A,
                                                        uint32_t *D, uint32_t cutoff,
                                                        unsigned long long *digest)
{
    __shared__ SnShared sh;
    tables_clear<SN_NW, 256>(sh.sm.s.tab);
    for (uint32_t ri = blockIdx.x; ri < count; ri += gridDim.x) small_subtree(sh, roots[ri], A, D, cutoff, digest);
}

// status bits a call that does not synchronise (a planned graph) reports in
// its device status word
constexpr uint32_t ST_UNFINISHED = 1u;   // an internal bucket needs a recursion step the device cannot take
constexpr uint32_t ST_DEVICE = 2u;       // a device failure word (bounded wait, stack) or a list overflow

// The internal buckets of a batch (its CLS_INTERNAL list) sorted on chip,
// each with its subtree, when they are on-chip nodes; any other one is
// reported as ST_UNFINISHED.  Used where the host does not read the list.
__global__ __launch_bounds__(SN_NT, 3) void k_internal_nodes(Batch<uint32_t> b, uint32_t *A, uint32_t *D,
                                                           uint32_t cutoff, unsigned long long *digest,
                                                           uint32_t *status)
{
    __shared__ SnShared sh;
    tables_clear<SN_NW, 256>(sh.sm.s.tab);
    const uint32_t cnt = min(b.ctr[CLS_INTERNAL], b.cap[CLS_INTERNAL]);
    for (uint32_t it = blockIdx.x; it < cnt; it += gridDim.x) {
        const BucketItem e = b.list[CLS_INTERNAL][it];
        const NodeDesc nd = b.nodes[e.node];
        uint32_t m = 1;
        while (m * m < e.size && m <= SN_MMAX) ++m;
        if (e.size <= SN_CAP && m <= cutoff) {
            small_subtree(sh, SmallNode{nd.off + e.lo, e.size, 0u, node_child_key(nd.key, 1, e.j)}, A, D, cutoff,
                          digest);
        } else if (threadIdx.x == 0) {
            atomicOr(status, ST_UNFINISHED);
        }
    }
}

// a batch's failure words (and, for a recursion step, its list overflows)
// into the status word
template <class K>
__global__ void k_status(Batch<K> b, uint32_t *status, int step)
{
    if (threadIdx.x != 0) return;
    uint32_t f = 0;
    if (b.ctr[CTR_BIG_FAIL]) f |= ST_DEVICE;
    if (step) {
        if (b.ctr[CTR_TR_FAIL] || b.ctr[CTR_FAIL]) f |= ST_DEVICE;
        for (int c = 0; c < NCLS; ++c)
            if (b.ctr[c] > b.cap[c]) f |= ST_DEVICE;
    }
    if (f) atomicOr(status, f);
}

// a copy of n words (the pristine initial counters of a planned call)
__global__ void k_copy_u32(uint32_t *dst, const uint32_t *src, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// ---- Base-case segments larger than one LDS sort (a whole array, or the
// instances of a batch when they are too few to fill the chip), on the whole
// grid.  One MSD split of each segment by the top 8 bits of x - min runs over
// all work-groups (chunk ranges, per-chunk digit counts, one scan per
// segment, a stable scatter into D); the parts are then items of the
// MSD-split kernel, which reads them from D.  Part j holds the keys
// min + j*2^shift .. min + (j+1)*2^shift - 1 (the first and last parts are
// given bounds open towards 0 and the largest key of the type).
constexpr int BS_NW = 4;
constexpr int BS_IPT = 16;
constexpr int BS_NT = BS_NW * WAVE;
constexpr uint32_t BS_CH = BS_NT * BS_IPT;          // 4096 keys a chunk
constexpr uint32_t BS_MAXG = BIG_CAP / BS_CH;       // chunks of the largest segment
static_assert(BS_MAXG <= (uint32_t)WAVE, "one lane per chunk in split_range");
using BsSm = SortSmem<BS_NW, BS_IPT>;

template <class K> struct BaseSplit {
    K *mm;                    // [chunk][2]: smallest and largest key of the chunk
    uint32_t *cnt;            // segment s at 256 * its first chunk: [d][g] keys of its chunk g with
                              // digit d, after the scan their first slot in the segment
    Span<K> *items;           // the parts of every segment (<= 256 each), resolved
    uint32_t *ctr;            // the counters of the part sort
    const uint64_t *segOff;   // per segment: first slot in A and D (null: one segment at 0)
    const uint32_t *segN;     // per segment: keys (<= BIG_CAP)
    const uint32_t *segChunk; // nseg + 1: prefix of the segments' chunk counts
    uint32_t nseg;
    uint32_t n;               // the one segment's keys (segOff null)
    uint32_t G;               // chunks of all segments
};

struct SegInfo {
    uint64_t off;
    uint32_t n, c0, G;        // keys, first chunk, chunks
};
template <class K>
__device__ inline SegInfo seg_info(const BaseSplit<K> &s, uint32_t seg)
{
    if (!s.segOff) return SegInfo{0ull, s.n, 0u, s.G};
    return SegInfo{s.segOff[seg], s.segN[seg], s.segChunk[seg], s.segChunk[seg + 1] - s.segChunk[seg]};
}
template <class K>
__device__ inline uint32_t seg_of_chunk(const BaseSplit<K> &s, uint32_t chunk)
{
    return s.segOff ? find_node(s.segChunk, s.nseg, chunk) : 0u;
}

// smallest key of the segment and the split shift (all threads)
template <class K>
__device__ inline void split_range(const BaseSplit<K> &s, const SegInfo &si, K &lo, K &hi, int &shift, K *sh)
{
    using T = KeyT<K>;
    if (threadIdx.x < WAVE) {
        const uint32_t l = lane_id();
        K a = l < si.G ? s.mm[2 * (si.c0 + l)] : (K)T::MAXV;
        K c = l < si.G ? s.mm[2 * (si.c0 + l) + 1] : (K)0;
        a = wave_min(a);
        c = wave_max(c);
        if (l == 0) { sh[0] = a; sh[1] = c; }
    }
    __syncthreads();
    lo = sh[0];
    hi = sh[1];
    const int bits = T::bitlen((K)(hi - lo));
    shift = bits > 8 ? bits - 8 : 0;
}

template <class K>
__global__ __launch_bounds__(BS_NT) void k_base_range(const K *A, BaseSplit<K> s)
{
    using T = KeyT<K>;
    __shared__ uint32_t red32[2 * BS_NW];
    __shared__ unsigned long long red64[2 * BS_NW];
    const uint32_t chunk = blockIdx.x;
    const SegInfo si = seg_info(s, seg_of_chunk(s, chunk));
    const uint32_t g = chunk - si.c0;
    if (chunk == 0)                                  // the scans add their parts into them
        for (uint32_t t = threadIdx.x; t < (uint32_t)CTR_WORDS; t += BS_NT) s.ctr[t] = 0u;
    K lo = (K)T::MAXV, hi = (K)0, x[BS_IPT];
#pragma unroll
    for (int i = 0; i < BS_IPT; ++i) {
        const uint32_t p = g * BS_CH + i * BS_NT + threadIdx.x;
        x[i] = p < si.n ? A[si.off + p] : (K)0;
    }
#pragma unroll
    for (int i = 0; i < BS_IPT; ++i)
        if (g * BS_CH + i * BS_NT + threadIdx.x < si.n) { lo = x[i] < lo ? x[i] : lo; hi = x[i] > hi ? x[i] : hi; }
    block_minmax<K, BS_NW>(lo, hi, red32, red64);
    if (threadIdx.x == 0) { s.mm[2 * chunk] = lo; s.mm[2 * chunk + 1] = hi; }
}

template <class K>
__global__ __launch_bounds__(BS_NT) void k_base_count(const K *A, BaseSplit<K> s)
{
    __shared__ uint32_t h[BS_NW][256];
    __shared__ K sh[2];
    const uint32_t chunk = blockIdx.x, tid = threadIdx.x;
    const SegInfo si = seg_info(s, seg_of_chunk(s, chunk));
    const uint32_t g = chunk - si.c0;
    K lo, hi;
    int shift;
    split_range(s, si, lo, hi, shift, sh);
    for (uint32_t i = tid; i < BS_NW * 256; i += BS_NT) (&h[0][0])[i] = 0;
    __syncthreads();
    uint32_t *wh = h[wave_id()];
    K x[BS_IPT];
#pragma unroll
    for (int i = 0; i < BS_IPT; ++i) {
        const uint32_t p = g * BS_CH + i * BS_NT + tid;
        x[i] = p < si.n ? A[si.off + p] : lo;
    }
#pragma unroll
    for (int i = 0; i < BS_IPT; ++i)
        if (g * BS_CH + i * BS_NT + tid < si.n) atomicAdd(&wh[(uint32_t)((K)(x[i] - lo) >> shift)], 1u);
    __syncthreads();
    uint32_t *cnt = s.cnt + 256ull * si.c0;
    for (uint32_t d = tid; d < 256; d += BS_NT) {
        uint32_t c = 0;
        for (int w = 0; w < BS_NW; ++w) c += h[w][d];
        cnt[d * si.G + g] = c;
    }
}

// One work-group per segment: exclusive scan of its [d][g] counts
// (digit-major, so the chunks of a digit follow each other: the scatter is
// stable), then its parts (largest first, appended to the part list).  With
// shift 0 every part holds one key value and is final after the scatter: no
// items.
template <class K>
__global__ __launch_bounds__(1024) void k_base_scan(BaseSplit<K> s)
{
    __shared__ uint32_t v[256 * BS_MAXG];
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t sz[256], st0[256];
    __shared__ uint32_t base_sh;
    __shared__ K sh[2];
    const uint32_t seg = blockIdx.x, tid = threadIdx.x;
    const SegInfo si = seg_info(s, seg);
    const uint32_t E = 256 * si.G;
    constexpr uint32_t PER = 256 * BS_MAXG / 1024;
    uint32_t *cnt = s.cnt + 256ull * si.c0;
    K lo, hi;
    int shift;
    split_range(s, si, lo, hi, shift, sh);
    uint32_t loc = 0, c[PER];
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {                 // loads first, in flight together
        const uint32_t i = tid * PER + q;
        c[q] = i < E ? cnt[i] : 0u;
    }
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
        v[tid * PER + q] = c[q];
        loc += c[q];
    }
    const uint32_t incl = wave_incl_scan(loc);
    if (lane_id() == WAVE - 1) wsum[wave_id()] = incl;
    __syncthreads();
    uint32_t run = incl - loc;
    for (uint32_t w = 0; w < wave_id(); ++w) run += wsum[w];
    for (uint32_t q = 0; q < PER; ++q) {
        const uint32_t i = tid * PER + q;
        const uint32_t c = v[i];
        v[i] = run;
        if (i < E) cnt[i] = run;
        run += c;
    }
    __syncthreads();
    if (tid < 256) {
        st0[tid] = v[tid * si.G];
        sz[tid] = (tid < 255 ? v[(tid + 1) * si.G] : si.n) - v[tid * si.G];
    }
    __syncthreads();
    uint32_t items = 0, rank = 0;
    if (tid < 256) {
        const uint32_t me = sz[tid];
        for (uint32_t e = 0; e < 256; ++e) {
            const uint32_t o = sz[e];
            rank += (o > me || (o == me && e < tid)) ? 1u : 0u;
            items += (shift > 0 && o > 0) ? 1u : 0u;
        }
    }
    if (tid == 0) {
        base_sh = items ? atomicAdd(&s.ctr[CLS_BIG], items) : 0u;
        if (items) atomicAdd(&s.ctr[2 * NCLS + CLS_BIG], si.n);
    }
    __syncthreads();
    if (tid < 256 && shift > 0 && sz[tid] > 0) {
        const uint32_t last = (uint32_t)((K)(hi - lo) >> shift);     // the highest non-empty digit
        const K plo = tid == 0 ? (K)0 : (K)(lo + ((K)tid << shift));
        const K phi = tid == last ? (K)KeyT<K>::MAXV : (K)(lo + ((K)(tid + 1) << shift) - 1);
        s.items[base_sh + rank] = Span<K>{si.off + st0[tid], sz[tid], 0u, plo, phi};
    }
}

template <class K, bool HV>
__global__ __launch_bounds__(BS_NT) void k_base_scatter(const K *A, const uint32_t *VA, K *D, uint32_t *VD,
                                                        BaseSplit<K> s)
{
    using T = KeyT<K>;
    __shared__ BsSm sm;
    __shared__ uint32_t gb[256];
    __shared__ K sh[2];
    const uint32_t chunk = blockIdx.x, tid = threadIdx.x;
    const SegInfo si = seg_info(s, seg_of_chunk(s, chunk));
    const uint32_t g = chunk - si.c0;
    K lo, hi;
    int shift;
    split_range(s, si, lo, hi, shift, sh);
    tables_clear<BS_NW, 256>(sm.s.tab);
    const uint32_t *cnt = s.cnt + 256ull * si.c0;
    for (uint32_t d = tid; d < 256; d += BS_NT) gb[d] = cnt[d * si.G + g];
    __syncthreads();
    const uint32_t c0 = g * BS_CH;
    const uint32_t chN = min(BS_CH, si.n - c0);
    const K *src = A + si.off;
    const uint32_t *vsrc = HV ? VA + si.off : nullptr;
    const int nrows = wave_rows<BS_IPT>(chN);
    RankTab<256> &tab = sm.s.tab[wave_id()];
    K kk[BS_IPT];
    uint32_t vv[BS_IPT], pos[BS_IPT];
#pragma unroll
    for (int r = 0; r < BS_IPT; ++r) {                          // loads first, in flight together
        const uint32_t p = item_pos<BS_NW, BS_IPT>(r);
        kk[r] = r < nrows && p < chN ? src[c0 + p] : (K)0;
        if (HV) vv[r] = r < nrows && p < chN ? vsrc[c0 + p] : 0u;
    }
#pragma unroll
    for (int r = 0; r < BS_IPT; ++r) {
        if (r < nrows) {
            const uint32_t p = item_pos<BS_NW, BS_IPT>(r);
            const uint32_t d = p < chN ? (uint32_t)((K)(kk[r] - lo) >> shift) : 255u;
            pos[r] = rank_row(tab, d);
        }
    }
    __syncthreads();
    scan_tables<BS_NW, 256>(sm.s.tab, sm.wsum);
#pragma unroll
    for (int r = 0; r < BS_IPT; ++r) {
        if (r < nrows) {
            const uint32_t p = item_pos<BS_NW, BS_IPT>(r);
            const uint32_t d = p < chN ? (uint32_t)((K)(kk[r] - lo) >> shift) : 255u;
            pos[r] += tab.off[d];
        }
    }
#pragma unroll
    for (int wd = 0; wd < T::WORDS; ++wd) {
#pragma unroll
        for (int r = 0; r < BS_IPT; ++r)
            if (r < nrows) sm.s.buf[pos[r]] = T::word(kk[r], wd);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < BS_IPT; ++r)
            if (r < nrows) kk[r] = T::set_word(kk[r], wd, sm.s.buf[item_pos<BS_NW, BS_IPT>(r)]);
        __syncthreads();
    }
    if (HV) {
#pragma unroll
        for (int r = 0; r < BS_IPT; ++r) if (r < nrows) sm.s.buf[pos[r]] = vv[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < BS_IPT; ++r) if (r < nrows) vv[r] = sm.s.buf[item_pos<BS_NW, BS_IPT>(r)];
    }
    // chunk-sorted position p holds a key of digit d: it goes to the chunk's
    // first slot of d plus its place among the chunk's keys of d
    K *dseg = D + si.off;
    uint32_t *vdseg = HV ? VD + si.off : nullptr;
#pragma unroll
    for (int r = 0; r < BS_IPT; ++r) {
        if (r < nrows) {
            const uint32_t p = item_pos<BS_NW, BS_IPT>(r);
            if (p < chN) {
                const uint32_t d = (uint32_t)((K)(kk[r] - lo) >> shift);
                const uint32_t at = gb[d] + (p - sm.s.tab[0].off[d]);
                dseg[at] = kk[r];
                if (HV) vdseg[at] = vv[r];
            }
        }
    }
}

// A whole (sub)array that is a base case: n <= cutoff, one work-group.
template <class K, bool HV>
__global__ __launch_bounds__(SORT_NT) void k_base_sort(uint32_t n, const K *A, const uint32_t *VA,
                                                        K *D, uint32_t *VD)
{
    __shared__ SortSm sm;
    K kk[SORT_IPT];
    uint32_t vv[SORT_IPT];
    tables_clear<SORT_NW, 256>(sm.s.tab);
    const int R = block_rows<SORT_NW, SORT_IPT>(n);
#pragma unroll
    for (int r = 0; r < SORT_IPT; ++r) {
        const uint32_t p = bpos(r, R);
        kk[r] = r < R && p < n ? A[p] : (K)0;
        if (HV) vv[r] = r < R && p < n ? VA[p] : 0u;
    }
    wait_vmem();
    __syncthreads();
    block_sort<K, HV, SORT_NW, SORT_IPT>(kk, vv, n, sm);
#pragma unroll
    for (int r = 0; r < SORT_IPT; ++r) {
        const uint32_t p = bpos(r, R);
        if (r < R && p < n) {
            D[p] = kk[r];
            if (HV) VD[p] = vv[r];
        }
    }
}

}  // namespace sqs
