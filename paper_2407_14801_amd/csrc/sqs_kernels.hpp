// sqs_kernels.hpp -- the HIP kernels of one SquareSort recursion step,
// batched over every internal node of that step (Alg. 1 of arXiv 2407.14801).
//
// A node owns the range [off, off+n) of both global arrays A (its input,
// clobbered) and D (its output).  For a batch of nodes the step runs:
//   k_sample         m-1 pivot draws per node from its input A
//   k_sort_pivots    sort them, strict flags (pivot equal to the next one)
//   k_colsort        sort each column A -> D and count, per column i and
//                    bucket block J, how many keys precede J; per column
//                    group g and bucket j, how many keys of g fall in j
//   k_colscan        prefix over groups per bucket, bucket totals
//   k_bucket_start   exclusive scan of totals: bucket j = [bs[j], bs[j+1])
//   k_transpose      SkewTranspose D -> A over (column group x bucket block)
//                    tiles, staged through LDS
//   k_bucket         per bucket: skip (empty), copy (single key value), sort
//                    in LDS (base case), or mark for the next batch
#pragma once

#include "sqs_device.hpp"

namespace sqs {

// ------------------------------------------------------------ configuration
constexpr int SORT_NW = 16;                  // waves of the sorting work-groups
constexpr int SORT_IPT = 16;                 // keys per thread
constexpr int SORT_NT = SORT_NW * WAVE;      // 1024 threads
constexpr int SORT_CAP = SORT_NT * SORT_IPT; // 16384 keys per LDS sort
constexpr int TG = 64;                       // columns per column group
constexpr int TB = 64;                       // buckets per bucket block
constexpr int TR_NW = 16;                    // waves of the transpose work-group
constexpr int TR_IPT = 8;                    // keys per thread per chunk
constexpr int TR_CH = TR_NW * WAVE * TR_IPT; // 8192 keys per transpose chunk

using SortSm = SortSmem<SORT_NW, SORT_IPT>;

// ------------------------------------------------------------ batch layout
struct NodeDesc {
    uint64_t off;      // first slot of the node in A and D
    uint64_t key;      // generator key of the node
    uint32_t n, m;     // size, columns (= buckets) = ceil(sqrt(n))
    uint32_t groups;   // ceil(m / TG)
    uint32_t nJ;       // ceil(m / TB)
    uint32_t piv;      // first pivot slot (m-1 slots)
    uint32_t bkt;      // first bucket slot (m+1 slots in bs, m in tot/cls)
    uint64_t src;      // first slot of the column/bucket-block offsets ((nJ+1)*m)
    uint64_t blk;      // first slot of the group/bucket counts (groups*m)
    uint32_t flags;    // NODE_COLS_SORTED: columns already sorted into D
    uint32_t pad;
};
constexpr uint32_t NODE_COLS_SORTED = 1u;

template <class K> struct Batch {
    const NodeDesc *nodes;
    uint32_t N;
    const uint32_t *pivStart;    // N+1 prefix of m-1
    const uint32_t *grpStart;    // N+1 prefix of groups
    const uint32_t *tileStart;   // N+1 prefix of groups*nJ
    const uint32_t *bucStart;    // N+1 prefix of m
    const uint32_t *digStart;    // N+1 prefix of digest chunks
    K *piv;
    uint8_t *strict;
    uint32_t *srcOff;   // [J][i] per node: keys of column i in buckets < J*TB
    uint32_t *blk;      // [g][j] per node: keys of group g in bucket j (then prefix over g)
    uint32_t *bs;       // [j] per node, m+1 entries
    uint32_t *tot;      // [j] per node
    uint8_t *cls;       // [j] per node: 0 empty, 1 single value, 2 base, 3 internal
    unsigned long long *H;
};

// largest k with prefix[k] <= item (prefix is non-decreasing, prefix[0] = 0)
__device__ inline uint32_t find_node(const uint32_t *prefix, uint32_t N, uint32_t item)
{
    uint32_t lo = 0, hi = N - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------ utility kernels
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
    b.piv[nd.piv + t] = A[nd.off + pivot_draw(nd.key, t, nd.n)];
}

// Sort the samples of one node (any correct sort; the paper uses MergeSort)
// and mark strict pivots.
template <class K>
__global__ __launch_bounds__(SORT_NT) void k_sort_pivots(Batch<K> b)
{
    __shared__ SortSm sm;
    const NodeDesc nd = b.nodes[blockIdx.x];
    const uint32_t cnt = nd.m - 1;
    K k[SORT_IPT];
    uint32_t v[SORT_IPT];
    rank_tables_init(sm.s.rt);
#pragma unroll
    for (int r = 0; r < SORT_IPT; ++r) {
        const uint32_t p = item_pos<SORT_NW, SORT_IPT>(r);
        k[r] = p < cnt ? b.piv[nd.piv + p] : (K)0;
    }
    __syncthreads();
    block_sort<K, false, SORT_NW, SORT_IPT>(k, v, cnt, sm);
#pragma unroll
    for (int r = 0; r < SORT_IPT; ++r) {
        const uint32_t p = item_pos<SORT_NW, SORT_IPT>(r);
        if (p < cnt) { b.piv[nd.piv + p] = k[r]; sm.k64[p] = (uint64_t)k[r]; }
    }
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < cnt; p += SORT_NT)
        b.strict[nd.piv + p] = (p + 1 < cnt && sm.k64[p] == sm.k64[p + 1]) ? 1 : 0;
}

// ------------------------------------------------------------ column phase
// One work-group per (node, column group).  Each column of the group is
// sorted in LDS (base case of the column children) unless the columns were
// already sorted by deeper recursion; then the sorted column is merged with
// the pivots by a galloping search per pivot.
template <class K, bool HV>
__global__ __launch_bounds__(SORT_NT) void k_colsort(Batch<K> b, const K *src, const uint32_t *vsrc,
                                                      K *dst, uint32_t *vdst, uint32_t cutoff)
{
    __shared__ SortSm sm;
    const uint32_t k = find_node(b.grpStart, b.N, blockIdx.x);
    const NodeDesc nd = b.nodes[k];
    const uint32_t g = blockIdx.x - b.grpStart[k];
    const uint32_t m = nd.m, n = nd.n, npiv = m - 1;
    const uint32_t i0 = g * TG;
    const uint32_t ncol = min((uint32_t)TG, m - i0);
    const bool cols_recursed = nd.flags & NODE_COLS_SORTED;
    const uint32_t ppt = (npiv + SORT_NT - 1) / SORT_NT;   // <= SORT_IPT
    const uint32_t t0 = threadIdx.x * ppt;

    K pv[SORT_IPT];
    bool ps[SORT_IPT];
    uint32_t P[SORT_IPT];
#pragma unroll
    for (int q = 0; q < SORT_IPT; ++q) {
        const uint32_t t = t0 + q;
        const bool ok = q < (int)ppt && t < npiv;
        pv[q] = ok ? b.piv[nd.piv + t] : (K)0;
        ps[q] = ok ? b.strict[nd.piv + t] != 0 : false;
        P[q] = 0;
    }
    rank_tables_init(sm.s.rt);
    __syncthreads();

    uint32_t total = 0;
    for (uint32_t c = 0; c < ncol; ++c) {
        const uint32_t i = i0 + c;
        const uint64_t lo = (uint64_t)i * m;
        const uint32_t len = lo < n ? (uint32_t)min((uint64_t)m, (uint64_t)n - lo) : 0u;
        total += len;
        if (len == 0) {
            for (uint32_t J = threadIdx.x; J <= nd.nJ; J += SORT_NT) b.srcOff[nd.src + (uint64_t)J * m + i] = 0;
            continue;
        }
        // columns larger than the cut-off were sorted by their own recursion
        const bool sorted = cols_recursed && len > cutoff;
        K kk[SORT_IPT];
        uint32_t vv[SORT_IPT];
        const uint64_t base = nd.off + lo;
        rank_tables_init(sm.s.rt);        // the previous column's search reused this LDS
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SORT_IPT; ++r) {
            const uint32_t p = item_pos<SORT_NW, SORT_IPT>(r);
            const bool ok = p < len;
            kk[r] = ok ? (sorted ? dst[base + p] : src[base + p]) : (K)0;
            if (HV) vv[r] = ok && !sorted ? vsrc[base + p] : 0u;
        }
        if (!sorted) {
            block_sort<K, HV, SORT_NW, SORT_IPT>(kk, vv, len, sm);
#pragma unroll
            for (int r = 0; r < SORT_IPT; ++r) {
                const uint32_t p = item_pos<SORT_NW, SORT_IPT>(r);
                if (p < len) {
                    dst[base + p] = kk[r];
                    if (HV) vdst[base + p] = vv[r];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SORT_IPT; ++r) {
            const uint32_t p = item_pos<SORT_NW, SORT_IPT>(r);
            if (p < len) { if (sizeof(K) == 4) sm.k32[p] = (uint32_t)kk[r]; else sm.k64[p] = (uint64_t)kk[r]; }
        }
        __syncthreads();
        // merge with the pivots: pos = number of keys at-or-below pivot t
        uint32_t prev = 0;
#pragma unroll
        for (int q = 0; q < SORT_IPT; ++q) {
            const uint32_t t = t0 + q;
            if (q < (int)ppt && t < npiv) {
                uint32_t a, e;
                if (q == 0) { a = 0; e = len; }
                else {
                    // gallop from the previous answer
                    a = prev; e = len;
                    uint32_t step = 1;
                    while (true) {
                        const uint32_t c2 = a + step - 1;
                        if (c2 >= len) break;
                        const K x = sizeof(K) == 4 ? (K)sm.k32[c2] : (K)sm.k64[c2];
                        if (!le_pivot(x, pv[q], ps[q])) { e = c2; break; }
                        a = c2 + 1;
                        step <<= 1;
                    }
                }
                while (a < e) {
                    const uint32_t mid = (a + e) >> 1;
                    const K x = sizeof(K) == 4 ? (K)sm.k32[mid] : (K)sm.k64[mid];
                    if (le_pivot(x, pv[q], ps[q])) a = mid + 1; else e = mid;
                }
                prev = a;
                P[q] += a;
                if ((t + 1) % TB == 0) b.srcOff[nd.src + (uint64_t)((t + 1) / TB) * m + i] = a;
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
    for (int q = 0; q < SORT_IPT; ++q) {
        const uint32_t t = t0 + q;
        if (q < (int)ppt && t < npiv) Pl[t] = P[q];
    }
    __syncthreads();
    uint32_t *blk = b.blk + nd.blk + (uint64_t)g * m;
#pragma unroll
    for (int q = 0; q < SORT_IPT; ++q) {
        const uint32_t t = t0 + q;
        if (q < (int)ppt && t < npiv) blk[t] = P[q] - (t > 0 ? Pl[t - 1] : 0u);
    }
    if (threadIdx.x == 0) blk[m - 1] = total - (npiv > 0 ? Pl[npiv - 1] : 0u);
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
    for (uint32_t g = 0; g < nd.groups; ++g) {
        uint32_t *p = b.blk + nd.blk + (uint64_t)g * nd.m + j;
        const uint32_t c = *p;
        *p = run;
        run += c;
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
    for (uint32_t q = 0; q < per; ++q) {
        if (j0 + q < m) {
            b.bs[nd.bkt + j0 + q] = run;
            if (bs64_out) bs64_out[j0 + q] = run;
            run += b.tot[nd.bkt + j0 + q];
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
template <class K> struct TileSmem {
    RankTables<TR_NW, TB> rt;
    uint32_t buf[TR_CH];
    uint8_t jl[TR_CH];
    uint32_t cOff[TG + 1];
    uint32_t aOf[TG];
    uint32_t dstb[TB];
    K piv[TB];
    uint8_t st[TB];
};

template <class K, bool HV>
__global__ __launch_bounds__(TR_NW * WAVE) void k_transpose(Batch<K> b, const K *src, const uint32_t *vsrc,
                                                            K *dst, uint32_t *vdst)
{
    __shared__ TileSmem<K> sm;
    using T = KeyT<K>;
    const uint32_t k = find_node(b.tileStart, b.N, blockIdx.x);
    const NodeDesc nd = b.nodes[k];
    const uint32_t tix = blockIdx.x - b.tileStart[k];
    const uint32_t g = tix / nd.nJ, J = tix % nd.nJ;
    const uint32_t m = nd.m;
    const uint32_t i0 = g * TG, ncol = min((uint32_t)TG, m - i0);
    const uint32_t j0 = J * TB, nb = min((uint32_t)TB, m - j0);
    const uint32_t npv = (j0 + nb <= m - 1) ? nb : nb - 1;   // real pivots of the block
    const uint32_t tid = threadIdx.x;

    rank_tables_init(sm.rt);
    if (tid < WAVE) {                      // one wave builds the run table
        uint32_t a = 0, len = 0;
        if (tid < ncol) {
            a = b.srcOff[nd.src + (uint64_t)J * m + i0 + tid];
            len = b.srcOff[nd.src + (uint64_t)(J + 1) * m + i0 + tid] - a;
        }
        const uint32_t incl = wave_incl_scan(len);
        if (tid < ncol) { sm.cOff[tid] = incl - len; sm.aOf[tid] = a; }
        if (tid == ncol - 1) sm.cOff[ncol] = incl;
    }
    if (tid < nb) {
        const uint32_t j = j0 + tid;
        sm.dstb[tid] = b.bs[nd.bkt + j] + b.blk[nd.blk + (uint64_t)g * m + j];
        if (tid < npv) { sm.piv[tid] = b.piv[nd.piv + j]; sm.st[tid] = b.strict[nd.piv + j]; }
    }
    __syncthreads();
    const uint32_t N = sm.cOff[ncol];

    for (uint32_t q0 = 0; q0 < N; q0 += TR_CH) {
        const uint32_t chN = min((uint32_t)TR_CH, N - q0);
        K kk[TR_IPT];
        uint32_t vv[TR_IPT], dig[TR_IPT], pos[TR_IPT];
#pragma unroll
        for (int r = 0; r < TR_IPT; ++r) {
            const uint32_t p = item_pos<TR_NW, TR_IPT>(r);
            kk[r] = (K)0;
            vv[r] = 0;
            dig[r] = TB - 1;
            if (p < chN) {
                const uint32_t q = q0 + p;
                uint32_t lo = 0, hi = ncol - 1;          // last column whose run starts at or before q
                while (lo < hi) {
                    const uint32_t mid = (lo + hi + 1) >> 1;
                    if (sm.cOff[mid] <= q) lo = mid; else hi = mid - 1;
                }
                const uint64_t rel = (uint64_t)(i0 + lo) * m + sm.aOf[lo] + (q - sm.cOff[lo]);
                const uint64_t at = nd.off + (rel < nd.n ? rel : 0);   // guard: stays inside the node
                kk[r] = src[at];
                if (HV) vv[r] = vsrc[at];
                uint32_t a = 0, e = npv;                  // bucket within the block
                while (a < e) {
                    const uint32_t mid = (a + e) >> 1;
                    if (le_pivot(kk[r], sm.piv[mid], sm.st[mid] != 0)) e = mid; else a = mid + 1;
                }
                dig[r] = a;
            }
        }
        rank_digits<TR_NW, TR_IPT, TB>(dig, pos, sm.rt);
#pragma unroll
        for (int wd = 0; wd < T::WORDS; ++wd) {
#pragma unroll
            for (int r = 0; r < TR_IPT; ++r) {
                sm.buf[pos[r]] = T::word(kk[r], wd);
                if (wd == 0) sm.jl[pos[r]] = (uint8_t)dig[r];
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < TR_IPT; ++r) kk[r] = T::set_word(kk[r], wd, sm.buf[item_pos<TR_NW, TR_IPT>(r)]);
            __syncthreads();
        }
        if (HV) {
#pragma unroll
            for (int r = 0; r < TR_IPT; ++r) sm.buf[pos[r]] = vv[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < TR_IPT; ++r) vv[r] = sm.buf[item_pos<TR_NW, TR_IPT>(r)];
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < TR_IPT; ++r) {
            const uint32_t p = item_pos<TR_NW, TR_IPT>(r);
            if (p < chN) {
                const uint32_t d = sm.jl[p];
                const uint64_t rel = (uint64_t)sm.dstb[d] + (p - sm.rt.offs[0][d]);
                if (rel < nd.n) {                                        // guard: stays inside the node
                    dst[nd.off + rel] = kk[r];
                    if (HV) vdst[nd.off + rel] = vv[r];
                }
            }
        }
        __syncthreads();
        if (tid < nb) {
            const uint32_t end = tid + 1 < TB ? sm.rt.offs[0][tid + 1] : (uint32_t)TR_CH;
            const uint32_t c = min(end, chN) - min(sm.rt.offs[0][tid], chN);
            sm.dstb[tid] += c;
        }
        __syncthreads();
    }
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
// A non-empty bucket admits exactly one key value (the appendix copies such
// buckets instead of recursing).  Inclusive bounds: U_j = s_j, or s_j - 1
// for a strict pivot, U_{m-1} = max; L_j = s_{j-1} + 1, or s_{j-1} after a
// strict pivot, L_0 = 0.
template <class K>
__device__ inline bool single_value_bucket(const Batch<K> &b, const NodeDesc &nd, uint32_t j)
{
    const K MAXV = (K)KeyT<K>::MAXV;
    const uint32_t m = nd.m;
    K lo, hi;
    if (j == 0) lo = 0;
    else { const K s = b.piv[nd.piv + j - 1]; lo = b.strict[nd.piv + j - 1] ? s : (K)(s + 1); }
    if (j == m - 1) hi = MAXV;
    else { const K s = b.piv[nd.piv + j]; hi = b.strict[nd.piv + j] ? (K)(s - 1) : s; }
    return lo == hi;
}

template <class K, bool HV>
__global__ __launch_bounds__(SORT_NT) void k_bucket(Batch<K> b, const K *A, const uint32_t *VA,
                                                     K *D, uint32_t *VD, uint32_t cutoff)
{
    __shared__ SortSm sm;
    const uint32_t k = find_node(b.bucStart, b.N, blockIdx.x);
    const NodeDesc nd = b.nodes[k];
    const uint32_t j = blockIdx.x - b.bucStart[k];
    const uint32_t lo = b.bs[nd.bkt + j], s = b.bs[nd.bkt + j + 1] - lo;
    const uint64_t base = nd.off + lo;
    uint8_t c;
    if (s == 0) c = 0;
    else if (single_value_bucket(b, nd, j)) {
        c = 1;
        for (uint32_t p = threadIdx.x; p < s; p += SORT_NT) {
            D[base + p] = A[base + p];
            if (HV) VD[base + p] = VA[base + p];
        }
    } else if (s <= cutoff) {
        c = 2;
        K kk[SORT_IPT];
        uint32_t vv[SORT_IPT];
        rank_tables_init(sm.s.rt);
#pragma unroll
        for (int r = 0; r < SORT_IPT; ++r) {
            const uint32_t p = item_pos<SORT_NW, SORT_IPT>(r);
            kk[r] = p < s ? A[base + p] : (K)0;
            if (HV) vv[r] = p < s ? VA[base + p] : 0u;
        }
        __syncthreads();
        block_sort<K, HV, SORT_NW, SORT_IPT>(kk, vv, s, sm);
#pragma unroll
        for (int r = 0; r < SORT_IPT; ++r) {
            const uint32_t p = item_pos<SORT_NW, SORT_IPT>(r);
            if (p < s) {
                D[base + p] = kk[r];
                if (HV) VD[base + p] = vv[r];
            }
        }
    } else c = 3;
    if (threadIdx.x == 0) b.cls[nd.bkt + j] = c;
}

// A whole (sub)array that is a base case: n <= cutoff, one work-group.
template <class K, bool HV>
__global__ __launch_bounds__(SORT_NT) void k_base_sort(uint32_t n, const K *A, const uint32_t *VA,
                                                        K *D, uint32_t *VD)
{
    __shared__ SortSm sm;
    K kk[SORT_IPT];
    uint32_t vv[SORT_IPT];
    rank_tables_init(sm.s.rt);
#pragma unroll
    for (int r = 0; r < SORT_IPT; ++r) {
        const uint32_t p = item_pos<SORT_NW, SORT_IPT>(r);
        kk[r] = p < n ? A[p] : (K)0;
        if (HV) vv[r] = p < n ? VA[p] : 0u;
    }
    __syncthreads();
    block_sort<K, HV, SORT_NW, SORT_IPT>(kk, vv, n, sm);
#pragma unroll
    for (int r = 0; r < SORT_IPT; ++r) {
        const uint32_t p = item_pos<SORT_NW, SORT_IPT>(r);
        if (p < n) {
            D[p] = kk[r];
            if (HV) VD[p] = vv[r];
        }
    }
}

}  // namespace sqs
