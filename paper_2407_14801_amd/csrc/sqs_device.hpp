// sqs_device.hpp -- device building blocks of libsquaresort (gfx950, wave64).
//
//  * the counter-based generator that draws pivot positions (SplitMix64 of
//    Steele, Lea and Flood, OOPSLA 2014, keyed per recursion node);
//  * key traits for u32 / u64 keys and the pivot rule;
//  * stable LSD radix sorts whose keys live in registers: a work-group sort
//    (up to NW*64*IPT keys) and a wave sort (up to 64*R keys, no barriers).
//
// Ranking is deterministic and stable without relying on the order in which
// the LDS serves colliding atomics.  Each wave owns a table with, per digit
// value, a 64-bit lane mask, a running count and an offset (three separate
// arrays).  For every 64-key row, each lane ORs its lane bit into its half of
// the mask of its digit (OR commutes, so the result does not depend on
// service order), reads the whole mask back, takes its rank among equal
// digits of the row with v_mbcnt, and every peer writes the same new count
// (old count + popcount of the mask) and clears the mask.  Rows are processed
// in position order, so ranks are stable; an exclusive scan of the counts
// then places every key.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sqs {

constexpr int WAVE = 64;

// ---------------------------------------------------------------- generator
__host__ __device__ inline uint64_t splitmix(uint64_t s)
{
    uint64_t z = s + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t node_child_key(uint64_t K, uint32_t phase, uint64_t i)
{
    return splitmix(K ^ splitmix(2 * i + phase));
}
// position of the t-th pivot draw of node K in an array of n items
__device__ inline uint32_t pivot_draw(uint64_t K, uint64_t t, uint32_t n)
{
    uint64_t u = splitmix(K ^ splitmix((1ull << 63) | t));
    return (uint32_t)__umul64hi(u, (uint64_t)n);
}
// draw t of sample attempt a under the Alg. 1 pivot rule (its own counter
// range: bits 63 and 62 set, the attempt in bits 32..61)
__device__ inline uint32_t pivot_draw_alg1(uint64_t K, uint32_t a, uint64_t t, uint32_t n)
{
    const uint64_t c = (3ull << 62) | ((uint64_t)(a & 0x3FFFFFFFu) << 32) | (t & 0xFFFFFFFFull);
    uint64_t u = splitmix(K ^ splitmix(c));
    return (uint32_t)__umul64hi(u, (uint64_t)n);
}

// ---------------------------------------------------------------- keys
template <class K> struct KeyT;
template <> struct KeyT<uint32_t> {
    static constexpr int WORDS = 1;
    static constexpr uint32_t MAXV = 0xFFFFFFFFu;
    __device__ static int bitlen(uint32_t x) { return x ? 32 - __clz(x) : 0; }
    __device__ static uint32_t word(uint32_t x, int) { return x; }
    __device__ static uint32_t set_word(uint32_t, int, uint32_t w) { return w; }
};
template <> struct KeyT<uint64_t> {
    static constexpr int WORDS = 2;
    static constexpr uint64_t MAXV = 0xFFFFFFFFFFFFFFFFull;
    __device__ static int bitlen(uint64_t x) { return x ? 64 - __clzll(x) : 0; }
    __device__ static uint32_t word(uint64_t x, int i) { return (uint32_t)(x >> (32 * i)); }
    __device__ static uint64_t set_word(uint64_t x, int i, uint32_t w)
    {
        return i == 0 ? ((x & 0xFFFFFFFF00000000ull) | w) : ((x & 0xFFFFFFFFull) | ((uint64_t)w << 32));
    }
};

// Pivot rule: key x belongs to bucket t or an earlier one iff x <= s_t, or
// x < s_t when the pivot is "strict" (followed by an equal pivot).
template <class K> __device__ inline bool le_pivot(K x, K s, bool strict)
{
    return strict ? (x < s) : (x <= s);
}

// ---------------------------------------------------------------- wave helpers
__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
// the wave index, as a wave-uniform (scalar) value
__device__ inline uint32_t wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE); }

// Waits until every vector memory access of the wave has completed.  Used
// right after a block of loads whose values feed per-row conditional code:
// without it the compiler cannot tell that the loads are complete on every
// path and waits for all memory accesses again before each later store,
// which serialises the stores.  (gfx9 encoding: vmcnt 0, expcnt and
// lgkmcnt at their maximum, i.e. not waited for.)
__device__ inline void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// orders this wave's LDS accesses before and after (no work-group barrier)
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint32_t rank_in_mask(uint32_t lo, uint32_t hi)
{
    return __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
}

// the value of lane l ^ j (j a power of two, a constant once unrolled):
// DPP lane moves inside rows of 16 lanes (j = 1, 2: quad permutations; 4: a
// half-row mirror then a quad reversal; 8: a row rotation by 8), a swizzle
// inside 32 lanes for 16, the LDS permute unit for 32 (for the bitonic
// networks of the on-chip nodes; the wave reductions keep the permute unit,
// which measured faster there)
__device__ inline uint32_t lane_xor(uint32_t x, int j)
{
    switch (j) {
    case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);    // quad_perm 1,0,3,2
    case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);    // quad_perm 2,3,0,1
    case 4: {
        const int t = __builtin_amdgcn_mov_dpp((int)x, 0x141, 0xF, 0xF, false);          // row_half_mirror
        return (uint32_t)__builtin_amdgcn_mov_dpp(t, 0x1B, 0xF, 0xF, false);             // quad_perm 3,2,1,0
    }
    case 8: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, false);   // row_ror 8
    case 16: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x401F);               // lane ^ 16 in 32
    default: return __shfl_xor(x, j, WAVE);
    }
}
template <class T> __device__ inline T wave_min(T v)
{
    for (int o = WAVE / 2; o > 0; o >>= 1) { T u = __shfl_xor(v, o, WAVE); v = u < v ? u : v; }
    return v;
}
template <class T> __device__ inline T wave_max(T v)
{
    for (int o = WAVE / 2; o > 0; o >>= 1) { T u = __shfl_xor(v, o, WAVE); v = u > v ? u : v; }
    return v;
}
// Inclusive scan over the 64 lanes (all lanes active): shifts within rows of
// 16 lanes, then the last lane of rows 0 and 2 into rows 1 and 3, then lane
// 31 into rows 2 and 3 (DPP row_shr / row_bcast, no LDS round trips).
__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}
__device__ inline unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// ---------------------------------------------------------------- ranking
// One wave's digit table: mask and count are zero between rows; off is
// written by the scan.  16 bytes per digit value.
template <int RDX> struct RankTab {
    unsigned long long mask[RDX];
    uint32_t cnt[RDX];
    uint32_t off[RDX];
};

// Rank one 64-key row against a wave's digit table: returns the count of
// equal digits in earlier rows plus the rank among equal digits of this row.
template <int RDX>
__device__ inline uint32_t rank_row(RankTab<RDX> &t, uint32_t d)
{
    const uint32_t l = lane_id();
    atomicOr(reinterpret_cast<uint32_t *>(&t.mask[d]) + (l >> 5), 1u << (l & 31));
    const unsigned long long pm = t.mask[d];
    const uint32_t old = t.cnt[d];
    t.cnt[d] = old + (uint32_t)__popcll(pm);
    t.mask[d] = 0ull;
    return old + rank_in_mask((uint32_t)pm, (uint32_t)(pm >> 32));
}

// clears one wave's table with that wave's lanes
template <int RDX>
__device__ inline void wave_table_clear(RankTab<RDX> &t)
{
    for (int i = lane_id(); i < RDX; i += WAVE) { t.mask[i] = 0ull; t.cnt[i] = 0u; }
}

// ---------------------------------------------------------------- block sort
// Work-group sort of up to CAP = NW*64*IPT keys.  Thread (w, lane) holds the
// keys at positions w*IPT*64 + r*64 + lane, r < IPT.  Shared memory: the
// per-wave digit tables and one 32-bit exchange buffer; once a sort has
// returned, the whole region may be reused.
template <int NW, int IPT> struct SortSmem {
    static constexpr int CAP = NW * WAVE * IPT;
    union {
        struct {
            RankTab<256> tab[NW];
            uint32_t buf[CAP];
            uint32_t pad[16];        // the bin sort's all-ones words after the last key
        } s;
        uint64_t k64[CAP];
        uint32_t k32[2 * CAP];
    };
    uint32_t wsum[NW];
    uint32_t red32[2 * NW];
    unsigned long long red64[2 * NW];
    // the bin sort's per-wave list of bins of more than 8 keys (start, size)
    static constexpr int BLW = NW >= 16 ? 64 : 32;
    uint2 bl[NW][BLW];
};

template <int NW, int IPT>
__device__ inline uint32_t item_pos(int r)
{
    // per-lane arithmetic on threadIdx (no scalar wave index), so that the
    // row-independent part is computed once rather than in every row's branch
    const uint32_t t = threadIdx.x;
    return (t / WAVE) * (IPT * WAVE) + (t % WAVE) + (uint32_t)r * WAVE;
}

// rows of the calling wave that hold at least one of the first `count` positions
template <int IPT>
__device__ inline int wave_rows(uint32_t count)
{
    const int64_t left = (int64_t)count - (int64_t)wave_id() * IPT * WAVE;
    if (left <= 0) return 0;
    const int64_t r = (left + WAVE - 1) / WAVE;
    return r < IPT ? (int)r : IPT;
}

// A block sort of `count` keys gives every wave R rows, the fewest that hold
// them (R <= IPT), so that all waves share the work.  Row r of the calling
// wave holds positions bpos(r, R) = (wave * R + r) * 64 + lane.
template <int NW, int IPT>
__device__ inline int block_rows(uint32_t count)
{
    const uint32_t R = (count + NW * WAVE - 1) / (NW * WAVE);
    return R < 1u ? 1 : (R > (uint32_t)IPT ? IPT : (int)R);
}
__device__ inline uint32_t bpos(int r, int R)
{
    const uint32_t t = threadIdx.x;
    return (t / WAVE) * (uint32_t)R * WAVE + (t % WAVE) + (uint32_t)r * WAVE;
}
// rows of the calling wave (of R) that hold at least one of the first count positions
__device__ inline int wave_rows_of(uint32_t count, int R)
{
    const int64_t left = (int64_t)count - (int64_t)wave_id() * R * WAVE;
    if (left <= 0) return 0;
    const int64_t r = (left + WAVE - 1) / WAVE;
    return r < R ? (int)r : R;
}

template <int NW, int RDX>
__device__ inline void tables_clear(RankTab<RDX> *tab)
{
    for (int i = threadIdx.x; i < NW * RDX; i += NW * WAVE) {
        tab[i / RDX].mask[i % RDX] = 0ull;
        tab[i / RDX].cnt[i % RDX] = 0u;
    }
}

// Work-group min and max.  Without trailing_sync the caller must pass a
// barrier before red32 / red64 are written again.
template <class K, int NW, bool trailing_sync = true>
__device__ inline void block_minmax(K &lo, K &hi, uint32_t *red32, unsigned long long *red64)
{
    lo = wave_min(lo);
    hi = wave_max(hi);
    const uint32_t w = wave_id();
    if (sizeof(K) == 4) {
        if (lane_id() == 0) { red32[w] = (uint32_t)lo; red32[NW + w] = (uint32_t)hi; }
        __syncthreads();
        uint32_t a = red32[0], b = red32[NW];
        for (int i = 1; i < NW; ++i) { a = min(a, red32[i]); b = max(b, red32[NW + i]); }
        lo = (K)a; hi = (K)b;
    } else {
        if (lane_id() == 0) { red64[w] = (unsigned long long)lo; red64[NW + w] = (unsigned long long)hi; }
        __syncthreads();
        unsigned long long a = red64[0], b = red64[NW];
        for (int i = 1; i < NW; ++i) { a = min(a, red64[i]); b = max(b, red64[NW + i]); }
        lo = (K)a; hi = (K)b;
    }
    if (trailing_sync) __syncthreads();
}

// Digit-major, wave-minor exclusive scan of the per-wave counts of RDX digit
// values: off := first position of (digit, wave); cnt := 0.  wsum has NW
// words.  Two barriers inside; call after a barrier that follows ranking.
template <int NW, int RDX>
__device__ inline void scan_tables(RankTab<RDX> *tab, uint32_t *wsum)
{
    static_assert(RDX <= NW * WAVE, "one thread per digit value");
    const uint32_t t = threadIdx.x;
    uint32_t c[NW], tot = 0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
        c[ww] = t < (uint32_t)RDX ? tab[ww].cnt[t] : 0u;
        tot += c[ww];
    }
    const uint32_t incl = wave_incl_scan(tot);
    if (lane_id() == WAVE - 1) wsum[wave_id()] = incl;
    __syncthreads();
    if (t < (uint32_t)RDX) {
        uint32_t run = incl - tot;
        for (uint32_t ww = 0; ww < wave_id(); ++ww) run += wsum[ww];
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            tab[ww].off[t] = run;
            tab[ww].cnt[t] = 0u;
            run += c[ww];
        }
    }
    __syncthreads();
}

// 8-bit digit at bit sh (a multiple of 8) of a key
__device__ inline uint32_t digit8(uint32_t x, int sh) { return (x >> sh) & 255u; }
__device__ inline uint32_t digit8(uint64_t x, int sh)
{
    const uint32_t w = sh < 32 ? (uint32_t)x : (uint32_t)(x >> 32);
    return (w >> (sh & 31)) & 255u;
}

// Stable LSD radix sort of `count` keys (and values) in registers, laid out
// by block_rows / bpos (callers load and store with the same layout);
// positions >= count are padding and stay at the end.  Only the bits in which the keys
// differ are sorted: keys are offset by their minimum and ceil(bits/8) 8-bit
// passes run.  Padding positions of the ranked rows hold the all-ones offset
// key, whose digit is 255 in every pass, so they stay behind every real key
// without a per-key test in the passes.  With `bounded`, [blo, bhi] is a
// caller-known range of the keys and replaces the block-wide min/max.  Tables
// must be clear on entry (tables_clear + barrier); they are clear again on
// return.  Ends with a barrier unless it returns at once (count <= 1 or a
// single key value).  On return only positions < count hold meaningful keys.
// With passes_out (and lo_out), the passes run and the offset: when at least
// one pass ran for keys without values, sm.s.buf holds the sorted keys minus
// lo (word 0 for 64-bit keys), and sm.s.tab[0].off[d] is the first position
// of the keys whose last-pass digit is d (padding sorts last).
template <class K, bool HV, int NW, int IPT>
__device__ void block_sort(K (&k)[IPT], uint32_t (&v)[IPT], uint32_t count, SortSmem<NW, IPT> &sm,
                           bool bounded = false, K blo = (K)0, K bhi = (K)0, K *lo_out = nullptr,
                           int *passes_out = nullptr)
{
    using T = KeyT<K>;
    const int R = block_rows<NW, IPT>(count);
    const int nrows = wave_rows_of(count, R);
    K lo = blo, hi = bhi;                          // bounded: every key lies in [blo, bhi]
    if (!bounded) {
        lo = (K)T::MAXV;
        hi = (K)0;
#pragma unroll
        for (int r = 0; r < IPT; ++r)
            if (r < nrows && bpos(r, R) < count) { lo = k[r] < lo ? k[r] : lo; hi = k[r] > hi ? k[r] : hi; }
        block_minmax<K, NW>(lo, hi, sm.red32, sm.red64);
    }
    if (passes_out) *passes_out = 0;
    if (count <= 1 || !(lo < hi)) return;          // already in order (uniform branch)
    const int passes = (T::bitlen((K)(hi - lo)) + 7) / 8;
    if (lo_out) *lo_out = lo;
    if (passes_out) *passes_out = passes;
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (r < nrows) k[r] = bpos(r, R) < count ? (K)(k[r] - lo) : (K)T::MAXV;
    RankTab<256> &tab = sm.s.tab[wave_id()];
    uint32_t pos[IPT];
    for (int ps = 0; ps < passes; ++ps) {
        const int sh = 8 * ps;
#pragma unroll
        for (int r = 0; r < IPT; ++r)
            if (r < nrows) pos[r] = rank_row(tab, digit8(k[r], sh));
        __syncthreads();
        scan_tables<NW, 256>(sm.s.tab, sm.wsum);
#pragma unroll
        for (int r = 0; r < IPT; ++r)
            if (r < nrows) pos[r] += tab.off[digit8(k[r], sh)];
        // move keys (and values) word by word through the exchange buffer
#pragma unroll
        for (int wd = 0; wd < T::WORDS; ++wd) {
#pragma unroll
            for (int r = 0; r < IPT; ++r)
                if (r < nrows) sm.s.buf[pos[r]] = T::word(k[r], wd);
            __syncthreads();
#pragma unroll
            for (int r = 0; r < IPT; ++r)
                if (r < nrows) k[r] = T::set_word(k[r], wd, sm.s.buf[bpos(r, R)]);
            __syncthreads();
        }
        if (HV) {
#pragma unroll
            for (int r = 0; r < IPT; ++r)
                if (r < nrows) sm.s.buf[pos[r]] = v[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < IPT; ++r)
                if (r < nrows) v[r] = sm.s.buf[bpos(r, R)];
            __syncthreads();
        }
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (r < nrows) k[r] = (K)(k[r] + lo);
}

// ------------------------------------------------------------ bin sort (u32)
// Batcher's odd-even merge sort over N registers (N a power of two),
// ascending: 5 / 19 / 63 compare-exchanges for N = 4 / 8 / 16 (a bitonic
// network needs 6 / 24 / 80).  Merging runs of length p, it compares the
// elements k apart (k = p, p/2, .., 1) that lie in the same run pair of
// length 2p, starting at offset k mod p.
template <int N>
__device__ inline void oddeven_regs(uint32_t (&x)[N])
{
#pragma unroll
    for (int p = 1; p < N; p <<= 1) {
#pragma unroll
        for (int k = p; k >= 1; k >>= 1) {
#pragma unroll
            for (int j = k % p; j + k < N; j += 2 * k) {
#pragma unroll
                for (int i = 0; i < k; ++i) {
                    const int lo = i + j, hi = i + j + k;
                    if (hi < N && lo / (2 * p) == hi / (2 * p)) {
                        const uint32_t a = x[lo], c = x[hi];
                        x[lo] = min(a, c);
                        x[hi] = max(a, c);
                    }
                }
            }
        }
    }
}

// Sorts the c <= N keys at buf[s ..), the keys of one bin (lanes with c < 2
// leave theirs alone).  It reads N words from s on without a bounds test:
// the words past the bin hold keys of later bins (sorted or not yet) or the
// all-ones words the bin sort put after the last key, all at least as large
// as the bin's keys, so the first c outputs of the network are the bin's
// keys in order; only those are written back.
template <int N>
__device__ inline void bin_net(uint32_t *buf, uint32_t s, uint32_t c)
{
    uint32_t x[N];
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = buf[s + j];
    oddeven_regs<N>(x);
#pragma unroll
    for (int j = 0; j < N; ++j)
        if ((uint32_t)j < c && c > 1) buf[s + j] = x[j];
}

constexpr int BIN_NET = 16;                  // largest bin sorted in registers (a 32-key
                                             // network needs twice the registers)
static_assert(BIN_NET <= 16, "the pad words of SortSmem and WaveSmem cover a network's reads");

// Sort of `count` 32-bit keys without values (block_rows / bpos layout) by
// bins of the key range: bin = (key - lo) >> sh for the fewest bins of equal
// width, about count/4 and at most bin_cap (uniform keys overfill a bin of
// 16 about once in a million bins; bins of one key value need no sort and
// have no size limit); every key takes its place in
// its bin from an LDS atomic add (equal keys are interchangeable when no
// values ride along, so the order among them does not matter), a scan lays
// the bins out, and every bin of at most BIN_NET keys is sorted in registers
// by one thread.  With `bounded`, [blo, bhi] is a caller-known range of the
// keys (as in block_sort).  Returns 0 when nothing is to be sorted (count <= 1
// or one key value), 2 when a bin holds more than BIN_NET keys (nothing has been
// moved; the digit tables are not clear), and 1 after sorting: then k holds
// the sorted keys, sm.s.buf the sorted keys minus lo, and the words
// bin_starts(sm)[0 .. nbin) the first position of every bin.  No LDS write
// is pending on return.
// bins of one sort: counts and starts share the digit tables' space
template <int NW, int IPT> constexpr int bin_cap()
{
    return (int)sizeof(RankTab<256>) * NW / 8 < 4096 ? (int)sizeof(RankTab<256>) * NW / 8 : 4096;
}
template <int NW, int IPT>
__device__ inline uint32_t *bin_starts(SortSmem<NW, IPT> &sm)
{
    return reinterpret_cast<uint32_t *>(sm.s.tab) + bin_cap<NW, IPT>();
}

template <int NW, int IPT>
__device__ int bin_sort(uint32_t (&k)[IPT], uint32_t count, SortSmem<NW, IPT> &sm, uint32_t &lo_out,
                        int &sh_out, uint32_t &nbin_out, bool bounded = false, uint32_t blo = 0u,
                        uint32_t bhi = 0u)
{
    constexpr int NT = NW * WAVE;
    constexpr int BIN_CAP = bin_cap<NW, IPT>();
    constexpr int BPT = BIN_CAP / NT;              // bins BPT*t .. BPT*t + BPT - 1 belong to thread t
    static_assert(BPT >= 1 && BPT * NT == BIN_CAP, "whole bins per thread");
    static_assert(2 * BIN_CAP * 4 <= (int)sizeof(sm.s.tab), "bin counts and starts fit the tables");
    const int R = block_rows<NW, IPT>(count);
    const int nrows = wave_rows_of(count, R);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(sm.s.tab);
    uint32_t *st = cnt + BIN_CAP;
    uint32_t lo = blo, hi = bhi;                   // bounded: every key lies in [blo, bhi]
    for (uint32_t i = threadIdx.x; i < (uint32_t)BIN_CAP; i += NT) cnt[i] = 0u;
    if (bounded) {
        __syncthreads();
    } else {
        lo = 0xffffffffu;
        hi = 0u;
#pragma unroll
        for (int r = 0; r < IPT; ++r)
            if (r < nrows && bpos(r, R) < count) { lo = min(lo, k[r]); hi = max(hi, k[r]); }
        // red32 is written again only after the barrier that follows the
        // atomic adds (or, on return, after a caller's barrier)
        block_minmax<uint32_t, NW, false>(lo, hi, sm.red32, sm.red64);
    }
    if (count <= 1 || !(lo < hi)) return 0;
    const int nb = min(max(KeyT<uint32_t>::bitlen(count) - 2, 1), KeyT<uint32_t>::bitlen(BIN_CAP) - 1);
    const int kb = KeyT<uint32_t>::bitlen(hi - lo);
    const int sh = kb > nb ? kb - nb : 0;
    const uint32_t nbin = ((hi - lo) >> sh) + 1u;
    uint32_t rk[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (r < nrows && bpos(r, R) < count) rk[r] = atomicAdd(&cnt[(k[r] - lo) >> sh], 1u);
    __syncthreads();
    const uint32_t t = threadIdx.x, w = wave_id();
    uint32_t c[BPT], tot = 0u;
    bool big = false;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
        const uint32_t bb = BPT * t + q;
        c[q] = bb < nbin ? cnt[bb] : 0u;
        tot += c[q];
        big |= c[q] > (uint32_t)BIN_NET;
    }
    const uint32_t incl = wave_incl_scan(tot);
    const bool over = sh > 0 && __ballot(big) != 0ull;   // a bin of one key value needs no sort
    if (lane_id() == WAVE - 1) { sm.wsum[w] = incl; sm.red32[w] = over ? 1u : 0u; }
    __syncthreads();
    uint32_t run = incl - tot;
    bool any = false;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
        if ((uint32_t)ww < w) run += sm.wsum[ww];
        any |= sm.red32[ww] != 0u;
    }
    if (any) return 2;                             // uniform over the work-group
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
        if (BPT * t + q < nbin) st[BPT * t + q] = run;
        run += c[q];
    }
    if (t < (uint32_t)BIN_NET) sm.s.buf[count + t] = 0xffffffffu;   // above every key (minus lo)
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (r < nrows && bpos(r, R) < count) {
            const uint32_t x = k[r] - lo;
            sm.s.buf[st[x >> sh] + rk[r]] = x;
        }
    __syncthreads();
    // Bins of at most 8 keys (all but about 2% for uniform keys) by 4- or
    // 8-key networks, as large as the wave's largest such bin needs; the
    // wave's larger bins are then listed and sorted together, one per lane,
    // by 16-key networks (or, past the list's room, iteration by iteration).
    // A network sized by every bin of the wave would mostly be the 16-key one.
    uint32_t bigit = 0u;                           // iterations whose bin holds more than 8 keys
    if (sh > 0) {
#pragma unroll 1
        for (int it = 0; it < BPT; ++it) {
            if ((uint32_t)it * NT >= nbin) break;     // no bin left (uniform)
            const uint32_t bb = t + (uint32_t)it * NT;
            const uint32_t cb = bb < nbin ? cnt[bb] : 0u;
            const uint32_t s = bb < nbin ? st[bb] : 0u;
            const bool big = cb > 8u;
            bigit |= (big ? 1u : 0u) << it;
            const uint32_t cs = big ? 0u : cb;
            const uint32_t cm = wave_max(cs);        // uniform within the wave
            if (cm <= 1u) continue;
            if (cm <= 4u) bin_net<4>(sm.s.buf, s, cs);
            else bin_net<8>(sm.s.buf, s, cs);
        }
        const uint32_t nbig = (uint32_t)__popc(bigit);
        const uint32_t incl = wave_incl_scan(nbig);
        const uint32_t tot = __shfl(incl, WAVE - 1, WAVE);
        if (tot > 0u) {
            constexpr int BLW = SortSmem<NW, IPT>::BLW;
            if (tot <= (uint32_t)BLW) {
                uint2 *bl = sm.bl[w];
                uint32_t o = incl - nbig;
#pragma unroll 1
                for (int it = 0; it < BPT; ++it) {
                    if ((bigit >> it) & 1u) {
                        const uint32_t bb = t + (uint32_t)it * NT;
                        bl[o++] = make_uint2(st[bb], cnt[bb]);
                    }
                }
                wave_lds_sync();
                const uint32_t l = lane_id();
                if (l < tot) {
                    const uint2 e = bl[l];
                    bin_net<16>(sm.s.buf, e.x, e.y);
                }
            } else {
#pragma unroll 1
                for (int it = 0; it < BPT; ++it) {
                    if (__ballot((bigit >> it) & 1u) == 0ull) continue;
                    const uint32_t bb = t + (uint32_t)it * NT;
                    const bool big = (bigit >> it) & 1u;
                    bin_net<16>(sm.s.buf, big ? st[bb] : 0u, big ? cnt[bb] : 0u);
                }
            }
        }
    }
    __syncthreads();
    // every row (positions past count read stale words of the buffer, which
    // stays in bounds: bpos(r, R) < NW * IPT * 64), so that no old key stays
    // live across the bin sorts
#pragma unroll
    for (int r = 0; r < IPT; ++r) k[r] = sm.s.buf[bpos(r, R)] + lo;
    lo_out = lo;
    sh_out = sh;
    nbin_out = nbin;
    return 1;
}

// Loads the keys (and values) at from[0 .. count) in block_rows / bpos layout.
template <class K, bool HV, int NW, int IPT>
__device__ inline void block_load(K (&k)[IPT], uint32_t (&v)[IPT], uint32_t count, const K *from,
                                  const uint32_t *vfrom)
{
    const int R = block_rows<NW, IPT>(count);
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t p = bpos(r, R);
        const bool ok = r < R && p < count;
        k[r] = ok ? from[p] : (K)0;
        if (HV) v[r] = ok ? vfrom[p] : 0u;
    }
    wait_vmem();
}

// Work-group LDS sort of `count` keys known to lie in [blo, bhi], loaded by
// block_load from `from`, which still holds them: by bins for 32-bit keys
// without values (when a bin is crowded, the keys are loaded again, so that
// the registers of the first load are free during the bin sort, and sorted
// by radix passes), by radix passes otherwise.  The digit tables must be
// clear on entry; on return they are clear only for the other key types.
template <class K, bool HV, int NW, int IPT>
__device__ inline void lds_sort(K (&k)[IPT], uint32_t (&v)[IPT], uint32_t count, SortSmem<NW, IPT> &sm, K blo,
                                K bhi, const K *from)
{
    if constexpr (sizeof(K) == 4 && !HV) {
        uint32_t lo, nbin;
        int sh;
        if (bin_sort<NW, IPT>(k, count, sm, lo, sh, nbin, true, (uint32_t)blo, (uint32_t)bhi) != 2) return;
        block_load<K, HV, NW, IPT>(k, v, count, from, nullptr);
        tables_clear<NW, 256>(sm.s.tab);
        __syncthreads();
    }
    block_sort<K, HV, NW, IPT>(k, v, count, sm, true, blo, bhi);
}

// ---------------------------------------------------------------- wave sort
// One wave sorts up to 64*R keys at positions r*64 + lane with its own table
// and buffer; no work-group barrier.  The table must be clear on entry and is
// clear on return (its counts; the offsets of the last pass remain).  With
// passes_out and lo_out as in block_sort: after at least one pass over keys
// without values, sm.buf holds the sorted keys minus lo (word 0) and
// sm.tab.off[d] the first position of last-pass digit d.
template <int R> struct WaveSmem {
    RankTab<256> tab;
    uint32_t buf[R * WAVE];
    uint32_t pad[16];                // the bin sort's all-ones words after the last key
};

template <class K, bool HV, int R>
__device__ void wave_sort(K (&k)[R], uint32_t (&v)[R], uint32_t count, WaveSmem<R> &sm, K *lo_out = nullptr,
                          int *passes_out = nullptr)
{
    using T = KeyT<K>;
    const uint32_t l = lane_id();
    const int nrows = (int)min((count + WAVE - 1) / WAVE, (uint32_t)R);
    K lo = (K)T::MAXV, hi = (K)0;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r < nrows && r * WAVE + l < count) { lo = k[r] < lo ? k[r] : lo; hi = k[r] > hi ? k[r] : hi; }
    lo = wave_min(lo);
    hi = wave_max(hi);
    if (passes_out) *passes_out = 0;
    if (count <= 1 || !(lo < hi)) return;
    const int passes = (T::bitlen((K)(hi - lo)) + 7) / 8;
    if (lo_out) *lo_out = lo;
    if (passes_out) *passes_out = passes;
    // offset keys; padding gets the all-ones key (digit 255 in every pass)
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r < nrows) k[r] = r * WAVE + l < count ? (K)(k[r] - lo) : (K)T::MAXV;
    uint32_t pos[R];
    for (int ps = 0; ps < passes; ++ps) {
        const int sh = 8 * ps;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r < nrows) pos[r] = rank_row(sm.tab, digit8(k[r], sh));
        wave_lds_sync();
        // exclusive scan over the 256 digit counts: lane l owns digits 4l..4l+3
        {
            const uint4 c = *reinterpret_cast<const uint4 *>(&sm.tab.cnt[4 * l]);
            const uint32_t s = c.x + c.y + c.z + c.w;
            const uint32_t run = wave_incl_scan(s) - s;
            *reinterpret_cast<uint4 *>(&sm.tab.off[4 * l]) =
                make_uint4(run, run + c.x, run + c.x + c.y, run + c.x + c.y + c.z);
            *reinterpret_cast<uint4 *>(&sm.tab.cnt[4 * l]) = make_uint4(0u, 0u, 0u, 0u);
        }
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r < nrows) pos[r] += sm.tab.off[digit8(k[r], sh)];
#pragma unroll
        for (int wd = 0; wd < T::WORDS; ++wd) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < nrows) sm.buf[pos[r]] = T::word(k[r], wd);
            wave_lds_sync();
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < nrows) k[r] = T::set_word(k[r], wd, sm.buf[r * WAVE + l]);
            wave_lds_sync();
        }
        if (HV) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < nrows) sm.buf[pos[r]] = v[r];
            wave_lds_sync();
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < nrows) v[r] = sm.buf[r * WAVE + l];
            wave_lds_sync();
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r < nrows) k[r] = (K)(k[r] + lo);
}

// Wave-level bin sort of up to 64*R 32-bit keys without values (positions
// r*64 + lane), as bin_sort with the wave's own table space: at most 256
// bins of about 4 keys, counts at the table's words [0, 256), starts at
// [256, 512), lane l scanning bins 4l .. 4l+3 and sorting bins l, l+64,
// l+128, l+192.  Returns 0 (nothing to sort), 1 (sorted: k, sm.buf = keys
// minus lo, bin starts at wave_bin_starts(sm)) or 2 (a crowded bin, nothing
// moved).  Either way the table is no longer clear: clear it
// (wave_table_clear) before the next wave_sort.
template <int R>
__device__ inline uint32_t *wave_bin_starts(WaveSmem<R> &sm)
{
    return reinterpret_cast<uint32_t *>(&sm.tab) + 256;
}

template <int R>
__device__ int wave_bin_sort(uint32_t (&k)[R], uint32_t count, WaveSmem<R> &sm, uint32_t &lo_out, int &sh_out,
                             uint32_t &nbin_out)
{
    static_assert(512 * 4 <= (int)sizeof(RankTab<256>), "counts and starts fit the table");
    const uint32_t l = lane_id();
    const int nrows = (int)min((count + WAVE - 1) / WAVE, (uint32_t)R);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(&sm.tab);
    uint32_t *st = cnt + 256;
    uint32_t lo = 0xffffffffu, hi = 0u;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r < nrows && r * WAVE + l < count) { lo = min(lo, k[r]); hi = max(hi, k[r]); }
    lo = wave_min(lo);
    hi = wave_max(hi);
    if (count <= 1 || !(lo < hi)) return 0;
    *reinterpret_cast<uint4 *>(&cnt[4 * l]) = make_uint4(0u, 0u, 0u, 0u);
    const int nb = min(max(KeyT<uint32_t>::bitlen(count) - 2, 1), 8);
    const int kb = KeyT<uint32_t>::bitlen(hi - lo);
    const int sh = kb > nb ? kb - nb : 0;
    const uint32_t nbin = ((hi - lo) >> sh) + 1u;
    wave_lds_sync();
    uint32_t rk[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r < nrows && r * WAVE + l < count) rk[r] = atomicAdd(&cnt[(k[r] - lo) >> sh], 1u);
    wave_lds_sync();
    const uint4 c = *reinterpret_cast<const uint4 *>(&cnt[4 * l]);   // bins >= nbin hold 0
    const bool big = c.x > (uint32_t)BIN_NET || c.y > (uint32_t)BIN_NET || c.z > (uint32_t)BIN_NET ||
                     c.w > (uint32_t)BIN_NET;
    if (sh > 0 && __ballot(big) != 0ull) return 2;   // uniform within the wave
    const uint32_t s4 = c.x + c.y + c.z + c.w;
    const uint32_t run = wave_incl_scan(s4) - s4;
    *reinterpret_cast<uint4 *>(&st[4 * l]) = make_uint4(run, run + c.x, run + c.x + c.y, run + c.x + c.y + c.z);
    if (l < (uint32_t)BIN_NET) sm.buf[count + l] = 0xffffffffu;      // above every key (minus lo)
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r < nrows && r * WAVE + l < count) {
            const uint32_t x = k[r] - lo;
            sm.buf[st[x >> sh] + rk[r]] = x;
        }
    wave_lds_sync();
    if (sh > 0) {
#pragma unroll 1
        for (uint32_t bb = l; bb - l < nbin; bb += WAVE) {
            const uint32_t cb = bb < nbin ? cnt[bb] : 0u;
            const uint32_t s = bb < nbin ? st[bb] : 0u;
            const uint32_t cm = wave_max(cb);
            if (cm <= 1u) continue;
            if (cm <= 4u) bin_net<4>(sm.buf, s, cb);
            else if (cm <= 8u) bin_net<8>(sm.buf, s, cb);
            else bin_net<16>(sm.buf, s, cb);
        }
        wave_lds_sync();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) k[r] = sm.buf[r * WAVE + l] + lo;   // every row: buf has 64*R words
    lo_out = lo;
    sh_out = sh;
    nbin_out = nbin;
    return 1;
}

}  // namespace sqs
