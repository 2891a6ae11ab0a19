// sqs_device.hpp -- device building blocks of libsquaresort (gfx950, wave64).
//
//  * the counter-based generator that draws pivot positions (SplitMix64 of
//    Steele, Lea and Flood, OOPSLA 2014, keyed per recursion node);
//  * key traits for u32 / u64 keys;
//  * a stable work-group radix sort whose keys live in registers and whose
//    LDS holds only the rank tables and one 32-bit exchange buffer.
//
// Ranking is deterministic and stable without relying on the order in which
// the LDS serves colliding atomics: for every 64-key row of a wave, each lane
// ORs its lane bit into a per-wave 64-bit mask of its digit (OR commutes, so
// the mask is the same whatever the service order), reads the mask back, and
// gets its rank among equal digits of the row with v_mbcnt and the row count
// with v_bcnt.  Rows are processed in order, so ranks follow the position
// order (wave, row, lane); a digit-major / wave-minor exclusive scan of the
// per-wave counts then gives every key its destination.
#pragma once

#include <hip/hip_runtime.h>
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

// ---------------------------------------------------------------- keys
template <class K> struct KeyT;
template <> struct KeyT<uint32_t> {
    static constexpr int BITS = 32;
    static constexpr int WORDS = 1;
    static constexpr uint32_t MAXV = 0xFFFFFFFFu;
    __device__ static int bitlen(uint32_t x) { return x ? 32 - __clz(x) : 0; }
    __device__ static uint32_t word(uint32_t x, int) { return x; }
    __device__ static uint32_t set_word(uint32_t, int, uint32_t w) { return w; }
};
template <> struct KeyT<uint64_t> {
    static constexpr int BITS = 64;
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
__device__ inline uint32_t lane_id() { return threadIdx.x & (WAVE - 1); }
__device__ inline uint32_t wave_id() { return threadIdx.x / WAVE; }

__device__ inline uint32_t rank_in_mask(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
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
__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    const uint32_t l = lane_id();
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t u = __shfl_up(v, o, WAVE);
        if (l >= (uint32_t)o) v += u;
    }
    return v;
}
__device__ inline unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// ---------------------------------------------------------------- rank tables
// Per-wave digit tables for a ranking pass over RDX digit values.
template <int NW, int RDX> struct RankTables {
    unsigned long long mask[NW][RDX];
    uint32_t cnt[NW][RDX];
    uint32_t offs[NW][RDX];
    uint32_t wsum[NW];
};

template <int NW, int RDX>
__device__ inline void rank_tables_init(RankTables<NW, RDX> &rt)
{
    for (int i = threadIdx.x; i < NW * RDX; i += NW * WAVE) {
        (&rt.mask[0][0])[i] = 0ull;
        (&rt.cnt[0][0])[i] = 0u;
    }
}

// Stable ranking of IPT digits per thread.  Thread (w, lane) holds the keys
// at positions w*IPT*64 + r*64 + lane.  On return pos[r] is the destination
// position of key r; offs[0][d] is the first position of digit d.  Requires
// the mask table zero and cnt zero on entry; leaves both zero.  Contains two
// work-group barriers.
template <int NW, int IPT, int RDX>
__device__ inline void rank_digits(const uint32_t (&dig)[IPT], uint32_t (&pos)[IPT],
                                   RankTables<NW, RDX> &rt)
{
    const uint32_t l = lane_id(), w = wave_id();
    const unsigned long long bit = 1ull << l;
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t d = dig[r];
        atomicOr(&rt.mask[w][d], bit);
        const unsigned long long pm =
            __hip_atomic_load(&rt.mask[w][d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const uint32_t old = rt.cnt[w][d];
        pos[r] = old + rank_in_mask(pm);
        rt.cnt[w][d] = old + (uint32_t)__popcll(pm);   // every peer stores the same value
        rt.mask[w][d] = 0ull;                            // likewise
    }
    __syncthreads();
    // digit-major, wave-minor exclusive scan of the per-wave counts
    constexpr int NT = NW * WAVE;
    static_assert(RDX <= NT, "one thread per digit");
    const uint32_t t = threadIdx.x;
    uint32_t c[NW];
    uint32_t tot = 0;
    if (t < (uint32_t)RDX) {
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) { c[ww] = rt.cnt[ww][t]; tot += c[ww]; }
    }
    const uint32_t incl = wave_incl_scan(tot);
    if (l == WAVE - 1) rt.wsum[w] = incl;
    __syncthreads();
    if (t < (uint32_t)RDX) {
        uint32_t run = incl - tot;
        for (uint32_t ww = 0; ww < w; ++ww) run += rt.wsum[ww];
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            rt.offs[ww][t] = run;
            run += c[ww];
            rt.cnt[ww][t] = 0u;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r) pos[r] += rt.offs[w][dig[r]];
}

// ---------------------------------------------------------------- block sort
// Shared memory of the block sort: rank tables plus a 32-bit exchange buffer
// of CAP words.  Once a sort is done the whole region may be reused.
template <int NW, int IPT> struct SortSmem {
    static constexpr int CAP = NW * WAVE * IPT;
    union {
        struct {
            RankTables<NW, 256> rt;
            uint32_t buf[CAP];
        } s;
        uint64_t k64[CAP];    // reuse after a sort: up to CAP 64-bit words
        uint32_t k32[2 * CAP];
    };
    uint32_t red32[2 * NW];
    unsigned long long red64[2 * NW];
};

template <int NW, int IPT>
__device__ inline uint32_t item_pos(int r)
{
    return wave_id() * (IPT * WAVE) + r * WAVE + lane_id();
}

template <class K, int NW>
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
    __syncthreads();
}

// Stable LSD radix sort of `count` keys (and values) held in registers at
// positions item_pos(r); positions >= count are padding and stay at the end.
// Only the bits in which the keys differ are sorted: the keys are offset by
// their minimum and ceil(bits(max-min)/8) 8-bit passes run.  rank tables must
// be zero on entry (rank_tables_init); they are zero again on return.  Ends
// with a barrier, after which the shared memory may be reused.
template <class K, bool HV, int NW, int IPT>
__device__ void block_sort(K (&k)[IPT], uint32_t (&v)[IPT], uint32_t count, SortSmem<NW, IPT> &sm)
{
    using T = KeyT<K>;
    K lo = (K)T::MAXV, hi = (K)0;
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (item_pos<NW, IPT>(r) < count) { lo = k[r] < lo ? k[r] : lo; hi = k[r] > hi ? k[r] : hi; }
    block_minmax<K, NW>(lo, hi, sm.red32, sm.red64);
    if (count <= 1 || !(lo < hi)) return;          // already in order (uniform branch)
    const int passes = (T::bitlen((K)(hi - lo)) + 7) / 8;
    uint32_t dig[IPT], pos[IPT];
    for (int ps = 0; ps < passes; ++ps) {
        const int sh = 8 * ps;
#pragma unroll
        for (int r = 0; r < IPT; ++r)
            dig[r] = item_pos<NW, IPT>(r) < count ? (uint32_t)(((K)(k[r] - lo) >> sh) & 255u) : 255u;
        rank_digits<NW, IPT, 256>(dig, pos, sm.s.rt);
        // move the keys (and values) word by word through the exchange buffer
#pragma unroll
        for (int wd = 0; wd < T::WORDS; ++wd) {
#pragma unroll
            for (int r = 0; r < IPT; ++r) sm.s.buf[pos[r]] = T::word(k[r], wd);
            __syncthreads();
#pragma unroll
            for (int r = 0; r < IPT; ++r) k[r] = T::set_word(k[r], wd, sm.s.buf[item_pos<NW, IPT>(r)]);
            __syncthreads();
        }
        if (HV) {
#pragma unroll
            for (int r = 0; r < IPT; ++r) sm.s.buf[pos[r]] = v[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < IPT; ++r) v[r] = sm.s.buf[item_pos<NW, IPT>(r)];
            __syncthreads();
        }
    }
}

}  // namespace sqs
