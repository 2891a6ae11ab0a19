// squaresort.hip -- libsquaresort: the C ABI (include/squaresort.h) and the
// host engine that drives SquareSort's recursion (Alg. 1, arXiv 2407.14801)
// on one MI355X.
//
// Recursion is breadth-wise: all internal nodes produced by one step form a
// batch that the kernels of sqs_kernels.hpp process together, so a step costs
// a fixed number of launches however many nodes it holds.  Column children
// that are internal themselves (m > cutoff) are processed as a nested batch
// before their parent's counting; bucket children that are internal form the
// next batch once the bucket sizes of the current one are known on the host
// (one small device-to-host copy per step).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/squaresort.h"
#include "sqs_kernels.hpp"

namespace sqs {
namespace {

// ------------------------------------------------------------ kernel timing
// Optional per-kernel timing: HIP events recorded on the launch stream around
// every launch, resolved at the call's synchronisation points.
struct Timing {
    bool on = false;
    std::mutex mu;
    struct Acc { double ms = 0; uint64_t launches = 0, units = 0; };
    std::map<std::string, Acc> acc;   // per kernel: time, launches, keys processed
    struct Pending { const char *name; hipEvent_t a, b; uint64_t units; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    hipEvent_t get()
    {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void resolve()
    {
        for (auto &p : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                auto &e = acc[p.name];
                e.ms += ms;
                e.launches += 1;
                e.units += p.units;
            }
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
};
Timing g_timing;

// ------------------------------------------------------------ host helpers
uint64_t ceil_isqrt_host(uint64_t n)
{
    uint64_t r = 0;
    for (int b = 31; b >= 0; --b) {
        const uint64_t c = r | (1ull << b);
        if (c * c <= n) r = c;
    }
    return r + (r * r < n ? 1 : 0);
}

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// SQS_DEBUG=1 in the environment prints one line per recursion step
bool debug_on()
{
    static const bool on = [] { const char *e = getenv("SQS_DEBUG"); return e && *e && *e != '0'; }();
    return on;
}
inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }
// shift that puts item sizes 1..cap into 256 bins (k_order_lists)
inline uint32_t shift_of(uint32_t cap)
{
    uint32_t bits = 0;
    while (bits < 32 && ((uint64_t)1 << bits) < cap) ++bits;     // 2^bits >= cap
    return bits > 8 ? bits - 8 : 0u;
}

// Work-groups per column group: the largest power of two <= cap that keeps
// groups * sub <= target (at least 1).
constexpr uint32_t COL_WG_BIG = 256;     // 16-wave column work-groups: one per CU
constexpr uint32_t COL_WG_SML = 1024;    // 4-wave column work-groups: a few per CU
inline uint32_t sub_groups(uint32_t groups, uint32_t target, uint32_t cap)
{
    uint32_t sub = 1;
    while (groups && sub * 2 <= cap && (uint64_t)groups * sub * 2 <= target) sub *= 2;
    return sub;
}

// A batch with at most this many base-case instances above one LDS sort
// splits each over the grid (k_base_*) instead of giving each one work-group.
constexpr size_t SPLIT_SEGS = 256;

// base-case class of a segment of n > 0 keys (n <= cut-off); wcap and m4cap
// are the tile choice's largest wave and mid4 buckets
inline int size_class(uint64_t n, uint32_t wcap, uint32_t m4cap)
{
    return n <= wcap ? CLS_SMALL : n <= m4cap ? CLS_MID4 : n <= (uint64_t)SORT_CAP ? CLS_MID : CLS_BIG;
}

// Tile choices (the sqs_params tile word, 0 = defaults): waves per
// work-group of the wave-level column kernel, and the largest bucket sorted
// by one wave and by one 4-wave work-group.  Every choice gives the same
// output and recursion tree.
struct Tile {
    int colw = SM_NW;
    uint32_t wcap = WCAP, m4cap = M4_CAP;
};
inline bool decode_tile(uint32_t w, Tile &t)
{
    if (w & ~(uint32_t)SQS_TILE_MASK) return false;
    const uint32_t cw = w & 3u, wc = (w >> 2) & 3u, m4 = (w >> 4) & 3u;
    if (cw > 2u || wc > 2u || m4 > 2u) return false;
    t.colw = cw == 0 ? SM_NW : cw == 1 ? 2 : 8;
    t.wcap = (uint32_t)WCAP >> wc;
    t.m4cap = M4_CAP >> m4;                 // never below wcap (1024 at most)
    return true;
}

struct HostNode {
    uint64_t off;
    uint32_t n;
    uint64_t key;
};

// Bump allocator over the caller's workspace (stack discipline).
struct Workspace {
    char *base = nullptr;
    uint64_t size = 0, top = 0;
    bool overflow = false;
    template <class T> T *take(uint64_t count)
    {
        const uint64_t at = align_up(top, 256);
        const uint64_t bytes = align_up(count * sizeof(T), 256);
        if (at + bytes > size) { overflow = true; return nullptr; }
        top = at + bytes;
        return reinterpret_cast<T *>(base + at);
    }
};

// Per-batch metadata bytes for one node of size n (as laid out in run_batch).
uint64_t node_meta_bytes(uint64_t n, uint64_t key_bytes)
{
    const uint64_t m = ceil_isqrt_host(n);
    const uint64_t groups = cdiv(m, TG), nJ = cdiv(m, TB);
    return sizeof(NodeDesc) + 7 * 4 + 8 + (m - 1 + PIV_ALIGN) * (key_bytes + 1) + 4 * m * (nJ + 1) +
           4 * groups * m + 4 * (m + 1) + 4 * m + 5 * sizeof(BucketItem) * m + 5 * (16 + 2 * key_bytes) * m +
           (3 * n / (2 * TR_CH) + 1) * (8 + 8 * TB) + 512 +
           sizeof(BucketItem) * (n / COPY_CH + 1) + 8;
}

// Upper bound of the metadata of one batch whose nodes are disjoint ranges of
// total size <= S, each node larger than the cut-off C.
uint64_t batch_bound(uint64_t S, uint64_t C, uint64_t key_bytes)
{
    if (S <= C) return 0;
    // the largest single node dominates the quadratic terms; the linear
    // terms are bounded by the count of nodes (< S / C) times a node of
    // size C+1 and by S / sqrt(C) for the m-proportional parts.
    const uint64_t big = node_meta_bytes(S, key_bytes);
    const uint64_t nodes = S / (C + 1) + 1;
    const uint64_t sq = ceil_isqrt_host(C + 1);
    const uint64_t per_m = key_bytes + 1 + 4 * 2 + 4 + 4 + 4 + 5 * sizeof(BucketItem) + 5 * (16 + 2 * key_bytes) + 8;   // generous
    return big + nodes * (sizeof(NodeDesc) + 64 + 4 * per_m) + (S / sq + nodes) * per_m * 2 +
           S / 8 + 32 * 256;
}

// the on-chip node list of a batch of total size S (nodes of more than C keys)
uint64_t small_list_bytes(uint64_t S, uint64_t C) { return align_up(sizeof(SmallNode) * (S / (C + 1) + 2), 256); }

uint64_t workspace_bound(uint64_t n, uint64_t C, uint64_t key_bytes)
{
    // n <= C needs no batch; the skew-transpose entry point still runs the
    // root step, so cover one node of n keys
    if (n <= C) {
        // a base case above one LDS sort: the grid-wide split's metadata
        const uint64_t G = cdiv(n, BS_CH);
        const uint64_t split = align_up(2 * G * key_bytes, 256) + align_up(256 * G * 4, 256) +
                               256 * (16 + 2 * key_bytes) + (8 << 10);
        return std::max(node_meta_bytes(std::max<uint64_t>(n, 2), key_bytes) + (64 << 10), split);
    }
    // nested batches: a chain of column recursions, each at most the size of n
    uint64_t chain = 1;
    for (uint64_t s = ceil_isqrt_host(n); s > C && chain < 8; s = ceil_isqrt_host(s)) ++chain;
    return chain * (batch_bound(n, C, key_bytes) + small_list_bytes(n, C)) + (1 << 20);
}

// ------------------------------------------------------------ engine
template <class K, bool HV> struct Engine {
    K *A;
    uint32_t *VA;
    K *D;
    uint32_t *VD;
    uint32_t cutoff;
    hipStream_t st;
    Workspace ws;
    bool digest;
    unsigned long long *digest_ptr;
    bool alg1 = false;     // the Alg. 1 pivot rule
    // skew-transpose mode: only the root's columns and transpose, columns
    // sorted in place in A, transpose A -> out
    bool skew_only = false;
    K *skew_out = nullptr;
    unsigned long long *skew_bs = nullptr;
    // skew mode: the columns of A come sorted (not sorted again); validate:
    // check that they are, and the output's bucket bounds
    bool cols_sorted = false;
    bool validate = false;
    Tile tile;
    // planned-graph mode: the launches are being captured into a graph that
    // is replayed later, so nothing may wait for the device: host data go up
    // synchronously at planning time (into workspace that is never reused),
    // counters that kernels change are restored by a kernel from a pristine
    // copy, failure words go to the device status word, and the internal
    // buckets of a step are finished on chip (k_internal_nodes)
    bool graph = false;
    uint32_t *status_ptr = nullptr;
    hipStream_t up = nullptr;          // planned graphs: the upload stream
    int upload(void *dst, const void *src, size_t bytes)
    {
        if (graph) {                     // on a stream of its own, outside the capture, waited for at once
            hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, up);
            if (e == hipSuccess) e = hipStreamSynchronize(up);
            if (e != hipSuccess && debug_on()) fprintf(stderr, "[sqs] plan upload: %s\n", hipGetErrorString(e));
            return e == hipSuccess ? SQS_OK : SQS_ERR_DEVICE;
        }
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess ? SQS_OK : SQS_ERR_DEVICE;
    }
    void release(uint64_t mark)
    {
        if (!graph) ws.top = mark;   // a graph replays every phase: nothing is reused
    }

    int check() const
    {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess && debug_on()) fprintf(stderr, "[sqs] launch: %s\n", hipGetErrorString(e));
        return e == hipSuccess ? SQS_OK : SQS_ERR_DEVICE;
    }

    // launch f() on st, bracketed by timing events when timing is enabled
    int cur_depth = 0;
    template <class F> void launch(const char *name0, uint64_t units, F f)
    {
        if (!g_timing.on || graph) { f(); return; }
        // kernels of deeper recursion steps are reported as name@d
        static thread_local std::string tmp;
        tmp = name0;
        if (cur_depth > 0) tmp += "@" + std::to_string(cur_depth);
        const char *name = intern(tmp);
        std::lock_guard<std::mutex> lk(g_timing.mu);
        hipEvent_t a = g_timing.get(), b = g_timing.get();
        if (a) hipEventRecord(a, st);
        f();
        if (b) hipEventRecord(b, st);
        if (a && b) g_timing.pending.push_back({name, a, b, units});
    }
    void resolve_timing()
    {
        if (!g_timing.on) return;
        std::lock_guard<std::mutex> lk(g_timing.mu);
        g_timing.resolve();
    }
    // corrects the units of this step's pending launch of a kernel
    void set_units(const char *name0, uint64_t units)
    {
        if (!g_timing.on) return;
        std::string nm = name0;
        if (cur_depth > 0) nm += "@" + std::to_string(cur_depth);
        std::lock_guard<std::mutex> lk(g_timing.mu);
        for (auto it = g_timing.pending.rbegin(); it != g_timing.pending.rend(); ++it)
            if (nm == it->name) { it->units = units; return; }
    }

    static const char *intern(const std::string &s)
    {
        static std::mutex mu;
        static std::vector<std::string *> names;
        std::lock_guard<std::mutex> lk(mu);
        for (auto *p : names) if (*p == s) return p->c_str();
        names.push_back(new std::string(s));
        return names.back()->c_str();
    }

    // Nodes that one work-group sorts with their whole subtree on chip (32-bit
    // keys without values, the default pivot rule, at most SN_CAP keys and
    // columns that are base cases): one launch of k_small_nodes; the others
    // are returned in rest.  The node list is taken from the workspace above
    // ws.top (the caller's frame releases it).
    int run_small(const std::vector<HostNode> &in, std::vector<HostNode> &rest)
    {
        rest.clear();
        if (!(sizeof(K) == 4 && !HV) || alg1 || skew_only) { rest = in; return SQS_OK; }
        std::vector<SmallNode> sn;
        uint64_t keys = 0;
        for (const HostNode &h : in) {
            if (h.n <= SN_CAP && ceil_isqrt_host(h.n) <= cutoff) {
                sn.push_back(SmallNode{h.off, h.n, 0u, h.key});
                keys += h.n;
            } else {
                rest.push_back(h);
            }
        }
        if (sn.empty()) return SQS_OK;
        SmallNode *dsn = ws.take<SmallNode>(sn.size());
        if (ws.overflow) return SQS_ERR_WORKSPACE;
        keep_.emplace_back(sn.size() * sizeof(SmallNode));
        memcpy(keep_.back().data(), sn.data(), sn.size() * sizeof(SmallNode));
        if (int rc = upload(dsn, keep_.back().data(), sn.size() * sizeof(SmallNode))) return rc;
        const uint32_t cnt = (uint32_t)sn.size();
        launch("k_small_nodes", keys, [&] {
            k_small_nodes<<<std::min<uint32_t>(cnt, 2048), SN_NT, 0, st>>>(
                dsn, cnt, reinterpret_cast<uint32_t *>(A), reinterpret_cast<uint32_t *>(D), cutoff,
                digest ? digest_ptr : nullptr); });
        return check();
    }

    int run_batch(const std::vector<HostNode> &nodes_in, int depth)
    {
        if (depth >= SQS_MAX_DEPTH) return SQS_ERR_DEPTH;
        cur_depth = depth;
        const uint64_t mark = ws.top;
        std::vector<HostNode> nodes;
        if (int rc = run_small(nodes_in, nodes)) return rc;
        if (nodes.empty()) {
            release(mark);                  // stream-ordered: later work may reuse the list's memory
            return SQS_OK;
        }
        const uint32_t N = (uint32_t)nodes.size();

        // ---- plan the batch on the host
        std::vector<NodeDesc> desc(N);
        // prefixes: piv, tile, buc, dig (N+1 each), then big/small index lists and group prefixes
        std::vector<uint32_t> bigIdx, smlIdx, bigGrp{0}, smlGrp{0};
        uint32_t bigM = 0;                             // largest m of the work-group-column nodes
        std::vector<uint32_t> pfx(4 * (N + 1), 0);
        uint32_t *pivS = &pfx[0], *tileS = &pfx[(N + 1)], *bucS = &pfx[2 * (N + 1)], *digS = &pfx[3 * (N + 1)];
        uint64_t srcTot = 0, blkTot = 0, keysTot = 0;
        uint32_t bktTot = 0;
        std::vector<HostNode> col_kids;
        // nodes with m > SORT_CAP: their pivots and base-case columns are sorted
        // as segments (one-bucket nodes) before the count
        std::vector<uint32_t> hugeIdx, hugeCol{0};
        std::vector<NodeDesc> pivSeg, colSeg;
        std::vector<BucketItem> pivLists[NCLS], colLists[NCLS];
        for (uint32_t k = 0; k < N; ++k) {
            const HostNode &h = nodes[k];
            NodeDesc &d = desc[k];
            d.off = h.off;
            d.key = h.key;
            d.n = h.n;
            d.m = (uint32_t)ceil_isqrt_host(h.n);
            d.groups = cdiv(d.m, TG);
            d.nJ = cdiv(d.m, TB);
            d.piv = pivS[k];
            d.bkt = bktTot;
            d.src = srcTot;
            d.blk = blkTot;
            d.flags = 0;
            d.sub = 1;
            const bool huge = d.m > (uint32_t)SORT_CAP;
            if (huge) {
                // columns do not fit one LDS sort: sorted into D first (the
                // Alg. 1 rule and the skew entry point keep the LDS-sized limit)
                if (skew_only || alg1) return SQS_ERR_UNSUPPORTED;
                d.flags |= NODE_HUGE | NODE_COLS_RECURSED;
                hugeIdx.push_back(k);
                hugeCol.push_back(hugeCol.back() + d.m);
                NodeDesc pn{};
                pn.off = d.piv;
                pn.n = d.m - 1;
                pn.m = 1;
                pivLists[CLS_BIG].push_back(BucketItem{(uint32_t)pivSeg.size(), 0u, 0u, d.m - 1});
                pivSeg.push_back(pn);
                NodeDesc cn{};
                cn.off = d.off;
                cn.n = d.n;
                cn.m = 1;
                const uint32_t cnode = (uint32_t)colSeg.size();
                colSeg.push_back(cn);
                for (uint32_t i = 0; i < d.m; ++i) {
                    const uint64_t lo = (uint64_t)i * d.m;
                    if (lo >= h.n) break;
                    const uint32_t len = (uint32_t)std::min<uint64_t>(d.m, h.n - lo);
                    if (len > cutoff) { col_kids.push_back({h.off + lo, len, node_child_key(h.key, 0, i)}); continue; }
                    const int cls = size_class(len, tile.wcap, tile.m4cap);
                    colLists[cls].push_back(BucketItem{cnode, 0u, (uint32_t)lo, len});
                }
            } else if (skew_only && cols_sorted) {
                d.flags |= NODE_COLS_RECURSED;             // taken as sorted (cut-off 0 below)
            } else if (!skew_only && d.m > cutoff) {
                d.flags |= NODE_COLS_RECURSED;
                for (uint32_t i = 0; i < d.m; ++i) {
                    const uint64_t lo = (uint64_t)i * d.m;
                    if (lo >= h.n) break;
                    const uint32_t len = (uint32_t)std::min<uint64_t>(d.m, h.n - lo);
                    // a short tail column may be a base case (sorted by the column kernel)
                    if (len > cutoff) col_kids.push_back({h.off + lo, len, node_child_key(h.key, 0, i)});
                }
            }
            if (huge) {
            } else if (d.m > (uint32_t)WCAP) {
                bigIdx.push_back(k);
                bigGrp.push_back(bigGrp.back() + d.groups);
                bigM = std::max(bigM, d.m);
            }
            else { smlIdx.push_back(k); smlGrp.push_back(smlGrp.back() + d.groups); }
            pivS[k + 1] = pivS[k] + (uint32_t)align_up(d.m - 1, PIV_ALIGN);   // 16-key aligned slots
            tileS[k + 1] = tileS[k] + d.groups * d.nJ;
            bucS[k + 1] = bucS[k] + d.m;
            digS[k + 1] = digS[k] + cdiv(h.n, 16384);
            bktTot += d.m + 1;
            keysTot += h.n;
            srcTot += (uint64_t)(d.nJ + 1) * d.m;
            blkTot += (uint64_t)d.groups * d.m;
        }
        const uint32_t NB = (uint32_t)bigIdx.size(), NS = (uint32_t)smlIdx.size();
        // Few column groups (a mid-size root): split each group over several
        // work-groups so that the column kernels fill the chip; they then add
        // their bucket counts into the group's (cleared below).
        const uint32_t subBig = sub_groups(bigGrp.back(), COL_WG_BIG, TG);
        const uint32_t subSml = sub_groups(smlGrp.back(), COL_WG_SML * SM_NW / tile.colw, TG / tile.colw);
        if (subBig > 1)
            for (uint32_t q = 0; q < NB; ++q) {
                desc[bigIdx[q]].sub = subBig;
                bigGrp[q + 1] = bigGrp[q] + desc[bigIdx[q]].groups * subBig;
            }
        if (subSml > 1)
            for (uint32_t q = 0; q < NS; ++q) {
                desc[smlIdx[q]].sub = subSml;
                smlGrp[q + 1] = smlGrp[q] + desc[smlIdx[q]].groups * subSml;
            }
        std::vector<uint32_t> idx;
        idx.reserve(pfx.size() + 2 * N + 2);
        idx.insert(idx.end(), pfx.begin(), pfx.end());
        const size_t oBigIdx = idx.size(); idx.insert(idx.end(), bigIdx.begin(), bigIdx.end());
        const size_t oBigGrp = idx.size(); idx.insert(idx.end(), bigGrp.begin(), bigGrp.end());
        const size_t oSmlIdx = idx.size(); idx.insert(idx.end(), smlIdx.begin(), smlIdx.end());
        const size_t oSmlGrp = idx.size(); idx.insert(idx.end(), smlGrp.begin(), smlGrp.end());
        const uint32_t NH = (uint32_t)hugeIdx.size();
        const size_t oHugeIdx = idx.size(); idx.insert(idx.end(), hugeIdx.begin(), hugeIdx.end());
        const size_t oHugeCol = idx.size(); idx.insert(idx.end(), hugeCol.begin(), hugeCol.end());

        // work-list capacities: every bucket may be small or single-valued;
        // mid buckets hold > WCAP keys and internal ones > cutoff keys
        const uint32_t capSmall = bucS[N];
        const uint32_t capCopy = (uint32_t)std::min<uint64_t>(0xFFFFFFFFull, bucS[N] + keysTot / COPY_CH + 1);
        const uint32_t capMid4 = (uint32_t)std::min<uint64_t>(bucS[N], keysTot / (tile.wcap + 1) + 1);
        const uint32_t capMid = (uint32_t)std::min<uint64_t>(bucS[N], keysTot / (tile.m4cap + 1) + 1);
        const uint32_t capBig = (uint32_t)std::min<uint64_t>(bucS[N], keysTot / (SORT_CAP + 1) + 1);
        const uint32_t capInt = (uint32_t)std::min<uint64_t>(bucS[N], keysTot / ((uint64_t)cutoff + 1) + 1);

        // ---- device metadata
        Batch<K> b;
        b.wcap = tile.wcap;
        b.m4cap = tile.m4cap;
        NodeDesc *dDesc = ws.take<NodeDesc>(N);
        uint32_t *dIdx = ws.take<uint32_t>(idx.size());
        b.piv = ws.take<K>(std::max<uint32_t>(pivS[N], 1));
        b.strict = ws.take<uint8_t>(std::max<uint32_t>(pivS[N], 1));
        b.srcOff = ws.take<uint32_t>(srcTot);
        b.blk = ws.take<uint32_t>(blkTot);
        b.bs = ws.take<uint32_t>(bktTot);
        b.tot = ws.take<uint32_t>(bktTot);
        b.list[CLS_COPY] = ws.take<BucketItem>(capCopy);
        b.list[CLS_SMALL] = ws.take<BucketItem>(capSmall);
        b.list[CLS_MID4] = ws.take<BucketItem>(capMid4);
        b.list[CLS_MID] = ws.take<BucketItem>(capMid);
        b.list[CLS_BIG] = ws.take<BucketItem>(capBig);
        b.list[CLS_INTERNAL] = ws.take<BucketItem>(capInt);
        b.cap[CLS_COPY] = capCopy; b.cap[CLS_SMALL] = capSmall; b.cap[CLS_MID4] = capMid4; b.cap[CLS_MID] = capMid;
        b.cap[CLS_BIG] = capBig; b.cap[CLS_INTERNAL] = capInt;
        for (int c = 0; c < NCLS; ++c) { b.span[c] = nullptr; b.ord[c] = nullptr; }
        b.bigInD = 0;
        b.span[CLS_MID4] = ws.take<Span<K>>(capMid4);
        b.span[CLS_MID] = ws.take<Span<K>>(capMid);
        b.ord[CLS_MID] = ws.take<Span<K>>(capMid);
        if (cutoff > (uint32_t)SORT_CAP) {
            b.span[CLS_BIG] = ws.take<Span<K>>(capBig);
            b.ord[CLS_BIG] = ws.take<Span<K>>(capBig);
        }
        b.ctr = ws.take<uint32_t>(CTR_WORDS);
        // heavy-tile transpose chunks: a tile above TR_HEAVY (three chunks) has
        // fewer than 1.5 * keys / TR_CH chunks, so the sum over tiles is below that
        b.trCap = (uint32_t)std::min<uint64_t>(0xFFFFFFFFull, 3 * keysTot / (2 * TR_CH) + 1);
        b.trItem = ws.take<uint32_t>(2 * (uint64_t)b.trCap);
        b.trRec = ws.take<unsigned long long>((uint64_t)b.trCap * TB);
        b.nmin = ws.take<K>(N);
        b.alg1 = alg1 ? 1u : 0u;
        b.H = ws.take<unsigned long long>(N);
        K *pivScratch = NH ? ws.take<K>(std::max<uint32_t>(pivS[N], 1)) : nullptr;
        if (ws.overflow) return SQS_ERR_WORKSPACE;
        b.nodes = dDesc;
        b.N = N;
        b.pivStart = dIdx;
        b.tileStart = dIdx + (N + 1);
        b.bucStart = dIdx + 2 * (N + 1);
        b.digStart = dIdx + 3 * (N + 1);
        b.bigIdx = dIdx + oBigIdx; b.bigGrp = dIdx + oBigGrp; b.NB = NB;
        b.smlIdx = dIdx + oSmlIdx; b.smlGrp = dIdx + oSmlGrp; b.NS = NS;
        if (int rc = upload(dDesc, desc.data(), N * sizeof(NodeDesc))) return rc;
        if (int rc = upload(dIdx, idx.data(), idx.size() * 4)) return rc;

        // ---- pivots (drawn from the node inputs before any child clobbers them)
        // counters (list sizes, take counters, key totals, the pivot-rule flag)
        k_fill_u32<<<1, 64, 0, st>>>(b.ctr, CTR_WORDS, 0u);
        if ((subBig > 1 || subSml > 1) && blkTot) k_fill_u32<<<cdiv(blkTot, 256), 256, 0, st>>>(b.blk, blkTot, 0u);
        if (alg1) {                                   // node minima for the Alg. 1 pivot rule
            if (sizeof(K) == 4) k_fill_u32<<<cdiv(N, 256), 256, 0, st>>>(reinterpret_cast<uint32_t *>(b.nmin), N, 0xFFFFFFFFu);
            else k_fill_u64<<<cdiv(N, 256), 256, 0, st>>>(reinterpret_cast<unsigned long long *>(b.nmin), N, ~0ull);
            launch("k_node_min", keysTot, [&] { k_node_min<K><<<digS[N], 256, 0, st>>>(b, A); });
        }
        if (pivS[N] > 0) launch("k_sample", pivS[N], [&] { k_sample<K><<<cdiv(pivS[N], 256), 256, 0, st>>>(b, A); });
        if (NB) launch("k_sort_pivots", pivS[N], [&] { k_sort_pivots_big<K><<<NB, SORT_NT, 0, st>>>(b, A); });
        if (NS) launch("k_sort_pivots_w", pivS[N], [&] { k_sort_pivots_small<K><<<cdiv(NS, SM_NW), SM_NW * WAVE, 0, st>>>(b, A); });
        if (int rc = check()) return rc;
        const uint32_t *dHugeIdx = dIdx + oHugeIdx, *dHugeCol = dIdx + oHugeCol;
        if (NH) {                                     // pivots of m > SORT_CAP nodes: MSD-split sorts, then flags
            if (int rc = sort_segments<false>(b.piv, nullptr, pivScratch, nullptr, pivSeg, pivLists)) return rc;
            for (uint32_t q = 0; q < NH; ++q) {
                const NodeDesc &d = desc[hugeIdx[q]];
                if (hipMemcpyAsync(b.piv + d.piv, pivScratch + d.piv, (uint64_t)(d.m - 1) * sizeof(K),
                                   hipMemcpyDeviceToDevice, st) != hipSuccess)
                    return SQS_ERR_DEVICE;
            }
            k_strict_flags<K><<<NH, 256, 0, st>>>(b, dHugeIdx);
            if (int rc = check()) return rc;
        }

        // ---- columns: internal column children first, then sort/count
        if (!col_kids.empty()) {
            if (int rc = run_batch(col_kids, depth + 1)) return rc;
            cur_depth = depth;
        }
        K *cdst = skew_only ? A : D;
        uint32_t *vcdst = skew_only ? VA : VD;
        // columns given sorted: every column counts as sorted by recursion
        const uint32_t colCut = skew_only && cols_sorted ? 0u : cutoff;
        if (skew_only && cols_sorted && validate)
            k_check_sorted<K><<<std::min<uint32_t>(cdiv(desc[0].n, 256), 4096), 256, 0, st>>>(
                A, desc[0].n, desc[0].m, b.ctr + CTR_PRE_FAIL);
        if (NH) {                                     // m > SORT_CAP: base-case columns A -> D, then the HBM count
            if (int rc = sort_segments<HV>(A, VA, D, VD, colSeg, colLists)) return rc;
            launch("k_blockoff", keysTot, [&] {
                k_blockoff<K><<<hugeCol.back(), 256, 0, st>>>(b, D, dHugeIdx, dHugeCol, NH); });
            launch("k_tilecount", keysTot, [&] { k_tilecount<K><<<tileS[N], TR_NW * WAVE, 0, st>>>(b, D); });
            if (int rc = check()) return rc;
        }
        if (NB) launch("k_colsort", keysTot, [&] {
            if constexpr (sizeof(K) == 8) {
                if (bigM <= (uint32_t)MergeCap<HV>::CAP) {   // every column fits the merge sort
                    k_colsort_big<K, HV, true><<<bigGrp.back(), SORT_NT, 0, st>>>(b, A, VA, cdst, vcdst, colCut);
                    return;
                }
            }
            k_colsort_big<K, HV><<<bigGrp.back(), SORT_NT, 0, st>>>(b, A, VA, cdst, vcdst, colCut); });
        if (NS) launch("k_colsort_w", keysTot, [&] {
            if (tile.colw == 2)
                k_colsort_small<K, HV, 2><<<smlGrp.back(), 2 * WAVE, 0, st>>>(b, A, VA, cdst, vcdst, colCut);
            else if (tile.colw == 8)
                k_colsort_small<K, HV, 8><<<smlGrp.back(), 8 * WAVE, 0, st>>>(b, A, VA, cdst, vcdst, colCut);
            else
                k_colsort_small<K, HV, SM_NW><<<smlGrp.back(), SM_NW * WAVE, 0, st>>>(b, A, VA, cdst, vcdst, colCut); });
        launch("k_colscan", bucS[N], [&] { k_colscan<K><<<cdiv(bucS[N], 256), 256, 0, st>>>(b); });
        launch("k_bucket_start", bucS[N], [&] { k_bucket_start<K><<<N, 1024, 0, st>>>(b, skew_only ? skew_bs : nullptr); });
        if (int rc = check()) return rc;

        // ---- SkewTranspose D -> A (skew mode: A -> out)
        if (skew_only) {
            launch("k_transpose", keysTot, [&] {
                k_tile_plan<K><<<cdiv(tileS[N], TR_NW), TR_NW * WAVE, 0, st>>>(b, tileS[N]);
                k_transpose<K, HV><<<tileS[N], TR_NW * WAVE, 0, st>>>(b, A, VA, skew_out, nullptr);
                k_transpose_heavy<K, HV><<<TR_EXTRA, TR_NW * WAVE, 0, st>>>(b, A, VA, skew_out, nullptr, tileS[N]); });
            if (validate)
                k_check_buckets<K><<<std::min<uint32_t>(cdiv(keysTot, 256), 4096), 256, 0, st>>>(b, skew_out);
            ws.top = mark;
            if (int rc = check()) return rc;
            // the host-side plan must outlive its upload
            uint32_t hc[CTR_WORDS];
            if (hipMemcpyAsync(hc, b.ctr, sizeof hc, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return SQS_ERR_DEVICE;
            resolve_timing();
            if (hc[CTR_PRE_FAIL]) return SQS_ERR_PRECOND;       // a column given as sorted is not
            if (alg1 && hc[CTR_FAIL]) return SQS_ERR_PRECOND;   // no valid Alg. 1 sample
            return hc[CTR_TR_FAIL] || hc[CTR_CHECK_FAIL] ? SQS_ERR_DEVICE : SQS_OK;
        }
        launch("k_transpose", keysTot, [&] {
            k_tile_plan<K><<<cdiv(tileS[N], TR_NW), TR_NW * WAVE, 0, st>>>(b, tileS[N]);
            k_transpose<K, HV><<<tileS[N], TR_NW * WAVE, 0, st>>>(b, D, VD, A, VA);
            k_transpose_heavy<K, HV><<<TR_EXTRA, TR_NW * WAVE, 0, st>>>(b, D, VD, A, VA, tileS[N]); });
        if (digest) {
            k_fill_u64<<<cdiv(N, 256), 256, 0, st>>>(b.H, N, 0ull);
            k_digest<K, HV><<<digS[N], 256, 0, st>>>(b, A, VA);
            k_digest_finish<K><<<cdiv(N, 256), 256, 0, st>>>(b, digest_ptr);
        }
        if (int rc = check()) return rc;

        // ---- buckets A -> D, by class
        launch("k_classify", bucS[N], [&] { k_classify<K><<<cdiv(bucS[N], CL_NT), CL_NT, 0, st>>>(b, cutoff); });
        launch("k_order_lists", bucS[N], [&] {
            k_order_lists<K><<<2, 1024, 0, st>>>(b, shift_of(SORT_CAP), shift_of(cutoff)); });
        launch("k_bucket_copy", keysTot, [&] { k_bucket_copy<K, HV><<<512, CP_NT, 0, st>>>(b, A, VA, D, VD); });
        launch("k_bucket_w", keysTot, [&] {
            k_bucket_small<K, HV><<<std::min<uint32_t>(cdiv(capSmall, SM_NW), 2048), SM_NW * WAVE, 0, st>>>(b, A, VA, D, VD); });
        launch("k_bucket4", keysTot, [&] {
            k_bucket_mid<K, HV, M4_NW, CLS_MID4><<<std::min<uint32_t>(capMid4, 2048), M4_NW * WAVE, 0, st>>>(b, A, VA, D, VD); });
        launch("k_bucket", keysTot, [&] {
            k_bucket_mid<K, HV, SORT_NW, CLS_MID><<<std::min<uint32_t>(capMid, 512), SORT_NT, 0, st>>>(b, A, VA, D, VD); });
        if constexpr (sizeof(K) == 4 && !HV) {
            if (cutoff > (uint32_t)SORT_CAP)             // the MSD-split list's smallest buckets, whole in LDS
                launch("k_bucket_wide", keysTot, [&] {
                    k_bucket_wide<<<std::min<uint32_t>(capBig, COL_WG_BIG), SORT_NT, 0, st>>>(
                        b, reinterpret_cast<const uint32_t *>(A), reinterpret_cast<uint32_t *>(D)); });
        }
        if (cutoff > (uint32_t)SORT_CAP)
            launch("k_bucket_big", keysTot, [&] {
                k_bucket_big<K, HV><<<std::min<uint32_t>(capBig, 512), BK_NT, 0, st>>>(b, A, VA, D, VD); });
        if (int rc = check()) return rc;

        // ---- internal buckets form the next batch
        if (graph) {                                     // finished on chip, or reported
            if constexpr (sizeof(K) == 4 && !HV) {
                launch("k_internal_nodes", keysTot, [&] {
                    k_internal_nodes<<<std::min<uint32_t>(std::max<uint32_t>(capInt, 1), 2048), SN_NT, 0, st>>>(
                        b, reinterpret_cast<uint32_t *>(A), reinterpret_cast<uint32_t *>(D), cutoff,
                        digest ? digest_ptr : nullptr, status_ptr); });
            }
            k_status<K><<<1, 64, 0, st>>>(b, status_ptr, 1);
            return check();
        }
        std::vector<uint32_t> hctr(CTR_WORDS);
        std::vector<BucketItem> hint(capInt);
        if (hipMemcpyAsync(hctr.data(), b.ctr, CTR_WORDS * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(hint.data(), b.list[CLS_INTERNAL], capInt * sizeof(BucketItem), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SQS_ERR_DEVICE;
        keep_.clear();                                   // the stream has run every upload
        // the bucket kernels processed the keys of their own class only
        set_units("k_bucket_copy", hctr[2 * NCLS + CLS_COPY]);
        set_units("k_bucket_w", hctr[2 * NCLS + CLS_SMALL]);
        set_units("k_bucket4", hctr[2 * NCLS + CLS_MID4]);
        set_units("k_bucket", hctr[2 * NCLS + CLS_MID]);
        set_units("k_bucket_wide", hctr[CTR_WIDE_KEYS]);
        set_units("k_bucket_big", hctr[2 * NCLS + CLS_BIG] - hctr[CTR_WIDE_KEYS]);
        resolve_timing();
        if (alg1 && hctr[CTR_FAIL]) return SQS_ERR_PRECOND;  // no valid Alg. 1 sample for some node
        if (hctr[CTR_TR_FAIL]) return SQS_ERR_DEVICE;          // a transpose chunk's wait ran out
        if (hctr[CTR_BIG_FAIL]) return SQS_ERR_DEVICE;         // an MSD-split stack overflow
        for (int c = 0; c < NCLS; ++c)
            if (hctr[c] > b.cap[c]) return SQS_ERR_DEVICE;   // cannot happen: capacities are bounds
        if (debug_on()) {
            fprintf(stderr, "[sqs] depth %d: %u nodes, %llu keys; buckets copy %u small %u mid %u big %u internal %u\n",
                    depth, N, (unsigned long long)keysTot, hctr[0], hctr[1], hctr[2], hctr[3], hctr[4]);
            if (bktTot <= 64) {
                std::vector<uint32_t> hb(bktTot), ht(bktTot), hblk(blkTot), hsrc(srcTot);
                hipMemcpy(hb.data(), b.bs, bktTot * 4, hipMemcpyDeviceToHost);
                hipMemcpy(ht.data(), b.tot, bktTot * 4, hipMemcpyDeviceToHost);
                hipMemcpy(hblk.data(), b.blk, blkTot * 4, hipMemcpyDeviceToHost);
                hipMemcpy(hsrc.data(), b.srcOff, srcTot * 4, hipMemcpyDeviceToHost);
                fprintf(stderr, "  bs:"); for (auto x : hb) fprintf(stderr, " %u", x);
                fprintf(stderr, "\n  tot:"); for (auto x : ht) fprintf(stderr, " %u", x);
                fprintf(stderr, "\n  blk:"); for (auto x : hblk) fprintf(stderr, " %u", x);
                fprintf(stderr, "\n  src:"); for (auto x : hsrc) fprintf(stderr, " %u", x);
                fprintf(stderr, "\n");
            }
        }
        hint.resize(hctr[CLS_INTERNAL]);
        std::sort(hint.begin(), hint.end(), [](const BucketItem &x, const BucketItem &y) {
            return x.node != y.node ? x.node < y.node : x.j < y.j;
        });
        std::vector<HostNode> next;
        next.reserve(hint.size());
        for (const BucketItem &e : hint)
            next.push_back({desc[e.node].off + e.lo, e.size, node_child_key(desc[e.node].key, 1, e.j)});
        release(mark);
        if (!next.empty()) return run_batch(next, depth + 1);
        return SQS_OK;
    }

    // Base-case segments larger than one LDS sort, on the whole grid: one MSD
    // split of each (A -> D), then the parts as items of the large-bucket
    // kernel, which reads them from D.  nseg == 1 with segOff null is a whole
    // array at 0 of n keys (nothing uploaded, so the call does not wait for
    // the stream); otherwise segOff / segN / segChunk are device arrays.
    int split_segments(uint32_t nseg, uint32_t G, uint64_t n1, const uint64_t *segOff, const uint32_t *segN,
                       const uint32_t *segChunk, uint64_t keys)
    {
        const uint64_t mark = ws.top;
        BaseSplit<K> s;
        s.nseg = nseg;
        s.n = (uint32_t)n1;
        s.G = G;
        s.segOff = segOff; s.segN = segN; s.segChunk = segChunk;
        s.mm = ws.take<K>(2 * (uint64_t)G);
        s.cnt = ws.take<uint32_t>(256 * (uint64_t)G);
        s.items = ws.take<Span<K>>(256 * (uint64_t)nseg);
        s.ctr = ws.take<uint32_t>(CTR_WORDS);
        release(mark);                     // stream-ordered: later work on this stream may reuse it
        if (ws.overflow) return SQS_ERR_WORKSPACE;
        Batch<K> b{};
        b.wcap = tile.wcap;
        b.m4cap = tile.m4cap;
        b.span[CLS_BIG] = s.items; b.cap[CLS_BIG] = 256 * nseg;
        b.ctr = s.ctr;
        b.bigInD = 1;
        launch("k_base_split", keys, [&] {
            k_base_range<K><<<G, BS_NT, 0, st>>>(A, s);
            k_base_count<K><<<G, BS_NT, 0, st>>>(A, s);
            k_base_scan<K><<<nseg, 1024, 0, st>>>(s);
            k_base_scatter<K, HV><<<G, BS_NT, 0, st>>>(A, VA, D, VD, s); });
        launch("k_bucket_big", keys, [&] {
            k_bucket_big<K, HV><<<std::min<uint32_t>(256 * nseg, 512), BK_NT, 0, st>>>(b, A, VA, D, VD); });
        if (int rc = check()) return rc;
        return read_fail(s.ctr);
    }
    // Reads a batch's failure words back (synchronising the stream): the
    // MSD-split kernel's stack overflow flag.
    int read_fail(const uint32_t *ctr)
    {
        if (graph) {                                     // reported through the status word
            Batch<K> sb{};
            sb.ctr = const_cast<uint32_t *>(ctr);
            k_status<K><<<1, 64, 0, st>>>(sb, status_ptr, 0);
            return check();
        }
        uint32_t f = 0;
        if (hipMemcpyAsync(&f, ctr + CTR_BIG_FAIL, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SQS_ERR_DEVICE;
        return f ? SQS_ERR_DEVICE : SQS_OK;
    }
    int sort_big_base(uint64_t n)
    {
        if (cdiv(n, BS_CH) > BS_MAXG) return SQS_ERR_ARG;   // cannot happen: n <= cutoff <= BIG_CAP
        if (int rc = split_segments(1, cdiv(n, BS_CH), n, nullptr, nullptr, nullptr, n)) return rc;
        if (g_timing.on && hipStreamSynchronize(st) == hipSuccess) resolve_timing();
        return SQS_OK;
    }

    int sort_root(uint64_t n, uint64_t seed)
    {
        if (n == 0) return SQS_OK;
        if (n > (uint64_t)SORT_CAP && n <= cutoff) return sort_big_base(n);
        if (n <= cutoff) {
            launch("k_base_sort", n, [&] { k_base_sort<K, HV><<<1, SORT_NT, 0, st>>>((uint32_t)n, A, VA, D, VD); });
            if (g_timing.on && hipStreamSynchronize(st) == hipSuccess) resolve_timing();
            return check();
        }
        std::vector<HostNode> root{{0, (uint32_t)n, splitmix(seed)}};
        return finish(run_batch(root, 0));
    }
    // a call whose last step left host copies that async uploads read (the
    // on-chip node list) waits for them before the copies are freed
    int finish(int rc)
    {
        if (!keep_.empty() && !graph) {
            if (hipStreamSynchronize(st) != hipSuccess && rc == SQS_OK) rc = SQS_ERR_DEVICE;
            keep_.clear();
        }
        return rc;
    }

    // Sorts independent segments src -> dst with the base-case kernels.  pn
    // are one-bucket nodes (m = 1, so a segment's key range is the whole
    // type) giving each segment's base; lists hold the segments by class
    // (small, mid, big).  Takes workspace; the caller keeps pn and lists
    // alive until the stream has run the uploads.
    template <bool HV2>
    int sort_segments(K *sA, uint32_t *sVA, K *sD, uint32_t *sVD, const std::vector<NodeDesc> &pn,
                      std::vector<BucketItem> (&lists)[NCLS])
    {
        Batch<K> b{};
        b.wcap = tile.wcap;
        b.m4cap = tile.m4cap;
        for (int c = CLS_MID4; c <= CLS_BIG; ++c)     // largest first, as k_order_lists orders device lists
            std::stable_sort(lists[c].begin(), lists[c].end(),
                             [](const BucketItem &x, const BucketItem &y) { return x.size > y.size; });
        NodeDesc *dDesc = ws.take<NodeDesc>(pn.size());
        for (int c = CLS_SMALL; c <= CLS_BIG; ++c) {
            b.list[c] = ws.take<BucketItem>(std::max<size_t>(lists[c].size(), 1));
            b.cap[c] = (uint32_t)lists[c].size();
        }
        uint32_t *ctr = ws.take<uint32_t>(CTR_WORDS);
        if (ws.overflow) return SQS_ERR_WORKSPACE;
        keep_.emplace_back(CTR_WORDS * 4, 0);
        uint32_t *hctr = reinterpret_cast<uint32_t *>(keep_.back().data());
        for (int c = CLS_SMALL; c <= CLS_BIG; ++c) hctr[c] = (uint32_t)lists[c].size();
        if (int rc = upload(dDesc, pn.data(), pn.size() * sizeof(NodeDesc))) return rc;
        if (graph) {                                     // the take counters change: restored every replay
            uint32_t *pctr = ws.take<uint32_t>(CTR_WORDS);
            if (ws.overflow) return SQS_ERR_WORKSPACE;
            if (int rc = upload(pctr, hctr, CTR_WORDS * 4)) return rc;
            k_copy_u32<<<1, 64, 0, st>>>(ctr, pctr, CTR_WORDS);
        } else if (int rc = upload(ctr, hctr, CTR_WORDS * 4)) {
            return rc;
        }
        for (int c = CLS_SMALL; c <= CLS_BIG; ++c)
            if (!lists[c].empty())
                if (int rc = upload(b.list[c], lists[c].data(), lists[c].size() * sizeof(BucketItem))) return rc;
        // the sorted classes read resolved spans (one-bucket nodes: the whole key range)
        for (int c = CLS_MID4; c <= CLS_BIG; ++c) {
            if (lists[c].empty()) continue;
            const size_t bytes = lists[c].size() * sizeof(Span<K>);
            keep_.emplace_back(bytes, 0);
            Span<K> *hs = reinterpret_cast<Span<K> *>(keep_.back().data());
            for (size_t q = 0; q < lists[c].size(); ++q) {
                const BucketItem &e = lists[c][q];
                hs[q] = Span<K>{pn[e.node].off + e.lo, e.size, 0u, (K)0, (K)KeyT<K>::MAXV};
            }
            b.span[c] = ws.take<Span<K>>(lists[c].size());
            if (ws.overflow) return SQS_ERR_WORKSPACE;
            if (int rc = upload(b.span[c], hs, bytes)) return rc;
        }
        b.nodes = dDesc;
        b.N = (uint32_t)pn.size();
        b.ctr = ctr;
        uint64_t keys[NCLS] = {};
        for (int c = CLS_SMALL; c <= CLS_BIG; ++c)
            for (const BucketItem &e : lists[c]) keys[c] += e.size;
        if (!lists[CLS_SMALL].empty())
            launch("k_bucket_w", keys[CLS_SMALL], [&] {
                k_bucket_small<K, HV2><<<std::min<uint32_t>(cdiv(b.cap[CLS_SMALL], SM_NW), 2048), SM_NW * WAVE, 0, st>>>(
                    b, sA, sVA, sD, sVD); });
        if (!lists[CLS_MID4].empty())
            launch("k_bucket4", keys[CLS_MID4], [&] {
                k_bucket_mid<K, HV2, M4_NW, CLS_MID4><<<std::min<uint32_t>(b.cap[CLS_MID4], 2048), M4_NW * WAVE, 0, st>>>(
                    b, sA, sVA, sD, sVD); });
        if (!lists[CLS_MID].empty())
            launch("k_bucket", keys[CLS_MID], [&] {
                k_bucket_mid<K, HV2, SORT_NW, CLS_MID><<<std::min<uint32_t>(b.cap[CLS_MID], 512), SORT_NT, 0, st>>>(
                    b, sA, sVA, sD, sVD); });
        if (!lists[CLS_BIG].empty()) {
            launch("k_bucket_big", keys[CLS_BIG], [&] {
                k_bucket_big<K, HV2><<<std::min<uint32_t>(b.cap[CLS_BIG], 512), BK_NT, 0, st>>>(b, sA, sVA, sD, sVD); });
            if (int rc = check()) return rc;
            return read_fail(ctr);
        }
        return check();
    }
    std::vector<std::vector<char>> keep_;      // host copies that async uploads read

    // Independent instances [offs[i], offs[i+1]) with seeds[i].  Each base-case
    // instance becomes a one-bucket node (m = 1, so its key range is the whole
    // type) on the bucket work lists; every other instance is a root node of
    // one shared first batch.  Nodes never interact, so instance i gets
    // exactly the result (and recursion tree) of sorting it alone.
    int sort_many(uint32_t count, const uint64_t *offs, const uint64_t *seeds)
    {
        std::vector<HostNode> roots;
        std::vector<NodeDesc> leaf;
        std::vector<BucketItem> lists[NCLS];
        for (uint32_t i = 0; i < count; ++i) {
            const uint64_t n = offs[i + 1] - offs[i];
            if (n == 0) continue;
            if (n > cutoff) { roots.push_back({offs[i], (uint32_t)n, splitmix(seeds[i])}); continue; }
            NodeDesc d{};
            d.off = offs[i];
            d.n = (uint32_t)n;
            d.m = 1;
            const int cls = size_class(n, tile.wcap, tile.m4cap);
            lists[cls].push_back(BucketItem{(uint32_t)leaf.size(), 0u, 0u, (uint32_t)n});
            leaf.push_back(d);
        }
        if (!leaf.empty()) {
            const uint64_t mark = ws.top;
            // Too few large leaves to fill the chip with one work-group each:
            // split each over the grid instead.
            std::vector<BucketItem> big;
            if (!lists[CLS_BIG].empty() && lists[CLS_BIG].size() <= SPLIT_SEGS) big.swap(lists[CLS_BIG]);
            bool rest = false;
            for (int c = 0; c < NCLS; ++c) rest |= !lists[c].empty();
            if (rest)
                if (int rc = sort_segments<HV>(A, VA, D, VD, leaf, lists)) return rc;
            if (!big.empty()) {
                const uint32_t ns = (uint32_t)big.size();
                keep_.emplace_back(ns * 8 + ns * 4 + (ns + 1) * 4, 0);
                char *hb = keep_.back().data();
                uint64_t *hOff = reinterpret_cast<uint64_t *>(hb);
                uint32_t *hN = reinterpret_cast<uint32_t *>(hb + ns * 8);
                uint32_t *hCh = hN + ns;
                uint64_t keys = 0;
                hCh[0] = 0;
                for (uint32_t q = 0; q < ns; ++q) {
                    hOff[q] = leaf[big[q].node].off;
                    hN[q] = big[q].size;
                    hCh[q + 1] = hCh[q] + cdiv(big[q].size, BS_CH);
                    keys += big[q].size;
                }
                char *dSeg = ws.take<char>(keep_.back().size());
                if (ws.overflow) return SQS_ERR_WORKSPACE;
                if (int rc = upload(dSeg, hb, keep_.back().size())) return rc;
                const uint64_t *dOff = reinterpret_cast<const uint64_t *>(dSeg);
                const uint32_t *dN = reinterpret_cast<const uint32_t *>(dSeg + ns * 8);
                if (int rc = split_segments(ns, hCh[ns], 0, dOff, dN, dN + ns, keys)) return rc;
            }
            if (!graph && hipStreamSynchronize(st) != hipSuccess) return SQS_ERR_DEVICE;   // host lists outlive the uploads
            keep_.clear();
            resolve_timing();
            release(mark);
        }
        if (!roots.empty()) return finish(run_batch(roots, 0));
        return SQS_OK;
    }
};

// Workspace of a batched call: the base-case lists, then (after they are
// released) the shared first batch of the other instances and its recursion.
uint64_t batched_workspace_bound(uint32_t count, const uint64_t *offs, uint64_t C, uint64_t key_bytes)
{
    uint64_t S = 0, big = 0, L = 0, nl = 0;
    for (uint32_t i = 0; i < count; ++i) {
        const uint64_t n = offs[i + 1] - offs[i];
        if (n > C) { S += n; big = std::max(big, n); }
        else if (n > (uint64_t)SORT_CAP) { L += n; ++nl; }
    }
    // leaf lists, plus the grid-wide split of the large leaves (chunk ranges
    // and counts per 4096 keys; node, pivots, flags and parts per leaf)
    const uint64_t split = (L / BS_CH + nl) * (2 * key_bytes + 256 * 4) +
                           nl * (256 * (16 + 2 * key_bytes) + 16) + (64 << 10);
    const uint64_t leaves = (uint64_t)count * (sizeof(NodeDesc) + 4 * sizeof(BucketItem) + 16 + 2 * key_bytes) +
                            12 * 256 + split;
    if (S == 0) return leaves;
    uint64_t chain = 1;
    for (uint64_t s = ceil_isqrt_host(big); s > C && chain < 8; s = ceil_isqrt_host(s)) ++chain;
    return std::max(leaves, chain * (batch_bound(S, C, key_bytes) + small_list_bytes(S, C)) + (1 << 20));
}

constexpr uint64_t key_bytes_of(int kind) { return kind == SQS_KIND_U32 ? 4 : 8; }

// the automatic (and largest) cut-off: a base case is sorted by one
// work-group, in LDS up to SORT_CAP keys and with MSD splits above
uint64_t max_cutoff_of(int kind) { return (kind >= SQS_KIND_U32 && kind <= SQS_KIND_KV) ? BIG_CAP : 0; }

uint64_t max_n_of(int kind)
{
    if (kind < SQS_KIND_U32 || kind > SQS_KIND_KV) return 0;
    // 32-bit positions inside a node; columns longer than one LDS sort are
    // sorted through HBM (NODE_HUGE)
    return 0xFFFFFFFFull;
}

// the skew entry point and the Alg. 1 pivot rule keep columns within one LDS sort
uint64_t max_n_lds(int kind)
{
    if (kind < SQS_KIND_U32 || kind > SQS_KIND_KV) return 0;
    return (uint64_t)SORT_CAP * SORT_CAP;
}

int resolve_cutoff(int kind, sqs_params *p, uint32_t *out)
{
    uint64_t c = p ? p->cutoff : 0;
    if (c == 0) c = max_cutoff_of(kind);
    if (c < 4 || c > max_cutoff_of(kind)) return SQS_ERR_ARG;
    Tile t;
    if (p && !decode_tile(p->tile, t)) return SQS_ERR_ARG;
    if (p) p->cutoff = c;
    *out = (uint32_t)c;
    return SQS_OK;
}

bool overlap(const void *a, uint64_t abytes, const void *b, uint64_t bbytes)
{
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    return x < y + bbytes && y < x + abytes;
}

// ------------------------------------------------------------ static scratch
// Scratch of squaresort_u32_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: kernels get the device address that
// hipGetSymbolAddress returns, looked up once per device with that device
// current and kept in scratch_ptr.
__device__ __align__(256) unsigned char scratch[SQS_STATIC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES];

// Device address of the current device's scratch.  The stream (if not null)
// must belong to the current device: the array is per device.
int static_scratch(hipStream_t stream, void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return SQS_ERR_DEVICE;
    if (stream) {
        hipDevice_t sdev = -1;
        if (hipStreamGetDevice(stream, &sdev) != hipSuccess) return SQS_ERR_DEVICE;
        if (sdev != dev) return SQS_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SQS_ERR_DEVICE;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return SQS_OK;
}

// The device address of pinned host memory (hipHostMalloc'd, so mapped into
// the device's address space); SQS_ERR_ARG for any other pointer.
template <class T> int host_array(T *&ptr)
{
    if (!ptr) return SQS_OK;
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
        (void)hipGetLastError();                 // clear the sticky error of an unknown pointer
        return SQS_ERR_ARG;
    }
    if (at.type != hipMemoryTypeHost) return SQS_ERR_ARG;
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, ptr, 0) != hipSuccess || !d) return SQS_ERR_ARG;
    ptr = static_cast<T *>(d);
    return SQS_OK;
}

template <class K, bool HV>
int run_sort(uint64_t n, K *in, uint32_t *vin, K *out, uint32_t *vout, uint64_t seed, sqs_params *p,
             void *stream, int kind)
{
    uint32_t C;
    if (int rc = resolve_cutoff(kind, p, &C)) return rc;
    if (n == 0) return SQS_OK;
    if (!in || !out || (HV && (!vin || !vout))) return SQS_ERR_ARG;
    if (p && (p->flags & SQS_FLAG_HOST_ARRAYS)) {        // the arrays stay in host memory
        if (int rc = host_array(in)) return rc;
        if (int rc = host_array(out)) return rc;
        if (int rc = host_array(vin)) return rc;
        if (int rc = host_array(vout)) return rc;
    }
    if (n > max_n_of(kind)) return SQS_ERR_UNSUPPORTED;
    if (overlap(in, n * sizeof(K), out, n * sizeof(K))) return SQS_ERR_ALIAS;
    if (HV && (overlap(vin, n * 4, vout, n * 4) || overlap(vin, n * 4, in, n * sizeof(K)) ||
               overlap(vin, n * 4, out, n * sizeof(K)) || overlap(vout, n * 4, in, n * sizeof(K)) ||
               overlap(vout, n * 4, out, n * sizeof(K))))
        return SQS_ERR_ALIAS;
    const uint64_t need = workspace_bound(n, C, sizeof(K) + (HV ? 4 : 0));
    if (n > (uint64_t)SORT_CAP && (!p || !p->workspace || p->workspace_bytes < need)) return SQS_ERR_WORKSPACE;
    const bool dig = p && (p->flags & SQS_FLAG_DIGEST);
    if (dig && !p->digest) return SQS_ERR_ARG;
    if (p && (p->flags & SQS_FLAG_COLS_SORTED)) return SQS_ERR_ARG;      // skew_transpose_u32 only
    const bool validate = p && (p->flags & SQS_FLAG_VALIDATE);
    if (validate && (!p->workspace || p->workspace_bytes < 256)) return SQS_ERR_WORKSPACE;
    Engine<K, HV> e;
    if (p) decode_tile(p->tile, e.tile);
    e.A = in; e.VA = vin; e.D = out; e.VD = vout;
    e.cutoff = C;
    e.st = (hipStream_t)stream;
    e.ws.base = p ? static_cast<char *>(p->workspace) : nullptr;
    e.ws.size = p ? p->workspace_bytes : 0;
    e.digest = dig;
    e.digest_ptr = dig ? reinterpret_cast<unsigned long long *>(p->digest) : nullptr;
    e.alg1 = p && (p->flags & SQS_FLAG_ALG1_PIVOTS);
    if (int rc = e.sort_root(n, seed)) return rc;
    if (!validate) return SQS_OK;
    // SQS_FLAG_VALIDATE: the output must be in key order
    e.ws.top = 0;
    uint32_t *flag = e.ws.template take<uint32_t>(1);
    if (!flag) return SQS_ERR_WORKSPACE;
    k_fill_u32<<<1, 64, 0, e.st>>>(flag, 1, 0u);
    k_check_sorted<K><<<std::min<uint64_t>(cdiv(n, 256), 4096), 256, 0, e.st>>>(out, n, n, flag);
    uint32_t bad = 0;
    if (hipGetLastError() != hipSuccess || hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, e.st) != hipSuccess ||
        hipStreamSynchronize(e.st) != hipSuccess)
        return SQS_ERR_DEVICE;
    return bad ? SQS_ERR_DEVICE : SQS_OK;
}

}  // namespace
}  // namespace sqs

using namespace sqs;

extern "C" {

uint64_t sqs_max_cutoff(int kind) { return max_cutoff_of(kind); }
uint64_t sqs_max_n(int kind) { return max_n_of(kind); }

uint64_t squaresort_workspace_bytes(uint64_t n, int kind, uint64_t cutoff)
{
    if (kind < SQS_KIND_U32 || kind > SQS_KIND_KV) return 0;
    if (cutoff == 0) cutoff = max_cutoff_of(kind);
    if (cutoff < 4) cutoff = 4;
    return workspace_bound(n, cutoff, key_bytes_of(kind) + (kind == SQS_KIND_KV ? 4 : 0));
}

int squaresort_u32(uint64_t n, uint32_t *in, uint32_t *out, uint64_t seed, sqs_params *params, void *stream)
{
    return run_sort<uint32_t, false>(n, in, nullptr, out, nullptr, seed, params, stream, SQS_KIND_U32);
}

int squaresort_u64(uint64_t n, uint64_t *in, uint64_t *out, uint64_t seed, sqs_params *params, void *stream)
{
    return run_sort<uint64_t, false>(n, in, nullptr, out, nullptr, seed, params, stream, SQS_KIND_U64);
}

int squaresort_kv(uint64_t n, uint64_t *keys_in, uint32_t *vals_in, uint64_t *keys_out, uint32_t *vals_out,
                  uint64_t seed, sqs_params *params, void *stream)
{
    return run_sort<uint64_t, true>(n, keys_in, vals_in, keys_out, vals_out, seed, params, stream, SQS_KIND_KV);
}

int skew_transpose_u32(uint64_t n, uint32_t *in, uint32_t *out, uint64_t *bucket_start, uint64_t seed,
                       sqs_params *params, void *stream)
{
    uint32_t C;
    if (int rc = resolve_cutoff(SQS_KIND_U32, params, &C)) return rc;
    if (n < 2 || !in || !out) return SQS_ERR_ARG;
    if (params && (params->flags & SQS_FLAG_HOST_ARRAYS)) return SQS_ERR_ARG;   // single sorts only
    if (n > max_n_lds(SQS_KIND_U32)) return SQS_ERR_UNSUPPORTED;
    if (overlap(in, n * 4, out, n * 4)) return SQS_ERR_ALIAS;
    const uint64_t m = ceil_isqrt_host(n);
    if (bucket_start && (overlap(bucket_start, (m + 1) * 8, in, n * 4) || overlap(bucket_start, (m + 1) * 8, out, n * 4)))
        return SQS_ERR_ALIAS;
    // one batch of the root alone, columns sorted completely in LDS
    const uint64_t need = node_meta_bytes(n, 4) + (64 << 10);
    if (!params || !params->workspace || params->workspace_bytes < need) return SQS_ERR_WORKSPACE;
    Engine<uint32_t, false> e;
    decode_tile(params->tile, e.tile);
    e.A = in; e.VA = nullptr; e.D = nullptr; e.VD = nullptr;
    e.cutoff = C;
    e.st = (hipStream_t)stream;
    e.ws.base = static_cast<char *>(params->workspace);
    e.ws.size = params->workspace_bytes;
    e.digest = false;
    e.digest_ptr = nullptr;
    e.skew_only = true;
    e.alg1 = params->flags & SQS_FLAG_ALG1_PIVOTS;
    e.skew_out = out;
    e.skew_bs = reinterpret_cast<unsigned long long *>(bucket_start);
    e.cols_sorted = params->flags & SQS_FLAG_COLS_SORTED;
    e.validate = params->flags & SQS_FLAG_VALIDATE;
    std::vector<HostNode> root{{0, (uint32_t)n, splitmix(seed)}};
    return e.run_batch(root, 0);
}

int squaresort_u32_noalloc(uint64_t n, uint32_t *in, uint32_t *out, uint64_t seed, sqs_params *params,
                           void *stream)
{
    sqs_params local{};
    if (params) local = *params;
    if (local.flags & SQS_FLAG_HOST_ARRAYS) return SQS_ERR_ARG;         // device arrays only
    uint32_t C;
    if (int rc = resolve_cutoff(SQS_KIND_U32, &local, &C)) return rc;
    // sizes whose scratch exceeds the static array are rejected up front
    if (n > (uint64_t)SORT_CAP && workspace_bound(n, C, 4) > SQS_STATIC_SCRATCH_BYTES) return SQS_ERR_WORKSPACE;
    void *scr = nullptr;
    if (int rc = static_scratch((hipStream_t)stream, &scr)) return rc;
    local.workspace = scr;
    local.workspace_bytes = SQS_STATIC_SCRATCH_BYTES;
    const int rc = run_sort<uint32_t, false>(n, in, nullptr, out, nullptr, seed, &local, stream, SQS_KIND_U32);
    if (params) params->cutoff = local.cutoff;
    return rc;
}

uint64_t squaresort_batched_workspace_bytes(uint32_t count, const uint64_t *offsets, int kind, uint64_t cutoff)
{
    if ((kind != SQS_KIND_U32 && kind != SQS_KIND_KV) || !offsets) return 0;
    if (cutoff == 0) cutoff = max_cutoff_of(kind);
    if (cutoff < 4) cutoff = 4;
    for (uint32_t i = 0; i < count; ++i) if (offsets[i + 1] < offsets[i]) return 0;
    return batched_workspace_bound(count, offsets, cutoff, key_bytes_of(kind) + (kind == SQS_KIND_KV ? 4 : 0));
}

}  // extern "C"

namespace sqs {
namespace {
template <class K, bool HV>
int run_batched(uint32_t count, const uint64_t *offsets, K *in, uint32_t *vin, K *out, uint32_t *vout,
                const uint64_t *seeds, sqs_params *params, void *stream, int kind)
{
    uint32_t C;
    if (int rc = resolve_cutoff(kind, params, &C)) return rc;
    if (count == 0) return SQS_OK;
    if (!offsets || !seeds || offsets[0] != 0) return SQS_ERR_ARG;
    for (uint32_t i = 0; i < count; ++i) {
        if (offsets[i + 1] < offsets[i]) return SQS_ERR_ARG;
        if (offsets[i + 1] - offsets[i] > max_n_of(kind)) return SQS_ERR_UNSUPPORTED;
    }
    const uint64_t total = offsets[count];
    if (total == 0) return SQS_OK;
    if (total > 0xFFFFFFFFull) return SQS_ERR_UNSUPPORTED;
    if (!in || !out || (HV && (!vin || !vout))) return SQS_ERR_ARG;
    const uint64_t kb = total * sizeof(K), vb = total * 4;
    if (overlap(in, kb, out, kb)) return SQS_ERR_ALIAS;
    if (HV && (overlap(vin, vb, vout, vb) || overlap(vin, vb, in, kb) || overlap(vin, vb, out, kb) ||
               overlap(vout, vb, in, kb) || overlap(vout, vb, out, kb)))
        return SQS_ERR_ALIAS;
    const uint64_t need = batched_workspace_bound(count, offsets, C, sizeof(K) + (HV ? 4 : 0));
    if (!params || !params->workspace || params->workspace_bytes < need) return SQS_ERR_WORKSPACE;
    const bool dig = params->flags & SQS_FLAG_DIGEST;
    if (dig && !params->digest) return SQS_ERR_ARG;
    if (params->flags & (SQS_FLAG_COLS_SORTED | SQS_FLAG_VALIDATE | SQS_FLAG_HOST_ARRAYS))
        return SQS_ERR_ARG;                                  // single-instance flags
    Engine<K, HV> e;
    decode_tile(params->tile, e.tile);
    e.A = in; e.VA = vin; e.D = out; e.VD = vout;
    e.cutoff = C;
    e.st = (hipStream_t)stream;
    e.ws.base = static_cast<char *>(params->workspace);
    e.ws.size = params->workspace_bytes;
    e.digest = dig;
    e.digest_ptr = dig ? reinterpret_cast<unsigned long long *>(params->digest) : nullptr;
    e.alg1 = params->flags & SQS_FLAG_ALG1_PIVOTS;
    return e.sort_many(count, offsets, seeds);
}
}  // namespace
}  // namespace sqs

extern "C" {

int squaresort_batched_u32(uint32_t count, const uint64_t *offsets, uint32_t *in, uint32_t *out,
                           const uint64_t *seeds, sqs_params *params, void *stream)
{
    return run_batched<uint32_t, false>(count, offsets, in, nullptr, out, nullptr, seeds, params, stream,
                                        SQS_KIND_U32);
}

int squaresort_batched_kv(uint32_t count, const uint64_t *offsets, uint64_t *keys_in, uint32_t *vals_in,
                          uint64_t *keys_out, uint32_t *vals_out, const uint64_t *seeds, sqs_params *params,
                          void *stream)
{
    return run_batched<uint64_t, true>(count, offsets, keys_in, vals_in, keys_out, vals_out, seeds, params,
                                       stream, SQS_KIND_KV);
}

// ------------------------------------------------------------ planned graphs
struct sqs_plan {
    hipStream_t cs = nullptr, up = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

uint64_t squaresort_batched_graph_workspace_bytes(uint32_t count, const uint64_t *offsets, uint64_t cutoff)
{
    if (!offsets) return 0;
    if (cutoff == 0) cutoff = max_cutoff_of(SQS_KIND_U32);
    if (cutoff < 4) cutoff = 4;
    for (uint32_t i = 0; i < count; ++i) if (offsets[i + 1] < offsets[i]) return 0;
    // every phase keeps its workspace (a replay runs all of them): at most
    // the base-case lists plus the recursion steps, each within the
    // batched bound
    return 2 * batched_workspace_bound(count, offsets, cutoff, 4);
}

int squaresort_batched_graph_u32(uint32_t count, const uint64_t *offsets, uint32_t *in, uint32_t *out,
                                 const uint64_t *seeds, sqs_params *params, uint32_t *status, sqs_plan **plan)
{
    if (!plan) return SQS_ERR_ARG;
    *plan = nullptr;
    uint32_t C;
    if (int rc = resolve_cutoff(SQS_KIND_U32, params, &C)) return rc;
    if (count == 0 || !offsets || !seeds || offsets[0] != 0 || !status || !params) return SQS_ERR_ARG;
    for (uint32_t i = 0; i < count; ++i) {
        if (offsets[i + 1] < offsets[i]) return SQS_ERR_ARG;
        // columns within one LDS sort: no recursion step through HBM counts
        if (offsets[i + 1] - offsets[i] > max_n_lds(SQS_KIND_U32)) return SQS_ERR_UNSUPPORTED;
    }
    const uint64_t total = offsets[count];
    if (total == 0 || total > 0xFFFFFFFFull) return total == 0 ? SQS_ERR_ARG : SQS_ERR_UNSUPPORTED;
    if (!in || !out) return SQS_ERR_ARG;
    if (overlap(in, total * 4, out, total * 4)) return SQS_ERR_ALIAS;
    if (params->flags & ~(uint32_t)SQS_FLAG_DIGEST) return SQS_ERR_ARG;
    const bool dig = params->flags & SQS_FLAG_DIGEST;
    if (dig && !params->digest) return SQS_ERR_ARG;
    const uint64_t need = squaresort_batched_graph_workspace_bytes(count, offsets, C);
    if (!params->workspace || params->workspace_bytes < need) return SQS_ERR_WORKSPACE;
    sqs_plan *pl = new sqs_plan;
    hipError_t se = hipStreamCreateWithFlags(&pl->cs, hipStreamNonBlocking);
    if (se == hipSuccess) se = hipStreamCreateWithFlags(&pl->up, hipStreamNonBlocking);
    if (se != hipSuccess) {
        if (debug_on()) fprintf(stderr, "[sqs] plan: stream %s\n", hipGetErrorString(se));
        sqs_plan_destroy(pl);
        return SQS_ERR_DEVICE;
    }
    const hipError_t be = hipStreamBeginCapture(pl->cs, hipStreamCaptureModeRelaxed);
    if (be != hipSuccess) {
        if (debug_on()) fprintf(stderr, "[sqs] plan: begin capture %s\n", hipGetErrorString(be));
        sqs_plan_destroy(pl);
        return SQS_ERR_DEVICE;
    }
    k_fill_u32<<<1, 64, 0, pl->cs>>>(status, 1, 0u);
    int rc;
    {
        Engine<uint32_t, false> e;
        e.A = in; e.VA = nullptr; e.D = out; e.VD = nullptr;
        decode_tile(params->tile, e.tile);
        e.cutoff = C;
        e.st = pl->cs;
        e.ws.base = static_cast<char *>(params->workspace);
        e.ws.size = params->workspace_bytes;
        e.digest = dig;
        e.digest_ptr = dig ? reinterpret_cast<unsigned long long *>(params->digest) : nullptr;
        e.graph = true;
        e.status_ptr = status;
        e.up = pl->up;
        rc = e.sort_many(count, offsets, seeds);
    }
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(pl->cs, &g);
    if (debug_on()) fprintf(stderr, "[sqs] plan: engine %d, end capture %s\n", rc, hipGetErrorString(ce));
    if (rc == SQS_OK && (ce != hipSuccess || !g)) rc = SQS_ERR_DEVICE;
    pl->graph = g;
    if (rc == SQS_OK) {
        const hipError_t ie = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            if (debug_on()) fprintf(stderr, "[sqs] plan: instantiate %s\n", hipGetErrorString(ie));
            rc = SQS_ERR_DEVICE;
        }
    }
    if (rc != SQS_OK) {
        sqs_plan_destroy(pl);
        return rc;
    }
    *plan = pl;
    return SQS_OK;
}

int sqs_plan_launch(sqs_plan *plan, void *stream)
{
    if (!plan || !plan->exec) return SQS_ERR_ARG;
    return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? SQS_OK : SQS_ERR_DEVICE;
}

int sqs_plan_destroy(sqs_plan *plan)
{
    if (!plan) return SQS_OK;
    int rc = SQS_OK;
    if (plan->exec && hipGraphExecDestroy(plan->exec) != hipSuccess) rc = SQS_ERR_DEVICE;
    if (plan->graph && hipGraphDestroy(plan->graph) != hipSuccess) rc = SQS_ERR_DEVICE;
    if (plan->cs && hipStreamDestroy(plan->cs) != hipSuccess) rc = SQS_ERR_DEVICE;
    if (plan->up && hipStreamDestroy(plan->up) != hipSuccess) rc = SQS_ERR_DEVICE;
    delete plan;
    return rc;
}

int sqs_timing_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.resolve();
    g_timing.acc.clear();
    g_timing.on = on != 0;
    return SQS_OK;
}

int64_t sqs_timing_report(char *buf, uint64_t len)
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.resolve();
    std::string js = "{";
    bool first = true;
    for (auto &kv : g_timing.acc) {
        char item[256];
        snprintf(item, sizeof item, "%s\"%s\": [%.6f, %llu, %llu]", first ? "" : ", ", kv.first.c_str(),
                 kv.second.ms, (unsigned long long)kv.second.launches, (unsigned long long)kv.second.units);
        js += item;
        first = false;
    }
    js += "}";
    if (buf && len > 0) {
        const uint64_t c = std::min<uint64_t>(len - 1, js.size());
        memcpy(buf, js.data(), c);
        buf[c] = 0;
    }
    return (int64_t)js.size();
}

const char *sqs_status_string(int s)
{
    switch (s) {
    case SQS_OK: return "ok";
    case SQS_ERR_ARG: return "invalid argument";
    case SQS_ERR_ALIAS: return "input and output overlap";
    case SQS_ERR_WORKSPACE: return "workspace missing or too small";
    case SQS_ERR_DEVICE: return "HIP launch or copy failed";
    case SQS_ERR_PRECOND: return "precondition failed (Alg. 1 pivot rule without distinct samples, or unsorted columns given as sorted)";
    case SQS_ERR_DEPTH: return "recursion too deep";
    case SQS_ERR_UNSUPPORTED: return "size not supported";
    default: return "unknown status";
    }
}

}  // extern "C"
