"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bit-exact on every check: sorted keys, key/value pairs in (key, original
index) order, the root SkewTranspose intermediate at the same seed, and the
recursion-tree digest at the same seed and cut-off.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2407_14801_amd import datagen

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def b():
    assert torch.cuda.is_available(), "these tests need the GPU"
    from paper_2407_14801_amd import binding
    return binding


@pytest.fixture(scope="module")
def ws(b):
    return b.Workspace(DEV)


def _say(*a):
    print(*a, flush=True)


def gpu_u32(b, ws, x, seed, cutoff, digest=False):
    inp = torch.from_numpy(np.ascontiguousarray(x, np.uint32).view(np.int32)).to(DEV)
    out = torch.empty_like(inp)
    dg = torch.zeros(1, dtype=torch.int64, device=DEV) if digest else None
    used = b.squaresort_u32(inp, out, seed=seed, cutoff=cutoff, ws=ws, digest=dg)
    torch.cuda.synchronize()
    res = out.cpu().numpy().view(np.uint32)
    if digest:
        return res, int(dg.cpu().numpy().view(np.uint64)[0]), used
    return res, used


def gpu_u64(b, ws, x, seed, cutoff, digest=False):
    inp = torch.from_numpy(np.ascontiguousarray(x, np.uint64).view(np.int64)).to(DEV)
    out = torch.empty_like(inp)
    dg = torch.zeros(1, dtype=torch.int64, device=DEV) if digest else None
    used = b.squaresort_u64(inp, out, seed=seed, cutoff=cutoff, ws=ws, digest=dg)
    torch.cuda.synchronize()
    res = out.cpu().numpy().view(np.uint64)
    if digest:
        return res, int(dg.cpu().numpy().view(np.uint64)[0]), used
    return res, used


def gpu_kv(b, ws, k, v, seed, cutoff, digest=False):
    ki = torch.from_numpy(np.ascontiguousarray(k, np.uint64).view(np.int64)).to(DEV)
    vi = torch.from_numpy(np.ascontiguousarray(v, np.uint32).view(np.int32)).to(DEV)
    ko, vo = torch.empty_like(ki), torch.empty_like(vi)
    dg = torch.zeros(1, dtype=torch.int64, device=DEV) if digest else None
    used = b.squaresort_kv(ki, vi, ko, vo, seed=seed, cutoff=cutoff, ws=ws, digest=dg)
    torch.cuda.synchronize()
    out = (ko.cpu().numpy().view(np.uint64), vo.cpu().numpy().view(np.uint32))
    if digest:
        return out + (int(dg.cpu().numpy().view(np.uint64)[0]), used)
    return out + (used,)


def gpu_skew(b, ws, x, seed):
    n = x.size
    m = oracle.ceil_isqrt(n)
    inp = torch.from_numpy(np.ascontiguousarray(x, np.uint32).view(np.int32)).to(DEV)
    out = torch.empty_like(inp)
    bs = torch.empty(m + 1, dtype=torch.int64, device=DEV)
    b.skew_transpose_u32(inp, out, bs, seed=seed, ws=ws)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32), bs.cpu().numpy().view(np.uint64)


# ------------------------------------------------------------------ u32
U32_CASES = [
    # (n, cutoff): spans base cases, one internal level, nested column
    # recursion (m > cutoff), ragged tails (n not a square, empty last column)
    (1, 0), (2, 0), (3, 4), (5, 4), (8, 4), (100, 4), (1000, 16), (4097, 64),
    (16384, 0), (16385, 0), (65537, 0), (65537, 64), (1_000_003, 0),
    ((1 << 20) + 3, 0), (3_000_017, 0), (130_000, 256),
    # whole array a base case sorted with MSD splits (16384 < n <= cutoff)
    (16_385, 0), (50_000, 0), (65_536, 0), (100_000, 0), (131_072, 0),
    (131_073, 0), (262_144, 0),
    # just above the automatic cut-off: one internal level with big buckets
    (262_145, 0),
    # buckets of 16K..64K keys (MSD-split base cases inside the bucket phase)
    ((1 << 24) + 5, 0), ((1 << 22) + 1, 20_000),
]


@pytest.mark.parametrize("n,cutoff", U32_CASES)
def test_u32_matches_oracle(b, ws, n, cutoff):
    _say(f"u32 n={n} cutoff={cutoff}")
    x = datagen.uniform_u32(n, seed=n)
    got, used = gpu_u32(b, ws, x, seed=3, cutoff=cutoff)
    assert np.array_equal(got, np.sort(x))
    want = oracle.squaresort_u32(x, 3, used)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("kind", ["perm", "binary", "uniform_n", "uniform_sqrt"])
def test_u32_paper_distributions(b, ws, kind):
    n = 300_007
    _say(f"u32 paper distribution {kind} n={n}")
    x = datagen.paper_u32(kind, n, seed=5)
    got, used = gpu_u32(b, ws, x, seed=2, cutoff=0)
    assert np.array_equal(got, np.sort(x))


def _degenerate(n):
    g = np.random.default_rng(n)
    return {
        "all_equal": np.full(n, 12345, np.uint32),
        "all_zero": np.zeros(n, np.uint32),
        "all_max": np.full(n, 2**32 - 1, np.uint32),
        "two_values": np.where(g.random(n) < 0.5, 7, 8).astype(np.uint32),
        "extremes": np.where(g.random(n) < 0.5, 0, 2**32 - 1).astype(np.uint32),
        "sorted": np.arange(n, dtype=np.uint32),
        "reversed": np.arange(n, dtype=np.uint32)[::-1].copy(),
        "organ_pipe": np.concatenate([np.arange(n // 2), np.arange(n - n // 2)[::-1]]).astype(np.uint32),
        "dup16": datagen.uniform_u32(n, seed=7, hi=1 << 16),
        "few_runs": np.repeat(g.integers(0, 2**32, size=50, dtype=np.uint64), n // 50 + 1)[:n].astype(np.uint32),
    }


@pytest.mark.parametrize("n,cutoff", [(200_003, 0), (70_000, 64), (2_000_003, 20_000)])
@pytest.mark.parametrize("name", list(_degenerate(10).keys()))
def test_u32_degenerate_inputs(b, ws, n, cutoff, name):
    _say(f"u32 degenerate {name} n={n} cutoff={cutoff}")
    x = _degenerate(n)[name]
    got, dg, used = gpu_u32(b, ws, x, seed=1, cutoff=cutoff, digest=True)
    want, wdg, _ = oracle.squaresort_u32(x, 1, used, want_digest=True)
    assert np.array_equal(got, want)
    assert dg == wdg


@pytest.mark.parametrize("n,cutoff", [(1 << 20, 64), (100_000, 16), (1 << 20, 0)])
def test_u32_digest_matches_oracle(b, ws, n, cutoff):
    """The recursion tree (pivots, layouts of every internal node) matches."""
    _say(f"u32 digest n={n} cutoff={cutoff}")
    x = datagen.uniform_u32(n, seed=1)
    got, dg, used = gpu_u32(b, ws, x, seed=1, cutoff=cutoff, digest=True)
    want, wdg, nodes = oracle.squaresort_u32(x, 1, used, want_digest=True)
    assert np.array_equal(got, want)
    assert dg == wdg, f"digest {dg:#x} != {wdg:#x} ({nodes} internal nodes)"


# ------------------------------------------------------------------ SkewTranspose
@pytest.mark.parametrize("n", [2, 4, 5, 17, 1000, 4096, 65541, 1 << 20, 3_000_001])
def test_skew_transpose_matches_oracle(b, ws, n):
    _say(f"skew n={n}")
    x = datagen.uniform_u32(n, seed=n + 1)
    got, bs = gpu_skew(b, ws, x, seed=7)
    want, wbs = oracle.root_intermediate(x.astype(np.uint64), seed=7)
    assert np.array_equal(bs, wbs)
    assert np.array_equal(got.astype(np.uint64), want)


@pytest.mark.parametrize("name", ["dup16", "two_values", "all_equal", "sorted", "few_runs"])
def test_skew_transpose_degenerate(b, ws, name):
    x = _degenerate(250_000)[name]
    _say(f"skew degenerate {name}")
    got, bs = gpu_skew(b, ws, x, seed=3)
    want, wbs = oracle.root_intermediate(x.astype(np.uint64), seed=3)
    assert np.array_equal(bs, wbs)
    assert np.array_equal(got.astype(np.uint64), want)


def test_skew_transpose_is_root_of_sort(b, ws):
    """The entry point's output is SquareSort's array A after the root step."""
    n = 500_000
    x = datagen.uniform_u32(n, seed=11)
    got, _ = gpu_skew(b, ws, x, seed=9)
    want_sort, used = gpu_u32(b, ws, x, seed=9, cutoff=0)
    want_root, _ = oracle.root_intermediate(x.astype(np.uint64), seed=9)
    assert np.array_equal(got.astype(np.uint64), want_root)
    assert np.array_equal(want_sort, np.sort(x))


# ------------------------------------------------------------------ u64, kv
@pytest.mark.parametrize("n,cutoff", [(1, 0), (7, 4), (5000, 16), (16385, 0), (300_001, 0), (70_001, 64),
                                      (40_000, 0), (120_000, 0), ((1 << 22) + 7, 30_000)])
def test_u64_matches_oracle(b, ws, n, cutoff):
    _say(f"u64 n={n} cutoff={cutoff}")
    x = datagen.uniform_u64(n, seed=n)
    x[: n // 10] = x[0]
    got, dg, used = gpu_u64(b, ws, x, seed=4, cutoff=cutoff, digest=True)
    want, wdg, _ = oracle.squaresort_u64(x, 4, used, want_digest=True)
    assert np.array_equal(got, want)
    assert np.array_equal(got, np.sort(x))
    assert dg == wdg


@pytest.mark.parametrize("n,cutoff", [(9, 4), (5000, 16), (40_000, 64), (300_007, 0), (60_000, 0),
                                      (125_000, 0), ((1 << 23) + 3, 0), ((1 << 21) + 5, 1000)])
def test_kv_matches_oracle(b, ws, n, cutoff):
    _say(f"kv n={n} cutoff={cutoff}")
    k, v = datagen.kv_mixture(n, seed=4)
    ko, vo, dg, used = gpu_kv(b, ws, k, v, seed=1, cutoff=cutoff, digest=True)
    order = np.argsort(k, kind="stable")
    assert np.array_equal(ko, k[order])
    assert np.array_equal(vo, v[order])
    wk, wv, wdg, _ = oracle.squaresort_kv(k, v, 1, used, want_digest=True)
    assert np.array_equal(ko, wk) and np.array_equal(vo, wv)
    assert dg == wdg


# ------------------------------------------------------------------ whole-array base cases
# A base case above one LDS sort is split once over the whole grid by the top
# 8 bits of x - min: key spans of 8 bits (every part one value), 9 bits,
# keys next to the largest value of the type, and a span of one value.
def _span_keys(n, name, seed):
    g = np.random.default_rng(seed)
    top = 2**32 - 1
    return {
        "span8": g.integers(1000, 1256, size=n).astype(np.uint32),
        "span9": g.integers(1000, 1512, size=n).astype(np.uint32),
        "near_max": (top - g.integers(0, 1 << 20, size=n)).astype(np.uint32),
        "max_and_near": np.where(g.random(n) < 0.3, top, top - g.integers(0, 300, size=n)).astype(np.uint32),
        "one_value": np.full(n, top - 1, np.uint32),
        "sparse_outlier": np.where(np.arange(n) == n // 2, top, g.integers(0, 1 << 12, size=n)).astype(np.uint32),
    }[name]


@pytest.mark.parametrize("n", [16_385, 150_001, 262_144])
@pytest.mark.parametrize("name", ["span8", "span9", "near_max", "max_and_near", "one_value", "sparse_outlier"])
def test_u32_base_split_ranges(b, ws, n, name):
    _say(f"u32 base split {name} n={n}")
    x = _span_keys(n, name, seed=n + 1)
    got, used = gpu_u32(b, ws, x, seed=3, cutoff=0)
    assert used >= n
    assert np.array_equal(got, np.sort(x))


def _crowded(n, name, seed):
    # inputs that crowd a key-range bin of a column, bucket or MSD part (more
    # than 16 keys inside one bin's width): half the keys in a narrow window
    # ("window*"), or uniform keys with a few values of very high
    # multiplicity (crowding columns) and a pool of values repeated about 64
    # times each (crowding buckets and parts) ("spiky")
    g = np.random.default_rng(seed)
    x = g.integers(0, 2**32, size=n, dtype=np.uint64)
    u = g.random(n)
    if name.startswith("window"):
        w = u < 0.5
        x[w] = 123_456_789 + g.integers(0, 1 << int(name[6:]), size=int(w.sum()))
    else:
        heavy = g.integers(0, 2**32, size=4, dtype=np.uint64)
        pool = g.integers(0, 2**32, size=max(1, n // 320), dtype=np.uint64)
        h = u < 0.2
        p = (u >= 0.2) & (u < 0.4)
        x[h] = heavy[g.integers(0, 4, size=int(h.sum()))]
        x[p] = pool[g.integers(0, pool.size, size=int(p.sum()))]
    return x.astype(np.uint32)


CROWDED_CASES = [(1 << 20, 0), (4_000_037, 0), ((1 << 22) + 1, 20_000), (300_001, 64), (200_000, 0)]


@pytest.mark.parametrize("n,cutoff", CROWDED_CASES)
@pytest.mark.parametrize("name", ["window8", "window16", "window24", "spiky"])
def test_u32_crowded_bins_digest(b, ws, n, cutoff, name):
    _say(f"u32 crowded {name} n={n} cutoff={cutoff}")
    x = _crowded(n, name, seed=n + len(name))
    got, dg, used = gpu_u32(b, ws, x, seed=5, cutoff=cutoff, digest=True)
    assert np.array_equal(got, np.sort(x))
    want, wdg, _ = oracle.squaresort_u32(x, 5, used, want_digest=True)
    assert dg == wdg


def test_u32_crowded_bins_large(b, ws):
    n = (1 << 24) + 5
    _say(f"u32 crowded spiky n={n}")
    x = _crowded(n, "spiky", seed=11)
    got, dg, used = gpu_u32(b, ws, x, seed=5, cutoff=0, digest=True)
    assert np.array_equal(got, np.sort(x))
    want, wdg, _ = oracle.squaresort_u32(x, 5, used, want_digest=True)
    assert dg == wdg


# Root buckets of 16385 .. 28672 32-bit keys are sorted whole in LDS by one
# bin sort; one with a crowded bin (more than 16 keys in one bin's width) is
# left to the MSD split.  The keys the wide-bucket kernel sorted are read from
# the library's per-kernel unit counts; the eligible buckets come from the
# oracle's root bucket starts at the same seed.
WIDE_MIN, WIDE_MAX = 16_384, 28_672


@pytest.mark.parametrize("name", ["uniform", "few_spikes", "spiky", "dup16", "dup14"])
def test_u32_wide_buckets(b, ws, name):
    n, seed, cutoff = (1 << 25) + 3, 7, 262_144
    _say(f"u32 wide buckets {name} n={n}")
    g = np.random.default_rng(21)
    if name == "spiky":                  # every large bucket crowds a bin: all go to the split
        x = _crowded(n, "spiky", seed=21)
    elif name.startswith("dup"):         # 2^16 values of 512 copies, 2^14 of 2048
        x = g.integers(0, 1 << int(name[3:]), size=n, dtype=np.uint64).astype(np.uint32)
    else:
        x = g.integers(0, 2**32, size=n, dtype=np.uint64)
        if name == "few_spikes":         # 200 values of 64 copies: a few buckets crowd a bin
            spikes = g.integers(0, 2**32, size=200, dtype=np.uint64)
            x[g.choice(n, 200 * 64, replace=False)] = np.repeat(spikes, 64)
        x = x.astype(np.uint32)
    _, bs = oracle.root_intermediate(x.astype(np.uint64), seed=seed)
    sz = np.diff(bs.astype(np.int64))
    eligible = int(sz[(sz > WIDE_MIN) & (sz <= WIDE_MAX)].sum())
    assert eligible > 0
    b.timing_enable(True)
    try:
        got, used = gpu_u32(b, ws, x, seed=seed, cutoff=cutoff)
        rep = b.timing_report()
    finally:
        b.timing_enable(False)
    assert used == cutoff
    assert np.array_equal(got, np.sort(x))
    wide = rep.get("k_bucket_wide", {}).get("units", 0)
    if name == "uniform":
        assert 0.95 * eligible <= wide <= eligible
    elif name == "few_spikes":
        assert 0 < wide < eligible
    elif name == "dup16":                # per value: no bin can crowd
        assert wide == eligible
    else:                                # spiky: crowded bins; dup14: ranges of at most 16 values
        assert wide == 0


@pytest.mark.parametrize("name", ["window8", "window16", "spiky"])
def test_skew_transpose_crowded(b, ws, name):
    n = (1 << 22) + 7
    _say(f"skew crowded {name}")
    x = _crowded(n, name, seed=3)
    got, bs = gpu_skew(b, ws, x, seed=9)
    want, wbs = oracle.root_intermediate(x.astype(np.uint64), seed=9)
    assert np.array_equal(bs, wbs)
    assert np.array_equal(got.astype(np.uint64), want)


@pytest.mark.parametrize("name", ["span8", "near_max", "one_value", "sparse_outlier"])
def test_kv_base_split_stable(b, ws, name):
    n = 200_001
    _say(f"kv base split {name} n={n}")
    k = _span_keys(n, name, seed=9).astype(np.uint64) << np.uint64(32)
    v = np.arange(n, dtype=np.uint32)
    ko, vo, used = gpu_kv(b, ws, k, v, seed=1, cutoff=0)
    order = np.argsort(k, kind="stable")
    assert np.array_equal(ko, k[order])
    assert np.array_equal(vo, v[order])


def test_u64_base_split_full_range(b, ws):
    n = 250_000
    _say(f"u64 base split full range n={n}")
    x = datagen.uniform_u64(n, seed=17)
    x[:100] = 2**64 - 1
    x[100:200] = 0
    got, used = gpu_u64(b, ws, x, seed=4, cutoff=0)
    assert used >= n
    assert np.array_equal(got, np.sort(x))


# ------------------------------------------------------------------ presorted inputs
# Presorted inputs put a column group's keys into a few bucket blocks: those
# SkewTranspose tiles hold many chunks, which other work-groups take as items
# whose destinations come from the tile's earlier chunks.  The intermediate
# order is checked exactly (against the oracle, or through the digest).
def _presorted(n, name, seed):
    g = np.random.default_rng(seed)
    u = np.sort(datagen.uniform_u32(n, seed=seed))
    if name == "sorted":
        return u
    if name == "reversed":
        return u[::-1].copy()
    if name == "near_sorted":              # 1% of positions swapped in pairs
        x = u.copy()
        p = g.permutation(n)[: (n // 100) * 2].reshape(-1, 2)
        x[p[:, 0]], x[p[:, 1]] = u[p[:, 1]], u[p[:, 0]]
        return x
    if name == "sawtooth":                 # 37 sorted runs
        return np.concatenate([np.sort(a) for a in np.array_split(datagen.uniform_u32(n, seed=seed), 37)])
    raise KeyError(name)


@pytest.mark.parametrize("name", ["sorted", "reversed", "near_sorted", "sawtooth"])
def test_skew_transpose_presorted(b, ws, name):
    n = 2_100_001
    _say(f"skew presorted {name} n={n}")
    x = _presorted(n, name, seed=5)
    got, bs = gpu_skew(b, ws, x, seed=3)
    want, wbs = oracle.root_intermediate(x.astype(np.uint64), seed=3)
    assert np.array_equal(bs, wbs)
    assert np.array_equal(got.astype(np.uint64), want)


@pytest.mark.parametrize("name", ["sorted", "near_sorted", "sawtooth"])
def test_u32_presorted_digest(b, ws, name):
    n = 4_000_037
    _say(f"u32 presorted {name} n={n}")
    x = _presorted(n, name, seed=6)
    got, dg, used = gpu_u32(b, ws, x, seed=2, cutoff=0, digest=True)
    assert np.array_equal(got, np.sort(x))
    want, wdg, _ = oracle.squaresort_u32(x, 2, used, want_digest=True)
    assert np.array_equal(got, want)
    assert dg == wdg


@pytest.mark.parametrize("n", [1_500_007, (1 << 22) + 1])
def test_kv_largest_keys_stable(b, ws, n):
    """Columns of the merge column sort whose lengths are not a multiple of
    a thread's run, with many keys equal to the largest 64-bit value (the
    value the sort pads with) among few others: equal keys keep their input
    order and the tree digest is the oracle's."""
    _say(f"kv largest keys n={n}")
    g = np.random.default_rng(n)
    top = np.uint64(2**64 - 1)
    k = np.where(g.random(n) < 0.6, top, top - g.integers(0, 50, size=n).astype(np.uint64)).astype(np.uint64)
    v = np.arange(n, dtype=np.uint32)
    ko, vo, dg, used = gpu_kv(b, ws, k, v, seed=3, cutoff=0, digest=True)
    order = np.argsort(k, kind="stable")
    assert np.array_equal(ko, k[order]) and np.array_equal(vo, v[order])
    _, _, wdg, _ = oracle.squaresort_kv(k, v, 3, used, want_digest=True)
    assert dg == wdg


def _clusters(size, seed):
    """16 clusters of `size` keys, cluster c in [c * 2^60, c * 2^60 + 2^20):
    the first split of a base case (top bits of x - min) gives 16 parts of
    `size` keys each, so the leaves have exactly that size."""
    g = np.random.default_rng(seed)
    k = (np.repeat(np.arange(16, dtype=np.uint64), size) << np.uint64(60)) + \
        g.integers(0, 1 << 20, size=16 * size).astype(np.uint64)
    return k[g.permutation(k.size)]


@pytest.mark.parametrize("size", [5000, 5632, 5633, 7000, 8100])
def test_kv_split_leaves_around_merge_capacity(b, ws, size):
    """Key/value leaves of the MSD split on both sides of the merge
    sort's capacity (5632 pairs; larger leaves take radix passes): stable
    order and the oracle's digest."""
    _say(f"kv split leaves size={size}")
    k = _clusters(size, seed=size)
    v = np.arange(k.size, dtype=np.uint32)
    ko, vo, dg, used = gpu_kv(b, ws, k, v, seed=2, cutoff=0, digest=True)
    order = np.argsort(k, kind="stable")
    assert np.array_equal(ko, k[order]) and np.array_equal(vo, v[order])
    _, _, wdg, _ = oracle.squaresort_kv(k, v, 2, used, want_digest=True)
    assert dg == wdg


@pytest.mark.parametrize("size", [7680, 7681, 8100])
def test_u64_split_leaves_around_merge_capacity(b, ws, size):
    """64-bit keys without values: leaves on both sides of the merge
    capacity (7680 keys)."""
    _say(f"u64 split leaves size={size}")
    x = _clusters(size, seed=size + 1)
    got, dg, used = gpu_u64(b, ws, x, seed=3, cutoff=0, digest=True)
    assert np.array_equal(got, np.sort(x))
    _, wdg, _ = oracle.squaresort_u64(x, 3, used, want_digest=True)
    assert dg == wdg


def test_kv_presorted_stable(b, ws):
    n = 3_000_017
    _say(f"kv presorted n={n}")
    k = np.sort(datagen.uniform_u64(n, seed=8) >> np.uint64(40))     # sorted, with duplicates
    v = np.arange(n, dtype=np.uint32)
    ko, vo, dg, used = gpu_kv(b, ws, k, v, seed=1, cutoff=0, digest=True)
    assert np.array_equal(ko, k) and np.array_equal(vo, v)
    _, _, wdg, _ = oracle.squaresort_kv(k, v, 1, used, want_digest=True)
    assert dg == wdg


# ------------------------------------------------------------------ determinism
def test_repeat_runs_identical(b, ws):
    x = datagen.uniform_u32(2_000_003, seed=2)
    a, da, _ = gpu_u32(b, ws, x, seed=5, cutoff=0, digest=True)
    c, dc, _ = gpu_u32(b, ws, x, seed=5, cutoff=0, digest=True)
    d, dd, _ = gpu_u32(b, ws, x, seed=6, cutoff=0, digest=True)
    assert np.array_equal(a, c) and da == dc
    assert np.array_equal(a, d) and da != dd
