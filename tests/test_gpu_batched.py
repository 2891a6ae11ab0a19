"""GPU parity of the batched form: many independent instances in one call.

Every instance must end exactly as a sort of that range alone would leave it
(numpy's sort, the oracle, and the single-instance entry point with the same
seed), and the digest of the batch must be the sum of the instances' oracle
digests (the same recursion trees).
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


def _batched(b, ws, keys, sizes, seeds, cutoff, digest=False, tile=0):
    offs = b.batched_offsets(sizes)
    inp = torch.from_numpy(keys.view(np.int32)).to(DEV)
    out = torch.empty_like(inp)
    dg = torch.zeros(1, dtype=torch.int64, device=DEV) if digest else None
    used = b.squaresort_batched_u32(inp, out, offs, seeds, cutoff=cutoff, ws=ws, digest=dg, tile=tile)
    torch.cuda.synchronize()
    res = out.cpu().numpy().view(np.uint32)
    d = int(dg.cpu().numpy().view(np.uint64)[0]) if digest else None
    return res, offs, used, d


def _single(b, ws, x, seed, cutoff):
    inp = torch.from_numpy(np.ascontiguousarray(x, np.uint32).view(np.int32)).to(DEV)
    out = torch.empty_like(inp)
    if x.size:
        b.squaresort_u32(inp, out, seed=seed, cutoff=cutoff, ws=ws)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


# every class of instance: empty, single key, wave sorts, work-group sorts,
# MSD-split base cases, internal roots, and sizes on each class boundary
MIXED = [0, 1, 2, 3, 64, 65, 1000, 1024, 1025, 5000, 16384, 16385, 50_000, 131_072, 131_073,
         300_000, 0, 7, 1_000_003, 4097]


@pytest.mark.parametrize("cutoff", [0, 4096])
def test_batched_mixed_classes(b, ws, cutoff):
    _say(f"batched mixed cutoff={cutoff}")
    sizes = np.array(MIXED, dtype=np.int64)
    keys = datagen.uniform_u32(int(sizes.sum()), seed=11)
    seeds = np.arange(len(sizes), dtype=np.uint64) * 7919 + 3
    got, offs, used, _ = _batched(b, ws, keys, sizes, seeds, cutoff)
    for i in range(len(sizes)):
        lo, hi = int(offs[i]), int(offs[i + 1])
        assert np.array_equal(got[lo:hi], np.sort(keys[lo:hi])), f"instance {i} (n={hi - lo})"
        assert np.array_equal(got[lo:hi], _single(b, ws, keys[lo:hi], int(seeds[i]), used)), f"instance {i}"


def test_batched_degenerate_instances(b, ws):
    _say("batched degenerate")
    parts = [np.full(70_000, 5, np.uint32), np.zeros(1, np.uint32), np.arange(200_000, dtype=np.uint32)[::-1].copy(),
             datagen.uniform_u32(150_000, seed=2, hi=16), np.array([3, 1, 2], np.uint32),
             np.where(np.arange(40_000) % 2 == 0, 0, 2**32 - 1).astype(np.uint32)]
    sizes = np.array([p.size for p in parts])
    keys = np.concatenate(parts)
    seeds = np.array([5, 6, 7, 8, 9, 10], dtype=np.uint64)
    got, offs, used, _ = _batched(b, ws, keys, sizes, seeds, 0)
    for i in range(len(parts)):
        lo, hi = int(offs[i]), int(offs[i + 1])
        assert np.array_equal(got[lo:hi], np.sort(keys[lo:hi])), f"instance {i}"


def test_batched_digest_is_sum_of_instance_trees(b, ws):
    """Fully recursive configuration (cut-off 64): the batch's digest equals
    the sum of the oracle's per-instance digests, and each output equals the
    oracle's."""
    _say("batched digest cutoff=64")
    sizes = datagen.log_uniform_sizes(40, 10, 30_000, seed=4)
    sizes[3] = 0
    keys = datagen.uniform_u32(int(sizes.sum()), seed=12)
    seeds = np.arange(1, len(sizes) + 1, dtype=np.uint64) * 1000003
    got, offs, used, dg = _batched(b, ws, keys, sizes, seeds, 64, digest=True)
    want = 0
    for i in range(len(sizes)):
        lo, hi = int(offs[i]), int(offs[i + 1])
        if hi == lo:
            continue
        w, wd, _ = oracle.squaresort_u32(keys[lo:hi], int(seeds[i]), used, want_digest=True)
        assert np.array_equal(got[lo:hi], w), f"instance {i}"
        want = (want + wd) & 0xFFFFFFFFFFFFFFFF
    assert dg == want


# tile words: each field off its default, and all three together
TILES = [dict(colw=2), dict(colw=8), dict(wcap=256), dict(wcap=512, m4cap=1024), dict(m4cap=2048),
         dict(colw=8, wcap=256, m4cap=1024)]


@pytest.mark.parametrize("fields", TILES, ids=lambda f: "-".join(f"{k}{v}" for k, v in f.items()))
def test_batched_tile_shapes_same_trees(b, ws, fields):
    """Every tile choice leaves each instance as the oracle does and adds
    the same digest (the tile word changes kernels and size classes, not the
    recursion tree): cut-off 64 runs every level through the wave-level
    column kernel, cut-off 0 puts buckets on every class boundary."""
    tile = b.tile_word(**fields)
    _say(f"batched tile {fields} word={tile}")
    sizes = np.array([0, 1, 200, 256, 257, 512, 513, 1024, 1025, 2048, 2049, 4096, 4097, 9000, 30_000, 70_000],
                     dtype=np.int64)
    keys = datagen.uniform_u32(int(sizes.sum()), seed=21)
    seeds = np.arange(1, len(sizes) + 1, dtype=np.uint64) * 7919
    got, offs, used, dg = _batched(b, ws, keys, sizes, seeds, 64, digest=True, tile=tile)
    want = 0
    for i in range(len(sizes)):
        lo, hi = int(offs[i]), int(offs[i + 1])
        if hi == lo:
            continue
        w, wd, _ = oracle.squaresort_u32(keys[lo:hi], int(seeds[i]), used, want_digest=True)
        assert np.array_equal(got[lo:hi], w), f"instance {i}"
        want = (want + wd) & 0xFFFFFFFFFFFFFFFF
    assert dg == want
    # automatic cut-off: base-case instances and buckets of every class
    sizes = datagen.log_uniform_sizes(300, 1 << 8, 1 << 18, seed=22)
    keys = datagen.uniform_u32(int(sizes.sum()), seed=23)
    seeds = np.arange(len(sizes), dtype=np.uint64) + 5
    got, offs, used, _ = _batched(b, ws, keys, sizes, seeds, 0, tile=tile)
    for i in range(len(sizes)):
        lo, hi = int(offs[i]), int(offs[i + 1])
        assert np.array_equal(got[lo:hi], np.sort(keys[lo:hi])), f"instance {i}"


def test_batched_log_uniform_workload(b, ws):
    """The batched workload's shape at reduced count: log-uniform sizes in
    [2^10, 2^20], uniform keys, automatic cut-off."""
    _say("batched log-uniform 512 instances")
    sizes = datagen.log_uniform_sizes(512, 1 << 10, 1 << 20, seed=7)
    keys = datagen.uniform_u32(int(sizes.sum()), seed=13)
    seeds = np.arange(len(sizes), dtype=np.uint64) + 1
    got, offs, used, _ = _batched(b, ws, keys, sizes, seeds, 0)
    for i in range(len(sizes)):
        lo, hi = int(offs[i]), int(offs[i + 1])
        assert np.array_equal(got[lo:hi], np.sort(keys[lo:hi])), f"instance {i}"


def _batched_kv(b, ws, k, v, sizes, seeds, cutoff, digest=False, tile=0):
    offs = b.batched_offsets(sizes)
    ki = torch.from_numpy(np.ascontiguousarray(k, np.uint64).view(np.int64)).to(DEV)
    vi = torch.from_numpy(np.ascontiguousarray(v, np.uint32).view(np.int32)).to(DEV)
    ko, vo = torch.empty_like(ki), torch.empty_like(vi)
    dg = torch.zeros(1, dtype=torch.int64, device=DEV) if digest else None
    used = b.squaresort_batched_kv(ki, vi, ko, vo, offs, seeds, cutoff=cutoff, ws=ws, digest=dg, tile=tile)
    torch.cuda.synchronize()
    d = int(dg.cpu().numpy().view(np.uint64)[0]) if digest else None
    return ko.cpu().numpy().view(np.uint64), vo.cpu().numpy().view(np.uint32), offs, used, d


@pytest.mark.parametrize("cutoff", [0, 4096])
def test_batched_kv_mixed_classes(b, ws, cutoff):
    """Key/value instances of every class (base cases split over the grid
    among them): each one is the stable sort of its range."""
    _say(f"batched kv mixed cutoff={cutoff}")
    sizes = np.array(MIXED, dtype=np.int64)
    k, _ = datagen.kv_mixture(int(sizes.sum()), seed=21)
    v = np.arange(k.size, dtype=np.uint32)
    seeds = np.arange(len(sizes), dtype=np.uint64) * 31 + 7
    gk, gv, offs, used, _ = _batched_kv(b, ws, k, v, sizes, seeds, cutoff)
    for i in range(len(sizes)):
        lo, hi = int(offs[i]), int(offs[i + 1])
        order = np.argsort(k[lo:hi], kind="stable")
        assert np.array_equal(gk[lo:hi], k[lo:hi][order]), f"instance {i} (n={hi - lo})"
        assert np.array_equal(gv[lo:hi], v[lo:hi][order]), f"instance {i} (n={hi - lo})"


@pytest.mark.parametrize("fields", [{}, dict(colw=2, wcap=256, m4cap=1024), dict(colw=8, wcap=512)],
                         ids=["default", "colw2-wcap256-m4cap1024", "colw8-wcap512"])
def test_batched_kv_digest_is_sum_of_instance_trees(b, ws, fields):
    _say(f"batched kv digest cutoff=64 tile {fields}")
    sizes = datagen.log_uniform_sizes(24, 10, 20_000, seed=9)
    k, _ = datagen.kv_mixture(int(sizes.sum()), seed=22)
    v = np.arange(k.size, dtype=np.uint32)
    seeds = np.arange(1, len(sizes) + 1, dtype=np.uint64) * 7777
    gk, gv, offs, used, dg = _batched_kv(b, ws, k, v, sizes, seeds, 64, digest=True, tile=b.tile_word(**fields))
    want = 0
    for i in range(len(sizes)):
        lo, hi = int(offs[i]), int(offs[i + 1])
        wk, wv, wd, _ = oracle.squaresort_kv(k[lo:hi], v[lo:hi], int(seeds[i]), used, want_digest=True)
        assert np.array_equal(gk[lo:hi], wk) and np.array_equal(gv[lo:hi], wv), f"instance {i}"
        want = (want + wd) & 0xFFFFFFFFFFFFFFFF
    assert dg == want


def test_batched_many_large_base_cases(b, ws):
    """More large base-case instances than the grid-wide split takes: each
    is sorted by one work-group of the MSD-split kernel."""
    _say("batched 300 large base cases")
    sizes = np.random.default_rng(3).integers(16_385, 60_000, size=300)
    keys = datagen.uniform_u32(int(sizes.sum()), seed=14)
    seeds = np.arange(len(sizes), dtype=np.uint64) + 11
    got, offs, used, _ = _batched(b, ws, keys, sizes, seeds, 0)
    assert used >= int(sizes.max())
    for i in range(len(sizes)):
        lo, hi = int(offs[i]), int(offs[i + 1])
        assert np.array_equal(got[lo:hi], np.sort(keys[lo:hi])), f"instance {i}"
