"""GPU parity at the full benchmark sizes, in the launch configuration that
bench.py times (automatic cut-off, one call per sort), against the oracle.

Each check is whole and bit-exact: the sorted output and the recursion-tree
digest of a sort (same seed and cut-off), the whole root SkewTranspose
intermediate and its bucket bounds (same seed).  The oracle spreads the
root's children over host threads (the bytes do not depend on it).
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2407_14801_amd import datagen

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
N28 = 1 << 28
N27 = 1 << 27
THREADS = max(1, min(16, int(os.environ.get("OMP_NUM_THREADS", "8"))))


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


def _input(hi, data_seed):
    return datagen.uniform_u32(N28, seed=data_seed, hi=hi) if hi else datagen.uniform_u32(N28, seed=data_seed)


@pytest.mark.parametrize("name,hi,data_seed", [("uniform", None, 2), ("dup16", 1 << 16, 3)])
def test_u32_full_size_matches_oracle(b, ws, name, hi, data_seed):
    """n = 2^28 u32 (uniform over [0, 2^32) and over [0, 2^16)): output and
    recursion-tree digest equal the oracle's at the same seed and cut-off."""
    _say(f"u32 {name} n=2^28 data_seed={data_seed} seed=1 auto cut-off")
    x = _input(hi, data_seed)
    inp = torch.from_numpy(x.view(np.int32)).to(DEV)
    out = torch.empty_like(inp)
    dg = torch.zeros(1, dtype=torch.int64, device=DEV)
    used = b.squaresort_u32(inp, out, seed=1, cutoff=0, ws=ws, digest=dg)
    torch.cuda.synchronize()
    del inp
    got = out.cpu().numpy().view(np.uint32)
    gdg = int(dg.cpu().numpy().view(np.uint64)[0])
    del out
    assert used == b.max_cutoff(b.KIND_U32)
    _say(f"  oracle on {THREADS} threads")
    with oracle.threads(THREADS):
        want, wdg, nodes = oracle.squaresort_u32(x, 1, used, want_digest=True)
    assert nodes >= 1
    assert np.array_equal(got, want)
    assert gdg == wdg


@pytest.mark.parametrize("name,hi,data_seed", [("uniform", None, 2), ("dup16", 1 << 16, 3)])
def test_u32_full_size_root_intermediate(b, ws, name, hi, data_seed):
    """The whole root SkewTranspose intermediate at 2^28 and its bucket
    bounds, against the oracle's."""
    _say(f"skew {name} n=2^28 data_seed={data_seed} seed=1")
    x = _input(hi, data_seed)
    m = oracle.ceil_isqrt(N28)
    inp = torch.from_numpy(x.view(np.int32)).to(DEV)
    out = torch.empty_like(inp)
    bs = torch.empty(m + 1, dtype=torch.int64, device=DEV)
    b.skew_transpose_u32(inp, out, bs, seed=1, ws=ws)
    torch.cuda.synchronize()
    del inp
    got = out.cpu().numpy().view(np.uint32)
    starts = bs.cpu().numpy().view(np.uint64)
    del out
    _say(f"  oracle root intermediate on {THREADS} threads")
    with oracle.threads(THREADS):
        want, wbs = oracle.root_intermediate(x.astype(np.uint64), seed=1)
    assert np.array_equal(starts, wbs)
    assert np.array_equal(got.astype(np.uint64), want)


def test_kv_mixture_full_size(b, ws):
    """2^27 (u64 key, u32 index) pairs of the key/value mixture: keys, values
    and digest equal the oracle's (stable order by key, then index)."""
    _say("kv mixture n=2^27 data_seed=4 seed=1 auto cut-off")
    k, v = datagen.kv_mixture(N27, seed=4)
    ki = torch.from_numpy(k.view(np.int64)).to(DEV)
    vi = torch.from_numpy(v.view(np.int32)).to(DEV)
    ko, vo = torch.empty_like(ki), torch.empty_like(vi)
    dg = torch.zeros(1, dtype=torch.int64, device=DEV)
    used = b.squaresort_kv(ki, vi, ko, vo, seed=1, cutoff=0, ws=ws, digest=dg)
    torch.cuda.synchronize()
    del ki, vi
    gk = ko.cpu().numpy().view(np.uint64)
    gv = vo.cpu().numpy().view(np.uint32)
    gdg = int(dg.cpu().numpy().view(np.uint64)[0])
    del ko, vo
    assert used == b.max_cutoff(b.KIND_KV)
    _say(f"  oracle on {THREADS} threads")
    with oracle.threads(THREADS):
        wk, wv, wdg, _ = oracle.squaresort_kv(k, v, 1, used, want_digest=True)
    assert np.array_equal(gk, wk)
    assert np.array_equal(gv, wv)
    assert gdg == wdg


@pytest.mark.parametrize("m", [13312, 13313])
def test_kv_merge_column_capacity(b, ws, m):
    """Key/value roots whose columns are exactly the merge column sort's
    capacity (13312 pairs) and one more (taken by the radix column kernel):
    the output is the stable sort (checked on the device against torch's
    stable sort of the keys in unsigned order)."""
    n = m * m
    _say(f"kv merge column capacity m={m} n={n}")
    g = torch.Generator(device=DEV)
    g.manual_seed(m)
    k = torch.randint(-(1 << 63), (1 << 63) - 1, (n,), dtype=torch.int64, device=DEV, generator=g)
    k[: n // 3] = k[: n // 3] & 0xFFFF                 # a third of the keys in 2^16 values
    v = torch.arange(n, dtype=torch.int32, device=DEV)
    ki, vi = k.clone(), v.clone()
    ko, vo = torch.empty_like(k), torch.empty_like(v)
    b.squaresort_kv(ki, vi, ko, vo, seed=5, cutoff=0, ws=ws)
    flip = torch.tensor(-(1 << 63), dtype=torch.int64, device=DEV)
    ws_sorted, order = torch.sort(k ^ flip, stable=True)
    assert torch.equal(ko, ws_sorted ^ flip)
    assert torch.equal(vo, v[order])
    del ki, vi, ko, vo, ws_sorted, order
    torch.cuda.synchronize()
