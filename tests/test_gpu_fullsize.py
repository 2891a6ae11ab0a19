"""GPU parity at the full benchmark sizes, in the launch configuration that
bench.py times (automatic cut-off, one call per sort).

The whole output is checked against what fixes it uniquely (numpy's sort for
keys; for key/value pairs the gather identity below), and the root
SkewTranspose intermediate, which depends on the seed, is checked on sampled
buckets that the oracle computes one by one (oracle.root_buckets).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2407_14801_amd import datagen

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
N28 = 1 << 28
N27 = 1 << 27


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


def _sorted_u32(b, ws, x, seed):
    inp = torch.from_numpy(x.view(np.int32)).to(DEV)
    out = torch.empty_like(inp)
    used = b.squaresort_u32(inp, out, seed=seed, cutoff=0, ws=ws)
    torch.cuda.synchronize()
    del inp
    return out.cpu().numpy().view(np.uint32), used


def _sample_buckets(m, rng, extra=4):
    sel = {0, 1, m // 2, m - 2, m - 1}
    sel.update(int(v) for v in rng.integers(0, m, size=extra))
    return np.array(sorted(sel), dtype=np.uint64)


@pytest.mark.parametrize("name,hi,data_seed", [("uniform", None, 2), ("dup16", 1 << 16, 3)])
def test_u32_full_size_sorted(b, ws, name, hi, data_seed):
    _say(f"u32 {name} n=2^28 data_seed={data_seed}")
    x = datagen.uniform_u32(N28, seed=data_seed, hi=hi) if hi else datagen.uniform_u32(N28, seed=data_seed)
    got, used = _sorted_u32(b, ws, x, seed=1)
    assert used == b.max_cutoff(b.KIND_U32)
    assert np.array_equal(got, np.sort(x))


@pytest.mark.parametrize("name,hi,data_seed", [("uniform", None, 2), ("dup16", 1 << 16, 3)])
def test_u32_full_size_root_buckets_sampled(b, ws, name, hi, data_seed):
    """Root intermediate at 2^28 on sampled buckets, against the oracle."""
    _say(f"skew {name} n=2^28 sampled buckets")
    x = datagen.uniform_u32(N28, seed=data_seed, hi=hi) if hi else datagen.uniform_u32(N28, seed=data_seed)
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
    assert starts[0] == 0 and starts[m] == N28 and np.all(np.diff(starts.astype(np.int64)) >= 0)
    sel = _sample_buckets(m, np.random.default_rng(data_seed))
    _, bounds, keys = oracle.root_buckets(x.astype(np.uint64), 1, sel)
    at = 0
    for s, (lo, hi_) in zip(sel, bounds):
        lo, hi_ = int(lo), int(hi_)
        assert (int(starts[s]), int(starts[s + 1])) == (lo, hi_), f"bucket {s}"
        assert np.array_equal(got[lo:hi_].astype(np.uint64), keys[at:at + hi_ - lo]), f"bucket {s}"
        at += hi_ - lo


def test_kv_mixture_full_size(b, ws):
    """2^27 (u64 key, u32 index) pairs: the output is the stable sort.

    With v the output values and k the output keys: v is a permutation of
    0..n-1, k[i] = keys_in[v[i]], k is non-decreasing, and v increases within
    every run of equal keys; these properties hold only for the stable sort.
    """
    _say("kv mixture n=2^27")
    k, v = datagen.kv_mixture(N27, seed=4)
    assert np.array_equal(v, np.arange(N27, dtype=np.uint32))
    ki = torch.from_numpy(k.view(np.int64)).to(DEV)
    vi = torch.from_numpy(v.view(np.int32)).to(DEV)
    ko, vo = torch.empty_like(ki), torch.empty_like(vi)
    used = b.squaresort_kv(ki, vi, ko, vo, seed=1, cutoff=0, ws=ws)
    torch.cuda.synchronize()
    del ki, vi
    gk = ko.cpu().numpy().view(np.uint64)
    gv = vo.cpu().numpy().view(np.uint32)
    del ko, vo
    assert used == b.max_cutoff(b.KIND_KV)
    assert np.array_equal(np.bincount(gv, minlength=N27), np.ones(N27, np.int64))
    assert np.array_equal(gk, k[gv])
    assert np.all(gk[1:] >= gk[:-1])
    eq = gk[1:] == gk[:-1]
    assert np.all(gv[1:][eq] > gv[:-1][eq])
