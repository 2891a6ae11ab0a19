"""SQS_FLAG_HOST_ARRAYS: the arrays stay in pinned host memory and the GPU
sorts them there (device memory holds the workspace only): output and
recursion-tree digest against the oracle, as for device arrays."""
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


def _pinned(x):
    t = torch.from_numpy(x).pin_memory()
    assert t.is_pinned()
    return t


@pytest.mark.parametrize("n,cutoff,hi", [(1000, 0, None), ((1 << 20) + 7, 64, None), (1 << 22, 0, None),
                                         (3_000_017, 0, 1 << 16), (300_001, 4096, None)])
def test_host_arrays_u32_match_oracle(b, ws, n, cutoff, hi):
    print(f"host arrays u32 n={n} cutoff={cutoff} hi={hi}", flush=True)
    x = datagen.uniform_u32(n, seed=n % 31 + 1, hi=hi) if hi else datagen.uniform_u32(n, seed=n % 31 + 1)
    inp = _pinned(x.view(np.int32).copy())
    out = _pinned(np.zeros(n, np.int32))
    dg = torch.zeros(1, dtype=torch.int64, device=DEV)
    used = b.squaresort_u32(inp, out, seed=3, cutoff=cutoff, ws=ws, digest=dg, host_arrays=True)
    torch.cuda.synchronize()
    want, wdg, _ = oracle.squaresort_u32(x, 3, used, want_digest=True)
    assert np.array_equal(out.numpy().view(np.uint32), want)
    assert int(dg.cpu().numpy().view(np.uint64)[0]) == wdg


def test_host_arrays_kv_match_oracle(b, ws):
    n = (1 << 20) + 3
    print(f"host arrays kv n={n}", flush=True)
    k, v = datagen.kv_mixture(n, seed=4)
    ki, vi = _pinned(k.view(np.int64).copy()), _pinned(v.view(np.int32).copy())
    ko, vo = _pinned(np.zeros(n, np.int64)), _pinned(np.zeros(n, np.int32))
    dg = torch.zeros(1, dtype=torch.int64, device=DEV)
    used = b.squaresort_kv(ki, vi, ko, vo, seed=2, ws=ws, digest=dg, host_arrays=True)
    torch.cuda.synchronize()
    wk, wv, wdg, _ = oracle.squaresort_kv(k, v, 2, used, want_digest=True)
    assert np.array_equal(ko.numpy().view(np.uint64), wk)
    assert np.array_equal(vo.numpy().view(np.uint32), wv)
    assert int(dg.cpu().numpy().view(np.uint64)[0]) == wdg


def test_host_arrays_reject_unpinned_memory(b, ws):
    """A pageable host buffer is not device-accessible: refused before any
    GPU work."""
    import ctypes
    x = np.arange(100, dtype=np.int32)
    y = np.zeros(100, dtype=np.int32)
    p = b.Params()
    p.flags = b.FLAG_HOST_ARRAYS
    rc = b.lib.squaresort_u32(100, x.ctypes.data, y.ctypes.data, 1, ctypes.byref(p), None)
    assert rc == -1
