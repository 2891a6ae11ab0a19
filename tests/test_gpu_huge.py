"""Nodes whose columns do not fit one LDS sort (m > 16384, n > 2^28): the
columns are sorted into D through HBM (base-case kernels or recursion) and
the bucket counts are taken from the sorted columns in HBM.  Checked against
numpy's sort, the stable-sort identities, and (once) the oracle's output and
recursion-tree digest."""
import numpy as np
import pytest
import torch

import oracle
from paper_2407_14801_amd import datagen

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
N_HUGE = (1 << 28) + 12_345            # m = 16385 columns


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


@pytest.fixture(scope="module")
def keys():
    return datagen.uniform_u32(N_HUGE, seed=31)


def _sort(b, ws, x, seed, cutoff, digest=False):
    inp = torch.from_numpy(x.view(np.int32)).to(DEV)
    out = torch.empty_like(inp)
    dg = torch.zeros(1, dtype=torch.int64, device=DEV) if digest else None
    used = b.squaresort_u32(inp, out, seed=seed, cutoff=cutoff, ws=ws, digest=dg)
    torch.cuda.synchronize()
    del inp
    res = out.cpu().numpy().view(np.uint32)
    return res, used, (int(dg.cpu().numpy().view(np.uint64)[0]) if digest else None)


@pytest.mark.parametrize("cutoff", [0, 4096])
def test_huge_u32_sorted(b, ws, keys, cutoff):
    """cut-off 0: columns of 16385 keys are MSD-split base cases; 4096: they
    are internal nodes of their own."""
    _say(f"huge u32 n={N_HUGE} cutoff={cutoff}")
    got, used, _ = _sort(b, ws, keys, 2, cutoff)
    assert np.array_equal(got, np.sort(keys))


def test_huge_u32_digest_matches_oracle(b, ws, keys):
    _say(f"huge u32 digest n={N_HUGE} (oracle run takes about a minute)")
    got, used, dg = _sort(b, ws, keys, 3, 0, digest=True)
    want, wdg, nodes = oracle.squaresort_u32(keys, 3, used, want_digest=True)
    assert np.array_equal(got, want)
    assert dg == wdg, f"{nodes} internal nodes"


def test_huge_kv_stable(b, ws):
    n = (1 << 28) + 999
    _say(f"huge kv n={n}")
    k, v = datagen.kv_mixture(n, seed=8)
    ki = torch.from_numpy(k.view(np.int64)).to(DEV)
    vi = torch.from_numpy(v.view(np.int32)).to(DEV)
    ko, vo = torch.empty_like(ki), torch.empty_like(vi)
    b.squaresort_kv(ki, vi, ko, vo, seed=1, cutoff=0, ws=ws)
    torch.cuda.synchronize()
    del ki, vi
    gk = ko.cpu().numpy().view(np.uint64)
    gv = vo.cpu().numpy().view(np.uint32)
    del ko, vo
    assert np.array_equal(np.bincount(gv, minlength=n), np.ones(n, np.int64))
    assert np.array_equal(gk, k[gv])
    assert np.all(gk[1:] >= gk[:-1])
    eq = gk[1:] == gk[:-1]
    assert np.all(gv[1:][eq] > gv[:-1][eq])


def test_huge_limits(b, ws):
    """The skew entry point and the Alg. 1 pivot rule keep columns within one
    LDS sort and report larger n as unsupported."""
    x = torch.zeros(N_HUGE, dtype=torch.int32, device=DEV)
    out = torch.empty_like(x)
    with pytest.raises(b.SquareSortError) as e:
        b.skew_transpose_u32(x, out, None, seed=1, ws=ws)
    assert e.value.status == -7
    with pytest.raises(b.SquareSortError) as e:
        b.squaresort_u32(x, out, seed=1, cutoff=0, ws=ws, pivot_rule="alg1")
    assert e.value.status == -7
