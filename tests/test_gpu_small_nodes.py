"""Nodes sorted on chip with their whole subtree (k_small_nodes: 32-bit keys,
at most 4096 keys, columns that are base cases): output and recursion-tree
digest against the oracle at the same seed and cut-off, for roots that are
such nodes, for column and bucket children that are, and for inputs whose
buckets are degenerate (runs of equal pivots, single values, sorted runs)."""
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


def _run(b, ws, x, seed, cutoff):
    inp = torch.from_numpy(x.view(np.int32)).to(DEV)
    out = torch.empty_like(inp)
    dg = torch.zeros(1, dtype=torch.int64, device=DEV)
    used = b.squaresort_u32(inp, out, seed=seed, cutoff=cutoff, ws=ws, digest=dg)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32), int(dg.cpu().numpy().view(np.uint64)[0]), used


# (n, cutoff): the root itself on chip (ceil sqrt n <= cutoff, n <= 4096);
# columns on chip below a batch root; buckets on chip; tiny cut-offs (deep
# on-chip trees); the largest on-chip node (4096 keys, m = 64)
CASES = [(65, 64), (1000, 32), (4000, 64), (4096, 64), (4097, 64), (20_000, 64), (300_001, 64),
         (1 << 20, 64), (5000, 8), (50_000, 16), (2000, 4), (100_003, 4), (4096, 4096), (70_000, 300)]


@pytest.mark.parametrize("n,cutoff", CASES)
def test_small_nodes_match_oracle(b, ws, n, cutoff):
    print(f"small nodes u32 n={n} cutoff={cutoff}", flush=True)
    x = datagen.uniform_u32(n, seed=n % 97 + 1)
    got, gdg, used = _run(b, ws, x, seed=5, cutoff=cutoff)
    want, wdg, nodes = oracle.squaresort_u32(x, 5, used, want_digest=True)
    assert used == cutoff
    assert np.array_equal(got, want)
    assert gdg == wdg


def _degenerate(n):
    g = np.random.default_rng(n)
    return {
        "all_equal": np.full(n, 77, np.uint32),
        "two_values": np.where(g.random(n) < 0.5, 3, 4).astype(np.uint32),
        "extremes": np.where(g.random(n) < 0.5, 0, 2**32 - 1).astype(np.uint32),
        "sorted": np.arange(n, dtype=np.uint32),
        "reversed": np.arange(n, dtype=np.uint32)[::-1].copy(),
        "few_values": g.integers(0, 9, size=n, dtype=np.uint64).astype(np.uint32),
        "dup8": datagen.uniform_u32(n, seed=3, hi=1 << 8),
    }


@pytest.mark.parametrize("name", ["all_equal", "two_values", "extremes", "sorted", "reversed", "few_values",
                                  "dup8"])
@pytest.mark.parametrize("n,cutoff", [(3000, 64), (40_000, 16), (200_000, 64)])
def test_small_nodes_degenerate(b, ws, n, cutoff, name):
    print(f"small nodes degenerate {name} n={n} cutoff={cutoff}", flush=True)
    x = _degenerate(n)[name]
    got, gdg, used = _run(b, ws, x, seed=2, cutoff=cutoff)
    want, wdg, _ = oracle.squaresort_u32(x, 2, used, want_digest=True)
    assert np.array_equal(got, want)
    assert gdg == wdg
