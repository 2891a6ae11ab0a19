"""The batched form as a planned graph (squaresort_batched_graph_u32 +
sqs_plan_launch): every replay, with eager work and synchronisations between
replays, gives the bytes and digest of the eager batched call and of the
oracle; internal buckets are finished on chip; a bucket beyond on-chip
capacity is reported through the status word."""
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


def _instances(count, lo, hi, seed):
    sizes = datagen.log_uniform_sizes(count, lo, hi, seed=seed)
    keys = datagen.uniform_u32(int(sizes.sum()), seed=seed + 100)
    return sizes, keys


# the last case: roots of 2^24..2^25 keys, whose largest buckets (16K..60K
# keys) go to the wide-bucket and MSD-split kernels, which mark the list
# entries they sorted; every replay rebuilds the lists on the device
@pytest.mark.parametrize("count,lo,hi,cutoff", [(300, 1 << 6, 1 << 18, 0), (200, 1 << 8, 1 << 16, 64),
                                                (32, 1 << 16, 1 << 20, 0), (40, 3, 30, 4), (50, 100, 600, 16),
                                                (2, 1 << 24, 1 << 25, 0)])
def test_graph_replays_match_eager_and_oracle(b, count, lo, hi, cutoff):
    print(f"graph count={count} sizes=[{lo},{hi}] cutoff={cutoff}", flush=True)
    sizes, keys = _instances(count, lo, hi, seed=count + lo)
    offs = b.batched_offsets(sizes)
    seeds = np.arange(11, 11 + count, dtype=np.uint64)
    base = torch.from_numpy(keys.view(np.int32)).to(DEV)
    # eager batched call
    ein, eout = base.clone(), torch.empty_like(base)
    edg = torch.zeros(1, dtype=torch.int64, device=DEV)
    used = b.squaresort_batched_u32(ein, eout, offs, seeds, cutoff=cutoff, digest=edg)
    torch.cuda.synchronize()
    want = eout.cpu().numpy().view(np.uint32)
    wdg = int(edg.cpu().numpy().view(np.uint64)[0])
    # oracle digest: the sum of the instances'
    odg = 0
    for i in range(count):
        x = keys[int(offs[i]):int(offs[i + 1])]
        if x.size == 0:
            continue
        _, d, _ = oracle.squaresort_u32(x, int(seeds[i]), used, want_digest=True)
        odg = (odg + d) % (1 << 64)
    assert wdg == odg
    # planned graph, replayed several times on fresh copies of the input
    gin, gout = torch.empty_like(base), torch.empty_like(base)
    gdg = torch.zeros(1, dtype=torch.int64, device=DEV)
    plan = b.BatchedGraph(gin, gout, offs, seeds, cutoff=cutoff, digest=gdg)
    assert plan.cutoff == used
    for rep in range(3):
        gin.copy_(base)
        gout.fill_(-1)
        gdg.zero_()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        assert int(plan.status.item()) == 0, rep
        assert np.array_equal(gout.cpu().numpy().view(np.uint32), want), rep
        assert int(gdg.cpu().numpy().view(np.uint64)[0]) == wdg, rep
        _ = (base.float() * 2).sum().item()         # eager work between replays
    plan.close()


def test_graph_reports_unfinished_buckets(b):
    """Buckets of more than 4096 keys that are internal (n = 2^24 at cut-off
    4096) cannot be finished without a host step: the status word says so."""
    n = 1 << 24
    keys = datagen.uniform_u32(n, seed=5)
    offs = np.array([0, n], dtype=np.uint64)
    seeds = np.array([1], dtype=np.uint64)
    base = torch.from_numpy(keys.view(np.int32)).to(DEV)
    gin, gout = base.clone(), torch.empty_like(base)
    plan = b.BatchedGraph(gin, gout, offs, seeds, cutoff=4096)
    plan.launch()
    torch.cuda.synchronize()
    assert int(plan.status.item()) & b.STATUS_UNFINISHED
    plan.close()


def test_graph_argument_errors(b):
    x = torch.zeros(16, dtype=torch.int32, device=DEV)
    with pytest.raises(b.SquareSortError):
        b.BatchedGraph(x, x, np.array([0, 16], dtype=np.uint64), np.array([1], dtype=np.uint64))
