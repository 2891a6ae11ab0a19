"""squaresort_u32_noalloc (scratch in the library's static per-GPU array)
against squaresort_u32 (caller workspace): same output and recursion-tree
digest, on two calls in a row, the second with a smaller input, and the
smaller one against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _run(fn, x, dev, **kw):
    import torch
    inp = torch.from_numpy(x.view(np.int32)).to(dev)
    out = torch.empty_like(inp)
    dg = torch.zeros(1, dtype=torch.int64, device=dev)
    used = fn(inp, out, digest=dg, **kw)
    torch.cuda.synchronize(dev)
    return out.cpu().numpy().view(np.uint32), int(dg.cpu().numpy().view(np.uint64)[0]), used


@pytest.mark.parametrize("first,second", [
    ((1 << 24, 0, 3), (100_003, 64, 5)),           # automatic cut-off, then the fully recursive form
    ((3_000_017, 4096, 7), (20_000, 0, 9)),         # a deeper tree, then one base-case work-group
])
def test_noalloc_matches_workspace_entry(first, second, orc):
    import torch
    from paper_2407_14801_amd import binding, datagen
    dev = torch.device("cuda:0")
    ws = binding.Workspace(dev)
    for (n, cutoff, seed) in (first, second):
        print(f"noalloc n={n} cutoff={cutoff} seed={seed}", flush=True)
        x = datagen.uniform_u32(n, seed=seed)
        got, gdg, gc = _run(binding.squaresort_u32_noalloc, x, dev, seed=seed, cutoff=cutoff)
        want, wdg, wc = _run(binding.squaresort_u32, x, dev, seed=seed, cutoff=cutoff, ws=ws)
        assert gc == wc
        assert np.array_equal(got, want)
        assert gdg == wdg
        assert np.array_equal(got, np.sort(x))
    # the second (smaller) call against the oracle's tree
    n, cutoff, seed = second
    x = datagen.uniform_u32(n, seed=seed)
    _, odg, _ = orc.squaresort_u32(x, seed, gc, want_digest=True)
    assert gdg == odg


def test_noalloc_validate_and_size_limit():
    import torch
    from paper_2407_14801_amd import binding, datagen
    dev = torch.device("cuda:0")
    x = datagen.uniform_u32(1_000_003, seed=11)
    inp = torch.from_numpy(x.view(np.int32)).to(dev)
    out = torch.empty_like(inp)
    binding.squaresort_u32_noalloc(inp, out, seed=2, validate=True)
    torch.cuda.synchronize(dev)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), np.sort(x))
    # more scratch than the static array holds: refused before any GPU work
    with pytest.raises(binding.SquareSortError) as e:
        binding.squaresort_u32_noalloc(inp, out, seed=2, cutoff=64)
    assert e.value.status == -3
