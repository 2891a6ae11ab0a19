"""Served form on the GPU: every request's result is the same alone and in
the mix (same seed, so bit-identical), and equal to the oracle's SquareSort
of its input (same seed and cut-off)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2407_14801_amd import datagen

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _requests(count, seed):
    from paper_2407_14801_amd.serve import Request
    specs = datagen.serve_requests(count, seed, lo=1 << 6, hi=1 << 18)
    reqs = []
    for s in specs:
        if s["kind"] == "u32":
            k = torch.from_numpy(s["keys"].view(np.int32)).to(DEV)
            v = None
        else:
            k = torch.from_numpy(s["keys"].view(np.int64)).to(DEV)
            v = torch.from_numpy(s["vals"].view(np.int32)).to(DEV)
        reqs.append(Request(id=s["id"], kind=s["kind"], n=s["n"], seed=s["seed"], keys=k, vals=v))
    return specs, reqs


def test_served_results_identical_alone_and_in_the_mix():
    assert torch.cuda.is_available()
    from paper_2407_14801_amd.serve import GpuExecutor, PlainExecutor, Request, Server, replay
    print("served: 48 mixed requests", flush=True)
    specs, reqs = _requests(48, seed=21)
    srv = Server(GpuExecutor(DEV)).start()
    # a burst: every request after the first arrives within 0.5 ms, while
    # the first batch is still on the device (each batch takes longer than
    # the gap between arrivals), so later ones join shared batches
    replay(srv, reqs, [0.0] + [0.002 + 0.00001 * i for i in range(len(reqs) - 1)])
    srv.drain(len(reqs))
    assert len({r.batch for r in reqs}) < len(reqs)                # some requests shared a batch
    alone = PlainExecutor(DEV)
    from paper_2407_14801_amd import binding
    for s, r in zip(specs, reqs):
        a = Request(id=r.id, kind=r.kind, n=r.n, seed=r.seed, keys=r.keys, vals=r.vals)
        alone(a.kind, [a])
        assert torch.equal(a.out_keys, r.out_keys), f"request {r.id}"
        if r.kind == "u32":
            want = oracle.squaresort_u32(s["keys"], r.seed, binding.max_cutoff(binding.KIND_U32))
            assert np.array_equal(r.out_keys.cpu().numpy().view(np.uint32), want), f"request {r.id}"
        else:
            assert torch.equal(a.out_vals, r.out_vals), f"request {r.id}"
            wk, wv = oracle.squaresort_kv(s["keys"], s["vals"], r.seed, binding.max_cutoff(binding.KIND_KV))
            assert np.array_equal(r.out_keys.cpu().numpy().view(np.uint64), wk), f"request {r.id}"
            assert np.array_equal(r.out_vals.cpu().numpy().view(np.uint32), wv), f"request {r.id}"
