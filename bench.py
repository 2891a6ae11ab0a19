#!/usr/bin/env python3
"""Benchmark of libsquaresort on one MI355X.

Default workload: SquareSort of n = 2^28 uint32 keys drawn i.i.d. uniform over
[0, 2^32) (data seed 2, pivot seed 1, automatic cut-off).  One step is one
full sort (every recursion level) of one resident copy of the input; the
input is clobbered by a sort, so W+K copies are staged in HBM before the
timed region.  Prints one JSON line.

  value        whole-job throughput, keys sorted per second (GKeys/s)
  roofline     the dominant kernel (largest share of device time) against the
               HBM peak: its algorithmic bytes (read + write of every key it
               processes) over its measured duration (HIP events on the launch
               stream, from the library's timing table)
  path_roofline  the whole step against the HBM roofline of the method:
               6 * w * n algorithmic bytes per HBM-resident level
  cpu_baseline the CPU oracle on a bounded sample of the same input
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sqlite3
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "u32_uniform": dict(kind="u32", log2n=28, dist="uniform[0,2^32)", data_seed=2),
    "u32_dup16": dict(kind="u32", log2n=28, dist="uniform[0,2^16)", data_seed=3),
    # the fully recursive configuration: every level of the tree runs (cut-off 64)
    "u32_recursive": dict(kind="u32", log2n=20, dist="uniform[0,2^32)", data_seed=1, cutoff=64),
    "kv_mixture": dict(kind="kv", log2n=27, dist="80% Zipf(1.1) over 2^20 u64 / 10% constant / "
                                                  "10% sorted run with 1% swaps", data_seed=4),
    # many independent instances in one call, against one call per instance
    "batched_u32": dict(kind="batched", count=4096, lo=1 << 10, hi=1 << 20, dist="uniform[0,2^32)",
                        data_seed=5),
    # Poisson request stream served with admission and continuous batching
    "served": dict(kind="served", lo=1 << 12, hi=1 << 24, data_seed=6, budget_gb=64),
    # the arrays in pinned host memory (SQS_FLAG_HOST_ARRAYS): sorted over the host link
    "u32_host": dict(kind="host", log2n=28, dist="uniform[0,2^32)", data_seed=2),
    # distinct keys under the Alg. 1 pivot rule, against the default rule
    "u32_perm_alg1": dict(kind="alg1", log2n=28, dist="permutation of 0..n-1 times an odd constant", data_seed=8),
}


# timing-table names of the library -> kernel symbols in rocprofv3 traces
KERNEL_SYMBOL = {"k_colsort": "k_colsort_big", "k_bucket_big": "k_bucket_big", "k_transpose": "k_transpose",
                 "k_bucket": "k_bucket_mid", "k_colsort_w": "k_colsort_small", "k_bucket_w": "k_bucket_small"}
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")


def source_hash():
    """Hash of the HIP sources: traffic counters are valid only for them."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2407_14801_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + fh.read())
    return h.hexdigest()[:16]


def _pmc_rows(db, counter):
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, grid_size, value from counters_collection "
                       "where counter_name = ?", (counter,)).fetchall()
    con.close()
    per = {}
    for d, k, g, v in rows:             # values may be split per shader engine / XCD: sum them
        e = per.setdefault(d, [k, g, 0.0])
        e[2] += v
    return list(per.values())


def traffic_from_dbs(fetch_db, write_db, kernel, calib_bytes):
    """HBM bytes per launch of `kernel` from a FETCH_SIZE run and a WRITE_SIZE
    run (KiB per dispatch), each scaled by what the same counter reads for the
    calibration copy of calib_bytes (the largest copy dispatch)."""
    sym = KERNEL_SYMBOL.get(kernel, kernel)
    out = {}
    for name, db in (("FETCH_SIZE", fetch_db), ("WRITE_SIZE", write_db)):
        rows = _pmc_rows(db, name)
        copies = [r for r in rows if "copyBuffer" in r[0]]
        cal = max(copies, key=lambda r: r[1])
        factor = calib_bytes / (cal[2] * 1024.0)
        ks = [r[2] for r in rows if sym + "<" in r[0]]
        out[name] = {"kib_per_launch": sum(ks) / len(ks), "launches": len(ks), "calib_kib": cal[2],
                     "scale": factor, "bytes_per_launch": sum(ks) / len(ks) * 1024.0 * factor}
    return out


def make_input(wl, n):
    from paper_2407_14801_amd import datagen
    if wl["kind"] == "u32":
        hi = 1 << 16 if "2^16" in wl["dist"] else 1 << 32
        return (datagen.uniform_u32(n, seed=wl["data_seed"], hi=hi),)
    return datagen.kv_mixture(n, seed=wl["data_seed"])


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, nproc


def cpu_threads():
    """Host threads for the oracle: the machine's CPU share (OMP_NUM_THREADS there),
    at most 16."""
    _, nproc = cpu_info()
    return max(1, min(16, int(os.environ.get("OMP_NUM_THREADS", nproc)), nproc))


def cpu_baseline(wl, host, cutoff, seed, log2_sample, gpu_out):
    """The CPU oracle, as it stands, on the machine's host cores: the whole input
    on P threads (the root's children spread over them; the reported value),
    its output compared byte for byte with the GPU's; on a 2^log2_sample
    prefix, the single-thread oracle (per-core figure), the P-thread oracle
    again (same bytes and digest) and std::sort / std::stable_sort (the
    paper's comparator) for context."""
    import oracle
    P = cpu_threads()
    model, nproc = cpu_info()
    n = host[0].size
    kv = wl["kind"] != "u32"
    unit = "GPairs/s" if kv else "GKeys/s"

    def run(keys, vals, threads):
        t0 = time.perf_counter()
        with oracle.threads(threads):
            if kv:
                ko, vo, dg, _ = oracle.squaresort_kv(keys, vals, seed, cutoff, want_digest=True)
            else:
                ko, dg, _ = oracle.squaresort_u32(keys, seed, cutoff, want_digest=True)
                vo = None
        return time.perf_counter() - t0, ko, vo, dg

    print(f"# cpu baseline: oracle on {P} threads, n={n}", file=sys.stderr, flush=True)
    t_full, ko, vo, _ = run(host[0], host[1] if kv else None, P)
    same_as_gpu = bool(np.array_equal(ko, gpu_out[0]) and (not kv or np.array_equal(vo, gpu_out[1])))
    del ko, vo
    s = min(1 << log2_sample, n)
    ks, vs = host[0][:s], (host[1][:s] if kv else None)
    print(f"# cpu baseline: single thread and {P} threads on {s} keys", file=sys.stderr, flush=True)
    t1, k1, v1, d1 = run(ks, vs, 1)
    tP, kP, vP, dP = run(ks, vs, P)
    identical = bool(np.array_equal(k1, kP) and d1 == dP and (not kv or np.array_equal(v1, vP)))
    del k1, v1, kP, vP
    t0 = time.perf_counter()
    if kv:
        oracle.std_stable_sort_kv(ks, vs)
    else:
        oracle.std_sort_u32(ks)
    t_std = time.perf_counter() - t0
    return {"value": round(n / t_full / 1e9, 6), "unit": unit, "cores": P, "kind": "oracle",
            "seconds": round(t_full, 3), "same_bytes_as_gpu": same_as_gpu,
            "sample": f"whole input (n = {n}) on {P} threads (the root's children spread over them)",
            "cpu_model": model, "nproc": nproc,
            "single_thread": {"n": s, "seconds": round(t1, 3), "value": round(s / t1 / 1e9, 6), "unit": unit,
                              "threaded_seconds": round(tP, 3), "identical_to_threaded": identical},
            "std_sort_single_thread": {"n": s, "what": "std::stable_sort by key" if kv else "std::sort",
                                       "seconds": round(t_std, 3), "value": round(s / t_std / 1e9, 6),
                                       "unit": unit}}


def roofline_of(timing, steps, w, traffic_key=None):
    """Per-kernel shares and the dominant kernel against the HBM peak."""
    kern = {}
    if not timing:
        return None, kern
    tot = sum(v["ms"] for v in timing.values())
    for k, v in timing.items():
        kern[k] = {"ms_per_step": v["ms"] / steps, "launches_per_step": v["launches"] / steps,
                   "share": v["ms"] / tot if tot else 0.0}
    dom = max(timing, key=lambda k: timing[k]["ms"])
    d = timing[dom]
    avg_ms = d["ms"] / d["launches"]
    bytes_per_launch = 2 * w * d["units"] / d["launches"]     # read + write of each key
    ach = bytes_per_launch / (avg_ms / 1e3) / 1e9
    traffic = None
    if traffic_key and os.path.exists(TRAFFIC_JSON):
        with open(TRAFFIC_JSON) as f:
            tr = json.load(f)
        if tr.get("source_hash") == source_hash() and tr.get("kernel") == dom and tr.get("workload") == traffic_key:
            traffic = int(tr["traffic_bytes_per_launch"])
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": traffic,
            "avg_launch_ms": round(avg_ms, 5), "alg_bytes_per_launch": int(bytes_per_launch)}
    return roof, kern


def bench_batched(args, wl):
    """4096 instances, sizes log-uniform in [2^10, 2^20], one batched call per
    step; the plain path (one call per instance, same seeds and cut-off) is
    timed on the same data and must give the same bytes."""
    import torch
    from paper_2407_14801_amd import autotune, binding, datagen
    dev = torch.device("cuda:0")
    sizes = datagen.log_uniform_sizes(wl["count"], wl["lo"], wl["hi"], seed=wl["data_seed"])
    total = int(sizes.sum())
    print(f"# generating {wl['count']} instances, {total} keys", file=sys.stderr, flush=True)
    keys = datagen.uniform_u32(total, seed=wl["data_seed"] + 1000)
    offs = binding.batched_offsets(sizes)
    seeds = np.arange(1, wl["count"] + 1, dtype=np.uint64)
    ws = binding.Workspace(dev)
    base = torch.from_numpy(keys.view(np.int32)).to(dev)
    cutoff, tile, tune = args.cutoff, 0, None
    if not args.no_autotune and not args.cutoff:
        print("# autotuning the cut-off and tile shapes", file=sys.stderr, flush=True)
        cutoff, tile, tune = autotune.tune_batched(base, offs, seeds, ws=ws)
    ins = [base.clone() for _ in range(args.warmup + args.steps)]
    out = torch.empty_like(base)
    for i in range(args.warmup):
        used = binding.squaresort_batched_u32(ins[i], out, offs, seeds, cutoff=cutoff, ws=ws, tile=tile)
    torch.cuda.synchronize()
    if not args.no_timing:
        binding.timing_enable(True)
    print(f"# timing {args.steps} batched steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        used = binding.squaresort_batched_u32(ins[i], out, offs, seeds, cutoff=cutoff, ws=ws, tile=tile)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = binding.timing_report() if not args.no_timing else {}
    binding.timing_enable(False)
    del ins
    ms = (t1 - t0) * 1e3 / args.steps

    # plain path: one call per instance on a fresh copy
    print(f"# timing {args.plain_steps} plain steps ({wl['count']} calls each)", file=sys.stderr, flush=True)
    plain_out = torch.empty_like(base)
    bounds = [(int(offs[i]), int(offs[i + 1])) for i in range(wl["count"])]
    plain_ms = []
    for r in range(args.plain_steps + 1):            # the first is a warm-up
        src = base.clone()
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for i, (lo, hi) in enumerate(bounds):
            binding.squaresort_u32(src[lo:hi], plain_out[lo:hi], seed=int(seeds[i]), cutoff=used, ws=ws,
                                   tile=tile)
        torch.cuda.synchronize()
        if r:
            plain_ms.append((time.perf_counter() - p0) * 1e3)
    same = bool(torch.equal(out, plain_out))

    # planned graph: the same call captured once, replayed (input restored
    # by an untimed copy before each replay; HIP events around the replay)
    print(f"# planned graph: {args.steps} replays", file=sys.stderr, flush=True)
    gin, gout = torch.empty_like(base), torch.empty_like(base)
    plan = binding.BatchedGraph(gin, gout, offs, seeds, cutoff=used, tile=tile)
    stream = torch.cuda.current_stream(dev)
    gms = []
    for r in range(args.warmup + args.steps):
        gin.copy_(base)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.launch()
        e1.record(stream)
        torch.cuda.synchronize()
        if r >= args.warmup:
            gms.append(e0.elapsed_time(e1))
    graph_status = int(plan.status.item())
    graph_same = bool(torch.equal(gout, out))
    plan.close()
    del gin, gout
    gmed = float(np.median(gms))
    o = out.to(torch.int64) & 0xFFFFFFFF
    ok = o[1:] >= o[:-1]
    starts = torch.from_numpy(offs[1:-1].astype(np.int64) - 1).to(dev)
    ok[starts[starts >= 0]] = True                    # instance boundaries may descend
    sorted_ok = bool(ok.all().item())

    w = 4
    roof, kern = roofline_of(timing, args.steps, w)
    b_alg = 6 * w * total
    pms = float(np.median(plain_ms))
    res = {
        "metric": "GKeys/s", "value": round(total / (ms / 1e3) / 1e9, 4), "unit": "GKeys/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"batched_u32_{wl['count']}x_loguniform[2^10,2^20]", "instances": wl["count"],
                   "total_keys": total, "key_dist": wl["dist"], "data_seed": wl["data_seed"],
                   "seeds": "1..count", "cutoff": int(used), "tile": binding.tile_fields(tile),
                   "autotune": tune},
        "plain_per_instance": {"value": round(total / (pms / 1e3) / 1e9, 4), "unit": "GKeys/s",
                               "ms_per_step": round(pms, 3), "calls_per_step": wl["count"]},
        "graph_replay": {"value": round(total / (gmed / 1e3) / 1e9, 4), "unit": "GKeys/s",
                         "ms_median": round(gmed, 4), "ms_p10": round(float(np.percentile(gms, 10)), 4),
                         "ms_p90": round(float(np.percentile(gms, 90)), 4), "replays": len(gms),
                         "status": graph_status, "same_bytes_as_batched": graph_same,
                         "how": "squaresort_batched_graph_u32 planned once, sqs_plan_launch per step; "
                                "HIP events around each replay"},
        "speedup_vs_plain": round(pms / ms, 3),
        "same_bytes_as_plain": same,
        "roofline": roof,
        "path_roofline": {"bytes_alg_per_level": b_alg, "levels": 1,
                          "achieved_gbs": round(b_alg / (ms / 1e3) / 1e9, 3), "peak_gbs": HBM_PEAK_GBS,
                          "frac": round(b_alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 5)},
        "kernels": {k: {kk: round(vv, 5) for kk, vv in v.items()} for k, v in kern.items()},
        "sorted_check": sorted_ok,
    }
    print(json.dumps(res), flush=True)


def bench_served(args, wl):
    """A Poisson stream of mixed requests (sizes log-uniform in [2^12, 2^24];
    70% u32, 30% key/value; keys uniform or Zipf(1.1)).  The plain path's
    capacity is measured first (each request alone, one call at a time); the
    stream then arrives at --serve-load times that capacity and is served
    twice at the same arrival times: plain (FIFO, one call per request) and
    served (admission by a 64 GB budget, continuous batching per kind, the
    two kinds overlapping on separate streams).  Every served result must
    equal the request's result alone."""
    import torch
    from paper_2407_14801_amd import datagen
    from paper_2407_14801_amd.serve import GpuExecutor, PlainExecutor, Request, Server, percentiles, replay
    dev = torch.device("cuda:0")
    count = args.serve_count
    print(f"# generating {count} requests", file=sys.stderr, flush=True)
    specs = datagen.serve_requests(count, wl["data_seed"], lo=wl["lo"], hi=wl["hi"])
    staged = []
    for s in specs:
        if s["kind"] == "u32":
            staged.append((torch.from_numpy(s["keys"].view(np.int32)).to(dev), None))
        else:
            staged.append((torch.from_numpy(s["keys"].view(np.int64)).to(dev),
                           torch.from_numpy(s["vals"].view(np.int32)).to(dev)))
    total = sum(s["n"] for s in specs)

    def fresh():
        return [Request(id=s["id"], kind=s["kind"], n=s["n"], seed=s["seed"], keys=k, vals=v)
                for s, (k, v) in zip(specs, staged)]

    # capacity of the plain path: every request alone (after one warm-up pass)
    plain = PlainExecutor(dev, args.cutoff)
    print("# alone (capacity)", file=sys.stderr, flush=True)
    for r in fresh()[: min(16, count)]:
        plain(r.kind, [r])
    alone = fresh()
    svc = []
    for r in alone:
        t0 = time.perf_counter()
        plain(r.kind, [r])
        svc.append(time.perf_counter() - t0)
    cap = 1.0 / float(np.mean(svc))                       # requests per second
    rate = args.serve_load * cap
    g = np.random.Generator(np.random.PCG64(wl["data_seed"] + 7))
    arrivals = np.cumsum(g.exponential(1.0 / rate, size=count))
    arrivals -= arrivals[0]

    def run(server, label):
        reqs = fresh()
        print(f"# {label} stream at {rate:.1f} req/s", file=sys.stderr, flush=True)
        server.start()
        t0 = replay(server, reqs, arrivals)
        server.drain(count)
        span = max(r.done for r in reqs) - t0
        lat = [r.latency * 1e3 for r in reqs]
        return reqs, {"keys_per_s_G": round(total / span / 1e9, 4), "span_s": round(span, 4),
                      **{k + "_ms": round(v, 3) for k, v in percentiles(lat).items()},
                      "mean_ms": round(float(np.mean(lat)), 3)}

    _, plain_stats = run(Server(PlainExecutor(dev, args.cutoff), max_batch_keys=0, lanes=("all",),
                                lane_of=lambda r: "all", budget_bytes=wl["budget_gb"] << 30), "plain")
    srv = Server(GpuExecutor(dev, args.cutoff), budget_bytes=wl["budget_gb"] << 30)
    served, served_stats = run(srv, "served")
    same = all(torch.equal(a.out_keys, b.out_keys) and (a.out_vals is None or torch.equal(a.out_vals, b.out_vals))
               for a, b in zip(alone, served))
    batches = len({r.batch for r in served})
    res = {
        "metric": "GKeys/s", "value": served_stats["keys_per_s_G"], "unit": "GKeys/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(served_stats["span_s"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32 | u64+u32",
        "data": "synthetic",
        "config": {"workload": "served_poisson_mixed", "requests": count, "total_keys": total,
                   "sizes": "log-uniform [2^12, 2^24]", "mix": "70% u32 / 30% u64+u32; uniform or Zipf(1.1) 1/2 each",
                   "budget_gb": wl["budget_gb"], "arrival_rate_req_s": round(rate, 2),
                   "load_vs_plain_capacity": args.serve_load, "plain_capacity_req_s": round(cap, 2)},
        "served": {**served_stats, "batches": batches, "peak_admitted_gb": round(srv.peak_used / 2**30, 3)},
        "plain_one_call_per_request": plain_stats,
        "alone_service_ms": {"mean": round(float(np.mean(svc)) * 1e3, 3),
                             **{k: round(v * 1e3, 3) for k, v in percentiles(svc).items()}},
        "same_results_alone_and_in_mix": bool(same),
    }
    print(json.dumps(res), flush=True)


def bench_alg1(args, wl):
    """n = 2^28 distinct u32 keys (a permutation, spread by an odd
    multiplier) sorted under the Alg. 1 pivot rule and under the default
    rule; the root's bucket sizes (Alg. 1 rule) against the Section 3.2
    bounds: Pr[n_i >= t sqrt n] <= e^{-0.9t+0.1}, Pr[n_1 <= s] <= e^2 s /
    sqrt n, sum n_i log n_i <= n log n / 2 + 4 e n (in expectation)."""
    import math
    import torch
    from paper_2407_14801_amd import binding
    dev = torch.device("cuda:0")
    log2n = args.log2n or wl["log2n"]
    n = 1 << log2n
    print(f"# generating a permutation of 2^{log2n}", file=sys.stderr, flush=True)
    g = np.random.Generator(np.random.PCG64(wl["data_seed"]))
    x = (g.permutation(n).astype(np.uint64) * 2654435761 % (1 << 32)).astype(np.uint32)
    base = torch.from_numpy(x.view(np.int32)).to(dev)
    out = torch.empty_like(base)
    ws = binding.Workspace(dev)
    res_rules = {}
    for rule in ("alg1", "replacement"):
        ins = [base.clone() for _ in range(args.warmup + args.steps)]
        for i in range(args.warmup):
            used = binding.squaresort_u32(ins[i], out, seed=1, cutoff=args.cutoff, ws=ws, pivot_rule=rule)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.warmup, args.warmup + args.steps):
            used = binding.squaresort_u32(ins[i], out, seed=1, cutoff=args.cutoff, ws=ws, pivot_rule=rule)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        o = out.to(torch.int64) & 0xFFFFFFFF
        res_rules[rule] = {"ms_per_step": round(ms, 4), "GKeys_s": round(n / ms / 1e6, 4), "cutoff": int(used),
                           "sorted_check": bool((o[1:] > o[:-1]).all().item())}
        del ins
    # root bucket sizes under the Alg. 1 rule, several seeds
    m = int(math.isqrt(n - 1)) + 1
    sizes = []
    for seed in range(1, 5):
        bs = torch.empty(m + 1, dtype=torch.int64, device=dev)
        src = base.clone()
        binding.skew_transpose_u32(src, out, bs, seed=seed, ws=ws, pivot_rule="alg1")
        torch.cuda.synchronize()
        sizes.append(np.diff(bs.cpu().numpy()))
        del src
    allsz = np.concatenate(sizes)
    rn = math.sqrt(n)
    tails = {str(t): {"measured": round(float(np.mean(allsz >= t * rn)), 6), "bound": round(math.exp(-0.9 * t + 0.1), 6)}
             for t in (1, 2, 3, 4, 6)}
    first = np.array([s[0] for s in sizes])
    ent = float(np.mean([np.sum(s * np.log2(s)) for s in sizes]))
    res = {
        "metric": "GKeys/s", "value": res_rules["alg1"]["GKeys_s"], "unit": "GKeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res_rules["alg1"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"squaresort_u32_perm_alg1_2^{log2n}", "n": n, "key_dist": wl["dist"],
                   "data_seed": wl["data_seed"], "seed": 1, "pivot_rule": "alg1"},
        "rules": res_rules,
        "root_buckets_alg1": {"seeds": 4, "m": m, "min_size": int(allsz.min()), "max_size": int(allsz.max()),
                              "upper_tail": tails,
                              "first_bucket_le_s": {str(s): {"measured": round(float(np.mean(first <= s)), 4),
                                                             "bound": round(math.e ** 2 * s / rn, 6)} for s in (2, 10, 30)},
                              "sum_ni_log2_ni": {"measured": round(ent, 1),
                                                 "bound": round(0.5 * n * math.log2(n) + 4 * math.e * n, 1)}},
    }
    print(json.dumps(res), flush=True)


def bench_host(args, wl):
    """n = 2^28 uniform u32 keys in pinned host memory, sorted there by the
    GPU (SQS_FLAG_HOST_ARRAYS; the workspace in HBM).  The input is restored
    from a pristine host copy before each step (untimed); HIP events around
    each call."""
    import torch
    from paper_2407_14801_amd import binding
    dev = torch.device("cuda:0")
    log2n = args.log2n or wl["log2n"]
    n = 1 << log2n
    print(f"# generating u32_host n=2^{log2n}", file=sys.stderr, flush=True)
    from paper_2407_14801_amd import datagen
    x = datagen.uniform_u32(n, seed=wl["data_seed"])
    pristine = torch.from_numpy(x.view(np.int32))
    inp = torch.empty(n, dtype=torch.int32).pin_memory()
    out = torch.empty(n, dtype=torch.int32).pin_memory()
    ws = binding.Workspace(dev)
    stream = torch.cuda.current_stream(dev)
    ms = []
    for r in range(args.warmup + args.steps):
        inp.copy_(pristine)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        cutoff = binding.squaresort_u32(inp, out, seed=1, cutoff=args.cutoff, ws=ws, host_arrays=True)
        e1.record(stream)
        torch.cuda.synchronize()
        if r >= args.warmup:
            ms.append(e0.elapsed_time(e1))
    o = out.numpy().view(np.uint32)
    sorted_ok = bool(np.all(o[1:] >= o[:-1]))
    med = float(np.median(ms))
    link = 6 * 4 * n                                   # 3 passes, each reading and writing the array
    res = {"metric": "GKeys/s", "value": round(n / (med / 1e3) / 1e9, 4), "unit": "GKeys/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(med, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"squaresort_u32_host_2^{log2n}", "n": n, "key_dist": wl["dist"],
                      "data_seed": wl["data_seed"], "seed": 1, "cutoff": cutoff,
                      "arrays": "pinned host memory (SQS_FLAG_HOST_ARRAYS); workspace in HBM"},
           "latency_ms": {"p10": round(float(np.percentile(ms, 10)), 3), "p50": round(med, 3),
                          "p90": round(float(np.percentile(ms, 90)), 3)},
           "host_link": {"bytes_alg": link, "achieved_gbs": round(link / (med / 1e3) / 1e9, 2),
                         "how": "6 * 4 * n bytes: three passes each reading and writing the array"},
           "sorted_check": sorted_ok}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="u32_uniform", choices=sorted(WORKLOADS))
    ap.add_argument("--log2n", type=int, default=None, help="override the size (2^k keys)")
    ap.add_argument("--cutoff", type=int, default=0, help="base-case cut-off (0 = the library's automatic choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched workload: library defaults instead of the tuned cut-off and tile shapes")
    ap.add_argument("--plain-steps", type=int, default=2, help="batched workload: timed one-call-per-instance steps")
    ap.add_argument("--serve-count", type=int, default=256, help="served workload: requests in the stream")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="served workload: arrival rate as a fraction of the plain path's capacity")
    ap.add_argument("--cpu-sample-log2", type=int, default=26)
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel timing pass")
    ap.add_argument("--kernel-steps", type=int, default=3,
                    help="steps of the separate per-kernel timing pass (launch events on)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, copy one input (n*w bytes) device-to-device: the known-size "
                         "kernel that scales rocprofv3 FETCH_SIZE / WRITE_SIZE readings")
    ap.add_argument("--traffic-dbs", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="rocprofv3 --pmc results of a --calib-copy run for FETCH_SIZE and WRITE_SIZE: "
                         "record the dominant kernel's HBM traffic in profiles/traffic.json and exit")
    ap.add_argument("--traffic-kernel", default="k_colsort")
    args = ap.parse_args()

    if args.traffic_dbs:
        wl = WORKLOADS[args.workload]
        log2n = args.log2n or wl["log2n"]
        calib = (1 << log2n) * (4 if wl["kind"] == "u32" else 8)
        t = traffic_from_dbs(args.traffic_dbs[0], args.traffic_dbs[1], args.traffic_kernel, calib)
        rec = {"kernel": args.traffic_kernel, "workload": f"squaresort_{args.workload}_2^{log2n}",
               "source_hash": source_hash(),
               "traffic_bytes_per_launch": t["FETCH_SIZE"]["bytes_per_launch"] + t["WRITE_SIZE"]["bytes_per_launch"],
               "counters": t}
        os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
        with open(TRAFFIC_JSON, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))
        return

    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU exchange is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_14801_amd import binding

    wl = WORKLOADS[args.workload]
    if wl["kind"] == "batched":
        return bench_batched(args, wl)
    if wl["kind"] == "served":
        return bench_served(args, wl)
    if wl["kind"] == "alg1":
        return bench_alg1(args, wl)
    if wl["kind"] == "host":
        return bench_host(args, wl)
    log2n = args.log2n or wl["log2n"]
    n = 1 << log2n
    dev = torch.device("cuda:0")
    seed = 1
    req_cutoff = args.cutoff or wl.get("cutoff", 0)
    print(f"# generating {args.workload} n=2^{log2n}", file=sys.stderr, flush=True)
    host = make_input(wl, n)
    ws = binding.Workspace(dev)
    kstep = 0 if args.no_timing else args.kernel_steps
    copies = args.warmup + args.steps + kstep
    want_digest = wl.get("cutoff") is not None          # the recursive workload checks its tree digest
    dg = torch.zeros(1, dtype=torch.int64, device=dev) if want_digest else None

    if wl["kind"] == "u32":
        base = torch.from_numpy(host[0].view(np.int32)).to(dev)
        ins = [base.clone() for _ in range(copies)]
        out = torch.empty_like(base)
        w = 4

        def step(i, digest=None):
            return binding.squaresort_u32(ins[i], out, seed=seed, cutoff=req_cutoff, ws=ws, digest=digest)
    else:
        bk = torch.from_numpy(host[0].view(np.int64)).to(dev)
        bv = torch.from_numpy(host[1].view(np.int32)).to(dev)
        ins = [(bk.clone(), bv.clone()) for _ in range(copies)]
        ko, vo = torch.empty_like(bk), torch.empty_like(bv)
        w = 12

        def step(i, digest=None):
            return binding.squaresort_kv(ins[i][0], ins[i][1], ko, vo, seed=seed, cutoff=req_cutoff, ws=ws,
                                         digest=digest)
    torch.cuda.synchronize()

    print(f"# warmup {args.warmup}", file=sys.stderr, flush=True)
    cutoff = 0
    for i in range(args.warmup):
        cutoff = step(i, dg if i == 0 else None)
    torch.cuda.synchronize()
    gpu_digest = int(dg.cpu().numpy().view(np.uint64)[0]) if want_digest else None

    # headline: K steps between two synchronisations, no per-kernel events;
    # per-step latency from HIP events on the stream the library launches on
    print(f"# timing {args.steps} steps", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream(dev)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j, i in enumerate(range(args.warmup, args.warmup + args.steps)):
        evs[j][0].record(stream)
        cutoff = step(i)
        evs[j][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_step = np.array([a.elapsed_time(c) for a, c in evs])

    # per-kernel times: a separate pass with the library's launch events on
    timing = {}
    if kstep:
        print(f"# per-kernel timing pass, {kstep} steps", file=sys.stderr, flush=True)
        binding.timing_enable(True)
        for i in range(args.warmup + args.steps, copies):
            step(i)
        torch.cuda.synchronize()
        timing = binding.timing_report()
        binding.timing_enable(False)
    if args.calib_copy:
        src = ins[0] if wl["kind"] == "u32" else ins[0][0]
        _c = src.clone()
        torch.cuda.synchronize()
        del _c
    del ins

    # the last output must be sorted (cheap device check)
    if wl["kind"] == "u32":
        o = out.to(torch.int64) & 0xFFFFFFFF
    else:   # compare unsigned 64-bit keys by flipping the sign bit
        o = ko.view(torch.int64) ^ torch.tensor(-(1 << 63), dtype=torch.int64, device=dev)
    sorted_ok = bool((o[1:] >= o[:-1]).all().item())
    del o

    ms = (t1 - t0) * 1e3 / args.steps
    value = n / (ms / 1e3) / 1e9
    b_alg = 6 * w * n
    path = {"bytes_alg_per_level": b_alg, "levels": 1, "achieved_gbs": b_alg / (ms / 1e3) / 1e9,
            "peak_gbs": HBM_PEAK_GBS}
    path["frac"] = path["achieved_gbs"] / HBM_PEAK_GBS

    roof, kern = roofline_of(timing, kstep, w, f"squaresort_{args.workload}_2^{log2n}")

    res = {
        "metric": "GKeys/s" if wl["kind"] == "u32" else "GPairs/s",
        "value": round(value, 4),
        "unit": "GKeys/s" if wl["kind"] == "u32" else "GPairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if wl["kind"] == "u32" else "u64+u32",
        "data": "synthetic",
        "config": {"workload": f"squaresort_{args.workload}_2^{log2n}", "n": n, "key_dist": wl["dist"],
                   "data_seed": wl["data_seed"], "seed": seed, "cutoff": cutoff},
        "latency_ms": {"p10": round(float(np.percentile(per_step, 10)), 4),
                       "p50": round(float(np.percentile(per_step, 50)), 4),
                       "p90": round(float(np.percentile(per_step, 90)), 4),
                       "how": "HIP events around each call on its stream; per-kernel events off"},
        "roofline": roof,
        "path_roofline": {k: (round(v, 5) if isinstance(v, float) else v) for k, v in path.items()},
        "kernels": {k: {kk: round(vv, 5) for kk, vv in v.items()} for k, v in kern.items()},
        "sorted_check": sorted_ok,
    }
    if timing:
        # device time per recursion depth (launches of deeper steps are named kernel@depth)
        depth = {}
        for k, v in timing.items():
            d = int(k.split("@")[1]) if "@" in k else 0
            depth[d] = depth.get(d, 0.0) + v["ms"] / kstep
        res["ms_per_depth"] = {str(d): round(t, 4) for d, t in sorted(depth.items())}
    gpu_out = None
    if want_digest or not args.no_cpu_baseline:
        gpu_out = ((out.cpu().numpy().view(np.uint32),) if wl["kind"] == "u32"
                   else (ko.cpu().numpy().view(np.uint64), vo.cpu().numpy().view(np.uint32)))
    if want_digest:
        import oracle
        print("# oracle digest", file=sys.stderr, flush=True)
        with oracle.threads(cpu_threads()):
            wout, wdg, nodes = oracle.squaresort_u32(host[0], seed, cutoff, want_digest=True)
        res["parity"] = {"digest": f"{gpu_digest:#018x}", "oracle_digest": f"{wdg:#018x}", "nodes": nodes,
                         "digest_equal": gpu_digest == wdg, "output_equal": bool(np.array_equal(wout, gpu_out[0]))}
    if not args.no_cpu_baseline:
        print("# cpu baseline", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(wl, host, cutoff, seed, min(args.cpu_sample_log2, log2n), gpu_out)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
