"""Served form: a request loop with admission by device-memory budget and
continuous batching.

Clients submit sort requests (uint32 keys, or uint64 key / uint32 value pairs)
whose inputs already sit in device memory.  The server admits requests in
arrival order while their device bytes fit the budget, and keeps one worker
per request kind (its own HIP stream): whenever a worker is free it takes
every admitted request of its kind that is waiting (up to a key cap), packs
them into one buffer and sorts them with one batched call, so requests that
arrive while others are on the GPU join the next batch and the two kinds
overlap on the device.  Each request is sorted with its own seed, so its
result is the same alone and in any mix.

The executor is pluggable (`execute(kind, requests)`), so the admission and
batching logic also runs without a GPU.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field


@dataclass
class Request:
    id: int
    kind: str                 # "u32" or "kv"
    n: int
    seed: int
    keys: object = None       # device tensor (int32 for u32, int64 for kv); not modified
    vals: object = None       # device int32 tensor for kv
    out_keys: object = None
    out_vals: object = None
    arrival: float = 0.0
    admitted: float = 0.0
    done: float = 0.0
    batch: int = -1           # id of the batch that served it
    ready: object = None      # event on the submitting thread's stream after the inputs were written

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def device_bytes(r: Request) -> int:
    """Device bytes a request holds while admitted: its input and output, and
    its share of the packed batch buffers and workspace (about 2x its data)."""
    per_key = 4 if r.kind == "u32" else 12
    return 4 * per_key * r.n


@dataclass
class Server:
    execute: object                      # callable(kind, list[Request]) -> None
    budget_bytes: int = 64 << 30
    max_batch_keys: int = 1 << 27      # 0: one request per batch
    lanes: tuple = ("u32", "kv")       # one worker per lane
    lane_of: object = None             # request -> lane (default: its kind)
    clock: object = time.perf_counter
    _lock: threading.Condition = field(default_factory=threading.Condition)
    _pending: list = field(default_factory=list)
    _ready: dict = field(default_factory=dict)
    _used: int = 0
    _stop: bool = False
    _threads: list = field(default_factory=list)
    _batches: int = 0
    done: list = field(default_factory=list)
    peak_used: int = 0

    def start(self):
        self._ready = {k: [] for k in self.lanes}
        for k in self.lanes:
            t = threading.Thread(target=self._worker, args=(k,), daemon=True)
            t.start()
            self._threads.append(t)
        return self

    def submit(self, r: Request):
        """Queue a request.  Its inputs may still be in flight on the caller's
        current stream: an event recorded there now is waited for before they
        are read.  Its outputs are complete once it is done; a consumer that
        uses them on another stream must record_stream them there."""
        if device_bytes(r) > self.budget_bytes:
            raise ValueError(f"request {r.id} needs more than the whole budget")
        if r.keys is not None and getattr(r.keys, "is_cuda", False):
            import torch
            r.ready = torch.cuda.Event()
            r.ready.record(torch.cuda.current_stream(r.keys.device))
        with self._lock:
            r.arrival = self.clock()
            self._pending.append(r)
            self._admit()
            self._lock.notify_all()

    def _admit(self):
        # arrival order; the head waits until it fits (no overtaking)
        while self._pending and self._used + device_bytes(self._pending[0]) <= self.budget_bytes:
            r = self._pending.pop(0)
            self._used += device_bytes(r)
            self.peak_used = max(self.peak_used, self._used)
            r.admitted = self.clock()
            self._ready[self.lane_of(r) if self.lane_of else r.kind].append(r)

    def _worker(self, lane):
        while True:
            with self._lock:
                while not self._ready[lane] and not self._stop:
                    self._lock.wait()
                if not self._ready[lane] and self._stop:
                    return
                batch, keys = [], 0
                q = self._ready[lane]
                while q and (not batch or keys + q[0].n <= self.max_batch_keys):
                    r = q.pop(0)
                    batch.append(r)
                    keys += r.n
                bid = self._batches
                self._batches += 1
            self.execute(batch[0].kind, batch)
            t = self.clock()
            with self._lock:
                for r in batch:
                    r.done = t
                    r.batch = bid
                    self._used -= device_bytes(r)
                    self.done.append(r)
                self._admit()
                self._lock.notify_all()

    def drain(self, count: int, timeout: float = 600.0):
        """Wait until `count` requests are done, then stop the workers."""
        end = time.perf_counter() + timeout
        with self._lock:
            while len(self.done) < count:
                if not self._lock.wait(timeout=max(0.0, end - time.perf_counter())):
                    raise TimeoutError(f"{len(self.done)} of {count} requests done")
            self._stop = True
            self._lock.notify_all()
        for t in self._threads:
            t.join()


def replay(server: Server, requests, arrivals):
    """Submit requests at their arrival offsets (seconds from now)."""
    t0 = time.perf_counter()
    for r, a in zip(requests, arrivals):
        delay = t0 + a - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        server.submit(r)
    return t0


def percentiles(values, ps=(50, 99)):
    import numpy as np
    v = np.asarray(values, dtype=np.float64)
    return {f"p{p}": float(np.percentile(v, p)) for p in ps}


# ------------------------------------------------------------------ GPU executors
class GpuExecutor:
    """Sorts a batch of same-kind requests with one batched call on this
    kind's stream: inputs are packed into one buffer, outputs are views of
    the packed result.  A batch of one request takes the single-instance
    call instead (the same bytes: an instance of a batch ends exactly as it
    would alone)."""

    def __init__(self, device, cutoff: int = 0):
        import torch
        from . import binding
        self.torch, self.b = torch, binding
        self.device = device
        self.cutoff = cutoff
        self.streams = {k: torch.cuda.Stream(device) for k in ("u32", "kv")}
        self.ws = {k: binding.Workspace(device) for k in ("u32", "kv")}

    def __call__(self, kind, batch):
        torch, b = self.torch, self.b
        import numpy as np
        st = self.streams[kind]
        for r in batch:                       # inputs written on the submitters' streams
            if r.ready is not None:
                st.wait_event(r.ready)
        with torch.cuda.stream(st):
            if len(batch) == 1:               # alone: the single-instance call (same bytes, no packing)
                r = batch[0]
                if kind == "u32":
                    src = r.keys.clone()      # the call clobbers its input
                    r.out_keys = torch.empty_like(src)
                    b.squaresort_u32(src, r.out_keys, seed=r.seed, cutoff=self.cutoff, ws=self.ws[kind])
                else:
                    ks, vs = r.keys.clone(), r.vals.clone()
                    r.out_keys, r.out_vals = torch.empty_like(ks), torch.empty_like(vs)
                    b.squaresort_kv(ks, vs, r.out_keys, r.out_vals, seed=r.seed, cutoff=self.cutoff,
                                    ws=self.ws[kind])
                st.synchronize()
                return
            sizes = [r.n for r in batch]
            offs = b.batched_offsets(sizes)
            seeds = np.array([r.seed for r in batch], dtype=np.uint64)
            total = int(offs[-1])
            if kind == "u32":
                pin = torch.empty(total, dtype=torch.int32, device=self.device)
                for r, o in zip(batch, offs[:-1]):
                    pin[int(o):int(o) + r.n].copy_(r.keys)
                pout = torch.empty_like(pin)
                b.squaresort_batched_u32(pin, pout, offs, seeds, cutoff=self.cutoff, ws=self.ws[kind])
                for r, o in zip(batch, offs[:-1]):
                    r.out_keys = pout[int(o):int(o) + r.n]
            else:
                kin = torch.empty(total, dtype=torch.int64, device=self.device)
                vin = torch.empty(total, dtype=torch.int32, device=self.device)
                for r, o in zip(batch, offs[:-1]):
                    kin[int(o):int(o) + r.n].copy_(r.keys)
                    vin[int(o):int(o) + r.n].copy_(r.vals)
                kout, vout = torch.empty_like(kin), torch.empty_like(vin)
                b.squaresort_batched_kv(kin, vin, kout, vout, offs, seeds, cutoff=self.cutoff, ws=self.ws[kind])
                for r, o in zip(batch, offs[:-1]):
                    r.out_keys = kout[int(o):int(o) + r.n]
                    r.out_vals = vout[int(o):int(o) + r.n]
        st.synchronize()


class PlainExecutor:
    """One single-instance call per request, one request at a time (the
    plain path the served form is compared with; use it with one lane and
    max_batch_keys = 0)."""

    def __init__(self, device, cutoff: int = 0):
        import torch
        from . import binding
        self.torch, self.b = torch, binding
        self.device = device
        self.cutoff = cutoff
        self.stream = torch.cuda.Stream(device)
        self.ws = binding.Workspace(device)
        self._mu = threading.Lock()

    def __call__(self, kind, batch):
        torch, b = self.torch, self.b
        with self._mu, torch.cuda.stream(self.stream):
            for r in batch:                   # inputs written on the submitters' streams
                if r.ready is not None:
                    self.stream.wait_event(r.ready)
            for r in batch:
                if r.kind == "u32":
                    src = r.keys.clone()
                    r.out_keys = torch.empty_like(src)
                    b.squaresort_u32(src, r.out_keys, seed=r.seed, cutoff=self.cutoff, ws=self.ws)
                else:
                    ks, vs = r.keys.clone(), r.vals.clone()
                    r.out_keys, r.out_vals = torch.empty_like(ks), torch.empty_like(vs)
                    b.squaresort_kv(ks, vs, r.out_keys, r.out_vals, seed=r.seed, cutoff=self.cutoff, ws=self.ws)
            self.stream.synchronize()
