"""Cut-off autotuner for the batched form.

The cut-off C decides which instances (and buckets) are base cases sorted in
one work-group and which become SquareSort nodes.  tune_batched_cutoff times
the batched entry point on the caller's instance sizes for each candidate C
(HIP events on the current stream, a pristine input restored before each
call) and returns the fastest with the whole table.  The outputs do not
depend on C; only the recursion tree and the time do.
"""
from __future__ import annotations

import numpy as np
import torch

DEFAULT_CANDIDATES = (4096, 16384, 65536, 131072, 262144)


def tune_batched_cutoff(pristine: torch.Tensor, offsets, seeds, candidates=DEFAULT_CANDIDATES,
                        reps: int = 3, ws=None):
    from . import binding
    scratch = torch.empty_like(pristine)
    out = torch.empty_like(pristine)
    ws = ws or binding.Workspace(pristine.device)
    table = {}
    stream = torch.cuda.current_stream(pristine.device)
    for c in candidates:
        times = []
        for r in range(reps + 1):            # the first call of a candidate is a warm-up
            scratch.copy_(pristine)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            binding.squaresort_batched_u32(scratch, out, offsets, seeds, cutoff=c, ws=ws)
            b.record(stream)
            torch.cuda.synchronize()
            if r:
                times.append(a.elapsed_time(b))
        table[int(c)] = float(np.median(times))
    best = min(table, key=table.get)
    return best, table
