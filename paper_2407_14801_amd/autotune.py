"""Cut-off and tile-shape autotuner for the batched form.

The cut-off C decides which instances (and buckets) are base cases sorted in
one work-group and which become SquareSort nodes; the tile word picks
template instances and size classes of the kernels (waves per work-group of
the wave-level column kernel, the largest bucket one wave sorts, the largest
one 4-wave work-group sorts).  Neither changes the output (nor, for the tile
word, the recursion tree); only the time.  The paper picks its cut-off by a
sweep (Section 4.2); the tuner does the same on the caller's instance sizes,
timing the batched entry point with HIP events on the current stream (a
pristine input restored before each call, the first call of a candidate a
warm-up), then sweeps each tile field in turn with the best cut-off and the
other fields held (coordinate descent).
"""
from __future__ import annotations

import numpy as np
import torch

DEFAULT_CANDIDATES = (4096, 16384, 65536, 131072, 262144)
TILE_FIELDS = (("colw", (4, 2, 8)), ("wcap", (1024, 512, 256)), ("m4cap", (4096, 2048, 1024)))


def _timer(pristine, offsets, seeds, reps, ws):
    from . import binding
    scratch = torch.empty_like(pristine)
    out = torch.empty_like(pristine)
    ws = ws or binding.Workspace(pristine.device)
    stream = torch.cuda.current_stream(pristine.device)

    def run(cutoff, tile):
        times = []
        for r in range(reps + 1):            # the first call of a candidate is a warm-up
            scratch.copy_(pristine)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            binding.squaresort_batched_u32(scratch, out, offsets, seeds, cutoff=cutoff, ws=ws, tile=tile)
            b.record(stream)
            torch.cuda.synchronize()
            if r:
                times.append(a.elapsed_time(b))
        return float(np.median(times))
    return run


def tune_batched_cutoff(pristine: torch.Tensor, offsets, seeds, candidates=DEFAULT_CANDIDATES,
                        reps: int = 3, ws=None):
    """The fastest cut-off among candidates (default tiles) and the table of
    median times."""
    run = _timer(pristine, offsets, seeds, reps, ws)
    table = {int(c): run(int(c), 0) for c in candidates}
    best = min(table, key=table.get)
    return best, table


def tune_batched(pristine: torch.Tensor, offsets, seeds, candidates=DEFAULT_CANDIDATES, reps: int = 3,
                 ws=None):
    """Cut-off, then each tile field in turn.  Returns (cutoff, tile word,
    record) where record holds every timed candidate."""
    from . import binding
    run = _timer(pristine, offsets, seeds, reps, ws)
    cut_table = {int(c): run(int(c), 0) for c in candidates}
    cutoff = min(cut_table, key=cut_table.get)
    best = {"colw": 4, "wcap": 1024, "m4cap": 4096}
    best_ms = cut_table[cutoff]
    tile_table = {}
    for name, values in TILE_FIELDS:
        for v in values:
            trial = dict(best, **{name: v})
            if trial == best:
                continue
            word = binding.tile_word(**trial)
            ms = run(cutoff, word)
            tile_table[str(word)] = {"fields": trial, "ms": ms}
            if ms < best_ms:
                best, best_ms = trial, ms
    word = binding.tile_word(**best)
    record = {"cutoff_ms": cut_table, "tile_ms": tile_table, "cutoff": cutoff, "tile": word,
              "tile_fields": best, "ms": best_ms}
    return cutoff, word, record
