"""Thin ctypes binding of libsquaresort (include/squaresort.h).

Argument marshalling only: device pointers and the current HIP stream are
taken from torch tensors; every step of the sort runs in the HIP library.
Importing this module raises if the library has not been built -- there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsquaresort.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libsquaresort.so not found at {LIB_PATH}; run paper_2407_14801_amd/build.py")

_lib = ctypes.CDLL(LIB_PATH)

KIND_U32, KIND_U64, KIND_KV = 0, 1, 2
FLAG_DIGEST = 1
FLAG_ALG1_PIVOTS = 2
FLAG_VALIDATE = 4
FLAG_COLS_SORTED = 8
FLAG_HOST_ARRAYS = 16
PIVOT_RULES = {"replacement": 0, "alg1": FLAG_ALG1_PIVOTS}
STATIC_SCRATCH_BYTES = 32 << 20          # SQS_STATIC_SCRATCH_BYTES
STATUS = {0: "SQS_OK", -1: "SQS_ERR_ARG", -2: "SQS_ERR_ALIAS", -3: "SQS_ERR_WORKSPACE",
          -4: "SQS_ERR_DEVICE", -5: "SQS_ERR_PRECOND", -6: "SQS_ERR_DEPTH", -7: "SQS_ERR_UNSUPPORTED"}


def tile_word(colw: int = 4, wcap: int = 1024, m4cap: int = 4096) -> int:
    """The sqs_params tile word (SQS_TILE_* fields): waves per work-group of
    the wave-level column kernel (4, 2 or 8), the largest bucket one wave
    sorts (1024, 512 or 256) and the largest one 4-wave work-group sorts
    (4096, 2048 or 1024)."""
    cw = {4: 0, 2: 1, 8: 2}[colw]
    wc = {1024: 0, 512: 1, 256: 2}[wcap]
    m4 = {4096: 0, 2048: 1, 1024: 2}[m4cap]
    return cw | (wc << 2) | (m4 << 4)


def tile_fields(word: int) -> dict:
    """Inverse of tile_word."""
    return {"colw": (4, 2, 8)[word & 3], "wcap": 1024 >> ((word >> 2) & 3), "m4cap": 4096 >> ((word >> 4) & 3)}


class Params(ctypes.Structure):
    _fields_ = [("cutoff", ctypes.c_uint64), ("flags", ctypes.c_uint32), ("tile", ctypes.c_uint32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64),
                ("digest", ctypes.c_void_p)]


_u64, _vp, _i = ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
_P = ctypes.POINTER(Params)
_SIGS = {
    "sqs_max_cutoff": (_u64, [_i]),
    "sqs_max_n": (_u64, [_i]),
    "squaresort_workspace_bytes": (_u64, [_u64, _i, _u64]),
    "squaresort_u32": (_i, [_u64, _vp, _vp, _u64, _P, _vp]),
    "squaresort_u64": (_i, [_u64, _vp, _vp, _u64, _P, _vp]),
    "squaresort_kv": (_i, [_u64, _vp, _vp, _vp, _vp, _u64, _P, _vp]),
    "skew_transpose_u32": (_i, [_u64, _vp, _vp, _vp, _u64, _P, _vp]),
    "squaresort_u32_noalloc": (_i, [_u64, _vp, _vp, _u64, _P, _vp]),
    "squaresort_batched_workspace_bytes": (_u64, [ctypes.c_uint32, _vp, _i, _u64]),
    "squaresort_batched_u32": (_i, [ctypes.c_uint32, _vp, _vp, _vp, _vp, _P, _vp]),
    "squaresort_batched_kv": (_i, [ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp, _vp, _P, _vp]),
    "squaresort_batched_graph_workspace_bytes": (_u64, [ctypes.c_uint32, _vp, _u64]),
    "squaresort_batched_graph_u32": (_i, [ctypes.c_uint32, _vp, _vp, _vp, _vp, _P, _vp, ctypes.POINTER(_vp)]),
    "sqs_plan_launch": (_i, [_vp, _vp]),
    "sqs_plan_destroy": (_i, [_vp]),
    "sqs_status_string": (ctypes.c_char_p, [_i]),
    "sqs_timing_enable": (_i, [_i]),
    "sqs_timing_report": (ctypes.c_int64, [ctypes.c_char_p, _u64]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class SquareSortError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)} ({_lib.sqs_status_string(status).decode()})")
        self.status = status


def _check(status: int, what: str):
    if status != 0:
        raise SquareSortError(status, what)


def max_cutoff(kind: int) -> int:
    return _lib.sqs_max_cutoff(kind)


def max_n(kind: int) -> int:
    return _lib.sqs_max_n(kind)


def workspace_bytes(n: int, kind: int, cutoff: int = 0) -> int:
    return _lib.squaresort_workspace_bytes(n, kind, cutoff)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Workspace:
    """Caller-owned device workspace, grown on demand (allocation happens
    here, outside the library)."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)
        return self.buf


def _params(n, kind, cutoff, ws, digest, pivot_rule="replacement", flags=0, tile=0):
    nbytes = workspace_bytes(n, kind, cutoff)
    buf = (ws or Workspace()).get(nbytes) if n > 0 else None
    p = Params()
    p.cutoff = cutoff
    p.flags = (FLAG_DIGEST if digest is not None else 0) | PIVOT_RULES[pivot_rule] | flags
    p.tile = tile
    p.workspace = None if buf is None else buf.data_ptr()
    p.workspace_bytes = 0 if buf is None else buf.numel()
    p.digest = None if digest is None else digest.data_ptr()
    return p, buf


def _check_dev(*ts, host=False):
    for t in ts:
        if host:
            if t.is_cuda or not t.is_pinned() or not t.is_contiguous():
                raise ValueError("host_arrays: tensors must be contiguous pinned host tensors")
        elif not t.is_cuda or not t.is_contiguous():
            raise ValueError("tensors must be contiguous device tensors")


def _stream_of(t):
    return _stream(t.device if t.is_cuda else torch.device("cuda", torch.cuda.current_device()))


def squaresort_u32(inp: torch.Tensor, out: torch.Tensor, seed: int = 1, cutoff: int = 0,
                   ws: Workspace | None = None, digest: torch.Tensor | None = None,
                   pivot_rule: str = "replacement", validate: bool = False, host_arrays: bool = False,
                   tile: int = 0) -> int:
    """Sort inp (uint32 bits in an int32 tensor; clobbered) into out.  Returns
    the cut-off used.  pivot_rule "alg1" selects the Alg. 1 pivot rule;
    validate sets SQS_FLAG_VALIDATE; host_arrays (SQS_FLAG_HOST_ARRAYS): inp
    and out are pinned host tensors, sorted in place there by the GPU."""
    _check_dev(inp, out, host=host_arrays)
    assert inp.dtype == torch.int32 and out.dtype == torch.int32 and inp.numel() == out.numel()
    n = inp.numel()
    fl = (FLAG_VALIDATE if validate else 0) | (FLAG_HOST_ARRAYS if host_arrays else 0)
    p, _keep = _params(n, KIND_U32, cutoff, ws, digest, pivot_rule, fl, tile)
    _check(_lib.squaresort_u32(n, _ptr(inp), _ptr(out), seed, ctypes.byref(p), _stream_of(inp)),
           "squaresort_u32")
    return p.cutoff


def squaresort_u32_noalloc(inp: torch.Tensor, out: torch.Tensor, seed: int = 1, cutoff: int = 0,
                           digest: torch.Tensor | None = None, pivot_rule: str = "replacement",
                           validate: bool = False) -> int:
    """squaresort_u32 with the library's static per-GPU scratch instead of a
    workspace (the call allocates nothing).  Returns the cut-off used."""
    _check_dev(inp, out)
    assert inp.dtype == torch.int32 and out.dtype == torch.int32 and inp.numel() == out.numel()
    p = Params()
    p.cutoff = cutoff
    p.flags = (FLAG_DIGEST if digest is not None else 0) | PIVOT_RULES[pivot_rule] | (FLAG_VALIDATE if validate else 0)
    p.digest = None if digest is None else digest.data_ptr()
    _check(_lib.squaresort_u32_noalloc(inp.numel(), _ptr(inp), _ptr(out), seed, ctypes.byref(p),
                                       _stream(inp.device)), "squaresort_u32_noalloc")
    return p.cutoff


def squaresort_u64(inp: torch.Tensor, out: torch.Tensor, seed: int = 1, cutoff: int = 0,
                   ws: Workspace | None = None, digest: torch.Tensor | None = None,
                   pivot_rule: str = "replacement", validate: bool = False) -> int:
    _check_dev(inp, out)
    assert inp.dtype == torch.int64 and out.dtype == torch.int64 and inp.numel() == out.numel()
    n = inp.numel()
    p, _keep = _params(n, KIND_U64, cutoff, ws, digest, pivot_rule, FLAG_VALIDATE if validate else 0)
    _check(_lib.squaresort_u64(n, _ptr(inp), _ptr(out), seed, ctypes.byref(p), _stream(inp.device)),
           "squaresort_u64")
    return p.cutoff


def squaresort_kv(keys_in, vals_in, keys_out, vals_out, seed: int = 1, cutoff: int = 0,
                  ws: Workspace | None = None, digest: torch.Tensor | None = None,
                  pivot_rule: str = "replacement", validate: bool = False, host_arrays: bool = False,
                  tile: int = 0) -> int:
    _check_dev(keys_in, vals_in, keys_out, vals_out, host=host_arrays)
    assert keys_in.dtype == torch.int64 and vals_in.dtype == torch.int32
    n = keys_in.numel()
    fl = (FLAG_VALIDATE if validate else 0) | (FLAG_HOST_ARRAYS if host_arrays else 0)
    p, _keep = _params(n, KIND_KV, cutoff, ws, digest, pivot_rule, fl, tile)
    _check(_lib.squaresort_kv(n, _ptr(keys_in), _ptr(vals_in), _ptr(keys_out), _ptr(vals_out), seed,
                              ctypes.byref(p), _stream_of(keys_in)), "squaresort_kv")
    return p.cutoff


def skew_transpose_u32(inp: torch.Tensor, out: torch.Tensor, bucket_start: torch.Tensor | None = None,
                       seed: int = 1, ws: Workspace | None = None, pivot_rule: str = "replacement",
                       validate: bool = False, cols_sorted: bool = False) -> None:
    """Root step up to SkewTranspose: columns of inp sorted in place (or,
    with cols_sorted, taken as given sorted), pivots drawn from the original
    inp, skew-transposed result in out.  validate checks the bucket bounds
    (and, with cols_sorted, that the columns are sorted)."""
    _check_dev(inp, out)
    n = inp.numel()
    fl = (FLAG_VALIDATE if validate else 0) | (FLAG_COLS_SORTED if cols_sorted else 0)
    p, _keep = _params(n, KIND_U32, 0, ws, None, pivot_rule, fl)
    _check(_lib.skew_transpose_u32(n, _ptr(inp), _ptr(out), _ptr(bucket_start), seed, ctypes.byref(p),
                                   _stream(inp.device)), "skew_transpose_u32")


def batched_offsets(sizes) -> "np.ndarray":
    """Host offsets (count+1, uint64) of instances packed back to back."""
    import numpy as np
    sizes = np.asarray(sizes, dtype=np.uint64)
    offs = np.zeros(sizes.size + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offs[1:])
    return offs


def batched_workspace_bytes(offsets, kind: int = KIND_U32, cutoff: int = 0) -> int:
    import numpy as np
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    return _lib.squaresort_batched_workspace_bytes(offs.size - 1, offs.ctypes.data, kind, cutoff)


def squaresort_batched_u32(inp: torch.Tensor, out: torch.Tensor, offsets, seeds, cutoff: int = 0,
                           ws: Workspace | None = None, digest: torch.Tensor | None = None,
                           tile: int = 0) -> int:
    """Sort the instances [offsets[i], offsets[i+1]) of inp (clobbered) into
    out, instance i with seeds[i] (host arrays); tile is the tile word
    (tile_word).  Returns the cut-off used."""
    import numpy as np
    _check_dev(inp, out)
    assert inp.dtype == torch.int32 and out.dtype == torch.int32 and inp.numel() == out.numel()
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    sd = np.ascontiguousarray(seeds, dtype=np.uint64)
    count = offs.size - 1
    assert sd.size == count and int(offs[-1]) == inp.numel()
    nbytes = batched_workspace_bytes(offs, KIND_U32, cutoff)
    buf = (ws or Workspace(inp.device)).get(nbytes)
    p = Params()
    p.cutoff = cutoff
    p.flags = FLAG_DIGEST if digest is not None else 0
    p.tile = tile
    p.workspace = buf.data_ptr()
    p.workspace_bytes = buf.numel()
    p.digest = None if digest is None else digest.data_ptr()
    _check(_lib.squaresort_batched_u32(count, offs.ctypes.data, _ptr(inp), _ptr(out), sd.ctypes.data,
                                       ctypes.byref(p), _stream(inp.device)), "squaresort_batched_u32")
    return p.cutoff


def squaresort_batched_kv(keys_in, vals_in, keys_out, vals_out, offsets, seeds, cutoff: int = 0,
                          ws: Workspace | None = None, digest: torch.Tensor | None = None,
                          tile: int = 0) -> int:
    """Key/value batched form (uint64 keys in int64 tensors, uint32 values in
    int32 tensors).  Returns the cut-off used."""
    import numpy as np
    _check_dev(keys_in, vals_in, keys_out, vals_out)
    assert keys_in.dtype == torch.int64 and vals_in.dtype == torch.int32
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    sd = np.ascontiguousarray(seeds, dtype=np.uint64)
    count = offs.size - 1
    assert sd.size == count and int(offs[-1]) == keys_in.numel()
    nbytes = batched_workspace_bytes(offs, KIND_KV, cutoff)
    buf = (ws or Workspace(keys_in.device)).get(nbytes)
    p = Params()
    p.cutoff = cutoff
    p.flags = FLAG_DIGEST if digest is not None else 0
    p.tile = tile
    p.workspace = buf.data_ptr()
    p.workspace_bytes = buf.numel()
    p.digest = None if digest is None else digest.data_ptr()
    _check(_lib.squaresort_batched_kv(count, offs.ctypes.data, _ptr(keys_in), _ptr(vals_in), _ptr(keys_out),
                                      _ptr(vals_out), sd.ctypes.data, ctypes.byref(p), _stream(keys_in.device)),
           "squaresort_batched_kv")
    return p.cutoff


STATUS_UNFINISHED, STATUS_DEVICE = 1, 2


def batched_graph_workspace_bytes(offsets, cutoff: int = 0) -> int:
    import numpy as np
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    return _lib.squaresort_batched_graph_workspace_bytes(offs.size - 1, offs.ctypes.data, cutoff)


class BatchedGraph:
    """squaresort_batched_graph_u32: the batched call planned once and
    captured into a HIP graph; launch() replays it on the current stream
    (sorting what inp holds then into out).  The buffers, workspace, digest
    and status tensors are bound to the plan and kept alive here."""

    def __init__(self, inp: torch.Tensor, out: torch.Tensor, offsets, seeds, cutoff: int = 0,
                 digest: torch.Tensor | None = None, tile: int = 0):
        import numpy as np
        _check_dev(inp, out)
        assert inp.dtype == torch.int32 and out.dtype == torch.int32 and inp.numel() == out.numel()
        self.offs = np.ascontiguousarray(offsets, dtype=np.uint64)
        self.seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
        count = self.offs.size - 1
        assert self.seeds.size == count and int(self.offs[-1]) == inp.numel()
        self.inp, self.out, self.digest = inp, out, digest
        self.ws = torch.empty(max(batched_graph_workspace_bytes(self.offs, cutoff), 1), dtype=torch.uint8,
                              device=inp.device)
        self.status = torch.zeros(1, dtype=torch.int32, device=inp.device)
        p = Params()
        p.cutoff = cutoff
        p.flags = FLAG_DIGEST if digest is not None else 0
        p.tile = tile
        p.workspace = self.ws.data_ptr()
        p.workspace_bytes = self.ws.numel()
        p.digest = None if digest is None else digest.data_ptr()
        torch.cuda.synchronize(inp.device)        # inputs and buffers ready before planning
        h = ctypes.c_void_p()
        _check(_lib.squaresort_batched_graph_u32(count, self.offs.ctypes.data, _ptr(inp), _ptr(out),
                                                 self.seeds.ctypes.data, ctypes.byref(p),
                                                 _ptr(self.status), ctypes.byref(h)), "squaresort_batched_graph_u32")
        self.handle = h
        self.cutoff = p.cutoff

    def launch(self) -> None:
        _check(_lib.sqs_plan_launch(self.handle, _stream(self.inp.device)), "sqs_plan_launch")

    def close(self) -> None:
        if getattr(self, "handle", None):
            _lib.sqs_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def timing_enable(on: bool = True) -> None:
    _lib.sqs_timing_enable(1 if on else 0)


def timing_report() -> dict:
    import json
    n = _lib.sqs_timing_report(None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    _lib.sqs_timing_report(buf, n + 1)
    return {k: {"ms": v[0], "launches": int(v[1]), "units": int(v[2])}
            for k, v in json.loads(buf.value.decode()).items()}


# raw entry points for tests that exercise the C ABI directly
lib = _lib
