"""The C-ABI library loads and exports every symbol its header declares; the
host-side argument checks return before any GPU work (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "squaresort.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int64_t|uint64_t|int|char|void)\s*\*?\s*(\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def b():
    from paper_2407_14801_amd import binding
    return binding


def test_every_declared_symbol_is_exported(b):
    names = _declared_functions()
    assert {"squaresort_u32", "squaresort_u64", "squaresort_kv", "skew_transpose_u32",
            "squaresort_workspace_bytes"} <= set(names)
    for name in names:
        assert hasattr(b.lib, name), name


def test_limits_and_workspace(b):
    for kind in (b.KIND_U32, b.KIND_U64, b.KIND_KV):
        assert b.max_cutoff(kind) >= 4096
        assert b.max_n(kind) >= 1 << 28
        small = b.workspace_bytes(1000, kind, 64)
        big = b.workspace_bytes(1 << 28, kind, 0)
        assert 0 < small < big
    assert b.max_cutoff(7) == 0 and b.workspace_bytes(10, 7, 0) == 0


def _params(cutoff=0, ws=None, nbytes=0):
    p = b_mod().Params()
    p.cutoff = cutoff
    p.workspace = ws
    p.workspace_bytes = nbytes
    return p


def b_mod():
    from paper_2407_14801_amd import binding
    return binding


def _call_u32(b, n, inp, out, p):
    return b.lib.squaresort_u32(n, inp, out, 1, ctypes.byref(p), None)


def test_argument_errors_before_gpu_work(b):
    fake_in, fake_out = 0x10000000, 0x20000000
    # n = 0 is a no-op even with null pointers
    assert _call_u32(b, 0, None, None, _params()) == 0
    # cut-off below 4 or above the maximum
    assert _call_u32(b, 10, fake_in, fake_out, _params(cutoff=3)) == -1
    assert _call_u32(b, 10, fake_in, fake_out, _params(cutoff=b.max_cutoff(0) + 1)) == -1
    # null pointers
    assert _call_u32(b, 10, None, fake_out, _params()) == -1
    # overlapping in/out
    assert _call_u32(b, 100, fake_in, fake_in + 8, _params()) == -2
    # too large
    assert _call_u32(b, b.max_n(0) + 1, fake_in, fake_out, _params()) == -7
    # internal node but no workspace
    n = b.max_cutoff(0) + 1
    assert _call_u32(b, n, fake_in, fake_in + 4 * n, _params()) == -3
    # cut-off echoed when automatic
    p = _params()
    assert _call_u32(b, 0, None, None, p) == 0 and p.cutoff == b.max_cutoff(0)
    # skew transpose needs n >= 2
    assert b.lib.skew_transpose_u32(1, fake_in, fake_out, None, 1, ctypes.byref(_params()), None) == -1
    assert b.lib.sqs_status_string(-3) == b"workspace missing or too small"


def test_batched_argument_errors_before_gpu_work(b):
    import numpy as np
    fake_in, fake_out = 0x10000000, 0x40000000

    def call(offs, seeds, inp=fake_in, out=fake_out, p=None):
        offs = np.ascontiguousarray(offs, dtype=np.uint64)
        seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
        p = p or _params()
        return b.lib.squaresort_batched_u32(offs.size - 1, offs.ctypes.data, inp, out,
                                            seeds.ctypes.data, ctypes.byref(p), None)

    # zero instances, or instances of total size 0, are no-ops
    assert b.lib.squaresort_batched_u32(0, None, None, None, None, ctypes.byref(_params()), None) == 0
    assert call([0, 0, 0], [1, 2], None, None) == 0
    # offsets must start at 0 and not decrease
    assert call([1, 5], [1]) == -1
    assert call([0, 9, 5], [1, 2]) == -1
    # one instance past the size limit, or a total of 2^32 keys or more
    assert call([0, b.max_n(0) + 1], [1]) == -7
    assert call([k << 28 for k in range(17)] + [(16 << 28) + 1], [1] * 17) == -7
    # overlapping input and output
    assert call([0, 100], [1], fake_in, fake_in + 64) == -2
    # workspace missing or too small; the size query agrees
    offs = np.array([0, 10, 200_000, 200_010], dtype=np.uint64)
    need = b.batched_workspace_bytes(offs)
    assert need > 0
    assert call(offs, [1, 2, 3]) == -3
    assert call(offs, [1, 2, 3], p=_params(ws=0x50000000, nbytes=need - 1)) == -3
    # base cases only: a list workspace, no batch metadata
    assert 0 < b.batched_workspace_bytes(np.array([0, 10, 20], dtype=np.uint64)) < need


def test_flag_errors_before_gpu_work(b):
    """Flags an entry point does not take are rejected before any GPU work:
    SQS_FLAG_COLS_SORTED outside skew_transpose_u32, the single-instance
    flags on the batched calls; SQS_FLAG_VALIDATE needs a workspace."""
    import numpy as np
    fake_in, fake_out = 0x10000000, 0x20000000
    p = _params()
    p.flags = b.FLAG_COLS_SORTED
    assert _call_u32(b, 100, fake_in, fake_out, p) == -1
    p = _params()
    p.flags = b.FLAG_VALIDATE
    assert _call_u32(b, 100, fake_in, fake_out, p) == -3
    offs = np.array([0, 10, 20], dtype=np.uint64)
    seeds = np.array([1, 2], dtype=np.uint64)
    for fl in (b.FLAG_VALIDATE, b.FLAG_COLS_SORTED):
        p = _params(ws=0x50000000, nbytes=1 << 30)
        p.flags = fl
        assert b.lib.squaresort_batched_u32(2, offs.ctypes.data, fake_in, fake_out, seeds.ctypes.data,
                                            ctypes.byref(p), None) == -1


def test_noalloc_argument_errors_before_gpu_work(b):
    """squaresort_u32_noalloc rejects a bad cut-off, and sizes whose scratch
    exceeds the static array, before it touches the GPU."""
    fake_in, fake_out = 0x10000000, 0x80000000
    lim = b.STATIC_SCRATCH_BYTES
    assert b.lib.squaresort_u32_noalloc(10, fake_in, fake_out, 1, ctypes.byref(_params(cutoff=3)), None) == -1
    assert b.workspace_bytes(1 << 24, b.KIND_U32, 0) <= lim < b.workspace_bytes(1 << 26, b.KIND_U32, 0)
    assert b.lib.squaresort_u32_noalloc(1 << 26, fake_in, fake_out, 1, ctypes.byref(_params()), None) == -3
    assert b.workspace_bytes(1 << 20, b.KIND_U32, 64) > lim
    assert b.lib.squaresort_u32_noalloc(1 << 20, fake_in, fake_out, 1, ctypes.byref(_params(cutoff=64)), None) == -3
    # params may be null (automatic cut-off): still rejected by size
    assert b.lib.squaresort_u32_noalloc(1 << 26, fake_in, fake_out, 1, None, None) == -3


def test_tile_word_errors_before_gpu_work(b):
    """Tile words with unknown bits or a field value of 3 are rejected before
    any GPU work; tile_word and tile_fields invert each other."""
    import numpy as np
    fake_in, fake_out = 0x10000000, 0x20000000
    offs = np.array([0, 10, 20], dtype=np.uint64)
    seeds = np.array([1, 2], dtype=np.uint64)
    for word in (3, 3 << 2, 3 << 4, 1 << 6, 1 << 31):
        p = _params()
        p.tile = word
        assert _call_u32(b, 100, fake_in, fake_out, p) == -1, word
        p = _params(ws=0x50000000, nbytes=1 << 30)
        p.tile = word
        assert b.lib.squaresort_batched_u32(2, offs.ctypes.data, fake_in, fake_out, seeds.ctypes.data,
                                            ctypes.byref(p), None) == -1, word
    for cw in (4, 2, 8):
        for wc in (1024, 512, 256):
            for m4 in (4096, 2048, 1024):
                assert b.tile_fields(b.tile_word(cw, wc, m4)) == {"colw": cw, "wcap": wc, "m4cap": m4}
    assert b.tile_word() == 0
