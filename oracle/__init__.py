"""CPU oracle of SquareSort (arXiv 2407.14801) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it and shares no code with it.

The arithmetic lives in ``squaresort_oracle.c`` (plain C, built by
``oracle/build.py`` into ``liboracle.so``); this module only marshals numpy
arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

u64 = ctypes.c_uint64
u32 = ctypes.c_uint32
vp = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "orc_sm64": (u64, [u64]),
        "orc_root_key": (u64, [u64]),
        "orc_child_key": (u64, [u64, u32, u64]),
        "orc_draw_pos": (u64, [u64, u64, u64]),
        "orc_draw_pos_alg1": (u64, [u64, u64, u64, u64]),
        "orc_squaresort_rule": (ctypes.c_int, [u64, vp, vp, vp, vp, u64, u64, u64, ctypes.c_int, vp, vp]),
        "orc_root_pivots_alg1": (ctypes.c_int, [u64, vp, u64, vp, vp, vp]),
        "orc_tree_stats_rule": (ctypes.c_int, [u64, vp, u64, u64, ctypes.c_int, u64, vp, vp, vp]),
        "orc_ceil_isqrt": (u64, [u64]),
        "orc_squaresort": (ctypes.c_int, [u64, vp, vp, vp, vp, u64, u64, vp, vp]),
        "orc_squaresort_u32": (ctypes.c_int, [u64, vp, vp, u64, u64, vp, vp]),
        "orc_squaresort_u64": (ctypes.c_int, [u64, vp, vp, u64, u64, vp, vp]),
        "orc_squaresort_kv": (ctypes.c_int, [u64, vp, vp, vp, vp, u64, u64, vp, vp]),
        "orc_root_pivots": (ctypes.c_int, [u64, vp, u64, vp, vp]),
        "orc_bucket_of": (u64, [u64, vp, vp, u64]),
        "orc_skew_transpose_explicit": (ctypes.c_int, [u64, vp, vp, vp, vp, vp, vp, vp, u32]),
        "orc_root_intermediate": (ctypes.c_int, [u64, vp, vp, vp, vp, vp, u64]),
        "orc_tree_stats": (ctypes.c_int, [u64, vp, u64, u64, u64, vp, vp, vp]),
        "orc_root_buckets": (ctypes.c_int, [u64, vp, u64, u64, vp, vp, vp]),
        "orc_stable_sort": (ctypes.c_int, [u64, vp, vp]),
        "orc_set_threads": (None, [u32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


# ---- std::sort (the paper's comparator; CPU-baseline context) --------------
_cpusort = None


def _load_cpusort():
    global _cpusort
    if _cpusort is None:
        path = os.path.join(_HERE, "libcpusort.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        lib.orc_std_sort_u32.restype = None
        lib.orc_std_sort_u32.argtypes = [u64, vp]
        lib.orc_std_stable_sort_kv.restype = ctypes.c_int
        lib.orc_std_stable_sort_kv.argtypes = [u64, vp, vp]
        _cpusort = lib
    return _cpusort


def std_sort_u32(x: np.ndarray) -> np.ndarray:
    y = np.array(x, dtype=np.uint32)
    _load_cpusort().orc_std_sort_u32(y.size, _p(y))
    return y


def std_stable_sort_kv(keys: np.ndarray, vals: np.ndarray):
    k = np.array(keys, dtype=np.uint64)
    v = np.array(vals, dtype=np.uint32)
    _load_cpusort().orc_std_stable_sort_kv(k.size, _p(k), _p(v))
    return k, v


# ---- threads ------------------------------------------------------------
class threads:
    """Context manager: the root node's children (and the column sorts of
    root_intermediate) run on `p` threads inside the block.  The bytes and
    the digest are the same as on one thread."""

    def __init__(self, p: int):
        self.p = max(1, int(p))

    def __enter__(self):
        _load().orc_set_threads(self.p)
        return self

    def __exit__(self, *exc):
        _load().orc_set_threads(1)
        return False


# ---- generator --------------------------------------------------------
def sm64(x: int) -> int:
    return _load().orc_sm64(x)


def root_key(seed: int) -> int:
    return _load().orc_root_key(seed)


def child_key(K: int, phase: int, i: int) -> int:
    return _load().orc_child_key(K, phase, i)


def draw_pos(K: int, t: int, n: int) -> int:
    return _load().orc_draw_pos(K, t, n)


def ceil_isqrt(n: int) -> int:
    return _load().orc_ceil_isqrt(n)


def draw_pos_alg1(K: int, a: int, t: int, n: int) -> int:
    return _load().orc_draw_pos_alg1(K, a, t, n)


RULES = {"replacement": 0, "alg1": 1}
ALG1_ATTEMPTS = 64


def _sort_rule(keys, vals, seed, cutoff, key_max, rule):
    k = np.array(keys, dtype=np.uint64)
    v = None if vals is None else np.array(vals, dtype=np.uint32)
    ko = np.empty_like(k)
    vo = None if v is None else np.empty_like(v)
    dg, nd = u64(0), u64(0)
    rc = _load().orc_squaresort_rule(k.size, _p(k), _p(v), _p(ko), _p(vo), seed, cutoff, key_max,
                                     RULES[rule], ctypes.addressof(dg), ctypes.addressof(nd))
    _check(rc, f"squaresort ({rule} pivots)")
    return ko, vo, dg.value, nd.value


# ---- sorts --------------------------------------------------------------
def squaresort_u32(x: np.ndarray, seed: int, cutoff: int, want_digest=False, rule="replacement"):
    if rule != "replacement":
        ko, _, dg, nd = _sort_rule(np.asarray(x, dtype=np.uint32), None, seed, cutoff, 2**32 - 1, rule)
        out = ko.astype(np.uint32)
        return (out, dg, nd) if want_digest else out
    x = np.ascontiguousarray(x, dtype=np.uint32)
    out = np.empty_like(x)
    dg, nd = u64(0), u64(0)
    rc = _load().orc_squaresort_u32(x.size, _p(x), _p(out), seed, cutoff,
                                    ctypes.addressof(dg), ctypes.addressof(nd))
    _check(rc, "squaresort_u32")
    return (out, dg.value, nd.value) if want_digest else out


def squaresort_u64(x: np.ndarray, seed: int, cutoff: int, want_digest=False, rule="replacement"):
    if rule != "replacement":
        ko, _, dg, nd = _sort_rule(x, None, seed, cutoff, 2**64 - 1, rule)
        return (ko, dg, nd) if want_digest else ko
    x = np.ascontiguousarray(x, dtype=np.uint64)
    out = np.empty_like(x)
    dg, nd = u64(0), u64(0)
    rc = _load().orc_squaresort_u64(x.size, _p(x), _p(out), seed, cutoff,
                                    ctypes.addressof(dg), ctypes.addressof(nd))
    _check(rc, "squaresort_u64")
    return (out, dg.value, nd.value) if want_digest else out


def squaresort_kv(keys: np.ndarray, vals: np.ndarray, seed: int, cutoff: int,
                  want_digest=False, rule="replacement"):
    if rule != "replacement":
        ko, vo, dg, nd = _sort_rule(keys, vals, seed, cutoff, 2**64 - 1, rule)
        return (ko, vo, dg, nd) if want_digest else (ko, vo)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    vals = np.ascontiguousarray(vals, dtype=np.uint32)
    ko, vo = np.empty_like(keys), np.empty_like(vals)
    dg, nd = u64(0), u64(0)
    rc = _load().orc_squaresort_kv(keys.size, _p(keys), _p(vals), _p(ko), _p(vo), seed, cutoff,
                                   ctypes.addressof(dg), ctypes.addressof(nd))
    _check(rc, "squaresort_kv")
    return (ko, vo, dg.value, nd.value) if want_digest else (ko, vo)


def stable_sort(keys: np.ndarray, vals: np.ndarray | None = None):
    k = np.array(keys, dtype=np.uint64)
    v = None if vals is None else np.array(vals, dtype=np.uint32)
    _check(_load().orc_stable_sort(k.size, _p(k), _p(v)), "stable_sort")
    return k if v is None else (k, v)


# ---- pivots, buckets, SkewTranspose --------------------------------------
def root_pivots(keys: np.ndarray, seed: int):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    m = ceil_isqrt(keys.size)
    piv = np.empty(m - 1, np.uint64)
    strict = np.empty(m - 1, np.uint8)
    _check(_load().orc_root_pivots(keys.size, _p(keys), seed, _p(piv), _p(strict)), "root_pivots")
    return piv, strict


def root_pivots_alg1(keys: np.ndarray, seed: int):
    """Root pivots under the Alg. 1 rule: (pivots, strict flags, attempts)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    m = ceil_isqrt(keys.size)
    piv = np.empty(m - 1, np.uint64)
    strict = np.empty(m - 1, np.uint8)
    att = u64(0)
    _check(_load().orc_root_pivots_alg1(keys.size, _p(keys), seed, _p(piv), _p(strict), ctypes.addressof(att)),
           "root_pivots_alg1")
    return piv, strict, att.value


def bucket_of(x: int, piv: np.ndarray, strict: np.ndarray) -> int:
    piv = np.ascontiguousarray(piv, dtype=np.uint64)
    strict = np.ascontiguousarray(strict, dtype=np.uint8)
    return _load().orc_bucket_of(x, _p(piv), _p(strict), piv.size)


def skew_transpose_explicit(src_keys, pivots, strict, threshold=4, src_vals=None):
    sk = np.ascontiguousarray(src_keys, dtype=np.uint64)
    sv = None if src_vals is None else np.ascontiguousarray(src_vals, dtype=np.uint32)
    piv = np.ascontiguousarray(pivots, dtype=np.uint64)
    st = np.ascontiguousarray(strict, dtype=np.uint8)
    n = sk.size
    m = ceil_isqrt(n)
    assert piv.size == m - 1 and st.size == m - 1
    dk = np.empty_like(sk)
    dv = None if sv is None else np.empty_like(sv)
    bs = np.empty(m + 1, np.uint64)
    rc = _load().orc_skew_transpose_explicit(n, _p(sk), _p(sv), _p(dk), _p(dv), _p(piv), _p(st),
                                             _p(bs), threshold)
    _check(rc, "skew_transpose_explicit")
    return (dk, bs) if sv is None else (dk, dv, bs)


def root_intermediate(keys, seed, vals=None):
    """SquareSort's array A right after the root's SkewTranspose."""
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32)
    n = k.size
    m = ceil_isqrt(n)
    ko = np.empty_like(k)
    vo = None if v is None else np.empty_like(v)
    bs = np.empty(m + 1, np.uint64)
    _check(_load().orc_root_intermediate(n, _p(k), _p(v), _p(ko), _p(vo), _p(bs), seed),
           "root_intermediate")
    return (ko, bs) if v is None else (ko, vo, bs)


def tree_stats(keys, seed, cutoff, max_depth=16, rule="replacement"):
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    cnt = np.zeros(max_depth, np.uint64)
    ssum = np.zeros(max_depth, np.uint64)
    depth = u64(0)
    _check(_load().orc_tree_stats_rule(k.size, _p(k), seed, cutoff, RULES[rule], max_depth, _p(cnt),
                                       _p(ssum), ctypes.addressof(depth)), "tree_stats")
    return cnt, ssum, depth.value


def root_buckets(keys, seed, sel):
    """Bounds and keys of selected buckets of the root intermediate, without
    building the whole intermediate.  Returns (sel, bounds[nsel, 2], keys)."""
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    sel = np.ascontiguousarray(np.sort(np.unique(sel)), dtype=np.uint64)
    bounds = np.empty((sel.size, 2), np.uint64)
    _check(_load().orc_root_buckets(k.size, _p(k), seed, sel.size, _p(sel), _p(bounds), None),
           "root_buckets")
    total = int((bounds[:, 1] - bounds[:, 0]).sum())
    out = np.empty(max(total, 1), np.uint64)
    _check(_load().orc_root_buckets(k.size, _p(k), seed, sel.size, _p(sel), _p(bounds), _p(out)),
           "root_buckets")
    return sel, bounds, out[:total]
