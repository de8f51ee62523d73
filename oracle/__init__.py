"""CPU oracle of the relational hot path: ctypes wrapper over oracle.c.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It never imports the product
package and the product never imports it; the two share only the seeded input
generator (module ``synth``).

Every function takes and returns numpy arrays (torch CPU tensors are accepted
and converted).  The C file holds the plain definitions; see its comments for
the passage of the paper each one follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_DIR, "oracle.c")
_LIB = os.path.join(_DIR, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, no -ffast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-Wno-implicit-fallthrough",
                               "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        L.or_fmix64.restype = C.c_uint64
        L.or_fmix64.argtypes = [C.c_uint64]
        L.or_murmur3_x64_128.argtypes = [C.c_void_p, C.c_int64, C.c_uint32, C.c_void_p]
        L.or_filter.restype = C.c_int64
        L.or_filter.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_int64,
                                C.c_void_p]
        L.or_partition.restype = C.c_int
        L.or_partition.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p]
        for f in (L.or_join_sortmerge, L.or_join_nested):
            f.restype = C.c_int64
            f.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                          C.c_void_p]
        for f in (L.or_groupby_sort, L.or_groupby_linear):
            f.restype = C.c_int64
            f.argtypes = [C.c_void_p, C.c_void_p]
        for f in (L.or_topk_sort, L.or_topk_select):
            f.restype = C.c_int64
            f.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int, C.c_void_p, C.c_void_p]
    return _lib


def _np(a, dtype=None):
    if a is None:
        return None
    if hasattr(a, "numpy"):
        a = a.detach().cpu().numpy()
    a = np.ascontiguousarray(a)
    if dtype is not None and a.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {a.dtype}")
    return a


def _p(a):
    return None if a is None else a.ctypes.data


def fmix64(k: int) -> int:
    return int(lib().or_fmix64(k & ((1 << 64) - 1)))


def murmur3_x64_128(data: bytes, seed: int) -> bytes:
    buf = C.create_string_buffer(data, len(data)) if data else C.create_string_buffer(1)
    out = (C.c_uint64 * 2)()
    lib().or_murmur3_x64_128(buf, len(data), seed, out)
    return int(out[0]).to_bytes(8, "little") + int(out[1]).to_bytes(8, "little")


def filter(col, lo: int, hi: int, sel_in=None):
    """Ascending row ids r (or entries of sel_in, in order) with lo <= col[r] < hi."""
    col = _np(col)
    assert col.dtype in (np.int32, np.int64)
    sel_in = _np(sel_in, np.int32)
    m = len(sel_in) if sel_in is not None else len(col)
    out = np.empty(max(m, 1), dtype=np.int32)
    cnt = lib().or_filter(_p(col), col.dtype.itemsize, len(col), lo, hi, _p(sel_in),
                          0 if sel_in is None else len(sel_in), _p(out))
    return out[:cnt].copy()


def partition(key, log2p: int, cols=()):
    """Stable hash partition; returns (key_out, [cols_out], rowid_out, offsets[P+1])."""
    key = _np(key, np.int64)
    cols = [_np(c) for c in cols]
    n = len(key)
    key_out = np.empty(n, dtype=np.int64)
    rowid = np.empty(n, dtype=np.int32)
    offsets = np.empty((1 << log2p) + 1, dtype=np.int64)
    outs = [np.empty_like(c) for c in cols]
    nc = len(cols)
    cin = (C.c_void_p * max(nc, 1))(*[_p(c) for c in cols])
    cout = (C.c_void_p * max(nc, 1))(*[_p(c) for c in outs])
    cb = (C.c_int32 * max(nc, 1))(*[c.dtype.itemsize for c in cols])
    rc = lib().or_partition(_p(key), n, log2p, nc, cin, cb, _p(key_out), cout, _p(rowid), _p(offsets))
    if rc != 0:
        raise MemoryError("oracle partition")
    return key_out, outs, rowid, offsets


class DuplicateKey(Exception):
    pass


def _join(fn, bkey, bpay, fk, sel):
    bkey = _np(bkey, np.int64)
    bpay = _np(bpay, np.int32)
    fk = _np(fk, np.int64)
    sel = _np(sel, np.int32)
    n = len(sel) if sel is not None else len(fk)
    prow = np.empty(max(n, 1), dtype=np.int32)
    pay = np.empty(max(n, 1), dtype=np.int32)
    cnt = fn(_p(bkey), _p(bpay), len(bkey), _p(fk), _p(sel), n, _p(prow), _p(pay))
    if cnt == -1:
        raise DuplicateKey("duplicate build key")
    if cnt < 0:
        raise MemoryError("oracle join")
    return prow[:cnt].copy(), pay[:cnt].copy()


def join(bkey, bpay, fk, sel=None):
    """Inner equi-join (sort-merge); (probe row, payload) pairs in probe order."""
    return _join(lib().or_join_sortmerge, bkey, bpay, fk, sel)


def join_nested(bkey, bpay, fk, sel=None):
    """Brute-force nested-loop join, for tiny inputs."""
    return _join(lib().or_join_nested, bkey, bpay, fk, sel)


class _GbIn(C.Structure):
    _fields_ = [("n", C.c_int64), ("rowid", C.c_void_p),
                ("key64", C.c_void_p), ("key64_by_rowid", C.c_int),
                ("key32", C.c_void_p), ("key32_by_rowid", C.c_int),
                ("qty", C.c_void_p), ("price", C.c_void_p), ("disc", C.c_void_p), ("rev_scale", C.c_int64)]


class _GbOut(C.Structure):
    _fields_ = [("key64", C.c_void_p), ("key32", C.c_void_p), ("count", C.c_void_p), ("sum_qty", C.c_void_p),
                ("sum_rev_lo", C.c_void_p), ("sum_rev_hi", C.c_void_p), ("avg_qty", C.c_void_p),
                ("avg_rev", C.c_void_p), ("cap", C.c_int64)]


def _groupby(fn, n, rowid, key64, key64_by_rowid, key32, key32_by_rowid, qty, price, disc, rev_scale, cap):
    rowid = _np(rowid, np.int32)
    key64 = _np(key64, np.int64)
    key32 = _np(key32, np.int32)
    qty, price, disc = _np(qty, np.int64), _np(price, np.int64), _np(disc, np.int64)
    if cap is None:
        cap = max(n, 1)
    out = {
        "key64": np.zeros(cap, np.int64) if key64 is not None else None,
        "key32": np.zeros(cap, np.int32) if key32 is not None else None,
        "count": np.zeros(cap, np.int64), "sum_qty": np.zeros(cap, np.int64),
        "sum_rev_lo": np.zeros(cap, np.uint64), "sum_rev_hi": np.zeros(cap, np.int64),
        "avg_qty": np.zeros(cap, np.float64), "avg_rev": np.zeros(cap, np.float64),
    }
    gi = _GbIn(n, _p(rowid), _p(key64), int(key64_by_rowid), _p(key32), int(key32_by_rowid),
               _p(qty), _p(price), _p(disc), rev_scale)
    go = _GbOut(_p(out["key64"]), _p(out["key32"]), _p(out["count"]), _p(out["sum_qty"]),
                _p(out["sum_rev_lo"]), _p(out["sum_rev_hi"]), _p(out["avg_qty"]), _p(out["avg_rev"]), cap)
    g = fn(C.byref(gi), C.byref(go))
    if g == -1:
        raise OverflowError("more groups than the capacity")
    if g < 0:
        raise MemoryError("oracle group-by")
    return {k: (v[:g].copy() if v is not None else None) for k, v in out.items()}


def groupby(n, qty, price, disc, rowid=None, key64=None, key64_by_rowid=False, key32=None,
            key32_by_rowid=False, rev_scale=100, cap=None):
    """Exact group-by aggregate, groups in ascending (key64, key32) order."""
    return _groupby(lib().or_groupby_sort, n, rowid, key64, key64_by_rowid, key32, key32_by_rowid,
                    qty, price, disc, rev_scale, cap)


def groupby_linear(n, qty, price, disc, rowid=None, key64=None, key64_by_rowid=False, key32=None,
                   key32_by_rowid=False, rev_scale=100, cap=None):
    """Brute-force group-by (linear group list), groups in first-seen order."""
    return _groupby(lib().or_groupby_linear, n, rowid, key64, key64_by_rowid, key32, key32_by_rowid,
                    qty, price, disc, rev_scale, cap)


def sum_rev_int(g: dict) -> list[int]:
    """The 128-bit revenue sums of a group result as Python ints."""
    lo = g["sum_rev_lo"].astype(np.uint64)
    hi = g["sum_rev_hi"].astype(np.int64)
    return [(int(h) << 64) + int(lo_) for lo_, h in zip(lo.tolist(), hi.tolist())]


def _topk(fn, val, sel, k, descending):
    val = _np(val, np.int64)
    sel = _np(sel, np.int32)
    n = len(sel) if sel is not None else len(val)
    vo = np.empty(max(k, 1), np.int64)
    ro = np.empty(max(k, 1), np.int32)
    cnt = fn(_p(val), _p(sel), n, k, int(descending), _p(vo), _p(ro))
    if cnt < 0:
        raise MemoryError("oracle top-k")
    return vo[:cnt].copy(), ro[:cnt].copy()


def topk(val, k, sel=None, descending=True):
    """(values, row ids) of the top-k selected rows; ties by ascending row id."""
    return _topk(lib().or_topk_sort, val, sel, k, descending)


def topk_select(val, k, sel=None, descending=True):
    """Brute-force top-k by repeated selection, for tiny inputs."""
    return _topk(lib().or_topk_select, val, sel, k, descending)


def pipeline(fact: dict, dim: dict, date_hi: int, rev_scale: int = 100, with_topk: int = 0):
    """filter(date < date_hi) -> join(fk = dim.key, payload dim.attr) -> group by attr
    (count, sum qty, sum revenue, averages) [-> top-k of price over the selection]."""
    sel = filter(fact["date"], -(1 << 31), date_hi)
    prow, pay = join(dim["key"], dim["attr"], fact["fk"], sel)
    g = groupby(len(prow), fact["qty"], fact["price"], fact["disc"], rowid=prow, key32=pay,
                rev_scale=rev_scale)
    out = {"sel": sel, "prow": prow, "payload": pay, "groups": g}
    if with_topk:
        out["topk"] = topk(fact["price"], with_topk, sel=sel)
    return out
