"""Python binding of libgq.so, the MI355X relational hot path.

Argument marshalling only: every step runs in the HIP kernels behind the C ABI
declared in include/gq.h.  Functions carry the C names (gq_filter,
gq_radix_partition, gq_join_build, gq_join_probe, gq_groupby_agg, gq_topk) and
take torch tensors that must live on a HIP device; PyTorch provides device
memory and the current stream, nothing else.  There is no CPU fallback: if
the library is missing, or a tensor is on the CPU, the call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgq.so")

GQ_OK = 0
GQ_ERR_INVALID_ARG = 1
GQ_ERR_CAPACITY = 2
GQ_ERR_WORKSPACE = 3
GQ_ERR_DUPLICATE_KEY = 4
GQ_ERR_HIP = 5
GQ_ERR_UNSUPPORTED = 6
GQ_ERR_INVALID_KEY = 7
GQ_ERR_TIMEOUT = 8
_NAMES = {0: "GQ_OK", 1: "GQ_ERR_INVALID_ARG", 2: "GQ_ERR_CAPACITY", 3: "GQ_ERR_WORKSPACE",
          4: "GQ_ERR_DUPLICATE_KEY", 5: "GQ_ERR_HIP", 6: "GQ_ERR_UNSUPPORTED", 7: "GQ_ERR_INVALID_KEY",
          8: "GQ_ERR_TIMEOUT"}

GQ_I32, GQ_I64 = 4, 8

EXPORTED = [
    "gq_ctx_create", "gq_ctx_destroy", "gq_last_error", "gq_status_word", "gq_set_wait_limit", "gq_set_timing",
    "gq_kernel_time",
    "gq_reset_timing", "gq_filter_workspace_bytes", "gq_filter", "gq_filter_noalloc",
    "gq_radix_partition_workspace_bytes",
    "gq_radix_partition", "gq_join_table_bytes", "gq_join_build_workspace_bytes", "gq_join_build", "gq_join_probe_workspace_bytes",
    "gq_join_probe_partitioned_workspace_bytes", "gq_join_probe_partitioned",
    "gq_join_probe", "gq_groupby_workspace_bytes", "gq_groupby_agg", "gq_topk_workspace_bytes", "gq_topk",
    "gq_default_tuning", "gq_batch_workspace_bytes", "gq_batch_join_agg", "gq_batch_autotune_workspace_bytes",
    "gq_batch_autotune", "gq_server_create", "gq_server_submit", "gq_server_wait", "gq_server_stats",
    "gq_server_destroy",
]

GQ_QUERY_FILTER_AGG, GQ_QUERY_JOIN_AGG, GQ_QUERY_JOIN2_AGG, GQ_QUERY_FILTER_TOPK = 1, 2, 3, 4


class GQError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class GroupbyIn(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_dev", C.c_void_p), ("rowid", C.c_void_p),
                ("key64", C.c_void_p), ("key64_by_rowid", C.c_int32),
                ("key32", C.c_void_p), ("key32_by_rowid", C.c_int32),
                ("qty", C.c_void_p), ("price", C.c_void_p), ("disc", C.c_void_p), ("rev_scale", C.c_int64),
                ("filter", C.c_void_p), ("filter_lo", C.c_int64), ("filter_hi", C.c_int64)]


class Groups(C.Structure):
    _fields_ = [("key64", C.c_void_p), ("key32", C.c_void_p), ("count", C.c_void_p), ("sum_qty", C.c_void_p),
                ("sum_rev_lo", C.c_void_p), ("sum_rev_hi", C.c_void_p), ("avg_qty", C.c_void_p),
                ("avg_rev", C.c_void_p), ("n_groups", C.c_void_p), ("capacity", C.c_int64)]


class Instance(C.Structure):
    _fields_ = [("dim_key", C.c_void_p), ("dim_attr", C.c_void_p), ("m", C.c_int64),
                ("fk", C.c_void_p), ("date", C.c_void_p), ("qty", C.c_void_p), ("price", C.c_void_p),
                ("disc", C.c_void_p), ("n", C.c_int64), ("date_lo", C.c_int64), ("date_hi", C.c_int64),
                ("rev_scale", C.c_int64), ("out", Groups)]


class ServerTables(C.Structure):
    _fields_ = [("fk", C.c_void_p), ("fk2", C.c_void_p), ("date", C.c_void_p), ("qty", C.c_void_p),
                ("price", C.c_void_p), ("disc", C.c_void_p), ("n", C.c_int64), ("dim1_table", C.c_void_p),
                ("dim1_table_bytes", C.c_size_t), ("dim2_table", C.c_void_p), ("dim2_table_bytes", C.c_size_t)]


class ServerCfg(C.Structure):
    _fields_ = [("tables", ServerTables), ("pool", C.c_void_p), ("pool_bytes", C.c_size_t),
                ("streams", C.c_int32), ("max_batch", C.c_int32), ("serial", C.c_int32)]


class Query(C.Structure):
    _fields_ = [("kind", C.c_int32), ("k", C.c_int32), ("date_hi", C.c_int64), ("max_groups", C.c_int64),
                ("groups", Groups), ("topk_val", C.c_void_p), ("topk_row", C.c_void_p), ("topk_n", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("load_factor", C.c_double), ("probe_tile", C.c_int32), ("build_tile", C.c_int32),
                ("init_tile", C.c_int32), ("lag", C.c_int32), ("fanout", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """The loaded libgq.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2506_09226_amd.build`")
        L = C.CDLL(LIB_PATH)
        st, vp, i64, i32, sz = C.c_int32, C.c_void_p, C.c_int64, C.c_int, C.c_size_t
        L.gq_ctx_create.restype = st
        L.gq_ctx_create.argtypes = [i32, C.POINTER(vp)]
        L.gq_ctx_destroy.restype = None
        L.gq_ctx_destroy.argtypes = [vp]
        L.gq_last_error.restype = C.c_char_p
        L.gq_last_error.argtypes = [vp]
        L.gq_status_word.restype = st
        L.gq_status_word.argtypes = [vp, vp, C.POINTER(C.c_int32)]
        L.gq_set_wait_limit.restype = st
        L.gq_set_wait_limit.argtypes = [vp, i64]
        L.gq_set_timing.restype = st
        L.gq_set_timing.argtypes = [vp, i32]
        L.gq_kernel_time.restype = st
        L.gq_kernel_time.argtypes = [vp, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.gq_reset_timing.restype = st
        L.gq_reset_timing.argtypes = [vp]
        L.gq_filter_workspace_bytes.restype = sz
        L.gq_filter_workspace_bytes.argtypes = [i64]
        L.gq_filter.restype = st
        L.gq_filter.argtypes = [vp, vp, i32, i64, vp, vp, i64, i64, vp, vp, vp, sz, vp]
        L.gq_filter_noalloc.restype = st
        L.gq_filter_noalloc.argtypes = [vp, vp, i32, i64, vp, vp, i64, i64, vp, vp, vp]
        L.gq_radix_partition_workspace_bytes.restype = sz
        L.gq_radix_partition_workspace_bytes.argtypes = [i64, i32]
        L.gq_radix_partition.restype = st
        L.gq_radix_partition.argtypes = [vp, vp, i64, i32, i32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.gq_join_table_bytes.restype = sz
        L.gq_join_table_bytes.argtypes = [i64, C.c_double]
        L.gq_join_build_workspace_bytes.restype = sz
        L.gq_join_build_workspace_bytes.argtypes = [i64, sz]
        L.gq_join_build.restype = st
        L.gq_join_build.argtypes = [vp, vp, vp, i64, vp, vp, vp, sz, vp, sz, vp]
        L.gq_join_probe_workspace_bytes.restype = sz
        L.gq_join_probe_workspace_bytes.argtypes = [i64]
        L.gq_join_probe.restype = st
        L.gq_join_probe.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, sz, vp]
        L.gq_join_probe_partitioned_workspace_bytes.restype = sz
        L.gq_join_probe_partitioned_workspace_bytes.argtypes = [i64]
        L.gq_join_probe_partitioned.restype = st
        L.gq_join_probe_partitioned.argtypes = [vp, vp, sz, vp, i64, vp, vp, i32, vp, vp, vp, vp, sz, vp]
        L.gq_groupby_workspace_bytes.restype = sz
        L.gq_groupby_workspace_bytes.argtypes = [i64, i64, i32, i32]
        L.gq_groupby_agg.restype = st
        L.gq_groupby_agg.argtypes = [vp, C.POINTER(GroupbyIn), i64, C.POINTER(Groups), vp, sz, vp]
        L.gq_topk_workspace_bytes.restype = sz
        L.gq_topk_workspace_bytes.argtypes = [i64, i32]
        L.gq_topk.restype = st
        L.gq_topk.argtypes = [vp, vp, vp, i64, vp, i32, i32, vp, vp, vp, vp, sz, vp]
        L.gq_default_tuning.restype = Tuning
        L.gq_default_tuning.argtypes = []
        L.gq_batch_workspace_bytes.restype = sz
        L.gq_batch_workspace_bytes.argtypes = [C.POINTER(Instance), i32, C.POINTER(Tuning)]
        L.gq_batch_join_agg.restype = st
        L.gq_batch_join_agg.argtypes = [vp, C.POINTER(Instance), i32, C.POINTER(Tuning), vp, vp, sz, vp]
        L.gq_batch_autotune_workspace_bytes.restype = sz
        L.gq_batch_autotune_workspace_bytes.argtypes = [C.POINTER(Instance), i32]
        L.gq_batch_autotune.restype = st
        L.gq_batch_autotune.argtypes = [vp, C.POINTER(Instance), i32, C.c_char_p, C.POINTER(Tuning),
                                        C.POINTER(C.c_double), vp, sz, vp]
        L.gq_server_create.restype = st
        L.gq_server_create.argtypes = [vp, C.POINTER(ServerCfg), C.POINTER(vp)]
        L.gq_server_submit.restype = st
        L.gq_server_submit.argtypes = [vp, C.POINTER(Query), C.POINTER(C.c_uint64)]
        L.gq_server_wait.restype = st
        L.gq_server_wait.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.gq_server_stats.restype = st
        L.gq_server_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]
        L.gq_server_destroy.restype = None
        L.gq_server_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda":
        raise TypeError("tensor must be on a HIP device (no CPU path)")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


class Context:
    """A gq_ctx on one device.  Not thread-safe: use one per host thread."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        rc = lib().gq_ctx_create(device, C.byref(h))
        if rc != GQ_OK:
            raise GQError(rc, "gq_ctx_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().gq_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int):
        if rc != GQ_OK:
            raise GQError(rc, lib().gq_last_error(self.handle).decode())

    def status(self) -> int:
        """Synchronize the current stream; return (and clear) the device status word."""
        out = C.c_int32()
        self.check(lib().gq_status_word(self.handle, _stream(self.device), C.byref(out)))
        return out.value

    def raise_status(self):
        s = self.status()
        if s != GQ_OK:
            raise GQError(s, "device-side error")

    def set_timing(self, on: bool):
        self.check(lib().gq_set_timing(self.handle, int(on)))

    def kernel_time(self, name: str):
        n, ms = C.c_int64(), C.c_double()
        self.check(lib().gq_kernel_time(self.handle, name.encode(), C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def reset_timing(self):
        self.check(lib().gq_reset_timing(self.handle))

    def set_wait_limit(self, polls: int):
        """Bound of device-side waits in polls (0 = the default); see gq.h."""
        self.check(lib().gq_set_wait_limit(self.handle, int(polls)))

    def workspace(self, nbytes: int) -> torch.Tensor:
        return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)


def _i64_scalar(ctx):
    return torch.zeros(1, dtype=torch.int64, device=ctx.device)


def gq_filter(ctx: Context, col, lo: int, hi: int, sel_in=None, n: int | None = None, n_dev=None,
              out=None, n_out=None, ws=None):
    """Selection vector of rows with lo <= col[r] < hi (see gq.h)."""
    dtype = {torch.int32: GQ_I32, torch.int64: GQ_I64}[col.dtype]
    if n is None:
        n = sel_in.numel() if sel_in is not None else col.numel()
    out = out if out is not None else torch.empty(max(n, 1), dtype=torch.int32, device=ctx.device)
    n_out = n_out if n_out is not None else _i64_scalar(ctx)
    need = lib().gq_filter_workspace_bytes(n)
    ws = ws if ws is not None else ctx.workspace(need)
    ctx.check(lib().gq_filter(ctx.handle, _ptr(col), dtype, n, _ptr(n_dev), _ptr(sel_in), lo, hi, _ptr(out),
                              _ptr(n_out), _ptr(ws), ws.numel(), _stream(ctx.device)))
    return out, n_out


def gq_filter_noalloc(ctx: Context, col, lo: int, hi: int, out, n_out, sel_in=None, n: int | None = None,
                      n_dev=None):
    """gq_filter with the library's static scratch instead of a workspace: the
    caller passes preallocated outputs, nothing is allocated."""
    dtype = {torch.int32: GQ_I32, torch.int64: GQ_I64}[col.dtype]
    if n is None:
        n = sel_in.numel() if sel_in is not None else col.numel()
    ctx.check(lib().gq_filter_noalloc(ctx.handle, _ptr(col), dtype, n, _ptr(n_dev), _ptr(sel_in), lo, hi, _ptr(out),
                                      _ptr(n_out), _stream(ctx.device)))
    return out, n_out


def gq_radix_partition(ctx: Context, key, log2_fanout: int, cols=(), rowid: bool = True, outs=None, ws=None):
    """Stable hash partition; returns (key_out, cols_out, rowid_out, offsets[P+1])."""
    n = key.numel()
    cols = list(cols)
    if outs is None:
        key_out = torch.empty_like(key)
        cols_out = [torch.empty_like(c) for c in cols]
        rowid_out = torch.empty(n, dtype=torch.int32, device=ctx.device) if rowid else None
        offsets = torch.empty((1 << log2_fanout) + 1, dtype=torch.int64, device=ctx.device)
    else:
        key_out, cols_out, rowid_out, offsets = outs
    nc = len(cols)
    cin = (C.c_void_p * max(nc, 1))(*[_ptr(c) for c in cols])
    cout = (C.c_void_p * max(nc, 1))(*[_ptr(c) for c in cols_out])
    cb = (C.c_int32 * max(nc, 1))(*[c.element_size() for c in cols])
    need = lib().gq_radix_partition_workspace_bytes(n, log2_fanout)
    ws = ws if ws is not None else ctx.workspace(need)
    ctx.check(lib().gq_radix_partition(ctx.handle, _ptr(key), n, log2_fanout, nc, cin, cb, _ptr(key_out), cout,
                                       _ptr(rowid_out), _ptr(offsets), _ptr(ws), ws.numel(), _stream(ctx.device)))
    return key_out, cols_out, rowid_out, offsets


def gq_join_table_bytes(m: int, load_factor: float = 0.5) -> int:
    return int(lib().gq_join_table_bytes(m, load_factor))


def gq_join_build(ctx: Context, key, payload, m: int | None = None, n_dev=None, sel=None, table=None,
                  load_factor: float = 0.5, ws=None):
    """Build the join hash table; returns the table tensor (device bytes)."""
    if m is None:
        m = sel.numel() if sel is not None else key.numel()
    if table is None:
        table = torch.empty(gq_join_table_bytes(m, load_factor), dtype=torch.uint8, device=ctx.device)
    if ws is None:
        ws = ctx.workspace(lib().gq_join_build_workspace_bytes(m, table.numel()))
    ctx.check(lib().gq_join_build(ctx.handle, _ptr(key), _ptr(payload), m, _ptr(n_dev), _ptr(sel), _ptr(table),
                                  table.numel(), _ptr(ws), ws.numel(), _stream(ctx.device)))
    return table


def gq_join_probe(ctx: Context, table, fk, sel=None, n: int | None = None, n_dev=None, prow=None, payload=None,
                  n_out=None, ws=None):
    """Probe; returns (prow_out, payload_out, n_out) in probe order."""
    if n is None:
        n = sel.numel() if sel is not None else fk.numel()
    prow = prow if prow is not None else torch.empty(max(n, 1), dtype=torch.int32, device=ctx.device)
    payload = payload if payload is not None else torch.empty(max(n, 1), dtype=torch.int32, device=ctx.device)
    n_out = n_out if n_out is not None else _i64_scalar(ctx)
    need = lib().gq_join_probe_workspace_bytes(n)
    ws = ws if ws is not None else ctx.workspace(need)
    ctx.check(lib().gq_join_probe(ctx.handle, _ptr(table), _ptr(fk), n, _ptr(n_dev), _ptr(sel), _ptr(prow),
                                  _ptr(payload), _ptr(n_out), _ptr(ws), ws.numel(), _stream(ctx.device)))
    return prow, payload, n_out


def gq_join_probe_partitioned(ctx: Context, table, fk, sel=None, n: int | None = None, n_dev=None,
                              log2_fanout: int = 0, prow=None, payload=None, n_out=None, ws=None):
    """Partitioned (LDS region) probe; returns (prow_out, payload_out, n_out),
    identical to gq_join_probe's output.  log2_fanout: radix bits of the hash
    partition the probe stream is in (0 if none)."""
    if n is None:
        n = sel.numel() if sel is not None else fk.numel()
    prow = prow if prow is not None else torch.empty(max(n, 1), dtype=torch.int32, device=ctx.device)
    payload = payload if payload is not None else torch.empty(max(n, 1), dtype=torch.int32, device=ctx.device)
    n_out = n_out if n_out is not None else _i64_scalar(ctx)
    need = lib().gq_join_probe_partitioned_workspace_bytes(n)
    ws = ws if ws is not None else ctx.workspace(need)
    ctx.check(lib().gq_join_probe_partitioned(ctx.handle, _ptr(table), table.numel() * table.element_size(),
                                              _ptr(fk), n, _ptr(n_dev), _ptr(sel), int(log2_fanout), _ptr(prow),
                                              _ptr(payload), _ptr(n_out), _ptr(ws), ws.numel(),
                                              _stream(ctx.device)))
    return prow, payload, n_out


@dataclass
class GroupResult:
    key64: torch.Tensor | None
    key32: torch.Tensor | None
    count: torch.Tensor
    sum_qty: torch.Tensor
    sum_rev_lo: torch.Tensor      # int64 tensor holding the unsigned low word's bits
    sum_rev_hi: torch.Tensor
    avg_qty: torch.Tensor
    avg_rev: torch.Tensor
    n_groups: torch.Tensor

    def host(self) -> dict:
        """Copy the first n_groups entries to host numpy arrays."""
        g = int(self.n_groups.item())
        out = {}
        for f in ("key64", "key32", "count", "sum_qty", "sum_rev_lo", "sum_rev_hi", "avg_qty", "avg_rev"):
            t = getattr(self, f)
            out[f] = None if t is None else t[:g].cpu().numpy()
        if out["sum_rev_lo"] is not None:
            out["sum_rev_lo"] = out["sum_rev_lo"].view("uint64")
        return out


def alloc_groups(ctx: Context, capacity: int, key64: bool, key32: bool) -> GroupResult:
    d = ctx.device
    e = lambda dt: torch.empty(capacity, dtype=dt, device=d)
    return GroupResult(e(torch.int64) if key64 else None, e(torch.int32) if key32 else None, e(torch.int64),
                       e(torch.int64), e(torch.int64), e(torch.int64), e(torch.float64), e(torch.float64),
                       torch.zeros(1, dtype=torch.int64, device=d))


def gq_groupby_agg(ctx: Context, qty, price, disc, n: int | None = None, n_dev=None, rowid=None, key64=None,
                   key64_by_rowid=False, key32=None, key32_by_rowid=False, rev_scale: int = 100,
                   max_groups: int = 1024, out: GroupResult | None = None, ws=None, filter_col=None,
                   filter_lo: int = 0, filter_hi: int = 0) -> GroupResult:
    """Exact group-by aggregate (see gq.h); returns device arrays + n_groups."""
    if n is None:
        n = rowid.numel() if rowid is not None else qty.numel()
    out = out if out is not None else alloc_groups(ctx, max_groups, key64 is not None, key32 is not None)
    gi = GroupbyIn(n, _ptr(n_dev), _ptr(rowid), _ptr(key64), int(key64_by_rowid), _ptr(key32), int(key32_by_rowid),
                   _ptr(qty), _ptr(price), _ptr(disc), rev_scale, _ptr(filter_col), filter_lo, filter_hi)
    go = Groups(_ptr(out.key64), _ptr(out.key32), _ptr(out.count), _ptr(out.sum_qty), _ptr(out.sum_rev_lo),
                _ptr(out.sum_rev_hi), _ptr(out.avg_qty), _ptr(out.avg_rev), _ptr(out.n_groups), out.count.numel())
    need = lib().gq_groupby_workspace_bytes(n, max_groups, int(key64 is not None), int(key32 is not None))
    ws = ws if ws is not None else ctx.workspace(need)
    ctx.check(lib().gq_groupby_agg(ctx.handle, C.byref(gi), max_groups, C.byref(go), _ptr(ws), ws.numel(),
                                   _stream(ctx.device)))
    return out


def gq_topk(ctx: Context, val, k: int, sel=None, n: int | None = None, n_dev=None, descending: bool = True,
            val_out=None, rowid_out=None, n_out=None, ws=None):
    """Top-k rows by value, ties by ascending row id; returns (val, rowid, n_out)."""
    if n is None:
        n = sel.numel() if sel is not None else val.numel()
    val_out = val_out if val_out is not None else torch.empty(k, dtype=torch.int64, device=ctx.device)
    rowid_out = rowid_out if rowid_out is not None else torch.empty(k, dtype=torch.int32, device=ctx.device)
    n_out = n_out if n_out is not None else _i64_scalar(ctx)
    need = lib().gq_topk_workspace_bytes(n, k)
    ws = ws if ws is not None else ctx.workspace(need)
    ctx.check(lib().gq_topk(ctx.handle, _ptr(val), _ptr(sel), n, _ptr(n_dev), k, int(descending), _ptr(val_out),
                            _ptr(rowid_out), _ptr(n_out), _ptr(ws), ws.numel(), _stream(ctx.device)))
    return val_out, rowid_out, n_out


def _groups_struct(g: GroupResult) -> Groups:
    return Groups(_ptr(g.key64), _ptr(g.key32), _ptr(g.count), _ptr(g.sum_qty), _ptr(g.sum_rev_lo),
                  _ptr(g.sum_rev_hi), _ptr(g.avg_qty), _ptr(g.avg_rev), _ptr(g.n_groups), g.count.numel())


def make_instances(specs) -> "C.Array":
    """specs: dicts with dim_key, dim_attr, fk, date, qty, price, disc (tensors),
    date_lo, date_hi, rev_scale and out (GroupResult with key32)."""
    arr = (Instance * len(specs))()
    for i, sp in enumerate(specs):
        arr[i] = Instance(_ptr(sp["dim_key"]), _ptr(sp["dim_attr"]), sp["dim_key"].numel(),
                          _ptr(sp["fk"]), _ptr(sp["date"]), _ptr(sp["qty"]), _ptr(sp["price"]), _ptr(sp["disc"]),
                          sp["fk"].numel(), sp["date_lo"], sp["date_hi"], sp.get("rev_scale", 100),
                          _groups_struct(sp["out"]))
    return arr


def gq_default_tuning() -> Tuning:
    return lib().gq_default_tuning()


def gq_batch_join_agg(ctx: Context, instances, tuning: Tuning | None = None, ws=None, inst_status=None):
    """Run all instances (a ctypes Instance array) in one persistent launch.
    inst_status (optional device int32[n]) receives each instance's status."""
    n = len(instances)
    tp = C.byref(tuning) if tuning is not None else None
    need = lib().gq_batch_workspace_bytes(instances, n, tp)
    if need == 0:
        raise GQError(GQ_ERR_INVALID_ARG, "invalid batch or tuning")
    ws = ws if ws is not None else ctx.workspace(need)
    if inst_status is not None and (inst_status.dtype != torch.int32 or inst_status.numel() < n):
        raise ValueError("inst_status must be a device int32 tensor with one entry per instance")
    ctx.check(lib().gq_batch_join_agg(ctx.handle, instances, n, tp, _ptr(inst_status), _ptr(ws), ws.numel(),
                                      _stream(ctx.device)))
    return ws


def gq_batch_autotune(ctx: Context, instances, cache_path: str | None = None, ws=None):
    """Fastest candidate tuning for these instances; returns (Tuning, ms)."""
    n = len(instances)
    need = lib().gq_batch_autotune_workspace_bytes(instances, n)
    ws = ws if ws is not None else ctx.workspace(need)
    best, ms = Tuning(), C.c_double()
    ctx.check(lib().gq_batch_autotune(ctx.handle, instances, n, cache_path.encode() if cache_path else None,
                                      C.byref(best), C.byref(ms), _ptr(ws), ws.numel(), _stream(ctx.device)))
    return best, ms.value
