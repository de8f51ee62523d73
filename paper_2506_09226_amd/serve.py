"""Served queries over resident tables: a thin wrapper of the gq_server_* ABI.

The scheduler (admission by workspace footprint, continuous batching into
shared scans, several HIP streams) runs in a native thread inside libgq.so;
this module only builds the C structs, allocates each query's output buffers
and collects latencies.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import torch

from . import (GQ_ERR_CAPACITY, GQ_OK, GQ_QUERY_FILTER_AGG, GQ_QUERY_FILTER_TOPK, Context, GQError, Query,
               ServerCfg, ServerTables, _groups_struct, _ptr, alloc_groups, lib)


@dataclass
class QuerySpec:
    kind: int
    date_hi: int
    max_groups: int = 64
    k: int = 100


@dataclass
class Submitted:
    spec: QuerySpec
    ticket: int
    struct: Query
    out: object = None                     # GroupResult or (val, row, n)
    latency: float = float("nan")
    status: int = -1
    extra: dict = field(default_factory=dict)


class Server:
    """ctx: a Context, or a device index (a Context is then created for it)."""

    def __init__(self, ctx, tables: dict, dim1_table: torch.Tensor, dim2_table: torch.Tensor,
                 pool: torch.Tensor, streams: int = 4, max_batch: int = 16, serial: bool = False):
        if not isinstance(ctx, Context):
            ctx = Context(int(ctx))
        self.ctx = ctx
        self.device = ctx.device
        self._keep = (tables, dim1_table, dim2_table, pool)
        t = ServerTables(_ptr(tables["fk"]), _ptr(tables["fk2"]), _ptr(tables["date"]), _ptr(tables["qty"]),
                         _ptr(tables["price"]), _ptr(tables["disc"]), tables["fk"].numel(), _ptr(dim1_table),
                         dim1_table.numel(), _ptr(dim2_table), dim2_table.numel())
        cfg = ServerCfg(t, _ptr(pool), pool.numel(), streams, max_batch, int(serial))
        h = C.c_void_p()
        torch.cuda.synchronize(self.device)
        ctx.check(lib().gq_server_create(ctx.handle, C.byref(cfg), C.byref(h)))
        self.h = h

    def alloc_output(self, spec: QuerySpec):
        if spec.kind == GQ_QUERY_FILTER_TOPK:
            return (torch.empty(spec.k, dtype=torch.int64, device=self.device),
                    torch.empty(spec.k, dtype=torch.int32, device=self.device),
                    torch.zeros(1, dtype=torch.int64, device=self.device))
        return alloc_groups(_Dev(self.device), spec.max_groups, spec.kind == GQ_QUERY_FILTER_AGG,
                            spec.kind != GQ_QUERY_FILTER_AGG)

    def submit(self, spec: QuerySpec, out=None) -> Submitted:
        out = out if out is not None else self.alloc_output(spec)
        if spec.kind == GQ_QUERY_FILTER_TOPK:
            q = Query(spec.kind, spec.k, spec.date_hi, 0, _empty_groups(), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]))
        else:
            q = Query(spec.kind, 0, spec.date_hi, spec.max_groups, _groups_struct(out), None, None, None)
        t = C.c_uint64()
        rc = lib().gq_server_submit(self.h, C.byref(q), C.byref(t))
        if rc != GQ_OK:
            raise GQError(rc, "gq_server_submit")
        return Submitted(spec, t.value, q, out)

    def wait(self, sub: Submitted) -> Submitted:
        st, lat = C.c_int32(), C.c_double()
        rc = lib().gq_server_wait(self.h, sub.ticket, C.byref(st), C.byref(lat))
        if rc != GQ_OK:
            raise GQError(rc, "gq_server_wait")
        sub.status, sub.latency = st.value, lat.value
        return sub

    def run(self, spec: QuerySpec, capacity: int | None = None, max_tries: int = 4) -> Submitted:
        """Submit and wait, with the caller's recovery from GQ_ERR_CAPACITY: the
        server already retries up to the output capacity, so a query that still
        reports it is submitted again with outputs (and group bound) twice as
        large, up to max_tries times."""
        cap = capacity or spec.max_groups
        for _ in range(max_tries):
            sp = QuerySpec(spec.kind, spec.date_hi, max_groups=min(spec.max_groups, cap), k=spec.k)
            out = self.alloc_output(QuerySpec(spec.kind, spec.date_hi, max_groups=cap, k=spec.k))
            sub = self.wait(self.submit(sp, out=out))
            if sub.status != GQ_ERR_CAPACITY or spec.kind == GQ_QUERY_FILTER_TOPK:
                sub.extra["capacity"] = cap
                return sub
            cap *= 2
        return sub

    def stats(self):
        d, b, m, r = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        lib().gq_server_stats(self.h, C.byref(d), C.byref(b), C.byref(m), C.byref(r))
        return {"done": d.value, "batches": b.value, "max_batch": m.value, "reruns": r.value}

    def close(self):
        if getattr(self, "h", None):
            lib().gq_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Dev:
    def __init__(self, device):
        self.device = device


def _empty_groups():
    from . import Groups
    return Groups()


def result_host(sub: Submitted) -> dict:
    """The query's result on the host (groups dict, or top-k values/rows)."""
    torch.cuda.synchronize()
    if sub.spec.kind == GQ_QUERY_FILTER_TOPK:
        v, r, n = sub.out
        k = int(n.item())
        return {"val": v[:k].cpu().numpy(), "row": r[:k].cpu().numpy()}
    return sub.out.host()
