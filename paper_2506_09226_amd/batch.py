"""Many independent join + aggregate instances: the batched persistent form and
the plain form (one launch chain per instance) over the same device tables.

Instance i reads rows [dim_offset, dim_offset + m) of the dimension columns and
[fact_offset, fact_offset + n) of the fact columns; it computes
filter(date_lo <= date < date_hi) -> join(fk = dim_key, payload dim_attr) ->
group by dim_attr (count, sum qty, exact sum revenue, averages).
"""
from __future__ import annotations

import torch

from . import (Context, GroupResult, alloc_groups, gq_batch_autotune, gq_batch_join_agg, gq_filter,
               gq_groupby_agg, gq_join_build, gq_join_probe, gq_join_table_bytes, lib, make_instances)


class BatchedJoinAgg:
    """All instances in one persistent launch (gq_batch_join_agg)."""

    def __init__(self, ctx: Context, cols: dict, layout, date_lo: int, date_hi: int, max_groups: int = 64):
        self.ctx = ctx
        self.outs = [alloc_groups(ctx, max_groups, False, True) for _ in layout]
        specs = []
        for (mo, m, no, n), out in zip(layout, self.outs):
            specs.append({"dim_key": cols["dim_key"][mo:mo + m], "dim_attr": cols["dim_attr"][mo:mo + m],
                          "fk": cols["fk"][no:no + n], "date": cols["date"][no:no + n],
                          "qty": cols["qty"][no:no + n], "price": cols["price"][no:no + n],
                          "disc": cols["disc"][no:no + n], "date_lo": date_lo, "date_hi": date_hi, "out": out})
        self.instances = make_instances(specs)
        self.inst_status = torch.zeros(len(layout), dtype=torch.int32, device=ctx.device)
        self.ws = None
        self.tuning = None

    def autotune(self, cache_path: str | None = None):
        self.tuning, ms = gq_batch_autotune(self.ctx, self.instances, cache_path)
        self.ws = None
        return self.tuning, ms

    def run(self):
        if self.ws is None:
            from ctypes import byref
            tp = byref(self.tuning) if self.tuning is not None else None
            need = lib().gq_batch_workspace_bytes(self.instances, len(self.instances), tp)
            self.ws = self.ctx.workspace(need)
        gq_batch_join_agg(self.ctx, self.instances, self.tuning, ws=self.ws, inst_status=self.inst_status)

    def statuses(self):
        """Each instance's status code of the last run (host list)."""
        return self.inst_status.cpu().tolist()

    def results(self):
        return [o.host() for o in self.outs]


class PlainPerInstance:
    """The same instances with the plain operators, one launch chain each:
    filter -> join build -> join probe -> group-by, all buffers allocated once."""

    def __init__(self, ctx: Context, cols: dict, layout, date_lo: int, date_hi: int, max_groups: int = 64,
                 load_factor: float = 0.5):
        self.ctx, self.cols, self.layout = ctx, cols, layout
        self.date_lo, self.date_hi, self.max_groups = date_lo, date_hi, max_groups
        d = ctx.device
        n_max = max(n for _, _, _, n in layout)
        m_max = max(m for _, m, _, _ in layout)
        L = lib()
        self.sel = torch.empty(max(n_max, 1), dtype=torch.int32, device=d)
        self.n_sel = torch.zeros(1, dtype=torch.int64, device=d)
        self.ws_filter = ctx.workspace(L.gq_filter_workspace_bytes(n_max))
        self.table = torch.empty(gq_join_table_bytes(m_max, load_factor), dtype=torch.uint8, device=d)
        self.load_factor = load_factor
        self.ws_build = ctx.workspace(max(L.gq_join_build_workspace_bytes(m, gq_join_table_bytes(m, load_factor))
                                          for _, m, _, _ in layout))
        self.prow = torch.empty(max(n_max, 1), dtype=torch.int32, device=d)
        self.pay = torch.empty(max(n_max, 1), dtype=torch.int32, device=d)
        self.n_join = torch.zeros(1, dtype=torch.int64, device=d)
        self.ws_probe = ctx.workspace(L.gq_join_probe_workspace_bytes(n_max))
        self.ws_gb = ctx.workspace(L.gq_groupby_workspace_bytes(n_max, max_groups, 0, 1))
        self.outs = [alloc_groups(ctx, max_groups, False, True) for _ in layout]

    def run(self):
        ctx, c = self.ctx, self.cols
        for (mo, m, no, n), out in zip(self.layout, self.outs):
            date = c["date"][no:no + n]
            fk = c["fk"][no:no + n]
            gq_filter(ctx, date, self.date_lo, self.date_hi, out=self.sel, n_out=self.n_sel, ws=self.ws_filter)
            tb = gq_join_table_bytes(m, self.load_factor)
            table = self.table[:tb]
            gq_join_build(ctx, c["dim_key"][mo:mo + m], c["dim_attr"][mo:mo + m], table=table, ws=self.ws_build)
            gq_join_probe(ctx, table, fk, sel=self.sel, n=n, n_dev=self.n_sel, prow=self.prow, payload=self.pay,
                          n_out=self.n_join, ws=self.ws_probe)
            gq_groupby_agg(ctx, c["qty"][no:no + n], c["price"][no:no + n], c["disc"][no:no + n], n=n,
                           n_dev=self.n_join, rowid=self.prow, key32=self.pay, max_groups=self.max_groups, out=out,
                           ws=self.ws_gb)

    def results(self):
        return [o.host() for o in self.outs]
