"""The plain per-operator form of the hot path: one launch chain per operator.

    partition(fact by fk)  ->  filter(date < date_hi)  ->  join build(dim)
    ->  probe(partitioned fk via the selection)  ->  group-by(dim attribute)
    ->  float64 averages  [->  top-k of price over the selection]

The probe is the single-pass one (gq_join_probe) or the partitioned one
(gq_join_probe_partitioned: table regions probed from LDS); both give the
same output.  "auto" takes the partitioned probe when the fact table was
radix-partitioned (then the probe stream is in region order), otherwise the
single-pass one.  "tune" times both on the first step's data (HIP events, one
host wait) and keeps the faster: a heavy key concentrates its table region's
probes on one workgroup of the partitioned form, while the single-pass form
reads a hot slot from cache.

All buffers and workspaces are allocated once, so a step allocates nothing and
never waits for the host: every count travels on the device.

With streams=2 the operators that do not depend on each other overlap: the
join build (it reads only the dimension table) runs on a second stream beside
the partition and filter, and the top-k (it needs only the filter's selection)
runs there beside the probe and group-by.  Events order them; each operator is
still its own launch chain, and the step ends when both streams are done
(joined into the caller's current stream).
"""
from __future__ import annotations

import torch

from . import (Context, alloc_groups, gq_filter, gq_groupby_agg, gq_join_build, gq_join_probe,
               gq_join_probe_partitioned, gq_join_table_bytes, gq_radix_partition, gq_topk, lib)

FACT_COLS = ("date", "qty", "price", "disc")


class PlainPipeline:
    def __init__(self, ctx: Context, fact: dict, dim: dict, date_hi: int, max_groups: int,
                 log2_fanout: int = 6, topk: int = 100, load_factor: float = 0.5, partition: bool = True,
                 probe: str = "auto", streams: int = 1):
        self.ctx, self.fact, self.dim = ctx, fact, dim
        self.date_hi, self.max_groups, self.log2p = date_hi, max_groups, log2_fanout
        self.k, self.partition = topk, partition
        if streams not in (1, 2):
            raise ValueError(f"streams must be 1 or 2, not {streams}")
        self.streams = streams
        d = ctx.device
        self.side = None
        n, m = fact["fk"].numel(), dim["key"].numel()
        self.n, self.m = n, m
        L = lib()
        if partition:
            self.p_key = torch.empty_like(fact["fk"])
            self.p_cols = [torch.empty_like(fact[c]) for c in FACT_COLS]
            self.p_rowid = torch.empty(n, dtype=torch.int32, device=d)
            self.p_off = torch.empty((1 << log2_fanout) + 1, dtype=torch.int64, device=d)
            self.ws_part = ctx.workspace(L.gq_radix_partition_workspace_bytes(n, log2_fanout))
        self.sel = torch.empty(max(n, 1), dtype=torch.int32, device=d)
        self.n_sel = torch.zeros(1, dtype=torch.int64, device=d)
        self.ws_filter = ctx.workspace(L.gq_filter_workspace_bytes(n))
        self.table = torch.empty(gq_join_table_bytes(m, load_factor), dtype=torch.uint8, device=d)
        self.ws_build = ctx.workspace(L.gq_join_build_workspace_bytes(m, self.table.numel()))
        self.prow = torch.empty(max(n, 1), dtype=torch.int32, device=d)
        self.pay = torch.empty(max(n, 1), dtype=torch.int32, device=d)
        self.n_join = torch.zeros(1, dtype=torch.int64, device=d)
        if probe == "auto":
            probe = "partitioned" if partition else "ordered"
        if probe not in ("ordered", "partitioned", "tune"):
            raise ValueError(f"probe must be auto, tune, ordered or partitioned, not {probe!r}")
        self.probe = probe
        self.probe_ms = None                     # with "tune": each form's time on the first step
        self.ws_probe = {}
        for form in (("ordered", "partitioned") if probe == "tune" else (probe,)):
            self.ws_probe[form] = ctx.workspace(L.gq_join_probe_partitioned_workspace_bytes(n)
                                                if form == "partitioned" else L.gq_join_probe_workspace_bytes(n))
        self.groups = alloc_groups(ctx, max_groups, False, True)
        self.ws_gb = ctx.workspace(L.gq_groupby_workspace_bytes(n, max_groups, 0, 1))
        if topk:
            self.tk_val = torch.empty(topk, dtype=torch.int64, device=d)
            self.tk_row = torch.empty(topk, dtype=torch.int32, device=d)
            self.tk_n = torch.zeros(1, dtype=torch.int64, device=d)
            self.ws_tk = ctx.workspace(L.gq_topk_workspace_bytes(n, topk))

    def columns(self):
        """The fact columns the filter/probe/aggregate read (partitioned or not)."""
        if self.partition:
            date, qty, price, disc = self.p_cols
            return self.p_key, date, qty, price, disc
        f = self.fact
        return f["fk"], f["date"], f["qty"], f["price"], f["disc"]

    def _build(self):
        gq_join_build(self.ctx, self.dim["key"], self.dim["attr"], table=self.table, ws=self.ws_build)

    def _topk(self, price):
        gq_topk(self.ctx, price, self.k, sel=self.sel, n=self.n, n_dev=self.n_sel, val_out=self.tk_val,
                rowid_out=self.tk_row, n_out=self.tk_n, ws=self.ws_tk)

    def _probe(self, form, fk):
        ctx = self.ctx
        if form == "partitioned":
            gq_join_probe_partitioned(ctx, self.table, fk, sel=self.sel, n=self.n, n_dev=self.n_sel,
                                      log2_fanout=self.log2p if self.partition else 0, prow=self.prow,
                                      payload=self.pay, n_out=self.n_join, ws=self.ws_probe[form])
        else:
            gq_join_probe(ctx, self.table, fk, sel=self.sel, n=self.n, n_dev=self.n_sel, prow=self.prow,
                          payload=self.pay, n_out=self.n_join, ws=self.ws_probe[form])

    def _tune_probe(self, fk, stream):
        """Run both probe forms (same output), time each, keep the faster."""
        ms = {}
        for form in ("ordered", "partitioned"):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            self._probe(form, fk)
            e1.record(stream)
            e1.synchronize()
            ms[form] = e0.elapsed_time(e1)
        self.probe_ms = ms
        self.probe = min(ms, key=ms.get)
        if self.probe == "ordered":              # the partitioned form ran last: redo the winner's output
            self._probe("ordered", fk)

    def step(self, streams: int | None = None):
        """One pass of the chain; `streams` overrides the pipeline's setting."""
        ctx, f = self.ctx, self.fact
        two = (streams or self.streams) == 2
        main = torch.cuda.current_stream(ctx.device)
        if two and self.side is None:
            self.side = torch.cuda.Stream(device=ctx.device)          # default priority
            self.ev_fork, self.ev_built, self.ev_sel, self.ev_done = (torch.cuda.Event() for _ in range(4))
        if two:                                          # build beside partition + filter
            self.ev_fork.record(main)
            self.side.wait_event(self.ev_fork)
            with torch.cuda.stream(self.side):
                self._build()
                self.ev_built.record(self.side)
        if self.partition:
            gq_radix_partition(ctx, f["fk"], self.log2p, [f[c] for c in FACT_COLS],
                               outs=(self.p_key, self.p_cols, self.p_rowid, self.p_off), ws=self.ws_part)
        fk, date, qty, price, disc = self.columns()
        gq_filter(ctx, date, -(1 << 31), self.date_hi, out=self.sel, n_out=self.n_sel, ws=self.ws_filter)
        if two:                                          # top-k beside probe + group-by
            self.ev_sel.record(main)
            if self.k:
                self.side.wait_event(self.ev_sel)
                with torch.cuda.stream(self.side):
                    self._topk(price)
            main.wait_event(self.ev_built)
        else:
            self._build()
        if self.probe == "tune":
            self._tune_probe(fk, main)
        else:
            self._probe(self.probe, fk)
        gq_groupby_agg(ctx, qty, price, disc, n=self.n, n_dev=self.n_join, rowid=self.prow, key32=self.pay,
                       max_groups=self.max_groups, out=self.groups, ws=self.ws_gb)
        if two:
            self.ev_done.record(self.side)
            main.wait_event(self.ev_done)
        elif self.k:
            self._topk(price)

    def capture(self, streams: int | None = None):
        """Capture one step into a HIP graph; replay() then runs the whole chain
        with one launch.  Every operator's work is kernels on the capturing
        stream (and the second stream, joined back by events), counts stay on
        the device and nothing is allocated, so a replay recomputes the step
        on whatever the input buffers hold.  The probe tuner decides first."""
        if self.probe == "tune":
            self.step(streams)
        torch.cuda.synchronize(self.ctx.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step(streams)
        torch.cuda.synchronize(self.ctx.device)
        self.graph = g

    def replay(self):
        self.graph.replay()

    def source_rows(self, rows: torch.Tensor) -> torch.Tensor:
        """Map row ids of the (possibly partitioned) columns to input row ids."""
        return self.p_rowid[rows.long()] if self.partition else rows
