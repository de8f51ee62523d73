"""Benchmark of the relational hot path on one MI355X.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--workload 1] [--no-cpu-baseline]
                    [--no-batched] [--no-served] [--mode plain|batch|serve|skew]

A step is one pass of the plain per-operator pipeline over the one-GPU share
(200M fact rows x 25M dim rows, ~1.5M groups, 64 buckets), inputs resident in
HBM before timing starts:

    radix partition (64 buckets, 4 columns + row id) -> filter (date < 1500)
    -> join build (25M keys) -> join probe -> group-by (exact int128 sums)
    -> float64 averages -> top-100 of price over the selection

Prints one JSON line.  `value` is the whole step's algorithmic HBM bytes (what
each operator must read and write once) divided by the step time.  Per-kernel
durations come from HIP events recorded on the stream each kernel runs on.

The same line carries the other two forms of the metric, measured in the same
run after the plain steps (each on its own resident tables, the previous
form's memory released first):
  "batched"  512 join+aggregate instances in one persistent launch (autotuned)
             against one launch chain per instance, results compared;
  "served"   the served mix over a 1.6-billion-row resident fact table under
             Poisson arrivals at 0.8 and 1.5 times the serial capacity, p50/p99
             latency and throughput against serial plain execution, results
             compared;
plus the GPU clocks read before and after the GPU work, and the CPU baseline:
the oracle timed on the host's cores, one core and all cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "HBM GB/s (% peak) for partition/join/group-by; served p50/p99 query latency"


def algorithmic_bytes(n: int, m: int, s_n: int, groups: int, k: int, partition: bool = True) -> dict:
    """Bytes each operator must move once (inputs read once, outputs written
    once, one 16-byte slot per build insert or probe lookup)."""
    ops = {
        "partition": (36 + 40) * n if partition else 0,        # 5 columns in, 5 columns + row id out
        "filter": 4 * n + 4 * s_n,                             # date in, selection out
        "join_build": (12 + 16) * m,                           # key + payload in, slot written
        "join_probe": (4 + 8 + 16 + 8) * s_n,                  # sel + fk in, slot read, pair out
        "groupby": (4 + 4 + 24) * s_n + 36 * groups,           # row id + key + 3 values in, groups out
        "topk": (4 + 8) * s_n + 12 * k,                        # sel + price in, k rows out
    }
    return ops


# kernels of each operator (HIP-event names); an operator's time is their sum
OP_KERNELS = {
    "partition": ["gq_partition_hist", "gq_partition_scan", "gq_partition_offsets", "gq_partition_scatter"],
    "filter": ["gq_filter"],
    "join_build": ["gq_join_build_init", "gq_join_build_insert", "gq_join_build_part_hist",
                   "gq_join_build_part_scan", "gq_join_build_part_offsets", "gq_join_build_part_scatter",
                   "gq_join_build_split", "gq_join_build_regions", "gq_join_build_overflow"],
    "join_probe": ["gq_join_probe", "gq_join_probe_split", "gq_join_probe_plan", "gq_join_probe_regions",
                   "gq_join_probe_compact"],
    "groupby": ["gq_groupby_hist", "gq_groupby_scan", "gq_groupby_scatter", "gq_groupby_tiles2", "gq_groupby_hist2",
                "gq_groupby_scan2", "gq_groupby_scatter2", "gq_groupby_side", "gq_groupby_chunks", "gq_groupby_bucket",
                "gq_groupby_emit", "gq_groupby_local"],
    "topk": ["gq_topk_local", "gq_topk_merge"],
}
KERNELS = ["gq_zero"] + [k for ks in OP_KERNELS.values() for k in ks]
# kernels that by themselves move their operator's whole algorithmic bytes
# (candidates for the roofline's dominant kernel)
KERNEL_OP = {"gq_partition_scatter": "partition", "gq_filter": "filter", "gq_join_probe": "join_probe",
             "gq_topk_local": "topk"}


def _file_sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, or None
    if there is none or the kernel's source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            a, b = line.split(":", 1)
            kv[a.strip()] = b.strip()
    src = os.path.join(ROOT, "paper_2506_09226_amd", "csrc", kv.get("source", ""))
    if not os.path.exists(src) or _file_sha(src) != kv.get("source_sha256_16"):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _sysfs_clocks() -> dict:
    """The current DPM level of each clock domain from the driver's sysfs
    files (read only), e.g. {"card0": {"sclk": "2400Mhz", ...}}."""
    import glob
    out = {}
    for path in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_*")):
        card = path.split("/")[4]
        dom = path.rsplit("pp_dpm_", 1)[1]
        try:
            cur = [ln.split(":", 1)[1].strip(" *\n") for ln in open(path) if ln.rstrip().endswith("*")]
        except OSError:
            continue
        if cur:
            out.setdefault(card, {})[dom] = cur[0]
    return out


_NO_CLOCKS = False


def gpu_clocks() -> dict:
    """Current GPU clocks, power and temperature as rocm-smi reports them,
    plus the sysfs DPM levels (read only; an error note if unavailable)."""
    import subprocess
    if _NO_CLOCKS:
        return {"skipped": "--no-clocks"}
    sysfs = _sysfs_clocks()
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--showpower", "--showtemp", "--json"],
                           capture_output=True, text=True, timeout=30)
        data = json.loads(r.stdout)
    except Exception as e:                                    # noqa: BLE001 - a missing tool is not an error
        return {"error": str(e)[:120], "sysfs_dpm": sysfs}
    out = {}
    for card, kv in data.items():
        if not isinstance(kv, dict):
            continue
        keep = {}
        for k, v in kv.items():
            kl = k.lower()
            if any(t in kl for t in ("sclk", "mclk", "fclk", "socclk", "power", "temperature (sensor junction)",
                                     "temperature (sensor memory)")):
                keep[k] = v
        out[card] = keep
    if sysfs:
        out["sysfs_dpm"] = sysfs
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_threads(cap: int = 16) -> int:
    """Host threads for the CPU baseline: the cores this process may use,
    at most `cap` (the host's share per GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


def cpu_baseline(w, shard_rows: int, threads: int) -> dict:
    """The oracle, as it stands, on the host's cores.  The fact table is cut
    into `threads` shards of `shard_rows` consecutive rows; each shard runs the
    whole plain pipeline (partition, filter, join with the full dimension
    table, group-by, top-k) in the single-threaded C oracle, on its own host
    thread, all shards at once.  Reported in the same unit as the GPU line
    (algorithmic GB/s over the shards' rows), next to one shard alone on one
    core.  The shards' partial groups are not merged (a merge of at most
    threads x groups partial sums, left out of the timing)."""
    import threading

    import torch

    import oracle
    import synth
    oracle.lib()
    dim = {k: v.numpy() for k, v in synth.dim_table(w.dim_m, w.dim_seed, w.attr_range).items()}
    shards = []
    for i in range(threads):
        rows = torch.arange(i * shard_rows, (i + 1) * shard_rows, dtype=torch.int64)
        shards.append({k: v.numpy() for k, v in synth.fact_columns(w.fact, rows).items()})

    def pipeline(fact, out, idx):
        pk, pcols, _, _ = oracle.partition(fact["fk"], w.log2_fanout,
                                           [fact[c] for c in ("date", "qty", "price", "disc")])
        pdate, pqty, pprice, pdisc = pcols
        sel = oracle.filter(pdate, -(1 << 31), w.date_hi)
        prow, pay = oracle.join(dim["key"], dim["attr"], pk, sel)
        g = oracle.groupby(len(prow), pqty, pprice, pdisc, rowid=prow, key32=pay)
        oracle.topk(pprice, 100, sel=sel)
        out[idx] = sum(algorithmic_bytes(len(pk), w.dim_m, len(sel), len(g["count"]), 100).values())

    one = [0]
    t0 = time.perf_counter()
    pipeline(shards[0], one, 0)
    dt1 = time.perf_counter() - t0
    res = [0] * threads
    ths = [threading.Thread(target=pipeline, args=(shards[i], res, i)) for i in range(threads)]
    t0 = time.perf_counter()
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    dtn = time.perf_counter() - t0
    return {"value": round(sum(res) / dtn / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{threads} shards of {shard_rows:,} consecutive fact rows ({threads * shard_rows:,} of "
                      f"{w.fact.n:,}), each joined with all {w.dim_m:,} dim rows; the same pipeline in the "
                      f"single-threaded C oracle, one host thread per shard, {dtn:.1f} s",
            "single_core": {"value": round(one[0] / dt1 / 1e9, 3), "unit": "GB/s", "cores": 1,
                            "sample": f"one shard of {shard_rows:,} rows, {dt1:.1f} s"}}


def copy_bandwidth(gib: int = 2, reps: int = 5) -> dict:
    """Read + write rate of a plain device-to-device copy of `gib` GiB,
    timed on the same box and in the same process as the steps: the practical
    ceiling that a bandwidth-bound kernel's fraction of the peak is set against."""
    import torch
    n = (gib << 30) // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    moved = 2 * n * 4
    del src, dst
    _release()
    gbs = moved / (ms * 1e6)
    return {"bytes_per_copy": moved, "ms": round(ms, 4), "GB/s": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def _timed(fn, steps, warm, stream):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _release():
    import gc

    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=1, choices=[0, 1])
    ap.add_argument("--mode", default="plain", choices=["plain", "batch", "serve", "skew"],
                    help="plain: the per-operator pipeline on one workload, with the batched and served forms "
                         "as sub-objects of its line; batch / serve: that form alone as the line; "
                         "skew: 100M Zipf(1.0) fact rows, composite-key group-by plus the 5%% pipeline")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--serve-queries", type=int, default=160)
    ap.add_argument("--serve-rows", type=int, default=1_600_000_000)
    ap.add_argument("--serve-streams", type=int, default=2, help="HIP streams of the served form")
    ap.add_argument("--no-batched", action="store_true", help="plain mode: leave out the batched sub-object")
    ap.add_argument("--no-served", action="store_true", help="plain mode: leave out the served sub-object")
    ap.add_argument("--cpu-shard-rows", type=int, default=0,
                    help="rows per CPU-baseline shard (0: the fact rows split evenly over the threads)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="0: the cores this process may use, at most 16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--probe", default="tune", choices=["tune", "auto", "ordered", "partitioned"],
                    help="join probe form (tune: both timed on the first warm-up step, the faster kept; "
                         "auto: partitioned on partitioned input)")
    ap.add_argument("--streams", type=int, default=1, choices=[1, 2],
                    help="plain form: 2 overlaps the join build and the top-k with the fact-side chain "
                         "(per-kernel times then include the overlap)")
    ap.add_argument("--load-factor", type=float, default=0.5, help="join hash table load factor bound")
    ap.add_argument("--graph", action="store_true",
                    help="plain form: time replays of the step captured as one HIP graph (no per-kernel times)")
    ap.add_argument("--no-partition", action="store_true",
                    help="variant: skip the radix partition and run filter/join/group-by on the input order")
    ap.add_argument("--no-clocks", action="store_true",
                    help="record no GPU clocks (rocm-smi is not started; for runs under a profiler)")
    ap.add_argument("--no-copy-ref", action="store_true",
                    help="plain form: skip the 2 GiB device copy timed after the steps (the practical ceiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (3 times) to calibrate HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library runs the per-GPU hot path "
              f"on one GPU's share; the multi-GPU exchange is not built", file=sys.stderr)
        sys.exit(2)
    global _NO_CLOCKS
    _NO_CLOCKS = args.no_clocks

    if args.mode == "batch":
        out = bench_batch(args)
        print(json.dumps(out), flush=True)
        return
    if args.mode == "serve":
        out = bench_serve(args)
        print(json.dumps(out), flush=True)
        return
    if args.mode == "skew":
        return bench_skew(args)
    clk0 = gpu_clocks()
    out = bench_plain(args)
    _release()
    if args.workload == 1 and not args.no_batched:
        out["batched"] = bench_batch(args, sub=True)
        _release()
    if args.workload == 1 and not args.no_served:
        out["served"] = bench_serve(args, sub=True)
        _release()
    out["gpu_clocks"] = {"start": clk0, **out["gpu_clocks"], "end": gpu_clocks()}
    if not args.no_cpu_baseline:
        import synth
        w = synth.workload(args.workload)
        threads = args.cpu_threads or cpu_threads()
        shard = min(args.cpu_shard_rows or w.fact.n, w.fact.n // threads)
        out["cpu_baseline"] = cpu_baseline(w, shard, threads)
    print(json.dumps(out), flush=True)


def bench_plain(args) -> dict:
    import torch

    import synth
    import paper_2506_09226_amd as gq
    from paper_2506_09226_amd.pipeline import PlainPipeline

    w = synth.workload(args.workload)
    torch.cuda.set_device(0)
    ctx = gq.Context(0)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")      # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t_gen = time.perf_counter()
    fact = synth.fact_table(w.fact, device="cuda")
    dim = synth.dim_table(w.dim_m, w.dim_seed, w.attr_range, device="cuda")
    torch.cuda.synchronize()
    print(f"# generated {w.fact.n:,} x {w.dim_m:,} rows in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr,
          flush=True)
    pl = PlainPipeline(ctx, fact, dim, w.date_hi, max_groups=w.attr_range, log2_fanout=w.log2_fanout, topk=100,
                       partition=not args.no_partition, probe=args.probe, streams=args.streams,
                       load_factor=args.load_factor)

    for _ in range(args.warmup):
        pl.step()
    if pl.probe == "tune":                      # the tuning step stays out of the timed region
        pl.step()
    torch.cuda.synchronize()
    ctx.raise_status()
    s_n = int(pl.n_sel.item())
    groups = int(pl.groups.n_groups.item())

    # timed region: whole steps, stream-ordered, no host waits inside
    stream = torch.cuda.current_stream()
    run_step = pl.step
    if args.graph:
        pl.capture()
        for _ in range(args.warmup):
            pl.replay()
        run_step = pl.replay
        args.no_timing = True                    # kernel events are not recorded inside a graph
    if not args.no_timing:
        ctx.reset_timing()
        ctx.set_timing(True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        run_step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    ctx.set_timing(False)
    ctx.raise_status()
    clk_steps = gpu_clocks()                   # read right after the timed steps, still in their clock state
    copy_ref = None if args.no_copy_ref else copy_bandwidth()
    print(f"# {args.steps} steps: {ms_step:.3f} ms/step (host wall {1e3 * wall / args.steps:.3f} ms/step)",
          file=sys.stderr, flush=True)
    by = algorithmic_bytes(w.fact.n, w.dim_m, s_n, groups, 100, partition=not args.no_partition)
    total_bytes = sum(by.values())
    kern = {}
    if not args.no_timing:
        for k in KERNELS:
            cnt, ms = ctx.kernel_time(k)
            if cnt:
                kern[k] = {"launches": cnt, "avg_ms": ms / cnt, "ms_per_step": ms / args.steps}
    ops = {}
    for op, ks in OP_KERNELS.items():
        ms = sum(kern[k]["ms_per_step"] for k in ks if k in kern)
        if ms > 0:
            ops[op] = {"ms": round(ms, 4), "bytes": by[op], "GB/s": round(by[op] / (ms * 1e6), 1),
                       "frac_of_peak": round(by[op] / (ms * 1e6) / HBM_PEAK_GBS, 4)}
    roofline = None
    cands = [k for k in KERNEL_OP if k in kern]
    if cands:
        dom = max(cands, key=lambda k: kern[k]["ms_per_step"])
        op = KERNEL_OP[dom]
        ach = by[op] / (kern[dom]["avg_ms"] * 1e6)
        roofline = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": load_traffic(dom, f"{w.fact.n // 1_000_000}M"),
                    "algorithmic_bytes_per_launch": by[op], "avg_ms": round(kern[dom]["avg_ms"], 4)}

    out = {
        "metric": METRIC,
        "value": round(total_bytes / (ms_step * 1e6), 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": w.name, "fact_rows": w.fact.n, "dim_rows": w.dim_m, "groups": groups,
                   "selected_rows": s_n, "buckets": 1 << w.log2_fanout, "filter": f"date < {w.date_hi}",
                   "topk": 100, "form": f"plain (one launch chain per operator, {args.streams} streams"
                                         f"{', captured as one HIP graph' if args.graph else ''})",
                   "partitioned": not args.no_partition, "probe": pl.probe, "probe_tuning_ms": pl.probe_ms,
                   "load_factor": args.load_factor,
                   "partition_items": int(os.environ.get("GQ_PARTITION_ITEMS", "16"))},
        "hbm_frac_of_peak": round(total_bytes / (ms_step * 1e6) / HBM_PEAK_GBS, 4),
        "algorithmic_bytes_per_step": total_bytes,
        "rows_per_s": round(w.fact.n / (ms_step * 1e-3)),
        "ops": ops,
        "kernels_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in kern.items()},
        "roofline": roofline,
        "cpu_baseline": None,
        "gpu_clocks": {"after_plain_steps": clk_steps},
        "copy_ref": copy_ref,
    }
    del pl, fact, dim
    ctx.close()
    return out


def bench_skew(args):
    """Skewed workload: 100M fact rows with Zipf(1.0) foreign keys over a 10M-row
    dimension.  A step is (i) the group-by over all rows on the composite key
    (fk, g32), about 10.6M groups, then (ii) filter (date < 128, 5%) -> join
    build -> probe -> group-by on the dimension attribute -> top-100."""
    import torch

    import synth
    import paper_2506_09226_amd as gq
    from paper_2506_09226_amd.pipeline import PlainPipeline

    w = synth.workload(2)
    torch.cuda.set_device(0)
    ctx = gq.Context(0)
    t_gen = time.perf_counter()
    fact = synth.fact_table(w.fact, device="cuda")
    dim = synth.dim_table(w.dim_m, w.dim_seed, w.attr_range, device="cuda")
    torch.cuda.synchronize()
    print(f"# generated {w.fact.n:,} x {w.dim_m:,} rows in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr,
          flush=True)
    n = w.fact.n
    max_groups = 16_000_000
    groups = gq.alloc_groups(ctx, max_groups, True, True)
    ws_gb = ctx.workspace(gq.lib().gq_groupby_workspace_bytes(n, max_groups, 1, 1))
    pl = PlainPipeline(ctx, fact, dim, w.date_hi, max_groups=w.attr_range, partition=False, topk=100,
                       streams=args.streams, probe=args.probe)

    def composite():
        gq.gq_groupby_agg(ctx, fact["qty"], fact["price"], fact["disc"], key64=fact["fk"], key32=fact["g32"],
                          max_groups=max_groups, out=groups, ws=ws_gb)

    stream = torch.cuda.current_stream()

    def timed(fn, steps, warm):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        ctx.raise_status()
        if not args.no_timing:
            ctx.reset_timing()
            ctx.set_timing(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ctx.set_timing(False)
        ctx.raise_status()
        kern = {}
        if not args.no_timing:
            for k in KERNELS:
                cnt, ms = ctx.kernel_time(k)
                if cnt:
                    kern[k] = round(ms / steps, 4)
        return e0.elapsed_time(e1) / steps, kern

    if pl.probe == "tune":                      # the tuning step stays out of the timed region
        pl.step()
    ms_gb, k_gb = timed(composite, args.steps, args.warmup)
    ms_pl, k_pl = timed(pl.step, args.steps, args.warmup)
    ng = int(groups.n_groups.item())
    s_n = int(pl.n_sel.item())
    by_gb = (8 + 4 + 24) * n + (8 + 4 + 32) * ng        # keys + values in; key + count + sums out
    by_pl = algorithmic_bytes(n, w.dim_m, s_n, int(pl.groups.n_groups.item()), 100, partition=False)
    total = by_gb + sum(by_pl.values())
    ms_step = ms_gb + ms_pl
    print(f"# composite group-by {ms_gb:.3f} ms ({ng:,} groups), pipeline {ms_pl:.3f} ms", file=sys.stderr,
          flush=True)
    out = {
        "metric": METRIC,
        "value": round(total / (ms_step * 1e6), 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": w.name, "fact_rows": n, "dim_rows": w.dim_m, "composite_groups": ng,
                   "selected_rows": s_n, "filter": f"date < {w.date_hi}", "topk": 100,
                   "form": f"plain (one launch chain per operator, {args.streams} streams)", "probe": pl.probe,
                   "probe_tuning_ms": pl.probe_ms},
        "hbm_frac_of_peak": round(total / (ms_step * 1e6) / HBM_PEAK_GBS, 4),
        "algorithmic_bytes_per_step": total,
        "composite_groupby": {"ms": round(ms_gb, 4), "bytes": by_gb, "GB/s": round(by_gb / (ms_gb * 1e6), 1),
                              "frac_of_peak": round(by_gb / (ms_gb * 1e6) / HBM_PEAK_GBS, 4),
                              "kernels_ms": k_gb},
        "pipeline": {"ms": round(ms_pl, 4), "bytes": sum(by_pl.values()),
                     "GB/s": round(sum(by_pl.values()) / (ms_pl * 1e6), 1), "kernels_ms": k_pl},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def batch_bytes(layout, sel_rows: int) -> int:
    """Algorithmic bytes of the fused filter -> probe -> aggregate per instance:
    build 12 B in + 16 B slot per key; probe 4 B date per fact row, then per
    selected row 8 B fk + 16 B slot + 24 B of values."""
    m = sum(l[1] for l in layout)
    n = sum(l[3] for l in layout)
    return 28 * m + 4 * n + 48 * sel_rows


def bench_batch(args, sub: bool = False) -> dict:
    """Batched workload: 512 join+aggregate instances in one persistent launch
    (autotuned) against one plain launch chain per instance.  sub=True: the
    object that the plain line carries as "batched"."""
    import numpy as np
    import torch

    import synth
    import paper_2506_09226_amd as gq
    from paper_2506_09226_amd.batch import BatchedJoinAgg, PlainPerInstance

    torch.cuda.set_device(0)
    ctx = gq.Context(0)
    spec = synth.BatchSpec(count=args.batch_count)
    t_gen = time.perf_counter()
    cols, layout = synth.batch_tables(spec, device="cuda")
    torch.cuda.synchronize()
    print(f"# generated {len(layout)} instances ({sum(l[1] for l in layout):,} build / "
          f"{sum(l[3] for l in layout):,} probe rows) in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr,
          flush=True)
    sel_rows = int((cols["date"] < spec.date_hi).sum().item())
    by = batch_bytes(layout, sel_rows)
    stream = torch.cuda.current_stream()

    b = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    tun, tune_ms = b.autotune(os.path.join(os.environ.get("TMPDIR", "/tmp"), "gq_batch_tuning.txt"))
    print(f"# autotuned: {tun.as_dict()} ({tune_ms:.2f} ms)", file=sys.stderr, flush=True)
    ms_b = _timed(b.run, args.steps, args.warmup, stream)
    ctx.raise_status()
    inst_ok = all(x == gq.GQ_OK for x in b.statuses())
    p = PlainPerInstance(ctx, cols, layout, 0, spec.date_hi)
    ms_p = _timed(p.run, max(1, args.steps // 2), 1, stream)
    ctx.raise_status()
    rb, rp = b.results(), p.results()
    same = inst_ok
    for x, y in zip(rb, rp):
        ox, oy = np.argsort(x["key32"]), np.argsort(y["key32"])
        for f in ("key32", "count", "sum_qty", "sum_rev_lo", "sum_rev_hi"):
            same &= bool(np.array_equal(x[f][ox], y[f][oy]))
    print(f"# batched {ms_b:.2f} ms, plain per instance {ms_p:.2f} ms", file=sys.stderr, flush=True)
    workload = (f"{len(layout)} join+aggregate instances, build log-uniform in [1e3, 2e6], probe 8-16x build, "
                f"date < {spec.date_hi}, group by dim attribute in [0, {spec.attr_range})")
    res = {"workload": workload, "instances": len(layout), "build_rows": sum(l[1] for l in layout),
           "probe_rows": sum(l[3] for l in layout), "selected_rows": sel_rows,
           "form": "batched (one persistent launch, autotuned)", "steps": args.steps, "warmup": args.warmup,
           "ms": round(ms_b, 4), "algorithmic_bytes": by, "GB/s": round(by / (ms_b * 1e6), 1),
           "frac_of_peak": round(by / (ms_b * 1e6) / HBM_PEAK_GBS, 4), "tuning": tun.as_dict(),
           "tuning_ms": round(tune_ms, 4),
           "tuning_search": "coordinate descent, 2 rounds: load factor {0.2,0.25,0.3,0.4,0.5,0.6,0.7}, probe tile "
                            "{8K..512K} rows, lag {1..512}, probe fan-out {1,2,4,8,16}, build tile {1K..64K}",
           "plain_per_instance": {"ms": round(ms_p, 3), "GB/s": round(by / (ms_p * 1e6), 1),
                                  "launch_chains": len(layout), "steps": max(1, args.steps // 2)},
           "speedup_vs_plain": round(ms_p / ms_b, 3), "results_equal": same}
    del b, p, cols
    ctx.close()
    if sub:
        return res
    return {"metric": METRIC, "value": res["GB/s"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": res["ms"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "int64", "data": "synthetic",
            "config": {"workload": workload, "instances": len(layout), "build_rows": res["build_rows"],
                       "probe_rows": res["probe_rows"], "selected_rows": sel_rows, "form": res["form"]},
            "hbm_frac_of_peak": res["frac_of_peak"], "algorithmic_bytes_per_step": by, "tuning": res["tuning"],
            "plain_per_instance": res["plain_per_instance"], "speedup_vs_plain": res["speedup_vs_plain"],
            "results_equal": same}


def bench_serve(args, sub: bool = False) -> dict:
    """Served mix vs serial plain execution under the same Poisson arrivals.
    sub=True: the object that the plain line carries as "served"."""
    import numpy as np
    import torch

    import synth
    import paper_2506_09226_amd as gq
    from paper_2506_09226_amd.serve import QuerySpec, Server, result_host

    torch.cuda.set_device(0)
    ctx = gq.Context(0)
    spec = synth.ServeSpec(n=args.serve_rows)
    t_gen = time.perf_counter()
    fact, dim1, dim2 = synth.serve_tables(spec, device="cuda")
    torch.cuda.synchronize()
    print(f"# generated {spec.n:,} fact rows and 2 x {spec.m:,} dim rows in {time.perf_counter() - t_gen:.1f} s",
          file=sys.stderr, flush=True)
    t1 = gq.gq_join_build(ctx, dim1["key"], dim1["attr"])
    t2 = gq.gq_join_build(ctx, dim2["key"], dim2["attr"])
    torch.cuda.synchronize()
    ctx.raise_status()
    del dim1, dim2
    torch.cuda.empty_cache()
    resident = sum(v.numel() * v.element_size() for v in fact.values()) + t1.numel() + t2.numel()
    free, total = torch.cuda.mem_get_info()
    pool = torch.empty(int(min(free - (8 << 30), 100 << 30)) & ~255, dtype=torch.uint8, device="cuda")
    print(f"# resident {resident / 1e9:.1f} GB (fact {spec.n:,} rows), pool {pool.numel() / 1e9:.1f} GB",
          file=sys.stderr, flush=True)
    qlist = [QuerySpec(k, hi, max_groups={1: 16, 2: spec.code_range, 3: 32, 4: 0}[k], k=100)
             for k, hi in synth.serve_queries(args.serve_queries, spec.seed)]

    def run(server, arrivals):
        subs, t0 = [], time.perf_counter()
        for q, at in zip(qlist, arrivals):
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            subs.append(server.submit(q))
        for s_ in subs:
            server.wait(s_)
        span = time.perf_counter() - t0
        lat = np.array([s_.latency for s_ in subs]) * 1e3
        ok = all(s_.status == gq.GQ_OK for s_ in subs)
        return subs, ok, {"qps": round(len(subs) / span, 2), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                          "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3)}

    # serial service time: each query alone, one at a time
    ser = Server(ctx, fact, t1, t2, pool, serial=True)
    warm = [ser.wait(ser.submit(q)) for q in qlist[:8]]
    iso = [ser.wait(ser.submit(q)).latency for q in qlist[:40]]
    t_bar = float(np.mean(iso))
    print(f"# serial service time {t_bar * 1e3:.2f} ms over {len(iso)} queries", file=sys.stderr, flush=True)
    out_loads = {}
    results_equal = True
    for load in (0.8, 1.5):
        arr = synth.poisson_arrivals(len(qlist), load / t_bar, spec.seed + int(load * 10))
        subs_s, ok_s, st_s = run(ser, arr)
        srv = Server(ctx, fact, t1, t2, pool, streams=args.serve_streams, max_batch=16)
        subs_b, ok_b, st_b = run(srv, arr)
        stats = srv.stats()
        srv.close()
        results_equal &= ok_s and ok_b
        for a, b in zip(subs_s, subs_b):
            ra, rb = result_host(a), result_host(b)
            if a.spec.kind == gq.GQ_QUERY_FILTER_TOPK:
                results_equal &= bool(np.array_equal(ra["row"], rb["row"]) and np.array_equal(ra["val"], rb["val"]))
            else:
                key = "key64" if a.spec.kind == gq.GQ_QUERY_FILTER_AGG else "key32"
                oa, ob = np.argsort(ra[key]), np.argsort(rb[key])
                for f in (key, "count", "sum_qty", "sum_rev_lo", "sum_rev_hi"):
                    results_equal &= bool(np.array_equal(ra[f][oa], rb[f][ob]))
        st_b.update({"batches": stats["batches"], "max_batch": stats["max_batch"], "reruns": stats["reruns"]})
        out_loads[f"{load}"] = {"offered_qps": round(load / t_bar, 2), "served": st_b, "serial": st_s}
        print(f"# load {load}: served {st_b} serial {st_s}", file=sys.stderr, flush=True)
    ser.close()
    main_load = out_loads["0.8"]
    workload = (f"served mix over {spec.n:,} resident fact rows, two dims of {spec.m:,} rows; 4 templates "
                f"(filter+agg, join+agg, two-join+agg, filter+top-100), selectivity U[1%,60%], Poisson arrivals "
                f"at 0.8 and 1.5 / serial service time")
    res = {"workload": workload, "resident_bytes": resident, "pool_bytes": pool.numel(), "queries": len(qlist),
           "form": f"served (continuous batching, shared scans, {args.serve_streams} streams) vs serial plain",
           "serial_service_ms": round(t_bar * 1e3, 3),
           "p50_ms": main_load["served"]["p50_ms"], "p99_ms": main_load["served"]["p99_ms"],
           "qps": main_load["served"]["qps"],
           "serial_p50_ms": main_load["serial"]["p50_ms"], "serial_p99_ms": main_load["serial"]["p99_ms"],
           "loads": out_loads, "results_equal": results_equal}
    del pool, fact, t1, t2
    ctx.close()
    if sub:
        return res
    return {"metric": METRIC, "value": res["qps"], "unit": "queries/s", "n_gpus": 1, "steps": len(qlist),
            "warmup": len(warm), "ms_per_step": main_load["served"]["mean_ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
            "config": {"workload": workload, "resident_bytes": resident, "pool_bytes": res["pool_bytes"],
                       "queries": len(qlist), "form": res["form"]},
            "p50_ms": res["p50_ms"], "p99_ms": res["p99_ms"], "serial_service_ms": res["serial_service_ms"],
            "loads": out_loads, "results_equal": results_equal}


if __name__ == "__main__":
    main()
