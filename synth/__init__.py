"""Seeded, counter-based synthetic inputs for the relational hot path.

This module is the only code shared by the CPU oracle and the HIP path. It holds
none of the method's arithmetic (no hashing for partitioning, no joins, no
aggregation): it only draws column values.

Every value is a pure function of (seed, stream, row), so any row can be
recomputed alone (the tests sample rows of 200M-row tables that way) and the
same call gives bit-identical columns on the CPU and on the GPU: all arithmetic
is wrapping int64 tensor arithmetic (torch), with logical shifts done by
masking, so the result does not depend on the device.

Mixing function: the SplitMix64 output function (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014), applied to the
counter ``seed*GOLDEN + stream*STREAM_STRIDE + row*GOLDEN``.  It is a bijection
of 64-bit words, which is what makes the dimension keys unique.

Distributions (all with the shapes of the workloads named in the design notes):
  uniform integer in [lo, hi]   multiply-high of a 31-bit draw: lo + ((x>>33)*R)>>31
  Zipf(s) over ranks 1..M       inverse CDF, binary search in a float64 CDF built
                                once on the host, u = (x>>11) * 2**-53
  log-uniform sizes             host-side float64, for instance sizes only
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
C1 = 0xBF58476D1CE4E5B9
C2 = 0x94D049BB133111EB
STREAM_STRIDE = 0xD1342543DE82EF95

# column stream ids (fixed per column name)
S_DIM_KEY, S_DIM_ATTR, S_FK_ROW, S_DATE, S_QTY, S_PRICE, S_DISC, S_G32, S_FK2_ROW = range(9)

INT64_MIN = -(1 << 63)


def _s64(u: int) -> int:
    """Unsigned 64-bit Python int -> the int64 with the same bits."""
    u &= MASK64
    return u - (1 << 64) if u >> 63 else u


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 bits."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def mix64(x: torch.Tensor) -> torch.Tensor:
    """SplitMix64 output function on int64 tensors (wrapping arithmetic)."""
    x = x ^ _srl(x, 30)
    x = x * _s64(C1)
    x = x ^ _srl(x, 27)
    x = x * _s64(C2)
    x = x ^ _srl(x, 31)
    return x


def mix64_int(x: int) -> int:
    """Scalar form of mix64 on Python ints (unsigned 64-bit in and out)."""
    x &= MASK64
    x ^= x >> 30
    x = (x * C1) & MASK64
    x ^= x >> 27
    x = (x * C2) & MASK64
    x ^= x >> 31
    return x


def splitmix64_sequence(seed: int, count: int) -> list[int]:
    """The textbook SplitMix64 generator (state += golden; output mix(state))."""
    out, state = [], seed & MASK64
    for _ in range(count):
        state = (state + GOLDEN) & MASK64
        out.append(mix64_int(state))
    return out


def raw(seed: int, stream: int, rows: torch.Tensor) -> torch.Tensor:
    """64 random bits (as int64) for each row index in ``rows`` (int64)."""
    base = _s64(seed * GOLDEN + stream * STREAM_STRIDE)
    return mix64(rows * _s64(GOLDEN) + base)


def uniform_int(seed: int, stream: int, rows: torch.Tensor, lo: int, hi: int) -> torch.Tensor:
    """Integer uniform in [lo, hi] (inclusive); hi - lo + 1 must be < 2**31."""
    r = hi - lo + 1
    assert 0 < r < (1 << 31)
    x = _srl(raw(seed, stream, rows), 33)          # 31 random bits
    return lo + ((x * r) >> 31)


def unit_float(seed: int, stream: int, rows: torch.Tensor) -> torch.Tensor:
    """float64 uniform in [0, 1): 53 random bits times 2**-53 (exact)."""
    x = _srl(raw(seed, stream, rows), 11)
    return x.to(torch.float64) * (2.0 ** -53)


def dim_key(seed: int, rows: torch.Tensor) -> torch.Tensor:
    """Unique int64 key of dimension row ``rows`` (bijective in the row index)."""
    return raw(seed, S_DIM_KEY, rows)


_ZIPF_CACHE: dict = {}


def zipf_cdf(m: int, s: float = 1.0) -> torch.Tensor:
    """float64 CDF of Zipf(s) over ranks 1..m, summed in a fixed order on the CPU."""
    key = (m, s)
    if key not in _ZIPF_CACHE:
        r = torch.arange(1, m + 1, dtype=torch.float64)
        w = r.pow(-s)
        c = torch.cumsum(w, 0)
        _ZIPF_CACHE[key] = c / c[-1]
    return _ZIPF_CACHE[key]


def zipf_row(seed: int, stream: int, rows: torch.Tensor, m: int, s: float = 1.0) -> torch.Tensor:
    """Dimension row (rank - 1) drawn Zipf(s) over m ranks; rank 1 -> row 0."""
    cdf = zipf_cdf(m, s).to(rows.device)
    u = unit_float(seed, stream, rows)
    idx = torch.searchsorted(cdf, u, right=True)
    return torch.clamp(idx, max=m - 1)


# ----------------------------------------------------------------------------
# Tables with the column shapes of the workloads
# ----------------------------------------------------------------------------

DATE_RANGE = 2557          # dates uniform in [0, 2557)
QTY_LO, QTY_HI = 1, 50
PRICE_LO, PRICE_HI = 100, 10_000_000
DISC_LO, DISC_HI = 0, 10


@dataclass
class FactSpec:
    n: int                  # fact rows
    m: int                  # dimension rows the foreign key points into
    seed: int
    zipf_s: float = 0.0     # 0 = uniform foreign keys
    g32_range: int = 0      # >0 adds the g32 column uniform in [0, g32_range)
    m2: int = 0             # >0 adds fk2 into a second dimension of m2 rows
    seed2: int = 0          # dimension seed for fk2


def fact_columns(spec: FactSpec, rows: torch.Tensor) -> dict:
    """Fact columns for the given row indices (int64 tensor, any device)."""
    sd = spec.seed
    if spec.zipf_s > 0:
        frow = zipf_row(sd, S_FK_ROW, rows, spec.m, spec.zipf_s)
    else:
        frow = uniform_int(sd, S_FK_ROW, rows, 0, spec.m - 1)
    cols = {
        "fk": dim_key(sd, frow),
        "date": uniform_int(sd, S_DATE, rows, 0, DATE_RANGE - 1).to(torch.int32),
        "qty": uniform_int(sd, S_QTY, rows, QTY_LO, QTY_HI),
        "price": uniform_int(sd, S_PRICE, rows, PRICE_LO, PRICE_HI),
        "disc": uniform_int(sd, S_DISC, rows, DISC_LO, DISC_HI),
    }
    if spec.g32_range > 0:
        cols["g32"] = uniform_int(sd, S_G32, rows, 0, spec.g32_range - 1).to(torch.int32)
    if spec.m2 > 0:
        r2 = uniform_int(sd, S_FK2_ROW, rows, 0, spec.m2 - 1)
        cols["fk2"] = dim_key(spec.seed2, r2)
    return cols


def fact_table(spec: FactSpec, device="cpu", chunk: int = 1 << 26) -> dict:
    """All fact rows, generated in chunks to bound temporaries."""
    out = None
    for start in range(0, spec.n, chunk):
        stop = min(spec.n, start + chunk)
        rows = torch.arange(start, stop, dtype=torch.int64, device=device)
        part = fact_columns(spec, rows)
        if out is None:
            out = {k: torch.empty(spec.n, dtype=v.dtype, device=device) for k, v in part.items()}
        for k, v in part.items():
            out[k][start:stop] = v
        del part, rows
    if out is None:
        out = {k: torch.empty(0, dtype=dt, device=device) for k, dt in
               (("fk", torch.int64), ("date", torch.int32), ("qty", torch.int64),
                ("price", torch.int64), ("disc", torch.int64))}
    return out


def dim_columns(seed: int, rows: torch.Tensor, attr_range: int) -> dict:
    key = dim_key(seed, rows)
    attr = uniform_int(seed, S_DIM_ATTR, rows, 0, attr_range - 1).to(torch.int32)
    return {"key": key, "attr": attr}


def dim_table(m: int, seed: int, attr_range: int, device="cpu") -> dict:
    rows = torch.arange(m, dtype=torch.int64, device=device)
    d = dim_columns(seed, rows, attr_range)
    if m and bool((d["key"] == INT64_MIN).any()):
        raise ValueError("generated key collides with the empty-slot sentinel")
    return d


def log_uniform_sizes(count: int, lo: float, hi: float, seed: int) -> list[int]:
    """floor(exp(U(ln lo, ln hi))) for each of ``count`` instances."""
    rows = torch.arange(count, dtype=torch.int64)
    u = unit_float(seed, 99, rows).tolist()
    return [int(math.floor(math.exp(math.log(lo) + x * (math.log(hi) - math.log(lo))))) for x in u]


def uniform_reals(count: int, lo: float, hi: float, seed: int, stream: int) -> list[float]:
    rows = torch.arange(count, dtype=torch.int64)
    u = unit_float(seed, stream, rows).tolist()
    return [lo + x * (hi - lo) for x in u]


# ----------------------------------------------------------------------------
# The workloads: seeds and sizes
# ----------------------------------------------------------------------------

SEED_BASE = 0x5EED0000


@dataclass
class Workload:
    name: str
    fact: FactSpec
    dim_m: int
    dim_seed: int
    attr_range: int
    date_hi: int            # filter keeps date < date_hi
    log2_fanout: int = 6


def workload(idx: int, scale: float = 1.0) -> Workload:
    """The plain-pipeline workloads; ``scale`` shrinks row counts for tests."""
    seed = SEED_BASE + idx
    if idx == 0:
        n, m, a = 1_048_576, 65_536, 25
        return Workload("small: 1,048,576 fact x 65,536 dim, 25 groups",
                        FactSpec(int(n * scale), max(1, int(m * scale)), seed), max(1, int(m * scale)),
                        seed, a, 1500)
    if idx == 1:
        n, m, a = 200_000_000, 25_000_000, 1_500_000
        mm = max(1, int(m * scale))
        return Workload("one GPU share: 200M fact x 25M dim, ~1.5M groups, 64 buckets",
                        FactSpec(int(n * scale), mm, seed), mm, seed, max(1, int(a * scale)), 1500)
    if idx == 2:
        n, m = 100_000_000, 10_000_000
        mm = max(1, int(m * scale))
        return Workload("skew: 100M fact, Zipf(1.0) FK over 10M dim, 5% filter",
                        FactSpec(int(n * scale), mm, seed, zipf_s=1.0, g32_range=2), mm, seed,
                        25, 128)
    raise ValueError(idx)


# ----------------------------------------------------------------------------
# Batched workload: many independent small join + aggregate instances
# ----------------------------------------------------------------------------

@dataclass
class BatchSpec:
    count: int = 512
    build_lo: float = 1e3
    build_hi: float = 2e6
    ratio_lo: float = 8.0
    ratio_hi: float = 16.0
    seed: int = SEED_BASE + 3
    attr_range: int = 25
    date_hi: int = 1500


def batch_sizes(spec: BatchSpec, scale: float = 1.0):
    """(m_i, n_i) per instance: m log-uniform in [build_lo, build_hi], n = round(m * U[ratio])."""
    ms = log_uniform_sizes(spec.count, spec.build_lo, spec.build_hi, spec.seed)
    rs = uniform_reals(spec.count, spec.ratio_lo, spec.ratio_hi, spec.seed, 98)
    out = []
    for m, r in zip(ms, rs):
        mm = max(1, int(m * scale))
        out.append((mm, int(round(mm * r))))
    return out


def batch_tables(spec: BatchSpec, device="cpu", scale: float = 1.0):
    """Dimension and fact columns of every instance, stored back to back in one
    tensor per column; returns (columns, [(dim_offset, m, fact_offset, n)])."""
    sizes = batch_sizes(spec, scale)
    M = sum(m for m, _ in sizes)
    N = sum(n for _, n in sizes)
    cols = {"dim_key": torch.empty(M, dtype=torch.int64, device=device),
            "dim_attr": torch.empty(M, dtype=torch.int32, device=device),
            "fk": torch.empty(N, dtype=torch.int64, device=device),
            "date": torch.empty(N, dtype=torch.int32, device=device),
            "qty": torch.empty(N, dtype=torch.int64, device=device),
            "price": torch.empty(N, dtype=torch.int64, device=device),
            "disc": torch.empty(N, dtype=torch.int64, device=device)}
    layout = []
    mo = no = 0
    for i, (m, n) in enumerate(sizes):
        seed = spec.seed + 1 + i
        d = dim_table(m, seed, spec.attr_range, device=device)
        cols["dim_key"][mo:mo + m] = d["key"]
        cols["dim_attr"][mo:mo + m] = d["attr"]
        f = fact_table(FactSpec(n, m, seed), device=device)
        for k in ("fk", "date", "qty", "price", "disc"):
            cols[k][no:no + n] = f[k]
        layout.append((mo, m, no, n))
        mo += m
        no += n
    return cols, layout


# ----------------------------------------------------------------------------
# Served workload: resident fact table with two foreign keys, two dimensions
# ----------------------------------------------------------------------------

@dataclass
class ServeSpec:
    n: int = 1_600_000_000          # fact rows
    m: int = 200_000_000            # rows of each dimension
    seed: int = SEED_BASE + 4
    code_range: int = 1_500_000     # dim1 attribute (join + aggregate groups)
    attr_range: int = 25            # dim2 attribute (two-join + aggregate groups)


def serve_tables(spec: ServeSpec, device="cpu"):
    """(fact columns with fk and fk2, dim1, dim2).  dim2 uses seed + 1."""
    fact = fact_table(FactSpec(spec.n, spec.m, spec.seed, m2=spec.m, seed2=spec.seed + 1), device=device)
    dim1 = dim_table(spec.m, spec.seed, spec.code_range, device=device)
    dim2 = dim_table(spec.m, spec.seed + 1, spec.attr_range, device=device)
    return fact, dim1, dim2


def serve_queries(count: int, seed: int, date_range: int = DATE_RANGE, kinds=(1, 2, 3, 4)):
    """(kind, date_hi) per query: template uniform over `kinds`, selectivity
    s uniform in [1%, 60%], date_hi = round(s * date_range)."""
    rows = torch.arange(count, dtype=torch.int64)
    ks = uniform_int(seed, 97, rows, 0, len(kinds) - 1).tolist()
    ss = uniform_reals(count, 0.01, 0.60, seed, 96)
    return [(kinds[k], int(round(s * date_range))) for k, s in zip(ks, ss)]


def poisson_arrivals(count: int, qps: float, seed: int):
    """Arrival times (s) of a Poisson process of rate qps (exponential gaps)."""
    u = unit_float(seed, 95, torch.arange(count, dtype=torch.int64)).tolist()
    t, out = 0.0, []
    for x in u:
        t += -math.log(1.0 - x) / qps
        out.append(t)
    return out
