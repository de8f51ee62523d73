"""The batched persistent form: every instance equals the oracle, the plain
per-instance form, and itself under every candidate tuning."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2506_09226_amd as gq
from paper_2506_09226_amd.batch import BatchedJoinAgg, PlainPerInstance

pytestmark = pytest.mark.gpu
AVG_RTOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = gq.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def small_batch():
    spec = synth.BatchSpec(count=48)
    cols, layout = synth.batch_tables(spec, device="cuda", scale=0.004)   # m in ~[4, 8000]
    return spec, cols, layout


def _sorted(h):
    o = np.argsort(h["key32"], kind="stable")
    return {k: (None if v is None else v[o]) for k, v in h.items()}


def _equal(a, b):
    for f in ("key32", "count", "sum_qty", "sum_rev_lo", "sum_rev_hi"):
        assert np.array_equal(a[f], b[f]), f
    for f in ("avg_qty", "avg_rev"):
        np.testing.assert_allclose(a[f], b[f], rtol=AVG_RTOL, atol=0)


def _oracle(cols_h, lay, spec):
    mo, m, no, n = lay
    date = cols_h["date"][no:no + n]
    sel = oracle.filter(date, 0, spec.date_hi)
    prow, pay = oracle.join(cols_h["dim_key"][mo:mo + m], cols_h["dim_attr"][mo:mo + m], cols_h["fk"][no:no + n], sel)
    return oracle.groupby(len(prow), cols_h["qty"][no:no + n], cols_h["price"][no:no + n],
                          cols_h["disc"][no:no + n], rowid=prow, key32=pay)


def test_batch_equals_oracle_and_plain(ctx, small_batch):
    spec, cols, layout = small_batch
    b = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    b.run()
    assert ctx.status() == gq.GQ_OK
    p = PlainPerInstance(ctx, cols, layout, 0, spec.date_hi)
    p.run()
    assert ctx.status() == gq.GQ_OK
    cols_h = {k: v.cpu().numpy() for k, v in cols.items()}
    for lay, gb, gp in zip(layout, b.results(), p.results()):
        e = _oracle(cols_h, lay, spec)
        _equal(_sorted(gb), e)
        _equal(_sorted(gp), e)


@pytest.mark.parametrize("lf,tile,lag,build,fanout", [(0.5, 4096, 0, 256, 1), (0.7, 16384, 3, 1024, 4),
                                                      (0.9, 8192, 1, 4096, 2), (0.3, 65536, 47, 256, 7),
                                                      (0.5, 4096, 5, 1024, 64)])
def test_batch_tunings_identical(ctx, small_batch, lf, tile, lag, build, fanout):
    spec, cols, layout = small_batch
    ref = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    ref.run()
    b = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    t = gq.gq_default_tuning()
    t.load_factor, t.probe_tile, t.lag, t.build_tile, t.init_tile, t.fanout = lf, tile, lag, build, 1024, fanout
    b.tuning = t
    b.run()
    assert ctx.status() == gq.GQ_OK
    for ga, gb in zip(ref.results(), b.results()):
        _equal(_sorted(ga), _sorted(gb))


def test_batch_large_instances_use_device_builds(ctx):
    """Instances big enough for the init/build work items (tables > 4096 slots),
    mixed with tiny ones and an empty fact side."""
    spec = synth.BatchSpec(count=6, build_lo=3000, build_hi=200_000, seed=synth.SEED_BASE + 77)
    cols, layout = synth.batch_tables(spec, device="cuda")
    layout = list(layout)
    mo, m, no, n = layout[0]
    layout[0] = (mo, m, no, 0)                     # no fact rows: zero groups
    b = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    b.run()
    assert ctx.status() == gq.GQ_OK
    cols_h = {k: v.cpu().numpy() for k, v in cols.items()}
    res = b.results()
    assert len(res[0]["count"]) == 0
    for lay, g in zip(layout[1:], res[1:]):
        _equal(_sorted(g), _oracle(cols_h, lay, spec))


def test_batch_signed_and_wide_revenues(ctx):
    """Signed quantities and revenues: most fit 64 bits (split LDS sums with
    negative high halves), a few need more (sent to the global table); group
    totals pass 2^64.  Equal to the oracle and to the plain form."""
    spec = synth.BatchSpec(count=8, build_lo=50, build_hi=20_000, seed=synth.SEED_BASE + 93)
    cols, layout = synth.batch_tables(spec, device="cuda")
    r = np.random.default_rng(93)
    nt = cols["price"].numel()
    price = r.integers(1, 1 << 55, size=nt, dtype=np.int64) * np.where(r.random(nt) < 0.4, -1, 1)
    wide = r.random(nt) < 0.03
    price[wide] = ((1 << 62) - r.integers(0, 1000, size=int(wide.sum()))) * np.where(r.random(int(wide.sum())) < 0.5,
                                                                                       -1, 1)
    cols["price"].copy_(torch.from_numpy(price))
    cols["qty"].copy_(torch.from_numpy(r.integers(-(1 << 40), 1 << 40, size=nt, dtype=np.int64)))
    cols["disc"].copy_(torch.from_numpy(r.integers(-20, 11, size=nt).astype(np.int64)))
    b = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    b.run()
    assert ctx.status() == gq.GQ_OK
    p = PlainPerInstance(ctx, cols, layout, 0, spec.date_hi)
    p.run()
    assert ctx.status() == gq.GQ_OK
    cols_h = {k: v.cpu().numpy() for k, v in cols.items()}
    big = False
    for lay, gb, gp in zip(layout, b.results(), p.results()):
        e = _oracle(cols_h, lay, spec)
        big |= any(abs(v) >= 1 << 64 for v in oracle.sum_rev_int(e))
        _equal(_sorted(gb), e)
        _equal(_sorted(gp), e)
    assert big


def test_batch_autotune_and_cache(ctx, small_batch, tmp_path):
    spec, cols, layout = small_batch
    b = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    path = str(tmp_path / "tune.txt")
    t1, ms1 = b.autotune(path)
    assert ms1 > 0 and t1.probe_tile % 4096 == 0
    b2 = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    t2, ms2 = b2.autotune(path)                     # served from the cache
    assert t2.as_dict() == t1.as_dict() and ms2 == pytest.approx(ms1, rel=1e-3)
    b2.run()
    ref = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    ref.run()
    for ga, gb in zip(ref.results(), b2.results()):
        _equal(_sorted(ga), _sorted(gb))


def test_batch_duplicate_key_reported(ctx):
    spec = synth.BatchSpec(count=3, build_lo=100, build_hi=10_000, seed=synth.SEED_BASE + 91)
    cols, layout = synth.batch_tables(spec, device="cuda")
    mo, m, _, _ = layout[1]
    cols["dim_key"][mo + 1] = cols["dim_key"][mo]
    b = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    b.run()
    assert ctx.status() == gq.GQ_ERR_DUPLICATE_KEY


@pytest.mark.parametrize("bad_big", [False, True])
def test_batch_error_flagged_per_instance(ctx, bad_big):
    """One instance with a duplicate build key (built in LDS, or by device
    compare-and-swap when its table is large): its own status says so, every
    other instance reports GQ_OK and equals the oracle."""
    spec = synth.BatchSpec(count=12, build_lo=200, build_hi=60_000, seed=synth.SEED_BASE + 95)
    cols, layout = synth.batch_tables(spec, device="cuda")
    sizes = [m for _, m, _, _ in layout]
    bad = int(np.argmax(sizes)) if bad_big else int(np.argmin(sizes))
    mo, m, _, _ = layout[bad]
    assert (m > 4096 // 2) == bad_big                   # an LDS-built table only when small
    orig = cols["dim_key"][mo + m - 1].clone()
    cols["dim_key"][mo + m - 1] = cols["dim_key"][mo]
    b = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    b.run()
    st = b.statuses()
    assert ctx.status() == gq.GQ_ERR_DUPLICATE_KEY
    assert st[bad] == gq.GQ_ERR_DUPLICATE_KEY
    assert all(x == gq.GQ_OK for i, x in enumerate(st) if i != bad)
    cols_h = {k: v.cpu().numpy() for k, v in cols.items()}
    for i, (lay, g) in enumerate(zip(layout, b.results())):
        if i != bad:
            _equal(_sorted(g), _oracle(cols_h, lay, spec))
    # the same batch without the error: every status back to GQ_OK, all exact
    cols["dim_key"][mo + m - 1] = orig
    b.run()
    assert ctx.status() == gq.GQ_OK and all(x == gq.GQ_OK for x in b.statuses())
    cols_h = {k: v.cpu().numpy() for k, v in cols.items()}
    _equal(_sorted(b.results()[bad]), _oracle(cols_h, layout[bad], spec))


def test_batch_int64_min_foreign_keys_match_nothing(ctx):
    """A foreign key equal to INT64_MIN (the empty-slot marker) must not
    match an empty slot: those rows drop out of the join, as in the oracle."""
    spec = synth.BatchSpec(count=6, build_lo=100, build_hi=50_000, seed=synth.SEED_BASE + 97)
    cols, layout = synth.batch_tables(spec, device="cuda")
    r = np.random.default_rng(97)
    nt = cols["fk"].numel()
    hit = torch.from_numpy(r.random(nt) < 0.1).cuda()
    cols["fk"].masked_fill_(hit, -(1 << 63))
    b = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    b.run()
    assert ctx.status() == gq.GQ_OK and all(x == gq.GQ_OK for x in b.statuses())
    cols_h = {k: v.cpu().numpy() for k, v in cols.items()}
    for lay, g in zip(layout, b.results()):
        _equal(_sorted(g), _oracle(cols_h, lay, spec))


def test_batch_wait_bound_forced_from_host(ctx):
    """The bounded wait of the batch kernel, forced from the host with a
    one-poll bound: probe and build items that find their inputs unfinished
    skip their work and report GQ_ERR_TIMEOUT, and the kernel still drains its
    queue and returns.  Back at the default bound the same batch is exact."""
    spec = synth.BatchSpec(count=24, build_lo=5_000, build_hi=200_000, seed=synth.SEED_BASE + 99)
    cols, layout = synth.batch_tables(spec, device="cuda")
    b = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    t = gq.gq_default_tuning()
    t.lag = 0                                  # probes queued right behind their own builds
    b.tuning = t
    ctx.set_wait_limit(1)
    try:
        b.run()
        torch.cuda.synchronize()
        st = b.statuses()
        word = ctx.status()
    finally:
        ctx.set_wait_limit(0)
    assert word == gq.GQ_ERR_TIMEOUT
    assert all(x in (gq.GQ_OK, gq.GQ_ERR_TIMEOUT) for x in st) and gq.GQ_ERR_TIMEOUT in st
    b.run()
    assert ctx.status() == gq.GQ_OK and all(x == gq.GQ_OK for x in b.statuses())
    cols_h = {k: v.cpu().numpy() for k, v in cols.items()}
    for lay, g in zip(layout, b.results()):
        _equal(_sorted(g), _oracle(cols_h, lay, spec))


def test_batch_full_size_sampled(ctx, tmp_path):
    """The benchmark's batched workload at full size (512 instances, build
    sizes log-uniform in [1e3, 2e6], probe sizes 8-16x build: 1.75G probe
    rows) in the benchmark's launch configuration (autotuned).  Every
    instance: its group counts and sums equal totals over its selected rows
    computed separately (every foreign key names a key of its own instance, so
    |join| = |selection|).  The smallest, the largest and one instance drawn
    at random: element by element against the oracle."""
    spec = synth.BatchSpec()
    cols, layout = synth.batch_tables(spec, device="cuda")
    assert len(layout) == 512
    b = BatchedJoinAgg(ctx, cols, layout, 0, spec.date_hi)
    b.autotune(str(tmp_path / "batch_tuning.txt"))
    b.run()
    torch.cuda.synchronize()
    assert ctx.status() == gq.GQ_OK
    res = b.results()
    keep = cols["date"] < spec.date_hi
    zero = torch.zeros((), dtype=torch.int64, device="cuda")
    cs_cnt = torch.cumsum(keep.to(torch.int64), 0)
    cs_qty = torch.cumsum(torch.where(keep, cols["qty"], zero), 0)
    cs_rev = torch.cumsum(torch.where(keep, cols["price"] * (100 - cols["disc"]), zero), 0)
    del keep
    ends = torch.tensor([no + n - 1 for _, _, no, n in layout], dtype=torch.int64, device="cuda")
    starts = torch.tensor([no - 1 for _, _, no, _ in layout], dtype=torch.int64, device="cuda")

    def seg(cs):
        hi = cs[ends].cpu().numpy()
        lo = np.where(starts.cpu().numpy() >= 0, cs[starts.clamp(min=0)].cpu().numpy(), 0)
        return hi - lo

    e_cnt, e_qty, e_rev = seg(cs_cnt), seg(cs_qty), seg(cs_rev)
    for i, g in enumerate(res):
        assert int(g["count"].sum()) == e_cnt[i], i
        assert int(g["sum_qty"].sum()) == e_qty[i], i
        assert bool((g["sum_rev_hi"] == 0).all()) and int(g["sum_rev_lo"].astype(np.int64).sum()) == e_rev[i], i
    del cs_cnt, cs_qty, cs_rev
    sizes = [m for _, m, _, _ in layout]
    pick = {int(np.argmin(sizes)), int(np.argmax(sizes)), int(np.random.default_rng(5).integers(0, len(layout)))}
    for i in sorted(pick):
        mo, m, no, n = layout[i]
        h = {k: cols[k][a:a + c].cpu().numpy() for k, a, c in
             (("dim_key", mo, m), ("dim_attr", mo, m), ("fk", no, n), ("date", no, n), ("qty", no, n),
              ("price", no, n), ("disc", no, n))}
        e = _oracle(h, (0, m, 0, n), spec)
        _equal(_sorted(res[i]), e)
