"""GPU parity of every operator against the CPU oracle, through the C ABI.

Integers, keys, row ids and 128-bit sums must match bit for bit; float64
averages within 1e-12 relative.  Sizes span several tiles plus a ragged tail
(tiles are 4096 or 8192 rows), and the degenerate cases (empty input, no
match, one group, ties, duplicate and invalid keys) are covered."""
import numpy as np
import pytest
import torch

import oracle
import paper_2506_09226_amd as gq

pytestmark = pytest.mark.gpu

AVG_RTOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = gq.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t, n=None):
    t = t if n is None else t[:n]
    return t.cpu().numpy()


def rng(seed):
    return np.random.default_rng(seed)


# ------------------------------------------------------------------ filter ---

@pytest.mark.parametrize("n", [0, 1, 63, 8191, 8192, 8193, 32767, 32768, 32769, 40963, 100_003, 1_000_000,
                               3_000_001])
@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_filter(ctx, n, dtype):
    r = rng(n)
    col = r.integers(0, 2557, size=n).astype(dtype)
    exp = oracle.filter(col, 100, 1500)
    out, cnt = gq.gq_filter(ctx, dev(col), 100, 1500)
    assert ctx.status() == gq.GQ_OK
    k = int(cnt.item())
    assert k == len(exp)
    assert np.array_equal(host(out, k), exp)


@pytest.mark.parametrize("n", [5000, 123_457])
def test_filter_with_selection_and_device_count(ctx, n):
    r = rng(7)
    col = r.integers(-1000, 1000, size=n).astype(np.int64)
    sel_in = np.sort(r.choice(n, size=n // 3, replace=False)).astype(np.int32)
    used = len(sel_in) - 17                                   # device count below the bound
    exp = oracle.filter(col, -10, 400, sel_in=sel_in[:used])
    n_dev = torch.tensor([used], dtype=torch.int64, device="cuda")
    out, cnt = gq.gq_filter(ctx, dev(col), -10, 400, sel_in=dev(sel_in), n_dev=n_dev)
    k = int(cnt.item())
    assert k == len(exp) and np.array_equal(host(out, k), exp)


@pytest.mark.parametrize("used", [0, 1, 8192, 40_000, 65_537])
def test_filter_device_count_far_below_bound(ctx, used):
    """The grid is sized by the bound (300,000 rows, ten groups of four tiles);
    the device count ends inside an early group, at a group edge, or at zero,
    and the groups past it do nothing."""
    n = 300_000
    col = rng(used + 3).integers(0, 2557, size=n).astype(np.int32)
    exp = oracle.filter(col[:used], 0, 1500)
    n_dev = torch.tensor([used], dtype=torch.int64, device="cuda")
    out, cnt = gq.gq_filter(ctx, dev(col), 0, 1500, n_dev=n_dev)
    assert ctx.status() == gq.GQ_OK
    k = int(cnt.item())
    assert k == len(exp) and np.array_equal(host(out, k), exp)


def test_filter_extremes(ctx):
    col = np.array([-(1 << 63), -1, 0, 1, (1 << 63) - 1] * 3000, dtype=np.int64)
    for lo, hi in [(-(1 << 63), (1 << 63) - 1), (0, 1), (5, 5), (1, -1)]:
        exp = oracle.filter(col, lo, hi)
        out, cnt = gq.gq_filter(ctx, dev(col), lo, hi)
        k = int(cnt.item())
        assert np.array_equal(host(out, k), exp)


# --------------------------------------------------------------- partition ---

@pytest.mark.parametrize("log2p", [0, 1, 3, 6, 8])
@pytest.mark.parametrize("n", [1, 4095, 4096, 4097, 70_001, 771 * 4096 + 1])
def test_partition(ctx, log2p, n):
    """Stable partition against the oracle; the largest size spans three
    whole rounds of 32-tile chunks dealt over the eight XCDs (768 tiles)
    plus a tail of tiles that keep their own index."""
    r = rng(n * 10 + log2p)
    key = r.integers(-(1 << 63), (1 << 63) - 1, size=n, dtype=np.int64)
    c32 = r.integers(0, 2557, size=n).astype(np.int32)
    c64 = r.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64)
    ek, (e32, e64), erow, eoff = oracle.partition(key, log2p, [c32, c64])
    k, (o32, o64), row, off = gq.gq_radix_partition(ctx, dev(key), log2p, [dev(c32), dev(c64)])
    assert ctx.status() == gq.GQ_OK
    assert np.array_equal(host(off), eoff)
    assert np.array_equal(host(k), ek)
    assert np.array_equal(host(row), erow)
    assert np.array_equal(host(o32), e32) and np.array_equal(host(o64), e64)


def test_partition_skewed_keys(ctx):
    """Few distinct keys: one bucket gets most rows; order must stay stable."""
    r = rng(5)
    key = r.choice(np.array([3, 3, 3, 3, 17, 99, -5], dtype=np.int64), size=50_000)
    ek, _, erow, eoff = oracle.partition(key, 6)
    k, _, row, off = gq.gq_radix_partition(ctx, dev(key), 6)
    assert np.array_equal(host(off), eoff) and np.array_equal(host(row), erow) and np.array_equal(host(k), ek)


def test_partition_empty(ctx):
    k, _, row, off = gq.gq_radix_partition(ctx, torch.empty(0, dtype=torch.int64, device="cuda"), 6)
    assert host(off).tolist() == [0] * 65


def test_partition_rejects_fanout(ctx):
    with pytest.raises(gq.GQError) as e:
        gq.gq_radix_partition(ctx, dev(np.zeros(10, np.int64)), 9)
    assert e.value.code == gq.GQ_ERR_UNSUPPORTED


# -------------------------------------------------------------------- join ---

def _dim(m, seed):
    r = rng(seed)
    keys = np.unique(r.integers(-(1 << 62), 1 << 62, size=m + m // 10 + 10, dtype=np.int64))
    keys = r.permutation(keys)[:m]
    pay = r.integers(0, 1 << 30, size=m).astype(np.int32)
    return keys, pay


@pytest.mark.parametrize("m,n", [(1, 10), (100, 10_000), (65_536, 300_001), (5000, 4096)])
def test_join_build_probe(ctx, m, n):
    r = rng(m + n)
    bkey, bpay = _dim(m, m)
    fk = np.where(r.random(n) < 0.8, bkey[r.integers(0, m, size=n)], r.integers(-(1 << 62), 1 << 62, size=n))
    fk = fk.astype(np.int64)
    sel = np.sort(r.choice(n, size=n // 2, replace=False)).astype(np.int32)
    table = gq.gq_join_build(ctx, dev(bkey), dev(bpay))
    for s in (None, sel):
        ep, ey = oracle.join(bkey, bpay, fk, s)
        prow, pay, cnt = gq.gq_join_probe(ctx, table, dev(fk), sel=None if s is None else dev(s))
        assert ctx.status() == gq.GQ_OK
        k = int(cnt.item())
        assert k == len(ep)
        assert np.array_equal(host(prow, k), ep) and np.array_equal(host(pay, k), ey)


def test_join_high_load_factor_and_device_counts(ctx):
    r = rng(3)
    bkey, bpay = _dim(57_000, 3)
    fk = bkey[r.integers(0, 57_000, size=200_000)]
    bsel = np.sort(r.choice(57_000, size=50_000, replace=False)).astype(np.int32)
    n_b = torch.tensor([49_000], dtype=torch.int64, device="cuda")
    table = gq.gq_join_build(ctx, dev(bkey), dev(bpay), sel=dev(bsel), n_dev=n_b, load_factor=0.9)
    used_b = bsel[:49_000]
    psel = np.arange(0, 200_000, 3, dtype=np.int32)
    n_p = torch.tensor([60_000], dtype=torch.int64, device="cuda")
    ep, ey = oracle.join(bkey[used_b], bpay[used_b], fk, psel[:60_000])
    prow, pay, cnt = gq.gq_join_probe(ctx, table, dev(fk), sel=dev(psel), n_dev=n_p)
    assert ctx.status() == gq.GQ_OK
    k = int(cnt.item())
    assert k == len(ep) and np.array_equal(host(prow, k), ep) and np.array_equal(host(pay, k), ey)


@pytest.fixture
def build_path(request, monkeypatch):
    monkeypatch.setenv("GQ_JOIN_BUILD", request.param)
    return request.param


@pytest.mark.parametrize("build_path", ["cas", "region"], indirect=True)
@pytest.mark.parametrize("m,lf", [(300_000, 0.5), (1_200_000, 0.5), (900_000, 0.9), (70_000, 0.9),
                                  (300_000, 0.2), (2_000_000, 0.0075)])
def test_join_build_paths(ctx, build_path, m, lf):
    """Both builds (device CAS; LDS regions after a radix sort by region)
    give tables on which the probe equals the oracle: regions sorted in one
    pass (2^8 regions and fewer), in two levels with 1, 2 and 8 bits in the
    second (2^9, 2^10 and 2^16 regions), and with region overflow at load
    factor 0.9."""
    r = rng(m)
    bkey, bpay = _dim(m, m + 1)
    n = 400_000
    fk = np.where(r.random(n) < 0.9, bkey[r.integers(0, m, size=n)], r.integers(-(1 << 62), 1 << 62, size=n))
    fk = fk.astype(np.int64)
    table = gq.gq_join_build(ctx, dev(bkey), dev(bpay), load_factor=lf)
    assert ctx.status() == gq.GQ_OK
    ep, ey = oracle.join(bkey, bpay, fk)
    prow, pay, cnt = gq.gq_join_probe(ctx, table, dev(fk))
    k = int(cnt.item())
    assert k == len(ep) and np.array_equal(host(prow, k), ep) and np.array_equal(host(pay, k), ey)


def _fmix64_inv_np(h):
    """Inverse of the MurmurHash3 64-bit finalizer: xor-shifts by 33 undo
    themselves, and each multiplier is undone by its inverse modulo 2^64."""
    h = h.astype(np.uint64)
    inv2 = np.uint64(pow(0xC4CEB9FE1A85EC53, -1, 1 << 64))
    inv1 = np.uint64(pow(0xFF51AFD7ED558CCD, -1, 1 << 64))
    h ^= h >> np.uint64(33)
    h *= inv2
    h ^= h >> np.uint64(33)
    h *= inv1
    h ^= h >> np.uint64(33)
    return h


@pytest.mark.parametrize("build_path", ["region"], indirect=True)
def test_join_region_build_uneven_buckets(ctx, build_path):
    """Keys whose hashes all have their top 4 bits clear fill 16 of the 256
    first-level buckets of the region sort and leave 240 empty; 2^22 slots
    give 2^10 regions, so each bucket is split 4 ways by the second level.
    The table still answers every probe as the oracle does."""
    r = rng(4242)
    m = 200_000
    h = np.unique(r.integers(0, 1 << 60, size=m + 1000, dtype=np.uint64))[:m]
    r.shuffle(h)
    bkey = _fmix64_inv_np(h).view(np.int64)
    assert np.array_equal(_fmix64_np(bkey.view(np.uint64)), h)            # the keys hash back
    assert not np.any(bkey == np.iinfo(np.int64).min)
    bpay = r.integers(-(1 << 31), (1 << 31) - 1, size=m).astype(np.int32)
    lf = 0.05
    assert gq.gq_join_table_bytes(m, lf) == 256 + (1 << 22) * 16       # 2^10 regions of 4096 slots
    table = gq.gq_join_build(ctx, dev(bkey), dev(bpay), load_factor=lf)
    assert ctx.status() == gq.GQ_OK
    n = 300_000
    fk = np.where(r.random(n) < 0.9, bkey[r.integers(0, m, size=n)], r.integers(-(1 << 62), 1 << 62, size=n))
    fk = fk.astype(np.int64)
    ep, ey = oracle.join(bkey, bpay, fk)
    prow, pay, cnt = gq.gq_join_probe(ctx, table, dev(fk))
    k = int(cnt.item())
    assert k == len(ep) and np.array_equal(host(prow, k), ep) and np.array_equal(host(pay, k), ey)


@pytest.mark.parametrize("build_path", ["region"], indirect=True)
def test_join_region_build_errors(ctx, build_path):
    keys = np.arange(300_000, dtype=np.int64) * 7 + 1
    keys[123_456] = keys[77]
    gq.gq_join_build(ctx, dev(keys), dev(np.zeros(300_000, np.int32)))
    assert ctx.status() == gq.GQ_ERR_DUPLICATE_KEY
    keys = np.arange(300_000, dtype=np.int64) * 7 + 1
    keys[5] = -(1 << 63)
    gq.gq_join_build(ctx, dev(keys), dev(np.zeros(300_000, np.int32)))
    assert ctx.status() == gq.GQ_ERR_INVALID_KEY


def test_join_duplicate_and_invalid_keys(ctx):
    gq.gq_join_build(ctx, dev(np.array([5, 6, 5], np.int64)), dev(np.zeros(3, np.int32)))
    assert ctx.status() == gq.GQ_ERR_DUPLICATE_KEY
    gq.gq_join_build(ctx, dev(np.array([5, -(1 << 63)], np.int64)), dev(np.zeros(2, np.int32)))
    assert ctx.status() == gq.GQ_ERR_INVALID_KEY
    assert ctx.status() == gq.GQ_OK                            # cleared by the read


def test_join_empty_sides(ctx):
    table = gq.gq_join_build(ctx, torch.empty(0, dtype=torch.int64, device="cuda"),
                             torch.empty(0, dtype=torch.int32, device="cuda"))
    prow, pay, cnt = gq.gq_join_probe(ctx, table, dev(np.arange(1000, dtype=np.int64)))
    assert int(cnt.item()) == 0
    prow, pay, cnt = gq.gq_join_probe(ctx, table, torch.empty(0, dtype=torch.int64, device="cuda"))
    assert int(cnt.item()) == 0


@pytest.mark.parametrize("m,n,order,fanout,lf", [
    (1000, 1, "random", 0, 0.5),                 # cache-resident table: the ordered probe
    (60_000, 300_001, "random", 6, 0.5),         # cache-resident table: the ordered probe
    (2_000_000, 3_000_000, "partitioned", 6, 0.5),   # 2^22 slots: 64 x 16 regions
    (700_000, 2_000_000, "partitioned", 6, 0.5),     # 2^21 slots: 64 x 8 regions
    (400_000, 1_000_000, "random", 0, 0.5),      # 2^20 slots, no high part: 256 regions, any order
    (2_000_000, 1_000_000, "random", 6, 0.5),    # wrong order for the hint: nearly all rows stray
    (2_000_000, 1_000_000, "random", 2, 0.5),    # 4 high parts: three quarters stray
    (1_800_000, 2_500_000, "partitioned", 6, 0.9),   # long probe runs: many cross a region's end
    (2_000_000, 3_000_000, "heavy", 6, 0.5),         # heavy keys: their regions are split into several items
    (1_800_000, 2_500_000, "heavy", 6, 0.9),
    (400_000, 1_000_000, "heavy", 0, 0.5),
])
def test_join_probe_partitioned(ctx, m, n, order, fanout, lf):
    """The partitioned probe returns exactly the output of the ordered probe
    (the oracle, in probe order): with and without a selection, with misses,
    with a device count, on a probe stream in radix-partition order and on a
    random one, with regions held in LDS and with the fallbacks, and with
    heavy keys (40%, 10% and 5% of the probes) whose regions the region pass
    splits across workgroups."""
    r = rng(m + 7 * n + fanout)
    bkey, bpay = _dim(m, m + 3)
    fk = np.where(r.random(n) < 0.85, bkey[r.integers(0, m, size=n)], r.integers(-(1 << 62), 1 << 62, size=n))
    fk = fk.astype(np.int64)
    if order == "heavy":
        u = r.random(n)
        fk[u < 0.40] = bkey[7]
        fk[(u >= 0.40) & (u < 0.50)] = bkey[m // 2]
        fk[(u >= 0.50) & (u < 0.55)] = bkey[m - 1]
    if order in ("partitioned", "heavy"):      # stable order by the top `fanout` hash bits, as after the partition
        fk = fk[np.argsort(_fmix64_np(fk) >> np.uint64(64 - fanout), kind="stable")]
    table = gq.gq_join_build(ctx, dev(bkey), dev(bpay), load_factor=lf)
    sel = np.sort(r.choice(n, size=(2 * n) // 3, replace=False)).astype(np.int32)
    for s in (None, sel):
        ep, ey = oracle.join(bkey, bpay, fk, s)
        prow, pay, cnt = gq.gq_join_probe_partitioned(ctx, table, dev(fk), sel=None if s is None else dev(s),
                                                      log2_fanout=fanout)
        assert ctx.status() == gq.GQ_OK
        k = int(cnt.item())
        assert k == len(ep)
        assert np.array_equal(host(prow, k), ep) and np.array_equal(host(pay, k), ey)
    h = len(sel) // 2
    n_dev = torch.tensor([h], dtype=torch.int64, device="cuda")
    ep, ey = oracle.join(bkey, bpay, fk, sel[:h])
    prow, pay, cnt = gq.gq_join_probe_partitioned(ctx, table, dev(fk), sel=dev(sel), n_dev=n_dev,
                                                  log2_fanout=fanout)
    k = int(cnt.item())
    assert k == len(ep)
    assert np.array_equal(host(prow, k), ep) and np.array_equal(host(pay, k), ey)


def test_join_probe_partitioned_table_size_checked(ctx):
    """A table size that does not match the table's header is reported."""
    bkey, bpay = _dim(2_000_000, 11)
    table = gq.gq_join_build(ctx, dev(bkey), dev(bpay))
    fk = dev(bkey[:100_000])
    gq.gq_join_probe_partitioned(ctx, table[:table.numel() - 4096], fk, log2_fanout=6)
    assert ctx.status() == gq.GQ_ERR_INVALID_ARG
    prow, pay, cnt = gq.gq_join_probe_partitioned(ctx, table, fk, log2_fanout=6)
    assert ctx.status() == gq.GQ_OK and int(cnt.item()) == 100_000


def test_join_probe_partitioned_empty(ctx):
    bkey, bpay = _dim(100, 5)
    table = gq.gq_join_build(ctx, dev(bkey), dev(bpay))
    prow, pay, cnt = gq.gq_join_probe_partitioned(ctx, table, torch.empty(0, dtype=torch.int64, device="cuda"))
    assert int(cnt.item()) == 0
    n_dev = torch.zeros(1, dtype=torch.int64, device="cuda")
    prow, pay, cnt = gq.gq_join_probe_partitioned(ctx, table, dev(bkey), n_dev=n_dev)
    assert int(cnt.item()) == 0


# ---------------------------------------------------------------- group-by ---

def _check_groups(res: gq.GroupResult, exp: dict, has64: bool, has32: bool):
    got = res.host()
    g = len(got["count"])
    assert g == len(exp["count"])
    if has64 and has32:
        order = np.lexsort((got["key32"], got["key64"]))
    elif has64:
        order = np.argsort(got["key64"], kind="stable")
    elif has32:
        order = np.argsort(got["key32"], kind="stable")
    else:
        order = np.arange(g)
    for f in ("key64", "key32", "count", "sum_qty", "sum_rev_lo", "sum_rev_hi"):
        if exp[f] is None:
            continue
        assert np.array_equal(got[f][order], exp[f]), f
    for f in ("avg_qty", "avg_rev"):
        np.testing.assert_allclose(got[f][order], exp[f], rtol=AVG_RTOL, atol=0)


def _gb_inputs(n, nv, seed, groups, big=False):
    r = rng(seed)
    rowid = r.integers(0, nv, size=n).astype(np.int32)
    key32 = r.integers(0, groups, size=n).astype(np.int32)
    key64 = (r.integers(0, 3, size=nv) * 1_000_000_007 - 7).astype(np.int64)
    if big:
        qty = r.integers(1 << 60, 1 << 62, size=nv, dtype=np.int64)
        price = r.integers((1 << 62) - 1000, 1 << 62, size=nv, dtype=np.int64)
        price[::5] *= -1
        disc = r.integers(-50, 11, size=nv).astype(np.int64)
    else:
        qty = r.integers(1, 51, size=nv).astype(np.int64)
        price = r.integers(100, 10_000_001, size=nv).astype(np.int64)
        disc = r.integers(0, 11, size=nv).astype(np.int64)
    return rowid, key32, key64, qty, price, disc


@pytest.mark.parametrize("n,groups", [(1, 1), (4097, 25), (300_000, 25), (200_000, 500), (250_003, 5000),
                                      (400_000, 150_000)])
def test_groupby_key32_via_rowid(ctx, n, groups):
    rowid, key32, _, qty, price, disc = _gb_inputs(n, 2 * n + 1, n + groups, groups)
    exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key32=key32)
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key32=dev(key32),
                            max_groups=groups)
    assert ctx.status() == gq.GQ_OK
    _check_groups(res, exp, False, True)


@pytest.mark.parametrize("max_groups", [64, 4000])
def test_groupby_composite_key_int128_carry(ctx, max_groups):
    n = 60_000
    rowid, key32, key64, qty, price, disc = _gb_inputs(n, n, 11, 7, big=True)
    exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key64=key64, key64_by_rowid=True, key32=key32)
    assert any(abs(v) >= 1 << 64 for v in oracle.sum_rev_int(exp))
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key64=dev(key64),
                            key64_by_rowid=True, key32=dev(key32), max_groups=max_groups)
    assert ctx.status() == gq.GQ_OK
    _check_groups(res, exp, True, True)


@pytest.mark.parametrize("max_groups", [16, 100_000])
def test_groupby_key64_direct_no_rowid(ctx, max_groups):
    n = 150_000
    r = rng(21)
    key64 = r.integers(-(1 << 63), (1 << 63) - 1, size=min(max_groups, 10), dtype=np.int64)[r.integers(0, min(max_groups, 10), size=n)]
    qty = r.integers(1, 51, size=n).astype(np.int64)
    price = r.integers(100, 10_000_001, size=n).astype(np.int64)
    disc = r.integers(0, 11, size=n).astype(np.int64)
    exp = oracle.groupby(n, qty, price, disc, key64=key64)
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), key64=dev(key64), max_groups=max_groups)
    _check_groups(res, exp, True, False)


@pytest.mark.parametrize("max_groups", [64, 100_000])
@pytest.mark.parametrize("composite", [False, True])
def test_groupby_extreme_keys(ctx, max_groups, composite):
    """Keys at the extremes of int64 and int32 (INT64_MIN, INT32_MIN among
    them) beside ordinary keys, on the small and the large path, key64 alone
    and composite: every group exact."""
    n = 120_000
    r = rng(23)
    k64s = np.array([-(1 << 63), (1 << 63) - 1, -1, 0, 1, 123_456_789_012], dtype=np.int64)
    k32s = np.array([-(1 << 31), (1 << 31) - 1, -1, 0, 7], dtype=np.int32)
    key64 = k64s[r.integers(0, len(k64s), size=n)]
    key32 = k32s[r.integers(0, len(k32s), size=n)] if composite else None
    qty = r.integers(1, 51, size=n).astype(np.int64)
    price = r.integers(100, 10_000_001, size=n).astype(np.int64)
    disc = r.integers(0, 11, size=n).astype(np.int64)
    exp = oracle.groupby(n, qty, price, disc, key64=key64, key32=key32)
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), key64=dev(key64),
                            key32=dev(key32) if composite else None, max_groups=max_groups)
    assert ctx.status() == gq.GQ_OK
    _check_groups(res, exp, True, composite)


@pytest.mark.parametrize("groups", [25, 5000])
def test_groupby_row_filter(ctx, groups):
    """Only rows whose value row passes filter_lo <= filter[v] < filter_hi."""
    n = 200_000
    rowid, key32, _, qty, price, disc = _gb_inputs(n, n, 55 + groups, groups)
    fcol = rng(5).integers(0, 2557, size=n).astype(np.int32)
    keep = np.nonzero(fcol[rowid] < 700)[0]
    exp = oracle.groupby(len(keep), qty, price, disc, rowid=rowid[keep], key32=key32[keep])
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key32=dev(key32),
                            max_groups=groups, filter_col=dev(fcol), filter_lo=0, filter_hi=700)
    assert ctx.status() == gq.GQ_OK
    _check_groups(res, exp, False, True)


def test_groupby_large_path_edges(ctx):
    """The large path (bucketed) with no key at all (one group), with a device
    row count of zero, and with a device row count well below the bound
    (only the first rows count)."""
    n = 100_003
    _, key32, _, qty, price, disc = _gb_inputs(n, n, 12, 3000)
    exp = oracle.groupby(n, qty, price, disc)
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), max_groups=5000)
    assert ctx.status() == gq.GQ_OK
    _check_groups(res, exp, False, False)
    n_dev = torch.zeros(1, dtype=torch.int64, device="cuda")
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), n_dev=n_dev, key32=dev(key32), max_groups=5000)
    assert ctx.status() == gq.GQ_OK and int(res.n_groups.item()) == 0
    part = 70_001
    n_dev.fill_(part)
    exp = oracle.groupby(part, qty, price, disc, key32=key32)
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), n_dev=n_dev, key32=dev(key32), max_groups=5000)
    assert ctx.status() == gq.GQ_OK
    _check_groups(res, exp, False, True)


@pytest.mark.parametrize("n", [32_767, 300_003])
def test_groupby_large_path_key32_by_rowid_filtered(ctx, n):
    """Large path with the key read at the value row (key32[rowid[j]]) and a
    row filter: chunk and tile edges (32K-row chunks, 4096-row tiles) with a
    ragged tail, every group exact."""
    r = rng(47)
    nv = 2 * n + 5
    rowid = r.integers(0, nv, size=n).astype(np.int32)
    keyv = r.integers(0, 20_000, size=nv).astype(np.int32)
    qty = r.integers(1, 51, size=nv).astype(np.int64)
    price = r.integers(100, 10_000_001, size=nv).astype(np.int64)
    disc = r.integers(0, 11, size=nv).astype(np.int64)
    fcol = r.integers(0, 2557, size=nv).astype(np.int32)
    keep = np.nonzero(fcol[rowid] < 1500)[0]
    exp = oracle.groupby(len(keep), qty, price, disc, rowid=rowid[keep], key32=keyv, key32_by_rowid=True)
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key32=dev(keyv),
                            key32_by_rowid=True, max_groups=40_000, filter_col=dev(fcol), filter_lo=0,
                            filter_hi=1500)
    assert ctx.status() == gq.GQ_OK
    _check_groups(res, exp, False, True)


def test_groupby_no_key_and_empty(ctx):
    n = 10_000
    _, _, _, qty, price, disc = _gb_inputs(n, n, 4, 1)
    exp = oracle.groupby(n, qty, price, disc)
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), max_groups=1)
    _check_groups(res, exp, False, False)
    n_dev = torch.zeros(1, dtype=torch.int64, device="cuda")
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), n_dev=n_dev, key32=dev(np.zeros(n, np.int32)),
                            max_groups=4)
    assert int(res.n_groups.item()) == 0


@pytest.mark.parametrize("composite", [False, True])
@pytest.mark.parametrize("max_groups", [1024, 4000])
@pytest.mark.parametrize("n", [1, 2048, 5000, 16383])
def test_groupby_large_path_few_rows(ctx, n, max_groups, composite):
    """The large path (max_groups above the small path's bound) on inputs of
    fewer than eight scatter tiles: the tiles are split over the eight XCD
    ranges, some of them empty."""
    # at most 900 distinct keys; composite keys pair 3 key64 values with 300 key32 values
    rowid, key32, key64, qty, price, disc = _gb_inputs(n, n + 3, 31 + n, 300 if composite else 900)
    if composite:
        exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key64=key64, key64_by_rowid=True, key32=key32)
        res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key64=dev(key64),
                                key64_by_rowid=True, key32=dev(key32), max_groups=max_groups)
    else:
        exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key32=key32)
        res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key32=dev(key32),
                                max_groups=max_groups)
    assert ctx.status() == gq.GQ_OK
    _check_groups(res, exp, composite, True)


def test_groupby_capacity_error(ctx):
    n = 5000
    key32 = np.arange(n, dtype=np.int32)
    v = np.ones(n, np.int64)
    gq.gq_groupby_agg(ctx, dev(v), dev(v), dev(v), key32=dev(key32), max_groups=100)
    assert ctx.status() == gq.GQ_ERR_CAPACITY


def _fmix64_np(x):
    x = x.astype(np.uint64)
    x ^= x >> np.uint64(33)
    x *= np.uint64(0xFF51AFD7ED558CCD)
    x ^= x >> np.uint64(33)
    x *= np.uint64(0xC4CEB9FE1A85EC53)
    x ^= x >> np.uint64(33)
    return x


def test_groupby_large_path_overflowing_buckets(ctx):
    """Thousands of keys that all hash into one bucket overflow that bucket's
    LDS table: the extra keys go to the global fallback table and the result
    stays exact."""
    r = rng(31)
    cand = r.integers(0, 1 << 31, size=4_000_000).astype(np.int64)
    with np.errstate(over="ignore"):
        h = _fmix64_np(cand.astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15))
    hot = np.unique(cand[(h >> np.uint64(57)) == 0])[:9000]          # top 7 bits 0: bucket 0 while P <= 128
    assert len(hot) == 9000
    n = 400_000
    other = r.integers(0, 1 << 31, size=50_000)
    keys = np.concatenate([hot, other]).astype(np.int32)
    key32 = keys[r.integers(0, len(keys), size=n)]
    nv = n
    rowid = r.integers(0, nv, size=n).astype(np.int32)
    qty = r.integers(1, 51, size=nv).astype(np.int64)
    price = r.integers(100, 10_000_001, size=nv).astype(np.int64)
    disc = r.integers(0, 11, size=nv).astype(np.int64)
    exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key32=key32)
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key32=dev(key32),
                            max_groups=250_000)
    assert ctx.status() == gq.GQ_OK
    _check_groups(res, exp, False, True)


def _hot_keys(r, count):
    """int32 keys whose group hash has its top 8 bits zero: with P <= 256
    buckets they all land in bucket 0 and overflow its LDS table."""
    cand = r.integers(0, 1 << 31, size=4_000_000).astype(np.int64)
    with np.errstate(over="ignore"):
        h = _fmix64_np(cand.astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15))
    hot = np.unique(cand[(h >> np.uint64(56)) == 0])[:count]
    assert len(hot) == count
    return hot


@pytest.mark.parametrize("composite", [False, True])
@pytest.mark.parametrize("overflow", [False, True])
def test_groupby_large_path_wide_rows(ctx, composite, overflow):
    """Rows whose qty needs more than 32 bits or whose revenue needs more than
    64 bits mix with ordinary rows in the same groups; some groups hold only
    such rows; with overflow, thousands of keys share one bucket and spill to
    the global table.  Every sum stays exact."""
    r = rng(61 + int(composite) + 2 * int(overflow))
    n = nv = 300_000
    keys = r.integers(0, 1 << 31, size=6000)
    if overflow:
        keys = np.concatenate([keys, _hot_keys(r, 9000)])
    keys = np.unique(keys).astype(np.int32)
    qty = r.integers(1, 51, size=nv).astype(np.int64)
    price = r.integers(100, 10_000_001, size=nv).astype(np.int64)
    disc = r.integers(0, 11, size=nv).astype(np.int64)
    wide = np.nonzero(r.random(nv) < 0.05)[0]
    half = len(wide) // 2
    qty[wide[:half]] = r.integers(1 << 33, 1 << 40, size=half) * np.where(r.random(half) < 0.3, -1, 1)
    price[wide[half:]] = ((1 << 62) - r.integers(0, 1000, size=len(wide) - half)) * \
        np.where(r.random(len(wide) - half) < 0.5, -1, 1)
    key32 = keys[r.integers(0, len(keys), size=n)]
    rowid = r.integers(0, nv, size=n).astype(np.int32)
    only_wide = np.isin(key32, keys[:50])                       # these groups see wide rows only
    rowid[only_wide] = wide[r.integers(0, len(wide), size=int(only_wide.sum()))]
    max_groups = 250_000 if overflow else 8000
    if composite:
        key64 = np.where(np.isin(key32, keys[:3000]), 0, key32.astype(np.int64) * 7 + 1).astype(np.int64)
        exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key64=key64, key32=key32)
        res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key64=dev(key64),
                                key32=dev(key32), max_groups=max_groups)
    else:
        exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key32=key32)
        res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key32=dev(key32),
                                max_groups=max_groups)
    assert ctx.status() == gq.GQ_OK
    assert any(abs(v) >= 1 << 63 for v in oracle.sum_rev_int(exp))
    _check_groups(res, exp, composite, True)


@pytest.mark.parametrize("composite,max_groups", [(False, 500_000), (True, 500_000), (False, 6_000_000),
                                                  (True, 6_000_000)])
def test_groupby_heavy_keys_split_buckets(ctx, composite, max_groups):
    """Zipf-like heavy keys: one key holds 40% of the rows, others 10% and 5%.
    Their buckets hold far more rows than the mean and are aggregated in
    chunks by several workgroups; the bucket's last chunk folds the others'
    partial groups into its LDS table; lanes of a wave on the same key combine
    before their LDS update.  Some heavy-key rows are too wide for a narrow
    record.  Exact against the oracle, with the one-level (500K groups) and
    the two-level (6M) scatter."""
    r = rng(71 + int(composite) + (2 if max_groups > 1_000_000 else 0))
    n = nv = 2_000_000
    keys = np.unique(r.integers(0, 1 << 31, size=200_000)).astype(np.int32)
    pick = r.random(n)
    key32 = keys[r.integers(0, len(keys), size=n)]
    key32[pick < 0.40] = keys[0]
    key32[(pick >= 0.40) & (pick < 0.50)] = keys[1]
    key32[(pick >= 0.50) & (pick < 0.55)] = keys[2]
    rowid = r.integers(0, nv, size=n).astype(np.int32)
    qty = r.integers(1, 51, size=nv).astype(np.int64)
    price = r.integers(100, 10_000_001, size=nv).astype(np.int64)
    disc = r.integers(0, 11, size=nv).astype(np.int64)
    heavy_rows = np.nonzero(pick < 0.40)[0][:300]
    qty[rowid[heavy_rows[:150]]] = 1 << 40                     # wide rows of the heaviest key
    price[rowid[heavy_rows[150:]]] = (1 << 62) - 5
    if composite:
        g32 = r.integers(0, 2, size=n).astype(np.int32)
        key64 = key32.astype(np.int64) * 1_000_003 - 11
        exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key64=key64, key32=g32)
        res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key64=dev(key64),
                                key32=dev(g32), max_groups=max_groups)
    else:
        exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key32=key32)
        res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key32=dev(key32),
                                max_groups=max_groups)
    assert ctx.status() == gq.GQ_OK
    assert exp["count"].max() >= 0.2 * n
    _check_groups(res, exp, composite, True)


@pytest.mark.parametrize("composite", [False, True])
def test_groupby_split_bucket_overflowing_lds(ctx, composite):
    """A bucket that is both split (a key with half of the rows) and too full
    for its LDS tables (9000 keys hashed into it): its chunks send rows to the
    global table, so every chunk's partial groups go there too and no key is
    written out twice.  Exact against the oracle."""
    r = rng(91 + int(composite))
    n = nv = 400_000
    hot = _hot_keys(r, 9000).astype(np.int32)
    other = np.unique(r.integers(0, 1 << 31, size=20_000)).astype(np.int32)
    keys = np.concatenate([hot, other])
    key32 = keys[r.integers(0, len(keys), size=n)]
    key32[r.random(n) < 0.5] = hot[0]                          # the heavy key, in the crowded bucket
    rowid = r.integers(0, nv, size=n).astype(np.int32)
    qty = r.integers(1, 51, size=nv).astype(np.int64)
    price = r.integers(100, 10_000_001, size=nv).astype(np.int64)
    disc = r.integers(0, 11, size=nv).astype(np.int64)
    if composite:
        key64 = np.where(np.isin(key32, hot), 0, key32.astype(np.int64) * 5 + 3).astype(np.int64)
        exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key64=key64, key32=key32)
        res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key64=dev(key64),
                                key32=dev(key32), max_groups=250_000)
    else:
        exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key32=key32)
        res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key32=dev(key32),
                                max_groups=250_000)
    assert ctx.status() == gq.GQ_OK
    assert exp["count"].max() >= 0.4 * n
    _check_groups(res, exp, composite, True)


@pytest.mark.parametrize("qlo", [-(1 << 31), 0])
@pytest.mark.parametrize("groups", [25, 5000, 150_000])
def test_groupby_signed_revenues_in_narrow_records(ctx, groups, qlo):
    """Revenues that fit 64 bits but not 32, of both signs, and quantities
    over all of int32 (or all non-negative int32, too wide to share a word
    with the count): every row stays a narrow record, the split low/high
    revenue sums carry nonzero (negative) high halves, and group totals pass
    2^64."""
    r = rng(88 + groups)
    n = nv = 300_000
    key32 = r.integers(0, groups, size=n).astype(np.int32)
    rowid = r.integers(0, nv, size=n).astype(np.int32)
    qty = r.integers(qlo, 1 << 31, size=nv).astype(np.int64)
    price = r.integers(1, 1 << 55, size=nv, dtype=np.int64) * np.where(r.random(nv) < 0.4, -1, 1)
    disc = r.integers(-20, 11, size=nv).astype(np.int64)
    exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key32=key32)
    if groups == 25:
        assert any(abs(v) >= 1 << 64 for v in oracle.sum_rev_int(exp))
    res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key32=dev(key32),
                            max_groups=groups)
    assert ctx.status() == gq.GQ_OK
    _check_groups(res, exp, False, True)


@pytest.mark.parametrize("composite", [False, True])
def test_groupby_wide_fanout(ctx, composite):
    """Millions of groups: more buckets than the tile-staged scatter takes
    (chunked histogram, direct scatter), with some rows too wide for a
    narrow record; exact against the oracle."""
    r = rng(77 + int(composite))
    n = nv = 6_000_000
    groups = 2_600_000
    keys = np.unique(r.integers(0, 1 << 31, size=groups)).astype(np.int32)
    key32 = keys[r.integers(0, len(keys), size=n)]
    rowid = r.integers(0, nv, size=n).astype(np.int32)
    qty = r.integers(1, 51, size=nv).astype(np.int64)
    price = r.integers(100, 10_000_001, size=nv).astype(np.int64)
    disc = r.integers(0, 11, size=nv).astype(np.int64)
    wide = np.nonzero(r.random(nv) < 0.001)[0]
    qty[wide] = 1 << 40
    if composite:
        key64 = (key32.astype(np.int64) * 1_000_003) ^ (1 << 50)
        exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key64=key64, key32=key32)
        res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key64=dev(key64),
                                key32=dev(key32), max_groups=3_000_000)
    else:
        exp = oracle.groupby(n, qty, price, disc, rowid=rowid, key32=key32)
        res = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), rowid=dev(rowid), key32=dev(key32),
                                max_groups=3_000_000)
    assert ctx.status() == gq.GQ_OK
    _check_groups(res, exp, composite, True)


def test_groupby_repeatable(ctx):
    """Integer results are identical run to run (no scheduling dependence)."""
    n = 500_000
    rowid, key32, _, qty, price, disc = _gb_inputs(n, n, 41, 3000)
    args = dict(rowid=dev(rowid), key32=dev(key32), max_groups=3000)
    first = None
    for _ in range(5):
        h = gq.gq_groupby_agg(ctx, dev(qty), dev(price), dev(disc), **args).host()
        o = np.argsort(h["key32"])
        cur = [h[f][o] for f in ("key32", "count", "sum_qty", "sum_rev_lo", "sum_rev_hi", "avg_qty", "avg_rev")]
        if first is None:
            first = cur
        else:
            assert all(np.array_equal(a, b) for a, b in zip(first, cur))


# ------------------------------------------------------------------- top-k ---

@pytest.mark.parametrize("n,k", [(0, 5), (3, 100), (100, 100), (50_000, 1), (1_000_003, 100), (300_000, 2048),
                                 (3_000_000, 2048), (2_500_001, 7)])
@pytest.mark.parametrize("desc", [True, False])
def test_topk(ctx, n, k, desc):
    r = rng(n + k)
    val = r.integers(-40, 40, size=max(n, 1)).astype(np.int64)     # heavy ties
    sel = np.sort(r.choice(max(n, 1), size=(n + 1) // 2, replace=False)).astype(np.int32) if n else None
    ev, er = oracle.topk(val[:n] if n else val[:0], k, sel=sel, descending=desc)
    v, row, cnt = gq.gq_topk(ctx, dev(val), k, sel=None if sel is None else dev(sel), n=0 if not n else None,
                             descending=desc)
    c = int(cnt.item())
    assert c == len(ev)
    assert np.array_equal(host(v, c), ev) and np.array_equal(host(row, c), er)


def test_topk_ascending_values_adversarial(ctx):
    """Increasing values in row order raise the threshold at every step."""
    n = 700_000
    val = np.arange(n, dtype=np.int64) * 3 - 5
    ev, er = oracle.topk(val, 100)
    v, row, cnt = gq.gq_topk(ctx, dev(val), 100)
    assert np.array_equal(host(v), ev) and np.array_equal(host(row), er)


def test_topk_extremes_and_device_count(ctx):
    val = np.array([-(1 << 63), (1 << 63) - 1, 0, (1 << 63) - 1, -1] * 1000, dtype=np.int64)
    n_dev = torch.tensor([4003], dtype=torch.int64, device="cuda")
    ev, er = oracle.topk(val[:4003], 7)
    v, row, cnt = gq.gq_topk(ctx, dev(val), 7, n_dev=n_dev)
    assert np.array_equal(host(v), ev) and np.array_equal(host(row), er)
    with pytest.raises(gq.GQError):
        gq.gq_topk(ctx, dev(val), 4000)
