"""Pins of the CPU oracle against facts that do not come from the oracle itself:
published hash values, closed forms, invariants, brute force on tiny inputs and
exact Python big-integer arithmetic.  CPU only."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

MASK = (1 << 64) - 1


def _golden_ints(path):
    vals = []
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            vals.append(int(line, 0))
    return vals


# ---------------------------------------------------------------- hash ----

def test_fmix64_published_murmur3_verification(golden_dir):
    (expected,) = _golden_ints(os.path.join(golden_dir, "murmur3_x64_128_verification.txt"))
    key = bytes(range(256))
    digests = b"".join(oracle.murmur3_x64_128(key[:i], 256 - i) for i in range(256))
    final = oracle.murmur3_x64_128(digests, 0)
    assert int.from_bytes(final[:4], "little") == expected


def test_fmix64_zero_and_bijection_on_sample():
    assert oracle.fmix64(0) == 0
    rng = np.random.default_rng(1)
    xs = [int(v) for v in rng.integers(0, 1 << 63, size=2000, dtype=np.int64)]
    hs = {oracle.fmix64(x) for x in xs}
    assert len(hs) == len(set(xs))


def _fmix64_inverse(h):
    """Inverse of the MurmurHash3 finalizer: undo xorshift-33 and the two odd
    multiplications (modular inverses), independent of the oracle's code."""
    c1, c2 = 0xFF51AFD7ED558CCD, 0xC4CEB9FE1A85EC53
    i1, i2 = pow(c1, -1, 1 << 64), pow(c2, -1, 1 << 64)

    def unxs33(x):
        return x ^ (x >> 33)          # x>>33 then >>66 == 0 for 64-bit words

    h = unxs33(h)
    h = (h * i2) & MASK
    h = unxs33(h)
    h = (h * i1) & MASK
    return unxs33(h)


def test_fmix64_inverse_roundtrip():
    rng = np.random.default_rng(2)
    for v in rng.integers(0, 1 << 63, size=200, dtype=np.int64):
        h = int(v) * 2 + 1
        assert oracle.fmix64(_fmix64_inverse(h)) == h


def _s64(u):
    return u - (1 << 64) if u >> 63 else u


def test_partition_constructed_buckets():
    """Keys built so that their hash has chosen top bits land in exactly those
    buckets: pins 'bucket = top log2P bits of fmix64(key)'."""
    log2p = 6
    rng = np.random.default_rng(3)
    want = rng.integers(0, 64, size=3000)
    low = rng.integers(0, 1 << 58, size=3000, dtype=np.int64)
    keys = np.array([_s64(_fmix64_inverse((int(b) << 58) | int(lo))) for b, lo in zip(want, low)],
                    dtype=np.int64)
    key_out, _, rowid, offs = oracle.partition(keys, log2p)
    counts = np.bincount(want, minlength=64)
    assert np.array_equal(np.diff(offs), counts)
    for b in range(64):
        rows = rowid[offs[b]:offs[b + 1]]
        assert np.array_equal(rows, np.nonzero(want == b)[0])   # stable: input order


# -------------------------------------------------------------- filter ----

def test_filter_closed_form_on_arange():
    col = np.arange(10_000, dtype=np.int32)
    for lo, hi in [(0, 10_000), (17, 4321), (5000, 5000), (-5, 3), (9_990, 20_000), (200, 100)]:
        exp = np.arange(max(lo, 0), max(min(hi, 10_000), max(lo, 0)), dtype=np.int32)
        assert np.array_equal(oracle.filter(col, lo, hi), exp)


def test_filter_brute_force_with_sel_in():
    rng = np.random.default_rng(4)
    for dt in (np.int32, np.int64):
        col = rng.integers(-50, 50, size=700).astype(dt)
        sel_in = np.sort(rng.choice(700, size=300, replace=False)).astype(np.int32)
        exp = [r for r in sel_in if -7 <= col[r] < 20]
        assert oracle.filter(col, -7, 20, sel_in=sel_in).tolist() == exp
        exp2 = [r for r in range(700) if -7 <= col[r] < 20]
        assert oracle.filter(col, -7, 20).tolist() == exp2


def test_filter_empty():
    assert len(oracle.filter(np.zeros(0, np.int32), 0, 10)) == 0


# ----------------------------------------------------------- partition ----

@pytest.mark.parametrize("log2p", [0, 1, 6, 9])
def test_partition_invariants(log2p):
    rng = np.random.default_rng(5 + log2p)
    n = 5000
    key = rng.integers(-(1 << 63), (1 << 63) - 1, size=n, dtype=np.int64)
    c32 = rng.integers(0, 1000, size=n).astype(np.int32)
    c64 = rng.integers(-(1 << 40), 1 << 40, size=n, dtype=np.int64)
    key_out, (o32, o64), rowid, offs = oracle.partition(key, log2p, [c32, c64])
    P = 1 << log2p
    assert offs[0] == 0 and offs[-1] == n and np.all(np.diff(offs) >= 0)
    assert np.array_equal(np.sort(rowid), np.arange(n))                # permutation
    assert np.array_equal(key_out, key[rowid])
    assert np.array_equal(o32, c32[rowid]) and np.array_equal(o64, c64[rowid])
    for b in range(P):
        seg = rowid[offs[b]:offs[b + 1]]
        assert np.all(np.diff(seg) > 0)                                 # stable
        for r in seg[:50]:
            h = oracle.fmix64(int(key[r]))
            assert (h >> (64 - log2p) if log2p else 0) == b


# ---------------------------------------------------------------- join ----

def test_join_cardinality_closed_form():
    """All foreign keys reference existing unique keys -> |join| == |sel|."""
    rng = np.random.default_rng(7)
    m = 4000
    bkey = rng.choice(np.arange(-10**12, 10**12, 7919, dtype=np.int64), size=m, replace=False)
    bpay = rng.integers(0, 25, size=m).astype(np.int32)
    fk = bkey[rng.integers(0, m, size=20_000)]
    sel = np.sort(rng.choice(20_000, size=9000, replace=False)).astype(np.int32)
    prow, pay = oracle.join(bkey, bpay, fk, sel)
    assert len(prow) == len(sel)
    assert np.array_equal(prow, sel)
    where = {int(k): i for i, k in enumerate(bkey)}
    assert all(pay[j] == bpay[where[int(fk[r])]] for j, r in enumerate(prow))


def test_join_matches_nested_loop_with_misses():
    rng = np.random.default_rng(8)
    for trial in range(5):
        m, n = int(rng.integers(0, 60)), int(rng.integers(0, 300))
        bkey = rng.choice(1000, size=m, replace=False).astype(np.int64)
        bpay = rng.integers(-5, 5, size=m).astype(np.int32)
        fk = rng.integers(0, 1000, size=n).astype(np.int64)
        sel = None if trial % 2 else np.sort(rng.choice(max(n, 1), size=n // 2, replace=False)).astype(np.int32)
        a = oracle.join(bkey, bpay, fk, sel)
        b = oracle.join_nested(bkey, bpay, fk, sel)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        exp = [(r, int(bpay[list(bkey).index(fk[r])])) for r in (sel if sel is not None else range(n))
               if fk[r] in set(bkey.tolist())]
        assert list(zip(a[0].tolist(), a[1].tolist())) == exp


def test_join_duplicate_key_detected():
    with pytest.raises(oracle.DuplicateKey):
        oracle.join(np.array([1, 2, 1], np.int64), np.zeros(3, np.int32), np.array([1], np.int64))
    with pytest.raises(oracle.DuplicateKey):
        oracle.join_nested(np.array([5, 5], np.int64), np.zeros(2, np.int32), np.array([1], np.int64))


# ------------------------------------------------------------- group-by ----

def _py_groupby(keys, qty, price, disc, scale=100):
    d = {}
    for k, q, p, s in zip(keys, qty, price, disc):
        c, sq, sr = d.get(k, (0, 0, 0))
        d[k] = (c + 1, sq + int(q), sr + int(p) * (scale - int(s)))
    return d


def test_groupby_matches_linear_scan_and_python_ints():
    rng = np.random.default_rng(9)
    n = 3000
    rowid = rng.permutation(n).astype(np.int32)
    k32 = rng.integers(0, 40, size=n).astype(np.int32)
    k64 = rng.integers(-3, 3, size=n).astype(np.int64)
    qty = rng.integers(1, 51, size=n).astype(np.int64)
    price = rng.integers(100, 10**7 + 1, size=n).astype(np.int64)
    disc = rng.integers(0, 11, size=n).astype(np.int64)
    g = oracle.groupby(n, qty, price, disc, rowid=rowid, key64=k64, key64_by_rowid=True, key32=k32)
    gl = oracle.groupby_linear(n, qty, price, disc, rowid=rowid, key64=k64, key64_by_rowid=True, key32=k32)
    order = np.lexsort((gl["key32"], gl["key64"]))
    for f in g:
        assert np.array_equal(g[f], gl[f][order]), f
    keys = [(int(k64[rowid[j]]), int(k32[j])) for j in range(n)]
    ref = _py_groupby(keys, qty[rowid], price[rowid], disc[rowid])
    assert len(ref) == len(g["count"])
    revs = oracle.sum_rev_int(g)
    for i, (a, b) in enumerate(zip(g["key64"].tolist(), g["key32"].tolist())):
        c, sq, sr = ref[(a, b)]
        assert g["count"][i] == c and g["sum_qty"][i] == sq and revs[i] == sr
        assert g["avg_qty"][i] == float(sq) / float(c)
        assert g["avg_rev"][i] == float(sr) / float(c)
    assert g["count"].sum() == n
    assert sum(revs) == sum(int(p) * (100 - int(s)) for p, s in zip(price, disc))


def test_groupby_int128_carry_exact():
    """Values near 2**62: per-group sums cross 2**64 and 2**127 boundaries are
    handled exactly (checked against Python big integers)."""
    rng = np.random.default_rng(10)
    n = 600
    price = rng.integers((1 << 62) - 1000, (1 << 62), size=n, dtype=np.int64)
    price[::7] *= -1                                   # some negative products
    disc = rng.integers(-60, 11, size=n).astype(np.int64)
    qty = rng.integers(1 << 60, (1 << 62), size=n, dtype=np.int64)   # int64 sum wraps
    key = rng.integers(0, 5, size=n).astype(np.int32)
    g = oracle.groupby(n, qty, price, disc, key32=key)
    revs = oracle.sum_rev_int(g)
    for i, k in enumerate(g["key32"].tolist()):
        idx = np.nonzero(key == k)[0]
        sr = sum(int(price[j]) * (100 - int(disc[j])) for j in idx)
        sq = sum(int(qty[j]) for j in idx)
        assert revs[i] == sr
        assert abs(sr) >= 1 << 64                      # the carry really happened
        assert int(g["sum_qty"][i]) == _s64(sq & MASK)  # wrapping int64
        assert g["avg_rev"][i] == float(sr) / len(idx)
        assert float(Fraction(sr, len(idx))) == pytest.approx(g["avg_rev"][i], rel=1e-15)


def test_groupby_no_key_is_one_group_and_empty_input():
    qty = np.array([1, 2, 3], np.int64)
    price = np.array([100, 200, 300], np.int64)
    disc = np.array([0, 10, 5], np.int64)
    g = oracle.groupby(3, qty, price, disc)
    assert g["count"].tolist() == [3] and g["sum_qty"].tolist() == [6]
    assert oracle.sum_rev_int(g) == [100 * 100 + 200 * 90 + 300 * 95]
    e = oracle.groupby(0, qty, price, disc, key32=np.zeros(3, np.int32))
    assert len(e["count"]) == 0


def test_groupby_capacity_overflow():
    with pytest.raises(OverflowError):
        oracle.groupby(4, np.ones(4, np.int64), np.ones(4, np.int64), np.zeros(4, np.int64),
                       key32=np.arange(4, dtype=np.int32), cap=3)


# ---------------------------------------------------------------- top-k ----

@pytest.mark.parametrize("descending", [True, False])
def test_topk_matches_python_sort_and_selection(descending):
    rng = np.random.default_rng(11)
    for n, k in [(0, 5), (3, 5), (500, 100), (2000, 37)]:
        val = rng.integers(-20, 20, size=n).astype(np.int64)       # many ties
        sel = np.sort(rng.choice(max(n, 1), size=n // 2 + (n > 0), replace=False)).astype(np.int32) if n else None
        rows = sel.tolist() if sel is not None else list(range(n))
        exp = sorted(rows, key=lambda r: ((-val[r] if descending else val[r]), r))[:k]
        v, r = oracle.topk(val, k, sel=sel, descending=descending)
        assert r.tolist() == exp and v.tolist() == [int(val[x]) for x in exp]
        v2, r2 = oracle.topk_select(val, k, sel=sel, descending=descending)
        assert r2.tolist() == exp and np.array_equal(v2, v)


def test_topk_extreme_values():
    val = np.array([-(1 << 63), (1 << 63) - 1, 0, (1 << 63) - 1, -1], np.int64)
    v, r = oracle.topk(val, 3)
    assert r.tolist() == [1, 3, 2]
    v, r = oracle.topk(val, 2, descending=False)
    assert r.tolist() == [0, 4]
