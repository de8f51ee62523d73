"""CPU tests of the exchange model (Sec. 3 of the paper).  The pins come from
outside the module: the worked skew example the paper prints, the boxed
closed forms of Eq. 1 and Eq. 2 written as throughputs, the equivalence of
Eq. 3 with comparing the two join times, the machine sums of Sec. 3.5 written
as the explicit triple sums over GPUs, and a Hockney fit on exact data."""
import itertools
import os

import numpy as np
import pytest

from paper_2506_09226_amd import model as M

GiB = float(1 << 30)
MiB = float(1 << 20)


def _golden(path):
    return [float(x) for x in open(path) if x.strip() and not x.startswith("#")]


def test_skew_gradient_matches_paper_example(golden_dir):
    f, V, k, first_mib, last_gib = _golden(os.path.join(golden_dir, "skew_gradient_example.txt"))
    N = int(V) * int(k)
    sizes = M.skew_gradient_sizes(N, f, N * GiB)
    assert round(sizes[0] / MiB) == first_mib
    assert round(sizes[-1] / GiB, 2) == last_gib
    assert sizes.sum() == pytest.approx(N * GiB, rel=1e-12)
    assert np.allclose(M.skew_gradient_sizes(N, 0.0, N * GiB), GiB)


@pytest.mark.parametrize("k,V", [(8, 1), (8, 2), (8, 5), (4, 3), (2, 1)])
def test_boxed_throughputs(k, V):
    """Eq. 1 and Eq. 2 as printed, against the time-based functions."""
    Bg, Bn, S = 400e9, 50e9, 3.7e12
    c = M.Cluster(k, V, Bg, Bn)
    N = k * V
    tb = M.throughput(S, M.broadcast_time(S, c))
    ts = M.throughput(S, M.shuffle_time(S, c))
    if V == 1:
        assert tb == pytest.approx(N / (N - 1) * Bg, rel=1e-12)
        assert ts == pytest.approx(N * N / (N - 1) * Bg, rel=1e-12)
    else:
        assert tb == pytest.approx(N / (N - 1) * min(Bn, Bg), rel=1e-12)
        assert ts == pytest.approx(V * V / (V - 1) * Bn, rel=1e-12)


def test_eq3_is_the_time_comparison():
    """Eq. 3 against T_b < T_s with the join times of Sec. 3.4 (network rate
    for both when V > 1; intra-machine rate for both when V = 1)."""
    Bn = 25e9
    rs = np.random.default_rng(3)
    for _ in range(2000):
        k = int(rs.integers(1, 9))
        V = int(rs.integers(1, 9))
        N = k * V
        if N == 1:
            continue
        R = float(rs.uniform(1, 100))
        S = float(rs.uniform(1, 100)) * float(rs.choice([1, 10, 100]))
        if V == 1:
            tb = (N - 1) * R / (N * Bn)
            tsh = (N - 1) * (R + S) / (N * N * Bn)
        else:
            tb = (N - 1) * R / (N * Bn)
            tsh = (V - 1) * (R + S) / (V * V * Bn)
        if abs(tb - tsh) < 1e-9 * tb:
            continue
        assert M.broadcast_join_wins(R, S, k, V) == (tb < tsh), (k, V, R, S)


def _triple_sums(Mx, k):
    """S_i and R_i of Sec. 3.5 as written: sums over j in [0,k), p != i in
    [0,V), q in [0,k) of m_{ij->pq} (send) and m_{pq->ij} (receive)."""
    N = Mx.shape[0]
    V = N // k
    send, recv = [], []
    for i in range(V):
        s = r = 0.0
        for j, p, q in itertools.product(range(k), range(V), range(k)):
            if p == i:
                continue
            s += Mx[i * k + j, p * k + q]
            r += Mx[p * k + q, i * k + j]
        send.append(s)
        recv.append(r)
    return np.array(send), np.array(recv)


@pytest.mark.parametrize("k,V", [(2, 2), (3, 4), (8, 2), (4, 1)])
def test_machine_sums_brute_force(k, V):
    rs = np.random.default_rng(k * 10 + V)
    Mx = rs.integers(0, 1000, size=(k * V, k * V)).astype(np.float64)
    s, r = M.machine_traffic(Mx, k)
    es, er = _triple_sums(Mx, k)
    assert np.array_equal(s, es) and np.array_equal(r, er)


@pytest.mark.parametrize("k,V", [(8, 1), (8, 2), (8, 4), (2, 3)])
def test_skewed_shuffle_reduces_to_eq2_without_skew(k, V):
    N, S = k * V, 1e12
    c = M.Cluster(k, V, 300e9, 40e9)
    even = M.equal_send_messages(np.full(N, S / N))
    assert M.shuffle_time_messages(even, c) == pytest.approx(M.shuffle_time(S, c), rel=1e-12)


def test_skewed_shuffle_paper_setting():
    """Sec. 5's skew case (f = 1, V = 4, k = 8, every GPU sends the same share
    to each receiver): the last machine sends the most, the first receives the
    most, and the shuffle takes the last machine's send bytes over B_n."""
    k, V, f = 8, 4, 1.0
    N = k * V
    sizes = M.skew_gradient_sizes(N, f, N * GiB)
    Mx = M.equal_send_messages(sizes)
    s, r = M.machine_traffic(Mx, k)
    assert int(np.argmax(s)) == V - 1 and int(np.argmax(r)) == 0
    node = sizes.reshape(V, k).sum(axis=1)
    assert s[-1] == pytest.approx(node[-1] * (N - k) / N, rel=1e-12)
    assert r[0] == pytest.approx(k * (sizes.sum() - node[0]) / N, rel=1e-12)
    c = M.Cluster(k, V, 300e9, 40e9)
    assert M.shuffle_time_messages(Mx, c) == pytest.approx(max(s.max(), r.max()) / 40e9, rel=1e-12)
    # skew only inside machines leaves the shuffle unchanged (Sec. 5)
    inner = np.tile(M.skew_gradient_sizes(k, f, k * GiB), V)
    assert M.shuffle_time_messages(M.equal_send_messages(inner), c) == \
        pytest.approx(M.shuffle_time(N * GiB, c), rel=1e-12)


def test_broadcast_ignores_placement_and_is_bound_by_slower_link():
    c = M.Cluster(8, 3, 100e9, 20e9)
    S = 5e11
    assert M.broadcast_time(S, c) == pytest.approx(23 * (S / 24) / 20e9, rel=1e-12)
    assert M.broadcast_time(S, M.Cluster(8, 3, 10e9, 20e9)) == pytest.approx(23 * (S / 24) / 10e9, rel=1e-12)


def test_hockney_fit_and_rate():
    L, cgap = 12e-6, 1 / 45e9
    ms = np.array([4e3, 6.4e4, 1e6, 1.6e7, 2.5e8])
    link = M.Link.fit(ms, L + cgap * ms)
    assert link.latency == pytest.approx(L, rel=1e-6) and link.gap == pytest.approx(cgap, rel=1e-9)
    assert link.rate(1e12) == pytest.approx(45e9, rel=1e-3)          # large messages: 1/c
    assert link.rate(1e3) < 0.1 * 45e9                               # small messages: latency bound
    # a Link in place of a constant rate: a shuffle's messages are S/N^2
    c = M.Cluster(8, 2, 400e9, link)
    S = 16 * 16 * 1e6
    assert M.shuffle_time(S, c) == pytest.approx(S * 1 / (4 * link.rate(1e6)), rel=1e-12)


def test_projection_plans():
    ops = {"partition": 3.7, "filter": 0.43, "join_build": 0.98, "join_probe": 2.9, "groupby": 4.0, "topk": 0.8}
    rows = M.project(ops, 200_000_000, 25_000_000, 1_500_000, gpus=(1, 8, 16))
    one = rows[0]
    assert one["shuffle_plan_ms"] == pytest.approx(sum(ops.values()), abs=1e-3)
    assert one["broadcast_plan_ms"] == pytest.approx(sum(ops.values()) - ops["partition"], abs=1e-3)
    # one machine of 8: |S|/|R| = 24 > N-1 = 7, so Eq. 3 broadcasts the dimension
    assert rows[1]["eq3"] == "broadcast"
    # two machines: (N-1)/(N-k) V - 1 = 15/8*2-1 = 2.75 < 24: still broadcast
    assert rows[2]["eq3"] == "broadcast"
    for r in rows[1:]:
        c = M.Cluster(8, r["machines"], M.MI355X_BG, M.MI355X_BN)
        N = r["gpus"]
        assert r["broadcast_exchange_ms"] == pytest.approx(1e3 * M.broadcast_time(N * 25e6 * 12, c), abs=1e-3)
        assert r["shuffle_plan_ms"] > one["shuffle_plan_ms"]
