"""The served form: every query's result is the same alone, in a concurrent
mix (continuous batching, shared scans, several streams), and in the serial
plain form; and equals the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2506_09226_amd as gq
from paper_2506_09226_amd.serve import QuerySpec, Server, result_host

pytestmark = pytest.mark.gpu
AVG_RTOL = 1e-12


@pytest.fixture(scope="module")
def served():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = gq.Context(0)
    spec = synth.ServeSpec(n=1_500_000, m=60_000, code_range=3000, attr_range=25, seed=synth.SEED_BASE + 40)
    fact, dim1, dim2 = synth.serve_tables(spec, device="cuda")
    t1 = gq.gq_join_build(ctx, dim1["key"], dim1["attr"])
    t2 = gq.gq_join_build(ctx, dim2["key"], dim2["attr"])
    torch.cuda.synchronize()
    assert ctx.status() == gq.GQ_OK
    pool = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    host = {"fact": {k: v.cpu().numpy() for k, v in fact.items()},
            "dim1": {k: v.cpu().numpy() for k, v in dim1.items()},
            "dim2": {k: v.cpu().numpy() for k, v in dim2.items()}}
    yield spec, fact, t1, t2, pool, host
    ctx.close()


def _queries(count, seed, spec):
    out = []
    for kind, hi in synth.serve_queries(count, seed):
        mg = {1: 16, 2: spec.code_range, 3: 32, 4: 0}[kind]
        out.append(QuerySpec(kind, hi, max_groups=mg, k=100))
    return out


def _oracle(q: QuerySpec, h):
    f = h["fact"]
    sel = oracle.filter(f["date"], -(1 << 31), q.date_hi)
    if q.kind == gq.GQ_QUERY_FILTER_TOPK:
        v, r = oracle.topk(f["price"], q.k, sel=sel)
        return {"val": v, "row": r}
    if q.kind == gq.GQ_QUERY_FILTER_AGG:
        return oracle.groupby(len(sel), f["qty"], f["price"], f["disc"], rowid=sel, key64=f["disc"],
                              key64_by_rowid=True)
    prow, pay = oracle.join(h["dim1"]["key"], h["dim1"]["attr"], f["fk"], sel)
    if q.kind == gq.GQ_QUERY_JOIN2_AGG:
        prow, pay = oracle.join(h["dim2"]["key"], h["dim2"]["attr"], f["fk2"], prow)
    return oracle.groupby(len(prow), f["qty"], f["price"], f["disc"], rowid=prow, key32=pay)


def _norm(q: QuerySpec, r: dict):
    if q.kind == gq.GQ_QUERY_FILTER_TOPK:
        return r
    key = "key64" if q.kind == gq.GQ_QUERY_FILTER_AGG else "key32"
    o = np.argsort(r[key], kind="stable")
    return {k: (None if v is None else v[o]) for k, v in r.items()}


def _same(q, a, b, avg_exact=False):
    if q.kind == gq.GQ_QUERY_FILTER_TOPK:
        assert np.array_equal(a["val"], b["val"]) and np.array_equal(a["row"], b["row"])
        return
    key = "key64" if q.kind == gq.GQ_QUERY_FILTER_AGG else "key32"
    for f in (key, "count", "sum_qty", "sum_rev_lo", "sum_rev_hi"):
        assert np.array_equal(a[f], b[f]), f
    for f in ("avg_qty", "avg_rev"):
        if avg_exact:
            assert np.array_equal(a[f], b[f]), f
        else:
            np.testing.assert_allclose(a[f], b[f], rtol=AVG_RTOL, atol=0)


def _run(server, qs, burst=True):
    if burst:
        subs = [server.submit(q) for q in qs]
        for s in subs:
            server.wait(s)
    else:
        subs = [server.wait(server.submit(q)) for q in qs]
    assert all(s.status == gq.GQ_OK for s in subs)
    assert all(s.latency > 0 for s in subs)
    return [_norm(s.spec, result_host(s)) for s in subs]


def test_served_alone_in_mix_serial_and_oracle(served):
    spec, fact, t1, t2, pool, h = served
    qs = _queries(40, 11, spec)
    srv = Server(0, fact, t1, t2, pool, streams=4, max_batch=16)
    mix = _run(srv, qs, burst=True)
    st = srv.stats()
    alone = _run(srv, qs, burst=False)
    srv.close()
    assert st["done"] == 40 and st["max_batch"] > 1 and st["batches"] < 40     # batching happened
    ser = Server(0, fact, t1, t2, pool, serial=True)
    serial = _run(ser, qs, burst=True)
    ser.close()
    for i, q in enumerate(qs):
        _same(q, mix[i], alone[i], avg_exact=True)                  # bit-identical alone and in the mix
        _same(q, mix[i], serial[i])
        if i < 16:
            _same(q, mix[i], _norm(q, _oracle(q, h)))


def test_served_admission_with_small_pool(served):
    """A pool that holds one join+aggregate batch at a time: queries queue for
    memory and still all complete with the right results."""
    spec, fact, t1, t2, pool, h = served
    qs = [QuerySpec(gq.GQ_QUERY_JOIN_AGG, hi, max_groups=spec.code_range) for hi in (300, 900, 1500, 2100, 2500)]
    need = 70 * fact["fk"].numel() + (16 << 20)                    # one batch (~44 B/row) fits, two do not
    small = pool[: min(pool.numel(), need)]
    srv = Server(0, fact, t1, t2, small, streams=4, max_batch=1)
    res = _run(srv, qs, burst=True)
    srv.close()
    for q, r in zip(qs[:2], res[:2]):
        _same(q, r, _norm(q, _oracle(q, h)))


def test_served_rejects_bad_queries(served):
    spec, fact, t1, t2, pool, h = served
    srv = Server(0, fact, t1, t2, pool)
    with pytest.raises(gq.GQError):
        srv.submit(QuerySpec(gq.GQ_QUERY_FILTER_TOPK, 100, k=1000))
    with pytest.raises(gq.GQError):
        srv.submit(QuerySpec(gq.GQ_QUERY_FILTER_AGG, 100, max_groups=5000))
    srv.close()
