"""The filter's no-allocation entry point (gq_filter_noalloc, static device
scratch) against the workspace entry point (gq_filter) and the oracle,
through the C ABI: two calls in a row, the second on a smaller input, so the
scratch left by the first call must be cleared by the second."""
import numpy as np
import pytest
import torch

import oracle
import paper_2506_09226_amd as gq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = gq.Context(0)
    yield c
    c.close()


def _both(ctx, col, lo, hi, sel_in=None, n=None, n_dev=None):
    m = n if n is not None else (sel_in.numel() if sel_in is not None else col.numel())
    out_a = torch.full((max(m, 1),), -1, dtype=torch.int32, device="cuda")
    out_b = torch.full((max(m, 1),), -2, dtype=torch.int32, device="cuda")
    na = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    nb = torch.full((1,), -2, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    gq.gq_filter(ctx, col, lo, hi, sel_in=sel_in, n=n, n_dev=n_dev, out=out_a, n_out=na)
    gq.gq_filter_noalloc(ctx, col, lo, hi, out_b, nb, sel_in=sel_in, n=n, n_dev=n_dev)
    assert ctx.status() == gq.GQ_OK
    ka, kb = int(na.item()), int(nb.item())
    assert ka == kb
    assert np.array_equal(out_a[:ka].cpu().numpy(), out_b[:kb].cpu().numpy())
    return out_b[:kb].cpu().numpy()


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_noalloc_equals_workspace_form_two_calls(ctx, dtype):
    r = np.random.default_rng(17)
    big = r.integers(0, 2557, size=3_000_001).astype(dtype)
    small = r.integers(0, 2557, size=40_961).astype(dtype)
    got = _both(ctx, torch.from_numpy(big).cuda(), 0, 1500)
    assert np.array_equal(got, oracle.filter(big, 0, 1500))
    got = _both(ctx, torch.from_numpy(small).cuda(), 100, 900)          # smaller: stale scratch must not leak
    assert np.array_equal(got, oracle.filter(small, 100, 900))


def test_noalloc_with_selection_device_count_and_empty(ctx):
    r = np.random.default_rng(18)
    col = r.integers(0, 2557, size=500_000).astype(np.int32)
    sel = np.sort(r.choice(500_000, size=200_000, replace=False)).astype(np.int32)
    used = 123_457
    n_dev = torch.tensor([used], dtype=torch.int64, device="cuda")
    got = _both(ctx, torch.from_numpy(col).cuda(), 0, 1000, sel_in=torch.from_numpy(sel).cuda(), n=len(sel),
                n_dev=n_dev)
    assert np.array_equal(got, oracle.filter(col, 0, 1000, sel_in=sel[:used]))
    got = _both(ctx, torch.from_numpy(col[:0].copy()).cuda(), 0, 1000)
    assert len(got) == 0


def test_noalloc_rejects_bad_arguments(ctx):
    col = torch.zeros(10, dtype=torch.int32, device="cuda")
    out = torch.empty(10, dtype=torch.int32, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(gq.GQError) as e:
        gq.gq_filter_noalloc(ctx, col, 0, 1, out, n_out, n=1 << 31)
    assert e.value.code == gq.GQ_ERR_INVALID_ARG
