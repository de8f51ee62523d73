"""The C ABI: libgq.so loads, exports every entry point include/gq.h declares,
and the host-side queries and argument checks behave.  No GPU needed (no
compute call is made)."""
import ctypes as C
import os
import re

import pytest

import paper_2506_09226_amd as gq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "gq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gq_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = gq.lib()
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(gq.EXPORTED) == names


def test_join_table_bytes():
    L = gq.lib()
    assert gq.gq_join_table_bytes(0, 0.5) == 256 + 64 * 16
    assert gq.gq_join_table_bytes(65_536, 0.5) == 256 + (1 << 17) * 16
    assert gq.gq_join_table_bytes(25_000_000, 0.5) == 256 + (1 << 26) * 16
    assert L.gq_join_table_bytes(10, 0.0) == 0 and L.gq_join_table_bytes(10, 0.95) == 0
    assert L.gq_join_table_bytes(-1, 0.5) == 0


def test_workspace_queries_monotone():
    L = gq.lib()
    for f, args in [(L.gq_filter_workspace_bytes, ()), (L.gq_join_probe_workspace_bytes, ())]:
        a, b = f(1000, *args), f(10_000_000, *args)
        assert 0 < a <= b and a % 256 == 0
    assert L.gq_radix_partition_workspace_bytes(1 << 20, 6) < L.gq_radix_partition_workspace_bytes(1 << 20, 8)
    assert L.gq_radix_partition_workspace_bytes(100, 9) == 0          # fan-out beyond 2^8
    small = L.gq_groupby_workspace_bytes(1 << 20, 25, 0, 1)
    large = L.gq_groupby_workspace_bytes(1 << 20, 1_500_000, 0, 1)
    assert 0 < small < large
    assert L.gq_topk_workspace_bytes(1 << 20, 100) > 0
    small = L.gq_join_build_workspace_bytes(1000, gq.gq_join_table_bytes(1000, 0.5))
    big = L.gq_join_build_workspace_bytes(25_000_000, gq.gq_join_table_bytes(25_000_000, 0.5))
    assert small == 256 and big > 25_000_000 * 24


def test_null_context_rejected():
    L = gq.lib()
    assert L.gq_filter(None, None, 4, 10, None, None, 0, 1, None, None, None, 0, None) == gq.GQ_ERR_INVALID_ARG
    assert L.gq_join_build(None, None, None, 0, None, None, None, 0, None, 0, None) == gq.GQ_ERR_INVALID_ARG
    assert L.gq_topk(None, None, None, 0, None, 1, 1, None, None, None, None, 0, None) == gq.GQ_ERR_INVALID_ARG
    assert L.gq_status_word(None, None, None) == gq.GQ_ERR_INVALID_ARG
    assert L.gq_last_error(None) == b""
    h = C.c_void_p()
    assert L.gq_ctx_create(-1, C.byref(h)) == gq.GQ_ERR_INVALID_ARG


def test_cpu_tensors_refused():
    import torch
    with pytest.raises(TypeError):
        gq._ptr(torch.zeros(4))
