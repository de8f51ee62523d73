"""The seeded input generator: published SplitMix64 values, device-independent
integer arithmetic and the distribution shapes.  CPU only."""
import math
import os

import numpy as np
import torch

import synth


def test_splitmix64_published_sequence(golden_dir):
    vals = [int(l) for l in open(os.path.join(golden_dir, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    assert synth.splitmix64_sequence(1234567, 5) == vals


def test_torch_mix_matches_python_ints():
    rng = np.random.default_rng(0)
    xs = rng.integers(-(1 << 63), (1 << 63) - 1, size=5000, dtype=np.int64)
    got = synth.mix64(torch.from_numpy(xs)).tolist()
    for x, g in zip(xs.tolist(), got):
        assert (g & synth.MASK64) == synth.mix64_int(x & synth.MASK64)


def test_uniform_ranges_and_means():
    rows = torch.arange(200_000)
    q = synth.uniform_int(7, synth.S_QTY, rows, 1, 50)
    assert int(q.min()) == 1 and int(q.max()) == 50
    assert abs(q.double().mean().item() - 25.5) < 0.1
    d = synth.uniform_int(7, synth.S_DATE, rows, 0, 2556)
    frac = (d < 1500).double().mean().item()
    assert abs(frac - 1500 / 2557) < 0.005


def test_dim_keys_unique_and_fk_reference_dim():
    m = 50_000
    d = synth.dim_table(m, 11, 25)
    assert torch.unique(d["key"]).numel() == m
    f = synth.fact_table(synth.FactSpec(20_000, m, 11))
    assert bool(torch.isin(f["fk"], d["key"]).all())


def test_rows_recomputable_alone():
    spec = synth.FactSpec(10_000, 1000, 5)
    full = synth.fact_table(spec)
    rows = torch.tensor([0, 17, 9999, 4242])
    part = synth.fact_columns(spec, rows)
    for k in full:
        assert torch.equal(full[k][rows], part[k])


def test_zipf_rank1_frequency():
    m, n = 10_000_000, 400_000
    rows = torch.arange(n)
    r = synth.zipf_row(3, synth.S_FK_ROW, rows, m)
    h = float(synth.zipf_cdf(m)[0])        # = 1 / H_m
    assert abs(1.0 / h - sum(1.0 / k for k in range(1, 1001)) - (math.log(m) - math.log(1000))) < 1e-3
    frac = (r == 0).double().mean().item()
    assert abs(frac - h) < 4 * math.sqrt(h * (1 - h) / n)
    assert int(r.min()) >= 0 and int(r.max()) < m
