"""CPU checks of the benchmark's contract: it refuses more than one GPU with a
message, and its algorithmic byte counts are the per-row figures the
measurements use."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_operator():
    n, m, s_n, g, k = 200_000_000, 25_000_000, 117_323_354, 1_500_000, 100
    by = bench.algorithmic_bytes(n, m, s_n, g, k)
    assert by["partition"] == 76 * n                       # 5 columns in (36 B), 5 columns + row id out (40 B)
    assert by["filter"] == 4 * n + 4 * s_n
    assert by["join_build"] == 28 * m                      # key + payload in, one 16-B slot
    assert by["join_probe"] == 36 * s_n                    # sel + fk in, one 16-B slot, pair out
    assert by["groupby"] == 32 * s_n + 36 * g
    assert by["topk"] == 12 * s_n + 12 * k
    assert bench.algorithmic_bytes(n, m, s_n, g, k, partition=False)["partition"] == 0
    assert sum(by.values()) == 26_609_162_936             # the bytes of one step of the 200M-row share


def test_cpu_baseline_uses_several_cores():
    """The CPU baseline runs the oracle's pipeline on one shard per thread and
    reports the thread count, the CPU model and the one-core figure."""
    import synth
    w = synth.workload(0, scale=1 / 64)
    r = bench.cpu_baseline(w, 4096, 2)
    assert r["cores"] == 2 and r["kind"] == "oracle" and r["value"] > 0
    assert r["single_core"]["cores"] == 1 and r["single_core"]["value"] > 0
    assert r["cpu_model"]
