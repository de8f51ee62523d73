"""CPU checks of the served path's error policy (csrc/gq_serve_policy.h):
what the server does with each query of a finished batch.  A small C++
driver that includes the header is compiled with g++ and run on a table of
cases; every case is forced from the host, no GPU is involved."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_09226_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")

DRIVER = r"""
#include <cstdio>
#include "gq_serve_policy.h"
int main() {
    int st, nq, agg, fits;
    long long mg, cap;
    while (std::scanf("%d %d %d %lld %lld %d", &st, &nq, &agg, &mg, &cap, &fits) == 6) {
        gq_retire_case c{st, nq, agg != 0, mg, cap, fits != 0};
        const gq_retire_action a = gq_retire_decide(c);
        std::printf("%d %lld\n", static_cast<int>(a), static_cast<long long>(gq_doubled_groups(mg, cap)));
    }
    return 0;
}
"""

COMPLETE, ALONE, DOUBLED = 0, 1, 2
OK, INVALID_ARG, CAPACITY, DUP, HIP, TIMEOUT = 0, 1, 2, 4, 5, 8


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("policy")
    src, exe = d / "drv.cpp", d / "drv"
    src.write_text(DRIVER)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", CSRC, "-I", INCLUDE, str(src), "-o", str(exe)])
    return str(exe)


def _decide(driver, cases):
    inp = "\n".join(" ".join(str(int(x)) for x in c) for c in cases) + "\n"
    out = subprocess.run([driver], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    return [tuple(int(v) for v in line.split()) for line in out if line.strip()]


def test_policy_table(driver):
    # (status, queries in batch, aggregate, max_groups, capacity, doubled fits) -> (action, doubled bound)
    cases = [
        ((OK, 5, 1, 100, 1000, 1), (COMPLETE, 200)),
        ((CAPACITY, 3, 1, 100, 1000, 1), (ALONE, 200)),        # a shared batch's error: each query alone
        ((DUP, 2, 1, 100, 1000, 1), (ALONE, 200)),
        ((TIMEOUT, 4, 0, 0, 0, 0), (ALONE, 0)),
        ((HIP, 4, 1, 100, 1000, 1), (COMPLETE, 200)),          # a launch failure is reported, not re-run
        ((CAPACITY, 1, 1, 100, 1000, 1), (DOUBLED, 200)),      # alone and overflowing: twice the bound
        ((CAPACITY, 1, 1, 600, 1000, 1), (DOUBLED, 1000)),     #   clamped to the output capacity
        ((CAPACITY, 1, 1, 1000, 1000, 1), (COMPLETE, 1000)),   #   outputs full: the caller's turn
        ((CAPACITY, 1, 1, 100, 1000, 0), (COMPLETE, 200)),     #   the doubled query no longer fits the pool
        ((CAPACITY, 1, 0, 0, 0, 1), (COMPLETE, 0)),            # top-k has no group bound
        ((INVALID_ARG, 1, 1, 100, 1000, 1), (COMPLETE, 200)),
    ]
    got = _decide(driver, [c for c, _ in cases])
    assert got == [e for _, e in cases]


def test_retry_sequence_reaches_capacity(driver):
    """Repeated overflows double the bound until the output capacity, then
    stop: at most log2(capacity / bound) + 1 runs."""
    mg, cap, runs = 3, 1000, 0
    while True:
        runs += 1
        (act, nxt), = _decide(driver, [(CAPACITY, 1, 1, mg, cap, 1)])
        if act != DOUBLED:
            break
        assert nxt > mg
        mg = nxt
    assert mg == cap and runs == 10
