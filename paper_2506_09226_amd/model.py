"""Analytical model of the data exchange steps (Sec. 3 of the paper), driven by
one GPU's measured operator times to project a multi-GPU step.

Notation (Sec. 3.1, Table 2): k GPUs per machine, V machines, N = k*V GPUs,
B_g the unidirectional rate at which one GPU reaches all its local peers
together, B_n the unidirectional network rate of one machine, S the bytes the
whole cluster exchanges, evenly spread unless a message matrix says otherwise.

  * broadcast (Sec. 3.2): a ring of N-1 steps moving S/N per hop, bound by
    the slower of the two link kinds; time (N-1)(S/N)/min(B_n, B_g), i.e.
    throughput N/(N-1) min(B_n, B_g) (Eq. 1); with one machine only B_g.
  * shuffle (Sec. 3.3): every GPU sends 1/N of its S/N to every GPU; remote
    sends are the slower ones, time S(V-1)/(V^2 B_n), throughput
    V^2/(V-1) B_n (Eq. 2); with one machine N^2/(N-1) B_g.
  * broadcast join vs shuffle join (Sec. 3.4): broadcasting R beats shuffling
    R and S when |S|/|R| > (N-1)/(N-k) V - 1 (Eq. 3); with one machine when
    |S|/|R| > N-1.
  * skew (Sec. 3.5): a broadcast ring is unaffected; a shuffle takes as long
    as the machine that sends or receives the most bytes over the network.
  * message sizes (Sec. 3.6): a link moves an m-byte message in L + c m
    (Hockney), so its rate is m / (L + c m); L and c are fitted to measured
    (m, t) pairs.

The one-machine skewed shuffle is not written out in the paper; here it is
the same rule one level down (the GPU that sends or receives the most bytes to
or from its local peers, at B_g), which reduces to the one-machine case of
Eq. 2 when every message is equal.

This module is arithmetic on floats and arrays; it runs on the CPU only.
"""
from __future__ import annotations

import argparse
import json
import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Link:
    """Hockney link: an m-byte message takes latency + gap * m seconds."""
    latency: float          # L, seconds
    gap: float              # c, seconds per byte

    def rate(self, m: float) -> float:
        """Bytes per second for messages of m bytes (Sec. 3.6)."""
        return m / (self.latency + self.gap * m)

    @staticmethod
    def fit(sizes, times) -> "Link":
        """Least-squares line t = L + c m through measured (m, t) pairs."""
        m = np.asarray(sizes, dtype=np.float64)
        t = np.asarray(times, dtype=np.float64)
        A = np.stack([np.ones_like(m), m], axis=1)
        (L, c), *_ = np.linalg.lstsq(A, t, rcond=None)
        return Link(float(L), float(c))


def _rate(b, m: float) -> float:
    """A link given as a constant rate (bytes/s) or as a Hockney Link."""
    return b.rate(m) if isinstance(b, Link) else float(b)


@dataclass(frozen=True)
class Cluster:
    k: int                  # GPUs per machine
    V: int                  # machines
    Bg: object              # bytes/s, or a Link (intra-machine, per GPU, all peers)
    Bn: object              # bytes/s, or a Link (network, per machine)

    @property
    def N(self) -> int:
        return self.k * self.V


def broadcast_time(S: float, c: Cluster) -> float:
    """Ring broadcast of S bytes spread over N GPUs (Sec. 3.2)."""
    N = c.N
    if N == 1:
        return 0.0
    m = S / N                                   # the message of each ring step
    bw = _rate(c.Bg, m) if c.V == 1 else min(_rate(c.Bn, m), _rate(c.Bg, m))
    return (N - 1) * m / bw


def shuffle_time(S: float, c: Cluster) -> float:
    """Even all-to-all of S bytes (Sec. 3.3): each GPU holds S/N and sends
    S/N^2 to every GPU."""
    N, V = c.N, c.V
    if N == 1:
        return 0.0
    m = S / (N * N)                             # point-to-point message size
    if V == 1:
        return S * (N - 1) / (N * N * _rate(c.Bg, m))
    return S * (V - 1) / (V * V * _rate(c.Bn, m))


def throughput(S: float, t: float) -> float:
    """Throughput of an exchange: the bytes S over its time (Sec. 3.1)."""
    return math.inf if t == 0 else S / t


def machine_traffic(M, k: int):
    """Bytes each machine sends to and receives from other machines, for a
    message matrix M[a, b] (GPU a to GPU b, GPU g on machine g // k): the sums
    S_i and R_i of Sec. 3.5."""
    M = np.asarray(M, dtype=np.float64)
    N = M.shape[0]
    node = np.arange(N) // k
    remote = node[:, None] != node[None, :]
    V = N // k
    send = np.array([M[(node == i)[:, None] & remote].sum() for i in range(V)])
    recv = np.array([M[remote & (node == i)[None, :]].sum() for i in range(V)])
    return send, recv


def shuffle_time_messages(M, c: Cluster) -> float:
    """Shuffle with an arbitrary message matrix (Sec. 3.5): the busiest
    machine's network bytes over B_n; on one machine, the busiest GPU's bytes
    to or from its peers over B_g."""
    M = np.asarray(M, dtype=np.float64)
    N = M.shape[0]
    if N != c.N:
        raise ValueError(f"message matrix is {N}x{N}, cluster has {c.N} GPUs")
    off = M[~np.eye(N, dtype=bool)]
    m = float(off.mean()) if off.size else 0.0
    if N == 1:
        return 0.0
    if c.V == 1:
        peer = M - np.diag(np.diag(M))
        busiest = max(peer.sum(axis=1).max(), peer.sum(axis=0).max())
        return busiest / _rate(c.Bg, m)
    send, recv = machine_traffic(M, c.k)
    return max(send.max(), recv.max()) / _rate(c.Bn, m)


def broadcast_join_wins(R: float, S: float, k: int, V: int) -> bool:
    """Eq. 3: broadcasting table R (|R| bytes) beats shuffling R and S."""
    N = k * V
    if N == 1:
        return False
    if V == 1:
        return S / R > N - 1
    return S / R > (N - 1) / (N - k) * V - 1


def skew_gradient_sizes(N: int, f: float, total: float) -> np.ndarray:
    """Initial placement of the skew experiment (Sec. 5): GPU i holds
    x + i f x bytes, with x chosen so the sizes sum to `total`."""
    i = np.arange(N, dtype=np.float64)
    x = total / (N + f * N * (N - 1) / 2)
    return x * (1 + f * i)


def equal_send_messages(sizes) -> np.ndarray:
    """Every GPU sends the same share of its data to each of the N GPUs."""
    sizes = np.asarray(sizes, dtype=np.float64)
    N = len(sizes)
    return np.repeat((sizes / N)[:, None], N, axis=1)


# ----------------------------------------------------------------------------
# Projection of the one-GPU-share step onto N GPUs (weak scaling: every GPU
# keeps its share; the exchanges grow with N)
# ----------------------------------------------------------------------------

# MI355X node, stated assumptions: 8 GPUs; 7 xGMI links of 153.6 GB/s per GPU,
# taken as bidirectional, so 76.8 GB/s each way and 537.6 GB/s to all peers;
# one 400 Gb/s NIC per GPU, so 400 GB/s per machine.
MI355X_K = 8
MI355X_BG = 7 * 76.8e9
MI355X_BN = 8 * 50e9


def project(ops_ms: dict, fact_rows: int, dim_rows: int, groups: int, gpus=(1, 8, 16, 32, 64),
            k: int = MI355X_K, Bg=MI355X_BG, Bn=MI355X_BN, fact_row_bytes: int = 36, dim_row_bytes: int = 12,
            group_bytes: int = 36) -> list:
    """Projected step time per GPU count, for both join plans.

    Shuffle plan: every GPU radix-partitions its fact share (the local half of
    the shuffle, measured), both tables are shuffled, and the local operators
    keep their measured one-GPU times (each GPU receives about its share).
    Broadcast plan: the dimension table is broadcast, no fact partition is
    needed, and each GPU builds its table over all N shares of the dimension
    (the build time scaled by N; the probe time kept, an optimistic bound).
    Both then shuffle the per-GPU partial groups by group key.  `eq3` is the
    plan Eq. 3 picks, which compares the exchange times alone."""
    rows = []
    part = ops_ms.get("partition", 0.0)
    build = ops_ms.get("join_build", 0.0)
    others = sum(v for key, v in ops_ms.items() if key not in ("partition", "join_build"))
    for N in gpus:
        V = max(1, N // k)
        kk = N if N < k else k
        c = Cluster(kk, V, Bg, Bn)
        R = N * dim_rows * dim_row_bytes
        S = N * fact_rows * fact_row_bytes
        t_groups = 1e3 * shuffle_time(N * min(groups, fact_rows) * group_bytes, c)
        t_shuf = 1e3 * (shuffle_time(R, c) + shuffle_time(S, c))
        t_bc = 1e3 * broadcast_time(R, c)
        shuffle_plan = part + build + others + t_shuf + t_groups
        bcast_plan = N * build + others + t_bc + t_groups
        eq3 = "broadcast" if broadcast_join_wins(R, S, kk, V) else "shuffle"
        best = min(shuffle_plan, bcast_plan)
        rows.append({"gpus": N, "machines": V, "eq3": eq3,
                     "shuffle_plan_ms": round(shuffle_plan, 3), "shuffle_exchange_ms": round(t_shuf, 3),
                     "broadcast_plan_ms": round(bcast_plan, 3), "broadcast_exchange_ms": round(t_bc, 3),
                     "group_exchange_ms": round(t_groups, 3),
                     "best": "broadcast" if bcast_plan < shuffle_plan else "shuffle",
                     "fact_rows_per_s": round(N * fact_rows / (best * 1e-3))})
    return rows


def main():
    ap = argparse.ArgumentParser(description="project a measured one-GPU step onto N MI355X GPUs")
    ap.add_argument("bench_json", help="a JSON line written by bench.py (plain form)")
    ap.add_argument("--gpus", default="1,8,16,32,64")
    a = ap.parse_args()
    d = json.loads(open(a.bench_json).read().strip().splitlines()[-1])
    ops = {k: v["ms"] for k, v in d["ops"].items()}
    cfg = d["config"]
    for r in project(ops, cfg["fact_rows"], cfg["dim_rows"], cfg["groups"],
                     tuple(int(x) for x in a.gpus.split(","))):
        print(json.dumps(r))


if __name__ == "__main__":
    main()
