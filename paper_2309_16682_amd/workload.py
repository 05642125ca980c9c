"""Seeded synthetic workloads shared by the tests, the benchmark and the serving
loop. Nothing here touches the generators' arithmetic: it only draws seeds,
request sizes and arrival times.

  batch keys     splitmix64(seed) (Steele, Lea, Flood 2014): generator g takes
                 outputs 2g and 2g+1 as the 4-word key [lo0, hi0, lo1, hi1].
  batch lengths  splitmix64(seed + 1), l = floor(exp(U ln(hi/lo) + ln lo)),
                 U = (u >> 11) 2^-53: log-uniform in [lo, hi).
  serving trace  Poisson arrivals (exponential gaps), log-uniform byte sizes
                 rounded to the element size, uniform state ids, a fraction of
                 jump requests by 2^k with k uniform in [kmin, kmax].
  rounds         a batch whose outputs exceed the device memory is written in
                 rounds over an output arena (plan_rounds).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int) -> np.ndarray:
    """First `count` outputs of splitmix64 started at `seed`."""
    with np.errstate(over="ignore"):
        s = np.uint64(seed) + _GOLDEN * np.arange(1, count + 1, dtype=np.uint64)
        z = (s ^ (s >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def batch_keys(count: int, seed: int = 42) -> np.ndarray:
    """(count, 4) uint32 init_by_array keys."""
    u = splitmix64(seed, 2 * count).reshape(count, 2)
    lo = (u & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    hi = (u >> np.uint64(32)).astype(np.uint32)
    return np.stack([lo[:, 0], hi[:, 0], lo[:, 1], hi[:, 1]], axis=1)


def uniform01(seed: int, count: int) -> np.ndarray:
    return (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * 2.0**-53


def batch_lengths(count: int, seed: int = 43, lo: float = 1e3, hi: float = 1e7) -> np.ndarray:
    """Log-uniform element counts in [lo, hi)."""
    u = uniform01(seed, count)
    return np.floor(np.exp(u * np.log(hi / lo) + np.log(lo))).astype(np.uint64)


@dataclass
class Request:
    rid: int
    t_arrival: float  # seconds from the start
    state: int
    kind: str  # "gen" or "jump"
    nelem: int  # elements to generate (gen)
    k: int  # jump exponent (jump)


def serving_trace(
    duration_s: float,
    rate_per_s: float = 20000.0,
    n_states: int = 4096,
    min_bytes: int = 4096,
    max_bytes: int = 256 << 20,
    elem_bytes: int = 8,
    jump_fraction: float = 0.1,
    kmin: int = 32,
    kmax: int = 256,
    seed: int = 11,
) -> list:
    """Poisson request stream for the serving loop."""
    rng = np.random.default_rng(seed)
    n = int(rate_per_s * duration_s * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, n))
    t = t[t < duration_s]
    n = len(t)
    u = rng.random(n)
    nbytes = np.exp(u * np.log(max_bytes / min_bytes) + np.log(min_bytes))
    nelem = np.maximum(1, (nbytes // elem_bytes)).astype(np.int64)
    states = rng.integers(0, n_states, n)
    is_jump = rng.random(n) < jump_fraction
    ks = rng.integers(kmin, kmax + 1, n)
    return [
        Request(i, float(t[i]), int(states[i]), "jump" if is_jump[i] else "gen", int(nelem[i]), int(ks[i]))
        for i in range(n)
    ]


def plan_rounds(lens: np.ndarray, arena_bytes: int, elem_bytes: int):
    """Deal the tasks (longest first) round-robin over R rounds and give each
    task a 256-byte aligned slice of the arena within its round."""
    total = int(sum(((int(n) * elem_bytes + 255) // 256) * 256 for n in lens))
    R = max(1, -(-total // arena_bytes))
    while True:
        order = np.argsort(-lens.astype(np.int64), kind="stable")
        rounds = [order[r::R] for r in range(R)]
        offs = {}
        ok = True
        for r, idx in enumerate(rounds):
            off = 0
            for i in idx:
                offs[int(i)] = off
                off += ((int(lens[i]) * elem_bytes + 255) // 256) * 256
            if off > arena_bytes:
                ok = False
                break
        if ok:
            return rounds, offs
        R += 1
