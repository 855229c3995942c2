"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the benchmark.

This module holds no arithmetic of the method (no modular multiplication, no
transform, no reduction).  It only draws pseudo-random 64-bit words and turns
them into coefficients:

* SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014) in its counter form: the k-th output of a stream with
  seed s is mix(s + (k + 1) * 0x9E3779B97F4A7C15).
* Uniform values in [0, q) by rejection: a word r is kept when
  r < q * floor(2^64 / q), and then r mod q is used, so every residue is equally
  likely.
* "Lazy" operands in [0, f * q) as x + q * r with x uniform in [0, q) and r
  uniform in [0, f): the representatives the paper's input_mod_factor allows.

Every (workload, polynomial, limb, operand) unit has its own seed, so a unit has
identical data whether it is generated alone or inside a batch.
"""
from __future__ import annotations

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MASK64 = (1 << 64) - 1


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Words offset .. offset+count-1 of the SplitMix64 stream with this seed."""
    k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & MASK64) + k * GOLDEN_GAMMA
        return _mix(state)


def unit_seed(*parts: int) -> int:
    """Derives one 64-bit seed from a tuple of non-negative integers."""
    s = 0x243F6A8885A308D3
    for p in parts:
        s = int(splitmix64((s ^ (int(p) & MASK64)) & MASK64, 1)[0])
    return s


def uniform_mod(seed: int, n: int, q: int) -> np.ndarray:
    """n values uniform in [0, q), drawn by rejection from the seed's stream."""
    if q < 1 or q > MASK64:
        raise ValueError("modulus out of range")
    limit = (((1 << 64) // q) * q)            # words >= limit are rejected
    out = np.empty(n, dtype=np.uint64)
    have, offset = 0, 0
    while have < n:
        want = n - have
        words = splitmix64(seed, want + 16, offset)
        offset += want + 16
        if limit <= MASK64:
            words = words[words < np.uint64(limit)]
        take = min(want, words.size)
        out[have:have + take] = words[:take] % np.uint64(q)
        have += take
    return out


def lazy_mod(seed: int, n: int, q: int, factor: int) -> np.ndarray:
    """n values in [0, factor * q): x + q * r, x uniform in [0, q), r uniform in [0, factor)."""
    if factor < 1 or factor * q > MASK64:
        raise ValueError("factor * q must fit in 64 bits")
    x = uniform_mod(seed, n, q)
    if factor == 1:
        return x
    r = uniform_mod(unit_seed(seed, 0x1A27), n, factor)
    with np.errstate(over="ignore"):
        return x + r * np.uint64(q)


def uniform_int(seed: int, n: int, lo: int, hi: int) -> np.ndarray:
    """n integers uniform in [lo, hi] (inclusive), e.g. ring sizes or limb counts."""
    return uniform_mod(seed, n, hi - lo + 1).astype(np.int64) + lo


def exponential(seed: int, n: int, mean: float) -> np.ndarray:
    """n exponential variates with the given mean (inter-arrival times of a Poisson stream)."""
    u = (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    return -mean * np.log1p(-u)
