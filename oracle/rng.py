"""Counter-based Gaussian stream for the sketch vectors (test infrastructure, see package header).

Alg. 4 draws a Gaussian vector omega in R^k for every stored solution; the paper names no
generator. Reading: SplitMix64 (Steele, Lea & Flood 2014) used as a counter-based generator,
out(seed, i) = mix(seed + i * 0x9E3779B97F4A7C15 mod 2^64), two outputs per draw mapped to
uniforms u = (floor(out / 2^11) + 1) 2^-53 in (0, 1], and the Box-Muller transform
z = sqrt(-2 ln u1) cos(2 pi u2). Draw a of solution s uses counters 2(64 s + a) + 1 and + 2
(k <= 64). Computed with the platform libm through Python's math module.

Pins (tests/test_oracle_subspace.py): the first SplitMix64 output for seed 0 is the
published 0xE220A8397B1DCDAF; sample mean and variance of 2^16 draws.
"""
from __future__ import annotations

import math

GAMMA = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1
KMAX = 64


def mix(z: int) -> int:
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def splitmix64(seed: int, i: int) -> int:
    return mix((seed + i * GAMMA) & MASK)


def uniform(seed: int, i: int) -> float:
    return ((splitmix64(seed, i) >> 11) + 1) * 2.0 ** -53


def gaussian(seed: int, s: int, a: int) -> float:
    i = 2 * (KMAX * s + a) + 1
    u1, u2 = uniform(seed, i), uniform(seed, i + 1)
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def omega(seed: int, s: int, k: int) -> list:
    if not 1 <= k <= KMAX:
        raise ValueError("k out of range")
    return [gaussian(seed, s, a) for a in range(k)]
