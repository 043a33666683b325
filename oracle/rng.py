"""Counter-based random signs for the randomized range finder (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  With state x and gamma
G = 0x9E3779B97F4A7C15 the n-th output (n = 0, 1, ...) of a generator seeded
with x is mix(x + (n + 1) * G), where mix(z) applies
z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
z ^= z >> 31 (all modulo 2^64).

Stream keys: key_0 = seed, key_{m+1} = out0(key_m XOR tag_m) for the tags of
one truncation (purpose, message, sweep, step, split), where out0(x) is the
first output of the generator seeded with x.  Sketch entry (i, j) of an
n x k matrix is taken from output number i*k + j of the generator seeded with
the stream key: bit 63 gives the sign of the real part, bit 62 the sign of
the imaginary part, and the entry is (+-1 +- 1j)/sqrt(2).
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def mix(z):
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def output(seed, n):
    """n-th output of SplitMix64 seeded with ``seed``."""
    return mix(seed + (n + 1) * GAMMA)


def stream_key(seed, tags):
    k = seed & MASK
    for t in tags:
        k = output(k ^ (t & MASK), 0)
    return k


def sign_matrix(key, n, k):
    """n x k complex sketch with entries (+-1 +- 1j)/sqrt(2)."""
    out = np.empty((n, k), complex)
    s = 1.0 / np.sqrt(2.0)
    for i in range(n):
        for j in range(k):
            z = output(key, i * k + j)
            re = -1.0 if (z >> 63) & 1 else 1.0
            im = -1.0 if (z >> 62) & 1 else 1.0
            out[i, j] = complex(re * s, im * s)
    return out
