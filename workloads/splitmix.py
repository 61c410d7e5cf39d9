"""SplitMix64 stream: the seeded source of every synthetic file and access list.

This module is the shared input generator. It holds no arithmetic of the page
cache, readahead or replacement method: it only defines which bytes the
synthetic files contain and which offsets the synthetic workloads read.

Definition (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014; the increment-then-mix form of Vigna's reference
``splitmix64.c``):

    output(seed, k) = mix(seed + k * 0x9E3779B97F4A7C15 mod 2**64),  k = 1, 2, ...
    mix(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
            z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31   (all mod 2**64)

File contents: byte ``o`` of a file with seed ``s`` is byte ``o mod 8``
(little-endian) of ``output(s, o // 8 + 1)``; the last output is truncated to
the file size.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB


def mix_int(z: int) -> int:
    """SplitMix64 finaliser on a Python int (mod 2**64)."""
    z &= MASK64
    z ^= z >> 30
    z = (z * M1) & MASK64
    z ^= z >> 27
    z = (z * M2) & MASK64
    z ^= z >> 31
    return z


def output_int(seed: int, k: int) -> int:
    """The k-th output (k >= 1) of the stream with the given seed."""
    return mix_int((seed + k * GAMMA) & MASK64)


def outputs(seed: int, k0: int, n: int) -> np.ndarray:
    """Outputs k0, k0+1, ..., k0+n-1 as a uint64 array (vectorised, wrapping)."""
    k = np.arange(k0, k0 + n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + k * np.uint64(GAMMA)
        z ^= z >> np.uint64(30)
        z *= np.uint64(M1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(M2)
        z ^= z >> np.uint64(31)
    return z


def file_bytes(seed: int, offset: int, length: int) -> bytes:
    """Bytes [offset, offset+length) of the (unbounded) stream file with this seed."""
    if length <= 0:
        return b""
    w0 = offset // 8
    w1 = (offset + length + 7) // 8
    words = outputs(seed, w0 + 1, w1 - w0).astype("<u8")
    raw = words.tobytes()
    s = offset - 8 * w0
    return raw[s:s + length]
