"""What gread() must deliver, and what the benchmark consumers compute from it.

Test infrastructure only (see the package docstring).

* gread(fd, offset, size) delivers exactly the file bytes
  [offset, min(offset + size, file_size)) -- a POSIX read at an offset, which is
  what the paper's GPU file API exposes to threadblocks (Sec. 2.2, "GPUfs").
  The oracle gets those bytes with a plain ``os.pread``.
* checksum: wrapping uint64 sum of the little-endian uint32 words of each
  delivered buffer, a trailing partial word zero-padded; a block's checksum is
  the sum over its reads in order (integer addition, so order-independent).
* histogram: uint32 count of each byte value over every byte a block receives.
"""
from __future__ import annotations

import os
from typing import Iterable

import numpy as np


def delivered(path: str, offset: int, size: int) -> bytes:
    """The bytes a read of ``size`` at ``offset`` returns (short at EOF, empty past it)."""
    fsize = os.path.getsize(path)
    if size <= 0 or offset >= fsize:
        return b""
    n = min(size, fsize - offset)
    fd = os.open(path, os.O_RDONLY)
    try:
        out = bytearray()
        while len(out) < n:
            chunk = os.pread(fd, n - len(out), offset + len(out))
            if not chunk:
                raise IOError(f"unexpected EOF in {path} at {offset + len(out)}")
            out += chunk
        return bytes(out)
    finally:
        os.close(fd)


def checksum_of(buf: bytes) -> int:
    """Wrapping u64 sum of LE u32 words; a trailing partial word is zero-padded."""
    pad = (-len(buf)) % 4
    b = buf + b"\0" * pad
    words = np.frombuffer(b, dtype="<u4").astype(np.uint64)
    with np.errstate(over="ignore"):
        return int(words.sum(dtype=np.uint64))


def histogram_of(buf: bytes) -> np.ndarray:
    """Count of each byte value 0..255 (uint32)."""
    a = np.frombuffer(buf, dtype=np.uint8)
    return np.bincount(a, minlength=256).astype(np.uint32)


def _rows(nb: int, blocks) -> list:
    return list(range(nb)) if blocks is None else list(blocks)


def block_checksums(path: str, offsets: np.ndarray, read_size: int,
                    blocks: Iterable[int] | None = None) -> np.ndarray:
    """Per-block u64 checksums; ``offsets[b, k]`` is block b's k-th read.

    If ``blocks`` is given only those rows are computed (the rest stay 0). Reads at the same
    offset deliver the same bytes, so each distinct offset's checksum is computed once."""
    nb = offsets.shape[0]
    out = np.zeros(nb, dtype=np.uint64)
    memo = {}
    for b in _rows(nb, blocks):
        s = 0
        for off in offsets[b]:
            o = int(off)
            if o not in memo:
                memo[o] = checksum_of(delivered(path, o, read_size))
            s = (s + memo[o]) & ((1 << 64) - 1)
        out[b] = np.uint64(s)
    return out


def block_histograms(path: str, offsets: np.ndarray, read_size: int,
                     blocks: Iterable[int] | None = None) -> np.ndarray:
    """Per-block 256-bin u32 histograms; rows not in ``blocks`` stay 0."""
    nb = offsets.shape[0]
    out = np.zeros((nb, 256), dtype=np.uint32)
    for b in _rows(nb, blocks):
        h = np.zeros(256, dtype=np.uint64)
        for off in offsets[b]:
            h += histogram_of(delivered(path, int(off), read_size))
        out[b] = h.astype(np.uint32)
    return out


def unit_outputs(paths: dict, units, nout: int) -> tuple:
    """Per-output-row checksum and histogram of a list of reads: ``units`` holds
    (file, out, offset, size) records; row ``out`` sums every read folded into it, the way the
    batch consumer does (integer sums, so the order of the reads does not matter). ``paths``
    maps a unit's file to its path. Reads of the same (file, offset, size) are computed once."""
    csum = [0] * nout
    hist = np.zeros((nout, 256), dtype=np.uint64)
    memo = {}
    for u in units:
        f, o, off, size = int(u["file"]), int(u["out"]), int(u["offset"]), int(u["size"])
        key = (f, off, size)
        if key not in memo:
            buf = delivered(paths[f], off, size)
            memo[key] = (checksum_of(buf), histogram_of(buf).astype(np.uint64))
        c, h = memo[key]
        csum[o] = (csum[o] + c) & ((1 << 64) - 1)
        hist[o] += h
    return np.array(csum, dtype=np.uint64), hist.astype(np.uint32)


def file_checksum(path: str, chunk: int = 64 << 20) -> int:
    """Checksum of the whole file: its bytes are one delivered buffer (chunks are multiples of
    4 bytes, so summing per chunk changes nothing)."""
    size = os.path.getsize(path)
    s = 0
    for off in range(0, size, chunk):
        s = (s + checksum_of(delivered(path, off, chunk))) & ((1 << 64) - 1)
    return s


def file_histogram(path: str, chunk: int = 64 << 20) -> np.ndarray:
    """Byte-value counts of the whole file (uint32; files here are below 4 GiB)."""
    size = os.path.getsize(path)
    h = np.zeros(256, dtype=np.uint64)
    for off in range(0, size, chunk):
        h += histogram_of(delivered(path, off, chunk))
    return h.astype(np.uint32)


def file_digest(path: str, chunk: int = 64 << 20) -> tuple:
    """(checksum, histogram) of the whole file in one pass over it (the two definitions
    above, applied to the same chunks)."""
    size = os.path.getsize(path)
    s = 0
    h = np.zeros(256, dtype=np.uint64)
    for off in range(0, size, chunk):
        buf = delivered(path, off, chunk)
        s = (s + checksum_of(buf)) & ((1 << 64) - 1)
        h += histogram_of(buf)
    return s, h.astype(np.uint32)
