"""Writes the stored expected values under tests/golden/ from the oracle alone.

Run from the repository root: ``python -m tests.golden.make_golden``. It generates the
synthetic input files (SplitMix64, the shared input generator), computes the values with
``oracle.data`` and writes one text file per fixture. Nothing here reads the HIP library.

Fixtures:
* c1_block_checksums.txt -- the plain method, small: a 64 MiB file (seed 1), 64 blocks,
  block b reads 64 KiB strides b, b + 64, ... (16 reads); each block's wrapping u64 sum of
  the little-endian u32 words it received, and the sum over blocks.
* c2_block0_first_stride_histogram.txt -- the larger-than-cache stream's file (seed 2):
  the 256-bin byte histogram of bytes [0, 131072), block 0's first 128 KiB read.
"""
from __future__ import annotations

import os
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import data  # noqa: E402
from workloads import configs  # noqa: E402

C2_HEAD = configs.FileSpec("c2head_seed2_1MiB.bin", 2, 1 << 20)   # the C2 file's first MiB


def c1_values(ddir: str):
    wl = configs.c1()
    path = configs.ensure_file(wl.file, ddir)
    return [int(x) for x in data.block_checksums(path, wl.offsets, wl.read_size)]


def c2_head_histogram(ddir: str):
    # byte o of a seed's file does not depend on the file's length, so the first MiB of the
    # 8 GiB file is the 1 MiB file of the same seed
    path = configs.ensure_file(C2_HEAD, ddir)
    return [int(x) for x in data.histogram_of(data.delivered(path, 0, 128 << 10))]


def write(ddir: str) -> None:
    cs = c1_values(ddir)
    with open(os.path.join(HERE, "c1_block_checksums.txt"), "w") as fh:
        fh.write("# C1: 64 MiB SplitMix64 file (seed 1), 64 blocks, block b reads 64 KiB strides\n"
                 "# b + 64 k (k = 0..15); per-block wrapping u64 sum of little-endian u32 words.\n"
                 "# Written by tests/golden/make_golden.py (oracle.data).\n")
        for b, v in enumerate(cs):
            fh.write(f"{b} {v}\n")
        fh.write(f"sum {sum(cs) & ((1 << 64) - 1)}\n")
    h = c2_head_histogram(ddir)
    with open(os.path.join(HERE, "c2_block0_first_stride_histogram.txt"), "w") as fh:
        fh.write("# C2 file (SplitMix64 seed 2): 256-bin histogram of bytes [0, 131072), the first\n"
                 "# 128 KiB read of block 0. Written by tests/golden/make_golden.py (oracle.data).\n")
        for v, c in enumerate(h):
            fh.write(f"{v} {c}\n")


def load_c1():
    vals, total = {}, None
    with open(os.path.join(HERE, "c1_block_checksums.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            if k == "sum":
                total = int(v)
            else:
                vals[int(k)] = int(v)
    return [vals[b] for b in range(len(vals))], total


def load_c2_head():
    out = [0] * 256
    with open(os.path.join(HERE, "c2_block0_first_stride_histogram.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            out[int(k)] = int(v)
    return out


if __name__ == "__main__":
    with tempfile.TemporaryDirectory(prefix="gfs_golden_") as d:
        write(d)
    print("wrote", os.path.join(HERE, "c1_block_checksums.txt"), "and",
          os.path.join(HERE, "c2_block0_first_stride_histogram.txt"))
