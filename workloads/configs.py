"""Synthetic workloads: files, cache geometry and per-block access lists.

Shared by the oracle and by the GPU tests/benchmarks. Nothing here computes a
page-cache, readahead or replacement decision; it only says which file bytes
exist and which (offset, size) reads each threadblock issues, in order.

Workload shapes (sizes are the ones the benchmark and parity tests use):

* ``c1`` plain method, small: 64 MiB file (seed 1), 64 KiB pages, 256 MiB cache,
  64 blocks x 256 threads; block b reads 64 KiB strides b, b+64, ... (16 reads);
  per-block u64 checksum.
* ``c2`` larger-than-cache stream: 8 GiB file (seed 2), 256 KiB pages, 2 GiB cache,
  1024 blocks; block b reads 128 KiB strides b + 1024 k, k = 0..63; per-block
  256-bin u32 byte histogram.
* ``c3a/c3b/c3c`` access-pattern sweep on a 4 GiB file (seed 3), 64 KiB pages,
  1 GiB cache, 1024 blocks x 256 threads: (a) block b reads its own 4 MiB chunk
  in 64 reads of 64 KiB; (b) 64 KiB strides b + 1024 k; (c) 2**20 reads of whole
  64 KiB pages, read i issued by block i mod 1024, page index = top 16 bits of
  SplitMix64 output i+1 with seed 1000003. Per-block u64 checksum.

Scaled-down variants (``*_small``) keep the pattern and the ratios that matter
(file larger than cache, several tiles and a ragged tail) at sizes the oracle
finishes in seconds.
"""
from __future__ import annotations

import dataclasses
import os
import shutil
import subprocess
from typing import Dict, Optional

import numpy as np

from . import splitmix

KiB = 1 << 10
MiB = 1 << 20
GiB = 1 << 30

CONSUMER_CHECKSUM = 0
CONSUMER_HISTOGRAM = 1
CONSUMER_NONE = 2          # the reads only: each block's buffer ends holding its last read


@dataclasses.dataclass(frozen=True)
class FileSpec:
    name: str
    seed: int
    size: int


@dataclasses.dataclass
class Workload:
    """One launch of the strided/list reader: B blocks, K reads each, fixed read size."""
    name: str
    file: FileSpec
    page_size: int
    cache_bytes: int
    blocks: int
    threads: int
    read_size: int
    offsets: np.ndarray            # uint64 [blocks, K]: block b's k-th read offset
    consumer: int                  # CONSUMER_CHECKSUM or CONSUMER_HISTOGRAM
    ra_cap_bytes: int = 16 * MiB   # readahead cap the benchmark uses for this workload

    @property
    def reads_per_block(self) -> int:
        return int(self.offsets.shape[1])

    @property
    def delivered_bytes(self) -> int:
        """Bytes gread() delivers over the whole launch (EOF-clamped)."""
        o = self.offsets.astype(np.int64)
        end = np.minimum(o + self.read_size, self.file.size)
        return int(np.maximum(end - o, 0).sum())


def strided_offsets(blocks: int, reads: int, stride: int) -> np.ndarray:
    """Block b's k-th read is stride number b + blocks*k."""
    b = np.arange(blocks, dtype=np.uint64)[:, None]
    k = np.arange(reads, dtype=np.uint64)[None, :]
    return (b + np.uint64(blocks) * k) * np.uint64(stride)


def chunked_offsets(blocks: int, reads: int, read_size: int) -> np.ndarray:
    """Block b reads its own contiguous chunk of reads*read_size bytes, in order."""
    b = np.arange(blocks, dtype=np.uint64)[:, None]
    k = np.arange(reads, dtype=np.uint64)[None, :]
    return (b * np.uint64(reads) + k) * np.uint64(read_size)


def random_page_offsets(blocks: int, nreads: int, npages_log2: int, page: int, seed: int) -> np.ndarray:
    """Read i goes to block i mod blocks; its page is the top npages_log2 bits of output i+1."""
    if nreads % blocks:
        raise ValueError("nreads must be a multiple of blocks")
    x = splitmix.outputs(seed, 1, nreads)
    pages = x >> np.uint64(64 - npages_log2)
    # read i -> block i % blocks, position i // blocks
    return (pages * np.uint64(page)).reshape(nreads // blocks, blocks).T.copy()


def c1() -> Workload:
    f = FileSpec("c1_seed1_64MiB.bin", 1, 64 * MiB)
    return Workload("c1", f, 64 * KiB, 256 * MiB, 64, 256, 64 * KiB,
                    strided_offsets(64, 16, 64 * KiB), CONSUMER_CHECKSUM)


def c2() -> Workload:
    f = FileSpec("c2_seed2_8GiB.bin", 2, 8 * GiB)
    return Workload("c2", f, 256 * KiB, 2 * GiB, 1024, 256, 128 * KiB,
                    strided_offsets(1024, 64, 128 * KiB), CONSUMER_HISTOGRAM)


def f3() -> Workload:
    """Small-page regime: a 1 GiB file (seed 4) through a 256 MiB cache of 4 KiB pages,
    1024 blocks reading 128 KiB strides b + 1024 k (8 reads each), per-block checksums.
    The page size here is the small one; the comparison runs the same reads with 64 KiB
    pages."""
    f = FileSpec("f3_seed4_1GiB.bin", 4, 1 * GiB)
    return Workload("f3", f, 4 * KiB, 256 * MiB, 1024, 256, 128 * KiB,
                    strided_offsets(1024, 8, 128 * KiB), CONSUMER_CHECKSUM)


def f3_small() -> Workload:
    """The small-page shape at a size the oracle finishes in seconds: a 3 MiB + 12 KiB + 40 B
    file (seed 4, a ragged last page) through a 512 KiB cache of 4 KiB pages (128 frames),
    8 blocks reading 32 KiB strides b + 8 k (8 pages per read, 13 reads each; the last
    stride is partial and some reads land past the end), per-block checksums."""
    size = 3 * MiB + 12 * KiB + 40
    f = FileSpec("f3s_seed4.bin", 4, size)
    stride = 32 * KiB
    nstrides = (size + stride - 1) // stride
    blocks = 8
    reads = (nstrides + blocks - 1) // blocks
    return Workload("f3_small", f, 4 * KiB, 512 * KiB, blocks, 256, stride,
                    strided_offsets(blocks, reads, stride), CONSUMER_CHECKSUM)


def _c3_file() -> FileSpec:
    return FileSpec("c3_seed3_4GiB.bin", 3, 4 * GiB)


def c3(pattern: str) -> Workload:
    f = _c3_file()
    if pattern == "a":
        off = chunked_offsets(1024, 64, 64 * KiB)
    elif pattern == "b":
        off = strided_offsets(1024, 64, 64 * KiB)
    elif pattern == "c":
        off = random_page_offsets(1024, 1 << 20, 16, 64 * KiB, 1000003)
    else:
        raise ValueError(pattern)
    return Workload("c3" + pattern, f, 64 * KiB, 1 * GiB, 1024, 256, 64 * KiB, off, CONSUMER_CHECKSUM)


# ---- scaled-down variants the oracle finishes in seconds --------------------------------

def c1_small() -> Workload:
    """C1 shape with a ragged tail: the file ends 24 KiB + 8 B into its last page."""
    size = 3 * MiB + 24 * KiB + 8
    f = FileSpec("c1s_seed1.bin", 1, size)
    stride = 64 * KiB
    nstrides = (size + stride - 1) // stride     # 49 strides, the last one partial
    blocks = 8
    reads = (nstrides + blocks - 1) // blocks    # 7 reads; some land at/after EOF
    return Workload("c1_small", f, 64 * KiB, 16 * MiB, blocks, 256, stride,
                    strided_offsets(blocks, reads, stride), CONSUMER_CHECKSUM)


def c2_small() -> Workload:
    """C2 shape at 1/128 scale: 64 MiB file through a 16 MiB cache (64 frames), histograms."""
    f = FileSpec("c2s_seed2.bin", 2, 64 * MiB)
    return Workload("c2_small", f, 256 * KiB, 16 * MiB, 64, 256, 128 * KiB,
                    strided_offsets(64, 8, 128 * KiB), CONSUMER_HISTOGRAM)


def c3_small(pattern: str) -> Workload:
    f = FileSpec("c3s_seed3.bin", 3, 16 * MiB)
    blocks = 32
    if pattern == "a":
        off = chunked_offsets(blocks, 8, 64 * KiB)
    elif pattern == "b":
        off = strided_offsets(blocks, 8, 64 * KiB)
    elif pattern == "c":
        off = random_page_offsets(blocks, 32 * 64, 8, 64 * KiB, 1000003)
    else:
        raise ValueError(pattern)
    return Workload("c3" + pattern + "_small", f, 64 * KiB, 4 * MiB, blocks, 256, 64 * KiB, off, CONSUMER_CHECKSUM)


@dataclasses.dataclass
class MixedWorkload:
    """Two files read at once through one persistent batch launch (the mixed case of Sec. 3.1,
    where one file is read sequentially and another at random): file 0 in consecutive pieces,
    file 1 in whole pages at random; the unit list interleaves one piece of file 0 with
    `ratio` random reads of file 1. Output row 0 folds file 0's reads, row 1 file 1's."""
    name: str
    seq: FileSpec
    rnd: FileSpec
    page_size: int
    cache_bytes: int
    piece: int                 # bytes per sequential read of file 0
    nrandom: int               # random page reads of file 1
    ratio: int
    seed: int                  # SplitMix64 seed of the random page indices

    def units(self) -> np.ndarray:
        """Records (file, out, offset, size) in launch order; file = 0 or 1 (the caller maps
        them to registered ids)."""
        seq_off = np.arange(0, self.seq.size, self.piece, dtype=np.uint64)
        npages = self.rnd.size // self.page_size
        bits = int(npages).bit_length() - 1
        if 1 << bits != npages:
            raise ValueError("file 1 must hold a power-of-two number of pages")
        pages = splitmix.outputs(self.seed, 1, self.nrandom) >> np.uint64(64 - bits)
        rnd_off = pages * np.uint64(self.page_size)
        dt = np.dtype([("file", "<u4"), ("out", "<u4"), ("offset", "<u8"), ("size", "<u8")])
        out = np.zeros(len(seq_off) + len(rnd_off), dtype=dt)
        k = i = j = 0
        while i < len(seq_off) or j < len(rnd_off):
            if i < len(seq_off):
                out[k] = (0, 0, seq_off[i], min(self.piece, self.seq.size - int(seq_off[i])))
                k += 1
                i += 1
            for _ in range(self.ratio):
                if j < len(rnd_off):
                    out[k] = (1, 1, rnd_off[j], self.page_size)
                    k += 1
                    j += 1
        return out


def f2() -> MixedWorkload:
    """2 GiB read in 1 MiB pieces (seed 5) beside 32768 random 64 KiB page reads of another
    2 GiB file (seed 6, page indices from SplitMix64 seed 1000006), 1 GiB cache."""
    return MixedWorkload("f2", FileSpec("f2a_seed5_2GiB.bin", 5, 2 * GiB), FileSpec("f2b_seed6_2GiB.bin", 6, 2 * GiB),
                         64 * KiB, 1 * GiB, 1 * MiB, 32768, 16, 1000006)


def f2_small() -> MixedWorkload:
    """The mixed case at 1/128 scale: 16 MiB in 256 KiB pieces beside 256 random page reads of
    a 16 MiB file, 8 MiB cache (128 frames)."""
    return MixedWorkload("f2_small", FileSpec("f2sa_seed5.bin", 5, 16 * MiB), FileSpec("f2sb_seed6.bin", 6, 16 * MiB),
                         64 * KiB, 8 * MiB, 256 * KiB, 256, 4, 1000006)


REGISTRY = {
    "c1": c1, "c2": c2,
    "c3a": lambda: c3("a"), "c3b": lambda: c3("b"), "c3c": lambda: c3("c"),
    "c1_small": c1_small, "c2_small": c2_small,
    "c3a_small": lambda: c3_small("a"), "c3b_small": lambda: c3_small("b"),
    "c3c_small": lambda: c3_small("c"), "f3": f3, "f3_small": f3_small,
}


def get(name: str) -> Workload:
    return REGISTRY[name]()


# ---- files on disk ----------------------------------------------------------------------

_HERE = os.path.dirname(os.path.abspath(__file__))
_GEN_SRC = os.path.join(_HERE, "genfile.c")
_GEN_BIN = os.path.join(_HERE, "genfile")
_PEAK_SRC = os.path.join(_HERE, "readpeak.c")
_PEAK_BIN = os.path.join(_HERE, "readpeak")


def data_dir() -> str:
    d = os.environ.get("GFS_DATA_DIR") or os.path.join(os.path.dirname(_HERE), "_data")
    os.makedirs(d, exist_ok=True)
    return d


def build_generator(force: bool = False) -> str:
    """Compile the C file writer with gcc (a build step; no method code inside)."""
    if force or not os.path.exists(_GEN_BIN) or os.path.getmtime(_GEN_BIN) < os.path.getmtime(_GEN_SRC):
        cc = shutil.which("gcc") or shutil.which("cc")
        if not cc:
            raise RuntimeError("no C compiler to build workloads/genfile")
        subprocess.check_call([cc, "-O2", "-o", _GEN_BIN, _GEN_SRC, "-lpthread"])
    return _GEN_BIN


def build_readpeak(force: bool = False) -> str:
    """Compile the C sequential-read timer (the storage bound of the benchmarks)."""
    if force or not os.path.exists(_PEAK_BIN) or os.path.getmtime(_PEAK_BIN) < os.path.getmtime(_PEAK_SRC):
        cc = shutil.which("gcc") or shutil.which("cc")
        if not cc:
            raise RuntimeError("no C compiler to build workloads/readpeak")
        subprocess.check_call([cc, "-O2", "-o", _PEAK_BIN, _PEAK_SRC, "-lpthread"])
    return _PEAK_BIN


def read_peak(paths, threads: int = 32, chunk: int = 4 << 20, limit: int = 8 << 30) -> float:
    """Sequential read rate (10^9 B/s) of the largest of `paths`, up to `limit` bytes in all,
    by `threads` native threads reading `chunk`-byte pieces (O_DIRECT where allowed)."""
    order = sorted(paths, key=os.path.getsize, reverse=True)
    pick, tot = [], 0
    for p in order:
        if tot >= limit:
            break
        pick.append(p)
        tot += os.path.getsize(p)
    out = subprocess.check_output([build_readpeak(), str(threads), str(chunk), str(limit), *pick], text=True)
    nbytes, secs = out.split()
    return int(nbytes) / float(secs) / 1e9


def ensure_file(spec: FileSpec, directory: Optional[str] = None, threads: int = 8) -> str:
    """Create the SplitMix64 file if it is missing or has the wrong size; return its path."""
    d = directory or data_dir()
    path = os.path.join(d, spec.name)
    if os.path.exists(path) and os.path.getsize(path) == spec.size:
        return path
    gen = build_generator()
    os.makedirs(d, exist_ok=True)
    subprocess.check_call([gen, path, str(spec.seed), str(spec.size), str(threads)])
    return path
