"""Pins for the data half of the oracle and for the shared input generator (CPU only).

What pins what:
* the published SplitMix64 vector (Vigna's reference, seed 1234567) pins the
  generator's arithmetic;
* the C file writer is checked byte for byte against the Python definition;
* the checksum / histogram definitions are checked on hand-made buffers;
* pread-based per-block checksums and histograms are checked against an
  independent pure-Python recomputation from the SplitMix64 closed form (no file
  I/O, no numpy), on a file with a ragged tail and reads at and past EOF.
"""
import os
import struct

import numpy as np
import pytest

from oracle import data
from workloads import configs, splitmix

MASK = (1 << 64) - 1


def test_splitmix_published_vector():
    # Published first outputs of splitmix64 with seed 1234567.
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423]
    assert [splitmix.output_int(1234567, k) for k in (1, 2, 3)] == expect
    assert [int(x) for x in splitmix.outputs(1234567, 1, 3)] == expect


def test_file_bytes_little_endian_layout():
    out1 = splitmix.output_int(1, 1)
    out2 = splitmix.output_int(1, 2)
    expect = struct.pack("<QQ", out1, out2)
    assert splitmix.file_bytes(1, 0, 16) == expect
    assert splitmix.file_bytes(1, 3, 7) == expect[3:10]
    assert expect.hex() == "c15c0289ec2d0a9167ec8e65a18debbe"


def test_generated_file_matches_definition(data_dir):
    spec = configs.FileSpec("pin_gen.bin", 7, (9 << 20) + 13)   # ragged: not a multiple of 8
    path = configs.ensure_file(spec, data_dir, threads=3)
    assert os.path.getsize(path) == spec.size
    with open(path, "rb") as fh:
        got = fh.read()
    assert got == splitmix.file_bytes(7, 0, spec.size)


def test_checksum_definition_on_handmade_buffers():
    assert data.checksum_of(b"") == 0
    assert data.checksum_of(struct.pack("<II", 1, 2)) == 3
    assert data.checksum_of(b"\x01\x02\x03") == 0x030201            # zero-padded partial word
    assert data.checksum_of(b"\xff" * 4 * 5) == 5 * 0xFFFFFFFF
    # wrap-around of the u64 sum: 2**32 + 1 words of 0xFFFFFFFF would be needed; instead check
    # the modular identity on a synthetic sum
    big = np.full(1 << 20, 0xFFFFFFFF, dtype="<u4").tobytes()
    assert data.checksum_of(big) == (0xFFFFFFFF << 20) & MASK


def test_histogram_definition_on_handmade_buffers():
    h = data.histogram_of(bytes([0, 0, 5, 255, 5, 5]))
    assert h.dtype == np.uint32 and h.shape == (256,)
    assert h[0] == 2 and h[5] == 3 and h[255] == 1 and int(h.sum()) == 6


def _closed_form_read(seed, fsize, off, size):
    """Pure-Python bytes of a read, straight from the generator definition."""
    if size <= 0 or off >= fsize:
        return b""
    end = min(off + size, fsize)
    out = bytearray()
    for o in range(off, end):
        w = splitmix.output_int(seed, o // 8 + 1)
        out.append((w >> (8 * (o % 8))) & 0xFF)
    return bytes(out)


def _closed_form_checksum(buf):
    s = 0
    for i in range(0, len(buf), 4):
        word = 0
        for j, byte in enumerate(buf[i:i + 4]):
            word |= byte << (8 * j)
        s = (s + word) & MASK
    return s


def test_block_checksums_vs_closed_form(data_dir):
    wl = configs.c1_small()
    path = configs.ensure_file(wl.file, data_dir)
    got = data.block_checksums(path, wl.offsets, wl.read_size, blocks=[0, 3, 7])
    for b in (0, 3, 7):
        s = 0
        for off in wl.offsets[b]:
            # word-level closed form: read offsets are multiples of 8, so word pairs are outputs
            off = int(off)
            end = min(off + wl.read_size, wl.file.size)
            if end <= off:
                continue
            full_words = (end - off) // 8
            for k in range(full_words):
                w = splitmix.output_int(wl.file.seed, off // 8 + k + 1)
                s = (s + (w & 0xFFFFFFFF) + (w >> 32)) & MASK
            tail = _closed_form_read(wl.file.seed, wl.file.size, off + 8 * full_words, end - off - 8 * full_words)
            s = (s + _closed_form_checksum(tail)) & MASK
        assert int(got[b]) == s, b
    # blocks not asked for stay zero
    assert int(got[1]) == 0


def test_reads_at_and_past_eof(data_dir):
    wl = configs.c1_small()
    path = configs.ensure_file(wl.file, data_dir)
    size = wl.file.size
    assert data.delivered(path, size, 100) == b""
    assert data.delivered(path, size + 4096, 100) == b""
    tail = data.delivered(path, size - 5, 64)
    assert tail == _closed_form_read(wl.file.seed, size, size - 5, 64) and len(tail) == 5
    assert data.delivered(path, 0, 0) == b""


def test_block_histograms_vs_closed_form(data_dir):
    wl = configs.c2_small()
    path = configs.ensure_file(wl.file, data_dir)
    got = data.block_histograms(path, wl.offsets, wl.read_size, blocks=[5])
    h = [0] * 256
    for off in wl.offsets[5]:
        off = int(off)
        for k in range(wl.read_size // 8):
            w = splitmix.output_int(wl.file.seed, off // 8 + k + 1)
            for t in range(8):
                h[(w >> (8 * t)) & 0xFF] += 1
    assert [int(x) for x in got[5]] == h
    assert int(got[5].sum()) == wl.reads_per_block * wl.read_size


def test_whole_file_checksum_and_histogram(data_dir):
    spec = configs.FileSpec("pin_whole.bin", 11, (3 << 20) + 40)
    path = configs.ensure_file(spec, data_dir)
    raw = splitmix.file_bytes(11, 0, spec.size)
    assert data.file_checksum(path, chunk=1 << 20) == _closed_form_checksum(raw)
    h = data.file_histogram(path, chunk=1 << 20)
    assert [int(x) for x in h] == [raw.count(bytes([v])) for v in range(256)]
