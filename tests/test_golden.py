"""Stored expected values (tests/golden/) against independent pins, and the oracle against them.

The C1 per-block checksums and the C2 spot histogram were first computed two independent
ways (vectorised numpy and pure-Python struct unpacking of the SplitMix64 closed form) when
the workloads were specified: block 0 = 562589286878686, block 1 = 562473151362049, block 2 =
563700609022817, block 3 = 563065335666973, block 63 = 562692025587906, sum over the 64 blocks
= 36027982716856646; bins 0..3 of the C2 spot histogram = 523, 546, 537, 506. Those numbers
are restated here as the pins; the stored files are written by tests/golden/make_golden.py
from oracle.data and must agree with them, and the oracle must reproduce the stored files.
"""
import numpy as np

from golden import make_golden
from oracle import data
from workloads import configs, splitmix

C1_PINS = {0: 562589286878686, 1: 562473151362049, 2: 563700609022817, 3: 563065335666973,
           63: 562692025587906}
C1_SUM = 36027982716856646
C2_BINS_0_3 = [523, 546, 537, 506]


def test_stored_c1_checksums_equal_the_pins():
    vals, total = make_golden.load_c1()
    assert len(vals) == 64
    for b, v in C1_PINS.items():
        assert vals[b] == v, b
    assert total == C1_SUM == sum(vals) & ((1 << 64) - 1)
    # magnitude: 16 reads of 16384 uniform u32 words per block, each ~2^31 on average
    # (standard deviation of a block sum: 512 * 2^32 / sqrt(12), about 2^39.3)
    assert all(abs(v - 16 * 16384 * 2 ** 31) < 2 ** 42 for v in vals)


def test_stored_c2_histogram_equals_the_pins():
    h = make_golden.load_c2_head()
    assert h[:4] == C2_BINS_0_3 and sum(h) == 128 << 10


def test_oracle_reproduces_stored_values(data_dir):
    vals, _ = make_golden.load_c1()
    assert make_golden.c1_values(data_dir) == vals
    assert make_golden.c2_head_histogram(data_dir) == make_golden.load_c2_head()


def test_c1_block0_from_closed_form():
    """Block 0's checksum straight from the generator definition (no file, no numpy)."""
    wl = configs.c1()
    s = 0
    for off in wl.offsets[0]:
        for k in range(wl.read_size // 8):
            w = splitmix.output_int(1, int(off) // 8 + k + 1)
            s = (s + (w & 0xFFFFFFFF) + (w >> 32)) & ((1 << 64) - 1)
    assert s == C1_PINS[0]


def test_unit_outputs_and_file_digest_agree_with_the_definitions(data_dir):
    spec = configs.FileSpec("pin_units.bin", 13, (2 << 20) + 20)
    path = configs.ensure_file(spec, data_dir)
    raw = splitmix.file_bytes(13, 0, spec.size)
    c, h = data.file_digest(path, chunk=1 << 19)
    assert c == data.file_checksum(path) and np.array_equal(h, data.file_histogram(path))
    assert np.array_equal(h, np.bincount(np.frombuffer(raw, np.uint8), minlength=256))
    # two rows: row 0 reads the file whole in two pieces, row 1 reads the same 4 KiB twice
    units = np.zeros(4, dtype=[("file", "<u4"), ("out", "<u4"), ("offset", "<u8"), ("size", "<u8")])
    units[0] = (0, 0, 0, 1 << 20)
    units[1] = (0, 0, 1 << 20, spec.size)            # short at EOF
    units[2] = (0, 1, 4096, 4096)
    units[3] = (0, 1, 4096, 4096)
    cs, hs = data.unit_outputs({0: path}, units, 2)
    assert int(cs[0]) == c and np.array_equal(hs[0], h)
    piece = raw[4096:8192]
    assert int(cs[1]) == (2 * data.checksum_of(piece)) & ((1 << 64) - 1)
    assert int(hs[1].sum()) == 8192
