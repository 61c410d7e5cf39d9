"""The batch planner (host-only C code in libgfs.so): units cover every file exactly once,
in pieces of at most unit_bytes, and about grid/blocks_per_file files are interleaved."""
import numpy as np
import pytest

from paper_2109_05366_amd import gfs


@pytest.mark.parametrize("bpf", [1, 4, 16, 1024])
def test_plan_covers_each_file_once(bpf):
    rng = np.random.default_rng(3)
    sizes = rng.integers(0, 5 << 20, size=37).astype(np.uint64) // 8 * 8
    sizes[5] = 0
    ids = np.arange(100, 137, dtype=np.uint32)
    unit = 256 << 10
    plan = gfs.gfs_batch_plan(sizes, ids, unit, 64, bpf)
    assert len(plan) == sum(int((s + unit - 1) // unit) for s in sizes)
    for i, s in enumerate(sizes):
        u = plan[plan["out"] == i]
        assert np.all(u["file"] == ids[i])
        assert np.all(u["size"] <= unit) and np.all(u["size"] > 0)
        got = sorted(zip(u["offset"].tolist(), u["size"].tolist()))
        pos = 0
        for off, sz in got:
            assert off == pos
            pos += sz
        assert pos == s
    # a file's units appear in offset order
    for i in range(len(sizes)):
        offs = plan[plan["out"] == i]["offset"]
        assert np.all(np.diff(offs.astype(np.int64)) > 0)


def test_plan_interleaves_grid_over_blocks_per_file_files():
    sizes = np.full(20, 64 << 20, dtype=np.uint64)
    ids = np.arange(20, dtype=np.uint32)
    plan = gfs.gfs_batch_plan(sizes, ids, 1 << 20, 64, 8)          # 8 files at a time
    head = plan[:64]
    assert len(set(head["out"].tolist())) == 8
    assert [int(x) for x in head["out"][:8]] == list(range(8))
    plan1 = gfs.gfs_batch_plan(sizes, ids, 1 << 20, 64, 64)        # one file at a time
    assert len(set(plan1[:64]["out"].tolist())) == 1


def test_plan_rejects_bad_arguments():
    with pytest.raises(OSError):
        gfs.gfs_batch_plan(np.array([10], np.uint64), np.array([0], np.uint32), 100, 64, 1)   # unit % 16
    with pytest.raises(OSError):
        gfs.gfs_batch_plan(np.array([10], np.uint64), np.array([0], np.uint32), 1 << 20, 64, 0)
