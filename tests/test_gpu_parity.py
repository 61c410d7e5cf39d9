"""GPU parity: the HIP page cache (through the C-ABI) against the CPU oracle.

Data parity is bit-exact (integers): every block's checksum or histogram and its
delivered byte count equal the oracle's pread-based values. Policy parity: in
serialized mode (test-only gate, one read at a time in (round, block) order) the
device trace equals the oracle model's predicted event sequence exactly.
"""
import os

import numpy as np
import pytest

from oracle.policy import PolicyModel, run_serialized
from paper_2109_05366_amd import gfs, runner
from workloads import configs

from gpu_util import canon, decode, expected

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gfs.lib()
    return torch


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


SMALL = ["c1_small", "c2_small", "c3a_small", "c3b_small", "c3c_small"]


@pytest.mark.parametrize("ra_pages", [0, 16])
@pytest.mark.parametrize("name", SMALL)
def test_small_parity(name, ra_pages, data_dir, cuda):
    wl = configs.get(name)
    path = configs.ensure_file(wl.file, data_dir)
    exp_out, exp_deliv = expected(wl, path)
    _say(f"{name} ra_pages={ra_pages}")
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_pages * wl.page_size, timeout_s=20)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
        st = cache.stats()
    assert st["timeouts"] == 0 and st["io_errors"] == 0, st
    np.testing.assert_array_equal(res.status, exp_deliv)
    np.testing.assert_array_equal(res.out, exp_out)
    assert st["delivered_bytes"] == int(exp_deliv.sum())
    assert st["fetched_pages"] == st["misses"] + st["ra_pages"]
    if ra_pages == 0:
        assert st["ra_pages"] == 0


@pytest.mark.parametrize("name,ra_pages", [
    ("c2_small", 0), ("c2_small", 16), ("c3c_small", 0), ("c3c_small", 8),
    ("c1_small", 8), ("c3a_small", 16), ("c3b_small", 4),
])
def test_serialized_trace_matches_model(name, ra_pages, data_dir, cuda):
    wl = configs.get(name)
    path = configs.ensure_file(wl.file, data_dir)
    _say(f"serialized {name} ra_pages={ra_pages}")
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_pages * wl.page_size,
                             ra_init_pages=4, streams=8, trace_level=2, trace_capacity=1 << 20,
                             timeout_s=20)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer, serialize=True)
        st = cache.stats()
        ev = cache.trace()
    assert st["trace_events"] == len(ev) < (1 << 20)
    exp_out, exp_deliv = expected(wl, path)
    np.testing.assert_array_equal(res.status, exp_deliv)
    np.testing.assert_array_equal(res.out, exp_out)
    C = wl.cache_bytes // wl.page_size
    model = PolicyModel(C, wl.page_size, ra_init_pages=min(4, ra_pages) if ra_pages else 4,
                        ra_cap_pages=ra_pages, streams_per_file=8)
    model.open(fid, wl.file.size)
    run_serialized(model, fid, wl.offsets, wl.read_size)
    got = canon(decode(ev))
    want = canon(model.events)
    assert len(got) == len(want)
    for i, (g, w) in enumerate(zip(got, want)):
        assert g == w, f"event {i}: gpu {g} != model {w}"
    assert st["misses"] == model.misses and st["hits"] == model.hits
    assert st["evictions"] == model.evictions and st["wasted_pages"] == model.wasted_pages
    assert st["fetched_pages"] == model.fetched_pages


def test_c1_full_parity(data_dir, cuda):
    wl = configs.c1()
    path = configs.ensure_file(wl.file, data_dir)
    exp_out, exp_deliv = expected(wl, path)
    for ra in (0, 16):
        _say(f"c1 ra_pages={ra}")
        cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra * wl.page_size, timeout_s=30)
        with gfs.PageCache(cfg) as cache:
            fid = cache.open(path)
            res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
            st = cache.stats()
            # warm re-run: every page is cached now (file fits), all hits
            res2 = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
            st2 = cache.stats()
        np.testing.assert_array_equal(res.out, exp_out)
        np.testing.assert_array_equal(res.status, exp_deliv)
        np.testing.assert_array_equal(res2.out, exp_out)
        assert st["evictions"] == 0 and st["fetched_pages"] == 1024    # closed form (i)
        assert st2["misses"] == st["misses"] and st2["fetched_pages"] == 1024


def test_gopen_path_and_errors(data_dir, cuda):
    wl = configs.c1_small()
    path = configs.ensure_file(wl.file, data_dir)
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, timeout_s=20)
    with gfs.PageCache(cfg) as cache:
        with pytest.raises(OSError):
            cache.open(path, flags=1)                 # only read-only opens
        with pytest.raises(OSError):
            cache.open(os.path.join(data_dir, "does_not_exist.bin"))
        fid = cache.open(path)
        # odd, unaligned offsets and a read that crosses EOF
        size = wl.file.size
        offs = np.array([[1, 65535 + 7, size - 100], [size, size + 12345, 3]], dtype=np.uint64)
        _say("unaligned reads")
        res = runner.run_list(cache, fid, offs, 4096 + 16, configs.CONSUMER_CHECKSUM)
        from oracle import data as odata
        for b in range(2):
            want = sum(odata.checksum_of(odata.delivered(path, int(o), 4096 + 16)) for o in offs[b]) & ((1 << 64) - 1)
            assert int(res.out[b]) == want
        cache.close_file(fid)
        with pytest.raises(OSError):
            cache.close_file(fid)


def test_tiny_cache_many_blocks_progress(data_dir, cuda):
    # 64 frames, 256 blocks each pinning a page: allocation must back off and still finish
    wl = configs.c3_small("b")
    path = configs.ensure_file(wl.file, data_dir)
    offs = configs.strided_offsets(256, 4, 64 << 10) % np.uint64(wl.file.size)
    _say("tiny cache, 256 blocks")
    cfg = runner.make_config(wl.page_size, 64 * wl.page_size, ra_cap_bytes=4 * wl.page_size, timeout_s=30)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        res = runner.run_list(cache, fid, offs, 64 << 10, configs.CONSUMER_CHECKSUM)
        st = cache.stats()
    from oracle import data as odata
    want = odata.block_checksums(path, offs, 64 << 10)
    np.testing.assert_array_equal(res.out, want)
    assert st["timeouts"] == 0


def test_reset_gives_cold_cache(data_dir, cuda):
    wl = configs.c2_small()
    path = configs.ensure_file(wl.file, data_dir)
    exp_out, _ = expected(wl, path)
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=16 * wl.page_size, timeout_s=20)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        for i in range(3):
            _say(f"reset round {i}")
            res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
            st = cache.stats()
            np.testing.assert_array_equal(res.out, exp_out)
            assert st["delivered_bytes"] == wl.delivered_bytes
            cache.reset()
            assert cache.stats()["misses"] == 0


@pytest.mark.parametrize("shift", [0, 40, 4096 + 12])
def test_multipage_reads_batched_hits(shift, data_dir, cuda):
    """Reads spanning many small pages (4 KiB pages, 96 KiB reads, some at offsets that are
    not page- or 16-byte-aligned): a cold pass mixes misses, joins and hits, a warm pass is
    all hits taken by the batched pass; both equal the oracle, and so does a pass with the
    policy trace on (one page at a time)."""
    from workloads.configs import Workload, FileSpec, strided_offsets, CONSUMER_CHECKSUM
    f = FileSpec("mp_seed21_6MiB.bin", 21, (6 << 20) + 1234)
    offs = strided_offsets(32, 2, 96 << 10) + shift
    wl = Workload("mp", f, 4 << 10, 2 << 20, 32, 256, 96 << 10, offs, CONSUMER_CHECKSUM)
    path = configs.ensure_file(wl.file, data_dir)
    exp_out, exp_deliv = expected(wl, path)
    for trace in (0, 1):
        cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=64 << 10, trace_level=trace,
                                 trace_capacity=(1 << 18) if trace else 0, timeout_s=20)
        with gfs.PageCache(cfg) as cache:
            fid = cache.open(path)
            cold = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
            warm = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
            st = cache.stats()
        for res in (cold, warm):
            np.testing.assert_array_equal(res.status, exp_deliv)
            np.testing.assert_array_equal(res.out, exp_out)
        assert st["timeouts"] == 0 and st["io_errors"] == 0
        assert st["hits"] > 0


@pytest.mark.parametrize("ra_pages", [0, 16])
def test_file_shrunk_under_the_cache_reports_eio(ra_pages, data_dir, cuda, tmp_path):
    """Failure handling forced from the host: a registered 4 MiB file is cut to 3 MiB + 100 B
    on disk, so the host reads of the pages past that point come back short. Blocks that read
    only below the cut get the right bytes; blocks that reach past it get -EIO (no hang, no
    wrong bytes); the cache is usable again after a reset."""
    import shutil
    from oracle import data as odata
    src = configs.ensure_file(configs.FileSpec("shrink_seed31_4MiB.bin", 31, 4 << 20), data_dir)
    path = str(tmp_path / "shrinking.bin")
    shutil.copyfile(src, path)
    page = 64 << 10
    offs = (np.arange(16 * 4, dtype=np.uint64) * np.uint64(page)).reshape(16, 4)   # block b: pages 4b..4b+3
    cfg = runner.make_config(page, 16 << 20, ra_cap_bytes=ra_pages * page, timeout_s=20)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        os.truncate(path, (3 << 20) + 100)
        _say(f"shrunk file, ra_pages={ra_pages}")
        res = runner.run_list(cache, fid, offs, page, configs.CONSUMER_CHECKSUM)
        st = cache.stats()
        assert st["io_errors"] > 0 and st["timeouts"] == 0
        for b in range(12):                                   # pages 0..47: below the cut
            assert int(res.status[b]) == 4 * page, b
            want = sum(odata.checksum_of(odata.delivered(src, int(o), page)) for o in offs[b]) & ((1 << 64) - 1)
            assert int(res.out[b]) == want, b
        for b in range(12, 16):                               # page 48 holds the cut
            assert int(res.status[b]) == -5, (b, int(res.status[b]))
        cache.close_file(fid)
        cache.reset()
        fid2 = cache.open(src)
        res2 = runner.run_list(cache, fid2, offs, page, configs.CONSUMER_CHECKSUM)
        want2 = odata.block_checksums(src, offs, page)
        np.testing.assert_array_equal(res2.out, want2)
        assert cache.stats()["io_errors"] == 0


@pytest.mark.parametrize("name", ["c2_small", "c3c_small"])
def test_partitioned_host_queue(name, data_dir, cuda):
    """GPUfs's partitioned request queue (a block posts into the slot of its block id, each
    host thread serves its own range of slots) delivers the same bytes."""
    wl = configs.get(name)
    path = configs.ensure_file(wl.file, data_dir)
    exp_out, exp_deliv = expected(wl, path)
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=8 * wl.page_size, host_threads=4,
                             rpc_slots=16, timeout_s=20)
    cfg.io_backend = gfs.GFS_IO_PREAD_PARTITIONED
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
        st = cache.stats()
    np.testing.assert_array_equal(res.status, exp_deliv)
    np.testing.assert_array_equal(res.out, exp_out)
    assert sum(st["host_thread_requests"]) == st["requests"]
