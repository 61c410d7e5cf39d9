"""GPU parity: the HIP page cache (through the C-ABI) against the CPU oracle.

Data parity is bit-exact (integers): every block's checksum or histogram and its
delivered byte count equal the oracle's pread-based values. Policy parity: in
serialized mode (test-only gate, one read at a time in (round, block) order) the
device trace equals the oracle model's predicted event sequence exactly.
"""
import os

import numpy as np
import pytest

from oracle.policy import PolicyModel, quota_cap, run_serialized
from paper_2109_05366_amd import gfs, runner
from workloads import configs

from golden import make_golden
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


@pytest.mark.parametrize("name,ra_pages,depth", [("c2_small", 16, 8), ("c3a_small", 16, 4), ("c3c_small", 0, 2)])
def test_io_uring_backend_parity(name, ra_pages, depth, data_dir, cuda):
    """The io_uring host backend (several reads in flight per host thread) delivers the same
    bytes as the pread one."""
    wl = configs.get(name)
    path = configs.ensure_file(wl.file, data_dir)
    exp_out, exp_deliv = expected(wl, path)
    _say(f"io_uring {name} ra_pages={ra_pages} depth={depth}")
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_pages * wl.page_size, timeout_s=20,
                             host_threads=2, io_backend=gfs.GFS_IO_URING, io_depth=depth,
                             io_chunk_bytes=256 << 10)
    try:
        cache = gfs.PageCache(cfg)
    except OSError as e:
        if e.errno == 38:   # ENOSYS: the box's kernel refuses io_uring
            pytest.skip("io_uring unavailable")
        raise
    with cache:
        fid = cache.open(path)
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
        st = cache.stats()
    assert st["timeouts"] == 0 and st["io_errors"] == 0, st
    np.testing.assert_array_equal(res.status, exp_deliv)
    np.testing.assert_array_equal(res.out, exp_out)
    assert st["host_bytes"] == st["request_bytes"] and st["host_requests"] == st["requests"]


DEFAULT_DET = (64, 64, 3)


@pytest.mark.parametrize("name,ra_pages,det,quota", [
    ("c2_small", 0, DEFAULT_DET, 1), ("c2_small", 16, DEFAULT_DET, 1), ("c3c_small", 0, DEFAULT_DET, 1),
    ("c3c_small", 8, DEFAULT_DET, 1), ("c1_small", 8, DEFAULT_DET, 1), ("c3a_small", 16, DEFAULT_DET, 1),
    ("c3b_small", 4, DEFAULT_DET, 1),
    # other detector constants: aggregate rule off (the context rule decides), and a short
    # memory with a small radius
    ("c3a_small", 16, (64, 64, 65), 1), ("c3c_small", 8, (16, 8, 2), 1), ("c2_small", 16, (8, 4, 2), 1),
    # the thrash guard: windows clipped to the cache's share per resident block
    ("c2_small", 16, DEFAULT_DET, 16), ("c3b_small", 8, DEFAULT_DET, 16),
])
def test_serialized_trace_matches_model(name, ra_pages, det, quota, data_dir, cuda):
    wl = configs.get(name)
    path = configs.ensure_file(wl.file, data_dir)
    _say(f"serialized {name} ra_pages={ra_pages} detector={det} quota={quota}")
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_pages * wl.page_size,
                             ra_init_pages=4, streams=8, trace_level=2, trace_capacity=1 << 20,
                             timeout_s=20, detector=det, quota_blocks=quota)
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
    cap = quota_cap(ra_pages, C, wl.blocks, quota) if ra_pages else 0
    model = PolicyModel(C, wl.page_size, ra_init_pages=min(4, cap) if cap else 4,
                        ra_cap_pages=cap, streams_per_file=8, recent=det[0], near_pages=det[1], near_min=det[2])
    model.open(fid, wl.file.size)
    run_serialized(model, fid, wl.offsets, wl.read_size)
    _compare_traces(ev, model, st)


@pytest.mark.parametrize("pattern,ra_pages,det", [
    ("strided", 16, DEFAULT_DET), ("random", 16, DEFAULT_DET), ("random", 16, (64, 64, 65)),
    ("random", 8, (8, 4, 2)),
])
def test_multipage_serialized_trace_matches_model(pattern, ra_pages, det, data_dir, cuda):
    """Reads of 8 pages of 4 KiB (32 KiB, unaligned to the read size in the random pattern,
    some past the end of the file): a window opened by a new stream or by the context rule
    covers at least the rest of the read that missed, on the device as in the model, miss
    for miss, hand visit for hand visit."""
    import dataclasses
    wl = configs.get("f3_small")
    if pattern == "random":
        wl = dataclasses.replace(wl, offsets=configs.random_page_offsets(wl.blocks, wl.blocks * 13, 10, 4096, 777))
    path = configs.ensure_file(wl.file, data_dir)
    _say(f"serialized multi-page {pattern} ra_pages={ra_pages} detector={det}")
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_pages * wl.page_size,
                             ra_init_pages=4, streams=8, trace_level=2, trace_capacity=1 << 20,
                             timeout_s=20, detector=det, quota_blocks=1)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer, serialize=True)
        st = cache.stats()
        ev = cache.trace()
    exp_out, exp_deliv = expected(wl, path)
    np.testing.assert_array_equal(res.status, exp_deliv)
    np.testing.assert_array_equal(res.out, exp_out)
    C = wl.cache_bytes // wl.page_size
    model = PolicyModel(C, wl.page_size, ra_init_pages=4, ra_cap_pages=ra_pages, streams_per_file=8,
                        recent=det[0], near_pages=det[1], near_min=det[2])
    model.open(fid, wl.file.size)
    run_serialized(model, fid, wl.offsets, wl.read_size)
    _compare_traces(ev, model, st)
    # the device logged each miss's read length (pages from the missed page on)
    reqs = [int(r["b"]) >> 32 for r in ev if int(r["op"]) == gfs.EV_MISS]
    assert max(reqs) > 1


@pytest.mark.parametrize("name,ra_pages", [
    ("c1_small", 8), ("c3a_small", 16), ("c3b_small", 8), ("c2_small", 16), ("c3c_small", 8),
])
def test_async_serialized_trace_matches_model(name, ra_pages, data_dir, cuda):
    """Asynchronous (marker-triggered) readahead, one access at a time: every marker taken,
    every window the stream advances to, and the rest of the trace equal the model's."""
    wl = configs.get(name)
    path = configs.ensure_file(wl.file, data_dir)
    _say(f"serialized async {name} ra_pages={ra_pages}")
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_pages * wl.page_size,
                             ra_init_pages=4, streams=8, trace_level=2, trace_capacity=1 << 20,
                             timeout_s=20, quota_blocks=1, ra_async=1)
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
    model = PolicyModel(C, wl.page_size, ra_init_pages=min(4, ra_pages), ra_cap_pages=ra_pages,
                        streams_per_file=8, ra_async=True)
    model.open(fid, wl.file.size)
    run_serialized(model, fid, wl.offsets, wl.read_size)
    _compare_traces(ev, model, st)
    assert st["ra_async_windows"] == model.advances
    assert st["joins"] == model.joins


@pytest.mark.parametrize("name,ra_pages", [("c2_small", 16), ("c3a_small", 16), ("c3b_small", 8),
                                           ("c3c_small", 8), ("c1_small", 8)])
def test_async_readahead_data(name, ra_pages, data_dir, cuda):
    """Asynchronous readahead with every block running at once: the delivered data equal the
    oracle's, windows were issued at markers, and every block finished its last one."""
    wl = configs.get(name)
    path = configs.ensure_file(wl.file, data_dir)
    exp_out, exp_deliv = expected(wl, path)
    _say(f"async data {name} ra_pages={ra_pages}")
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_pages * wl.page_size, timeout_s=20,
                             ra_async=1)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        for rep in range(2):   # cold, then with whatever the first pass left cached
            res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
            st = cache.stats()
            assert st["timeouts"] == 0 and st["io_errors"] == 0, st
            np.testing.assert_array_equal(res.status, exp_deliv)
            np.testing.assert_array_equal(res.out, exp_out)
        # every request was read by the host and every frame published: nothing is left filling
        assert st["host_requests"] == st["requests"]
    if name in ("c3a_small", "c1_small"):
        assert st["ra_async_windows"] > 0


def _compare_traces(ev, model, st):
    """The device trace equals the model's event sequence (hand visits with what they found),
    and every miss logged the model's detector inputs and rule."""
    got = canon(decode(ev))
    want = canon(model.events)
    assert len(got) == len(want)
    for i, (g, w) in enumerate(zip(got, want)):
        assert g == w, f"event {i}: gpu {g} != model {w}"
    packed = [int(r["frame"]) for r in ev if int(r["op"]) == gfs.EV_MISS]
    dec = [(x & 0xFF, (x >> 8) & 0xFFFF, x >> 24) for x in packed]
    assert dec == model.decisions
    assert st["misses"] == model.misses and st["hits"] == model.hits
    assert st["evictions"] == model.evictions and st["wasted_pages"] == model.wasted_pages
    assert st["fetched_pages"] == model.fetched_pages


@pytest.mark.parametrize("name,advice", [("c3b_small", "random"), ("c3c_small", "sequential"),
                                         ("c3c_small", "random"), ("c3a_small", "sequential")])
def test_fadvise_serialized_trace_matches_model(name, advice, data_dir, cuda):
    """gfs_fadvise (Sec. 4.1: a posix_fadvise-style hint switches prefetching off): RANDOM turns readahead off for
    the file (every miss fetches its page alone), SEQUENTIAL opens every new stream with the
    initial window; the device trace equals the model run with the same advice."""
    from oracle.policy import ADV_RANDOM, ADV_SEQUENTIAL
    wl = configs.get(name)
    path = configs.ensure_file(wl.file, data_dir)
    ra_pages = 8
    _say(f"fadvise {advice} {name}")
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_pages * wl.page_size,
                             trace_level=2, trace_capacity=1 << 20, timeout_s=20, quota_blocks=1)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        cache.fadvise(fid, gfs.GFS_ADV_RANDOM if advice == "random" else gfs.GFS_ADV_SEQUENTIAL)
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer, serialize=True)
        st = cache.stats()
        ev = cache.trace()
    exp_out, exp_deliv = expected(wl, path)
    np.testing.assert_array_equal(res.status, exp_deliv)
    np.testing.assert_array_equal(res.out, exp_out)
    C = wl.cache_bytes // wl.page_size
    model = PolicyModel(C, wl.page_size, ra_init_pages=4, ra_cap_pages=ra_pages, streams_per_file=8)
    model.open(fid, wl.file.size, advice=ADV_RANDOM if advice == "random" else ADV_SEQUENTIAL)
    run_serialized(model, fid, wl.offsets, wl.read_size)
    _compare_traces(ev, model, st)
    if advice == "random":
        assert st["ra_pages"] == 0 and st["misses"] == st["fetched_pages"]


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
        # the stored golden values (tests/golden/, pinned on the CPU)
        golden, total = make_golden.load_c1()
        assert [int(x) for x in res.out] == golden
        assert int(res.out.sum(dtype=np.uint64)) == total


def test_host_open_errors_and_unaligned_reads(data_dir, cuda):
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


def _probe_lib():
    import ctypes
    from paper_2109_05366_amd import build as b
    if not os.path.exists(b.PROBE_LIB):
        raise RuntimeError(f"{b.PROBE_LIB} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(b.PROBE_LIB)
    vp = ctypes.c_void_p
    L.gfs_test_api_probe.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_uint32, vp, vp, vp]
    L.gfs_test_api_probe.restype = ctypes.c_int
    return L


@pytest.mark.parametrize("threads", [256, 64, 96])
def test_device_gopen_by_path_and_error_returns(threads, data_dir, cuda):
    """A user kernel opens a registered file by path with gopen (Sec. 2.2), reads through the
    descriptor and closes it; the device-side error returns are the documented ones: -EROFS
    for a non-read-only open (prefetching only for read-only files, Sec. 4), -ENOENT for a
    path or id that is not registered, -EBADF for a bad descriptor in gread and gclose, 0 at
    the end of the file, and -EINVAL from gread in a block whose size is not a multiple of
    64 threads."""
    torch = cuda
    from oracle import data as odata
    wl = configs.c1_small()
    path = configs.ensure_file(wl.file, data_dir)
    L = _probe_lib()
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, timeout_s=20)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        other = configs.ensure_file(configs.FileSpec("probe_other_seed5.bin", 5, 1 << 20), data_dir)
        fid2 = cache.open(other)
        cache.close_file(fid2)                         # id fid2: below max_files, not registered
        p_dev = torch.tensor(list(path.encode()) + [0], dtype=torch.uint8, device="cuda")
        m_dev = torch.tensor(list((path + ".missing").encode()) + [0], dtype=torch.uint8, device="cuda")
        off, size = 3 * (64 << 10) + 40, (100 << 10) + 16
        buf = torch.zeros(size + 64, dtype=torch.uint8, device="cuda")
        out = torch.full((10,), -999, dtype=torch.int64, device="cuda")
        _say(f"api probe, {threads} threads")
        rc = L.gfs_test_api_probe(cache.handle, p_dev.data_ptr(), m_dev.data_ptr(), fid2, off, size, wl.file.size,
                                  threads, buf.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        assert rc == 0
        torch.cuda.synchronize()
        o = out.cpu().tolist()
        st = cache.stats()
    assert o[0] == fid
    assert o[1] == -30 and o[2] == -2                  # -EROFS, -ENOENT
    assert o[7] == -9 and o[8] == 0 and o[9] == -2     # gclose(bad) -EBADF, gclose ok, gopen_id -ENOENT
    if threads % 64:
        assert o[3] == -9 and o[4] == -9               # descriptors are checked first
        assert o[5] == -22 and o[6] == -22             # -EINVAL: not a multiple of 64 threads
    else:
        assert o[3] == -9 and o[4] == -9               # -EBADF
        assert o[5] == size and o[6] == 0
        assert bytes(buf[:size].cpu().numpy()) == odata.delivered(path, off, size)
        assert st["timeouts"] == 0 and st["io_errors"] == 0


def test_close_drops_pages_before_the_id_is_reused(data_dir, cuda):
    """gfs_close drops the file's cached pages: a different file opened next gets the same id,
    and reading it without a cache reset returns its own bytes, not the closed file's."""
    from oracle import data as odata
    a = configs.c1_small()
    b_spec = configs.FileSpec("reuse_seed23.bin", 23, a.file.size)
    pa = configs.ensure_file(a.file, data_dir)
    pb = configs.ensure_file(b_spec, data_dir)
    want_a = odata.block_checksums(pa, a.offsets, a.read_size)
    want_b = odata.block_checksums(pb, a.offsets, a.read_size)
    assert not np.array_equal(want_a, want_b)
    for ra in (0, 8):
        cfg = runner.make_config(a.page_size, a.cache_bytes, ra_cap_bytes=ra * a.page_size, timeout_s=20)
        with gfs.PageCache(cfg) as cache:
            fa = cache.open(pa)
            _say(f"reuse: read A, ra={ra}")
            np.testing.assert_array_equal(runner.run_list(cache, fa, a.offsets, a.read_size, a.consumer).out, want_a)
            np.testing.assert_array_equal(runner.run_list(cache, fa, a.offsets, a.read_size, a.consumer).out, want_a)
            s0 = cache.stats()
            cache.close_file(fa)
            fb = cache.open(pb)
            assert fb == fa                            # the id is reused
            _say("reuse: read B under the same id, no reset")
            res = runner.run_list(cache, fb, a.offsets, a.read_size, a.consumer)
            s1 = cache.stats()
            np.testing.assert_array_equal(res.out, want_b)
            assert s1["fetched_pages"] - s0["fetched_pages"] == s0["fetched_pages"]   # all of B fetched
            # and the first file, opened again (another id now), reads right too
            fa2 = cache.open(pa)
            np.testing.assert_array_equal(runner.run_list(cache, fa2, a.offsets, a.read_size, a.consumer).out,
                                          want_a)


def test_wait_timeout_gives_etimedout_and_every_block_exits(data_dir, cuda):
    """Failure handling forced from the host: a 2 us device wait limit is far below a host
    read, so blocks give up with -ETIMEDOUT (the kernel's own bounded waits; every block
    returns) and no block delivers wrong bytes; after a reset the cache serves the same reads
    correctly with the default limit."""
    wl = configs.c2_small()
    path = configs.ensure_file(wl.file, data_dir)
    exp_out, exp_deliv = expected(wl, path)
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=8 * wl.page_size, timeout_ns=2000)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        _say("2 us wait limit")
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
        st = cache.stats()
        timed_out = res.status == -110
        assert timed_out.any() and st["timeouts"] > 0
        ok = ~timed_out
        np.testing.assert_array_equal(res.status[ok], exp_deliv[ok])
        np.testing.assert_array_equal(res.out[ok], exp_out[ok])
        assert set(res.status[timed_out].tolist()) == {-110}
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=8 * wl.page_size, timeout_s=20)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
        st = cache.stats()
    assert st["timeouts"] == 0
    np.testing.assert_array_equal(res.out, exp_out)


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


@pytest.mark.parametrize("name", ["c1_small", "c2_small"])
def test_buffer_reader_matches_oracle(name, data_dir, cuda):
    """The CPU-I/O comparator's kernel (the same reads and consumers over a device copy of the
    file) gives the oracle's outputs, including reads at and past the end of the file and an
    unaligned read."""
    torch = cuda
    wl = configs.get(name)
    path = configs.ensure_file(wl.file, data_dir)
    offs = wl.offsets.copy()
    offs[0, 0] += np.uint64(3)                          # an unaligned read
    exp_out = (odata_mod().block_checksums if wl.consumer == 0 else odata_mod().block_histograms)(
        path, offs, wl.read_size)
    with open(path, "rb") as fh:
        raw = np.frombuffer(fh.read(), dtype=np.uint8)
    data = torch.from_numpy(raw.copy()).to("cuda")
    o_dev = torch.from_numpy(offs.view(np.int64)).to("cuda")
    out = torch.zeros(wl.blocks * (1 if wl.consumer == 0 else 256), dtype=torch.int64 if wl.consumer == 0
                      else torch.int32, device="cuda")
    status = torch.zeros(wl.blocks, dtype=torch.int64, device="cuda")
    gfs.gfs_launch_buffer_reader(data.data_ptr(), len(raw), o_dev.data_ptr(), wl.blocks, wl.reads_per_block,
                                 wl.read_size, 256, wl.consumer, out.data_ptr(), status.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    got = got.view(np.uint64) if wl.consumer == 0 else got.view(np.uint32).reshape(wl.blocks, 256)
    np.testing.assert_array_equal(got, exp_out)


@pytest.mark.parametrize("ra_pages", [0, 16])
def test_reads_only_consumer_leaves_each_blocks_last_read(ra_pages, data_dir, cuda):
    """Consumer 2 (the reads alone, as the all-hit benchmark times them): every block's buffer
    ends holding what its reads put there in order (a short read at the end of the file
    overwrites only its prefix, a read past it nothing), cold and then all hits."""
    wl = configs.get("c1_small")
    path = configs.ensure_file(wl.file, data_dir)
    _, exp_deliv = expected(wl, path)
    fill = 0xA5
    want = np.full((wl.blocks, wl.read_size), fill, dtype=np.uint8)
    for b in range(wl.blocks):
        for off in wl.offsets[b]:
            got = odata_mod().delivered(path, int(off), wl.read_size)
            want[b, :len(got)] = np.frombuffer(got, dtype=np.uint8)
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_pages * wl.page_size, timeout_s=20)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        r = runner.ListReader(wl.offsets, wl.read_size, configs.CONSUMER_NONE)
        for label in ("cold", "warm"):
            _say(f"reads only, {label}, ra_pages={ra_pages}")
            r.buf.fill_(fill)
            r.launch(cache, fid)
            res = r.result()
            np.testing.assert_array_equal(res.status, exp_deliv)
            np.testing.assert_array_equal(res.out, want)
        st = cache.stats()
    assert st["timeouts"] == 0 and st["io_errors"] == 0, st
    assert st["delivered_bytes"] == 2 * int(exp_deliv.sum())


@pytest.mark.parametrize("timers", [0, 1])
def test_page_timers_only_when_asked(timers, data_dir, cuda):
    """The per-page split of gread's time (acquire, copy-out, unpin) is measured only in a
    context created with page_timers; the data are the same either way."""
    wl = configs.get("c1_small")
    path = configs.ensure_file(wl.file, data_dir)
    exp_out, exp_deliv = expected(wl, path)
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=16 * wl.page_size, timeout_s=20,
                             page_timers=timers)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        for _ in range(2):   # cold, then all hits
            res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
            np.testing.assert_array_equal(res.status, exp_deliv)
            np.testing.assert_array_equal(res.out, exp_out)
        st = cache.stats()
    split = [st["t_acquire_ns"], st["t_copy_ns"], st["t_unpin_ns"]]
    if timers:
        assert min(split) > 0, split
    else:
        assert split == [0, 0, 0], split


def odata_mod():
    from oracle import data as odata
    return odata
