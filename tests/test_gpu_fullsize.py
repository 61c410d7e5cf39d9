"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

Outputs are checked on sampled blocks against the oracle's pread-based values (each
block one by one), every block against properties that hold at any size (delivered bytes,
histogram totals), and the concurrent policy trace of the C2 stream is replayed against
the model's rules (oracle.replay): frame histories in hand-ticket order, eviction victims,
readahead windows, request runs.
"""
import numpy as np
import pytest

from oracle import replay
from paper_2109_05366_amd import gfs, runner
from workloads import configs

from gpu_util import decode_replay, expected

pytestmark = pytest.mark.gpu

RA_CAP_LARGE = 16 << 20                # windows of 64 pages
HOST_THREADS = 32       # bench.py's launch configuration
IO_CHUNK = 4 << 20
RPC_SLOTS = 64


@pytest.fixture(scope="module")
def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gfs.lib()
    return torch


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _sample(blocks, n, seed):
    rng = np.random.default_rng(seed)
    return sorted(set(int(x) for x in rng.integers(0, blocks, size=n)) | {0, blocks - 1})


@pytest.mark.parametrize("ra_cap", ["bench", RA_CAP_LARGE, 0])
def test_c2_full_size_parity_and_trace_replay(ra_cap, data_dir, cuda):
    wl = configs.c2()
    if ra_cap == "bench":
        ra_cap = wl.ra_cap_bytes          # the cap bench.py runs this workload with
    path = configs.ensure_file(wl.file, data_dir)
    _say(f"c2 full size, ra cap {ra_cap >> 20} MiB")
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_cap, host_threads=HOST_THREADS,
                             rpc_slots=RPC_SLOTS, trace_level=1, trace_capacity=1 << 21, timeout_s=60,
                             io_chunk_bytes=IO_CHUNK)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer, threads=wl.threads)
        st = cache.stats()
        ev = cache.trace()
    assert st["timeouts"] == 0 and st["io_errors"] == 0
    per_block = wl.reads_per_block * wl.read_size
    np.testing.assert_array_equal(res.status, np.full(wl.blocks, per_block))
    np.testing.assert_array_equal(res.out.sum(axis=1, dtype=np.uint64), np.full(wl.blocks, per_block))
    sample = _sample(wl.blocks, 10, 7)
    want, _ = expected(wl, path, blocks=sample)
    np.testing.assert_array_equal(res.out[sample], want[sample])
    # policy: replay the concurrent trace against the rules
    assert st["trace_events"] == len(ev) < (1 << 21)
    C = wl.cache_bytes // wl.page_size
    N = wl.file.size // wl.page_size
    tr = decode_replay(ev)
    rc = replay.replay_clock(tr, C)
    assert rc["allocations"] == st["fetched_pages"] >= N
    assert len(rc["evictions"]) == st["evictions"] == st["fetched_pages"] - C
    assert rc["wasted_pages"] == st["wasted_pages"]
    ra_pages = ra_cap // wl.page_size
    rr = replay.replay_readahead(tr, min(4, ra_pages) if ra_pages else 4, ra_pages, 8,
                                 {fid: wl.file.size}, wl.page_size)
    assert rr["exact"] + rr["shape_only"] == st["misses"]
    assert replay.replay_requests(tr) == st["requests"]
    _say(f"c2 replay ok: {st['misses']} misses ({rr['exact']} windows exact), "
         f"{len(rc['evictions'])} evictions, {st['fetched_pages']} pages fetched")


@pytest.mark.parametrize("ra_cap", ["bench", 0])
@pytest.mark.parametrize("pattern", ["a", "b", "c"])
def test_c3_full_size_parity(pattern, ra_cap, data_dir, cuda):
    wl = configs.c3(pattern)
    if ra_cap == "bench":
        ra_cap = wl.ra_cap_bytes
    path = configs.ensure_file(wl.file, data_dir)
    _say(f"c3{pattern} full size, ra cap {ra_cap >> 20} MiB")
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_cap, host_threads=HOST_THREADS,
                             rpc_slots=RPC_SLOTS, timeout_s=90, io_chunk_bytes=IO_CHUNK)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer, threads=wl.threads)
        st = cache.stats()
    assert st["timeouts"] == 0 and st["io_errors"] == 0
    np.testing.assert_array_equal(res.status, np.full(wl.blocks, wl.reads_per_block * wl.read_size))
    sample = _sample(wl.blocks, 6 if pattern == "c" else 24, 11)
    want, _ = expected(wl, path, blocks=sample)
    np.testing.assert_array_equal(res.out[sample], want[sample])
    C = wl.cache_bytes // wl.page_size
    assert st["fetched_pages"] == st["misses"] + st["ra_pages"]
    assert st["evictions"] == max(0, st["fetched_pages"] - C)
    assert st["delivered_bytes"] == wl.delivered_bytes
