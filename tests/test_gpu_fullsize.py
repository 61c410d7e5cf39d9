"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

Every block's output is compared with the oracle's pread-based value, element by element,
and the concurrent policy trace of the C2 stream is replayed against the model's rules
(oracle.replay): frame histories in hand-ticket order, each hand visit's action against
what it found, eviction victims, every readahead window exactly (the context rule's
history is in the trace), request runs. The C2 replay runs at two settings of the detector
constants, so that the model is shown to predict the kernel at more than one setting.
"""
import numpy as np
import pytest

from oracle import replay
from oracle.policy import quota_cap
from paper_2109_05366_amd import gfs, runner
from workloads import configs

from gpu_util import decode_replay, expected

pytestmark = pytest.mark.gpu

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


_ORACLE = {}


def _oracle(wl, path):
    """Every block's expected output, computed once per workload and file."""
    key = (wl.name, path)
    if key not in _ORACLE:
        _say(f"oracle: {wl.name}, all {wl.blocks} blocks")
        _ORACLE[key] = expected(wl, path)
    return _ORACLE[key]


@pytest.mark.parametrize("setting", ["bench", "other_detector", "no_readahead"])
def test_c2_full_size_parity_and_trace_replay(setting, data_dir, cuda):
    wl = configs.c2()
    ra_cap = 0 if setting == "no_readahead" else wl.ra_cap_bytes
    det = (16, 16, 2) if setting == "other_detector" else (64, 64, 3)
    quota = 1 if setting == "other_detector" else 0       # guard off / the device's resident blocks
    path = configs.ensure_file(wl.file, data_dir)
    want, want_deliv = _oracle(wl, path)
    _say(f"c2 full size, {setting}: cap {ra_cap >> 20} MiB, detector {det}, quota {quota}")
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_cap, host_threads=HOST_THREADS,
                             rpc_slots=RPC_SLOTS, trace_level=1, trace_capacity=1 << 21, timeout_s=60,
                             io_chunk_bytes=IO_CHUNK, detector=det, quota_blocks=quota)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        resident = cache.config().ra_quota_blocks
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer, threads=wl.threads)
        st = cache.stats()
        ev = cache.trace()
    assert st["timeouts"] == 0 and st["io_errors"] == 0
    np.testing.assert_array_equal(res.status, want_deliv)
    np.testing.assert_array_equal(res.out, want)           # every block's histogram
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
    cap = quota_cap(ra_pages, C, wl.blocks, resident) if ra_pages else 0
    rr = replay.replay_readahead(tr, min(4, cap) if cap else 4, cap, 8, {fid: wl.file.size}, wl.page_size,
                                 recent=det[0], near_pages=det[1], near_min=det[2])
    assert rr["exact"] == st["misses"] and rr["shape_only"] == 0
    assert replay.replay_requests(tr) == st["requests"]
    _say(f"c2 replay ok: {st['misses']} decisions all exact {rr['by_rule']}, "
         f"{len(rc['evictions'])} evictions, {st['fetched_pages']} pages fetched, window cap {cap} pages")


@pytest.mark.parametrize("ra_cap", ["bench", 0])
@pytest.mark.parametrize("pattern", ["a", "b", "c"])
def test_c3_full_size_parity(pattern, ra_cap, data_dir, cuda):
    wl = configs.c3(pattern)
    if ra_cap == "bench":
        ra_cap = wl.ra_cap_bytes
    path = configs.ensure_file(wl.file, data_dir)
    want, want_deliv = _oracle(wl, path)
    _say(f"c3{pattern} full size, ra cap {ra_cap >> 20} MiB")
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=ra_cap, host_threads=HOST_THREADS,
                             rpc_slots=RPC_SLOTS, timeout_s=90, io_chunk_bytes=IO_CHUNK)
    with gfs.PageCache(cfg) as cache:
        fid = cache.open(path)
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer, threads=wl.threads)
        st = cache.stats()
    assert st["timeouts"] == 0 and st["io_errors"] == 0
    np.testing.assert_array_equal(res.status, want_deliv)
    np.testing.assert_array_equal(res.out, want)           # every block's checksum
    C = wl.cache_bytes // wl.page_size
    assert st["fetched_pages"] == st["misses"] + st["ra_pages"]
    assert st["evictions"] == max(0, st["fetched_pages"] - C)
    assert st["delivered_bytes"] == wl.delivered_bytes
