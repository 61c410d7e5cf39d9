"""GPU parity of the private-buffer policy (the paper's Sec. 4.1 prefetcher with Sec. 5.1
per-block replacement): delivered data equal the oracle's for every block, and in serialized
mode the device's trace (misses with their request sizes, evictions in each block's
least-recently-allocated order, allocations, private-buffer fills, host requests) and its
counters equal the model's (oracle/private.py)."""
import numpy as np
import pytest

from gpu_util import expected
from oracle.private import PrivatePolicyModel, run_serialized
from paper_2109_05366_amd import gfs, runner
from workloads import configs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gfs.lib()
    return torch


def _decode(ev):
    out = []
    for r in ev:
        op = int(r["op"])
        blk, f, p, fr, a = int(r["block"]), int(r["file"]), int(r["page"]), int(r["frame"]), int(r["a"])
        if op == 1:
            out.append(("HIT", blk, f, p, fr))
        elif op == 3:
            out.append(("MISS", blk, f, p, a))
        elif op == 4 and (a & 0xFF) == 3:
            out.append(("EVICT", blk, fr, f, p))
        elif op == 5:
            out.append(("ALLOC", blk, f, p, fr))
        elif op == 8:
            out.append(("PBHIT", blk, f, p, fr))
        elif op == 6:
            out.append(("REQ", blk, f, p, a))
        else:
            raise AssertionError(f"unexpected trace record op {op} in serialized mode")
    return out


def _config(wl, prefetch, slots, trace=False):
    return runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=prefetch * wl.page_size,
                              policy=gfs.GFS_POLICY_PRIVATE, private_slots=slots,
                              trace_level=2 if trace else 0, trace_capacity=(1 << 20) if trace else 0,
                              timeout_s=30)


@pytest.mark.parametrize("name,prefetch,slots", [
    ("c1_small", 4, 8), ("c2_small", 0, 64), ("c2_small", 3, 64), ("c3a_small", 7, 32),
    ("c3b_small", 4, 32), ("c3c_small", 2, 32),
])
def test_private_policy_data(name, prefetch, slots, data_dir, cuda):
    wl = configs.get(name)
    path = configs.ensure_file(wl.file, data_dir)
    _say(f"private {name} prefetch={prefetch} slots={slots}")
    with gfs.PageCache(_config(wl, prefetch, slots)) as cache:
        fid = cache.open(path)
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)
        st = cache.stats()
        res2 = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer)   # warm, reused slots
        st2 = cache.stats()
    exp_out, exp_deliv = expected(wl, path)
    assert st["timeouts"] == 0 and st["io_errors"] == 0
    np.testing.assert_array_equal(res.status, exp_deliv)
    np.testing.assert_array_equal(res.out, exp_out)
    np.testing.assert_array_equal(res2.out, exp_out)
    assert st["requests"] + st["private_hits"] == st["misses"]
    if prefetch == 0:
        assert st["private_hits"] == 0


@pytest.mark.parametrize("name,prefetch,slots", [
    ("c3a_small", 7, 32), ("c3a_small", 0, 32), ("c2_small", 3, 64), ("c1_small", 4, 8), ("c3c_small", 2, 32),
])
def test_private_policy_serialized_trace(name, prefetch, slots, data_dir, cuda):
    wl = configs.get(name)
    path = configs.ensure_file(wl.file, data_dir)
    _say(f"private serialized {name} prefetch={prefetch}")
    with gfs.PageCache(_config(wl, prefetch, slots, trace=True)) as cache:
        fid = cache.open(path)
        res = runner.run_list(cache, fid, wl.offsets, wl.read_size, wl.consumer, serialize=True)
        st = cache.stats()
        ev = cache.trace()
    assert st["trace_events"] == len(ev) < (1 << 20)
    exp_out, _ = expected(wl, path)
    np.testing.assert_array_equal(res.out, exp_out)
    model = PrivatePolicyModel(wl.cache_bytes // wl.page_size, wl.page_size, prefetch, slots)
    model.open(fid, wl.file.size)
    run_serialized(model, fid, wl.offsets, wl.read_size)
    got = _decode(ev)
    assert len(got) == len(model.events)
    for i, (g, w) in enumerate(zip(got, model.events)):
        assert g == w, f"event {i}: gpu {g} != model {w}"
    assert st["misses"] == model.misses and st["hits"] == model.hits
    assert st["requests"] == model.requests and st["request_bytes"] == model.request_bytes
    assert st["private_hits"] == model.pb_hits and st["evictions"] == model.evictions
    assert st["ra_pages"] == model.pb_pages and st["private_wasted"] == model.wasted
