"""GPU parity of the serving loop: every request's checksum equals the oracle's checksum of
its file, alone or in the mix; the records obey the admission rule (arrival order, budget);
time stamps are ordered; a zero-byte file and repeated files are served; an unregistered
file is refused before anything runs."""
import errno
import os

import numpy as np
import pytest

from oracle import data as odata
from oracle import serve as oserve
from paper_2109_05366_amd import gfs, runner
from workloads import configs, manifest

pytestmark = pytest.mark.gpu

PAGE = 64 << 10


@pytest.fixture(scope="module")
def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gfs.lib()
    return torch


@pytest.fixture(scope="module")
def pool(data_dir):
    m = manifest.load("serve_small")
    paths = [configs.ensure_file(configs.FileSpec(f["name"], f["seed"], f["size"]), data_dir) for f in m["files"]]
    want = np.array([odata.file_checksum(p) for p in paths], dtype=np.uint64)
    return m, paths, want


def _cache(budget, ra_cap=4 << 20, page=PAGE):
    cfg = runner.make_config(page, max(budget // page * page, 64 * page), ra_cap_bytes=ra_cap, rpc_slots=16,
                             timeout_s=60)
    return gfs.PageCache(cfg)


def _check_records(recs, sizes, files, want, budget, page):
    assert np.all(recs["result"] == np.asarray(sizes, dtype=np.int64)[files]), recs["result"]
    np.testing.assert_array_equal(recs["csum"], want[files])
    reserved = [oserve.reservation(int(sizes[f]), page) for f in files]
    assert list(recs["reserved"]) == reserved
    oserve.check_admission(recs["arrival_ns"], recs["admit_ns"], recs["done_ns"], recs["seq"], recs["reserved"],
                           budget)
    # the first page lands between admission and completion (device clock mapped to the host's)
    slack = 200_000
    assert np.all(recs["first_ns"].astype(np.int64) + slack >= recs["admit_ns"].astype(np.int64))
    assert np.all(recs["first_ns"] <= recs["done_ns"] + slack)


@pytest.mark.parametrize("chunk", [256 << 10, 1 << 20])
def test_serve_small_mix(pool, cuda, chunk):
    m, paths, want = pool
    sizes = [f["size"] for f in m["files"]]
    files = np.array([r["file"] for r in m["requests"]])
    arrivals = [r["t_ns"] for r in m["requests"]]
    budget = m["budget_bytes"]
    print(f"[gpu] serve_small chunk={chunk} n={len(files)}", flush=True)
    with _cache(budget) as cache:
        ids = [cache.open(p) for p in paths]
        recs, summ = runner.serve(cache, [ids[f] for f in files], arrivals, budget, chunk_bytes=chunk)
        st = cache.stats()
    print(f"[gpu] summary {summ} latency {runner.latency_ms(recs)}", flush=True)
    assert st["timeouts"] == 0 and st["io_errors"] == 0
    _check_records(recs, sizes, files, want, budget, PAGE)
    assert summ["delivered_bytes"] == int(np.asarray(sizes)[files].sum())
    assert summ["peak_reserved"] <= max(budget, max(sizes) + PAGE)
    assert st["evictions"] > 0          # the pool is four times the cache


def test_alone_equals_mix(pool, cuda):
    m, paths, want = pool
    files = np.array([r["file"] for r in m["requests"]])
    arrivals = [r["t_ns"] for r in m["requests"]]
    budget = m["budget_bytes"]
    with _cache(budget) as cache:
        ids = [cache.open(p) for p in paths]
        mix, _ = runner.serve(cache, [ids[f] for f in files], arrivals, budget)
        for j in (0, 7, len(files) - 1):
            cache.reset()
            alone, _ = runner.serve(cache, [ids[files[j]]], [0], budget)
            assert int(alone["csum"][0]) == int(mix["csum"][j]) == int(want[files[j]]), j
            assert alone["result"][0] == mix["result"][j]


def test_zero_byte_and_repeated_files(pool, cuda, data_dir):
    m, paths, want = pool
    empty = os.path.join(data_dir, "serve_empty.bin")
    open(empty, "wb").close()
    budget = 64 << 20
    with _cache(budget) as cache:
        ids = [cache.open(p) for p in paths[:3]]
        eid = cache.open(empty)
        seq = [ids[0], eid, ids[0], ids[1], eid, ids[1], ids[2], ids[0]]
        recs, summ = runner.serve(cache, seq, [0] * len(seq), budget)
        st = cache.stats()
    exp = {ids[0]: int(want[0]), ids[1]: int(want[1]), ids[2]: int(want[2]), eid: 0}
    assert [int(c) for c in recs["csum"]] == [exp[i] for i in seq]
    assert recs["result"][1] == 0 and recs["result"][4] == 0
    assert st["hits"] > 0               # repeats are served from the cache


def test_unregistered_file_is_refused(cuda):
    with _cache(64 << 20) as cache:
        with pytest.raises(OSError) as ei:
            runner.serve(cache, [5], [0], 64 << 20)
        assert ei.value.errno == errno.EBADF


def test_full_serve_sample(data_dir, cuda):
    """The first 120 requests of the serving workload at its full size (pool, budget, page
    size); every request's checksum equals the oracle's checksum of its file."""
    m = manifest.load("serve")
    paths = [configs.ensure_file(configs.FileSpec(f["name"], f["seed"], f["size"]), data_dir) for f in m["files"]]
    sizes = [f["size"] for f in m["files"]]
    files = np.array([r["file"] for r in m["requests"]])[:120]
    arrivals = [r["t_ns"] for r in m["requests"]][:120]
    budget = m["budget_bytes"]
    page = 256 << 10
    print(f"[gpu] serve full: {len(files)} requests, budget {budget >> 30} GiB", flush=True)
    with _cache(budget, ra_cap=16 << 20, page=page) as cache:
        ids = [cache.open(p) for p in paths]
        recs, summ = runner.serve(cache, [ids[f] for f in files], arrivals, budget)
        st = cache.stats()
    print(f"[gpu] serve full: {summ['delivered_bytes'] / summ['span_ns']:.2f} GB/s {runner.latency_ms(recs)}",
          flush=True)
    assert st["timeouts"] == 0 and st["io_errors"] == 0
    assert np.all(recs["result"] == np.asarray(sizes, dtype=np.int64)[files])
    oserve.check_admission(recs["arrival_ns"], recs["admit_ns"], recs["done_ns"], recs["seq"], recs["reserved"],
                           budget)
    # the oracle's checksum of every file the requests read (threads: pread and numpy's sums
    # release the interpreter lock)
    from concurrent.futures import ThreadPoolExecutor
    used = sorted(set(files.tolist()))
    with ThreadPoolExecutor(8) as ex:
        want = dict(zip(used, ex.map(lambda f: odata.file_checksum(paths[f]), used)))
    for i, f in enumerate(files.tolist()):
        assert int(recs["csum"][i]) == want[f], (f, i)
