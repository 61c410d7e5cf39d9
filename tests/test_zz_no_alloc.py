"""The serving loop's entry point that allocates nothing (gfs_serve_run_noalloc) gives the
same per-request results as gfs_serve_run on the same stream, on two calls in a row through
one context, the second with fewer requests over a different part of the pool (the scratch
array and the mailbox keep the first call's contents, which the second must not see); and
it refuses runs beyond its fixed limits."""
import errno

import numpy as np
import pytest

from oracle import data as odata
from paper_2109_05366_amd import gfs, runner
from workloads import configs, manifest

pytestmark = pytest.mark.gpu

PAGE = 64 << 10
CHUNK = 64 << 10      # 512 blocks x 64 KiB of chunk buffers fit the scratch array


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


def _cache(budget):
    cfg = runner.make_config(PAGE, max(budget // PAGE * PAGE, 64 * PAGE), ra_cap_bytes=4 << 20, rpc_slots=16,
                             timeout_s=60)
    return gfs.PageCache(cfg)


def _same(a, b, sizes, files, want):
    """Both runs delivered every request whole with the oracle's checksum, and were admitted
    alike (same order and reservations)."""
    for recs in (a, b):
        np.testing.assert_array_equal(recs["result"], np.asarray(sizes, dtype=np.int64)[files])
        np.testing.assert_array_equal(recs["csum"], want[files])
    for k in ("csum", "result", "seq", "reserved"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_noalloc_matches_serve_run_twice(pool, cuda):
    m, paths, want = pool
    sizes = [f["size"] for f in m["files"]]
    files = np.array([r["file"] for r in m["requests"]])
    arrivals = np.array([r["t_ns"] for r in m["requests"]], dtype=np.uint64)
    budget = m["budget_bytes"]
    # second call: fewer requests, the pool's files in another order, arriving sooner
    files2 = files[::-1][: len(files) // 3].copy()
    arrivals2 = arrivals[: len(files2)] // 2
    with _cache(budget) as cache:
        ids = np.array([cache.open(p) for p in paths])
        for k, (fl, ar) in enumerate(((files, arrivals), (files2, arrivals2))):
            print(f"[gpu] noalloc call {k}: n={len(fl)} chunk={CHUNK}", flush=True)
            cache.reset()
            ref, _ = runner.serve(cache, ids[fl], ar, budget, chunk_bytes=CHUNK)
            cache.reset()
            got, summ = runner.serve(cache, ids[fl], ar, budget, chunk_bytes=CHUNK, noalloc=True)
            st = cache.stats()
            assert st["timeouts"] == 0 and st["io_errors"] == 0
            assert summ["delivered_bytes"] == int(np.asarray(sizes)[fl].sum())
            _same(ref, got, sizes, fl, want)


def test_noalloc_limits(pool, cuda):
    m, paths, _ = pool
    with _cache(m["budget_bytes"]) as cache:
        fid = cache.open(paths[0])
        n = gfs.GFS_SERVE_NOALLOC_MAX_REQUESTS + 1
        with pytest.raises(OSError) as e:
            runner.serve(cache, [fid] * n, np.zeros(n, dtype=np.uint64), m["budget_bytes"], chunk_bytes=CHUNK,
                         noalloc=True)
        assert e.value.errno == errno.E2BIG
        # 512 blocks x 1 MiB chunk buffers do not fit the 64 MiB array
        with pytest.raises(OSError) as e:
            runner.serve(cache, [fid], [0], m["budget_bytes"], chunk_bytes=1 << 20, grid=512, noalloc=True)
        assert e.value.errno == errno.E2BIG
