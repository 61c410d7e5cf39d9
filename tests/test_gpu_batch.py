"""GPU parity of the batched persistent launch (many files of uneven sizes, one kernel):
per-file checksums and histograms equal the oracle's whole-file values, for several page
sizes, readahead caps and blocks-per-file settings, with a cache that holds the batch and
one that does not, and for the configuration the autotuner picks."""
import os

import numpy as np
import pytest

from oracle import data as odata
from paper_2109_05366_amd import autotune, gfs, runner
from workloads import configs, manifest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gfs.lib()
    return torch


def _files(name, data_dir):
    m = manifest.load(name)
    paths, sizes = [], []
    for f in m["files"]:
        paths.append(configs.ensure_file(configs.FileSpec(f["name"], f["seed"], f["size"]), data_dir))
        sizes.append(f["size"])
    return m, paths, sizes


@pytest.fixture(scope="module")
def small_batch(data_dir):
    m, paths, sizes = _files("batch_small", data_dir)
    want_c = np.array([odata.file_checksum(p) for p in paths], dtype=np.uint64)
    want_h = np.stack([odata.file_histogram(p) for p in paths])
    return m, paths, sizes, want_c, want_h


@pytest.mark.parametrize("cfg", [(64 << 10, 1 << 20, 1), (256 << 10, 4 << 20, 4), (2 << 20, 16 << 20, 16)])
@pytest.mark.parametrize("cache_mib", [256, 32])
def test_batch_small_parity(cfg, cache_mib, small_batch, cuda):
    m, paths, sizes, want_c, want_h = small_batch
    # the cache must hold at least 64 pages; 128 MiB of 2 MiB pages is still below the batch
    cache_bytes = max(cache_mib << 20, 64 * cfg[0])
    print(f"[gpu] batch_small cfg={cfg} cache={cache_bytes >> 20} MiB", flush=True)
    bb = autotune.BatchBench(paths, sizes, cache_bytes, rpc_slots=16)
    gbs, res, st = bb.run(cfg)
    assert st["timeouts"] == 0 and st["io_errors"] == 0
    assert int(res.status.sum()) == sum(sizes)
    np.testing.assert_array_equal(res.csum, want_c)
    np.testing.assert_array_equal(res.hist, want_h)
    if cache_mib == 32:
        assert st["evictions"] > 0


def test_autotuned_config_is_correct(small_batch, cuda):
    m, paths, sizes, want_c, want_h = small_batch
    bb = autotune.BatchBench(paths, sizes, 256 << 20, rpc_slots=16)
    r = autotune.coordinate_descent(bb.measure, spaces=((64 << 10, 1 << 20), (1 << 20, 4 << 20), (1, 8)),
                                    max_passes=1)
    print(f"[gpu] autotune best {r.best} {r.best_value:.2f} GB/s over {len(r.history)} runs", flush=True)
    gbs, res, st = bb.run(r.best)
    np.testing.assert_array_equal(res.csum, want_c)
    np.testing.assert_array_equal(res.hist, want_h)


def test_batch_full_c4(data_dir, cuda):
    m, paths, sizes = _files("batch", data_dir)
    print(f"[gpu] c4: {len(paths)} files, {sum(sizes) / 2**30:.2f} GiB", flush=True)
    bb = autotune.BatchBench(paths, sizes, m["cache_bytes"], rpc_slots=32)
    gbs, res, st = bb.run((256 << 10, 16 << 20, 4))
    print(f"[gpu] c4 batched: {gbs:.2f} GB/s; oracle over every file", flush=True)
    assert st["timeouts"] == 0 and st["io_errors"] == 0
    assert int(res.status.sum()) == sum(sizes)
    for i, p in enumerate(paths):                       # every file, checksum and histogram
        c, h = odata.file_digest(p)
        assert int(res.csum[i]) == c, i
        np.testing.assert_array_equal(res.hist[i], h)


@pytest.mark.parametrize("advice", [("normal", "normal"), ("sequential", "random"), ("normal", "random")])
def test_mixed_sequential_and_random_files(advice, data_dir, cuda):
    """The mixed case (Sec. 3.1: one file read in order, another at random) in one persistent
    launch, with per-file readahead hints (Sec. 4: posix_fadvise-like): each output row equals
    the oracle's sum over the reads folded into it, and with RANDOM advice the random file is
    read one page per miss (no readahead pages for it)."""
    torch = cuda
    wl = configs.f2_small()
    pa, pb = configs.ensure_file(wl.seq, data_dir), configs.ensure_file(wl.rnd, data_dir)
    units = wl.units()
    want_c, want_h = odata.unit_outputs({0: pa, 1: pb}, units, 2)
    adv = {"normal": gfs.GFS_ADV_NORMAL, "sequential": gfs.GFS_ADV_SEQUENTIAL, "random": gfs.GFS_ADV_RANDOM}
    print(f"[gpu] f2_small advice {advice}", flush=True)
    cfg = runner.make_config(wl.page_size, wl.cache_bytes, ra_cap_bytes=1 << 20, timeout_s=30)
    with gfs.PageCache(cfg) as cache:
        ids = [cache.open(pa), cache.open(pb)]
        for i, a in enumerate(advice):
            cache.fadvise(ids[i], adv[a])
        u = units.copy()
        u["file"] = np.array(ids, dtype=np.uint32)[units["file"]]
        rd = runner.BatchReader(None, None, wl.piece, 1, units=u, nout=2)
        rd.launch(cache)
        res = rd.result()
        st = cache.stats()
    assert st["timeouts"] == 0 and st["io_errors"] == 0
    assert int(res.status.sum()) == int(units["size"].sum())
    np.testing.assert_array_equal(res.csum, want_c)
    np.testing.assert_array_equal(res.hist, want_h)
    if advice[1] == "random":
        # readahead pages can only come from the sequential file (16 MiB = 256 pages)
        assert st["ra_pages"] <= wl.seq.size // wl.page_size
