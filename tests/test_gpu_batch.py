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
    print(f"[gpu] c4 batched: {gbs:.2f} GB/s", flush=True)
    assert st["timeouts"] == 0 and st["io_errors"] == 0
    assert int(res.status.sum()) == sum(sizes)
    np.testing.assert_array_equal(res.hist.sum(axis=1, dtype=np.uint64), np.array(sizes, dtype=np.uint64))
    order = np.argsort(sizes)
    sample = sorted(set(order[:4].tolist()) | {int(order[len(order) // 2])})
    for i in sample:
        assert int(res.csum[i]) == odata.file_checksum(paths[i]), i
        np.testing.assert_array_equal(res.hist[i], odata.file_histogram(paths[i]))
