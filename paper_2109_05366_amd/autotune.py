"""Autotuner for the batched persistent launch: page size, readahead cap, blocks per file.

The search is coordinate descent over the discrete grid: starting from a middle point it
sweeps one parameter at a time with the others fixed, keeps the best value, and repeats
the sweeps until a full pass brings no improvement (or the pass limit is reached). Each
evaluation is one cold pass of the batch (cache reset, files re-read from storage),
measured in delivered GB/s; configurations that fail validation (window larger than the
library's limit) are skipped. The measure function is supplied by the caller, so the same
search drives the real batch on the GPU and the CPU tests of the search itself.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

from . import gfs, runner

PAGE_SIZES = (64 << 10, 256 << 10, 1 << 20, 2 << 20)
RA_CAPS = (1 << 20, 4 << 20, 16 << 20, 64 << 20)
BLOCKS_PER_FILE = (1, 2, 4, 8, 16)

Config = Tuple[int, int, int]          # (page_size, ra_cap_bytes, blocks_per_file)


def valid(cfg: Config) -> bool:
    page, cap, bpf = cfg
    return cap % page == 0 and cap // page <= gfs.GFS_MAX_WINDOW_PAGES and bpf >= 1


@dataclasses.dataclass
class SearchResult:
    best: Config
    best_value: float
    history: List[Tuple[Config, float]]


def coordinate_descent(measure: Callable[[Config], float],
                       spaces: Sequence[Sequence[int]] = (PAGE_SIZES, RA_CAPS, BLOCKS_PER_FILE),
                       start: Optional[Config] = None, max_passes: int = 2) -> SearchResult:
    cache: Dict[Config, float] = {}
    history: List[Tuple[Config, float]] = []

    def score(cfg: Config) -> float:
        if cfg not in cache:
            cache[cfg] = measure(cfg) if valid(cfg) else float("-inf")
            history.append((cfg, cache[cfg]))
        return cache[cfg]

    cur = list(start or tuple(sp[len(sp) // 2] for sp in spaces))
    best_v = score(tuple(cur))
    for _ in range(max_passes):
        improved = False
        for dim, space in enumerate(spaces):
            for v in space:
                cand = list(cur)
                cand[dim] = v
                s = score(tuple(cand))
                if s > best_v:
                    best_v, cur, improved = s, cand, True
        if not improved:
            break
    return SearchResult(best=tuple(cur), best_value=best_v, history=history)


class BatchBench:
    """Cold passes of a file batch through the persistent kernel on the GPU."""

    def __init__(self, paths: Sequence[str], sizes: Sequence[int], cache_bytes: int, host_threads: int = 8,
                 rpc_slots: int = 32, threads: int = 256):
        self.paths = list(paths)
        self.sizes = [int(s) for s in sizes]
        self.cache_bytes = cache_bytes
        self.host_threads = host_threads
        self.rpc_slots = rpc_slots
        self.threads = threads
        self.total = sum(self.sizes)

    def run(self, cfg: Config, passes: int = 1):
        """Returns (GB/s over the timed passes, BatchResult of the last pass, stats)."""
        import torch
        page, cap, bpf = cfg
        cache_bytes = self.cache_bytes // page * page
        conf = runner.make_config(page, cache_bytes, ra_cap_bytes=cap, host_threads=self.host_threads,
                                  rpc_slots=self.rpc_slots, timeout_s=120)
        with gfs.PageCache(conf) as cache:
            ids = [cache.open(p) for p in self.paths]
            unit = max(page, 256 << 10)
            br = runner.BatchReader(ids, self.sizes, unit, bpf, threads=self.threads)
            dt = 0.0
            for _ in range(passes):
                cache.reset()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                br.launch(cache)
                res = br.result()
                dt += time.perf_counter() - t0
            st = cache.stats()
        return passes * self.total / dt / 1e9, res, st

    def run_per_file(self, cfg: Config) -> float:
        """The plain form for comparison: one cold pass with a separate launch per file (each
        over the whole grid, blocks_per_file = the grid), one after another. GB/s."""
        import torch
        page, cap, _ = cfg
        cache_bytes = self.cache_bytes // page * page
        conf = runner.make_config(page, cache_bytes, ra_cap_bytes=cap, host_threads=self.host_threads,
                                  rpc_slots=self.rpc_slots, timeout_s=120)
        with gfs.PageCache(conf) as cache:
            ids = [cache.open(p) for p in self.paths]
            unit = max(page, 256 << 10)
            readers = [runner.BatchReader([i], [s], unit, 1 << 20, threads=self.threads)
                       for i, s in zip(ids, self.sizes)]
            cache.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for br in readers:
                br.launch(cache)
                br.result()
            dt = time.perf_counter() - t0
        return self.total / dt / 1e9

    def measure(self, cfg: Config) -> float:
        return self.run(cfg)[0]
