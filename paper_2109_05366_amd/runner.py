"""Launch a list-reader workload through the C-ABI (marshalling and torch allocations only)."""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import gfs


def make_config(page_size: int, cache_bytes: int, ra_cap_bytes: int = 16 << 20, ra_init_pages: int = 4,
                streams: int = 8, host_threads: int = 8, rpc_slots: int = 64,
                o_direct: int = gfs.GFS_DIRECT_PREFER, trace_level: int = 0, trace_capacity: int = 0,
                timeout_s: float = 30.0, policy: int = gfs.GFS_POLICY_SHARED,
                private_slots: int = 512, io_chunk_bytes: int = 2 << 20, max_files: int = 64,
                detector=(64, 64, 3), quota_blocks: int = 0, timeout_ns: int = 0,
                io_backend: int = gfs.GFS_IO_PREAD, io_depth: int = 8, ra_async: int = 0,
                page_timers: int = 0) -> gfs.gfs_config:
    """detector = (ra_recent, ra_near_pages, ra_near_min); quota_blocks = the thrash guard's
    resident-block count (0: the device's, 1: off); timeout_ns overrides timeout_s; io_depth =
    reads in flight per host thread with the io_uring backend; ra_async = 1 for marker-triggered
    (asynchronous) readahead."""
    cap_pages = min(ra_cap_bytes // page_size, gfs.GFS_MAX_WINDOW_PAGES)
    init = min(ra_init_pages, cap_pages) if cap_pages else 0
    return gfs.gfs_config_default(
        page_size=page_size, cache_bytes=cache_bytes, ra_cap_bytes=cap_pages * page_size,
        ra_init_bytes=init * page_size, streams_per_file=streams, host_threads=host_threads,
        rpc_slots=rpc_slots, o_direct=o_direct, trace_level=trace_level,
        trace_capacity=trace_capacity, wait_timeout_ns=int(timeout_ns or timeout_s * 1e9), policy=policy,
        private_slots=private_slots, io_chunk_bytes=io_chunk_bytes, max_files=max_files,
        ra_recent=detector[0], ra_near_pages=detector[1], ra_near_min=detector[2],
        ra_quota_blocks=quota_blocks, io_backend=io_backend, io_depth=io_depth, ra_async=ra_async,
        page_timers=page_timers)


@dataclasses.dataclass
class ListResult:
    out: np.ndarray        # checksums [blocks] uint64 or histograms [blocks, 256] uint32
    status: np.ndarray     # int64 [blocks]: bytes delivered or -errno


class ListReader:
    """Device buffers for one list-reader launch shape: offsets, user buffers, outputs."""

    def __init__(self, offsets: np.ndarray, read_size: int, consumer: int, threads: int = 256,
                 device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.blocks, self.reads = offsets.shape
        self.read_size = read_size
        self.consumer = consumer
        self.threads = threads
        self.offsets = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).to(device)
        self.buf = torch.empty(self.blocks * read_size, dtype=torch.uint8, device=device)
        if consumer == 0:
            self.out = torch.zeros(self.blocks, dtype=torch.int64, device=device)
        elif consumer == 1:
            self.out = torch.zeros(self.blocks * 256, dtype=torch.int32, device=device)
        else:
            self.out = None   # consumer 2: the reads only; the buffers hold each block's last read
        self.status = torch.zeros(self.blocks, dtype=torch.int64, device=device)
        self.turn = torch.zeros(1, dtype=torch.int64, device=device)

    def launch(self, cache: gfs.PageCache, file_id: int, stream=None, serialize: bool = False) -> None:
        s = stream if stream is not None else self.torch.cuda.current_stream()
        if serialize:
            self.turn.zero_()
        gfs.gfs_launch_list_reader(cache.ctx, file_id, self.offsets.data_ptr(), self.blocks, self.reads,
                                   self.read_size, self.threads, self.consumer, self.buf.data_ptr(),
                                   self.out.data_ptr() if self.out is not None else 0, self.status.data_ptr(),
                                   self.turn.data_ptr() if serialize else 0, s.cuda_stream)

    def result(self) -> ListResult:
        self.torch.cuda.synchronize()
        st = self.status.cpu().numpy()
        if self.consumer == 0:
            out = self.out.cpu().numpy().view(np.uint64).copy()
        elif self.consumer == 1:
            out = self.out.cpu().numpy().view(np.uint32).reshape(self.blocks, 256).copy()
        else:
            out = self.buf.cpu().numpy().reshape(self.blocks, self.read_size).copy()
        return ListResult(out=out, status=st)


def run_list(cache: gfs.PageCache, file_id: int, offsets: np.ndarray, read_size: int, consumer: int,
             threads: int = 256, serialize: bool = False) -> ListResult:
    r = ListReader(offsets, read_size, consumer, threads)
    r.launch(cache, file_id, serialize=serialize)
    return r.result()


@dataclasses.dataclass
class BatchResult:
    csum: np.ndarray       # uint64 [files]
    hist: np.ndarray       # uint32 [files, 256]
    status: np.ndarray     # int64 [grid]
    units: int


class BatchReader:
    """Device buffers and unit plan for one persistent batch launch over registered files."""

    def __init__(self, file_ids, sizes, unit_bytes: int, blocks_per_file: int, grid: int = 0,
                 threads: int = 256, device: str = "cuda:0", units=None, nout: int = 0):
        """units: an explicit unit list (UNIT_DTYPE records, file = registered id) with nout
        output rows, instead of the plan gfs_batch_plan makes for whole files."""
        import torch
        self.torch = torch
        self.threads = threads
        self.grid = grid or gfs.gfs_batch_grid(threads)
        self.unit_bytes = unit_bytes
        self.nfiles = nout if units is not None else len(sizes)
        if units is not None:
            plan = np.ascontiguousarray(units).astype(gfs.UNIT_DTYPE)
        else:
            plan = gfs.gfs_batch_plan(sizes, file_ids, unit_bytes, self.grid, blocks_per_file)
        self.nunits = len(plan)
        self.units = torch.from_numpy(plan.view(np.uint8).copy()).to(device)
        self.buf = torch.empty(self.grid * unit_bytes, dtype=torch.uint8, device=device)
        self.counter = torch.zeros(1, dtype=torch.int64, device=device)
        self.csum = torch.zeros(self.nfiles, dtype=torch.int64, device=device)
        self.hist = torch.zeros(self.nfiles * 256, dtype=torch.int32, device=device)
        self.status = torch.zeros(self.grid, dtype=torch.int64, device=device)

    def launch(self, cache: gfs.PageCache, stream=None) -> None:
        s = stream if stream is not None else self.torch.cuda.current_stream()
        self.csum.zero_()
        self.hist.zero_()
        gfs.gfs_launch_batch(cache.ctx, self.units.data_ptr(), self.nunits, self.grid, self.threads,
                             self.unit_bytes, self.buf.data_ptr(), self.counter.data_ptr(),
                             self.csum.data_ptr(), self.hist.data_ptr(), self.status.data_ptr(), s.cuda_stream)

    def result(self) -> BatchResult:
        self.torch.cuda.synchronize()
        return BatchResult(csum=self.csum.cpu().numpy().view(np.uint64).copy(),
                           hist=self.hist.cpu().numpy().view(np.uint32).reshape(self.nfiles, 256).copy(),
                           status=self.status.cpu().numpy(), units=self.nunits)


def serve(cache: gfs.PageCache, file_ids, arrival_ns, budget_bytes: int, chunk_bytes: int = 1 << 20,
          grid: int = 0, threads: int = 256, idle_timeout_s: float = 60.0, stream=None, noalloc: bool = False):
    """Run a request stream through gfs_serve_run (gfs_serve_run_noalloc if noalloc). file_ids[i]
    is request i's registered file, arrival_ns[i] its arrival time. Returns (records, summary)
    as the binding gives them."""
    import torch
    req = np.zeros(len(file_ids), dtype=gfs.SERVE_REQUEST_DTYPE)
    req["file_id"] = np.asarray(file_ids, dtype=np.uint32)
    req["arrival_ns"] = np.asarray(arrival_ns, dtype=np.uint64)
    params = gfs.gfs_serve_params(budget_bytes=budget_bytes, chunk_bytes=chunk_bytes, grid=grid, threads=threads,
                                  idle_timeout_ns=int(idle_timeout_s * 1e9))
    s = stream if stream is not None else torch.cuda.current_stream()
    run = gfs.gfs_serve_run_noalloc if noalloc else gfs.gfs_serve_run
    return run(cache.ctx, req, params, s.cuda_stream)


def latency_ms(records: np.ndarray) -> dict:
    """p50/p99 of time to first page and of completion, from arrival, in milliseconds."""
    ttfp = (records["first_ns"].astype(np.float64) - records["arrival_ns"]) / 1e6
    done = (records["done_ns"].astype(np.float64) - records["arrival_ns"]) / 1e6
    return {"ttfp_p50": float(np.percentile(ttfp, 50)), "ttfp_p99": float(np.percentile(ttfp, 99)),
            "done_p50": float(np.percentile(done, 50)), "done_p99": float(np.percentile(done, 99))}
