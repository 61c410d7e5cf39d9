"""Python binding of libgfs.so (ctypes): the C-ABI of include/gfs.h, same names.

Argument marshalling only: every step of the page-cache path runs in the library's HIP
kernels and host threads. PyTorch provides device memory and streams. If the library is
not built this module raises at first use; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgfs.so")

GFS_ABI_VERSION = 5
GFS_O_RDONLY = 0
GFS_ADV_NORMAL, GFS_ADV_RANDOM, GFS_ADV_SEQUENTIAL = 0, 1, 2
GFS_DIRECT_OFF, GFS_DIRECT_ON, GFS_DIRECT_PREFER = 0, 1, 2
GFS_POLICY_SHARED, GFS_POLICY_PRIVATE = 0, 1
GFS_IO_PREAD, GFS_IO_PREAD_PARTITIONED, GFS_IO_URING = 0, 1, 2
GFS_MAX_WINDOW_PAGES = 1024

EV_HIT, EV_JOIN, EV_MISS, EV_HAND, EV_ALLOC, EV_REQ, EV_NOFRAME = 1, 2, 3, 4, 5, 6, 7
RA_RULE_OFF, RA_RULE_ZONE, RA_RULE_AGGREGATE, RA_RULE_CONTEXT, RA_RULE_NEW = 0, 1, 2, 3, 4
HAND_FREE, HAND_SKIP, HAND_CLEAR, HAND_EVICT = 0, 1, 2, 3


class gfs_config(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("streams_per_file", C.c_uint32),
        ("page_size", C.c_uint64), ("cache_bytes", C.c_uint64),
        ("ra_init_bytes", C.c_uint64), ("ra_cap_bytes", C.c_uint64),
        ("host_threads", C.c_uint32), ("rpc_slots", C.c_uint32),
        ("io_backend", C.c_uint32), ("o_direct", C.c_uint32),
        ("trace_level", C.c_uint32), ("trace_capacity", C.c_uint32),
        ("wait_timeout_ns", C.c_uint64), ("policy", C.c_uint32), ("private_slots", C.c_uint32),
        ("io_chunk_bytes", C.c_uint32), ("max_files", C.c_uint32),
        ("ra_recent", C.c_uint32), ("ra_near_pages", C.c_uint32), ("ra_near_min", C.c_uint32),
        ("ra_quota_blocks", C.c_uint32), ("ra_async", C.c_uint32), ("io_depth", C.c_uint32),
        ("page_timers", C.c_uint32),
    ]


_STAT_U64 = ["hits", "joins", "misses", "ra_pages", "fetched_pages", "evictions", "wasted_pages",
             "hand_visits", "requests", "request_bytes", "delivered_bytes", "retries", "noframe",
             "timeouts", "io_errors", "trace_events", "host_requests", "host_bytes", "host_read_ns",
             "t_lock_ns", "t_crit_ns", "t_alloc_ns", "t_slot_ns", "t_host_ns", "t_pull_ns", "t_join_ns",
             "t_decide_ns", "t_run_ns", "t_unlock_ns", "lock_acquired", "lock_left", "t_acquire_ns", "t_copy_ns",
             "t_unpin_ns", "private_hits", "private_wasted",
             "host_errors", "host_last_errno"]


class gfs_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in _STAT_U64] + [
        ("host_spins", C.c_uint64 * 64), ("host_threads", C.c_uint32), ("direct_io", C.c_uint32),
        ("host_thread_requests", C.c_uint64 * 64), ("ra_async_windows", C.c_uint64)]


UNIT_DTYPE = np.dtype([("file", "<u4"), ("out", "<u4"), ("offset", "<u8"), ("size", "<u8")])

SERVE_REQUEST_DTYPE = np.dtype([("file_id", "<u4"), ("pad", "<u4"), ("arrival_ns", "<u8")])
SERVE_RECORD_DTYPE = np.dtype([("csum", "<u8"), ("result", "<i8"), ("arrival_ns", "<u8"), ("admit_ns", "<u8"),
                               ("first_ns", "<u8"), ("done_ns", "<u8"), ("seq", "<u8"), ("reserved", "<u8")])


class gfs_serve_params(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("chunk_bytes", C.c_uint64), ("grid", C.c_uint32),
                ("threads", C.c_uint32), ("idle_timeout_ns", C.c_uint64)]


class gfs_serve_summary(C.Structure):
    _fields_ = [("span_ns", C.c_uint64), ("delivered_bytes", C.c_uint64), ("peak_reserved", C.c_uint64),
                ("peak_pending", C.c_uint32), ("grid", C.c_uint32), ("clock_skew_ns", C.c_uint64)]


EVENT_DTYPE = np.dtype([("op", "<u4"), ("block", "<u4"), ("file", "<u4"), ("page", "<u4"),
                        ("frame", "<u4"), ("a", "<u4"), ("b", "<u8")])

_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = C.CDLL(LIB_PATH)
    vp, u32, u64, i32, sz = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int, C.c_size_t
    L.gfs_config_default.argtypes = [C.POINTER(gfs_config)]
    L.gfs_config_default.restype = None
    L.gfs_device_bytes.argtypes = [C.POINTER(gfs_config), C.POINTER(sz), C.POINTER(sz)]
    L.gfs_init.argtypes = [C.POINTER(gfs_config), vp, vp, vp, C.POINTER(vp)]
    L.gfs_open.argtypes = [vp, C.c_char_p, i32, C.POINTER(i32)]
    L.gfs_fadvise.argtypes = [vp, i32, i32]
    L.gfs_close.argtypes = [vp, i32]
    L.gfs_device_handle.argtypes = [vp]
    L.gfs_device_handle.restype = vp
    L.gfs_stats_read.argtypes = [vp, C.POINTER(gfs_stats)]
    L.gfs_trace_read.argtypes = [vp, vp, sz, C.POINTER(sz)]
    L.gfs_reset_cache.argtypes = [vp]
    L.gfs_shutdown.argtypes = [vp]
    L.gfs_launch_list_reader.argtypes = [vp, i32, vp, u32, u32, u64, u32, i32, vp, vp, vp, vp, vp]
    L.gfs_launch_buffer_reader.argtypes = [vp, u64, vp, u32, u32, u64, u32, i32, vp, vp, vp]
    L.gfs_batch_plan.argtypes = [vp, vp, u32, u64, u32, u32, vp, u64, C.POINTER(u64)]
    L.gfs_launch_batch.argtypes = [vp, vp, u64, u32, u32, u64, vp, vp, vp, vp, vp, vp]
    L.gfs_batch_grid.argtypes = [u32, C.POINTER(u32)]
    L.gfs_file_size.argtypes = [vp, i32, C.POINTER(u64)]
    L.gfs_get_config.argtypes = [vp, C.POINTER(gfs_config)]
    L.gfs_serve_run.argtypes = [vp, vp, u32, C.POINTER(gfs_serve_params), vp, C.POINTER(gfs_serve_summary), vp]
    L.gfs_serve_run_noalloc.argtypes = L.gfs_serve_run.argtypes
    for name in ("gfs_device_bytes", "gfs_init", "gfs_open", "gfs_fadvise", "gfs_close",
                 "gfs_stats_read", "gfs_trace_read", "gfs_reset_cache", "gfs_shutdown",
                 "gfs_launch_list_reader", "gfs_launch_buffer_reader", "gfs_batch_plan", "gfs_launch_batch",
                 "gfs_batch_grid",
                 "gfs_file_size", "gfs_get_config", "gfs_serve_run", "gfs_serve_run_noalloc"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise OSError(-rc, f"{what}: {os.strerror(-rc)}")
    return rc


# ---- thin wrappers, one per C function ---------------------------------------------------

def gfs_config_default(**overrides) -> gfs_config:
    cfg = gfs_config()
    lib().gfs_config_default(C.byref(cfg))
    for k, v in overrides.items():
        if not hasattr(cfg, k):
            raise AttributeError(k)
        setattr(cfg, k, v)
    return cfg


def gfs_device_bytes(cfg: gfs_config) -> Tuple[int, int]:
    fb, mb = C.c_size_t(0), C.c_size_t(0)
    _check(lib().gfs_device_bytes(C.byref(cfg), C.byref(fb), C.byref(mb)), "gfs_device_bytes")
    return fb.value, mb.value


def gfs_init(cfg: gfs_config, frames_dev: int, meta_dev: int, stream: int) -> int:
    ctx = C.c_void_p(0)
    _check(lib().gfs_init(C.byref(cfg), C.c_void_p(frames_dev), C.c_void_p(meta_dev),
                          C.c_void_p(stream), C.byref(ctx)), "gfs_init")
    return ctx.value


def gfs_open(ctx: int, path: str, flags: int = GFS_O_RDONLY) -> int:
    fid = C.c_int(-1)
    _check(lib().gfs_open(C.c_void_p(ctx), path.encode(), flags, C.byref(fid)), f"gfs_open({path})")
    return fid.value


def gfs_fadvise(ctx: int, file_id: int, advice: int) -> None:
    _check(lib().gfs_fadvise(C.c_void_p(ctx), file_id, advice), "gfs_fadvise")


def gfs_close(ctx: int, file_id: int) -> None:
    _check(lib().gfs_close(C.c_void_p(ctx), file_id), "gfs_close")


def gfs_device_handle(ctx: int) -> int:
    return lib().gfs_device_handle(C.c_void_p(ctx))


def gfs_stats_read(ctx: int) -> Dict[str, object]:
    s = gfs_stats()
    _check(lib().gfs_stats_read(C.c_void_p(ctx), C.byref(s)), "gfs_stats_read")
    out: Dict[str, object] = {n: int(getattr(s, n)) for n in _STAT_U64}
    out["host_threads"] = int(s.host_threads)
    out["host_spins"] = [int(x) for x in s.host_spins[: s.host_threads]]
    out["host_thread_requests"] = [int(x) for x in s.host_thread_requests[: s.host_threads]]
    out["direct_io"] = int(s.direct_io)
    out["ra_async_windows"] = int(s.ra_async_windows)
    return out


def gfs_trace_read(ctx: int, max_events: int) -> np.ndarray:
    buf = np.zeros(max_events, dtype=EVENT_DTYPE)
    n = C.c_size_t(0)
    _check(lib().gfs_trace_read(C.c_void_p(ctx), C.c_void_p(buf.ctypes.data), buf.nbytes, C.byref(n)),
           "gfs_trace_read")
    return buf[: n.value // EVENT_DTYPE.itemsize].copy()


def gfs_reset_cache(ctx: int) -> None:
    _check(lib().gfs_reset_cache(C.c_void_p(ctx)), "gfs_reset_cache")


def gfs_shutdown(ctx: int) -> None:
    _check(lib().gfs_shutdown(C.c_void_p(ctx)), "gfs_shutdown")


def gfs_launch_list_reader(ctx: int, file_id: int, offsets_dev: int, blocks: int, reads: int,
                           read_size: int, threads: int, consumer: int, buf_dev: int, out_dev: int,
                           status_dev: int, turn_dev: int, stream: int) -> None:
    _check(lib().gfs_launch_list_reader(C.c_void_p(ctx), file_id, C.c_void_p(offsets_dev), blocks, reads,
                                        read_size, threads, consumer, C.c_void_p(buf_dev),
                                        C.c_void_p(out_dev), C.c_void_p(status_dev),
                                        C.c_void_p(turn_dev or 0), C.c_void_p(stream)),
           "gfs_launch_list_reader")


def gfs_launch_buffer_reader(data_dev: int, data_size: int, offsets_dev: int, blocks: int, reads: int,
                             read_size: int, threads: int, consumer: int, out_dev: int, status_dev: int,
                             stream: int) -> None:
    _check(lib().gfs_launch_buffer_reader(C.c_void_p(data_dev), data_size, C.c_void_p(offsets_dev), blocks, reads,
                                          read_size, threads, consumer, C.c_void_p(out_dev), C.c_void_p(status_dev),
                                          C.c_void_p(stream)), "gfs_launch_buffer_reader")


def gfs_batch_plan(sizes, ids, unit_bytes: int, grid: int, blocks_per_file: int) -> np.ndarray:
    sizes = np.ascontiguousarray(sizes, dtype=np.uint64)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    if sizes.shape != ids.shape:
        raise ValueError("sizes and ids differ in length")
    n = C.c_uint64(0)
    rc = lib().gfs_batch_plan(C.c_void_p(sizes.ctypes.data), C.c_void_p(ids.ctypes.data), len(sizes), unit_bytes,
                              grid, blocks_per_file, None, 0, C.byref(n))
    if rc not in (0, -28):
        _check(rc, "gfs_batch_plan")
    out = np.zeros(n.value, dtype=UNIT_DTYPE)
    _check(lib().gfs_batch_plan(C.c_void_p(sizes.ctypes.data), C.c_void_p(ids.ctypes.data), len(sizes),
                                unit_bytes, grid, blocks_per_file, C.c_void_p(out.ctypes.data), len(out),
                                C.byref(n)), "gfs_batch_plan")
    return out[: n.value]


def gfs_launch_batch(ctx: int, units_dev: int, nunits: int, grid: int, threads: int, unit_bytes: int,
                     buf_dev: int, counter_dev: int, csum_dev: int, hist_dev: int, status_dev: int,
                     stream: int) -> None:
    _check(lib().gfs_launch_batch(C.c_void_p(ctx), C.c_void_p(units_dev), nunits, grid, threads, unit_bytes,
                                  C.c_void_p(buf_dev), C.c_void_p(counter_dev), C.c_void_p(csum_dev),
                                  C.c_void_p(hist_dev), C.c_void_p(status_dev), C.c_void_p(stream)),
           "gfs_launch_batch")


def gfs_batch_grid(threads: int) -> int:
    g = C.c_uint32(0)
    _check(lib().gfs_batch_grid(threads, C.byref(g)), "gfs_batch_grid")
    return g.value


def gfs_file_size(ctx: int, file_id: int) -> int:
    v = C.c_uint64(0)
    _check(lib().gfs_file_size(C.c_void_p(ctx), file_id, C.byref(v)), "gfs_file_size")
    return v.value


def gfs_get_config(ctx: int) -> gfs_config:
    cfg = gfs_config()
    _check(lib().gfs_get_config(C.c_void_p(ctx), C.byref(cfg)), "gfs_get_config")
    return cfg


def _serve(name: str, ctx: int, requests: np.ndarray, params: gfs_serve_params,
           stream: int) -> Tuple[np.ndarray, Dict[str, int]]:
    reqs = np.ascontiguousarray(requests, dtype=SERVE_REQUEST_DTYPE)
    out = np.zeros(len(reqs), dtype=SERVE_RECORD_DTYPE)
    summ = gfs_serve_summary()
    _check(getattr(lib(), name)(C.c_void_p(ctx), C.c_void_p(reqs.ctypes.data), len(reqs), C.byref(params),
                                C.c_void_p(out.ctypes.data), C.byref(summ), C.c_void_p(stream)), name)
    return out, {n: int(getattr(summ, n)) for n, _ in gfs_serve_summary._fields_}


def gfs_serve_run(ctx: int, requests: np.ndarray, params: gfs_serve_params,
                  stream: int) -> Tuple[np.ndarray, Dict[str, int]]:
    """requests: SERVE_REQUEST_DTYPE array; returns (SERVE_RECORD_DTYPE records, summary)."""
    return _serve("gfs_serve_run", ctx, requests, params, stream)


def gfs_serve_run_noalloc(ctx: int, requests: np.ndarray, params: gfs_serve_params,
                          stream: int) -> Tuple[np.ndarray, Dict[str, int]]:
    """As gfs_serve_run, through the entry point that allocates nothing (state in the
    library's fixed scratch array and the context's mailbox)."""
    return _serve("gfs_serve_run_noalloc", ctx, requests, params, stream)


GFS_SERVE_NOALLOC_MAX_REQUESTS = 16384
GFS_SERVE_NOALLOC_SCRATCH_BYTES = 64 << 20


# ---- convenience: a cache over torch-allocated device memory ----------------------------

class PageCache:
    """Owns the torch allocations a context needs; closes the context on close()."""

    def __init__(self, cfg: gfs_config, device: str = "cuda:0", stream=None):
        import torch
        self.cfg = cfg
        fb, mb = gfs_device_bytes(cfg)
        self.frames = torch.empty(fb, dtype=torch.uint8, device=device)
        self.meta = torch.empty(mb, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.ctx = gfs_init(cfg, self.frames.data_ptr(), self.meta.data_ptr(), self.stream.cuda_stream)
        self.handle = gfs_device_handle(self.ctx)

    def open(self, path: str, flags: int = GFS_O_RDONLY) -> int:
        return gfs_open(self.ctx, path, flags)

    def fadvise(self, fid: int, advice: int) -> None:
        gfs_fadvise(self.ctx, fid, advice)

    def close_file(self, fid: int) -> None:
        gfs_close(self.ctx, fid)

    def stats(self) -> Dict[str, object]:
        return gfs_stats_read(self.ctx)

    def config(self) -> gfs_config:
        return gfs_get_config(self.ctx)

    def trace(self, max_events: Optional[int] = None) -> np.ndarray:
        return gfs_trace_read(self.ctx, max_events or int(self.cfg.trace_capacity))

    def reset(self) -> None:
        gfs_reset_cache(self.ctx)

    def close(self) -> None:
        if self.ctx:
            gfs_shutdown(self.ctx)
            self.ctx = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
