"""CPU-side checks of the C-ABI library: it loads, exports every declared symbol, and its
host-side configuration logic behaves as documented (no GPU calls)."""
import ctypes
import errno
import os
import re

import pytest

from paper_2109_05366_amd import gfs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in ("gfs.h",):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?(?:struct\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\*?\s*(gfs_[a-z_0-9]+)\s*\(",
                             src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = gfs.lib()
    names = _declared_functions()
    assert "gfs_init" in names and "gfs_launch_list_reader" in names and len(names) >= 12
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/gfs.h but not exported"


def test_config_default_values():
    cfg = gfs.gfs_config_default()
    assert cfg.abi_version == gfs.GFS_ABI_VERSION
    assert cfg.page_size == 64 << 10 and cfg.cache_bytes == 256 << 20
    assert cfg.ra_init_bytes == 4 * cfg.page_size and cfg.ra_cap_bytes == 16 << 20
    assert cfg.streams_per_file == 8 and cfg.host_threads == 8 and cfg.rpc_slots == 64
    assert ctypes.sizeof(gfs.gfs_config) == 120
    assert cfg.policy == gfs.GFS_POLICY_SHARED and cfg.private_slots == 512
    assert cfg.io_chunk_bytes == 2 << 20
    assert gfs.EVENT_DTYPE.itemsize == 32


def test_device_bytes_layout_scales_with_frames():
    f1, m1 = gfs.gfs_device_bytes(gfs.gfs_config_default(cache_bytes=256 << 20))
    f2, m2 = gfs.gfs_device_bytes(gfs.gfs_config_default(cache_bytes=512 << 20))
    assert f1 == 256 << 20 and f2 == 512 << 20
    # frame words, tags and fill tags (24 B per frame) + the table: 8 B entries, at least 4
    # per frame plus 8192 for reservations in flight, a power of two of 16-entry buckets
    # (32768 entries for 4096 frames, 65536 for 8192)
    assert m2 - m1 == 4096 * (8 + 8 + 8) + 8 * (65536 - 32768)
    f3, m3 = gfs.gfs_device_bytes(gfs.gfs_config_default(trace_level=1, trace_capacity=1000))
    assert m3 - m1 >= 1000 * 32


@pytest.mark.parametrize("field,value", [
    ("abi_version", 99), ("page_size", 3000), ("page_size", 1 << 12 - 1), ("page_size", 4 << 20),
    ("cache_bytes", 0), ("cache_bytes", 100 << 10), ("cache_bytes", (64 << 10) * 63),
    ("streams_per_file", 0), ("streams_per_file", 9), ("ra_cap_bytes", 100),
    ("ra_cap_bytes", (64 << 10) * 1025), ("host_threads", 0), ("host_threads", 65),
    ("rpc_slots", 0), ("o_direct", 3), ("trace_level", 3), ("io_backend", 3), ("policy", 2),
    ("io_depth", 0), ("io_depth", 257),
])
def test_invalid_configs_rejected(field, value):
    cfg = gfs.gfs_config_default()
    setattr(cfg, field, value)
    with pytest.raises(OSError) as e:
        gfs.gfs_device_bytes(cfg)
    assert e.value.errno == errno.EINVAL


def test_readahead_init_must_fit_cap():
    cfg = gfs.gfs_config_default(ra_cap_bytes=4 * (64 << 10), ra_init_bytes=8 * (64 << 10))
    with pytest.raises(OSError):
        gfs.gfs_device_bytes(cfg)
    cfg = gfs.gfs_config_default(ra_cap_bytes=0, ra_init_bytes=0)   # readahead off
    assert gfs.gfs_device_bytes(cfg)[0] == cfg.cache_bytes


def test_null_arguments_rejected_without_gpu():
    lib = gfs.lib()
    assert lib.gfs_init(None, None, None, None, None) == -errno.EINVAL
    assert lib.gfs_open(None, b"x", 0, None) == -errno.EINVAL
    assert lib.gfs_shutdown(None) == -errno.EINVAL
    assert lib.gfs_device_handle(None) is None


def test_policy_and_queue_limits():
    P = 64 << 10
    ok = gfs.gfs_config_default(policy=gfs.GFS_POLICY_PRIVATE, private_slots=64, cache_bytes=64 * P)
    f, _ = gfs.gfs_device_bytes(ok)
    assert f == 64 * P + 64 * ok.ra_cap_bytes          # the private buffers live with the frames
    for bad in (dict(private_slots=0), dict(private_slots=65, cache_bytes=64 * P)):   # quota < 1 frame
        cfg = gfs.gfs_config_default(policy=gfs.GFS_POLICY_PRIVATE, **bad)
        with pytest.raises(OSError):
            gfs.gfs_device_bytes(cfg)
    cfg = gfs.gfs_config_default(io_backend=gfs.GFS_IO_PREAD_PARTITIONED, host_threads=8, rpc_slots=4)
    with pytest.raises(OSError):                        # every host thread needs its own slots
        gfs.gfs_device_bytes(cfg)
    gfs.gfs_device_bytes(gfs.gfs_config_default(io_backend=gfs.GFS_IO_PREAD_PARTITIONED, host_threads=4,
                                                rpc_slots=64))
    for chunk in (64 << 10, 8 << 20, 64 << 20):
        gfs.gfs_device_bytes(gfs.gfs_config_default(io_chunk_bytes=chunk))
    for bad in (dict(io_chunk_bytes=0), dict(io_chunk_bytes=(1 << 20) + 512), dict(io_chunk_bytes=32 << 10),
                dict(io_chunk_bytes=128 << 20), dict(max_files=0), dict(max_files=1025), dict(ra_recent=0),
                dict(ra_recent=65), dict(ra_near_min=0), dict(ra_near_min=66), dict(ra_near_pages=(1 << 20) + 1),
                dict(ra_async=2)):
        with pytest.raises(OSError):
            gfs.gfs_device_bytes(gfs.gfs_config_default(**bad))


def test_metadata_scales_with_max_files():
    """Per-file metadata (record, miss lock and its 4096 queue slots, claims, path, and one
    bit per page for 2^19 pages, set when a page is evicted after use) is sized by max_files:
    about 98 KiB per file, so 64 files take ~6 MiB rather than the 1024-file maximum's
    ~98 MiB."""
    _, m64 = gfs.gfs_device_bytes(gfs.gfs_config_default(max_files=64))
    _, m1024 = gfs.gfs_device_bytes(gfs.gfs_config_default(max_files=1024))
    per_file = (m1024 - m64) / 960
    assert 97 << 10 < per_file < 99 << 10, per_file
    assert m64 < m1024 / 8


def test_detector_defaults():
    cfg = gfs.gfs_config_default()
    assert (cfg.ra_recent, cfg.ra_near_pages, cfg.ra_near_min) == (64, 64, 3)
    assert cfg.ra_quota_blocks == 0 and cfg.ra_async == 0 and cfg.max_files == 64 and cfg.page_timers == 0
