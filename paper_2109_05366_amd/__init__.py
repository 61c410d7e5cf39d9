"""MI355X-native GPU file page cache with a readahead prefetcher (arXiv 2109.05366).

libgfs.so (HIP, gfx950) holds the method: the device page table, frames, readahead
detector, clock replacement, request ring client and copy-out (include/gfs_device.h),
and the host runtime serving the ring (csrc/gfs_host.cpp). ``gfs`` is its ctypes
binding; ``runner`` launches the list-reader workloads through it.
"""
