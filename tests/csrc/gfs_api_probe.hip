// A user kernel of the device API, for the tests: it opens a registered file by path with
// gopen (Sec. 2.2: a threadblock opens, reads and closes files with POSIX-like calls made by
// all of its threads) and records what each call returns, including the error returns.
// Built by the package's build step into tests/libgfs_api_probe.so; takes the device handle
// that gfs_device_handle returns.
#include <errno.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "gfs.h"
#include "gfs_device.h"

namespace {

// out[0]  gopen(path, GFS_O_RDONLY)          a descriptor
// out[1]  gopen(path, flags 1)                -EROFS: only read-only opens
// out[2]  gopen(missing, GFS_O_RDONLY)        -ENOENT: not registered
// out[3]  gread(bad_fd, ...)                  -EBADF: an id below max_files that is not registered
// out[4]  gread(-1, ...)                      -EBADF
// out[5]  gread(fd, off, size, buf)           bytes delivered (buf holds them)
// out[6]  gread(fd, eof_off, 64, buf2)        0 at or past the end of the file
// out[7]  gclose(1 << 20)                     -EBADF
// out[8]  gclose(fd)                          0
// out[9]  gopen_id(bad_fd, GFS_O_RDONLY)      -ENOENT
__global__ void __launch_bounds__(GFS_MAX_BLOCK_THREADS) api_probe_kernel(const gfs_dev* d, const char* path,
                                                                          const char* missing, int bad_fd,
                                                                          uint64_t off, uint64_t size,
                                                                          uint64_t eof_off, uint8_t* buf,
                                                                          int64_t* out) {
  const bool t0 = threadIdx.x == 0;
  const int fd = gopen(d, path, GFS_O_RDONLY);
  const int e_rofs = gopen(d, path, 1);
  const int e_noent = gopen(d, missing, GFS_O_RDONLY);
  const int64_t e_bad = gread(d, bad_fd, 0, 16, buf);
  const int64_t e_neg = gread(d, -1, 0, 16, buf);
  const int64_t got = fd >= 0 ? gread(d, fd, off, size, buf) : -1;
  const int64_t at_eof = fd >= 0 ? gread(d, fd, eof_off, 64, buf + size) : -1;
  const int c_bad = gclose(d, 1 << 20);
  const int c_ok = fd >= 0 ? gclose(d, fd) : -1;
  const int e_id = gopen_id(d, bad_fd, GFS_O_RDONLY);
  if (t0) {
    out[0] = fd;
    out[1] = e_rofs;
    out[2] = e_noent;
    out[3] = e_bad;
    out[4] = e_neg;
    out[5] = got;
    out[6] = at_eof;
    out[7] = c_bad;
    out[8] = c_ok;
    out[9] = e_id;
  }
}

}  // namespace

// One block of `threads` threads (a multiple of 64 for reads to run; any other count makes
// gread return -EINVAL). Pointers are device pointers; buf holds size + 64 bytes; out holds
// 10 values. Returns 0 or -EIO if the launch failed.
extern "C" int gfs_test_api_probe(const void* dev_handle, const char* path_dev, const char* missing_dev,
                                  int bad_fd, uint64_t off, uint64_t size, uint64_t eof_off, uint32_t threads,
                                  void* buf, int64_t* out, void* stream) {
  if (!dev_handle || !path_dev || !missing_dev || !buf || !out || threads == 0 ||
      threads > GFS_MAX_BLOCK_THREADS)
    return -EINVAL;
  hipLaunchKernelGGL(api_probe_kernel, dim3(1), dim3(threads), 0, (hipStream_t)stream, (const gfs_dev*)dev_handle,
                     path_dev, missing_dev, bad_fd, off, size, eof_off, (uint8_t*)buf, out);
  return hipGetLastError() == hipSuccess ? 0 : -EIO;
}
