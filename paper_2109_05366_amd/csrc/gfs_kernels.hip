// Kernels of the library: metadata zeroing and the list-reader workload that drives gread
// (the benchmark consumer: per-block checksum or byte histogram of everything delivered).
#include <errno.h>

#include <hip/hip_runtime.h>

#include "gfs.h"
#include "gfs_device.h"
#include "gfs_layout.h"
#include "gfs_consumers.h"

extern "C" int gfs_internal_zero(void* p, size_t bytes, hipStream_t s);

namespace {

using gfs_consumers::block_sum_u64;
using gfs_consumers::checksum_part;
using gfs_consumers::histogram_part;

__global__ void zero_kernel(uint64_t* p, uint64_t n8) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n8; i += stride) p[i] = 0;
}

// Drop one file's pages: frames whose tag belongs to it become FREE (version bumped), and its
// page-table entries (mapped pages and reservations) are cleared. Runs with no reader kernel
// in flight, so plain accesses suffice.
__global__ void purge_file_kernel(const gfs_dev* d, uint32_t nframes, uint64_t pt_entries, uint32_t file) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t prefix = (uint64_t)file + 1;
  const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (uint64_t i = i0; i < nframes; i += stride) {
    const uint64_t w = d->fword[i];
    if ((w & GFS_FW_STATE) != GFS_FS_FREE && (d->ftag[i] >> GFS_KEY_PAGE_BITS) == prefix) {
      d->fword[i] = (((w >> GFS_FW_VER_SHIFT) + 1) << GFS_FW_VER_SHIFT) | GFS_FS_FREE;
      d->ftag[i] = 0;
      d->ffill[i] = 0;
    }
  }
  for (uint64_t i = i0; i < pt_entries; i += stride) {
    const uint64_t e = d->pt[i];
    if (e && (e >> (GFS_ENTRY_FRAME_BITS + GFS_KEY_PAGE_BITS)) == prefix) d->pt[i] = 0;
  }
}

__global__ void __launch_bounds__(GFS_MAX_BLOCK_THREADS, 2) list_reader_kernel(const gfs_dev* d, int file_id, const uint64_t* offsets,
                                   uint32_t reads, uint64_t read_size, int consumer,
                                   uint8_t* buf, void* out, int64_t* status, uint64_t* turn) {
  __shared__ uint32_t hist[256];
  __shared__ uint64_t red[16];
  __shared__ int gate_err;
  __shared__ uint64_t offs[64];   /* the block's next read offsets, fetched 64 at a time */
  const uint32_t b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  uint8_t* mybuf = buf + (uint64_t)b * read_size;
  if (consumer == 1)
    for (uint32_t i = tid; i < 256; i += nt) hist[i] = 0;
  __syncthreads();
  const int fd = gopen_id(d, file_id, GFS_O_RDONLY);
  int64_t err = fd < 0 ? fd : 0;
  int64_t total = 0;
  uint64_t csum = 0;
  const uint64_t t0 = wall_clock64();
  for (uint32_t k = 0; k < reads && err == 0; ++k) {
    if ((k & 63) == 0) {
      // one round trip for the next 64 offsets instead of one before every read (every thread
      // has passed gread's barriers since it read the previous ones)
      if (tid < 64 && k + tid < reads) offs[tid] = offsets[(uint64_t)b * reads + k + tid];
      __syncthreads();
    }
    const uint64_t my_turn = (uint64_t)k * gridDim.x + b;
    if (turn) {
      if (tid == 0) {
        uint32_t n = 0;
        int e = 0;
        while (__hip_atomic_load(turn, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != my_turn) {
          if (gfsd::expired(d, t0)) {
            e = -gfsd::kETIMEDOUT;
            break;
          }
          gfsd::nap(n);
        }
        gate_err = e;
      }
      __syncthreads();
      if (gate_err) {
        err = gate_err;
        break;
      }
    }
    const int64_t r = gread(d, fd, offs[k & 63], read_size, mybuf);
    // serialized runs: an asynchronous window this read issued is in place before the next
    // block's turn, so that every access sees the cache the one-at-a-time order implies
    if (turn) (void)gfsd::async_finish_block(d, gfsd::block_state());
    if (turn && tid == 0)
      __hip_atomic_store(turn, my_turn + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (r < 0) {
      err = r;
      break;
    }
    total += r;
    if (consumer == 0) csum += checksum_part(mybuf, (uint64_t)r, tid, nt);
    else if (consumer == 1) histogram_part(mybuf, (uint64_t)r, tid, nt, hist);
    __syncthreads();
  }
  if (fd >= 0) gclose(d, fd);
  if (consumer == 0) {
    // block reduction of the per-thread sums
    for (int off = 32; off > 0; off >>= 1) csum += __shfl_xor(csum, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = csum;
    __syncthreads();
    if (tid == 0) {
      uint64_t s = 0;
      for (uint32_t w = 0; w < (nt + 63) / 64; ++w) s += red[w];
      ((uint64_t*)out)[b] = s;
    }
  } else if (consumer == 1) {
    __syncthreads();
    for (uint32_t i = tid; i < 256; i += nt) ((uint32_t*)out)[(uint64_t)b * 256 + i] = hist[i];
  }
  if (tid == 0) status[b] = err ? err : total;
}

// The same reads and consumers as list_reader_kernel, taken straight from a copy of the file
// in device memory instead of through gread: the GPU half of the CPU-I/O comparator, where
// host code reads the file and copies it to the GPU before the kernel runs (the paper's
// "CPU I/O" baseline, Sec. 6).
__global__ void __launch_bounds__(GFS_MAX_BLOCK_THREADS, 2) buffer_reader_kernel(const uint8_t* data, uint64_t size,
                                                                              const uint64_t* offsets, uint32_t reads,
                                                                              uint64_t read_size, int consumer,
                                                                              void* out, int64_t* status) {
  __shared__ uint32_t hist[256];
  __shared__ uint64_t red[16];
  const uint32_t b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  if (consumer == 1)
    for (uint32_t i = tid; i < 256; i += nt) hist[i] = 0;
  __syncthreads();
  int64_t total = 0;
  uint64_t csum = 0;
  for (uint32_t k = 0; k < reads; ++k) {
    const uint64_t off = offsets[(uint64_t)b * reads + k];
    if (off >= size) continue;
    const uint64_t n = read_size < size - off ? read_size : size - off;
    const uint8_t* p = data + off;
    total += (int64_t)n;
    if ((((uintptr_t)p) & 15) == 0) {
      if (consumer == 0) csum += checksum_part(p, n, tid, nt);
      else histogram_part(p, n, tid, nt, hist);
    } else if (consumer == 0) {
      for (uint64_t w = 4ull * tid; w < n; w += 4ull * nt) {
        uint32_t word = 0;
        for (int i = 0; i < 4; ++i)
          if (w + i < n) word |= (uint32_t)p[w + i] << (8 * i);
        csum += word;
      }
    } else {
      for (uint64_t j = tid; j < n; j += nt) atomicAdd(&hist[p[j]], 1u);
    }
  }
  __syncthreads();
  if (consumer == 0) {
    const uint64_t s = block_sum_u64(csum, red, tid, nt);
    if (tid == 0) ((uint64_t*)out)[b] = s;
  } else {
    for (uint32_t i = tid; i < 256; i += nt) ((uint32_t*)out)[(uint64_t)b * 256 + i] = hist[i];
  }
  if (tid == 0) status[b] = total;
}

// Persistent batch reader: blocks take units in order from one device counter; a block
// keeps its descriptor and its partial checksum/histogram while consecutive units belong
// to the same file, and adds them into that file's output row when it moves on.
__global__ void __launch_bounds__(GFS_MAX_BLOCK_THREADS, 2) batch_reader_kernel(const gfs_dev* d, const gfs_unit* units, uint64_t nunits,
                                    uint64_t* counter, uint8_t* buf, uint64_t unit_bytes,
                                    uint64_t* csum, uint32_t* hist, int64_t* status) {
  __shared__ uint32_t lhist[256];
  __shared__ uint64_t red[16];
  __shared__ uint64_t s_unit;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  uint8_t* mybuf = buf + (uint64_t)blockIdx.x * unit_bytes;
  for (uint32_t i = tid; i < 256; i += nt) lhist[i] = 0;
  int fd = -1;
  uint32_t cur_file = 0xffffffffu, cur_out = 0;
  uint64_t part = 0;
  int64_t err = 0, total = 0;
  bool dirty = false;
  while (true) {
    if (tid == 0) s_unit = __hip_atomic_fetch_add(counter, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint64_t u = s_unit;
    __syncthreads();
    if (u >= nunits) break;
    const gfs_unit un = units[u];
    if (un.file != cur_file) {
      if (dirty) {
        const uint64_t s = block_sum_u64(part, red, tid, nt);
        if (tid == 0) __hip_atomic_fetch_add(&csum[cur_out], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        for (uint32_t i = tid; i < 256; i += nt) {
          if (lhist[i]) atomicAdd(&hist[(uint64_t)cur_out * 256 + i], lhist[i]);
          lhist[i] = 0;
        }
        part = 0;
        dirty = false;
      }
      if (fd >= 0) gclose(d, fd);
      fd = gopen_id(d, (int)un.file, GFS_O_RDONLY);
      if (fd < 0) {
        err = fd;
        break;
      }
      cur_file = un.file;
      cur_out = un.out;
    }
    const int64_t r = gread(d, fd, un.offset, un.size, mybuf);
    if (r < 0) {
      err = r;
      break;
    }
    total += r;
    part += checksum_part(mybuf, (uint64_t)r, tid, nt);
    histogram_part(mybuf, (uint64_t)r, tid, nt, lhist);
    dirty = true;
    __syncthreads();
  }
  if (dirty) {
    const uint64_t s = block_sum_u64(part, red, tid, nt);
    if (tid == 0) __hip_atomic_fetch_add(&csum[cur_out], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    for (uint32_t i = tid; i < 256; i += nt)
      if (lhist[i]) atomicAdd(&hist[(uint64_t)cur_out * 256 + i], lhist[i]);
  }
  if (fd >= 0) gclose(d, fd);
  if (tid == 0) status[blockIdx.x] = err ? err : total;
}

}  // namespace

extern "C" int gfs_launch_batch(gfs_ctx* ctx, const gfs_unit* units, uint64_t nunits, uint32_t grid,
                                uint32_t threads, uint64_t unit_bytes, void* buf, uint64_t* counter,
                                uint64_t* csum, uint32_t* hist, int64_t* status, void* hip_stream) {
  if (!ctx || !units || !buf || !counter || !csum || !hist || !status) return -EINVAL;
  if (grid == 0 || grid > (1u << 20) || threads == 0 || threads % 64 || threads > GFS_MAX_BLOCK_THREADS) return -EINVAL;
  if (unit_bytes == 0 || unit_bytes % 16) return -EINVAL;
  if (((uintptr_t)buf | (uintptr_t)counter | (uintptr_t)csum) & 7) return -EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  const int rc = gfs_internal_zero(counter, 8, s);
  if (rc) return rc;
  hipLaunchKernelGGL(batch_reader_kernel, dim3(grid), dim3(threads), 0, s, gfs_device_handle(ctx), units,
                     nunits, counter, (uint8_t*)buf, unit_bytes, csum, hist, status);
  return hipGetLastError() == hipSuccess ? 0 : -EIO;
}

extern "C" int gfs_launch_buffer_reader(const void* data_dev, uint64_t data_size, const uint64_t* offsets,
                                        uint32_t blocks, uint32_t reads, uint64_t read_size, uint32_t threads,
                                        int consumer, void* out, int64_t* status, void* hip_stream) {
  if (!data_dev || !offsets || !out || !status) return -EINVAL;
  if (blocks == 0 || blocks > (1u << 20) || reads == 0) return -EINVAL;
  if (threads == 0 || threads % 64 || threads > GFS_MAX_BLOCK_THREADS) return -EINVAL;
  if (read_size == 0 || (consumer != 0 && consumer != 1)) return -EINVAL;
  if (((uintptr_t)out) & 15) return -EINVAL;
  hipLaunchKernelGGL(buffer_reader_kernel, dim3(blocks), dim3(threads), 0, (hipStream_t)hip_stream,
                     (const uint8_t*)data_dev, data_size, offsets, reads, read_size, consumer, out, status);
  return hipGetLastError() == hipSuccess ? 0 : -EIO;
}

extern "C" int gfs_batch_grid(uint32_t threads, uint32_t* grid) {
  if (!grid || threads == 0 || threads % 64 || threads > GFS_MAX_BLOCK_THREADS) return -EINVAL;
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -EIO;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_reader_kernel, (int)threads, 0) != hipSuccess)
    return -EIO;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -EIO;
  *grid = (uint32_t)(per_cu > 0 ? per_cu : 1) * (uint32_t)cus;
  return 0;
}

extern "C" int gfs_internal_purge_file(const gfs_dev* ddev, uint32_t nframes, uint64_t pt_entries, uint32_t file,
                                       hipStream_t s) {
  const uint64_t n = pt_entries > nframes ? pt_entries : nframes;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(purge_file_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, ddev, nframes, pt_entries, file);
  return hipGetLastError() == hipSuccess ? 0 : -EIO;
}

// Blocks of the list-reader kernel at `threads` threads that fit on the current device at
// once: the thrash guard's default count of blocks sharing the cache.
extern "C" int gfs_internal_resident_blocks(uint32_t threads, uint32_t* blocks) {
  int dev = 0, per_cu = 0, cus = 0;
  if (!blocks) return -EINVAL;
  if (hipGetDevice(&dev) != hipSuccess) return -EIO;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, list_reader_kernel, (int)threads, 0) != hipSuccess)
    return -EIO;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -EIO;
  *blocks = (uint32_t)(per_cu > 0 ? per_cu : 1) * (uint32_t)cus;
  return 0;
}

extern "C" int gfs_internal_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes % 8) return -EINVAL;
  const uint64_t n8 = bytes / 8;
  if (n8 == 0) return 0;
  uint64_t blocks = (n8 + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(zero_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, (uint64_t*)p, n8);
  return hipGetLastError() == hipSuccess ? 0 : -EIO;
}

extern "C" int gfs_launch_list_reader(gfs_ctx* ctx, int file_id, const uint64_t* offsets,
                                      uint32_t blocks, uint32_t reads, uint64_t read_size,
                                      uint32_t threads, int consumer, void* buf, void* out,
                                      int64_t* status, uint64_t* turn, void* hip_stream) {
  if (!ctx || !offsets || !buf || (!out && consumer != 2) || !status) return -EINVAL;
  if (blocks == 0 || blocks > (1u << 20) || reads == 0) return -EINVAL;
  if (threads == 0 || threads % 64 || threads > GFS_MAX_BLOCK_THREADS) return -EINVAL;
  if (read_size == 0 || read_size % 16) return -EINVAL;
  if (consumer < 0 || consumer > 2) return -EINVAL;
  if (((uintptr_t)buf | (uintptr_t)out) & 15) return -EINVAL;
  if (turn) {
    // the serialising gate waits on other blocks: every block must be resident at once
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, list_reader_kernel, (int)threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return -EIO;
    if ((uint64_t)blocks > (uint64_t)per_cu * (uint64_t)cus) return -EINVAL;
  }
  const gfs_dev* d = gfs_device_handle(ctx);
  hipLaunchKernelGGL(list_reader_kernel, dim3(blocks), dim3(threads), 0, (hipStream_t)hip_stream, d,
                     file_id, offsets, reads, read_size, consumer, (uint8_t*)buf, out, status, turn);
  return hipGetLastError() == hipSuccess ? 0 : -EIO;
}
