// Kernels of the library: metadata zeroing and the list-reader workload that drives gread
// (the benchmark consumer: per-block checksum or byte histogram of everything delivered).
#include <errno.h>

#include <hip/hip_runtime.h>

#include "gfs.h"
#include "gfs_device.h"
#include "gfs_layout.h"

namespace {

__global__ void zero_kernel(uint64_t* p, uint64_t n8) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n8; i += stride) p[i] = 0;
}

// Fold a delivered buffer into the block's consumer state.
// checksum: wrapping u64 sum of LE u32 words, a trailing partial word zero-padded.
__device__ __forceinline__ uint64_t checksum_part(const uint8_t* buf, uint64_t n, uint32_t tid,
                                                  uint32_t nt) {
  uint64_t s = 0;
  const uint64_t n16 = n >> 4;
  const gfsd::v4u* v = (const gfsd::v4u*)buf;
  for (uint64_t i = tid; i < n16; i += nt) {
    const gfsd::v4u x = v[i];
    s += (uint64_t)x.x + x.y + x.z + x.w;
  }
  // remaining bytes (n not a multiple of 16): whole words, then the zero-padded last word
  const uint64_t rem0 = n16 << 4;
  for (uint64_t w = rem0 + 4ull * tid; w < n; w += 4ull * nt) {
    uint32_t word = 0;
    for (int b = 0; b < 4; ++b)
      if (w + b < n) word |= (uint32_t)buf[w + b] << (8 * b);
    s += word;
  }
  return s;
}

__device__ __forceinline__ void histogram_part(const uint8_t* buf, uint64_t n, uint32_t tid,
                                               uint32_t nt, uint32_t* hist) {
  const uint64_t n16 = n >> 4;
  const gfsd::v4u* v = (const gfsd::v4u*)buf;
  for (uint64_t i = tid; i < n16; i += nt) {
    const gfsd::v4u x = v[i];
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int b = 0; b < 4; ++b) atomicAdd(&hist[(w[k] >> (8 * b)) & 0xff], 1u);
  }
  for (uint64_t j = (n16 << 4) + tid; j < n; j += nt) atomicAdd(&hist[buf[j]], 1u);
}

__global__ void list_reader_kernel(const gfs_dev* d, int file_id, const uint64_t* offsets,
                                   uint32_t reads, uint64_t read_size, int consumer,
                                   uint8_t* buf, void* out, int64_t* status, uint64_t* turn) {
  __shared__ uint32_t hist[256];
  __shared__ uint64_t red[16];
  __shared__ int gate_err;
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
    const int64_t r = gread(d, fd, offsets[(uint64_t)b * reads + k], read_size, mybuf);
    if (turn && tid == 0)
      __hip_atomic_store(turn, my_turn + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (r < 0) {
      err = r;
      break;
    }
    total += r;
    if (consumer == 0) csum += checksum_part(mybuf, (uint64_t)r, tid, nt);
    else histogram_part(mybuf, (uint64_t)r, tid, nt, hist);
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
  } else {
    __syncthreads();
    for (uint32_t i = tid; i < 256; i += nt) ((uint32_t*)out)[(uint64_t)b * 256 + i] = hist[i];
  }
  if (tid == 0) status[b] = err ? err : total;
}

}  // namespace

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
  if (!ctx || !offsets || !buf || !out || !status) return -EINVAL;
  if (blocks == 0 || blocks > (1u << 20) || reads == 0) return -EINVAL;
  if (threads == 0 || threads % 64 || threads > 1024) return -EINVAL;
  if (read_size == 0 || read_size % 16) return -EINVAL;
  if (consumer != 0 && consumer != 1) return -EINVAL;
  if (((uintptr_t)buf | (uintptr_t)out) & 15) return -EINVAL;
  const gfs_dev* d = gfs_device_handle(ctx);
  hipLaunchKernelGGL(list_reader_kernel, dim3(blocks), dim3(threads), 0, (hipStream_t)hip_stream, d,
                     file_id, offsets, reads, read_size, consumer, (uint8_t*)buf, out, status, turn);
  return hipGetLastError() == hipSuccess ? 0 : -EIO;
}
