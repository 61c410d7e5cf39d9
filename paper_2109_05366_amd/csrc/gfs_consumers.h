// Benchmark consumers of delivered bytes, shared by the workload kernels: the wrapping
// u64 checksum of little-endian u32 words (a trailing partial word zero-padded), the byte
// histogram, and a block-wide sum. They are not part of the page cache.
#ifndef GFS_CONSUMERS_H
#define GFS_CONSUMERS_H

#include <hip/hip_runtime.h>

#include "gfs_device.h"

namespace gfs_consumers {

// Fold a delivered buffer into the block's consumer state.
// checksum: wrapping u64 sum of LE u32 words, a trailing partial word zero-padded.
__device__ __forceinline__ uint64_t checksum_part(const uint8_t* buf, uint64_t n, uint32_t tid,
                                                  uint32_t nt) {
  uint64_t s = 0;
  const uint64_t n16 = n >> 4;
  const gfsd::gv4u* v = (const gfsd::gv4u*)buf;   /* user buffers are global memory */
  uint64_t i = tid;
  for (; i + 7ull * nt < n16; i += 8ull * nt) {
    gfsd::v4u x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = v[i + (uint64_t)k * nt];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += (uint64_t)x[k].x + x[k].y + x[k].z + x[k].w;
  }
  for (; i + 3ull * nt < n16; i += 4ull * nt) {
    gfsd::v4u x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = v[i + (uint64_t)k * nt];
#pragma unroll
    for (int k = 0; k < 4; ++k) s += (uint64_t)x[k].x + x[k].y + x[k].z + x[k].w;
  }
  for (; i < n16; i += nt) {
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
  const gfsd::gv4u* v = (const gfsd::gv4u*)buf;
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

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* red, uint32_t tid, uint32_t nt) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  uint64_t s = 0;
  if (tid == 0)
    for (uint32_t w = 0; w < (nt + 63) / 64; ++w) s += red[w];
  return s;   /* valid in thread 0 */
}

}  // namespace gfs_consumers

#endif  // GFS_CONSUMERS_H
