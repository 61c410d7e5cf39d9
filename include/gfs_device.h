/* gfs_device.h -- device side of the GPU file page cache: gopen / gread / gclose.
 *
 * Include from HIP code compiled for gfx950. The functions are block-collective
 * (Sec. 2.2: each threadblock issues a file call by invoking it from all of its
 * threads): every thread of the block must call them with the same arguments, and
 * every thread gets the same result. Blocks must have a multiple of 64 threads. A
 * kernel must obtain its descriptor with gopen/gopen_id before calling gread, and
 * should gclose it at the end: the block's statistics are flushed there.
 *
 *   int     gopen (const gfs_dev* d, const char* path, int flags);
 *       Resolve a path registered with gfs_open (path: NUL-terminated, device-readable
 *       memory) to a descriptor. flags must be GFS_O_RDONLY (-EROFS otherwise); an
 *       unknown path gives -ENOENT.
 *   int     gopen_id(const gfs_dev* d, int file_id, int flags);
 *       Same, from the id gfs_open returned.
 *   int64_t gread (const gfs_dev* d, int fd, uint64_t offset, uint64_t size, void* dst);
 *       Copy file bytes [offset, min(offset+size, file size)) to dst (device memory of
 *       at least that many bytes; 16-byte alignment of dst and offset takes the vector
 *       path). Returns the byte count (short only at EOF, 0 at or past it) or -EBADF,
 *       -EINVAL, -EIO (host read failed), -ENOSPC (the page's table buckets stayed full of
 *       other misses' reservations until the wait limit), -ETIMEDOUT (a wait exceeded the
 *       configured timeout; the cache must then be reset).
 *   int     gclose(const gfs_dev* d, int fd);
 *
 * How a read is served (Sec. 2.2 and Sec. 4.1): the request is divided into pages; each
 * page is looked up in the hashed page table and, on a hit, pinned and copied out. On a
 * miss the block takes the file's miss lock, asks the readahead detector for a window,
 * reserves the run of unmapped window pages around the miss in the page table, and
 * unlocks; it then gives the reserved pages frames with the clock hand (evicting in
 * place, Sec. 5.1), posts one request for the run to the host ring and waits for it
 * (synchronous prefetch, Sec. 4), pulls the fetched bytes from pinned staging into the
 * frames, publishes them, and copies its own page out. Blocks that find a page whose
 * frame is reserved or still being filled wait for it instead of fetching it again.
 *
 * Calling kernels: gread is inlined into its caller and its miss path needs about 220
 * VGPRs; give the kernel __launch_bounds__(GFS_MAX_BLOCK_THREADS) or less, or the compiler
 * caps registers lower and spills every call's state to scratch memory.
 */
#ifndef GFS_DEVICE_H
#define GFS_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gfs.h"
#include "gfs_layout.h"

namespace gfsd {

constexpr int kENOENT = 2, kEIO = 5, kEBADF = 9, kEINVAL = 22, kENOSPC = 28, kEROFS = 30,
              kETIMEDOUT = 110;
constexpr uint32_t kMaxWindow = GFS_MAX_WINDOW_PAGES;
constexpr uint64_t kFrameMask = (1ull << GFS_ENTRY_FRAME_BITS) - 1;
/* page-table entry frame value of a page reserved by a miss that has no frame yet */
constexpr uint32_t kReserved = (uint32_t)kFrameMask;

/* Per-block state in LDS, shared by gopen/gread/gclose within one kernel. */
struct BlockState {
  int64_t status;           /* 0 or -errno for the current page */
  int64_t result;           /* host read result for the request this block pulls */
  uint64_t first_page;      /* first page of the request span */
  uint64_t gen;             /* ring generation of the request */
  int32_t frame;            /* pinned frame of the current page */
  int32_t pull;             /* 1: pull this block's own request; 2: help pull one frame;
                               3: fill the frame from the private buffer; 4: pull a private-policy
                               request (page into the frame, the rest into the private buffer) */
  uint32_t slot;            /* ring slot of the request */
  uint32_t list_n;          /* pages in list[] that got frames (a prefix) */
  uint32_t file;
  int32_t open_result;
  int32_t open_fd;          /* the descriptor gopen returned last (-1: none), and its file's */
  uint64_t open_size;       /* size, read once: a registered file cannot be closed while a
                               kernel holds it open, so gread need not read them again */
  uint64_t ctr[GFS_C_COUNT];    /* block-local statistics, added to the globals by gclose */
  uint32_t list[kMaxWindow];    /* run pages: the demanded page, then the rest ascending */
  uint32_t lframe[kMaxWindow];  /* frame given to list[k], or GFS_NO_FRAME */
  uint32_t lslot[kMaxWindow];   /* page-table slot reserved for list[k] (0xffffffff: none);
                                   after allocation, the indices of the frames this block pulls */
  uint32_t nclaim;              /* entries of lslot[] claimed for pulling */
  uint32_t help_page;           /* page of the frame a helping block pulls */
  int32_t pslot;                /* private policy: the block's slot (-1: none) */
  int32_t bframe[64];           /* batched hits: frame pinned for page base + i, or -1 */
  uint32_t trig;                /* asynchronous readahead: this page access took a marker */
  uint32_t a_pending;           /* 1: this block has an asynchronous request outstanding, whose
                                   pages and frames are list[0..a_n) / lframe[0..a_n) */
  uint32_t a_slot, a_n, a_file;
  int32_t a_status;
  uint64_t a_gen, a_first;
  uint64_t tagkey;              /* nonzero: frame is pinned VALID and its tag is still to be
                                   compared with this key (the hit's copy carries the check) */
  uint64_t pinw;                /* the frame word the pin returned (for the hit's bit updates) */
  int32_t tag_ok;               /* the check's outcome, for every thread of the block */
  uint64_t read_last;           /* last page of the gread in progress: a readahead window
                                   opened by a miss covers the read up to it */
};

/* the lock queue's size assumes every block that calls gread holds this much LDS */
static_assert(sizeof(BlockState) >= GFS_BLOCK_LDS_MIN, "per-block state below the LDS bound the lock queue assumes");

__device__ __forceinline__ BlockState* block_state() {
  __shared__ BlockState gfs_block_state;
  return &gfs_block_state;
}

/* ------------------------------------------------------------------ thread / wave ids */
__device__ __forceinline__ uint32_t thread_id() {
  return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
}
__device__ __forceinline__ uint32_t block_threads() { return blockDim.x * blockDim.y * blockDim.z; }
__device__ __forceinline__ uint32_t block_id() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}
__device__ __forceinline__ uint32_t lane() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

/* ------------------------------------------------------------------ atomics (agent scope) */
__device__ __forceinline__ uint64_t ld_rlx(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_acq(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
/* Spin loops poll with relaxed loads and take one acquire fence once the awaited value is
   seen: an agent-scope acquire invalidates the XCD's L2, and hundreds of waiting blocks
   polling with acquire loads would keep every block's cached data flushed. */
__device__ __forceinline__ void acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void acquire_system() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, ""); }
/* Ordering for the miss lock's critical section, whose shared reads and writes are all
   agent-scope atomics (the detector state, the window claims, the page table, the queue
   slots): these are performed coherently across the XCDs, so passing the lock on needs
   only the holder's earlier atomics to have completed before the grant is written, and
   taking it needs only the later reads to be issued after the grant was seen. The wait
   for outstanding memory operations gives both, without the L2 write-back and
   invalidation that agent-scope fences add for plain (cached) accesses. The workgroup
   fences keep the compiler from moving memory operations across the wait. */
__device__ __forceinline__ void drain_atomics() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0x0F70);   /* vmcnt(0): every load, store and atomic done */
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
__device__ __forceinline__ uint32_t ld_rlx32(uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas64(uint64_t* p, uint64_t& expected, uint64_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_ACQ_REL,
                                              __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas64_rlx(uint64_t* p, uint64_t& expected, uint64_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas32(uint32_t* p, uint32_t& expected, uint32_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_ACQ_REL,
                                              __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t fadd64(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
/* block-local statistics: only thread 0 of the block (lane 0 of wave 0) adds */
__device__ __forceinline__ void bcount(BlockState* bs, int c, uint64_t v) { bs->ctr[c] += v; }

/* ------------------------------------------------------------------ waiting */
__device__ __forceinline__ void nap(uint32_t& n) {
  if (n < 8) __builtin_amdgcn_s_sleep(2);
  else if (n < 64) __builtin_amdgcn_s_sleep(16);
  else __builtin_amdgcn_s_sleep(127);
  ++n;
}
/* shorter naps for the miss lock, whose holder keeps it for a few microseconds */
__device__ __forceinline__ void nap_short(uint32_t& n) {
  if (n < 16) __builtin_amdgcn_s_sleep(2);
  else __builtin_amdgcn_s_sleep(24);
  ++n;
}
__device__ __forceinline__ bool expired(const gfs_dev* d, uint64_t t0) {
  return wall_clock64() - t0 > d->timeout_ticks;
}

/* ------------------------------------------------------------------ trace */
__device__ __forceinline__ void trace_ev(const gfs_dev* d, uint32_t level, uint32_t op,
                                         uint32_t block, uint32_t file, uint32_t page,
                                         uint32_t frame, uint32_t a, uint64_t b) {
  if (d->trace_level < level) return;
  const uint64_t i = fadd64(&d->g->trace_n, 1);
  if (i >= d->trace_cap) return;
  gfs_event* e = ((gfs_event*)d->trace) + i;
  e->op = op;
  e->block = block;
  e->file = file;
  e->page = page;
  e->frame = frame;
  e->a = a;
  e->b = b;
}

/* ------------------------------------------------------------------ hashed page table
 * Two candidate buckets of 16 entries (128 B) per key; an entry is key<<24 | frame and is
 * changed only by atomics. Lookups take no lock. A file's keys are inserted only under
 * that file's miss lock, first as reservations (frame field kReserved), so one key is never
 * inserted twice; the reserving block later stores the frame into its own entry, or
 * clears it. An evicting block clears the entry of the frame it claimed. */
__device__ __forceinline__ uint64_t page_key(uint32_t file, uint64_t page) {
  return ((uint64_t)(file + 1) << GFS_KEY_PAGE_BITS) | page;
}
__device__ __forceinline__ uint64_t key_hash(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}
__device__ __forceinline__ void key_buckets_m(uint32_t mask, uint64_t key, uint32_t& b1, uint32_t& b2) {
  const uint64_t h = key_hash(key);
  b1 = (uint32_t)h & mask;
  b2 = (uint32_t)(h >> 32) & mask;
  if (b2 == b1) b2 = b1 ^ 1u;
}
__device__ __forceinline__ void key_buckets(const gfs_dev* d, uint64_t key, uint32_t& b1,
                                            uint32_t& b2) {
  key_buckets_m(d->nbuckets_mask, key, b1, b2);
}
__device__ __forceinline__ uint64_t* slot_ptr(const gfs_dev* d, uint32_t b1, uint32_t b2, int i) {
  return d->pt + (uint64_t)(i < GFS_BUCKET_SLOTS ? b1 : b2) * GFS_BUCKET_SLOTS + (i & 15);
}

/* wave-collective: lanes 0-15 read bucket 1, lanes 16-31 bucket 2; uniform result: the
 * frame, kReserved, or -1 when absent */
__device__ __forceinline__ int32_t pt_lookup_at(uint64_t* pt, uint32_t mask, uint64_t key) {
  uint32_t b1, b2;
  key_buckets_m(mask, key, b1, b2);
  const uint32_t l = lane();
  uint64_t e = 0;
  if (l < 32) e = ld_rlx(pt + (uint64_t)(l < GFS_BUCKET_SLOTS ? b1 : b2) * GFS_BUCKET_SLOTS + (l & 15));
  const uint64_t m = __ballot(l < 32 && (e >> GFS_ENTRY_FRAME_BITS) == key);
  if (m == 0) return -1;
  const uint64_t hit = __shfl(e, __ffsll((unsigned long long)m) - 1, 64);
  return (int32_t)(hit & kFrameMask);
}
__device__ int32_t pt_lookup_wave(const gfs_dev* d, uint64_t key) {
  return pt_lookup_at(d->pt, d->nbuckets_mask, key);
}

/* per lane: the 32 candidate entries of a key, loaded together (one round trip) */
__device__ __forceinline__ void pt_load_lane(const gfs_dev* d, uint32_t b1, uint32_t b2,
                                             uint64_t e[2 * GFS_BUCKET_SLOTS]) {
#pragma unroll
  for (int i = 0; i < 2 * GFS_BUCKET_SLOTS; ++i) e[i] = ld_rlx(slot_ptr(d, b1, b2, i));
}

/* per lane: true if key has an entry (a frame or a reservation) */
__device__ bool pt_present_lane(const gfs_dev* d, uint64_t key) {
  uint32_t b1, b2;
  key_buckets(d, key, b1, b2);
  uint64_t e[2 * GFS_BUCKET_SLOTS];
  pt_load_lane(d, b1, b2, e);
  bool hit = false;
#pragma unroll
  for (int i = 0; i < 2 * GFS_BUCKET_SLOTS; ++i) hit |= (e[i] >> GFS_ENTRY_FRAME_BITS) == key;
  return hit;
}

/* per lane: the frame key maps to, kReserved, or -1 when absent */
__device__ int32_t pt_find_lane(const gfs_dev* d, uint64_t key) {
  uint32_t b1, b2;
  key_buckets(d, key, b1, b2);
  uint64_t e[2 * GFS_BUCKET_SLOTS];
  pt_load_lane(d, b1, b2, e);
  int32_t f = -1;
#pragma unroll
  for (int i = 0; i < 2 * GFS_BUCKET_SLOTS; ++i)
    if ((e[i] >> GFS_ENTRY_FRAME_BITS) == key) f = (int32_t)(e[i] & kFrameMask);
  return f;
}

/* per lane, under key's file lock: reserve key; returns the global slot index or -1 if
 * both buckets are full */
__device__ int64_t pt_reserve_lane(const gfs_dev* d, uint64_t key) {
  const uint64_t ent = (key << GFS_ENTRY_FRAME_BITS) | kReserved;
  uint32_t b1, b2;
  key_buckets(d, key, b1, b2);
  for (int attempt = 0; attempt < 256; ++attempt) {
    uint64_t e[2 * GFS_BUCKET_SLOTS];
    pt_load_lane(d, b1, b2, e);
    int cnt1 = 0, cnt2 = 0, f1 = -1, f2 = -1;
#pragma unroll
    for (int i = 0; i < GFS_BUCKET_SLOTS; ++i) {
      if (e[i]) ++cnt1;
      else if (f1 < 0) f1 = i;
      if (e[GFS_BUCKET_SLOTS + i]) ++cnt2;
      else if (f2 < 0) f2 = GFS_BUCKET_SLOTS + i;
    }
    int pick = cnt2 < cnt1 ? f2 : f1;   /* less loaded bucket, ties to the first */
    if (pick < 0) pick = f1 >= 0 ? f1 : f2;
    if (pick < 0) return -1;
    uint64_t expect = 0;
    uint64_t* sp = slot_ptr(d, b1, b2, pick);
    if (cas64_rlx(sp, expect, ent)) return (int64_t)(sp - d->pt);
  }
  return -1;
}

/* per lane: clear the entry key -> frame (the caller owns it) */
__device__ bool pt_delete_lane(const gfs_dev* d, uint64_t key, uint32_t frame) {
  const uint64_t ent = (key << GFS_ENTRY_FRAME_BITS) | frame;
  uint32_t b1, b2;
  key_buckets(d, key, b1, b2);
  uint64_t e[2 * GFS_BUCKET_SLOTS];
  pt_load_lane(d, b1, b2, e);
  int at = -1;
#pragma unroll
  for (int i = 0; i < 2 * GFS_BUCKET_SLOTS; ++i)
    if (at < 0 && e[i] == ent) at = i;
  if (at < 0) return false;
  uint64_t expect = ent;
  return cas64_rlx(slot_ptr(d, b1, b2, at), expect, 0ull);
}

/* ------------------------------------------------------------------ frame words */
enum { PIN_RETRY = 0, PIN_VALID = 1, PIN_FILLING = 2, PIN_ERROR = 3, PIN_VALID_UNCHECKED = 4 };

/* Pins are counted with fetch-and-add and fetch-and-subtract, so a pin costs one atomic
 * round trip and dropping one costs none (the wave does not wait for it). Every other change
 * of a frame word is a compare-and-swap against the word just read, or an addition (the
 * allocator's CLAIMED -> FILLING step), so a pin taken and dropped at any moment is never
 * lost: a block that pins a frame which turns out not to hold its page (or is not FILLING
 * or VALID) just drops the pin again. The clock hand claims only frames with no pins. */

/* Drop a pin. Relaxed: the caller's reads of the frame have completed (a block barrier
 * waits for them) before this is issued, and unpinning publishes nothing. */
/* ------------------------------------------------------------------ evicted-after-use bits
 * One bit per page of a file: set when the clock evicts the page after it was consumed (its
 * prefetch mark cleared by a pin, or it was the demanded page). A window leaves such pages
 * out of its run, unless the demanded page (the marker page, for an asynchronous window) is
 * one of them: a page a reader consumed and the cache dropped lies behind that reader, and a
 * demanded one means the file is being read again. */
__device__ __forceinline__ uint64_t* shadow_word(const gfs_dev* d, uint32_t file, uint64_t q) {
  return d->shadow + (uint64_t)file * (GFS_SHADOW_PAGES / 64) + (q >> 6);
}
__device__ __forceinline__ bool shadow_lane(const gfs_dev* d, uint32_t file, uint64_t q) {
  if (q >= GFS_SHADOW_PAGES) return false;
  return ((ld_rlx(shadow_word(d, file, q)) >> (q & 63)) & 1ull) != 0;
}
__device__ __forceinline__ void shadow_set_lane(const gfs_dev* d, uint32_t file, uint64_t q) {
  if (q < GFS_SHADOW_PAGES)
    __hip_atomic_fetch_or(shadow_word(d, file, q), 1ull << (q & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void frame_unpin(const gfs_dev* d, uint32_t f) {
  __hip_atomic_fetch_sub(&d->fword[f], GFS_FW_PIN_ONE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

/* Pin frame f if it is filling or valid and still holds key; sets the reference bit and
 * clears the prefetched mark (the page has now been demanded). Acquire: a valid frame's
 * bytes, published with release by the block that filled it, are visible afterwards, and
 * the tag is read after the pin is in place (a frame cannot be claimed while pinned). */
__device__ int frame_pin(const gfs_dev* d, uint32_t f, uint64_t key, uint64_t* w_out = nullptr) {
  uint64_t* fw = &d->fword[f];
  const uint64_t w = __hip_atomic_fetch_add(fw, GFS_FW_PIN_ONE, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  if (w_out) *w_out = w;
  const uint64_t st = w & GFS_FW_STATE;
  if ((st != GFS_FS_FILLING && st != GFS_FS_VALID) || ld_rlx(&d->ftag[f]) != key) {
    frame_unpin(d, f);
    return PIN_RETRY;
  }
  if (st == GFS_FS_VALID && (w & GFS_FW_ERR)) {
    frame_unpin(d, f);   /* the host read of this page failed */
    return PIN_ERROR;
  }
  /* idempotent bit updates; the wave does not wait for them */
  if (!(w & GFS_FW_REF))
    __hip_atomic_fetch_or(fw, GFS_FW_REF, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (w & GFS_FW_RA)
    __hip_atomic_fetch_and(fw, ~GFS_FW_RA, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return st == GFS_FS_VALID ? PIN_VALID : PIN_FILLING;
}

/* The bit updates of a demand pin: set the reference bit, clear the prefetched mark (the page
   has now been demanded). Idempotent; the wave does not wait for them. */
__device__ __forceinline__ void frame_pin_bits(const gfs_dev* d, uint32_t f, uint64_t w) {
  uint64_t* fw = &d->fword[f];
  if (!(w & GFS_FW_REF))
    __hip_atomic_fetch_or(fw, GFS_FW_REF, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (w & GFS_FW_RA)
    __hip_atomic_fetch_and(fw, ~GFS_FW_RA, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

/* Pin frame f for a hit whose tag comparison travels with the copy: a VALID frame without
 * the error bit is left pinned and reported PIN_VALID_UNCHECKED (w receives the word the pin
 * returned); the caller loads the frame's tag together with the first loads of its copy and
 * keeps the copy only if the tag is key (a pinned frame cannot be claimed, so the tag read
 * after the pin is the one the bytes belong to), then applies frame_pin_bits. Any other state
 * goes through frame_pin's checks. Saves frame_pin's dependent tag load on every hit. */
__device__ int frame_pin_fast(const gfs_dev* d, uint32_t f, uint64_t key, uint64_t& w_out) {
  uint64_t* fw = &d->fword[f];
  const uint64_t w = __hip_atomic_fetch_add(fw, GFS_FW_PIN_ONE, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  w_out = w;
  const uint64_t st = w & GFS_FW_STATE;
  if (st == GFS_FS_VALID && !(w & GFS_FW_ERR)) return PIN_VALID_UNCHECKED;
  if ((st != GFS_FS_FILLING && st != GFS_FS_VALID) || ld_rlx(&d->ftag[f]) != key) {
    frame_unpin(d, f);
    return PIN_RETRY;
  }
  if (st == GFS_FS_VALID) {
    frame_unpin(d, f);   /* the host read of this page failed */
    return PIN_ERROR;
  }
  frame_pin_bits(d, f, w);
  return PIN_FILLING;
}

/* Lane: the pinned frame's word showed the marker bit; clear it. True for the one block whose
   clearing took it (that block advances the stream). */
__device__ __forceinline__ bool mark_take_lane(const gfs_dev* d, uint32_t f) {
  const uint64_t old = __hip_atomic_fetch_and(&d->fword[f], ~GFS_FW_MARK, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return (old & GFS_FW_MARK) != 0;
}

/* One clock step at frame f (per lane). FREE or EVICT leave the frame CLAIMED by the
 * caller; EVICT reports the victim's key and prefetched mark. `seen` receives what the step
 * decided on, for the trace: the reference bit << 1 | pinned << 2 | lost race << 3 |
 * state << 4 (the word was read, then a compare-and-swap against it failed: SKIP). */
__device__ int hand_visit(const gfs_dev* d, uint32_t f, uint64_t& vkey, uint32_t& vra, uint32_t& seen) {
  uint64_t* fw = &d->fword[f];
  uint64_t w = ld_rlx(fw);
  const uint64_t tag = ld_rlx(&d->ftag[f]);   /* loaded with the word; used only on EVICT */
  const uint64_t st = w & GFS_FW_STATE;
  const uint64_t claimed = (((w >> GFS_FW_VER_SHIFT) + 1) << GFS_FW_VER_SHIFT) | GFS_FS_CLAIMED;
  seen = ((w & GFS_FW_REF) ? 2u : 0u) | ((w & GFS_FW_PINS) ? 4u : 0u) | ((uint32_t)st << 4);
  if (w & GFS_FW_PINS) return GFS_HAND_SKIP;
  if (st == GFS_FS_FREE) {
    if (cas64(fw, w, claimed)) return GFS_HAND_FREE;
    seen |= 8u;
    return GFS_HAND_SKIP;
  }
  if (st != GFS_FS_VALID) return GFS_HAND_SKIP;
  if (w & GFS_FW_REF) {
    if (cas64_rlx(fw, w, (w & ~GFS_FW_REF) + GFS_FW_VER_ONE)) return GFS_HAND_CLEAR;
    seen |= 8u;
    return GFS_HAND_SKIP;
  }
  const uint64_t old = w;
  if (!cas64(fw, w, claimed)) {
    seen |= 8u;
    return GFS_HAND_SKIP;
  }
  /* the tag read with the word is still the frame's: a tag is rewritten only by the block
     that claims the frame, and the CAS just succeeded against the word read with it */
  vkey = tag;
  vra = (old & GFS_FW_RA) ? 1u : 0u;
  return GFS_HAND_EVICT;
}

/* Wait (lane) until the pinned frame f is VALID. 0, -EIO or -ETIMEDOUT (pin dropped on error). */
__device__ int64_t wait_valid_lane(const gfs_dev* d, uint32_t f, uint64_t t0) {
  uint32_t n = 0;
  while (true) {
    const uint64_t w = ld_rlx(&d->fword[f]);
    if ((w & GFS_FW_STATE) == GFS_FS_VALID) {
      acquire_agent();   /* the frame's bytes, published before VALID */
      if (w & GFS_FW_ERR) {
        frame_unpin(d, f);
        return -kEIO;
      }
      return 0;
    }
    if (expired(d, t0)) {
      frame_unpin(d, f);
      return -kETIMEDOUT;
    }
    nap(n);
  }
}

/* ------------------------------------------------------------------ per-file miss lock
 * A FIFO ticket lock whose waiters can leave the queue. Blocks get the lock in ticket
 * order, which keeps the readers of a file together (an unfair lock lets a few blocks run
 * far ahead and spreads the misses over the whole file). Each ticket has a 64-bit queue
 * slot (GFS_LOCK_SLOTS per file, more than the blocks the device can hold at once). A
 * waiter announces the page it missed in its slot ("waiting n, page"); the holder passes
 * the lock by writing "granted n" into the slot of ticket n. A waiter whose page appears
 * in the table while it waits (another block's window covered it) writes "left n" instead,
 * by compare-and-swap against the grant, and goes to the pin path. A holder that has just
 * claimed a window marks the waiters right behind it whose pages lie in that window
 * "covered n" (their pages are about to be reserved, so the lock has nothing to decide for
 * them) and passes the lock to the first ticket that is neither left nor covered. Ticket 0
 * of a cold file holds the lock at once. The low word of every slot value carries the
 * ticket, so stale values of earlier tickets never match. */

enum { LOCK_OWN = 0, LOCK_LEFT = 1, LOCK_TIMEOUT = 2, LOCK_COVERED = 3 };

__device__ __forceinline__ uint64_t lock_granted(uint64_t n) { return (uint64_t)(((uint32_t)n << 2) | 1u); }
__device__ __forceinline__ uint64_t lock_left(uint64_t n) { return (uint64_t)(((uint32_t)n << 2) | 2u); }
__device__ __forceinline__ uint64_t lock_covered(uint64_t n) { return (uint64_t)(((uint32_t)n << 2) | 3u); }
__device__ __forceinline__ uint64_t lock_waiting(uint64_t n, uint64_t page) {
  return (1ull << 63) | (page << 32) | (uint64_t)((uint32_t)n << 2);
}
__device__ __forceinline__ uint64_t* lock_slot(const gfs_dev* d, uint32_t file, uint64_t n) {
  return d->lockq + (uint64_t)file * GFS_LOCK_SLOTS + (n & (GFS_LOCK_SLOTS - 1));
}

/* Lane 0: leave the queue if ticket t is not granted yet; true if it is out of the queue
   (left, or marked covered by the holder), false if the lock was granted meanwhile (then
   the caller holds it). */
__device__ bool lock_try_leave_lane(const gfs_dev* d, uint32_t file, uint64_t t) {
  uint64_t* sl = lock_slot(d, file, t);
  uint64_t v = __hip_atomic_load(sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (v != lock_granted(t)) {
    if (v == lock_covered(t)) return true;
    if (__hip_atomic_compare_exchange_strong(sl, &v, lock_left(t), __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return true;
  }
  return false;
}

/* Wave-collective. Waits for the file's miss lock for page `page` (key `key`); while
 * waiting, looks up `key` in the table now and then and leaves the queue if it appeared.
 * Returns LOCK_OWN (ticket set), LOCK_LEFT, LOCK_COVERED (the holder's window covers the
 * page) or LOCK_TIMEOUT (left the queue after the wait timeout). */
__device__ int lock_file_wave(const gfs_dev* d, uint32_t file, uint64_t key, uint64_t page, uint64_t t0,
                              uint64_t& ticket, bool may_leave = true);
/* Wave-collective: pass the lock on; [lo, hi) is the window the holder has just claimed
   (lo == hi: none). has_pre: lane l's `pre` is the value of the slot of ticket + 1 + l, read
   earlier under the lock, and the first look uses it instead of reading the slots again. */
__device__ void unlock_file_wave(const gfs_dev* d, uint32_t file, uint64_t ticket, uint64_t lo, uint64_t hi,
                                 bool has_pre = false, uint64_t pre = 0);

__device__ int32_t pt_lookup_wave(const gfs_dev* d, uint64_t key);

__device__ int lock_file_wave(const gfs_dev* d, uint32_t file, uint64_t key, uint64_t page, uint64_t t0,
                              uint64_t& ticket, bool may_leave) {
  uint64_t t = 0;
  if (lane() == 0)
    t = __hip_atomic_fetch_add(&d->locks[file].next, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  t = __shfl(t, 0, 64);
  ticket = t;
  int res = LOCK_OWN;
  if (t != 0) {
    uint64_t* sl = lock_slot(d, file, t);
    /* announce the page, unless the grant is already there */
    int own = 0;
    if (lane() == 0) {
      uint64_t v = __hip_atomic_load(sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      while (v != lock_granted(t)) {
        if (__hip_atomic_compare_exchange_strong(sl, &v, lock_waiting(t, page), __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          break;
      }
      own = v == lock_granted(t) ? 1 : 0;
    }
    own = __shfl(own, 0, 64);
    for (uint32_t n = 0; !own; ++n) {
      int st = -1;   /* -1: keep waiting */
      if (lane() == 0) {
        const uint64_t v = __hip_atomic_load(sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v == lock_granted(t)) st = LOCK_OWN;
        else if (v == lock_covered(t)) st = LOCK_COVERED;
      }
      st = __shfl(st, 0, 64);
      if (st < 0 && (n & 7) == 7) {
        /* the page may have been reserved by a window that covers it */
        const bool present = may_leave && pt_lookup_wave(d, key) >= 0;
        const bool late = expired(d, t0);
        if (present || late) {
          int out = 0;
          if (lane() == 0) out = lock_try_leave_lane(d, file, t) ? 1 : 0;
          out = __shfl(out, 0, 64);
          st = out ? (present ? LOCK_LEFT : LOCK_TIMEOUT) : LOCK_OWN;
        }
      }
      if (st >= 0) {
        res = st;
        break;
      }
      if (lane() == 0) {
        if (n < 64) __builtin_amdgcn_s_sleep(2);
        else __builtin_amdgcn_s_sleep(16);
      }
    }
  }
  drain_atomics();
  return res;
}

/* Wave-collective: pass the lock to the first later ticket that is still waiting for it
 * and whose page is outside [lo, hi). Without a window the next ticket gets the grant by
 * one exchange, and only if that waiter had left does the wave read the following slots,
 * 64 at a time, for the first ticket still in the queue. With a window the wave reads the
 * slots first: tickets that left or were marked covered are passed over, waiting tickets
 * whose announced page lies in the window are marked covered (a compare-and-swap that
 * loses only to the waiter leaving), and the first other ticket gets the grant; if that
 * waiter left just before the exchange, the scan goes on after it. A ticket that has not
 * announced its page yet is granted the lock like any other. */
/* lq: the file's queue slots, ticket n in lq[n mod GFS_LOCK_SLOTS] */
__device__ void unlock_slots_wave(uint64_t* lq, uint64_t ticket, uint64_t lo, uint64_t hi, bool has_pre,
                                  uint64_t pre) {
  drain_atomics();
  const uint32_t l = lane();
  uint64_t n = ticket + 1;
  bool look = hi > lo;
  while (true) {
    if (look) {
      const uint64_t nl = n + l;
      uint64_t* sl = lq + (nl & (GFS_LOCK_SLOTS - 1));
      uint64_t v = has_pre && n == ticket + 1 ? pre : ld_rlx(sl);
      const uint64_t pg = (v >> 32) & 0x7fffffffull;
      const bool gone = v == lock_left(nl) || v == lock_covered(nl);
      const bool cov = hi > lo && (v >> 63) && (uint32_t)v == ((uint32_t)nl << 2) && pg >= lo && pg < hi;
      const uint64_t skip = __ballot(gone || cov);
      const uint32_t first = ~skip ? (uint32_t)__builtin_ctzll(~skip) : 64u;
      if (cov && l < first) {
        /* loses only to the waiter leaving, which takes it out of the queue as well */
        (void)__hip_atomic_compare_exchange_strong(sl, &v, lock_covered(nl), __ATOMIC_RELAXED,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (first == 64) {
        n += 64;
        continue;
      }
      n += first;
    }
    uint64_t old = 0;
    if (l == 0)
      old = __hip_atomic_exchange(lq + (n & (GFS_LOCK_SLOTS - 1)), lock_granted(n), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
    old = __shfl(old, 0, 64);
    if (old != lock_left(n)) return;
    ++n;   /* that waiter had left: look for the next one still in the queue */
    look = true;
  }
}
/* the same, given the file instead of its queue slots */
__device__ void unlock_file_wave(const gfs_dev* d, uint32_t file, uint64_t ticket, uint64_t lo, uint64_t hi,
                                 bool has_pre, uint64_t pre) {
  unlock_slots_wave(d->lockq + (uint64_t)file * GFS_LOCK_SLOTS, ticket, lo, hi, has_pre, pre);
}

/* ------------------------------------------------------------------ readahead detector
 * Wave-collective, under the file's miss lock. Streams live in the file record; lane i
 * looks at stream slot i. Sec. 2.3 (Linux readahead: per-descriptor sequential streams,
 * window doubled up to a maximum, several interleaved readers followed on one file) and
 * Sec. 4 (GPU-side window, RANDOM hint disables it). A miss inside a stream's zone
 * [next, next+size) doubles that stream's window. Otherwise a new stream replaces an empty
 * or the least recently used slot: if several of the file's recent misses are near p the
 * file is being read in aggregate by many blocks and the window is the cap-sized aligned
 * chunk around p; else the history of cached pages right behind p sizes it (context
 * readahead); with neither, it opens with the initial window at offset 0 or under
 * SEQUENTIAL advice, else with one page. The context rule needs more cached history than
 * the req pages from p to the end of the read that missed (a shorter one may be a random
 * read next to cached pages), and a context or new window covers at least those req pages
 * (Sec. 2.3: the prefetcher reads at least what the caller asked for), up to the cap. */
/* Per lane: the file's detector state, loaded together (lane i: recent miss i, stream
   slot i); the decision below uses it after the caller's acquire fence. */
struct RaState {
  uint32_t advice, clk, rn;
  uint64_t r, s_next;
  uint32_t s_size, s_last, s_valid, s_marker;
};
__device__ __forceinline__ RaState ra_load_lane(gfs_file_dev* fe, uint32_t nrec, uint32_t nstreams) {
  const uint32_t l = lane();
  RaState st{};
  st.advice = ld_rlx32(&fe->advice);
  if (l == 0) st.clk = ld_rlx32(&fe->clock);
  st.rn = ld_rlx32(&fe->recent_n);
  if (l < nrec) st.r = ld_rlx(&fe->recent[l]);
  if (l < nstreams) {
    gfs_stream* sp = &fe->streams[l];
    st.s_next = ld_rlx(&sp->next);
    st.s_size = ld_rlx32(&sp->size);
    st.s_last = ld_rlx32(&sp->last_use);
    st.s_valid = ld_rlx32(&sp->valid);
    st.s_marker = ld_rlx32(&sp->marker);
  }
  return st;
}

/* Which rule decided a window (GFS_RA_RULE_*, recorded in the trace with the detector's inputs). */
enum { RA_RULE_OFF = GFS_RA_RULE_OFF, RA_RULE_ZONE = GFS_RA_RULE_ZONE, RA_RULE_AGGREGATE = GFS_RA_RULE_AGGREGATE,
       RA_RULE_CONTEXT = GFS_RA_RULE_CONTEXT, RA_RULE_NEW = GFS_RA_RULE_NEW };

/* The largest window a decision may take: the configured cap, clipped to the share of the
   cache one resident block may hold (Sec. 5.1's quota: cache pages over the blocks reading at
   once, the smaller of the launch's grid and the configured resident count), so that the
   windows of all resident readers together do not exceed the cache. */
__device__ __forceinline__ uint32_t ra_cap_eff(const gfs_dev* d) {
  const uint64_t grid = (uint64_t)gridDim.x * gridDim.y * gridDim.z;
  const uint64_t r = grid < d->ra_quota_blocks ? grid : d->ra_quota_blocks;
  uint64_t q = d->nframes / (r ? r : 1);
  if (q < 1) q = 1;
  return d->ra_cap < q ? d->ra_cap : (uint32_t)q;
}

/* The detector's constants, read before a block takes the miss lock, so that the holder's
   decision waits on no load of them. */
struct RaParams {
  uint32_t cap, nrec, nstreams, near_min, init;
  uint64_t radius;
};
__device__ __forceinline__ RaParams ra_params(const gfs_dev* d) {
  RaParams q;
  q.cap = ra_cap_eff(d);
  q.nrec = d->ra_recent;
  q.nstreams = d->streams;
  q.near_min = d->ra_near_min;
  q.init = d->ra_init;
  q.radius = d->ra_near_pages;
  return q;
}

/* Wave-collective: how many consecutive pages right behind p are in the table (64 per round),
 * up to max(ceil(cap / 2), min(req, cap) + 1): enough to tell whether the history is longer
 * than the read that missed (req pages from p), and to size a context window min(2h, cap).
 * The miss path counts them before it takes the file's miss lock, while it would wait
 * anyway, so the lock's holder probes no table entries for this: the count is the table as
 * the block saw it when it missed (with accesses made one at a time, the same as under the
 * lock), and the decision uses it alone. */
__device__ uint32_t ra_history_wave(const gfs_dev* d, uint32_t file, uint64_t p, uint32_t req) {
  const uint32_t l = lane();
  const uint32_t cap = ra_cap_eff(d);
  const uint32_t r = req < cap ? req : cap;
  const uint32_t hmax = (cap + 1) / 2 > r + 1 ? (cap + 1) / 2 : r + 1;
  uint32_t h = 0;
  while (h < hmax) {
    const uint64_t back = (uint64_t)h + 1 + l;
    bool mapped = false;
    if (back <= p && h + l < hmax) mapped = pt_present_lane(d, page_key(file, p - back));
    const uint64_t m = __ballot(mapped);
    const uint32_t run = (~m == 0ull) ? 64u : (uint32_t)__builtin_ctzll(~m);
    h += run;
    if (run < 64) break;
  }
  return h < hmax ? h : hmax;
}

__device__ void ra_decide_wave(gfs_file_dev* fe, uint64_t p, uint32_t req, uint32_t hist,
                               const RaParams& rp, const RaState& st, uint64_t& ws, uint32_t& wn, uint32_t& near_out,
                               uint32_t& h_out, uint32_t& rule_out, int& slot_out) {
  const uint32_t advice = st.advice;
  ws = p;
  wn = 1;
  near_out = 0;
  h_out = 0;
  rule_out = RA_RULE_OFF;
  slot_out = -1;
  if (rp.cap == 0 || advice == GFS_ADV_RANDOM) return;
  const uint32_t l = lane();
  const uint32_t cap = rp.cap;
  const uint32_t nrec = rp.nrec;
  uint32_t clk = st.clk;
  const uint32_t rn = st.rn;
  const uint64_t r = st.r;
  const uint64_t s_next = st.s_next;
  const uint32_t s_size = st.s_size, s_last = st.s_last, s_valid = st.s_valid;
  clk = __shfl(clk, 0, 64) + 1;
  /* how many of the file's last misses lie near p; then remember p */
  const uint64_t radius = rp.radius;
  const bool near_l = l < nrec && l < rn && r + radius >= p && r <= p + radius;
  const uint32_t near = (uint32_t)__popcll(__ballot(near_l));
  near_out = near;
  if (l == 0) {
    st_rlx32(&fe->clock, clk);
    st_rlx(&fe->recent[rn % nrec], p);
    st_rlx32(&fe->recent_n, rn + 1);
  }
  const bool cov = l < rp.nstreams && s_valid && s_next <= p && p < s_next + s_size;
  const uint64_t cm = __ballot(cov);
  int j;
  if (cm) {
    /* p is inside a stream's zone: double that stream's window from its frontier */
    j = __ffsll((unsigned long long)cm) - 1;
    const uint64_t nx = __shfl(s_next, j, 64);
    const uint32_t sz = __shfl(s_size, j, 64);
    ws = nx;
    wn = 2 * sz < cap ? 2 * sz : cap;
    rule_out = RA_RULE_ZONE;
  } else {
    const uint64_t inv = __ballot(l < rp.nstreams && !s_valid);
    if (inv) {
      j = __ffsll((unsigned long long)inv) - 1;
    } else {
      uint64_t k = l < rp.nstreams ? (((uint64_t)s_last << 8) | l) : ~0ull;
      for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(k, off, 64);
        k = o < k ? o : k;
      }
      j = (int)(k & 0xff);
    }
    if (near >= rp.near_min) {
      /* many blocks missing close together: the file is read in aggregate (interleaved
         strides); take the cap-sized chunk aligned around p */
      wn = cap;
      ws = p - p % cap;
      rule_out = RA_RULE_AGGREGATE;
    } else {
      /* context: the consecutive cached pages right behind p (hist, counted by
         ra_history_wave); a stream that no slot tracks shows up as that history */
      const uint32_t h = hist;
      /* a history no longer than the read itself may be chance (a random read next to
         cached pages): only a longer one makes p a stream's continuation. Either way the
         window covers at least the rest of the read that missed (req pages from p), as a
         read larger than a page asks for them all */
      const uint32_t r = req < cap ? req : cap;
      uint32_t w0;
      if (h > r) {
        w0 = 2 * h;
        rule_out = RA_RULE_CONTEXT;
      } else {
        w0 = (p == 0 || advice == GFS_ADV_SEQUENTIAL) ? rp.init : 1u;
        rule_out = RA_RULE_NEW;
      }
      if (w0 < r) w0 = r;
      if (w0 > cap) w0 = cap;
      if (w0 < 1) w0 = 1;
      ws = p;
      wn = w0;
      h_out = h;
    }
  }
  if (l == 0) {
    gfs_stream* s = &fe->streams[j];
    st_rlx(&s->next, ws + wn);
    st_rlx32(&s->size, wn);
    st_rlx32(&s->last_use, clk);
    st_rlx32(&s->valid, 1u);
  }
  slot_out = j;
}

/* ------------------------------------------------------------------ clock allocation
 * Wave-collective, outside the miss lock. Gives frames to bs->list[0..n) in order: each
 * round takes as many consecutive hand tickets as pages remain, visits those frames in
 * parallel, and hands the k-th successful ticket to the next unserved page, which is the
 * order a one-at-a-time hand would produce. Each page that gets a frame is tagged, made
 * FILLING (pinned for the demanded page, marked prefetched otherwise) and its reserved
 * table entry is pointed at the frame. Returns how many pages got frames (a prefix of the
 * list); stops after 2 * nframes visits without enough frames. */
__device__ uint32_t alloc_wave(const gfs_dev* d, uint32_t file, uint64_t demand, BlockState* bs,
                               uint32_t n, uint32_t bid, uint64_t mark = ~0ull) {
  const uint32_t l = lane();
  uint32_t assigned = 0;
  uint64_t visits = 0;
  uint32_t evicted = 0, wasted = 0;
  const uint64_t limit = 2ull * d->nframes;
  while (assigned < n && visits < limit) {
    const uint32_t need = (n - assigned) < 64u ? (n - assigned) : 64u;
    uint64_t base = 0;
    if (l == 0) base = fadd64(&d->g->hand, need);
    base = __shfl(base, 0, 64);
    int act = -1;
    uint32_t f = 0;
    uint64_t vkey = 0;
    uint32_t vra = 0, seen = 0;
    const uint64_t t = base + l;
    if (l < need) {
      f = (uint32_t)(t % d->nframes);
      act = hand_visit(d, f, vkey, vra, seen);
      if (act == GFS_HAND_EVICT) {
        const uint32_t vf = (uint32_t)(vkey >> GFS_KEY_PAGE_BITS) - 1u;
        const uint32_t vp = (uint32_t)(vkey & ((1ull << GFS_KEY_PAGE_BITS) - 1));
        trace_ev(d, 1, GFS_EV_HAND, bid, vf, vp, f, GFS_HAND_EVICT | (vra << 8) | (seen << 8), t);
      } else {
        trace_ev(d, 1, GFS_EV_HAND, bid, 0xffffffffu, 0xffffffffu, f, (uint32_t)act | (seen << 8), t);
      }
    }
    const bool ok = (act == GFS_HAND_FREE || act == GFS_HAND_EVICT);
    const uint64_t sm = __ballot(ok);
    evicted += (uint32_t)__popcll(__ballot(act == GFS_HAND_EVICT));
    wasted += (uint32_t)__popcll(__ballot(act == GFS_HAND_EVICT && vra));
    if (ok) {
      const uint32_t k = assigned + (uint32_t)__popcll(sm & lanemask_lt());
      const uint64_t q = bs->list[k];
      if (act == GFS_HAND_EVICT) {
        pt_delete_lane(d, vkey, f);
        if (!vra)
          shadow_set_lane(d, (uint32_t)(vkey >> GFS_KEY_PAGE_BITS) - 1u, vkey & ((1ull << GFS_KEY_PAGE_BITS) - 1));
      }
      const uint64_t key = page_key(file, q);
      st_rlx(&d->ftag[f], key);
      st_rlx(&d->ffill[f], 0ull);   /* the request that fills it is not known yet */
      /* CLAIMED (no flags, no pins of ours) -> FILLING, version + 1, pinned for the demanded
         page, prefetched mark otherwise; an addition keeps pins other blocks hold briefly */
      const uint64_t delta = (GFS_FS_FILLING - GFS_FS_CLAIMED) + GFS_FW_VER_ONE +
                             (q == demand ? GFS_FW_PIN_ONE : GFS_FW_RA) + (q == mark ? GFS_FW_MARK : 0ull);
      __hip_atomic_fetch_add(&d->fword[f], delta, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      st_rel(d->pt + bs->lslot[k], (key << GFS_ENTRY_FRAME_BITS) | f);
      bs->lframe[k] = f;
      trace_ev(d, 1, GFS_EV_ALLOC, bid, file, (uint32_t)q, f, q == demand ? 0u : 1u, t);
    }
    if (l == 0) bcount(bs, GFS_C_HAND, need);
    assigned += (uint32_t)__popcll(sm);
    visits += need;
  }
  if (l == 0) {
    bcount(bs, GFS_C_EVICTIONS, evicted);
    bcount(bs, GFS_C_WASTED, wasted);
  }
  wave_sync_lds();
  return assigned;
}

/* ------------------------------------------------------------------ vector copy */
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

/* Block-cooperative copy of n bytes; both pointers 16-byte aligned and in global memory
 * (frames, user buffers). Global rather than generic accesses let loads and stores be
 * waited on separately, so eight 16-byte loads per lane are in flight per round.
 * kStream: the source is read with nontemporal loads, which do not keep its lines in the
 * caches; the copy-out of a frame uses it, so that streaming page bytes through does not
 * push the page table and frame words out of L2 (all-hit pass: +3 % with the reads alone,
 * +6 % with a consumer reading the user buffer back, lookup and pin 0.3 us shorter). */
typedef __attribute__((address_space(1))) v4u gv4u;

template <bool kStream = false>
__device__ __forceinline__ void copy_block_aligned(uint8_t* dst, const uint8_t* src, uint64_t n,
                                                   uint32_t tid, uint32_t nt) {
  const uint64_t n16 = n >> 4;
  const gv4u* s = (const gv4u*)src;
  gv4u* o = (gv4u*)dst;
  uint64_t i = tid;
  for (; i + 7ull * nt < n16; i += 8ull * nt) {
    v4u a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (kStream) a[k] = __builtin_nontemporal_load(&s[i + (uint64_t)k * nt]);
      else a[k] = s[i + (uint64_t)k * nt];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) o[i + (uint64_t)k * nt] = a[k];
  }
  for (; i < n16; i += nt) o[i] = s[i];
  for (uint64_t j = (n16 << 4) + tid; j < n; j += nt) dst[j] = src[j];
}

/* The copy-out of a frame's bytes to a user buffer (any alignment). */
__device__ __forceinline__ void copy_block(uint8_t* dst, const uint8_t* src, uint64_t n,
                                           uint32_t tid, uint32_t nt) {
  if ((((uintptr_t)dst | (uintptr_t)src) & 15) == 0) {
    copy_block_aligned<true>(dst, src, n, tid, nt);
  } else {
    for (uint64_t j = tid; j < n; j += nt) dst[j] = src[j];
  }
}

/* Lane: this block holds a pin on frame f (page p), which another block's request is
 * filling. Wait for it to become VALID; meanwhile, once the request's host read is done,
 * try to take over copying this frame's bytes from staging (the PULL bit), so that blocks
 * waiting on a large window pull its pages in parallel. Leaves in bs: status, frame, and
 * pull = 2 with slot/gen/first_page/result when this block must pull frame f. */
__device__ void join_or_help_lane(const gfs_dev* d, uint32_t f, uint64_t p, uint64_t t0,
                                  BlockState* bs) {
  uint64_t* fw = &d->fword[f];
  uint32_t n = 0;
  bs->frame = (int32_t)f;
  bs->pull = 0;
  while (true) {
    uint64_t w = ld_rlx(fw);
    if ((w & GFS_FW_STATE) == GFS_FS_VALID) {
      acquire_agent();   /* the frame's bytes, published before VALID */
      if (w & GFS_FW_ERR) {
        frame_unpin(d, f);
        bs->status = -kEIO;
      } else {
        bs->status = 0;
      }
      return;
    }
    if (!(w & GFS_FW_PULL)) {
      const uint64_t ff = ld_rlx(&d->ffill[f]);
      if (ff >> 63) {
        /* an asynchronous request: nobody publishes it, so look at the host's completion in
           the ring slot itself (the slot cannot be reused while this frame is filling) */
        const uint32_t s = (uint32_t)((ff >> 40) & 0x7fffff) - 1;
        const uint64_t gen = ff & ((1ull << 40) - 1);
        gfs_rpc_slot* rs = &d->ring[s];
        if (__hip_atomic_load(&rs->done_seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) == gen) {
          acquire_system();   /* the staged bytes and the result, written before done_seq */
          if (cas64(fw, w, (w | GFS_FW_PULL) + GFS_FW_VER_ONE)) {
            bs->status = 0;
            bs->pull = 2;
            bs->slot = s;
            bs->gen = gen;
            bs->first_page = rs->offset >> d->page_shift;
            bs->result = rs->result;
            bs->help_page = (uint32_t)p;
            return;
          }
          continue;
        }
      } else if (ff) {
        const uint32_t s = (uint32_t)(ff >> 40) - 1;
        gfs_req_dev* rq = &d->reqd[s];
        const uint64_t ready = ld_rlx(&rq->ready);
        if (ready != 0 && (ready & ((1ull << 40) - 1)) == (ff & ((1ull << 40) - 1))) {
          acquire_agent();   /* the request record, published before ready */
          if (cas64(fw, w, (w | GFS_FW_PULL) + GFS_FW_VER_ONE)) {
            bs->status = 0;
            bs->pull = 2;
            bs->slot = s;
            bs->gen = ready;
            bs->first_page = rq->first_page;
            bs->result = rq->result;
            bs->help_page = (uint32_t)p;
            return;
          }
          continue;
        }
      }
    }
    if (expired(d, t0)) {
      frame_unpin(d, f);
      bcount(bs, GFS_C_TIMEOUTS, 1);
      bs->status = -kETIMEDOUT;
      return;
    }
    nap(n);
  }
}

/* Wave-collective, under the file's miss lock, for a window of at most 64 pages with p
 * absent: find the run of absent pages around p inside [ws, ws + wn) and reserve them.
 * Lane i loads both buckets of page ws + i once; the run is read off the ballot of
 * present pages; each run lane takes a free entry of its less loaded bucket from the
 * loaded copy with one compare-and-swap (and reloads only if that swap loses a race).
 * Fills bs->list/lslot/lframe in allocation order (p first, then the rest ascending);
 * returns the run length and sets failed if some page found both buckets full. */
__device__ uint32_t reserve_run_small_wave(const gfs_dev* d, uint32_t file, uint64_t p, uint64_t ws,
                                           uint32_t wn, BlockState* bs, uint32_t& failed) {
  const uint32_t l = lane();
  const uint64_t q = ws + l;
  const uint64_t key = page_key(file, q);
  const uint64_t ent = (key << GFS_ENTRY_FRAME_BITS) | kReserved;
  uint32_t b1 = 0, b2 = 0;
  uint64_t e[2 * GFS_BUCKET_SLOTS];
  bool present = false, gone = false;
  if (l < wn) {
    key_buckets(d, key, b1, b2);
    pt_load_lane(d, b1, b2, e);
    gone = shadow_lane(d, file, q);
#pragma unroll
    for (int i = 0; i < 2 * GFS_BUCKET_SLOTS; ++i) present |= (e[i] >> GFS_ENTRY_FRAME_BITS) == key;
  }
  const uint32_t pi = (uint32_t)(p - ws);
  uint64_t pm = __ballot(l < wn && present);
  const uint64_t gm = __ballot(gone);
  if (((gm >> pi) & 1ull) == 0) pm |= gm;     /* pages evicted after use stop it, unless p is one */
  if (wn < 64) pm |= ~0ull << wn;             /* pages outside the window stop the run */
  pm &= ~(1ull << pi);                         /* p itself is absent (probed under the lock) */
  const uint64_t below = pm & ((1ull << pi) - 1);
  const uint64_t above = pi == 63 ? 0ull : (pm >> (pi + 1)) << (pi + 1);
  const uint32_t a = below ? 64u - (uint32_t)__builtin_clzll(below) : 0u;
  const uint32_t b = above ? (uint32_t)__builtin_ctzll(above) - 1u : 63u;
  const uint32_t n = b - a + 1;
  uint32_t bad = 0;
  if (l >= a && l <= b) {
    const uint32_t i = l == pi ? 0u : (l < pi ? l - a + 1 : l - a);
    int64_t slot = -1;
    int cnt1 = 0, cnt2 = 0, f1 = -1, f2 = -1;
#pragma unroll
    for (int k = 0; k < GFS_BUCKET_SLOTS; ++k) {
      if (e[k]) ++cnt1;
      else if (f1 < 0) f1 = k;
      if (e[GFS_BUCKET_SLOTS + k]) ++cnt2;
      else if (f2 < 0) f2 = GFS_BUCKET_SLOTS + k;
    }
    int pick = cnt2 < cnt1 ? f2 : f1;
    if (pick < 0) pick = f1 >= 0 ? f1 : f2;
    if (pick >= 0) {
      uint64_t expect = 0;
      uint64_t* sp = slot_ptr(d, b1, b2, pick);
      if (cas64_rlx(sp, expect, ent)) slot = (int64_t)(sp - d->pt);
      else slot = pt_reserve_lane(d, key);    /* the entry was taken meanwhile: reload */
    }
    bs->list[i] = (uint32_t)q;
    bs->lslot[i] = slot < 0 ? 0xffffffffu : (uint32_t)slot;
    bs->lframe[i] = GFS_NO_FRAME;
    bad = slot < 0 ? 1u : 0u;
  }
  failed = bad;
  return n;
}

/* ------------------------------------------------------------------ ring slots
 * Ticketed requests use the first S = sync_slots slots. Shared ring (default): one ticket
 * counter, ticket t uses slot t mod S in generation t / S + 1. Partitioned (GPUfs's queue):
 * block b always posts into slot b mod S, whose own counter gives the generation; the ticket
 * is then (generation - 1) * S + slot, so the same two helpers recover slot and generation.
 * The remaining slots belong to asynchronous windows: a window takes a free one without
 * waiting (or is not issued), because its pages are pulled only when readers reach them, and a
 * ticketed request queued behind such a slot could wait for readers that wait for it. */
__device__ __forceinline__ void ring_ticket_lane(const gfs_dev* d, uint32_t bid, uint64_t& tk) {
  const uint32_t S = d->sync_slots;
  if (d->partitioned) {
    const uint32_t s = bid % S;
    tk = fadd64(&d->slot_tail[s], 1) * S + s;
  } else {
    tk = fadd64(&d->g->ring_tail, 1);
  }
}
__device__ __forceinline__ uint32_t ring_slot(const gfs_dev* d, uint32_t, uint64_t tk) {
  return (uint32_t)(tk % d->sync_slots);
}
__device__ __forceinline__ uint64_t ring_gen(const gfs_dev* d, uint64_t tk) { return tk / d->sync_slots + 1; }

/* Lane: take a free slot of the asynchronous windows (busy 0 -> 1), starting at the block's
   own; -1 if every one is held. The slot's next generation is one past its last completed. */
__device__ int32_t async_slot_take_lane(const gfs_dev* d, uint32_t bid) {
  const uint32_t A = d->rpc_slots - d->sync_slots;
  for (uint32_t i = 0; i < A; ++i) {
    const uint32_t s = d->sync_slots + (bid + i) % A;
    uint64_t* b = &d->reqd[s].busy;
    uint64_t z = 0;
    if (ld_rlx(b) == 0 && cas64(b, z, 1ull)) return (int32_t)s;
  }
  return -1;
}

/* ------------------------------------------------------------------ private policy
 * The paper's design (Sec. 4.1 and Sec. 5.1). A miss reserves the one page in the table
 * without the file's lock (reserve_unique_wave); the frame comes from the block's own share
 * of the frames,
 * least recently allocated first (a frame another block has pinned is passed over); the
 * bytes come from the block's private buffer if it holds the page, else from a host read of
 * the page plus the static prefetch size, whose tail becomes the new private buffer. */

__device__ int64_t reserve_unique_wave(const gfs_dev* d, uint64_t key);

/* Lane: claim frame f of the block's share: FREE, or VALID with no pins (its page is
   evicted; the reference bit plays no part). CLAIMED on success. */
__device__ int lra_visit(const gfs_dev* d, uint32_t f, uint64_t& vkey, uint32_t& vra) {
  uint64_t* fw = &d->fword[f];
  uint64_t w = ld_rlx(fw);
  const uint64_t tag = ld_rlx(&d->ftag[f]);
  const uint64_t st = w & GFS_FW_STATE;
  const uint64_t claimed = (((w >> GFS_FW_VER_SHIFT) + 1) << GFS_FW_VER_SHIFT) | GFS_FS_CLAIMED;
  if (w & GFS_FW_PINS) return GFS_HAND_SKIP;
  if (st == GFS_FS_FREE) return cas64(fw, w, claimed) ? GFS_HAND_FREE : GFS_HAND_SKIP;
  if (st != GFS_FS_VALID) return GFS_HAND_SKIP;
  const uint64_t old = w;
  if (!cas64(fw, w, claimed)) return GFS_HAND_SKIP;
  vkey = tag;
  vra = (old & GFS_FW_RA) ? 1u : 0u;
  return GFS_HAND_EVICT;
}

/* Wave 0: the miss path of the private policy. 0: done (bs filled in), 1: look again,
   2: timed out. */
__device__ int miss_private_wave(const gfs_dev* d, uint32_t file, uint64_t p, uint64_t key, uint64_t fsize,
                                 BlockState* bs, uint32_t bid, uint64_t t0, uint32_t& naps) {
  const uint32_t l = lane();
  /* the page's table entry, made unique without the file's lock (the policy decides nothing
     under it: the window is the static prefetch after p, into the block's own buffer) */
  const uint64_t tr0 = wall_clock64();
  const int64_t slot = reserve_unique_wave(d, key);
  if (l == 0) bcount(bs, GFS_T_RUN, wall_clock64() - tr0);
  if (slot == -1) return 1;   /* another block's entry: go to the pin path */
  if (slot < 0) {
    /* both buckets of the key are full: reservations of misses in flight come and go, so
       back off and look again; only a table still full at the wait limit is an error */
    if (!expired(d, t0)) {
      if (l == 0) {
        bcount(bs, GFS_C_RETRIES, 1);
        nap(naps);
      }
      return 1;
    }
    if (l == 0) {
      bs->status = -kENOSPC;
      bs->pull = 0;
      bs->frame = -1;
    }
    return 0;
  }
  int status = 0;
  if (l == 0) {
    gfs_pslot* ps = &d->pslots[bs->pslot];
    const uint64_t npages = d->files[file].npages;
    const uint32_t cap = d->ra_cap;
    const uint32_t span = (uint32_t)((npages - p) < (uint64_t)(1 + cap) ? (npages - p) : (uint64_t)(1 + cap));
    const bool in_pb = ps->n && ps->file == file && ps->first <= p && p < ps->first + ps->n;
    trace_ev(d, 1, GFS_EV_MISS, bid, file, (uint32_t)p, 0, in_pb ? 1u : span, p);
    /* a frame of the block's share, least recently allocated first */
    const uint64_t ta0 = wall_clock64();
    const uint32_t q = d->quota;
    const uint32_t base = (uint32_t)bs->pslot * q;
    int32_t fr = -1;
    for (uint32_t i = 0; i < 2 * q && fr < 0; ++i) {
      const uint32_t idx = ps->lra_next;
      ps->lra_next = idx + 1 == q ? 0 : idx + 1;
      const uint32_t f = base + idx;
      uint64_t vkey = 0;
      uint32_t vra = 0;
      const int act = lra_visit(d, f, vkey, vra);
      if (act == GFS_HAND_EVICT) {
        pt_delete_lane(d, vkey, f);
        bcount(bs, GFS_C_EVICTIONS, 1);
        const uint32_t vf = (uint32_t)(vkey >> GFS_KEY_PAGE_BITS) - 1u;
        const uint32_t vp = (uint32_t)(vkey & ((1ull << GFS_KEY_PAGE_BITS) - 1));
        trace_ev(d, 1, GFS_EV_HAND, bid, vf, vp, f, GFS_HAND_EVICT, idx);
      } else if (act == GFS_HAND_SKIP) {
        trace_ev(d, 1, GFS_EV_HAND, bid, 0xffffffffu, 0xffffffffu, f, GFS_HAND_SKIP, idx);
      }
      if (act == GFS_HAND_FREE || act == GFS_HAND_EVICT) fr = (int32_t)f;
    }
    bcount(bs, GFS_C_HAND, 1);
    if (fr < 0) {
      /* every frame of the share is pinned by other blocks: give the page back, retry */
      st_rel(d->pt + slot, 0ull);
      bcount(bs, GFS_C_NOFRAME, 1);
      status = 1;
    } else {
      st_rlx(&d->ftag[fr], key);
      st_rlx(&d->ffill[fr], 0ull);
      __hip_atomic_fetch_add(&d->fword[fr], (GFS_FS_FILLING - GFS_FS_CLAIMED) + GFS_FW_VER_ONE + GFS_FW_PIN_ONE,
                             __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      st_rel(d->pt + slot, (key << GFS_ENTRY_FRAME_BITS) | (uint64_t)fr);
      trace_ev(d, 1, GFS_EV_ALLOC, bid, file, (uint32_t)p, (uint32_t)fr, 0, (uint64_t)ps->lra_next);
      bcount(bs, GFS_T_ALLOC, wall_clock64() - ta0);
      bcount(bs, GFS_C_MISSES, 1);
      bs->frame = fr;
      bs->file = file;
      bs->status = 0;
      if (in_pb) {
        trace_ev(d, 1, GFS_EV_PBHIT, bid, file, (uint32_t)p, (uint32_t)fr, 0, 0);
        bcount(bs, GFS_C_PB_HITS, 1);
        bs->pull = 3;
        bs->help_page = (uint32_t)p;
      } else {
        /* one request: the page and the prefetch that follows it */
        const uint64_t off0 = p << d->page_shift;
        uint64_t len = (uint64_t)span << d->page_shift;
        if (off0 + len > fsize) len = fsize - off0;
        uint64_t tk;
        ring_ticket_lane(d, bid, tk);
        const uint32_t s = ring_slot(d, bid, tk);
        const uint64_t gen = ring_gen(d, tk);
        uint32_t nn = 0;
        const uint64_t ts0 = wall_clock64();
        while (ld_rlx(&d->slot_free[s]) != gen - 1) {
          if (expired(d, t0)) {
            status = 2;
            break;
          }
          nap(nn);
        }
        acquire_agent();   /* the slot's last users are done with its staging */
        bcount(bs, GFS_T_SLOT, wall_clock64() - ts0);
        if (status == 0) {
          gfs_rpc_slot* rs = &d->ring[s];
          rs->file_id = file;
          rs->npages = span;
          rs->offset = off0;
          rs->length = len;
          rs->ticket = tk;
          __hip_atomic_store(&rs->req_seq, gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
          trace_ev(d, 1, GFS_EV_REQ, bid, file, (uint32_t)p, GFS_NO_FRAME, span, tk);
          bcount(bs, GFS_C_REQUESTS, 1);
          bcount(bs, GFS_C_REQ_BYTES, len);
          bcount(bs, GFS_C_FETCHED, 1);
          const uint64_t th0 = wall_clock64();
          while (__hip_atomic_load(&rs->done_seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != gen) {
            if (expired(d, t0)) {
              status = 2;
              break;
            }
            nap(nn);
          }
          acquire_system();   /* the staged bytes, written by the host before done_seq */
          bcount(bs, GFS_T_HOST, wall_clock64() - th0);
          if (status == 0) bs->result = rs->result;
        }
        if (status == 0) {
          bs->pull = 4;
          bs->slot = s;
          bs->gen = gen;
          bs->first_page = p;
          bs->list_n = span;
        } else {
          /* the frame stays FILLING with the pin; the cache must be reset after a timeout */
          bs->status = -kETIMEDOUT;
          bs->pull = 0;
          bcount(bs, GFS_C_TIMEOUTS, 1);
        }
      }
    }
  }
  status = __shfl(status, 0, 64);
  if (status == 1) {
    if (expired(d, t0)) return 2;
    if (l == 0) nap(naps);
    return 1;
  }
  return 0;
}

/* Wave 0, after the run's pages got frames (bs->list/lframe[0..got), the demanded page first):
 * post one request for the span of those pages, tell blocks waiting on its frames which request
 * fills them, wait for the host, and publish the finished read for the helpers. Leaves in bs:
 * status, the demanded page's frame, pull = 1 (this block pulls the request). Returns 0. */
__device__ int post_wait_wave(const gfs_dev* d, uint32_t file, uint64_t fsize, BlockState* bs, uint32_t bid,
                              uint64_t t0, uint32_t got) {
  const uint32_t l = lane();
  /* span of the pages that got frames: p and a contiguous piece of the run */
  uint64_t lo = ~0ull, hi = 0;
  for (uint32_t k = l; k < got; k += 64) {
    const uint64_t q = bs->list[k];
    lo = q < lo ? q : lo;
    hi = q > hi ? q : hi;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t olo = __shfl_xor(lo, off, 64), ohi = __shfl_xor(hi, off, 64);
    lo = olo < lo ? olo : lo;
    hi = ohi > hi ? ohi : hi;
  }
  /* post the request for the span [lo, hi] and wait for the host */
  const uint32_t span = (uint32_t)(hi - lo + 1);
  const uint64_t off0 = lo << d->page_shift;
  uint64_t len = (uint64_t)span << d->page_shift;
  if (off0 + len > fsize) len = fsize - off0;
  int64_t status = 0;
  uint64_t tk = 0;
  if (l == 0) {
    ring_ticket_lane(d, bid, tk);
    const uint32_t s = ring_slot(d, bid, tk);
    const uint64_t gen = ring_gen(d, tk);
    uint32_t nn = 0;
    const uint64_t ts0 = wall_clock64();
    while (ld_rlx(&d->slot_free[s]) != gen - 1) {
      if (expired(d, t0)) {
        status = -kETIMEDOUT;
        break;
      }
      nap(nn);
    }
    acquire_agent();   /* the slot's last users are done with its staging */
    bcount(bs, GFS_T_SLOT, wall_clock64() - ts0);
    if (status == 0) {
      gfs_rpc_slot* rs = &d->ring[s];
      rs->file_id = file;
      rs->npages = span;
      rs->offset = off0;
      rs->length = len;
      rs->ticket = tk;
      __hip_atomic_store(&rs->req_seq, gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      trace_ev(d, 1, GFS_EV_REQ, bid, file, (uint32_t)lo, GFS_NO_FRAME, span, tk);
      bcount(bs, GFS_C_MISSES, 1);
      bcount(bs, GFS_C_REQUESTS, 1);
      bcount(bs, GFS_C_REQ_BYTES, len);
      bcount(bs, GFS_C_FETCHED, got);
      bcount(bs, GFS_C_RA_PAGES, got - 1);
    }
  }
  status = __shfl(status, 0, 64);
  tk = __shfl(tk, 0, 64);
  const uint32_t s = ring_slot(d, bid, tk);
  const uint64_t gen = ring_gen(d, tk);
  if (status == 0) {
    /* tell waiting blocks which request fills each frame: (slot + 1) << 40 | gen */
    const uint64_t fill = ((uint64_t)(s + 1) << 40) | (gen & ((1ull << 40) - 1));
    for (uint32_t k = l; k < got; k += 64) st_rel(&d->ffill[bs->lframe[k]], fill);
  }
  if (l == 0) {
    if (status == 0) {
      gfs_rpc_slot* rs = &d->ring[s];
      uint32_t nn = 0;
      const uint64_t th0 = wall_clock64();
      while (__hip_atomic_load(&rs->done_seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) !=
             gen) {
        if (expired(d, t0)) {
          status = -kETIMEDOUT;
          break;
        }
        nap(nn);
      }
      acquire_system();   /* the staged bytes, written by the host before done_seq */
      bcount(bs, GFS_T_HOST, wall_clock64() - th0);
      if (status == 0) {
        bs->result = rs->result;
        /* let blocks waiting on frames of this request pull their own pages */
        gfs_req_dev* rq = &d->reqd[s];
        rq->result = bs->result;
        rq->first_page = lo;
        rq->file = file;
        __hip_atomic_store(&rq->remaining, got, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st_rel(&rq->ready, gen);
      }
    }
    if (status) bcount(bs, GFS_C_TIMEOUTS, 1);
    bs->status = status;
    bs->frame = (int32_t)bs->lframe[0];
    bs->pull = status == 0 ? 1 : 0;
    bs->slot = s;
    bs->gen = gen;
    bs->first_page = lo;
    bs->list_n = got;
    bs->file = file;
  }
  return 0;
}

/* Wave-collective, without the miss lock: reserve the table entry of key if no entry for it
 * exists, so that one block alone fetches the page. Lanes 0-31 load the key's two buckets; lane
 * 0 takes a free entry of the less loaded bucket by compare-and-swap; once that swap has been
 * performed the lanes look again, and if another block's entry for the same key is there the
 * reservation is withdrawn. Of two blocks that reserve one key at once, the later swap sees the
 * earlier one, so at most one reservation stays (both may withdraw; both then look again).
 * Returns the entry's index, -1 when the key has (or just got) another entry, -2 when both
 * buckets stayed full. */
__device__ int64_t reserve_unique_wave(const gfs_dev* d, uint64_t key) {
  uint32_t b1, b2;
  key_buckets(d, key, b1, b2);
  const uint32_t l = lane();
  const uint64_t ent = (key << GFS_ENTRY_FRAME_BITS) | kReserved;
  for (int attempt = 0; attempt < 64; ++attempt) {
    uint64_t e = 0;
    if (l < 32) e = ld_rlx(slot_ptr(d, b1, b2, (int)l));
    if (__ballot(l < 32 && (e >> GFS_ENTRY_FRAME_BITS) == key)) return -1;
    const uint64_t free1 = __ballot(l < 16 && e == 0), free2 = __ballot(l >= 16 && l < 32 && e == 0);
    const uint32_t used1 = 16u - (uint32_t)__popcll(free1), used2 = 16u - (uint32_t)__popcll(free2);
    uint64_t fm = used2 < used1 ? free2 : free1;   /* less loaded bucket, ties to the first */
    if (fm == 0) fm = free1 ? free1 : free2;
    if (fm == 0) return -2;
    const int pick = __builtin_ctzll(fm);
    uint64_t* sp = slot_ptr(d, b1, b2, pick);
    int won = 0;
    if (l == 0) {
      uint64_t z = 0;
      won = cas64_rlx(sp, z, ent) ? 1 : 0;
    }
    won = __shfl(won, 0, 64);
    if (!won) continue;   /* the entry was taken meanwhile: look again */
    drain_atomics();      /* the swap is performed before the second look goes out */
    uint64_t e2 = 0;
    if (l < 32 && (int)l != pick) e2 = ld_rlx(slot_ptr(d, b1, b2, (int)l));
    if (__ballot(l < 32 && (int)l != pick && (e2 >> GFS_ENTRY_FRAME_BITS) == key)) {
      if (l == 0) {
        uint64_t x = ent;
        (void)cas64_rlx(sp, x, 0ull);
      }
      return -1;
    }
    return (int64_t)(sp - d->pt);
  }
  return -2;
}

/* Wave 0: the miss path of a file whose windows are one page (readahead off, or RANDOM advice):
 * no detector decision to make, so no miss lock; the page's reservation is made unique by
 * reserve_unique_wave. Same results and trace events as the locked path for such a file.
 * Returns as miss_shared_wave. */
__device__ int miss_one_page_wave(const gfs_dev* d, uint32_t file, uint64_t p, uint64_t key, uint64_t fsize,
                                  BlockState* bs, uint32_t bid, uint64_t t0, uint32_t& naps) {
  const uint32_t l = lane();
  const uint64_t tr0 = wall_clock64();
  const int64_t slot = reserve_unique_wave(d, key);
  if (slot == -1) return 1;   /* another block's entry: go to the pin path */
  if (slot < 0) {
    /* both buckets full of other misses' reservations: back off; -ENOSPC at the wait limit */
    if (!expired(d, t0)) {
      if (l == 0) {
        bcount(bs, GFS_C_RETRIES, 1);
        nap(naps);
      }
      return 1;
    }
    if (l == 0) {
      bs->status = -kENOSPC;
      bs->pull = 0;
      bs->frame = -1;
    }
    return 0;
  }
  if (l == 0) {
    trace_ev(d, 1, GFS_EV_MISS, bid, file, (uint32_t)p, (uint32_t)RA_RULE_OFF << 24, 1, p);
    bs->list[0] = (uint32_t)p;
    bs->lslot[0] = (uint32_t)slot;
    bs->lframe[0] = GFS_NO_FRAME;
  }
  wave_sync_lds();
  const uint64_t tl3 = wall_clock64();
  if (l == 0) bcount(bs, GFS_T_RUN, tl3 - tr0);
  const uint32_t got = alloc_wave(d, file, p, bs, 1, bid);
  if (l == 0) bcount(bs, GFS_T_ALLOC, wall_clock64() - tl3);
  if (got == 0) {
    /* every frame pinned or filling: give the page back and retry the access */
    if (l == 0) {
      st_rel(d->pt + slot, 0ull);
      bcount(bs, GFS_C_NOFRAME, 1);
    }
    if (expired(d, t0)) return 2;
    if (l == 0) nap(naps);
    return 1;
  }
  return post_wait_wave(d, file, fsize, bs, bid, t0, 1);
}

/* Wave 0: the shared policy's miss path for page p of `file` (key), found absent from the
 * table: take the file's miss lock, decide and claim the window, reserve and allocate its
 * run, post the request and wait for the host. Out of line: it runs once per host request
 * and holds most of the library's registers, which the hit path then does not have to share.
 * Returns 0 when bs is filled in (status, frame, pull), 1 to look the page up again, 2 when
 * the wait timed out. */
__device__ __attribute__((noinline)) int miss_shared_wave(const gfs_dev* d, uint32_t file, uint64_t p,
                                                          uint64_t key, uint64_t fsize, BlockState* bs,
                                                          uint32_t bid, uint64_t t0, uint32_t& naps) {
  if (d->ra_cap == 0 || ld_rlx32(&d->files[file].advice) == GFS_ADV_RANDOM)
    return miss_one_page_wave(d, file, p, key, fsize, bs, bid, t0, naps);
  const uint32_t l = lane();
  /* the pages of the read that missed, from p on */
  const uint64_t rl = bs->read_last;
  const uint32_t req = rl >= p ? (rl - p + 1 < 0xffffffffull ? (uint32_t)(rl - p + 1) : 0xffffffffu) : 1u;
  /* the cached history behind p, counted before the lock (see ra_history_wave) */
  const uint32_t hist_pre = ra_history_wave(d, file, p, req);
  const RaParams rp = ra_params(d);
  /* what the critical section needs from the device and file records, read now: after the
     grant's acquire, each would be a load from memory on the path every waiter waits on */
  gfs_file_dev* const fe = &d->files[file];
  uint64_t* const clp = d->claims[file].e;
  uint64_t* const lq = d->lockq + (uint64_t)file * GFS_LOCK_SLOTS;
  uint64_t* const pt = d->pt;
  const uint32_t ptmask = d->nbuckets_mask;
  const uint64_t npages = fe->npages;
  const bool tracing = d->trace_level >= 1;
  const bool async_on = d->ra_async != 0;
  const uint64_t tl0 = wall_clock64();
  uint64_t ticket;
  const int lk = lock_file_wave(d, file, key, p, t0, ticket);
  const uint64_t tl1 = wall_clock64();
  if (l == 0) bcount(bs, GFS_T_LOCK, tl1 - tl0);
  if (lk == LOCK_TIMEOUT) return 2;
  if (lk == LOCK_LEFT) {
    if (l == 0) bcount(bs, GFS_C_LOCK_LEFT, 1);
    return 1;   /* the page was reserved while this block waited: go to the pin path */
  }
  if (lk == LOCK_COVERED) {
    /* the holder's window covers the page: wait until its reservation shows in the
       table or no running claim covers the page any more, then look again */
    if (l == 0) bcount(bs, GFS_C_LOCK_LEFT, 1);
    uint32_t nw = 0;
    while (pt_lookup_wave(d, key) < 0 && !expired(d, t0)) {
      uint64_t cl = 0;
      if (l < GFS_CLAIMS) cl = ld_rlx(&d->claims[file].e[l]);
      const uint64_t c_lo = cl >> 32, c_hi = (cl >> 32) + ((cl & 0xffffffffull) >> 1);
      if (__ballot(l < GFS_CLAIMS && (cl & 1ull) && c_lo <= p && p < c_hi) == 0) break;
      if (l == 0) nap_short(nw);
    }
    acquire_agent();   /* the reservations, published before the claim was cleared */
    return 1;
  }
  if (l == 0) bcount(bs, GFS_C_LOCKS, 1);
  /* every block waiting on this file's lock waits for this wave: let it issue first */
  __builtin_amdgcn_s_setprio(3);
  /* one round: the detector state and the file's window claims; then, ordered after the
     claims, the table probe (a claim cleared after its reservations means they show) */
  const RaState ras = ra_load_lane(fe, rp.nrec, rp.nstreams);
  uint64_t cl = 0;
  if (l < GFS_CLAIMS) cl = ld_rlx(&clp[l]);
  /* the queue slots behind this ticket, read now for the hand-off: a waiter that arrives or
     leaves after this read is handled by the grant's exchange (it returns what the slot
     holds), and a stale "waiting" value only makes the covered mark's compare-and-swap fail */
  const uint64_t qv = ld_rlx(lq + ((ticket + 1 + l) & (GFS_LOCK_SLOTS - 1)));
  drain_atomics();   /* the table probe below goes out after the claims were read */
  const bool cl_on = l < GFS_CLAIMS && (cl & 1ull);
  const uint64_t cl_lo = cl >> 32, cl_hi = (cl >> 32) + ((cl & 0xffffffffull) >> 1);
  const bool covered = __ballot(cl_on && cl_lo <= p && p < cl_hi) != 0;
  const uint64_t free_cl = __ballot(l < GFS_CLAIMS && !cl_on);
  const bool present = pt_lookup_at(pt, ptmask, key) >= 0;
  if (present || covered || free_cl == 0) {
    /* filled, reserved, or about to be reserved by a window being claimed: go to the pin
       path (after a nap if the claim is still running) */
    unlock_slots_wave(lq, ticket, 0, 0, false, 0);
    __builtin_amdgcn_s_setprio(0);
    if (l == 0) bcount(bs, GFS_T_CRIT, wall_clock64() - tl1);
    if (!present) {
      if (expired(d, t0)) return 2;
      if (l == 0) nap(naps);
    }
    return 1;
  }
  /* miss: decide the window, clip it to stay out of running claims, claim it, unlock */
  uint64_t ws;
  uint32_t wn, near, hist, rule;
  int rslot;
  const uint64_t td0 = wall_clock64();
  ra_decide_wave(fe, p, req, hist_pre, rp, ras, ws, wn, near, hist, rule, rslot);
  const uint64_t td1 = wall_clock64();
  if (l == 0) bcount(bs, GFS_T_DECIDE, td1 - td0);
  if (ws + wn > npages) wn = (uint32_t)(npages - ws);
  /* asynchronous readahead: the page after the demanded one is the stream's marker */
  uint64_t mark = ~0ull;
  if (async_on && rslot >= 0) {
    mark = p + 1 < ws + wn ? p + 1 : ~0ull;
    if (l == 0) st_rlx32(&fe->streams[rslot].marker, mark == ~0ull ? GFS_NO_MARKER : (uint32_t)mark);
  }
  if (tracing && l == 0)
    trace_ev(d, 1, GFS_EV_MISS, bid, file, (uint32_t)p, (near & 0xffu) | (hist << 8) | (rule << 24), wn,
             ws | ((uint64_t)req << 32));
  uint64_t cws = ws, cwe = ws + wn;
  {
    uint64_t lo_b = cl_on && cl_hi <= p ? cl_hi : 0;
    uint64_t hi_b = cl_on && cl_lo > p ? cl_lo : ~0ull;
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t a = __shfl_xor(lo_b, off, 64), b = __shfl_xor(hi_b, off, 64);
      lo_b = a > lo_b ? a : lo_b;
      hi_b = b < hi_b ? b : hi_b;
    }
    cws = cws > lo_b ? cws : lo_b;
    cwe = cwe < hi_b ? cwe : hi_b;
  }
  const uint32_t cj = (uint32_t)__builtin_ctzll(free_cl);
  uint64_t* claim = &clp[cj];
  if (l == 0) st_rlx(claim, (cws << 32) | ((cwe - cws) << 1) | 1ull);
  const uint64_t tu0 = wall_clock64();
  unlock_slots_wave(lq, ticket, cws, cwe, true, qv);
  __builtin_amdgcn_s_setprio(0);
  const uint64_t tl2 = wall_clock64();
  if (l == 0) {
    bcount(bs, GFS_T_CRIT, tl2 - tl1);
    bcount(bs, GFS_T_UNLOCK, tl2 - tu0);
  }
  /* reserve the run of unmapped pages around p inside the claimed window */
  const uint32_t cwn = (uint32_t)(cwe - cws);
  uint32_t n = 0, failed = 0;
  if (cwn <= 64) {
    /* one round: lane i loads the buckets of window page cws + i, the run around p is
       read off the ballot of present pages, and each run lane reserves its page from
       the buckets it already holds */
    n = reserve_run_small_wave(d, file, p, cws, cwn, bs, failed);
  } else {
    /* pages evicted after use end the run too, unless p is one */
    const bool clip = !shadow_lane(d, file, p);
    uint64_t a = p;
    for (uint64_t base = p; base > cws;) {
      const bool valid = (uint64_t)l < base - cws;
      bool stop = !valid;
      if (valid)
        stop = pt_present_lane(d, page_key(file, base - 1 - l)) | (clip && shadow_lane(d, file, base - 1 - l));
      const uint64_t sm = __ballot(stop);
      const uint32_t k = sm ? (uint32_t)__builtin_ctzll(sm) : 64u;
      a = base - k;
      if (k < 64) break;
      base -= 64;
    }
    uint64_t b = p;
    for (uint64_t base = p + 1; base < cwe;) {
      const bool valid = (uint64_t)l < cwe - base;
      bool stop = !valid;
      if (valid) stop = pt_present_lane(d, page_key(file, base + l)) | (clip && shadow_lane(d, file, base + l));
      const uint64_t sm = __ballot(stop);
      const uint32_t k = sm ? (uint32_t)__builtin_ctzll(sm) : 64u;
      b = base + k - 1;
      if (k < 64) break;
      base += 64;
    }
    n = (uint32_t)(b - a + 1);
    /* allocation order: the demanded page first, then the rest of the run ascending */
    for (uint32_t i = l; i < n; i += 64) {
      uint64_t q;
      if (i == 0) q = p;
      else if (i <= p - a) q = a + i - 1;
      else q = a + i;
      const int64_t slot = pt_reserve_lane(d, page_key(file, q));
      bs->list[i] = (uint32_t)q;
      bs->lslot[i] = slot < 0 ? 0xffffffffu : (uint32_t)slot;
      bs->lframe[i] = GFS_NO_FRAME;
      failed |= slot < 0 ? 1u : 0u;
    }
  }
  failed = (uint32_t)(__ballot(failed != 0) != 0);
  /* the reservations are in the table: release the claim */
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (l == 0) st_rlx(claim, 0ull);
  wave_sync_lds();
  const uint64_t tl3 = wall_clock64();
  if (l == 0) bcount(bs, GFS_T_RUN, tl3 - tl2);
  /* a reservation can fail only if both buckets are full: keep the prefix before the
     first failure (the demanded page comes first) and drop the rest */
  uint32_t keep = n;
  if (failed) {
    uint32_t firstbad = n;
    for (uint32_t i = l; i < n; i += 64)
      if (bs->lslot[i] == 0xffffffffu) firstbad = i < firstbad ? i : firstbad;
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t o = __shfl_xor(firstbad, off, 64);
      firstbad = o < firstbad ? o : firstbad;
    }
    keep = firstbad;
  }
  const uint32_t got = keep ? alloc_wave(d, file, p, bs, keep, bid, mark) : 0;
  if (l == 0) bcount(bs, GFS_T_ALLOC, wall_clock64() - tl3);
  /* release reservations that got no frame (the table was full or no frame was free) */
  for (uint32_t i = got + l; i < n; i += 64) {
    if (bs->lslot[i] != 0xffffffffu)
      st_rel(d->pt + bs->lslot[i], 0ull);
  }
  if (got == 0) {
    if (l == 0) bcount(bs, keep ? GFS_C_NOFRAME : GFS_C_RETRIES, 1);
    if (keep == 0 && expired(d, t0)) {
      /* the demanded page's buckets stayed full until the wait limit */
      if (l == 0) {
        bs->status = -kENOSPC;
        bs->pull = 0;
        bs->frame = -1;
      }
      return 0;
    }
    if (expired(d, t0)) return 2;
    if (l == 0) nap(naps);
    return 1;   /* buckets full of reservations in flight, or every frame pinned or
                   filling: back off and retry the access */
  }
  if (got < n && l == 0)
    trace_ev(d, 1, GFS_EV_NOFRAME, bid, file, bs->list[got], GFS_NO_FRAME, 0, 0);
  return post_wait_wave(d, file, fsize, bs, bid, t0, got);
}

/* ------------------------------------------------------------------ one page, wave 0
 * Leaves in bs: status; on success the pinned frame, and pull = 1 when this block posted
 * the request and must pull it. */
__device__ void acquire_page_wave(const gfs_dev* d, uint32_t file, uint64_t p, uint64_t fsize,
                                  BlockState* bs, uint32_t bid) {
  const uint64_t key = page_key(file, p);
  const uint32_t l = lane();
  uint64_t t0 = 0;   /* the wait deadline's start: read at the first step that may wait */
  uint32_t naps = 0;
  /* untraced runs check a hit's tag with its copy (frame_pin_fast) */
  const bool fast = d->trace_level == 0;
  if (l == 0) {
    bs->tagkey = 0;
    bs->trig = 0;
  }
  while (true) {
    int32_t f = pt_lookup_wave(d, key);
    if (f >= 0 && (uint32_t)f != kReserved) {
      int r = PIN_RETRY;
      uint64_t w = 0;
      if (l == 0) r = fast ? frame_pin_fast(d, (uint32_t)f, key, w) : frame_pin(d, (uint32_t)f, key, &w);
      r = __shfl(r, 0, 64);
      if (r == PIN_VALID_UNCHECKED) {
        if (l == 0) {
          bs->frame = f;
          bs->status = 0;
          bs->pull = 0;
          bs->tagkey = key;
          bs->pinw = w;
        }
        return;
      }
      if (t0 == 0) t0 = wall_clock64();
      if (r == PIN_VALID) {
        if (l == 0) {
          bcount(bs, GFS_C_HITS, 1);
          trace_ev(d, 2, GFS_EV_HIT, bid, file, (uint32_t)p, (uint32_t)f, 0, 0);
          bs->frame = f;
          bs->status = 0;
          bs->pull = 0;
          if (d->ra_async && (w & GFS_FW_MARK)) bs->trig = mark_take_lane(d, (uint32_t)f) ? 1u : 0u;
        }
        return;
      }
      if (r == PIN_FILLING) {
        if (l == 0) {
          bcount(bs, GFS_C_JOINS, 1);
          trace_ev(d, 2, GFS_EV_JOIN, bid, file, (uint32_t)p, (uint32_t)f, 0, 0);
          if (d->ra_async && (w & GFS_FW_MARK)) bs->trig = mark_take_lane(d, (uint32_t)f) ? 1u : 0u;
          const uint64_t tj0 = wall_clock64();
          join_or_help_lane(d, (uint32_t)f, p, t0, bs);
          bcount(bs, GFS_T_JOIN, wall_clock64() - tj0);
        }
        return;
      }
      if (r == PIN_ERROR) {
        if (l == 0) {
          bs->status = -kEIO;
          bs->frame = -1;
          bs->pull = 0;
        }
        return;
      }
      if (l == 0) bcount(bs, GFS_C_RETRIES, 1);
    }
    if (t0 == 0) t0 = wall_clock64();
    if (f >= 0 && (uint32_t)f != kReserved) {
      /* the pin lost a race (the frame changed under it): wait a little and look again */
    } else if (f < 0 && d->policy == GFS_POLICY_PRIVATE) {
      const int r = miss_private_wave(d, file, p, key, fsize, bs, bid, t0, naps);
      if (r == 0) return;
      if (r == 2) break;
      continue;
    } else if (f < 0 && bs->a_pending) {
      /* a block posts a request only with no asynchronous request of its own outstanding (so
         that no block waits for a ring slot that only it would free): the block finishes that
         request first and then looks again */
      if (l == 0) {
        bs->status = 0;
        bs->pull = 5;
        bs->frame = -1;
      }
      return;
    } else if (f < 0) {
      const int r = miss_shared_wave(d, file, p, key, fsize, bs, bid, t0, naps);
      if (r == 0) return;
      if (r == 2) break;
      continue;
    }
    /* reserved by another block's miss, or a lost race: wait a little and look again */
    if (expired(d, t0)) break;
    if (l == 0) nap(naps);
  }
  if (l == 0) {
    bcount(bs, GFS_C_TIMEOUTS, 1);
    bs->status = -kETIMEDOUT;
    bs->pull = 0;
    bs->frame = -1;
  }
}

/* Bytes of page q held in the staging of a request whose span starts at first (clamped to
 * what the host returned and to the file). */
__device__ __forceinline__ uint64_t staged_bytes(const gfs_dev* d, uint64_t q, uint64_t first,
                                                 int64_t result, uint64_t fsize) {
  const uint64_t P = d->page_size;
  const uint64_t rel = (q - first) * P;
  int64_t avail = result - (int64_t)rel;
  if (avail < 0) avail = 0;
  uint64_t pb = fsize - (q << d->page_shift);
  if (pb > P) pb = P;
  return (uint64_t)avail < pb ? (uint64_t)avail : pb;
}
__device__ __forceinline__ bool staged_short(const gfs_dev* d, uint64_t q, uint64_t first,
                                             int64_t result, uint64_t fsize) {
  const uint64_t P = d->page_size;
  uint64_t pb = fsize - (q << d->page_shift);
  if (pb > P) pb = P;
  return result < 0 || (uint64_t)result < (q - first) * P + pb;
}

/* Wave 0: claim the request's frames that no helping block has taken (PULL bit); their
 * indices go to bs->lslot[0..nclaim). A frame counts as the request's only while its fill word
 * names the request (fill): once helpers have published it, the clock may have given it to
 * another request, which the caller must not touch. The word is read first (acquire) and the
 * fill word after it, and the claim is a compare-and-swap against that word, so a frame that
 * changed hands in between is not claimed. */
__device__ void claim_pulls_wave(const gfs_dev* d, BlockState* bs, uint64_t fill) {
  const uint32_t l = lane();
  uint32_t nclaim = 0;
  for (uint32_t base = 0; base < bs->list_n; base += 64) {
    const uint32_t k = base + l;
    bool won = false;
    if (k < bs->list_n) {
      const uint32_t f = bs->lframe[k];
      uint64_t* fw = &d->fword[f];
      uint64_t w = ld_acq(fw);
      while ((w & GFS_FW_STATE) == GFS_FS_FILLING && !(w & GFS_FW_PULL) && ld_rlx(&d->ffill[f]) == fill) {
        if (cas64(fw, w, (w | GFS_FW_PULL) + GFS_FW_VER_ONE)) {
          won = true;
          break;
        }
      }
    }
    const uint64_t m = __ballot(won);
    if (won) bs->lslot[nclaim + __popcll(m & lanemask_lt())] = k;
    nclaim += (uint32_t)__popcll(m);
  }
  if (l == 0) bs->nclaim = nclaim;
  wave_sync_lds();
}

/* Block-collective: copy claimed pages from the ring slot's staging into their frames.
 * pull == 1: the frames listed in lslot[0..nclaim); pull == 2: the one helped frame. */
__device__ void block_pull(const gfs_dev* d, const BlockState* bs, uint64_t fsize) {
  const uint32_t tid = thread_id(), nt = block_threads();
  const uint64_t P = d->page_size;
  const uint8_t* stg = d->staging + (uint64_t)bs->slot * d->max_req_bytes;
  if (bs->pull == 2) {
    const uint64_t q = bs->help_page;
    copy_block_aligned(d->frames + (uint64_t)(uint32_t)bs->frame * P, stg + (q - bs->first_page) * P,
                       staged_bytes(d, q, bs->first_page, bs->result, fsize), tid, nt);
    return;
  }
  for (uint32_t c = 0; c < bs->nclaim; ++c) {
    const uint32_t k = bs->lslot[c];
    const uint64_t q = bs->list[k];
    copy_block_aligned(d->frames + (uint64_t)bs->lframe[k] * P, stg + (q - bs->first_page) * P,
                       staged_bytes(d, q, bs->first_page, bs->result, fsize), tid, nt);
  }
}

/* Lane: publish a pulled frame VALID (reference bit set, ERR if the host read came short). */
__device__ __forceinline__ void publish_frame(const gfs_dev* d, uint32_t f, bool short_read) {
  uint64_t* fw = &d->fword[f];
  uint64_t w = ld_rlx(fw);
  while (true) {
    uint64_t nw = ((w & ~(GFS_FW_STATE | GFS_FW_PULL)) | GFS_FS_VALID | GFS_FW_REF) + GFS_FW_VER_ONE;
    if (short_read) nw |= GFS_FW_ERR;
    if (cas64(fw, w, nw)) break;
  }
}

/* Lane 0 (after the frames are published): count them off the request; the block that
 * publishes the last one frees the ring slot. */
__device__ __forceinline__ void request_done_lane(const gfs_dev* d, uint32_t s, uint64_t gen,
                                                  uint32_t cnt) {
  if (cnt == 0) return;
  const uint32_t before = __hip_atomic_fetch_sub(&d->reqd[s].remaining, cnt, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
  if (before == cnt) {
    st_rel(&d->slot_free[s], gen);
    if (s >= d->sync_slots) st_rel(&d->reqd[s].busy, 0ull);   /* an asynchronous window's slot */
  }
}

/* Wave 0, after the block's pull, a fence by every thread and a barrier: publish the frames
 * this block pulled and count them off. Returns the status of this block's page: for its
 * own request the demanded page (list[0]), which a helper may be pulling, so it may wait.
 * On an error the block's pin on its page has been dropped. */
__device__ int64_t publish_pull_wave(const gfs_dev* d, BlockState* bs, uint64_t fsize,
                                     uint64_t t0) {
  const uint32_t l = lane();
  uint32_t bad = 0;
  int64_t st = 0;
  if (bs->pull == 2) {
    if (l == 0) {
      const bool sh = staged_short(d, bs->help_page, bs->first_page, bs->result, fsize);
      publish_frame(d, (uint32_t)bs->frame, sh);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      request_done_lane(d, bs->slot, bs->gen, 1);
      bad = sh ? 1u : 0u;
      st = sh ? -kEIO : 0;
      if (sh) frame_unpin(d, (uint32_t)bs->frame);
    }
  } else {
    for (uint32_t c = l; c < bs->nclaim; c += 64) {
      const uint32_t k = bs->lslot[c];
      const bool sh = staged_short(d, bs->list[k], bs->first_page, bs->result, fsize);
      publish_frame(d, bs->lframe[k], sh);
      bad += sh ? 1u : 0u;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (l == 0) {
      request_done_lane(d, bs->slot, bs->gen, bs->nclaim);
      /* the demanded page: pulled here, or by a helper that may still be copying it (an
         asynchronous request has none: frame -1) */
      if (bs->frame >= 0) {
        st = wait_valid_lane(d, (uint32_t)bs->frame, t0);
        if (st == -kETIMEDOUT) bcount(bs, GFS_C_TIMEOUTS, 1);
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off, 64);
  if (l == 0) bcount(bs, GFS_C_IOERR, bad);
  return __shfl(st, 0, 64);
}

/* Block-collective: the private policy's fills. pull 3: the page from the block's private
 * buffer into its frame; pull 4: the staged request's first page into the frame and the
 * rest of the span into the private buffer. */
__device__ void private_pull(const gfs_dev* d, const BlockState* bs, uint64_t fsize) {
  const uint32_t tid = thread_id(), nt = block_threads();
  const uint64_t P = d->page_size;
  const uint32_t f = (uint32_t)bs->frame;
  const gfs_pslot* ps = &d->pslots[bs->pslot];
  uint8_t* pb = d->pbuf + (uint64_t)bs->pslot * d->ra_cap * P;
  if (bs->pull == 3) {
    const uint64_t q = bs->help_page;
    uint64_t n = fsize - (q << d->page_shift);
    if (n > P) n = P;
    copy_block_aligned(d->frames + (uint64_t)f * P, pb + (q - ps->first) * P, n, tid, nt);
    return;
  }
  const uint8_t* stg = d->staging + (uint64_t)bs->slot * d->max_req_bytes;
  copy_block_aligned(d->frames + (uint64_t)f * P, stg,
                     staged_bytes(d, bs->first_page, bs->first_page, bs->result, fsize), tid, nt);
  const int64_t rest = bs->result - (int64_t)P;
  if (rest > 0) copy_block_aligned(pb, stg + P, (uint64_t)rest, tid, nt);
}

/* Thread 0, after private_pull and a block barrier: publish the frame; for a host request,
 * free its ring slot and make the rest of the span the private buffer (only whole pages
 * unless the read stopped at the end of the file). 0 or -EIO (the pin is then dropped). */
__device__ int64_t private_publish_lane(const gfs_dev* d, BlockState* bs, uint64_t fsize) {
  gfs_pslot* ps = &d->pslots[bs->pslot];
  const uint32_t f = (uint32_t)bs->frame;
  if (bs->pull == 3) {
    publish_frame(d, f, false);
    ps->used += 1;
    return 0;
  }
  const uint64_t P = d->page_size;
  const bool short_page = staged_short(d, bs->first_page, bs->first_page, bs->result, fsize);
  publish_frame(d, f, short_page);
  if (short_page) bcount(bs, GFS_C_IOERR, 1);
  st_rel(&d->slot_free[bs->slot], bs->gen);
  const uint64_t off0 = bs->first_page << d->page_shift;
  uint64_t expect = (uint64_t)bs->list_n * P;
  if (expect > fsize - off0) expect = fsize - off0;
  const int64_t rest = bs->result - (int64_t)P;
  uint32_t n = 0;
  if (rest > 0) n = (uint32_t)((bs->result == (int64_t)expect) ? ((uint64_t)rest + P - 1) / P : (uint64_t)rest / P);
  bcount(bs, GFS_C_PB_WASTED, ps->n - ps->used);
  bcount(bs, GFS_C_RA_PAGES, n);
  ps->file = bs->file;
  ps->first = bs->first_page + 1;
  ps->n = n;
  ps->used = 0;
  if (short_page) {
    frame_unpin(d, f);
    return -kEIO;
  }
  return 0;
}

/* ------------------------------------------------------------------ asynchronous readahead
 * Sec. 2.3: Linux reads the next window while the reader still consumes the current one. A
 * stream's marker page (the page after the demanded one in a demand window, the first page
 * of an asynchronous window) carries GFS_FW_MARK from its allocation; the first block whose
 * access finds it clears it and, after copying its own page, advances the stream: window
 * [next, next + min(2 size, cap)), the run of unmapped pages from its start, posted to the
 * host with nobody waiting. Blocks that need one of its pages join the frame and pull it from
 * staging once the host is done (the ring slot says so); the block that posted the request
 * pulls the rest when it next needs to post, reaches the next marker, or closes the file. */

/* Wave-collective, outside the lock: reserve the run of unmapped pages that starts at ws,
   within [ws, ws + n), ascending into bs->list/lslot/lframe; returns its length and sets
   failed if a page found both buckets full. */
__device__ uint32_t reserve_from_wave(const gfs_dev* d, uint32_t file, uint64_t ws, uint32_t n, bool clip,
                                      BlockState* bs, uint32_t& failed) {
  const uint32_t l = lane();
  uint32_t count = 0, bad = 0;
  for (uint32_t base = 0; base < n; base += 64) {
    const bool valid = base + l < n;
    const uint64_t q = ws + base + l;
    const uint64_t key = page_key(file, q);
    uint32_t b1 = 0, b2 = 0;
    uint64_t e[2 * GFS_BUCKET_SLOTS];
    bool present = false, gone = false;
    if (valid) {
      key_buckets(d, key, b1, b2);
      pt_load_lane(d, b1, b2, e);
      gone = clip && shadow_lane(d, file, q);
#pragma unroll
      for (int i = 0; i < 2 * GFS_BUCKET_SLOTS; ++i) present |= (e[i] >> GFS_ENTRY_FRAME_BITS) == key;
    }
    const uint64_t stop = __ballot(!valid || present || gone);
    const uint32_t k = stop ? (uint32_t)__builtin_ctzll(stop) : 64u;
    if (l < k) {
      int cnt1 = 0, cnt2 = 0, f1 = -1, f2 = -1;
#pragma unroll
      for (int i = 0; i < GFS_BUCKET_SLOTS; ++i) {
        if (e[i]) ++cnt1;
        else if (f1 < 0) f1 = i;
        if (e[GFS_BUCKET_SLOTS + i]) ++cnt2;
        else if (f2 < 0) f2 = GFS_BUCKET_SLOTS + i;
      }
      int pick = cnt2 < cnt1 ? f2 : f1;
      if (pick < 0) pick = f1 >= 0 ? f1 : f2;
      int64_t slot = -1;
      if (pick >= 0) {
        uint64_t expect = 0;
        uint64_t* sp = slot_ptr(d, b1, b2, pick);
        if (cas64_rlx(sp, expect, (key << GFS_ENTRY_FRAME_BITS) | kReserved)) slot = (int64_t)(sp - d->pt);
        else slot = pt_reserve_lane(d, key);
      }
      bs->list[base + l] = (uint32_t)q;
      bs->lslot[base + l] = slot < 0 ? 0xffffffffu : (uint32_t)slot;
      bs->lframe[base + l] = GFS_NO_FRAME;
      bad |= slot < 0 ? 1u : 0u;
    }
    count = base + k;
    if (k < 64) break;
  }
  failed = (uint32_t)(__ballot(bad != 0) != 0);
  return count;
}

/* Wave 0, with no asynchronous request of the block outstanding: the block's access found
   marker page m of file `file`. Advance the stream whose marker m still is (lowest slot),
   reserve and allocate the window's unmapped run, and post it to the host without waiting;
   the request becomes the block's outstanding one. Gives up quietly when no stream names m,
   the window is empty, a running claim holds its first page, or no frame is free. */
__device__ __attribute__((noinline)) void async_issue_wave(const gfs_dev* d, uint32_t file, uint64_t m, uint64_t fsize, BlockState* bs,
                                 uint32_t bid, uint64_t t0) {
  const uint32_t l = lane();
  /* a slot of its own first: with none free the window is not issued (readers then miss at
     its first page and the stream goes on synchronously) */
  int32_t aslot = -1;
  if (l == 0) aslot = async_slot_take_lane(d, bid);
  aslot = __shfl(aslot, 0, 64);
  if (aslot < 0) return;
  const uint32_t s = (uint32_t)aslot;
  uint64_t ticket;
  /* the waiter announces no page of any window, so no holder marks it covered */
  const int lk = lock_file_wave(d, file, 0, 0x7fffffffull, t0, ticket, false);
  if (lk != LOCK_OWN) {
    if (l == 0) st_rel(&d->reqd[s].busy, 0ull);
    return;
  }
  __builtin_amdgcn_s_setprio(3);
  const RaState ras = ra_load_lane(&d->files[file], d->ra_recent, d->streams);
  uint64_t cl = 0;
  if (l < GFS_CLAIMS) cl = ld_rlx(&d->claims[file].e[l]);
  const uint64_t npages = d->files[file].npages;
  /* the window leaves out pages evicted after use, unless the marker page is one */
  const bool clip = !shadow_lane(d, file, m);
  drain_atomics();
  const uint64_t sm = __ballot(l < d->streams && ras.s_valid && ras.s_marker == (uint32_t)m);
  if (sm == 0) {
    unlock_file_wave(d, file, ticket, 0, 0);
    __builtin_amdgcn_s_setprio(0);
    if (l == 0) st_rel(&d->reqd[s].busy, 0ull);
    return;
  }
  const int j = __ffsll((unsigned long long)sm) - 1;
  const uint32_t clk = __shfl(ras.clk, 0, 64) + 1;
  const uint64_t ws = __shfl(ras.s_next, j, 64);
  const uint32_t sz = __shfl(ras.s_size, j, 64);
  const uint32_t cap = ra_cap_eff(d);
  const uint32_t wn = 2 * sz < cap ? 2 * sz : cap;
  gfs_file_dev* fe = &d->files[file];
  if (l == 0) {
    gfs_stream* st = &fe->streams[j];
    st_rlx(&st->next, ws + wn);
    st_rlx32(&st->size, wn);
    st_rlx32(&st->last_use, clk);
    st_rlx32(&st->marker, (uint32_t)ws);
    st_rlx32(&fe->clock, clk);
  }
  const uint32_t wnc = ws < npages ? (uint32_t)((npages - ws) < wn ? (npages - ws) : wn) : 0u;
  if (l == 0) {
    trace_ev(d, 1, GFS_EV_ADV, bid, file, (uint32_t)m, 0, wnc, ws);
    bcount(bs, GFS_C_ADVANCES, 1);
  }
  /* a running claim on the first page: that block is fetching it; else stop at the next claim */
  const bool cl_on = l < GFS_CLAIMS && (cl & 1ull);
  const uint64_t cl_lo = cl >> 32, cl_hi = (cl >> 32) + ((cl & 0xffffffffull) >> 1);
  const bool held = __ballot(cl_on && cl_lo <= ws && ws < cl_hi) != 0;
  const uint64_t free_cl = __ballot(l < GFS_CLAIMS && !cl_on);
  uint64_t hi_b = cl_on && cl_lo > ws ? cl_lo : ~0ull;
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t b = __shfl_xor(hi_b, off, 64);
    hi_b = b < hi_b ? b : hi_b;
  }
  const uint64_t cwe = ws + wnc < hi_b ? ws + wnc : hi_b;
  if (wnc == 0 || held || free_cl == 0 || cwe <= ws) {
    unlock_file_wave(d, file, ticket, 0, 0);
    __builtin_amdgcn_s_setprio(0);
    if (l == 0) st_rel(&d->reqd[s].busy, 0ull);
    return;
  }
  const uint32_t cj = (uint32_t)__builtin_ctzll(free_cl);
  uint64_t* claim = &d->claims[file].e[cj];
  if (l == 0) st_rlx(claim, (ws << 32) | ((cwe - ws) << 1) | 1ull);
  unlock_file_wave(d, file, ticket, ws, cwe);
  __builtin_amdgcn_s_setprio(0);
  uint32_t failed = 0;
  const uint32_t n = reserve_from_wave(d, file, ws, (uint32_t)(cwe - ws), clip, bs, failed);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (l == 0) st_rlx(claim, 0ull);
  wave_sync_lds();
  uint32_t keep = n;
  if (failed) {
    uint32_t firstbad = n;
    for (uint32_t i = l; i < n; i += 64)
      if (bs->lslot[i] == 0xffffffffu) firstbad = i < firstbad ? i : firstbad;
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t o = __shfl_xor(firstbad, off, 64);
      firstbad = o < firstbad ? o : firstbad;
    }
    keep = firstbad;
  }
  /* no demanded page: every page is prefetched; the window's first page is the new marker */
  const uint32_t got = keep ? alloc_wave(d, file, ~0ull, bs, keep, bid, ws) : 0;
  for (uint32_t i = got + l; i < n; i += 64)
    if (bs->lslot[i] != 0xffffffffu) st_rel(d->pt + bs->lslot[i], 0ull);
  if (got == 0) {
    if (l == 0) st_rel(&d->reqd[s].busy, 0ull);
    return;
  }
  if (got < n && l == 0) trace_ev(d, 1, GFS_EV_NOFRAME, bid, file, bs->list[got], GFS_NO_FRAME, 0, 0);
  /* the pages that got frames are [ws, ws + got) */
  const uint64_t off0 = ws << d->page_shift;
  uint64_t len = (uint64_t)got << d->page_shift;
  if (off0 + len > fsize) len = fsize - off0;
  /* the slot is this window's alone: its staging is free once its last request was counted
     off (that cleared busy), and its next generation is one past the last completed */
  acquire_agent();
  const uint64_t gen = ld_rlx(&d->slot_free[s]) + 1;
  const uint64_t tk = (gen - 1) * d->rpc_slots + s;   /* for the trace only */
  if (l == 0)   /* frames count themselves off the request as they are published */
    __hip_atomic_store(&d->reqd[s].remaining, got, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t fill = (1ull << 63) | ((uint64_t)(s + 1) << 40) | (gen & ((1ull << 40) - 1));
  for (uint32_t k = l; k < got; k += 64) st_rel(&d->ffill[bs->lframe[k]], fill);
  if (l == 0) {
    gfs_rpc_slot* rs = &d->ring[s];
    rs->file_id = file;
    rs->npages = got;
    rs->offset = off0;
    rs->length = len;
    rs->ticket = tk;
    __hip_atomic_store(&rs->req_seq, gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    trace_ev(d, 1, GFS_EV_REQ, bid, file, (uint32_t)ws, GFS_NO_FRAME, got, tk);
    bcount(bs, GFS_C_REQUESTS, 1);
    bcount(bs, GFS_C_REQ_BYTES, len);
    bcount(bs, GFS_C_FETCHED, got);
    bcount(bs, GFS_C_RA_PAGES, got);
    bs->a_pending = 1;
    bs->a_slot = s;
    bs->a_gen = gen;
    bs->a_first = ws;
    bs->a_n = got;
    bs->a_file = file;
  }
}

/* Block-collective: finish the block's outstanding asynchronous request, if any: wait for the
   host, pull every frame no other block has claimed, publish them. 0 or -ETIMEDOUT. */
__device__ __attribute__((noinline)) int64_t async_finish_block(const gfs_dev* d, BlockState* bs) {
  const uint32_t tid = thread_id();
  __syncthreads();
  if (!bs->a_pending) return 0;
  const uint64_t t0 = wall_clock64();
  if (tid == 0) {
    gfs_rpc_slot* rs = &d->ring[bs->a_slot];
    uint32_t nn = 0;
    int st = 0;
    const uint64_t th0 = wall_clock64();
    /* the slot's generations only grow: one past a_gen means the host finished this request,
       blocks that joined its frames pulled and published every one of them, and the slot went
       to a later request (nothing is left to claim: no frame's fill word names this one) */
    uint64_t ds;
    while ((int64_t)((ds = __hip_atomic_load(&rs->done_seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) -
                     bs->a_gen) < 0) {
      if (expired(d, t0)) {
        st = -kETIMEDOUT;
        break;
      }
      nap(nn);
    }
    acquire_system();   /* the staged bytes, written by the host before done_seq */
    bcount(bs, GFS_T_HOST, wall_clock64() - th0);
    if (st) bcount(bs, GFS_C_TIMEOUTS, 1);
    if (st == 0 && ds != bs->a_gen) st = 1;   /* done, and nothing left to pull */
    bs->a_status = st;
    bs->result = rs->result;
    bs->slot = bs->a_slot;
    bs->gen = bs->a_gen;
    bs->first_page = bs->a_first;
    bs->list_n = bs->a_n;
    bs->frame = -1;
    bs->pull = 1;
  }
  __syncthreads();
  int64_t st = bs->a_status;
  if (st == 0) {
    const uint64_t fsize = d->files[bs->a_file].size;
    if (tid < 64)
      claim_pulls_wave(d, bs, (1ull << 63) | ((uint64_t)(bs->a_slot + 1) << 40) | (bs->a_gen & ((1ull << 40) - 1)));
    __syncthreads();
    block_pull(d, bs, fsize);
    __threadfence();
    __syncthreads();
    if (tid < 64) (void)publish_pull_wave(d, bs, fsize, t0);
  }
  __syncthreads();
  if (tid == 0) {
    bs->a_pending = 0;
    bs->pull = 0;
  }
  __syncthreads();
  return st < 0 ? st : 0;
}

}  // namespace gfsd

/* ====================================================================== public API */

__device__ int gopen_id(const gfs_dev* d, int file_id, int flags) {
  gfsd::BlockState* bs = gfsd::block_state();
  if (gfsd::thread_id() == 0) {
    int v;
    if (flags != GFS_O_RDONLY) {
      v = -gfsd::kEROFS;
    } else if (file_id < 0 || (uint32_t)file_id >= d->max_files ||
               gfsd::ld_rlx32(&d->files[file_id].open) == 0) {
      v = -gfsd::kENOENT;
    } else {
      __hip_atomic_fetch_add(&d->files[file_id].handles, 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      v = file_id;
    }
    bs->pslot = -1;
    if (v >= 0 && d->policy == GFS_POLICY_PRIVATE) {
      /* the block's private slot: its own frames and private buffer until gclose. A slot
         given back by a block that just ended may not show yet: look again, with naps,
         until the wait timeout */
      const uint64_t t0 = wall_clock64();
      uint32_t naps = 0;
      while (bs->pslot < 0) {
        for (uint32_t i = 0; i < d->npslots && bs->pslot < 0; ++i) {
          const uint32_t s = (gfsd::block_id() + i) % d->npslots;
          uint32_t z = 0;
          if (gfsd::ld_rlx32(&d->pslots[s].owner) == 0 && gfsd::cas32(&d->pslots[s].owner, z, 1u))
            bs->pslot = (int32_t)s;
        }
        if (bs->pslot >= 0 || gfsd::expired(d, t0)) break;
        gfsd::nap(naps);
      }
      if (bs->pslot < 0) {
        __hip_atomic_fetch_sub(&d->files[file_id].handles, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v = -gfsd::kENOSPC;
      } else {
        gfs_pslot* ps = &d->pslots[bs->pslot];
        ps->n = 0;   /* a new owner starts with an empty private buffer */
        ps->used = 0;
      }
    }
    for (int c = 0; c < GFS_C_COUNT; ++c) bs->ctr[c] = 0;
    bs->pull = 0;
    bs->trig = 0;
    bs->a_pending = 0;   /* an asynchronous request is finished by gclose, before the next gopen */
    bs->open_result = v;
    bs->open_fd = v;
    bs->open_size = v >= 0 ? d->files[v].size : 0;
  }
  __syncthreads();
  const int v = bs->open_result;
  __syncthreads();
  return v;
}

__device__ int gopen(const gfs_dev* d, const char* path, int flags) {
  gfsd::BlockState* bs = gfsd::block_state();
  if (gfsd::thread_id() == 0) {
    int id = -1;
    for (uint32_t i = 0; i < d->max_files && id < 0; ++i) {
      if (gfsd::ld_rlx32(&d->files[i].open) == 0) continue;
      const char* nm = d->names + (uint64_t)i * GFS_NAME_MAX;
      uint32_t j = 0;
      while (j < GFS_NAME_MAX && nm[j] == path[j] && nm[j] != 0) ++j;
      if (j < GFS_NAME_MAX && nm[j] == 0 && path[j] == 0) id = (int)i;
    }
    bs->open_result = id;
  }
  __syncthreads();
  const int id = bs->open_result;
  __syncthreads();
  if (flags != GFS_O_RDONLY) return -gfsd::kEROFS;
  if (id < 0) return -gfsd::kENOENT;
  return gopen_id(d, id, flags);
}

__device__ int gclose(const gfs_dev* d, int fd) {
  if (fd < 0 || (uint32_t)fd >= d->max_files) return -gfsd::kEBADF;
  gfsd::BlockState* bs = gfsd::block_state();
  /* an asynchronous request still outstanding is pulled in before the block lets go */
  (void)gfsd::async_finish_block(d, bs);
  __syncthreads();
  if (gfsd::thread_id() == 0) {
    __hip_atomic_fetch_sub(&d->files[fd].handles, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (d->policy == GFS_POLICY_PRIVATE && bs->pslot >= 0) {
      gfs_pslot* ps = &d->pslots[bs->pslot];
      bs->ctr[GFS_C_PB_WASTED] += ps->n - ps->used;   /* the private buffer is dropped */
      ps->n = 0;
      ps->used = 0;
      __hip_atomic_store(&ps->owner, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      bs->pslot = -1;
    }
    for (int c = 0; c < GFS_C_COUNT; ++c) {
      if (bs->ctr[c]) gfsd::fadd64(&d->g->ctr[c], bs->ctr[c]);
      bs->ctr[c] = 0;
    }
    bs->open_fd = -1;
  }
  __syncthreads();
  return 0;
}

__device__ __attribute__((always_inline)) int64_t gread(const gfs_dev* d, int fd, uint64_t offset,
                                                        uint64_t size, void* dst) {
  using namespace gfsd;
  BlockState* bs = block_state();
  if (fd < 0 || (uint32_t)fd >= d->max_files) return -kEBADF;
  uint64_t fsize;
  if (fd == bs->open_fd) {
    fsize = bs->open_size;   /* checked by gopen */
  } else {
    gfs_file_dev* fe = &d->files[fd];
    if (ld_rlx32(&fe->open) == 0) return -kEBADF;
    fsize = fe->size;
  }
  const uint32_t nt = block_threads();
  if (nt & 63u) return -kEINVAL;
  if (size == 0 || offset >= fsize) return 0;
  const uint64_t end = (size > fsize - offset) ? fsize : offset + size;
  const uint32_t tid = thread_id();
  const uint32_t bid = block_id();
  const uint64_t P = d->page_size;
  const uint32_t sh_bits = d->page_shift;
  const uint64_t pfirst = offset >> sh_bits, plast = (end - 1) >> sh_bits;
  int64_t err = 0;
  /* Reads of several pages first take every page that is cached and valid in one pass:
     lane i of wave 0 looks up and pins page base + i, the block copies all of them, and
     the pins are dropped together. The remaining pages (misses, frames being filled) go
     through the one-page path below, in order. Off while the policy trace is recorded, so
     that a traced run makes its accesses one at a time in page order. */
  const bool batched = plast > pfirst && d->trace_level == 0;
  if (batched) {
    const uint32_t cnt = (uint32_t)((plast - pfirst + 1) < 64 ? (plast - pfirst + 1) : 64);
    const uint64_t tb0 = d->page_timers ? wall_clock64() : 0;
    if (tid < 64) {
      int32_t f = -1;
      if (tid < cnt) {
        const uint64_t key = page_key((uint32_t)fd, pfirst + tid);
        f = pt_find_lane(d, key);
        if (f >= 0 && (uint32_t)f != kReserved) {
          uint64_t w = 0;
          const int r = frame_pin(d, (uint32_t)f, key, &w);
          if (r != PIN_VALID || (d->ra_async && (w & GFS_FW_MARK))) {
            /* the one-page path joins a filling frame, and takes a marker page's mark */
            if (r == PIN_FILLING || r == PIN_VALID) frame_unpin(d, (uint32_t)f);
            f = -1;
          }
        } else {
          f = -1;
        }
      }
      bs->bframe[tid] = f;
      const uint64_t got = __ballot(f >= 0);
      if (tid == 0) bcount(bs, GFS_C_HITS, (uint64_t)__popcll(got));
    }
    __syncthreads();
    /* whole pages: one pass over all their 16-byte units, eight in flight per thread */
    const bool aligned = ((((uintptr_t)dst) | offset) & 15) == 0;
    const uint32_t ush = sh_bits - 4;
    const uint64_t total = (uint64_t)cnt << ush;
    if (aligned) {
      for (uint64_t u0 = tid; u0 < total; u0 += 8ull * nt) {
        v4u a[8];
        bool ok[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const uint64_t u = u0 + (uint64_t)j * nt;
          const uint32_t i = (uint32_t)(u >> ush);
          const uint64_t pos = ((pfirst + i) << sh_bits) + ((u & ((1ull << ush) - 1)) << 4);
          const int32_t f = u < total ? bs->bframe[i] : -1;
          ok[j] = f >= 0 && pos >= offset && pos + 16 <= end;
          if (ok[j]) a[j] = ((const gv4u*)(d->frames + (uint64_t)f * P))[u & ((1ull << ush) - 1)];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const uint64_t u = u0 + (uint64_t)j * nt;
          const uint64_t pos = ((pfirst + (u >> ush)) << sh_bits) + ((u & ((1ull << ush) - 1)) << 4);
          if (ok[j]) ((gv4u*)((uint8_t*)dst + (pos - offset)))[0] = a[j];
        }
      }
    }
    /* bytes the unit pass left: unaligned buffers, and the ends of partly covered pages */
    for (uint32_t i = 0; i < cnt; ++i) {
      const int32_t f = bs->bframe[i];
      if (f < 0) continue;
      const uint64_t pbase = (pfirst + i) << sh_bits;
      const uint64_t lo = offset > pbase ? offset : pbase;
      const uint64_t hi = end < pbase + P ? end : pbase + P;
      if (!aligned) {
        copy_block((uint8_t*)dst + (lo - offset), d->frames + (uint64_t)f * P + (lo - pbase), hi - lo, tid, nt);
      } else {
        /* units cover [lo16, hi16): copy the head and tail bytes outside them */
        const uint64_t lo16 = (lo + 15) & ~15ull, hi16 = hi & ~15ull;
        for (uint64_t b = lo + tid; b < (lo16 < hi ? lo16 : hi); b += nt)
          ((uint8_t*)dst)[b - offset] = d->frames[(uint64_t)f * P + (b - pbase)];
        for (uint64_t b = (hi16 > lo16 ? hi16 : lo16) + tid; b < hi; b += nt)
          ((uint8_t*)dst)[b - offset] = d->frames[(uint64_t)f * P + (b - pbase)];
      }
    }
    __syncthreads();
    if (tid < cnt && bs->bframe[tid] >= 0) frame_unpin(d, (uint32_t)bs->bframe[tid]);
    if (tid == 0 && d->page_timers) bcount(bs, GFS_T_COPY, wall_clock64() - tb0);
    __syncthreads();
  }
  if (tid == 0) bs->read_last = plast;   /* read by wave 0's miss path, after this store */
  for (uint64_t p = pfirst; p <= plast; ++p) {
    if (batched && p - pfirst < 64 && bs->bframe[p - pfirst] >= 0) continue;
    const bool ptm = d->page_timers != 0;
    const uint64_t ta0 = ptm ? wall_clock64() : 0;
    if (tid < 64) acquire_page_wave(d, (uint32_t)fd, p, fsize, bs, bid);
    __syncthreads();
    if (bs->pull == 5) {
      /* a miss while this block's asynchronous request is outstanding: finish it, look again */
      const int64_t e = async_finish_block(d, bs);
      if (e < 0) {
        err = e;
        break;
      }
      --p;   /* the same page again (unsigned wrap at 0 is undone by the loop's ++p) */
      continue;
    }
    if (bs->pull >= 3) {
      const uint64_t tp0 = wall_clock64();
      private_pull(d, bs, fsize);
      __threadfence();
      __syncthreads();
      if (tid == 0) {
        const int64_t st = private_publish_lane(d, bs, fsize);
        if (st < 0) bs->status = st;
        bs->pull = 0;
        bcount(bs, GFS_T_PULL, wall_clock64() - tp0);
      }
      __syncthreads();
    } else if (bs->pull) {
      const uint64_t tp0 = wall_clock64();
      if (bs->pull == 1) {
        if (tid < 64)
          claim_pulls_wave(d, bs, ((uint64_t)(bs->slot + 1) << 40) | (bs->gen & ((1ull << 40) - 1)));
        __syncthreads();
      }
      block_pull(d, bs, fsize);
      __threadfence();
      __syncthreads();
      if (tid < 64) {
        const int64_t st = publish_pull_wave(d, bs, fsize, wall_clock64());
        if (tid == 0) {
          if (st < 0) bs->status = st;
          bs->pull = 0;
          bcount(bs, GFS_T_PULL, wall_clock64() - tp0);
        }
      }
      __syncthreads();
    }

    const int64_t st = bs->status;
    const int32_t f = bs->frame;
    if (st < 0) {
      err = st;
      __syncthreads();
      break;
    }
    const uint64_t ta1 = ptm ? wall_clock64() : 0;
    const uint64_t pbase = p << sh_bits;
    const uint64_t lo = offset > pbase ? offset : pbase;
    const uint64_t hi = end < pbase + P ? end : pbase + P;
    /* a hit pinned with its tag unchecked: thread 0's tag load goes out just before its share
       of the copy, so the check costs no round trip of its own; if the frame turns out to hold
       another page (reused between the lookup and the pin), the bytes copied to dst are
       overwritten by the next look (gread has not returned, so nobody may read dst yet) */
    const uint64_t tk = bs->tagkey;
    uint64_t tag = 0;
    if (tk && tid == 0) tag = ld_rlx(&d->ftag[f]);
    copy_block((uint8_t*)dst + (lo - offset), d->frames + (uint64_t)f * P + (lo - pbase), hi - lo,
               tid, nt);
    if (tk && tid == 0) {
      const bool ok = tag == tk;
      bs->tag_ok = ok ? 1 : 0;
      if (ok && d->ra_async && (bs->pinw & GFS_FW_MARK)) bs->trig = mark_take_lane(d, (uint32_t)f) ? 1u : 0u;
    }
    __syncthreads();
    const bool trig = bs->trig != 0;
    if (tk && !bs->tag_ok) {
      __syncthreads();
      if (tid == 0) {
        frame_unpin(d, (uint32_t)f);
        bcount(bs, GFS_C_RETRIES, 1);
      }
      --p;   /* look the same page up again (unsigned wrap at 0 is undone by the loop's ++p) */
      continue;
    }
    if (tid == 0) {
      if (tk) {
        frame_pin_bits(d, (uint32_t)f, bs->pinw);
        bcount(bs, GFS_C_HITS, 1);
      }
      if (ptm) {
        const uint64_t ta2 = wall_clock64();
        frame_unpin(d, (uint32_t)f);
        bcount(bs, GFS_T_ACQUIRE, ta1 - ta0);
        bcount(bs, GFS_T_COPY, ta2 - ta1);
        bcount(bs, GFS_T_UNPIN, wall_clock64() - ta2);
      } else {
        frame_unpin(d, (uint32_t)f);
      }
    }
    if (trig) {
      /* this access took its stream's marker: finish the block's previous asynchronous
         request, then issue the stream's next window without waiting for it */
      const int64_t e = async_finish_block(d, bs);
      if (e < 0) {
        err = e;
        break;
      }
      if (tid < 64) async_issue_wave(d, (uint32_t)fd, p, fsize, bs, bid, wall_clock64());
      __syncthreads();
    }
  }
  if (err) return err;
  if (tid == 0) bcount(bs, GFS_C_DELIVERED, end - offset);
  return (int64_t)(end - offset);
}

#endif /* GFS_DEVICE_H */
