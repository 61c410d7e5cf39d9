/* gfs_layout.h -- memory layout shared by the host runtime and the device library.
 *
 * Internal to the library (users include gfs.h and gfs_device.h). Everything here is
 * plain data: the device handle, the per-file and global records in HBM, the frame
 * word and page-table entry encodings, and the request-ring slot in pinned host memory.
 *
 * HBM layout of the metadata region (offsets computed by the host, stored in gfs_dev):
 *   gfs_globals                      384 B
 *   gfs_dev (the handle)             512 B
 *   files[max_files]                 768 B each
 *   locks[max_files]                 128 B each (miss ticket locks)
 *   lockq[max_files][GFS_LOCK_SLOTS] u64   queue slots of the miss locks (32 KiB per file)
 *   claims[max_files]                128 B each (windows being reserved)
 *   pslots[private_slots]            64 B each (private policy)
 *   names[max_files]                 GFS_NAME_MAX B each (registered paths)
 *   fword[nframes]  u64              frame word (state, pins, ref, ra, version)
 *   ftag[nframes]   u64              key of the page held (valid while not FREE)
 *   pt[nbuckets*16] u64              hashed page table, 16-entry buckets (128 B)
 *   ffill[nframes]  u64              ring slot and generation filling the frame (0: not yet known)
 *   slot_free[rpc_slots] u64         generation of the last completed use of each ring slot
 *   slot_tail[rpc_slots] u64         partitioned queue: requests posted into each slot
 *   reqd[rpc_slots]                  64 B: a finished host read, for blocks that help pull it
 *   trace[trace_capacity]            32 B records
 * Frames (cache_bytes) are a separate caller allocation. The ring and staging live in
 * pinned, device-mapped host memory owned by the context.
 */
#ifndef GFS_LAYOUT_H
#define GFS_LAYOUT_H

#include <stdint.h>

/* ---- frame word (64 bit), changed only by compare-and-swap, version bumped each time ---- */
#define GFS_FS_FREE 0ull
#define GFS_FS_CLAIMED 1ull   /* owned by an allocator; not pinnable, not visible */
#define GFS_FS_FILLING 2ull   /* mapped, data on its way; pinnable (joiners wait) */
#define GFS_FS_VALID 3ull     /* mapped, data present */
#define GFS_FW_STATE 0x3ull
#define GFS_FW_REF (1ull << 2)   /* clock reference bit */
#define GFS_FW_RA (1ull << 3)    /* prefetched, not yet demanded */
#define GFS_FW_ERR (1ull << 4)   /* the host read for this page failed */
#define GFS_FW_PULL (1ull << 5)  /* filling, and a block is copying the bytes into the frame */
#define GFS_FW_MARK (1ull << 6)  /* asynchronous readahead: the page is its stream's marker; the
                                    first block to find it advances the stream */
#define GFS_FW_PIN_SHIFT 8
#define GFS_FW_PIN_ONE (1ull << GFS_FW_PIN_SHIFT)
#define GFS_FW_PINS (0xffffull << GFS_FW_PIN_SHIFT)
#define GFS_FW_VER_SHIFT 32
#define GFS_FW_VER_ONE (1ull << GFS_FW_VER_SHIFT)

/* ---- page key and page-table entry ----
 * key = (file+1) << 28 | page   (39 bits, never 0)
 * entry = key << 24 | frame      (0 = empty slot)                                  */
#define GFS_KEY_PAGE_BITS 28
#define GFS_ENTRY_FRAME_BITS 24
#define GFS_BUCKET_SLOTS 16
#define GFS_NO_FRAME 0xffffffffu

typedef struct gfs_globals {
  uint64_t hand;          /* clock hand ticket counter */
  uint64_t ring_tail;     /* request ring ticket counter */
  uint64_t trace_n;       /* trace records appended (including dropped) */
  uint64_t pad0[5];
  uint64_t ctr[40];       /* device counters, GFS_C_* */
} gfs_globals;

enum {
  GFS_C_HITS = 0, GFS_C_JOINS, GFS_C_MISSES, GFS_C_RA_PAGES, GFS_C_FETCHED, GFS_C_EVICTIONS,
  GFS_C_WASTED, GFS_C_HAND, GFS_C_REQUESTS, GFS_C_REQ_BYTES, GFS_C_DELIVERED, GFS_C_RETRIES,
  GFS_C_NOFRAME, GFS_C_TIMEOUTS, GFS_C_IOERR,
  /* wall-clock ticks summed over blocks, by phase of the miss path */
  GFS_T_LOCK, GFS_T_CRIT, GFS_T_ALLOC, GFS_T_SLOT, GFS_T_HOST, GFS_T_PULL, GFS_T_JOIN,
  /* readahead decision and unlock (parts of GFS_T_CRIT); run finding + reservation
     (after the unlock, under a window claim) */
  GFS_T_DECIDE, GFS_T_RUN, GFS_T_UNLOCK,
  GFS_C_LOCKS,       /* miss locks taken */
  GFS_C_LOCK_LEFT,   /* waits for a miss lock given up because the page appeared */
  /* every page gread serves, summed over blocks: finding and pinning it (hit, join or
     miss, including pulls), copying it out, dropping the pin */
  GFS_T_ACQUIRE, GFS_T_COPY, GFS_T_UNPIN,
  GFS_C_PB_HITS,     /* private policy: misses filled from the private buffer */
  GFS_C_PB_WASTED,   /* private policy: private-buffer pages dropped unused */
  GFS_C_ADVANCES,    /* asynchronous readahead: windows issued at a marker page */
  GFS_C_COUNT
};
typedef char gfs_counters_fit[(GFS_C_COUNT <= 40) ? 1 : -1];   /* gfs_globals.ctr */

/* room for the readahead detector's recent misses (the configured count, ra_recent, is at
   most this: one per lane of the deciding wave) */
#define GFS_RECENT_MISSES 64

typedef struct gfs_stream {
  uint64_t next;          /* first page after the last window */
  uint32_t size;          /* last window length (pages) */
  uint32_t last_use;      /* per-file decision clock at last use */
  uint32_t valid;
  uint32_t marker;        /* asynchronous readahead: the page whose first access advances the
                             stream (GFS_NO_MARKER: none) */
} gfs_stream;             /* 24 B */
#define GFS_NO_MARKER 0xffffffffu

typedef struct gfs_file_dev {
  uint64_t size;          /* bytes */
  uint32_t npages;
  uint32_t open;          /* 1 while registered */
  uint32_t advice;        /* GFS_ADV_* */
  uint32_t pad0;
  uint32_t clock;         /* readahead decision counter (stream last_use) */
  uint32_t handles;       /* device gopen count minus gclose count */
  gfs_stream streams[8];  /* 192 B */
  uint64_t recent[GFS_RECENT_MISSES];  /* pages of the last misses (ring) */
  uint32_t recent_n;      /* misses pushed into the ring so far */
  uint32_t pad[7];
} gfs_file_dev;           /* 768 B */

/* per-file miss lock: a ticket lock on a cache line of its own, so that waiters polling
   it do not slow the holder's accesses to the file record */
typedef struct gfs_file_lock {
  uint64_t next;          /* tickets handed out */
  uint64_t pad[15];
} gfs_file_lock;          /* 128 B */

/* queue slots of each file's miss lock (u64 each); at least the number of blocks that can
   wait on one lock at once. Every block that calls gread holds at least GFS_BLOCK_LDS_MIN
   bytes of LDS for its per-block state, so a CU holds at most LDS / GFS_BLOCK_LDS_MIN such
   blocks (12 on a 160 KiB CU, 3072 on 256 CUs); gfs_init checks the device. */
#define GFS_LOCK_SLOTS 4096u

/* pages per file whose eviction after use is remembered, one bit each (64 KiB per file id);
   later pages of a larger file are not tracked */
#define GFS_SHADOW_PAGES (1u << 19)
#define GFS_BLOCK_LDS_MIN 12288u

/* window claims: a block that decided a window under the miss lock records it here and
   reserves the window's pages after unlocking; other misses inside an active claim wait for
   it, and later windows are clipped to stay out of it. Entry = start << 32 | len << 1 | 1
   (0 = free). */
#define GFS_CLAIMS 16

/* private policy: one per slot; the slot's frames are [slot * quota, (slot + 1) * quota) and
   its private buffer holds pages [first, first + n) of file `file` */
typedef struct gfs_pslot {
  uint32_t owner;         /* 1 while a block holds the slot */
  uint32_t file;
  uint64_t first;
  uint32_t n;             /* pages in the buffer */
  uint32_t used;          /* of them, taken into the cache */
  uint32_t lra_next;      /* next frame of the share to (re)allocate */
  uint32_t pad[9];
} gfs_pslot;              /* 64 B */
typedef struct gfs_file_claims {
  uint64_t e[GFS_CLAIMS];
} gfs_file_claims;        /* 128 B */

#define GFS_NAME_MAX 256     /* registered path, NUL-terminated, for gopen(path) */

/* request ring slot in pinned host memory: the device writes the first cache line,
 * the host the second */
typedef struct gfs_rpc_slot {
  uint64_t req_seq;       /* generation, published last (system-scope release) */
  uint32_t file_id;
  uint32_t npages;        /* pages in the span */
  uint64_t offset;        /* file byte offset of the first page */
  uint64_t length;        /* bytes to read (span, clamped to EOF) */
  uint64_t ticket;
  uint64_t pad0[3];
  uint64_t done_seq;      /* generation completed, published last by the host */
  int64_t result;         /* bytes read, or -errno */
  uint64_t t_claim_ns;
  uint64_t t_done_ns;
  uint64_t pad1[4];
} gfs_rpc_slot;           /* 128 B */

/* a ring slot's finished host read, published by the requester so that blocks waiting on
   frames of the request can copy their own pages from staging */
typedef struct gfs_req_dev {
  uint64_t ready;         /* generation whose bytes are in staging */
  int64_t result;         /* host read result (bytes or -errno) */
  uint64_t first_page;    /* first page of the span */
  uint32_t remaining;     /* frames of the request not yet published */
  uint32_t file;
  uint64_t busy;          /* slots of asynchronous windows: 1 while a window holds the slot */
  uint64_t pad[3];
} gfs_req_dev;            /* 64 B */

typedef struct gfs_dev {
  uint64_t page_size;
  uint32_t page_shift;
  uint32_t nframes;
  uint32_t nbuckets_mask;       /* buckets - 1 (power of two) */
  uint32_t streams;
  uint32_t ra_init;             /* pages */
  uint32_t ra_cap;              /* pages; 0 = readahead off */
  uint32_t rpc_slots;
  uint32_t max_req_pages;
  uint32_t trace_level;
  uint32_t trace_cap;
  uint32_t max_files;           /* file ids below this are valid */
  uint32_t ra_recent;           /* detector: misses remembered per file (<= GFS_RECENT_MISSES) */
  uint32_t ra_near_pages;       /* detector: "near" radius */
  uint32_t ra_near_min;         /* detector: near misses that mark aggregate reading */
  uint32_t ra_quota_blocks;     /* thrash guard: resident blocks the cache is shared by */
  uint32_t ra_async;            /* 1: marker-triggered (asynchronous) readahead */
  uint32_t sync_slots;          /* ring slots [0, sync_slots) take ticketed requests; the rest are
                                   the asynchronous windows' own (taken without waiting) */
  uint32_t page_timers;         /* gfs_config.page_timers */
  uint64_t max_req_bytes;
  uint64_t timeout_ticks;       /* wall_clock64 ticks */
  uint8_t* frames;
  uint64_t* fword;
  uint64_t* ftag;
  uint64_t* pt;
  gfs_globals* g;
  gfs_file_dev* files;
  gfs_file_lock* locks;
  uint64_t* lockq;              /* [max_files][GFS_LOCK_SLOTS] miss-lock queue slots */
  gfs_file_claims* claims;      /* [max_files] windows being reserved */
  uint64_t* shadow;             /* [max_files][GFS_SHADOW_PAGES / 64]: bit set once the page was
                                   evicted after it was consumed (cleared with the cache) */
  gfs_pslot* pslots;            /* private policy: [private_slots] */
  uint8_t* pbuf;                /* private policy: [private_slots][ra_cap pages] in the frames allocation */
  uint32_t policy;              /* GFS_POLICY_* */
  uint32_t npslots;             /* private slots */
  uint32_t quota;               /* frames per private slot */
  uint32_t partitioned;         /* 1: a block posts into the slot of its block id */
  uint64_t* slot_free;
  uint64_t* slot_tail;          /* partitioned queue: requests posted into each slot so far */
  uint64_t* ffill;              /* per frame: (slot + 1) << 40 | generation of the request filling
                                   it, bit 63 set for an asynchronous request (0: not yet known) */
  gfs_req_dev* reqd;
  uint32_t* req_frames;
  void* trace;                  /* gfs_event[trace_cap] */
  char* names;                  /* [max_files][GFS_NAME_MAX] registered paths */
  gfs_rpc_slot* ring;           /* device-visible address of the pinned ring */
  uint8_t* staging;             /* device-visible address of the pinned staging */
} gfs_dev;

#endif /* GFS_LAYOUT_H */
