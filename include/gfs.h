/* gfs.h -- host C-ABI of the GPU-resident file page cache with readahead.
 *
 * The operation (Sec. 2.2 of the paper, "GPUfs"): GPU threadblocks read files
 * through a POSIX-like call made by every thread of the block; the library keeps
 * a page cache in GPU memory, serves hits from it, and forwards misses to host
 * threads that read the file and hand the data to the GPU. Sec. 4 adds a GPU-side
 * readahead prefetcher (a miss asks the host for the page plus a prefetch
 * window), enabled for read-only files and switchable off by an fadvise-style
 * hint; Sec. 5 adds a replacement mechanism that reuses frames in place so files
 * larger than the cache stream through.
 *
 * This header is the host side: create a cache over caller-owned device memory,
 * register files, read statistics and the event trace, reset, shut down. The
 * device side (gopen/gread/gclose, called from HIP kernels) is in gfs_device.h.
 * Workload launchers used by the benchmarks and tests are declared at the end.
 *
 * Conventions for every function returning int: 0 on success or a negative errno
 * value; out-parameters are left untouched on error. All pointers are plain host
 * or device addresses as stated per argument; no call takes ownership of caller
 * memory unless stated. Host calls on one context are not thread-safe with each
 * other, except gfs_stats.
 */
#ifndef GFS_H
#define GFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GFS_ABI_VERSION 5u

/* limits of the encoding (page-table entry = file:11 | page:28 | frame:24 bits) */
#define GFS_MAX_FILES 1024u
#define GFS_MAX_PAGES_PER_FILE (1u << 28)
#define GFS_MAX_FRAMES (1u << 24)
#define GFS_MAX_STREAMS 8u
#define GFS_MAX_WINDOW_PAGES 1024u   /* readahead cap, in pages */
#define GFS_MAX_RECENT 64u           /* detector: recent misses remembered per file (one per lane) */

/* Threads per block of the library's workload kernels. gread is inlined into its caller;
 * at 256 threads the compiler keeps the whole miss path in registers (about 220 VGPRs, no
 * scratch), where a 1024-thread bound would cap it at 128 and spill to scratch memory. */
#define GFS_MAX_BLOCK_THREADS 256u

/* open flags and fadvise advice */
#define GFS_O_RDONLY 0
#define GFS_ADV_NORMAL 0
#define GFS_ADV_SEQUENTIAL 2
#define GFS_ADV_RANDOM 1

/* host read backends */
#define GFS_IO_PREAD 0              /* any idle host thread takes the next request (ring order) */
#define GFS_IO_PREAD_PARTITIONED 1  /* GPUfs's queue (Sec. 3.3): a block posts into the slot of its
                                       block id (mod rpc_slots); host thread i serves only its own
                                       contiguous range of slots, one request at a time */
#define GFS_IO_URING 2              /* as GFS_IO_PREAD, but each host thread keeps io_depth reads in
                                       flight on its own io_uring (Sec. 4.1 has the host read the
                                       whole span; this overlaps its pieces on one thread) */

/* cache policies */
#define GFS_POLICY_SHARED 0    /* readahead windows into the shared page cache, global clock */
#define GFS_POLICY_PRIVATE 1   /* the paper's design (Sec. 4.1, Sec. 5.1): every threadblock
                                  prefetches into a private buffer and replaces pages in its own
                                  least-recently-allocated share of the frames */

/* o_direct modes */
#define GFS_DIRECT_OFF 0      /* buffered reads */
#define GFS_DIRECT_ON 1       /* O_DIRECT; gfs_open fails if the file system refuses it */
#define GFS_DIRECT_PREFER 2   /* O_DIRECT where the file system supports it, else buffered */

typedef struct gfs_config {
  uint32_t abi_version;          /* must be GFS_ABI_VERSION */
  uint32_t streams_per_file;     /* readahead streams tracked per file, 1..GFS_MAX_STREAMS */
  uint64_t page_size;            /* bytes; power of two, 4 KiB .. 2 MiB */
  uint64_t cache_bytes;          /* bytes of frames; a multiple of page_size, >= 64 pages */
  uint64_t ra_init_bytes;        /* first window of a stream at offset 0 or SEQUENTIAL advice */
  uint64_t ra_cap_bytes;         /* largest window; 0 switches readahead off (demand paging) */
  uint32_t host_threads;         /* host I/O threads polling the request ring, 1..64 */
  uint32_t rpc_slots;            /* request ring slots (each has its own staging buffer), 1..4096 */
  uint32_t io_backend;           /* GFS_IO_PREAD or GFS_IO_PREAD_PARTITIONED */
  uint32_t o_direct;             /* GFS_DIRECT_* */
  uint32_t trace_level;          /* 0 off, 1 policy events, 2 also hits/joins */
  uint32_t trace_capacity;       /* events kept in the device trace ring (32 B each) */
  uint64_t wait_timeout_ns;      /* device waits give up with -ETIMEDOUT after this long; 0 = 10 s */
  uint32_t policy;               /* GFS_POLICY_* */
  uint32_t private_slots;        /* GFS_POLICY_PRIVATE: per-block slots (private buffer + frame
                                    share), at least the blocks resident at once; 1..65536 */
  uint32_t io_chunk_bytes;       /* a host request is read in pieces of this size, each by
                                    whichever host thread is free (so one request keeps several
                                    reads in flight); with GFS_IO_PREAD, a request that would
                                    make fewer pieces than there are idle threads is cut into
                                    equal shares for them instead, none below 256 KiB; a
                                    multiple of 4 KiB, 64 KiB .. 64 MiB; each host thread holds
                                    one bounce buffer of this size for O_DIRECT reads */
  uint32_t max_files;            /* files registered at once (ids 0..max_files-1), 1..GFS_MAX_FILES;
                                    sizes the per-file metadata (about 34 KiB per file) */
  /* Readahead detector (Sec. 2.3: Linux also follows several readers that interleave on one
     file, by heuristics the paper does not spell out; these are the constants of this library's
     aggregate-reading rule). A
     miss at page p whose file has at least ra_near_min of its last ra_recent misses within
     ra_near_pages pages of p opens the window as the aligned chunk around p. */
  uint32_t ra_recent;            /* misses remembered per file, 1..GFS_MAX_RECENT */
  uint32_t ra_near_pages;        /* "near" radius in pages, 0..2^20 */
  uint32_t ra_near_min;          /* near misses that make the file read in aggregate, 1..ra_recent+1
                                    (ra_recent + 1 switches the rule off) */
  /* Thrash guard (Sec. 5.1: each resident threadblock's share of the cache is cache / resident
     threadblocks): a window is at most cache_pages / R pages, R = min(blocks in the launch,
     ra_quota_blocks). 0 = the device's resident blocks of 256-thread reader kernels (found at
     gfs_init); 1 = no guard (R = 1). */
  uint32_t ra_quota_blocks;
  uint32_t ra_async;             /* 0 = synchronous prefetch (the paper's choice, Sec. 4
                                    "Asynchronous operation": a missing block waits for its whole
                                    window); 1 = asynchronous, marker-triggered (Linux's way,
                                    Sec. 2.3): the page after a demand miss, and the first page of
                                    each asynchronous window, is its stream's marker; the first
                                    block to reach it issues the stream's next window and does not
                                    wait for it. Such windows use a quarter of the ring slots
                                    (at least one) of their own and are skipped while all of
                                    those are held. Shared policy only, rpc_slots >= 2 (-EINVAL
                                    otherwise). A block
                                    keeps at most one such window outstanding and pulls it in at
                                    gclose at the latest, so kernels must gclose before they end
                                    or gopen again. */
  uint32_t io_depth;             /* GFS_IO_URING: reads each host thread keeps in flight, 1..256
                                    (each holds an io_chunk_bytes bounce buffer for O_DIRECT) */
  uint32_t page_timers;          /* 1: gread times every page it serves, split into acquire,
                                    copy-out and unpin (t_acquire_ns, t_copy_ns, t_unpin_ns in
                                    gfs_stats); 0 (default): those stay 0, and an all-hit read
                                    saves the clock reads (~3 % of its time) */
} gfs_config;

/* Fill *cfg with defaults: 64 KiB pages (the best GPUfs page size for sequential reads,
 * Sec. 3.1), 256 MiB cache, readahead 4 pages (the 16 KB first fetch of Sec. 3.2's example,
 * at 4 KB pages) growing by doubling to 16 MiB (Linux's window growth, Sec. 2.3), 8 streams
 * per file (Sec. 2.3: several streams per descriptor), 8 host threads, 64 slots, 2 MiB host
 * read pieces, O_DIRECT preferred, trace off, shared policy (512 private slots if the
 * private policy is chosen), 64 files, detector constants 64/64/3, the device's resident
 * blocks for the thrash guard, synchronous prefetch (Sec. 4).
 *
 * GFS_POLICY_PRIVATE: a miss that the block's private buffer cannot serve asks the host for
 * the page plus ra_cap_bytes that follow it (PREFETCH_SIZE, static); the page goes into the
 * cache, the rest into the block's private buffer; a later miss of the same block on a page
 * held there is filled from it without a host request. Frames are split evenly among
 * private_slots; a block (one slot, taken at gopen, given back at gclose) reuses its own
 * frames in allocation order. The frames allocation then also holds the private buffers:
 * private_slots * ra_cap_bytes more bytes (gfs_device_bytes reports the total). */
void gfs_config_default(gfs_config* cfg);

typedef struct gfs_ctx gfs_ctx;
struct gfs_dev;

/* Device memory the caller must provide for a configuration (Sec. 2.2: the page cache lives in
 * GPU memory; Sec. 5.1: its frames are reused in place): the frame pool
 * (cache_bytes, plus the private buffers under GFS_POLICY_PRIVATE; 256-byte aligned) and
 * the metadata region (page table, frame words,
 * tags, per-file state, counters, trace ring). -EINVAL if the configuration is invalid. */
int gfs_device_bytes(const gfs_config* cfg, size_t* frames_bytes, size_t* meta_bytes);

/* Create a cache (Sec. 2.2: the GPU page cache, the shared CPU-GPU request queue, and the
 * host threads that poll it and read files for the GPU). frames_dev and meta_dev are device
 * pointers (e.g. from PyTorch) of at
 * least the sizes gfs_device_bytes reports; they stay owned by the caller and must
 * outlive the context. hip_stream is the hipStream_t the library uses for its own
 * set-up work (may be NULL for the null stream). The call initialises the metadata,
 * allocates the pinned request ring and staging buffers, and starts the host I/O
 * threads. Errors: -EINVAL (bad config/pointers), -ENOMEM (pinned memory), -EIO (HIP). */
int gfs_init(const gfs_config* cfg, void* frames_dev, void* meta_dev, void* hip_stream,
             gfs_ctx** out);

/* Register a file for device reads (the host half of Sec. 2.2's open). flags must be
 * GFS_O_RDONLY (Sec. 4, page cache coherency: prefetching is enabled only for read-only
 * files; there is no write path): anything else gives
 * -EROFS. The path is copied. *file_id receives the id that gopen resolves the same
 * path to, and that the workload launchers take. Must not run concurrently with
 * kernels using the context. Errors: -ENFILE (table full), -errno from open/fstat,
 * -EFBIG (more pages than the encoding holds). */
int gfs_open(gfs_ctx* ctx, const char* path, int flags, int* file_id);

/* Readahead hint for a registered file (Sec. 4.1: for files not read in order the paper lets
 * the user switch its prefetcher off with a posix_fadvise-style hint):
 * GFS_ADV_RANDOM switches readahead off for it, GFS_ADV_SEQUENTIAL opens every new
 * stream with the initial window, GFS_ADV_NORMAL restores the default. */
int gfs_fadvise(gfs_ctx* ctx, int file_id, int advice);

/* Unregister a file (the host half of Sec. 2.2's close). Every cached page, reservation and
 * readahead stream of the file is dropped and its frames become free, because a later
 * gfs_open may hand the same id to another file. Must not run concurrently with kernels
 * using the context. -EBADF if file_id is not registered, -EBUSY if a kernel still holds it
 * open (gopen without gclose; the file stays registered), -EIO on a HIP error. */
int gfs_close(gfs_ctx* ctx, int file_id);

/* Device pointer to the cache handle; pass it to kernels that call gopen/gread/gclose (Sec.
 * 2.2: GPU threadblocks call the file API). NULL if ctx is NULL; valid until gfs_shutdown. */
const struct gfs_dev* gfs_device_handle(gfs_ctx* ctx);

typedef struct gfs_stats {
  /* device counters */
  uint64_t hits;              /* page lookups served from a valid frame */
  uint64_t joins;             /* page lookups that waited for a frame being filled */
  uint64_t misses;            /* page lookups that issued a host request */
  uint64_t ra_pages;          /* pages fetched ahead of demand */
  uint64_t fetched_pages;     /* pages filled from the host (demand + readahead) */
  uint64_t evictions;         /* frames reused for another page */
  uint64_t wasted_pages;      /* prefetched pages evicted before any demand access */
  uint64_t hand_visits;       /* clock hand steps */
  uint64_t requests;          /* host requests posted */
  uint64_t request_bytes;     /* bytes asked of the host (span of each request) */
  uint64_t delivered_bytes;   /* bytes gread copied to user buffers */
  uint64_t retries;           /* lookups retried after a lost race */
  uint64_t noframe;           /* allocations that found every frame pinned or filling */
  uint64_t timeouts;          /* device waits that gave up */
  uint64_t io_errors;         /* host reads that failed or came back short */
  uint64_t trace_events;      /* events recorded (including dropped ones) */
  /* host counters */
  uint64_t host_requests;     /* requests served by the host threads */
  uint64_t host_bytes;        /* bytes the host read from files */
  uint64_t host_read_ns;      /* summed time inside pread */
  /* device time by phase of the miss path, summed over blocks (ns) */
  uint64_t t_lock_ns;         /* waiting for a file's miss lock */
  uint64_t t_crit_ns;         /* holding it (readahead decision, run, reservations) */
  uint64_t t_alloc_ns;        /* clock allocation and table updates */
  uint64_t t_slot_ns;         /* waiting for a free ring slot */
  uint64_t t_host_ns;         /* waiting for the host read */
  uint64_t t_pull_ns;         /* pulling staging into frames and publishing them */
  uint64_t t_join_ns;         /* waiting on frames other blocks are filling */
  uint64_t t_decide_ns;       /* part of t_crit: the readahead decision */
  uint64_t t_run_ns;          /* finding and reserving the run (after the unlock, under a claim) */
  uint64_t t_unlock_ns;       /* part of t_crit: releasing the miss lock */
  uint64_t lock_acquired;     /* miss locks taken */
  uint64_t lock_left;         /* lock waits given up because another block's window covered the page */
  /* time of every page gread serves, summed over blocks (ns) */
  uint64_t t_acquire_ns;      /* finding and pinning it: hit, join or miss, pulls included */
  uint64_t t_copy_ns;         /* copying it to the caller's buffer */
  uint64_t t_unpin_ns;        /* dropping the pin */
  /* GFS_POLICY_PRIVATE */
  uint64_t private_hits;      /* misses filled from the block's private buffer */
  uint64_t private_wasted;    /* private-buffer pages dropped without being used */
  uint64_t host_errors;       /* host reads that returned an error */
  uint64_t host_last_errno;   /* errno of the last failed host read (0 if none) */
  uint64_t host_spins[64];    /* per host thread: polls of the ring before its first request */
  uint32_t host_threads;
  uint32_t direct_io;         /* 1 if the last gfs_open used O_DIRECT */
  uint64_t host_thread_requests[64];   /* per host thread: requests it started serving */
  uint64_t ra_async_windows;  /* asynchronous readahead: windows issued at a marker page */
} gfs_stats;

/* Snapshot the counters (the quantities Sec. 3 and Sec. 6 measure: hits and misses of the GPU
 * page cache, prefetched and wasted pages, host requests and bytes, each host thread's polls
 * before its first request as in Sec. 3.3). Call when no kernel using the context is
 * running; -EINVAL on NULL arguments, -EIO on a HIP error. */
int gfs_stats_read(gfs_ctx* ctx, gfs_stats* out);

/* Trace record (32 bytes), written by device code when trace_level > 0. */
typedef struct gfs_event {
  uint32_t op;      /* GFS_EV_* */
  uint32_t block;   /* flattened blockIdx of the caller */
  uint32_t file;
  uint32_t page;
  uint32_t frame;   /* 0xffffffff when not applicable */
  uint32_t a;       /* op-specific: window length, hand action, ra bit, ... */
  uint64_t b;       /* op-specific: window start, hand ticket, request ticket, ... */
} gfs_event;

enum {
  GFS_EV_HIT = 1,    /* file,page,frame                                         */
  GFS_EV_JOIN = 2,   /* file,page,frame                                         */
  GFS_EV_MISS = 3,   /* file,page; a = window length (EOF-clamped), b = window start |
                        req << 32, req = pages of the read from page on (readahead on);
                        frame = near | h << 8 | rule << 24: the detector's inputs and choice --
                        near = the file's recent misses near page, h = cached pages right
                        behind page (counted only when no stream zone or the aggregate rule
                        applies), rule = GFS_RA_RULE_* */
  GFS_EV_HAND = 4,   /* frame; b = ticket; file,page = victim (EVICT); a = action | x << 8,
                        x = victim prefetched (EVICT) | ref bit seen << 1 | pinned << 2 |
                        lost a compare-and-swap << 3 | frame state seen << 4 */
  GFS_EV_ALLOC = 5,  /* file,page,frame; a = ra (1 if prefetched), b = hand ticket */
  GFS_EV_REQ = 6,    /* file, page = first page, a = pages in span, b = ring ticket */
  GFS_EV_NOFRAME = 7, /* file,page: window cut short, no frame left             */
  GFS_EV_PBHIT = 8,   /* private policy: file,page,frame filled from the private buffer */
  GFS_EV_ADV = 9      /* asynchronous readahead: file, page = the marker page whose access
                         advanced a stream; a = window length (EOF-clamped), b = window start */
};
/* readahead rules (GFS_EV_MISS): off (readahead off or RANDOM advice), a stream's zone,
   aggregate reading, context (cached history behind the page), a new stream (W0 or 1) */
enum { GFS_RA_RULE_OFF = 0, GFS_RA_RULE_ZONE = 1, GFS_RA_RULE_AGGREGATE = 2, GFS_RA_RULE_CONTEXT = 3,
       GFS_RA_RULE_NEW = 4 };
enum { GFS_HAND_FREE = 0, GFS_HAND_SKIP = 1, GFS_HAND_CLEAR = 2, GFS_HAND_EVICT = 3 };

/* Copy up to cap_bytes of recorded events (in record order) to host memory dst; *n_bytes
 * receives the bytes copied (whole records). The trace is the GPU I/O trace that Sec. 3.3
 * records and replays on the CPU; here it carries the policy's decisions for the CPU model
 * to replay. Call when no kernel using the context runs. -EINVAL, -EIO. */
int gfs_trace_read(gfs_ctx* ctx, void* dst, size_t cap_bytes, size_t* n_bytes);

/* Drop every cached page, readahead stream, counter and trace record (cold start: Sec. 6
 * flushes the page cache before every run; file reads then use O_DIRECT or come after
 * POSIX_FADV_DONTNEED). Registered files stay registered. Call when no kernel using the
 * context runs. -EINVAL, -EIO. */
int gfs_reset_cache(gfs_ctx* ctx);

/* Stop the host threads (Sec. 2.2), free the ring and staging, close files, free the
 * context. Kernels using the handle must have completed. -EINVAL if ctx is NULL. */
int gfs_shutdown(gfs_ctx* ctx);

/* ---- workload launchers (the benchmark consumers of gread; not part of the method) ----
 *
 * The workloads follow the paper's microbenchmark (Sec. 6.1): threadblocks each read their
 * share of a file in fixed-size strides, in order.
 *
 * gfs_launch_list_reader: one kernel of `blocks` threadblocks x `threads` threads
 * (a multiple of 64, <= GFS_MAX_BLOCK_THREADS). Block b calls gread(file, offsets[b*reads + k],
 * read_size, buf + b*read_size) for k = 0..reads-1 in order and folds every delivered
 * buffer into its consumer output:
 *   consumer 0 (checksum): out is uint64[blocks]; wrapping sum of the delivered
 *     little-endian uint32 words, a trailing partial word zero-padded;
 *   consumer 1 (histogram): out is uint32[blocks*256]; count of each byte value;
 *   consumer 2 (none): the reads only; out is not touched (may be NULL), and buf + b*read_size
 *     holds what block b's last read delivered.
 * status (int64[blocks]) receives the total bytes delivered to the block, or the first
 * negative errno gread returned. turn, if not NULL, serialises the reads: read k of
 * block b waits until *turn == k*blocks + b and then increments it (test-only; every
 * block must be resident at once: -EINVAL if `blocks` exceeds what the device holds).
 * All pointers are device pointers; the kernel is
 * enqueued on hip_stream and the call returns without waiting. -EINVAL on bad shapes. */
int gfs_launch_list_reader(gfs_ctx* ctx, int file_id, const uint64_t* offsets, uint32_t blocks,
                           uint32_t reads, uint64_t read_size, uint32_t threads, int consumer,
                           void* buf, void* out, int64_t* status, uint64_t* turn,
                           void* hip_stream);

/* gfs_launch_buffer_reader: the list reader's reads and consumers taken straight from a copy
 * of the file in device memory (data_dev, data_size bytes) instead of through gread; reads at
 * or past data_size deliver nothing, reads crossing it are cut short, exactly like gread at
 * the end of a file. This is the GPU half of the paper's CPU-I/O baseline (Sec. 6: the CPU
 * reads the file and copies it to the GPU, then the kernel runs). Arguments as for
 * gfs_launch_list_reader (offsets need no alignment; consumers 0 and 1 only); no context.
 * -EINVAL on bad shapes. */
int gfs_launch_buffer_reader(const void* data_dev, uint64_t data_size, const uint64_t* offsets, uint32_t blocks,
                             uint32_t reads, uint64_t read_size, uint32_t threads, int consumer, void* out,
                             int64_t* status, void* hip_stream);

/* ---- batched persistent launch (many files, one kernel) ----
 *
 * A unit is one gread of one file: bytes [offset, offset+size) of file `file`, folded into
 * output row `out` (per-file checksum and histogram). */
typedef struct gfs_unit {
  uint32_t file;      /* registered file id */
  uint32_t out;       /* output row */
  uint64_t offset;
  uint64_t size;
} gfs_unit;           /* 24 B */

/* Plan the unit order of a batch (host only, no GPU; a launch shape of this library, which
 * the paper, launching one kernel per application, does not have): files in the given order are cut
 * into units of at most unit_bytes; `grid / blocks_per_file` files are read at a time,
 * their units interleaved round-robin, and a finished file's place is taken by the next
 * one, so that a grid pulling units in order has about blocks_per_file blocks on each
 * file. sizes: host array of nfiles file sizes; ids: host array of the registered file ids
 * (out row i belongs to sizes[i]); out: host array of cap units; *nout receives the count.
 * -EINVAL on bad arguments, -ENOSPC if cap is too small (*nout then holds the count needed). */
int gfs_batch_plan(const uint64_t* sizes, const uint32_t* ids, uint32_t nfiles, uint64_t unit_bytes,
                   uint32_t grid, uint32_t blocks_per_file, gfs_unit* out, uint64_t cap,
                   uint64_t* nout);

/* gfs_launch_batch (every unit is one block-level gread, Sec. 2.2; the persistent launch over
 * many files is this library's own shape): one persistent kernel of `grid` blocks x `threads`
 * threads (a multiple
 * of 64, <= GFS_MAX_BLOCK_THREADS); blocks take units from units[0..nunits) in order through the device
 * counter *counter (reset by the call), gread each into their own buf + b*unit_bytes, and
 * fold the bytes into csum[out] (wrapping u64 sum of LE u32 words) and hist[out*256 + v]
 * (u32 byte counts) with atomics. status (int64[grid]) receives the bytes each block read
 * or the first negative errno. All pointers are device pointers; csum and hist must be
 * zeroed by the caller; enqueued on hip_stream without waiting. -EINVAL on bad shapes. */
int gfs_launch_batch(gfs_ctx* ctx, const gfs_unit* units, uint64_t nunits, uint32_t grid,
                     uint32_t threads, uint64_t unit_bytes, void* buf, uint64_t* counter,
                     uint64_t* csum, uint32_t* hist, int64_t* status, void* hip_stream);

/* Blocks of `threads` threads that fit on the device at once for the batch kernel (the grid
 * a persistent launch should use; Sec. 3.3 shows why the resident count matters: blocks not
 * yet resident leave their host threads idle); -EINVAL on a bad thread count, -EIO on a HIP
 * error. */
int gfs_batch_grid(uint32_t threads, uint32_t* grid);

/* Size in bytes of a registered file (host only; the size gread clamps to, Sec. 2.2's POSIX
 * read semantics). -EBADF if file_id is not registered, -EINVAL if size is NULL. */
int gfs_file_size(gfs_ctx* ctx, int file_id, uint64_t* size);

/* The configuration the context was created with (host only), with ra_quota_blocks resolved
 * to the count in use when it was 0 (the resident blocks of Sec. 5.1's quota). -EINVAL on
 * NULL arguments. */
int gfs_get_config(gfs_ctx* ctx, gfs_config* out);

/* ---- serving loop (a stream of whole-file read requests, one persistent kernel) ----
 *
 * The paper has no serving loop; this one is built from its parts: every request is a
 * stream of block-level greads (Sec. 2.2), admission keeps the bytes of unfinished requests
 * within the cache (Sec. 5: files larger than the cache stream through frames reused in
 * place), and the readahead detector serves each request's sequential stream (Sec. 4).
 *
 * Every request reads one registered file from start to end through gread, in chunks of
 * chunk_bytes, and yields the wrapping u64 sum of the file's little-endian u32 words (a
 * trailing partial word zero-padded). Requests arrive at given times; the host admits them
 * in arrival order while the cache bytes reserved by admitted, unfinished requests (file
 * size rounded up to whole pages) plus the next request's stay within budget_bytes (a
 * request is always admitted when nothing else is in flight). One persistent kernel of
 * `grid` blocks serves every admitted request: blocks take (request, chunk) units, oldest
 * request first, and newly admitted requests join between chunks. */
typedef struct gfs_serve_request {
  uint32_t file_id;       /* registered file */
  uint32_t pad;
  uint64_t arrival_ns;    /* arrival time after the start of the run; non-decreasing */
} gfs_serve_request;      /* 16 B */

typedef struct gfs_serve_params {
  uint64_t budget_bytes;     /* cache bytes admitted requests may reserve (> 0) */
  uint64_t chunk_bytes;      /* bytes per gread, a multiple of 16, <= 64 MiB */
  uint32_t grid;             /* persistent blocks (0: as many as fit on the device) */
  uint32_t threads;          /* threads per block, a multiple of 64, <= GFS_MAX_BLOCK_THREADS */
  uint64_t idle_timeout_ns;  /* the kernel gives up when the host is silent this long (0: 60 s) */
} gfs_serve_params;

typedef struct gfs_serve_record {
  uint64_t csum;          /* checksum of the file's bytes */
  int64_t result;         /* bytes delivered, or -errno of the first failed gread */
  uint64_t arrival_ns;    /* times after the start of the run, host clock */
  uint64_t admit_ns;      /* the host handed the request to the kernel */
  uint64_t first_ns;      /* the file's first page delivered (device clock mapped to the host's;
                             0 if that read failed) */
  uint64_t done_ns;       /* the host saw the request complete */
  uint64_t seq;           /* admission order */
  uint64_t reserved;      /* cache bytes reserved for it */
} gfs_serve_record;       /* 64 B */

typedef struct gfs_serve_summary {
  uint64_t span_ns;          /* start of the run to the last completion */
  uint64_t delivered_bytes;  /* summed over requests */
  uint64_t peak_reserved;    /* largest reservation total reached */
  uint32_t peak_pending;     /* longest admission queue */
  uint32_t grid;             /* blocks the kernel ran with */
  uint64_t clock_skew_ns;    /* uncertainty of the device-to-host clock mapping */
} gfs_serve_summary;

/* Run a whole request stream and return when every request has completed (blocking).
 * reqs: host array of n requests (1 <= n <= 2^20); out: host array of n records, in the
 * order of reqs; summary may be NULL. Times are replayed on the host clock from the moment
 * the kernel is seen running. The call allocates its own device and pinned buffers and frees
 * them before returning; the kernel runs on hip_stream, which must not carry other work that
 * waits on it. Errors: -EINVAL (bad arguments), -EBADF (a file not registered), -ENOMEM,
 * -EIO (HIP error), -ETIMEDOUT (the kernel stopped serving); per-request failures are
 * reported in out[i].result with the call returning 0. */
int gfs_serve_run(gfs_ctx* ctx, const gfs_serve_request* reqs, uint32_t n, const gfs_serve_params* params,
                  gfs_serve_record* out, gfs_serve_summary* summary, void* hip_stream);

/* ---- the serving loop without allocation ----
 *
 * For callers that cannot allocate memory during a run (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same run as gfs_serve_run, with the
 * same arguments, results and errors, but the call allocates nothing. Its device state
 * (request table, control words, block status, one chunk buffer per block) lives in a
 * fixed array of GFS_SERVE_NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds
 * until the process ends; its pinned mailbox (submissions and completion records for up to
 * GFS_SERVE_NOALLOC_MAX_REQUESTS requests) and host bookkeeping are allocated once, by
 * gfs_init. The scratch array is shared by every call on that GPU and the mailbox by every
 * call on that context: calls that overlap on one GPU race and must not be made. Each call
 * clears what it needs zeroed. The context's device must be current (-EINVAL otherwise).
 * -E2BIG if n exceeds GFS_SERVE_NOALLOC_MAX_REQUESTS, or if the run's device state,
 * 64 B per request + 1 KiB + 8 B per block + chunk_bytes per block (each part rounded up to
 * 256 B), exceeds GFS_SERVE_NOALLOC_SCRATCH_BYTES (e.g. 512 blocks fit chunks up to 120 KiB). */
#define GFS_SERVE_NOALLOC_MAX_REQUESTS 16384u
#define GFS_SERVE_NOALLOC_SCRATCH_BYTES (64ull << 20)
int gfs_serve_run_noalloc(gfs_ctx* ctx, const gfs_serve_request* reqs, uint32_t n,
                          const gfs_serve_params* params, gfs_serve_record* out, gfs_serve_summary* summary,
                          void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* GFS_H */
