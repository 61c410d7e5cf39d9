// gfs_hostio.h -- the host half of the request ring: the I/O threads that serve the device's
// read requests (Sec. 2.2: host threads poll the shared CPU-GPU request queue and read the
// file for the GPU; Sec. 4.1: the host reads the whole requested span).
//
// Differences from the paper's host side, on purpose: any idle host thread takes any posted
// request (the paper's per-thread slot partition left threads idle, Sec. 3.3); one read
// covers a whole readahead span instead of one page per read, cut into pieces that any idle
// thread reads; the data goes straight into the slot's staging, which the GPU pulls from.
//
// Internal to the library. There is no HIP here: to this code the ring and the staging are
// host memory (pinned and device-mapped in the library, ordinary memory in the CPU tests that
// drive it from host threads standing in for GPU blocks).
#ifndef GFS_HOSTIO_H
#define GFS_HOSTIO_H

#include <errno.h>
#include <linux/io_uring.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <sys/mman.h>
#include <sys/syscall.h>
#include <time.h>
#include <unistd.h>

#include <atomic>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "gfs.h"
#include "gfs_layout.h"

namespace gfs_hostio {

constexpr uint64_t kDirectAlign = 4096;

inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }
inline uint64_t now_ns() {
  timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (uint64_t)t.tv_sec * 1000000000ull + (uint64_t)t.tv_nsec;
}

/* a registered file as the I/O threads see it */
struct HostFile {
  std::atomic<int> fd{-1};
  bool open = false;
  bool direct = false;
  uint64_t size = 0;
  std::string path;
};

/* a request larger than one piece is split; any I/O thread may read any piece */
struct Chunk {
  uint32_t slot;
  uint64_t gen;
  uint64_t off;       /* file offset */
  uint64_t len;
  uint64_t dst;       /* byte offset in the slot's staging */
};
struct Track {
  std::atomic<uint32_t> remaining{0};
  std::atomic<int64_t> total{0};
  std::atomic<int64_t> err{0};
};

/* The I/O engine of one context. Set the configuration and the ring, staging and file table
   pointers, call init(), then start_threads(); stop_threads() joins them. */
struct HostIo {
  uint32_t rpc_slots = 0;
  uint32_t host_threads = 0;        /* 1..64 */
  uint32_t io_backend = GFS_IO_PREAD;
  uint32_t io_depth = 1;            /* GFS_IO_URING: reads in flight per thread, 1..256 */
  uint64_t io_chunk_bytes = 0;      /* piece size, a multiple of kDirectAlign */
  uint64_t min_piece_bytes = 256 << 10;   /* GFS_IO_PREAD: the smallest piece a request is cut
                                             into when threads would otherwise sit idle (a
                                             multiple of kDirectAlign) */
  uint64_t max_req_bytes = 0;       /* staging bytes per slot */
  gfs_rpc_slot* ring = nullptr;     /* rpc_slots slots */
  uint8_t* staging = nullptr;       /* rpc_slots * max_req_bytes */
  HostFile* files = nullptr;        /* GFS_MAX_FILES entries */

  std::vector<std::thread> threads;
  std::unique_ptr<std::atomic<uint64_t>[]> claimed;   // per ring slot: last generation a thread took
  std::unique_ptr<Track[]> track;
  std::atomic<bool> stop{false};
  std::atomic<uint64_t> host_requests{0}, host_bytes{0}, host_read_ns{0}, host_errors{0};
  std::atomic<int64_t> host_last_errno{0};
  std::atomic<uint64_t> spins[64];
  std::atomic<uint64_t> thread_requests[64];
  std::mutex qmu;
  std::deque<Chunk> queue;
  std::atomic<uint32_t> queued{0};
  std::atomic<uint32_t> busy{0};    /* GFS_IO_PREAD threads reading a piece right now */
  std::atomic<uint64_t> host_pieces{0};   /* pieces read (a request is one or more) */

  /* per-slot state; -ENOMEM if it cannot be allocated */
  int init() {
    track.reset(new (std::nothrow) Track[rpc_slots]);
    claimed.reset(new (std::nothrow) std::atomic<uint64_t>[rpc_slots]);
    for (auto& x : spins) x.store(0);
    for (auto& x : thread_requests) x.store(0);
    return track && claimed ? 0 : -ENOMEM;
  }
  void clear_counters() {
    host_requests = 0;
    host_bytes = 0;
    host_read_ns = 0;
    host_errors = 0;
    host_last_errno = 0;
    for (auto& x : spins) x.store(0);
  }
};

// Read file bytes [off, off+len) into dst (pinned staging). Returns bytes read (short only
// at end of file) or -errno. Direct reads cannot target the GPU driver's pinned pages (the
// kernel refuses to pin them for DMA, EFAULT), so they go through the thread's aligned
// bounce buffer in chunks and are copied into staging; buffered reads go straight in.
inline int64_t read_span(int fd, bool direct, uint8_t* dst, uint64_t off, uint64_t len, uint8_t* bounce,
                  uint64_t chunk) {
  uint64_t done = 0;
  if (!direct) {
    while (done < len) {
      const ssize_t r = pread(fd, dst + done, len - done, (off_t)(off + done));
      if (r < 0) {
        if (errno == EINTR) continue;
        return -(int64_t)errno;
      }
      if (r == 0) break;
      done += (uint64_t)r;
    }
    return (int64_t)done;
  }
  while (done < len) {
    const uint64_t want = len - done < chunk ? align_up(len - done, kDirectAlign) : chunk;
    ssize_t r;
    do {
      r = pread(fd, bounce, want, (off_t)(off + done));
    } while (r < 0 && errno == EINTR);
    if (r < 0) return -(int64_t)errno;
    if (r == 0) break;
    uint64_t take = (uint64_t)r;
    if (take > len - done) take = len - done;
    memcpy(dst + done, bounce, take);
    done += take;
    if ((uint64_t)r < want) break;   // end of file
  }
  return (int64_t)done;
}

inline void cpu_relax() { __builtin_ia32_pause(); }

// Account one finished chunk (r = bytes read or -errno); the thread that finishes a request's
// last chunk publishes its result to the device.
inline void finish_chunk(HostIo* c, const Chunk& ch, int64_t r) {
  gfs_rpc_slot* rs = &c->ring[ch.slot];
  Track& tr = c->track[ch.slot];
  if (r < 0) {
    tr.err.store(r, std::memory_order_relaxed);
    c->host_errors.fetch_add(1, std::memory_order_relaxed);
    c->host_last_errno.store(-r, std::memory_order_relaxed);
  } else {
    tr.total.fetch_add(r, std::memory_order_relaxed);
    c->host_bytes.fetch_add((uint64_t)r, std::memory_order_relaxed);
  }
  if (tr.remaining.fetch_sub(1, std::memory_order_acq_rel) == 1) {
    const int64_t e = tr.err.load(std::memory_order_relaxed);
    rs->result = e ? e : tr.total.load(std::memory_order_relaxed);
    rs->t_done_ns = now_ns();
    __atomic_store_n(&rs->done_seq, ch.gen, __ATOMIC_RELEASE);
    c->host_requests.fetch_add(1, std::memory_order_relaxed);
  }
}

// The registered file a request names, or null (its descriptor in *fd, -1 if closed).
inline HostFile* request_file(HostIo* c, uint32_t slot, int* fd) {
  const uint32_t fid = c->ring[slot].file_id;
  HostFile* hf = fid < GFS_MAX_FILES ? &c->files[fid] : nullptr;
  *fd = hf ? hf->fd.load(std::memory_order_acquire) : -1;
  return hf;
}

// Read one chunk of a request into the slot's staging, then account it.
inline void run_chunk(HostIo* c, const Chunk& ch, uint8_t* bounce) {
  int fd;
  HostFile* hf = request_file(c, ch.slot, &fd);
  int64_t r;
  if (fd < 0) {
    r = -EBADF;
  } else {
    const uint64_t t0 = now_ns();
    r = read_span(fd, hf->direct, c->staging + (uint64_t)ch.slot * c->max_req_bytes + ch.dst,
                  ch.off, ch.len, bounce, c->io_chunk_bytes);
    c->host_read_ns.fetch_add(now_ns() - t0, std::memory_order_relaxed);
    c->host_pieces.fetch_add(1, std::memory_order_relaxed);
  }
  finish_chunk(c, ch, r);
}

inline bool pop_chunk(HostIo* c, Chunk* out) {
  if (c->queued.load(std::memory_order_relaxed) == 0) return false;
  std::lock_guard<std::mutex> g(c->qmu);
  if (c->queue.empty()) return false;
  *out = c->queue.front();
  c->queue.pop_front();
  c->queued.fetch_sub(1, std::memory_order_relaxed);
  return true;
}

// Partitioned queue (GPUfs's, Sec. 3.3): thread idx serves only the slots
// [idx*S/N, (idx+1)*S/N), in turn, each request whole by itself.
inline void io_thread_partitioned(HostIo* c, int idx) {
  const uint32_t NS = c->rpc_slots, N = c->host_threads;
  const uint32_t lo = (uint32_t)((uint64_t)idx * NS / N), hi = (uint32_t)((uint64_t)(idx + 1) * NS / N);
  std::vector<uint64_t> want(hi - lo, 1);   // next generation of each own slot
  bool first = true;
  uint64_t spins = 0;
  const uint64_t chunk = c->io_chunk_bytes;
  uint8_t* bounce = (uint8_t*)aligned_alloc(kDirectAlign, chunk);
  if (!bounce) return;
  while (!c->stop.load(std::memory_order_relaxed)) {
    bool served = false;
    for (uint32_t s = lo; s < hi; ++s) {
      gfs_rpc_slot* rs = &c->ring[s];
      const uint64_t gen = want[s - lo];
      if (__atomic_load_n(&rs->req_seq, __ATOMIC_ACQUIRE) != gen) continue;
      if (first) {
        c->spins[idx].store(spins, std::memory_order_relaxed);
        first = false;
      }
      c->thread_requests[idx].fetch_add(1, std::memory_order_relaxed);
      rs->t_claim_ns = now_ns();
      const uint64_t off = rs->offset, len = rs->length;
      const uint64_t n = len > c->max_req_bytes ? 0 : (len + chunk - 1) / chunk;
      Track& tr = c->track[s];
      tr.total.store(0, std::memory_order_relaxed);
      tr.err.store(n == 0 && len ? -EINVAL : 0, std::memory_order_relaxed);
      tr.remaining.store(n ? (uint32_t)n : 1u, std::memory_order_release);
      if (n == 0) {
        run_chunk(c, {s, gen, off, 0, 0}, bounce);
      } else {
        for (uint64_t i = 0; i < n; ++i) {
          const uint64_t o = i * chunk;
          run_chunk(c, {s, gen, off + o, (len - o) < chunk ? (len - o) : chunk, o}, bounce);
        }
      }
      want[s - lo] = gen + 1;
      served = true;
    }
    if (!served) {
      ++spins;
      if (spins < (1u << 20)) cpu_relax();
      else usleep(50);
    }
  }
  free(bounce);
}

// One host I/O thread: read queued chunks when there are any; otherwise look over the ring
// for a posted request that no thread has taken (starting after the slot it served last, so
// every slot is visited in turn), take it with a compare-and-swap on the slot's claimed
// generation, split it into chunks, queue all but the first, and read the first. Taking
// any posted request, rather than waiting on the next ticket in ring order, keeps a thread
// from idling behind a slot whose block has not posted yet.
// Look over the ring for a posted request no thread has taken (starting at *pos, so every slot
// is visited in turn) and take it with a compare-and-swap on the slot's claimed generation;
// split it into chunks, queue all but the first and return the first in *first_chunk.
// False if nothing is posted.
inline bool claim_request(HostIo* c, int idx, uint32_t* pos, Chunk* first_chunk) {
  const uint32_t NS = c->rpc_slots;
  const uint64_t chunk = c->io_chunk_bytes;
  int32_t got = -1;
  uint64_t gen = 0;
  for (uint32_t k = 0; k < NS && got < 0; ++k) {
    const uint32_t s = *pos + k < NS ? *pos + k : *pos + k - NS;
    const uint64_t g = __atomic_load_n(&c->ring[s].req_seq, __ATOMIC_ACQUIRE);
    uint64_t prev = g - 1;
    if (g != 0 && c->claimed[s].load(std::memory_order_relaxed) == prev &&
        c->claimed[s].compare_exchange_strong(prev, g, std::memory_order_acq_rel)) {
      got = (int32_t)s;
      gen = g;
    }
  }
  if (got < 0) return false;
  const uint32_t s = (uint32_t)got;
  *pos = s + 1 < NS ? s + 1 : 0;
  c->thread_requests[idx].fetch_add(1, std::memory_order_relaxed);
  gfs_rpc_slot* rs = &c->ring[s];
  rs->t_claim_ns = now_ns();
  const uint64_t off = rs->offset, len = rs->length;
  /* pieces of io_chunk_bytes; but when fewer pieces than idle threads (this one included)
     would result, smaller ones, down to min_piece_bytes, so that every idle thread reads a
     share: a storage device serves more reads in flight faster, and a readahead window is
     otherwise read by one thread while others wait for work */
  uint64_t piece = chunk;
  if (c->io_backend == GFS_IO_PREAD && len > c->min_piece_bytes) {
    const uint32_t nt = c->host_threads;
    const uint32_t taken = c->busy.load(std::memory_order_relaxed) + c->queued.load(std::memory_order_relaxed);
    const uint32_t idle = nt > taken ? nt - taken : 1u;
    if (idle > 1) {
      uint64_t share = (len + idle - 1) / idle;
      share = (share + c->min_piece_bytes - 1) / c->min_piece_bytes * c->min_piece_bytes;
      if (share < piece) piece = share;
    }
  }
  const uint64_t n = len > c->max_req_bytes ? 0 : (len + piece - 1) / piece;
  Track& tr = c->track[s];
  tr.total.store(0, std::memory_order_relaxed);
  tr.err.store(n == 0 && len ? -EINVAL : 0, std::memory_order_relaxed);
  tr.remaining.store(n ? (uint32_t)n : 1u, std::memory_order_release);
  if (n > 1) {
    std::lock_guard<std::mutex> g(c->qmu);
    for (uint64_t i = 1; i < n; ++i) {
      const uint64_t o = i * piece;
      c->queue.push_back({s, gen, off + o, (len - o) < piece ? (len - o) : piece, o});
    }
    c->queued.fetch_add((uint32_t)(n - 1), std::memory_order_relaxed);
  }
  *first_chunk = {s, gen, off, n ? (len < piece ? len : piece) : 0, 0};
  return true;
}

inline void idle_step(uint64_t& spins) {
  ++spins;
  if (spins < (1u << 20)) cpu_relax();
  else usleep(50);   // long idle: stop burning the core, at some wake-up latency
}

inline void io_thread(HostIo* c, int idx) {
  bool first = true;
  uint64_t spins = 0;
  uint32_t pos = (uint32_t)((uint64_t)idx * c->rpc_slots / c->host_threads);
  uint8_t* bounce = (uint8_t*)aligned_alloc(kDirectAlign, c->io_chunk_bytes);
  if (!bounce) return;
  Chunk ch;
  while (!c->stop.load(std::memory_order_relaxed)) {
    if (pop_chunk(c, &ch)) {
      c->busy.fetch_add(1, std::memory_order_relaxed);
      run_chunk(c, ch, bounce);
      c->busy.fetch_sub(1, std::memory_order_relaxed);
      continue;
    }
    if (!claim_request(c, idx, &pos, &ch)) {
      idle_step(spins);
      continue;
    }
    if (first) {
      c->spins[idx].store(spins, std::memory_order_relaxed);
      first = false;
    }
    c->busy.fetch_add(1, std::memory_order_relaxed);
    run_chunk(c, ch, bounce);
    c->busy.fetch_sub(1, std::memory_order_relaxed);
  }
  free(bounce);
}

// ---- io_uring backend: one submission ring per host thread, io_depth reads in flight ----
//
// The ring is driven through the raw system calls (io_uring_setup / io_uring_enter and the
// kernel's shared queues), with no helper library. A thread fills its free entries with
// chunks (queued pieces first, then newly claimed requests), submits them together, and
// reaps completions; a piece read short before the end of its file is submitted again for
// the rest. Direct reads land in the entry's aligned bounce buffer (the driver's pinned
// staging cannot take O_DIRECT DMA) and are copied into staging; buffered reads go straight
// into staging.
struct Uring {
  int fd = -1;
  void* sq_map = nullptr;
  void* cq_map = nullptr;
  size_t sq_len = 0, cq_len = 0, sqe_len = 0;
  io_uring_sqe* sqes = nullptr;
  uint32_t *sq_head = nullptr, *sq_tail = nullptr, *sq_mask = nullptr, *sq_array = nullptr;
  uint32_t *cq_head = nullptr, *cq_tail = nullptr, *cq_mask = nullptr;
  io_uring_cqe* cqes = nullptr;

  int setup(unsigned entries) {
    io_uring_params p;
    memset(&p, 0, sizeof p);
    fd = (int)syscall(__NR_io_uring_setup, entries, &p);
    if (fd < 0) return -errno;
    sq_len = p.sq_off.array + p.sq_entries * sizeof(uint32_t);
    cq_len = p.cq_off.cqes + p.cq_entries * sizeof(io_uring_cqe);
    const bool single = (p.features & IORING_FEAT_SINGLE_MMAP) != 0;
    if (single) sq_len = cq_len = sq_len > cq_len ? sq_len : cq_len;
    sq_map = mmap(nullptr, sq_len, PROT_READ | PROT_WRITE, MAP_SHARED | MAP_POPULATE, fd, IORING_OFF_SQ_RING);
    if (sq_map == MAP_FAILED) {
      sq_map = nullptr;
      return fail(-errno);
    }
    if (single) {
      cq_map = sq_map;
    } else {
      cq_map = mmap(nullptr, cq_len, PROT_READ | PROT_WRITE, MAP_SHARED | MAP_POPULATE, fd, IORING_OFF_CQ_RING);
      if (cq_map == MAP_FAILED) {
        cq_map = nullptr;
        return fail(-errno);
      }
    }
    sqe_len = p.sq_entries * sizeof(io_uring_sqe);
    void* sq = mmap(nullptr, sqe_len, PROT_READ | PROT_WRITE, MAP_SHARED | MAP_POPULATE, fd, IORING_OFF_SQES);
    if (sq == MAP_FAILED) return fail(-errno);
    sqes = (io_uring_sqe*)sq;
    uint8_t* s8 = (uint8_t*)sq_map;
    uint8_t* c8 = (uint8_t*)cq_map;
    sq_head = (uint32_t*)(s8 + p.sq_off.head);
    sq_tail = (uint32_t*)(s8 + p.sq_off.tail);
    sq_mask = (uint32_t*)(s8 + p.sq_off.ring_mask);
    sq_array = (uint32_t*)(s8 + p.sq_off.array);
    cq_head = (uint32_t*)(c8 + p.cq_off.head);
    cq_tail = (uint32_t*)(c8 + p.cq_off.tail);
    cq_mask = (uint32_t*)(c8 + p.cq_off.ring_mask);
    cqes = (io_uring_cqe*)(c8 + p.cq_off.cqes);
    return 0;
  }
  int fail(int e) {
    teardown();
    return e;
  }
  void teardown() {
    if (sqes) munmap(sqes, sqe_len);
    if (cq_map && cq_map != sq_map) munmap(cq_map, cq_len);
    if (sq_map) munmap(sq_map, sq_len);
    if (fd >= 0) close(fd);
    sqes = nullptr;
    sq_map = cq_map = nullptr;
    fd = -1;
  }
  /* queue one read (the caller keeps at most `entries` in flight, so the queue has room) */
  void push_read(int file, void* dst, uint32_t len, uint64_t off, uint64_t tag) {
    const uint32_t tail = *sq_tail;
    const uint32_t i = tail & *sq_mask;
    io_uring_sqe* e = &sqes[i];
    memset(e, 0, sizeof *e);
    e->opcode = IORING_OP_READ;
    e->fd = file;
    e->addr = (uint64_t)(uintptr_t)dst;
    e->len = len;
    e->off = off;
    e->user_data = tag;
    sq_array[i] = i;
    __atomic_store_n(sq_tail, tail + 1, __ATOMIC_RELEASE);
  }
  /* submit `n` queued reads; wait for at least `wait` completions */
  int enter(uint32_t n, uint32_t wait) {
    while (true) {
      const long r = syscall(__NR_io_uring_enter, fd, n, wait, wait ? IORING_ENTER_GETEVENTS : 0, nullptr, 0);
      if (r >= 0) return (int)r;
      if (errno != EINTR) return -errno;
    }
  }
  /* the next completion, if any: true and (tag, res) */
  bool pop(uint64_t* tag, int32_t* res) {
    const uint32_t head = *cq_head;
    if (head == __atomic_load_n(cq_tail, __ATOMIC_ACQUIRE)) return false;
    const io_uring_cqe* e = &cqes[head & *cq_mask];
    *tag = e->user_data;
    *res = e->res;
    __atomic_store_n(cq_head, head + 1, __ATOMIC_RELEASE);
    return true;
  }
};

/* 0 if this process may create an io_uring, else -errno (kernels can switch it off) */
inline int uring_available() {
  Uring u;
  const int rc = u.setup(1);
  if (rc == 0) u.teardown();
  return rc;
}

/* one read in flight on a thread's ring: which chunk, where it stands */
struct UringEntry {
  bool busy = false;
  Chunk ch{};
  uint64_t done = 0;      /* bytes of the chunk read so far */
  uint64_t t0 = 0;
  bool direct = false;
  uint64_t fsize = 0;
  uint8_t* bounce = nullptr;
};

inline bool uring_submit_entry(HostIo* c, Uring& u, UringEntry& e, uint32_t k, int fd) {
  const uint64_t rest = e.ch.len - e.done;
  uint8_t* stage = c->staging + (uint64_t)e.ch.slot * c->max_req_bytes + e.ch.dst + e.done;
  if (e.direct) {
    // whole aligned blocks from an aligned offset (every chunk starts aligned and a resubmit
    // follows a read of whole blocks); the bounce buffer holds one piece
    u.push_read(fd, e.bounce, (uint32_t)align_up(rest, kDirectAlign), e.ch.off + e.done, k);
  } else {
    u.push_read(fd, stage, (uint32_t)rest, e.ch.off + e.done, k);
  }
  return true;
}

inline void io_thread_uring(HostIo* c, int idx) {
  const uint32_t depth = c->io_depth < 1 ? 1 : c->io_depth;
  Uring u;
  if (u.setup(depth) != 0) {
    c->host_errors.fetch_add(1, std::memory_order_relaxed);
    c->host_last_errno.store(ENOSYS, std::memory_order_relaxed);
    return;
  }
  std::vector<UringEntry> ent(depth);
  bool ok = true;
  for (auto& e : ent) {
    e.bounce = (uint8_t*)aligned_alloc(kDirectAlign, c->io_chunk_bytes);
    ok = ok && e.bounce;
  }
  bool first = true;
  uint64_t spins = 0;
  uint32_t pos = (uint32_t)((uint64_t)idx * c->rpc_slots / c->host_threads);
  uint32_t inflight = 0;
  while (ok && !(c->stop.load(std::memory_order_relaxed) && inflight == 0)) {
    // fill free entries with work (none once asked to stop: drain what is in flight)
    uint32_t queued = 0;
    for (uint32_t k = 0; k < depth && !c->stop.load(std::memory_order_relaxed); ++k) {
      UringEntry& e = ent[k];
      if (e.busy) continue;
      Chunk ch;
      if (!pop_chunk(c, &ch)) {
        if (!claim_request(c, idx, &pos, &ch)) break;
        if (first) {
          c->spins[idx].store(spins, std::memory_order_relaxed);
          first = false;
        }
      }
      int fd;
      HostFile* hf = request_file(c, ch.slot, &fd);
      if (fd < 0 || ch.len == 0) {
        finish_chunk(c, ch, fd < 0 ? -EBADF : 0);
        --k;   // the entry is still free
        continue;
      }
      e.busy = true;
      e.ch = ch;
      e.done = 0;
      e.t0 = now_ns();
      e.direct = hf->direct;
      e.fsize = hf->size;
      uring_submit_entry(c, u, e, k, fd);
      ++queued;
      ++inflight;
    }
    if (inflight == 0) {
      idle_step(spins);
      continue;
    }
    // submit; wait for a completion only when nothing new could be started
    const int r = u.enter(queued, queued ? 0 : 1);
    if (r < 0) {
      // the ring itself failed: fail every read in flight and stop this thread
      for (uint32_t k = 0; k < depth; ++k)
        if (ent[k].busy) {
          ent[k].busy = false;
          finish_chunk(c, ent[k].ch, r);
        }
      inflight = 0;
      break;
    }
    uint64_t tag;
    int32_t res;
    while (u.pop(&tag, &res)) {
      if (tag >= depth || !ent[tag].busy) continue;
      UringEntry& e = ent[tag];
      if (res == -EINTR || res == -EAGAIN) {
        int fd;
        request_file(c, e.ch.slot, &fd);
        if (fd >= 0) {
          uring_submit_entry(c, u, e, (uint32_t)tag, fd);
          u.enter(1, 0);
          continue;
        }
        res = -EBADF;
      }
      int64_t out;
      bool again = false;
      if (res < 0) {
        out = res;
      } else {
        uint64_t take = (uint64_t)res;
        if (take > e.ch.len - e.done) take = e.ch.len - e.done;
        if (e.direct && take)
          memcpy(c->staging + (uint64_t)e.ch.slot * c->max_req_bytes + e.ch.dst + e.done, e.bounce, take);
        e.done += take;
        // short before the end of the piece and of the file: read the rest (whole blocks
        // only for direct reads, whose offset must stay aligned)
        const uint64_t at = e.ch.off + e.done;
        again = res > 0 && e.done < e.ch.len && at < e.fsize && (!e.direct || e.done % kDirectAlign == 0);
        out = (int64_t)e.done;
      }
      if (again) {
        int fd;
        request_file(c, e.ch.slot, &fd);
        if (fd >= 0) {
          uring_submit_entry(c, u, e, (uint32_t)tag, fd);
          u.enter(1, 0);
          continue;
        }
      }
      c->host_read_ns.fetch_add(now_ns() - e.t0, std::memory_order_relaxed);
      e.busy = false;
      --inflight;
      finish_chunk(c, e.ch, out);
    }
  }
  for (auto& e : ent) free(e.bounce);
  u.teardown();
}

inline void start_threads(HostIo* c) {
  c->stop.store(false);
  for (uint32_t i = 0; i < c->rpc_slots; ++i) c->claimed[i].store(0);
  for (uint32_t i = 0; i < c->host_threads; ++i)
    c->threads.emplace_back(c->io_backend == GFS_IO_PREAD_PARTITIONED ? io_thread_partitioned
                            : c->io_backend == GFS_IO_URING          ? io_thread_uring
                                                                     : io_thread,
                            c, (int)i);
}

inline void stop_threads(HostIo* c) {
  c->stop.store(true);
  for (auto& t : c->threads) t.join();
  c->threads.clear();
  std::lock_guard<std::mutex> g(c->qmu);
  c->queue.clear();
  c->queued.store(0);
}

}  // namespace gfs_hostio

#endif  // GFS_HOSTIO_H
