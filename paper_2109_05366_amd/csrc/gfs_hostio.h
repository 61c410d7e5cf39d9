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
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
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
  uint64_t io_chunk_bytes = 0;      /* piece size, a multiple of kDirectAlign */
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

// Read one chunk of a request into the slot's staging; the thread that finishes a
// request's last chunk publishes its result to the device.
inline void run_chunk(HostIo* c, const Chunk& ch, uint8_t* bounce) {
  gfs_rpc_slot* rs = &c->ring[ch.slot];
  Track& tr = c->track[ch.slot];
  const uint32_t fid = rs->file_id;
  HostFile* hf = fid < GFS_MAX_FILES ? &c->files[fid] : nullptr;
  const int fd = hf ? hf->fd.load(std::memory_order_acquire) : -1;
  int64_t r;
  if (fd < 0) {
    r = -EBADF;
  } else {
    const uint64_t t0 = now_ns();
    r = read_span(fd, hf->direct, c->staging + (uint64_t)ch.slot * c->max_req_bytes + ch.dst,
                  ch.off, ch.len, bounce, c->io_chunk_bytes);
    c->host_read_ns.fetch_add(now_ns() - t0, std::memory_order_relaxed);
  }
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
inline void io_thread(HostIo* c, int idx) {
  const uint32_t NS = c->rpc_slots;
  bool first = true;
  uint64_t spins = 0;
  uint32_t pos = (uint32_t)((uint64_t)idx * NS / c->host_threads);
  const uint64_t chunk = c->io_chunk_bytes;
  uint8_t* bounce = (uint8_t*)aligned_alloc(kDirectAlign, chunk);
  if (!bounce) return;
  Chunk ch;
  while (!c->stop.load(std::memory_order_relaxed)) {
    if (pop_chunk(c, &ch)) {
      run_chunk(c, ch, bounce);
      continue;
    }
    int32_t got = -1;
    uint64_t gen = 0;
    for (uint32_t k = 0; k < NS && got < 0; ++k) {
      const uint32_t s = pos + k < NS ? pos + k : pos + k - NS;
      const uint64_t g = __atomic_load_n(&c->ring[s].req_seq, __ATOMIC_ACQUIRE);
      uint64_t prev = g - 1;
      if (g != 0 && c->claimed[s].load(std::memory_order_relaxed) == prev &&
          c->claimed[s].compare_exchange_strong(prev, g, std::memory_order_acq_rel)) {
        got = (int32_t)s;
        gen = g;
      }
    }
    if (got < 0) {
      ++spins;
      if (spins < (1u << 20)) cpu_relax();
      else usleep(50);   // long idle: stop burning the core, at some wake-up latency
      continue;
    }
    const uint32_t s = (uint32_t)got;
    pos = s + 1 < NS ? s + 1 : 0;
    if (first) {
      c->spins[idx].store(spins, std::memory_order_relaxed);
      first = false;
    }
    c->thread_requests[idx].fetch_add(1, std::memory_order_relaxed);
    gfs_rpc_slot* rs = &c->ring[s];
    rs->t_claim_ns = now_ns();
    const uint64_t off = rs->offset, len = rs->length;
    const uint64_t n = len > c->max_req_bytes ? 0 : (len + chunk - 1) / chunk;
    Track& tr = c->track[s];
    tr.total.store(0, std::memory_order_relaxed);
    tr.err.store(n == 0 && len ? -EINVAL : 0, std::memory_order_relaxed);
    tr.remaining.store(n ? (uint32_t)n : 1u, std::memory_order_release);
    if (n > 1) {
      std::lock_guard<std::mutex> g(c->qmu);
      for (uint64_t i = 1; i < n; ++i) {
        const uint64_t o = i * chunk;
        c->queue.push_back({s, gen, off + o, (len - o) < chunk ? (len - o) : chunk, o});
      }
      c->queued.fetch_add((uint32_t)(n - 1), std::memory_order_relaxed);
    }
    run_chunk(c, {s, gen, off, n ? (len < chunk ? len : chunk) : 0, 0}, bounce);
  }
  free(bounce);
}

inline void start_threads(HostIo* c) {
  c->stop.store(false);
  for (uint32_t i = 0; i < c->rpc_slots; ++i) c->claimed[i].store(0);
  for (uint32_t i = 0; i < c->host_threads; ++i)
    c->threads.emplace_back(c->io_backend == GFS_IO_PREAD_PARTITIONED ? io_thread_partitioned : io_thread, c,
                            (int)i);
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
