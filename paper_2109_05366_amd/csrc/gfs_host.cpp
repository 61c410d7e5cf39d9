// Host runtime of the GPU file page cache: context set-up, file registry, and the host
// I/O threads that serve the device's request ring (Sec. 2.2: host threads poll the shared
// CPU-GPU request queue and read the file for the GPU; Sec. 4.1: the host reads the whole
// requested span, and the GPU side places every page of it in the cache).
//
// Differences from the paper's host side, on purpose: any idle host thread takes any posted
// request (the paper's per-thread slot partition left threads idle, Sec. 3.3);
// one read covers a whole readahead span instead of one page per read; the data is read
// straight into pinned staging that the GPU pulls from, so the host issues no copy calls.
#include <errno.h>
#include <fcntl.h>
#include <sched.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
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

#include <hip/hip_runtime.h>

#include "gfs.h"
#include "gfs_layout.h"

extern "C" int gfs_internal_zero(void* p, size_t bytes, hipStream_t s);
extern "C" int gfs_internal_resident_blocks(uint32_t threads, uint32_t* blocks);
extern "C" int gfs_internal_purge_file(const gfs_dev* ddev, uint32_t nframes, uint64_t pt_entries, uint32_t file,
                                       hipStream_t s);

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint64_t kDirectAlign = 4096;

uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }
uint64_t now_ns() {
  timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (uint64_t)t.tv_sec * 1000000000ull + (uint64_t)t.tv_nsec;
}
bool pow2(uint64_t v) { return v && !(v & (v - 1)); }
uint32_t log2u(uint64_t v) {
  uint32_t s = 0;
  while ((1ull << s) < v) ++s;
  return s;
}

struct Layout {
  uint64_t nframes = 0, nbuckets = 0, ra_init = 0, ra_cap = 0, max_req_pages = 0;
  uint64_t max_req_bytes = 0;
  uint64_t quota = 0;              /* private policy: frames per slot */
  uint64_t pbuf_bytes = 0;         /* private policy: all private buffers */
  uint64_t off_globals = 0, off_dev = 0, off_files = 0, off_locks = 0, off_lockq = 0, off_claims = 0, off_pslots = 0, off_names = 0, off_fword = 0,
           off_ftag = 0, off_pt = 0, off_ffill = 0, off_slot_free = 0, off_slot_tail = 0, off_reqd = 0, off_trace = 0,
           meta_bytes = 0;
};

int make_layout(const gfs_config* c, Layout* L) {
  if (!c || c->abi_version != GFS_ABI_VERSION) return -EINVAL;
  const uint64_t P = c->page_size;
  if (!pow2(P) || P < 4096 || P > (2ull << 20)) return -EINVAL;
  if (c->cache_bytes == 0 || c->cache_bytes % P) return -EINVAL;
  L->nframes = c->cache_bytes / P;
  if (L->nframes < 64 || L->nframes > GFS_MAX_FRAMES - 1) return -EINVAL;
  if (c->streams_per_file < 1 || c->streams_per_file > GFS_MAX_STREAMS) return -EINVAL;
  if (c->ra_cap_bytes % P || c->ra_init_bytes % P) return -EINVAL;
  L->ra_cap = c->ra_cap_bytes / P;
  L->ra_init = c->ra_init_bytes / P;
  if (L->ra_cap > GFS_MAX_WINDOW_PAGES) return -EINVAL;
  if (L->ra_cap && (L->ra_init < 1 || L->ra_init > L->ra_cap)) return -EINVAL;
  if (c->host_threads < 1 || c->host_threads > 64) return -EINVAL;
  if (c->rpc_slots < 1 || c->rpc_slots > 4096) return -EINVAL;
  if (c->io_backend != GFS_IO_PREAD && c->io_backend != GFS_IO_PREAD_PARTITIONED) return -EINVAL;
  if (c->io_backend == GFS_IO_PREAD_PARTITIONED && c->host_threads > c->rpc_slots) return -EINVAL;
  if (c->o_direct > GFS_DIRECT_PREFER) return -EINVAL;
  if (c->trace_level > 2) return -EINVAL;
  if (c->io_chunk_bytes % kDirectAlign || c->io_chunk_bytes < (64u << 10) || c->io_chunk_bytes > (64u << 20))
    return -EINVAL;
  if (c->max_files < 1 || c->max_files > GFS_MAX_FILES) return -EINVAL;
  if (c->ra_recent < 1 || c->ra_recent > GFS_MAX_RECENT) return -EINVAL;
  if (c->ra_near_pages > (1u << 20) || c->ra_near_min < 1 || c->ra_near_min > c->ra_recent + 1) return -EINVAL;
  if (c->ra_async > 1) return -EINVAL;
  if (c->ra_async) return -ENOTSUP;   /* marker-triggered prefetch is not built (see gfs.h) */
  if (c->policy == GFS_POLICY_SHARED) {
    L->max_req_pages = L->ra_cap ? L->ra_cap : 1;
  } else if (c->policy == GFS_POLICY_PRIVATE) {
    // a request is the missed page plus the static prefetch that follows it
    if (c->private_slots < 1 || c->private_slots > 65536) return -EINVAL;
    L->quota = L->nframes / c->private_slots;
    if (L->quota < 1) return -EINVAL;
    L->max_req_pages = 1 + L->ra_cap;
    L->pbuf_bytes = (uint64_t)c->private_slots * L->ra_cap * P;
  } else {
    return -EINVAL;
  }
  L->max_req_bytes = L->max_req_pages * P;
  // page table: 4 entries per frame, plus room for the reservations of misses in flight
  // (a page is reserved before it gets a frame; with a small cache, blocks that miss at once
  // can hold more reservations than there are frames), 16-entry buckets, power-of-two count
  uint64_t nb = 2;
  while (nb * GFS_BUCKET_SLOTS < 4 * L->nframes + 2 * GFS_LOCK_SLOTS) nb <<= 1;
  L->nbuckets = nb;
  uint64_t o = 0;
  L->off_globals = o; o = align_up(o + sizeof(gfs_globals), kAlign);
  L->off_dev = o; o = align_up(o + sizeof(gfs_dev), kAlign);
  const uint64_t nf = c->max_files;
  L->off_files = o; o = align_up(o + sizeof(gfs_file_dev) * nf, kAlign);
  L->off_locks = o; o = align_up(o + sizeof(gfs_file_lock) * nf, kAlign);
  L->off_lockq = o; o = align_up(o + 8ull * GFS_LOCK_SLOTS * nf, kAlign);
  L->off_claims = o; o = align_up(o + sizeof(gfs_file_claims) * nf, kAlign);
  L->off_pslots = o;
  if (c->policy == GFS_POLICY_PRIVATE) o = align_up(o + sizeof(gfs_pslot) * c->private_slots, kAlign);
  L->off_names = o; o = align_up(o + (uint64_t)GFS_NAME_MAX * nf, kAlign);
  L->off_fword = o; o = align_up(o + 8 * L->nframes, kAlign);
  L->off_ftag = o; o = align_up(o + 8 * L->nframes, kAlign);
  L->off_pt = o; o = align_up(o + 8 * GFS_BUCKET_SLOTS * L->nbuckets, kAlign);
  L->off_ffill = o; o = align_up(o + 8 * L->nframes, kAlign);
  L->off_slot_free = o; o = align_up(o + 8ull * c->rpc_slots, kAlign);
  L->off_slot_tail = o; o = align_up(o + 8ull * c->rpc_slots, kAlign);
  L->off_reqd = o; o = align_up(o + sizeof(gfs_req_dev) * (uint64_t)c->rpc_slots, kAlign);
  L->off_trace = o; o = align_up(o + sizeof(gfs_event) * (uint64_t)c->trace_capacity, kAlign);
  L->meta_bytes = o;
  return 0;
}

struct HostFile {
  std::atomic<int> fd{-1};
  bool open = false;
  bool direct = false;
  uint64_t size = 0;
  std::string path;
};

}  // namespace

struct gfs_ctx {
  gfs_config cfg{};
  Layout L;
  int device = 0;
  hipStream_t stream = nullptr;
  uint8_t* frames = nullptr;
  uint8_t* meta = nullptr;
  gfs_dev hdev{};
  gfs_dev* ddev = nullptr;
  gfs_rpc_slot* ring = nullptr;   // host address (pinned, mapped)
  uint8_t* staging = nullptr;     // host address (pinned, mapped)
  HostFile files[GFS_MAX_FILES];
  std::vector<std::thread> threads;
  std::unique_ptr<std::atomic<uint64_t>[]> claimed;   // per ring slot: last generation a thread took
  std::atomic<bool> stop{false};
  std::atomic<uint64_t> host_requests{0}, host_bytes{0}, host_read_ns{0}, host_errors{0};
  std::atomic<int64_t> host_last_errno{0};
  std::atomic<uint64_t> spins[64];
  std::atomic<uint64_t> thread_requests[64];
  bool last_direct = false;
  int clock_khz = 100000;
  /* a request larger than one chunk is split; any I/O thread may read any chunk */
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
  std::mutex qmu;
  std::deque<Chunk> queue;
  std::atomic<uint32_t> queued{0};
  std::unique_ptr<Track[]> track;
};

namespace {

// Read file bytes [off, off+len) into dst (pinned staging). Returns bytes read (short only
// at end of file) or -errno. Direct reads cannot target the GPU driver's pinned pages (the
// kernel refuses to pin them for DMA, EFAULT), so they go through the thread's aligned
// bounce buffer in chunks and are copied into staging; buffered reads go straight in.
int64_t read_span(int fd, bool direct, uint8_t* dst, uint64_t off, uint64_t len, uint8_t* bounce,
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
void run_chunk(gfs_ctx* c, const gfs_ctx::Chunk& ch, uint8_t* bounce) {
  gfs_rpc_slot* rs = &c->ring[ch.slot];
  gfs_ctx::Track& tr = c->track[ch.slot];
  const uint32_t fid = rs->file_id;
  HostFile* hf = fid < GFS_MAX_FILES ? &c->files[fid] : nullptr;
  const int fd = hf ? hf->fd.load(std::memory_order_acquire) : -1;
  int64_t r;
  if (fd < 0) {
    r = -EBADF;
  } else {
    const uint64_t t0 = now_ns();
    r = read_span(fd, hf->direct, c->staging + (uint64_t)ch.slot * c->L.max_req_bytes + ch.dst,
                  ch.off, ch.len, bounce, c->cfg.io_chunk_bytes);
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

bool pop_chunk(gfs_ctx* c, gfs_ctx::Chunk* out) {
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
void io_thread_partitioned(gfs_ctx* c, int idx) {
  const uint32_t NS = c->cfg.rpc_slots, N = c->cfg.host_threads;
  const uint32_t lo = (uint32_t)((uint64_t)idx * NS / N), hi = (uint32_t)((uint64_t)(idx + 1) * NS / N);
  std::vector<uint64_t> want(hi - lo, 1);   // next generation of each own slot
  bool first = true;
  uint64_t spins = 0;
  const uint64_t chunk = c->cfg.io_chunk_bytes;
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
      const uint64_t n = len > c->L.max_req_bytes ? 0 : (len + chunk - 1) / chunk;
      gfs_ctx::Track& tr = c->track[s];
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
void io_thread(gfs_ctx* c, int idx) {
  const uint32_t NS = c->cfg.rpc_slots;
  bool first = true;
  uint64_t spins = 0;
  uint32_t pos = (uint32_t)((uint64_t)idx * NS / c->cfg.host_threads);
  const uint64_t chunk = c->cfg.io_chunk_bytes;
  uint8_t* bounce = (uint8_t*)aligned_alloc(kDirectAlign, chunk);
  if (!bounce) return;
  gfs_ctx::Chunk ch;
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
    const uint64_t n = len > c->L.max_req_bytes ? 0 : (len + chunk - 1) / chunk;
    gfs_ctx::Track& tr = c->track[s];
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

void start_threads(gfs_ctx* c) {
  c->stop.store(false);
  for (uint32_t i = 0; i < c->cfg.rpc_slots; ++i) c->claimed[i].store(0);
  for (uint32_t i = 0; i < c->cfg.host_threads; ++i)
    c->threads.emplace_back(c->cfg.io_backend == GFS_IO_PREAD_PARTITIONED ? io_thread_partitioned : io_thread, c,
                            (int)i);
}

void stop_threads(gfs_ctx* c) {
  c->stop.store(true);
  for (auto& t : c->threads) t.join();
  c->threads.clear();
  std::lock_guard<std::mutex> g(c->qmu);
  c->queue.clear();
  c->queued.store(0);
}

int hip_ok(hipError_t e) { return e == hipSuccess ? 0 : -EIO; }

int upload_file_record(gfs_ctx* c, int id, const gfs_file_dev& rec) {
  gfs_file_dev* dst = (gfs_file_dev*)(c->meta + c->L.off_files) + id;
  if (hipMemcpyAsync(dst, &rec, sizeof rec, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return -EIO;
  return hip_ok(hipStreamSynchronize(c->stream));
}

int download_file_record(gfs_ctx* c, int id, gfs_file_dev* rec) {
  const gfs_file_dev* src = (const gfs_file_dev*)(c->meta + c->L.off_files) + id;
  if (hipMemcpyAsync(rec, src, sizeof *rec, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return -EIO;
  return hip_ok(hipStreamSynchronize(c->stream));
}

// clear one file id's miss lock, its queue slots and its window claims (no kernel running)
int zero_file_locks(gfs_ctx* c, int id) {
  const Layout& L = c->L;
  int rc = gfs_internal_zero(c->meta + L.off_locks + sizeof(gfs_file_lock) * (uint64_t)id, sizeof(gfs_file_lock),
                             c->stream);
  if (!rc)
    rc = gfs_internal_zero(c->meta + L.off_lockq + 8ull * GFS_LOCK_SLOTS * (uint64_t)id, 8ull * GFS_LOCK_SLOTS,
                           c->stream);
  if (!rc)
    rc = gfs_internal_zero(c->meta + L.off_claims + sizeof(gfs_file_claims) * (uint64_t)id,
                           sizeof(gfs_file_claims), c->stream);
  return rc;
}

// zero the dynamic state: counters, hand, ring tail, frames, tags, table, slots, trace
int zero_dynamic(gfs_ctx* c) {
  const Layout& L = c->L;
  int rc = gfs_internal_zero(c->meta + L.off_globals, sizeof(gfs_globals), c->stream);
  // miss locks, their queue slots, window claims, private slots
  if (!rc) rc = gfs_internal_zero(c->meta + L.off_locks, L.off_names - L.off_locks, c->stream);
  if (!rc) rc = gfs_internal_zero(c->meta + L.off_fword, L.off_trace - L.off_fword, c->stream);
  if (!rc && c->cfg.trace_capacity)
    rc = gfs_internal_zero(c->meta + L.off_trace, sizeof(gfs_event) * (uint64_t)c->cfg.trace_capacity, c->stream);
  if (!rc) rc = hip_ok(hipStreamSynchronize(c->stream));
  memset(c->ring, 0, sizeof(gfs_rpc_slot) * c->cfg.rpc_slots);
  return rc;
}

}  // namespace

extern "C" {

void gfs_config_default(gfs_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof *cfg);
  cfg->abi_version = GFS_ABI_VERSION;
  cfg->streams_per_file = 8;
  cfg->page_size = 64 << 10;
  cfg->cache_bytes = 256ull << 20;
  cfg->ra_init_bytes = 4 * cfg->page_size;
  cfg->ra_cap_bytes = 16ull << 20;
  cfg->host_threads = 8;
  cfg->rpc_slots = 64;
  cfg->io_backend = GFS_IO_PREAD;
  cfg->o_direct = GFS_DIRECT_PREFER;
  cfg->trace_level = 0;
  cfg->trace_capacity = 0;
  cfg->wait_timeout_ns = 0;
  cfg->policy = GFS_POLICY_SHARED;
  cfg->private_slots = 512;
  cfg->io_chunk_bytes = 2u << 20;
  cfg->max_files = 64;
  cfg->ra_recent = 64;
  cfg->ra_near_pages = 64;
  cfg->ra_near_min = 3;
  cfg->ra_quota_blocks = 0;
  cfg->ra_async = 0;
}

int gfs_device_bytes(const gfs_config* cfg, size_t* frames_bytes, size_t* meta_bytes) {
  Layout L;
  const int rc = make_layout(cfg, &L);
  if (rc) return rc;
  if (frames_bytes) *frames_bytes = cfg->cache_bytes + L.pbuf_bytes;
  if (meta_bytes) *meta_bytes = L.meta_bytes;
  return 0;
}

int gfs_init(const gfs_config* cfg, void* frames_dev, void* meta_dev, void* hip_stream,
             gfs_ctx** out) {
  if (!out || !frames_dev || !meta_dev) return -EINVAL;
  if (((uintptr_t)frames_dev | (uintptr_t)meta_dev) & (kAlign - 1)) return -EINVAL;
  Layout L;
  int rc = make_layout(cfg, &L);
  if (rc) return rc;
  gfs_ctx* c = new (std::nothrow) gfs_ctx();
  if (!c) return -ENOMEM;
  for (auto& s : c->spins) s.store(0);
  for (auto& s : c->thread_requests) s.store(0);
  c->cfg = *cfg;
  c->L = L;
  c->stream = (hipStream_t)hip_stream;
  c->frames = (uint8_t*)frames_dev;
  c->meta = (uint8_t*)meta_dev;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return -EIO; }
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) != hipSuccess || khz <= 0) {
    delete c;
    return -EIO;
  }
  // every block the device can hold at once may wait on one file's miss lock: each needs
  // its own queue slot. A block that calls gread holds at least GFS_BLOCK_LDS_MIN bytes of
  // LDS and one wave, which bounds the blocks per CU.
  int cus = 0, thr_per_cu = 0, lds_per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
      hipDeviceGetAttribute(&thr_per_cu, hipDeviceAttributeMaxThreadsPerMultiProcessor, c->device) != hipSuccess ||
      hipDeviceGetAttribute(&lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, c->device) !=
          hipSuccess) {
    delete c;
    return -EIO;
  }
  {
    uint64_t per_cu = (uint64_t)(thr_per_cu / 64);
    const uint64_t by_lds = (uint64_t)lds_per_cu / GFS_BLOCK_LDS_MIN;
    if (lds_per_cu > 0 && by_lds < per_cu) per_cu = by_lds;
    if ((uint64_t)cus * per_cu > GFS_LOCK_SLOTS) {
      delete c;
      return -EINVAL;
    }
  }
  uint32_t quota_blocks = cfg->ra_quota_blocks;
  if (quota_blocks == 0) {
    // the blocks of the library's 256-thread reader kernels that fit on the device at once
    if (gfs_internal_resident_blocks(GFS_MAX_BLOCK_THREADS, &quota_blocks) != 0 || quota_blocks == 0) {
      delete c;
      return -EIO;
    }
  }
  const uint64_t ring_bytes = sizeof(gfs_rpc_slot) * (uint64_t)cfg->rpc_slots;
  const uint64_t staging_bytes = L.max_req_bytes * (uint64_t)cfg->rpc_slots;
  if (hipHostMalloc((void**)&c->ring, ring_bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    delete c;
    return -ENOMEM;
  }
  if (hipHostMalloc((void**)&c->staging, staging_bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    (void)hipHostFree(c->ring);
    delete c;
    return -ENOMEM;
  }
  void* dring = nullptr;
  void* dstg = nullptr;
  if (hipHostGetDevicePointer(&dring, c->ring, 0) != hipSuccess ||
      hipHostGetDevicePointer(&dstg, c->staging, 0) != hipSuccess) {
    (void)hipHostFree(c->staging);
    (void)hipHostFree(c->ring);
    delete c;
    return -EIO;
  }
  gfs_dev& h = c->hdev;
  memset(&h, 0, sizeof h);
  h.page_size = cfg->page_size;
  h.page_shift = log2u(cfg->page_size);
  h.nframes = (uint32_t)L.nframes;
  h.nbuckets_mask = (uint32_t)(L.nbuckets - 1);
  h.streams = cfg->streams_per_file;
  h.ra_init = (uint32_t)L.ra_init;
  h.ra_cap = (uint32_t)L.ra_cap;
  h.rpc_slots = cfg->rpc_slots;
  h.max_req_pages = (uint32_t)L.max_req_pages;
  h.trace_level = cfg->trace_level;
  h.trace_cap = cfg->trace_capacity;
  h.max_files = cfg->max_files;
  h.ra_recent = cfg->ra_recent;
  h.ra_near_pages = cfg->ra_near_pages;
  h.ra_near_min = cfg->ra_near_min;
  h.ra_quota_blocks = quota_blocks;
  c->cfg.ra_quota_blocks = quota_blocks;   /* gfs_get_config reports the resolved count */
  h.max_req_bytes = L.max_req_bytes;
  c->clock_khz = khz;
  const uint64_t tns = cfg->wait_timeout_ns ? cfg->wait_timeout_ns : 10000000000ull;
  h.timeout_ticks = tns / 1000 * (uint64_t)khz / 1000;
  h.frames = c->frames;
  h.g = (gfs_globals*)(c->meta + L.off_globals);
  h.files = (gfs_file_dev*)(c->meta + L.off_files);
  h.locks = (gfs_file_lock*)(c->meta + L.off_locks);
  h.lockq = (uint64_t*)(c->meta + L.off_lockq);
  h.claims = (gfs_file_claims*)(c->meta + L.off_claims);
  h.policy = cfg->policy;
  if (cfg->policy == GFS_POLICY_PRIVATE) {
    h.pslots = (gfs_pslot*)(c->meta + L.off_pslots);
    h.pbuf = c->frames + cfg->cache_bytes;
    h.npslots = cfg->private_slots;
    h.quota = (uint32_t)L.quota;
  }
  h.names = (char*)(c->meta + L.off_names);
  h.fword = (uint64_t*)(c->meta + L.off_fword);
  h.ftag = (uint64_t*)(c->meta + L.off_ftag);
  h.pt = (uint64_t*)(c->meta + L.off_pt);
  h.slot_free = (uint64_t*)(c->meta + L.off_slot_free);
  h.slot_tail = (uint64_t*)(c->meta + L.off_slot_tail);
  h.partitioned = cfg->io_backend == GFS_IO_PREAD_PARTITIONED ? 1u : 0u;
  h.ffill = (uint64_t*)(c->meta + L.off_ffill);
  h.reqd = (gfs_req_dev*)(c->meta + L.off_reqd);
  h.trace = c->meta + L.off_trace;
  h.ring = (gfs_rpc_slot*)dring;
  h.staging = (uint8_t*)dstg;
  c->ddev = (gfs_dev*)(c->meta + L.off_dev);
  rc = gfs_internal_zero(c->meta, L.meta_bytes, c->stream);
  if (!rc && hipMemcpyAsync(c->ddev, &h, sizeof h, hipMemcpyHostToDevice, c->stream) != hipSuccess) rc = -EIO;
  if (!rc) rc = hip_ok(hipStreamSynchronize(c->stream));
  if (rc) {
    (void)hipHostFree(c->staging);
    (void)hipHostFree(c->ring);
    delete c;
    return rc;
  }
  memset(c->ring, 0, ring_bytes);
  c->track.reset(new (std::nothrow) gfs_ctx::Track[cfg->rpc_slots]);
  c->claimed.reset(new (std::nothrow) std::atomic<uint64_t>[cfg->rpc_slots]);
  if (!c->track || !c->claimed) {
    (void)hipHostFree(c->staging);
    (void)hipHostFree(c->ring);
    delete c;
    return -ENOMEM;
  }
  start_threads(c);
  *out = c;
  return 0;
}

int gfs_open(gfs_ctx* c, const char* path, int flags, int* file_id) {
  if (!c || !path || !file_id) return -EINVAL;
  if (flags != GFS_O_RDONLY) return -EROFS;
  const size_t plen = strlen(path);
  if (plen == 0 || plen >= GFS_NAME_MAX) return -ENAMETOOLONG;
  int id = -1;
  for (int i = 0; i < (int)c->cfg.max_files; ++i)
    if (!c->files[i].open) { id = i; break; }
  if (id < 0) return -ENFILE;
  bool direct = false;
  int fd = -1;
  if (c->cfg.o_direct != GFS_DIRECT_OFF) {
    fd = open(path, O_RDONLY | O_DIRECT | O_CLOEXEC);
    if (fd >= 0) direct = true;
    else if (c->cfg.o_direct == GFS_DIRECT_ON || errno != EINVAL) return -errno;
  }
  if (fd < 0) {
    fd = open(path, O_RDONLY | O_CLOEXEC);
    if (fd < 0) return -errno;
  }
  struct stat st;
  if (fstat(fd, &st) != 0) { const int e = errno; close(fd); return -e; }
  const uint64_t size = (uint64_t)st.st_size;
  const uint64_t npages = (size + c->cfg.page_size - 1) / c->cfg.page_size;
  if (npages >= GFS_MAX_PAGES_PER_FILE) { close(fd); return -EFBIG; }
  posix_fadvise(fd, 0, 0, POSIX_FADV_DONTNEED);
  gfs_file_dev rec;
  memset(&rec, 0, sizeof rec);
  rec.size = size;
  rec.npages = (uint32_t)npages;
  rec.open = 1;
  rec.advice = GFS_ADV_NORMAL;
  char name[GFS_NAME_MAX];
  memset(name, 0, sizeof name);
  memcpy(name, path, plen);
  int rc = zero_file_locks(c, id);
  if (!rc) rc = upload_file_record(c, id, rec);
  if (!rc && hipMemcpyAsync(c->meta + c->L.off_names + (uint64_t)id * GFS_NAME_MAX, name, GFS_NAME_MAX,
                            hipMemcpyHostToDevice, c->stream) != hipSuccess)
    rc = -EIO;
  if (!rc) rc = hip_ok(hipStreamSynchronize(c->stream));
  if (rc) { close(fd); return rc; }
  HostFile& hf = c->files[id];
  hf.open = true;
  hf.direct = direct;
  hf.size = size;
  hf.path = path;
  hf.fd.store(fd, std::memory_order_release);
  c->last_direct = direct;
  *file_id = id;
  return 0;
}

int gfs_fadvise(gfs_ctx* c, int file_id, int advice) {
  if (!c || file_id < 0 || file_id >= (int)GFS_MAX_FILES || !c->files[file_id].open) return -EBADF;
  if (advice != GFS_ADV_NORMAL && advice != GFS_ADV_RANDOM && advice != GFS_ADV_SEQUENTIAL) return -EINVAL;
  gfs_file_dev rec;
  int rc = download_file_record(c, file_id, &rec);
  if (rc) return rc;
  rec.advice = (uint32_t)advice;
  return upload_file_record(c, file_id, rec);
}

int gfs_file_size(gfs_ctx* c, int file_id, uint64_t* size) {
  if (!c || file_id < 0 || file_id >= (int)GFS_MAX_FILES || !c->files[file_id].open) return -EBADF;
  if (!size) return -EINVAL;
  *size = c->files[file_id].size;
  return 0;
}

int gfs_get_config(gfs_ctx* c, gfs_config* out) {
  if (!c || !out) return -EINVAL;
  *out = c->cfg;
  return 0;
}

int gfs_close(gfs_ctx* c, int file_id) {
  if (!c || file_id < 0 || file_id >= (int)GFS_MAX_FILES || !c->files[file_id].open) return -EBADF;
  gfs_file_dev rec;
  int rc = download_file_record(c, file_id, &rec);
  if (rc) return rc;
  if (rec.handles != 0) return -EBUSY;
  // A page key is (id, page), and a later gfs_open may give this id to another file: drop
  // every cached page, reservation and frame of the file now, so that no read of the next
  // file under this id can find them, and clear the id's detector and lock state.
  memset(&rec, 0, sizeof rec);
  rc = upload_file_record(c, file_id, rec);
  if (!rc) rc = gfs_internal_purge_file(c->ddev, (uint32_t)c->L.nframes, c->L.nbuckets * GFS_BUCKET_SLOTS,
                                        (uint32_t)file_id, c->stream);
  if (!rc) rc = zero_file_locks(c, file_id);
  if (!rc) rc = hip_ok(hipStreamSynchronize(c->stream));
  if (rc) return rc;
  HostFile& hf = c->files[file_id];
  const int fd = hf.fd.exchange(-1);
  if (fd >= 0) close(fd);
  hf.open = false;
  hf.path.clear();
  return 0;
}

const struct gfs_dev* gfs_device_handle(gfs_ctx* c) { return c ? c->ddev : nullptr; }

int gfs_stats_read(gfs_ctx* c, gfs_stats* out) {
  if (!c || !out) return -EINVAL;
  gfs_globals g;
  if (hipMemcpyAsync(&g, c->meta + c->L.off_globals, sizeof g, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return -EIO;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return -EIO;
  gfs_stats s;
  memset(&s, 0, sizeof s);
  s.hits = g.ctr[GFS_C_HITS];
  s.joins = g.ctr[GFS_C_JOINS];
  s.misses = g.ctr[GFS_C_MISSES];
  s.ra_pages = g.ctr[GFS_C_RA_PAGES];
  s.fetched_pages = g.ctr[GFS_C_FETCHED];
  s.evictions = g.ctr[GFS_C_EVICTIONS];
  s.wasted_pages = g.ctr[GFS_C_WASTED];
  s.hand_visits = g.ctr[GFS_C_HAND];
  s.requests = g.ctr[GFS_C_REQUESTS];
  s.request_bytes = g.ctr[GFS_C_REQ_BYTES];
  s.delivered_bytes = g.ctr[GFS_C_DELIVERED];
  s.retries = g.ctr[GFS_C_RETRIES];
  s.noframe = g.ctr[GFS_C_NOFRAME];
  s.timeouts = g.ctr[GFS_C_TIMEOUTS];
  s.io_errors = g.ctr[GFS_C_IOERR];
  s.trace_events = g.trace_n;
  s.host_requests = c->host_requests.load();
  s.host_bytes = c->host_bytes.load();
  s.host_read_ns = c->host_read_ns.load();
  const double ns_per_tick = 1e6 / (double)c->clock_khz;
  s.t_lock_ns = (uint64_t)(g.ctr[GFS_T_LOCK] * ns_per_tick);
  s.t_crit_ns = (uint64_t)(g.ctr[GFS_T_CRIT] * ns_per_tick);
  s.t_alloc_ns = (uint64_t)(g.ctr[GFS_T_ALLOC] * ns_per_tick);
  s.t_slot_ns = (uint64_t)(g.ctr[GFS_T_SLOT] * ns_per_tick);
  s.t_host_ns = (uint64_t)(g.ctr[GFS_T_HOST] * ns_per_tick);
  s.t_pull_ns = (uint64_t)(g.ctr[GFS_T_PULL] * ns_per_tick);
  s.t_join_ns = (uint64_t)(g.ctr[GFS_T_JOIN] * ns_per_tick);
  s.t_decide_ns = (uint64_t)(g.ctr[GFS_T_DECIDE] * ns_per_tick);
  s.t_run_ns = (uint64_t)(g.ctr[GFS_T_RUN] * ns_per_tick);
  s.t_unlock_ns = (uint64_t)(g.ctr[GFS_T_UNLOCK] * ns_per_tick);
  s.lock_acquired = g.ctr[GFS_C_LOCKS];
  s.lock_left = g.ctr[GFS_C_LOCK_LEFT];
  s.t_acquire_ns = (uint64_t)(g.ctr[GFS_T_ACQUIRE] * ns_per_tick);
  s.t_copy_ns = (uint64_t)(g.ctr[GFS_T_COPY] * ns_per_tick);
  s.t_unpin_ns = (uint64_t)(g.ctr[GFS_T_UNPIN] * ns_per_tick);
  s.private_hits = g.ctr[GFS_C_PB_HITS];
  s.private_wasted = g.ctr[GFS_C_PB_WASTED];
  s.host_errors = c->host_errors.load();
  s.host_last_errno = (uint64_t)c->host_last_errno.load();
  for (uint32_t i = 0; i < 64; ++i) s.host_spins[i] = c->spins[i].load();
  for (uint32_t i = 0; i < 64; ++i) s.host_thread_requests[i] = c->thread_requests[i].load();
  s.host_threads = c->cfg.host_threads;
  s.direct_io = c->last_direct ? 1 : 0;
  *out = s;
  return 0;
}

int gfs_trace_read(gfs_ctx* c, void* dst, size_t cap_bytes, size_t* n_bytes) {
  if (!c || (!dst && cap_bytes) || !n_bytes) return -EINVAL;
  uint64_t n = 0;
  if (hipMemcpyAsync(&n, c->meta + c->L.off_globals + offsetof(gfs_globals, trace_n), 8,
                     hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return -EIO;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return -EIO;
  if (n > c->cfg.trace_capacity) n = c->cfg.trace_capacity;
  uint64_t bytes = n * sizeof(gfs_event);
  if (bytes > cap_bytes) bytes = cap_bytes / sizeof(gfs_event) * sizeof(gfs_event);
  if (bytes) {
    if (hipMemcpyAsync(dst, c->meta + c->L.off_trace, bytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      return -EIO;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return -EIO;
  }
  *n_bytes = bytes;
  return 0;
}

int gfs_reset_cache(gfs_ctx* c) {
  if (!c) return -EINVAL;
  stop_threads(c);
  int rc = zero_dynamic(c);
  // clear readahead streams, locks and clocks of registered files
  for (int i = 0; !rc && i < (int)c->cfg.max_files; ++i) {
    if (!c->files[i].open) continue;
    gfs_file_dev rec;
    rc = download_file_record(c, i, &rec);
    if (rc) break;
    const uint32_t advice = rec.advice;
    const uint32_t handles = rec.handles;
    memset(&rec, 0, sizeof rec);
    rec.size = c->files[i].size;
    rec.npages = (uint32_t)((rec.size + c->cfg.page_size - 1) / c->cfg.page_size);
    rec.open = 1;
    rec.advice = advice;
    rec.handles = handles;
    rc = upload_file_record(c, i, rec);
    if (c->files[i].direct) posix_fadvise(c->files[i].fd.load(), 0, 0, POSIX_FADV_DONTNEED);
  }
  c->host_requests = 0;
  c->host_bytes = 0;
  c->host_read_ns = 0;
  c->host_errors = 0;
  c->host_last_errno = 0;
  for (auto& s : c->spins) s.store(0);
  start_threads(c);
  return rc;
}

int gfs_shutdown(gfs_ctx* c) {
  if (!c) return -EINVAL;
  stop_threads(c);
  for (auto& f : c->files) {
    const int fd = f.fd.exchange(-1);
    if (fd >= 0) close(fd);
  }
  (void)hipHostFree(c->staging);
  (void)hipHostFree(c->ring);
  delete c;
  return 0;
}

}  // extern "C"

// ---- batch planning (host only) --------------------------------------------------------
extern "C" int gfs_batch_plan(const uint64_t* sizes, const uint32_t* ids, uint32_t nfiles,
                              uint64_t unit_bytes, uint32_t grid, uint32_t blocks_per_file,
                              gfs_unit* out, uint64_t cap, uint64_t* nout) {
  if (!sizes || !ids || !nout || nfiles == 0 || unit_bytes == 0 || unit_bytes % 16 || grid == 0 ||
      blocks_per_file == 0)
    return -EINVAL;
  uint64_t need = 0;
  for (uint32_t i = 0; i < nfiles; ++i) need += (sizes[i] + unit_bytes - 1) / unit_bytes;
  *nout = need;
  if (need > cap || (need && !out)) return -ENOSPC;
  uint32_t lanes = grid / blocks_per_file;
  if (lanes == 0) lanes = 1;
  struct Lane {
    uint32_t file;
    uint64_t next;
    bool busy;
  };
  std::vector<Lane> lane(lanes, Lane{0, 0, false});
  uint32_t next_file = 0;
  auto refill = [&](Lane& ln) {
    while (next_file < nfiles && sizes[next_file] == 0) ++next_file;
    if (next_file < nfiles) {
      ln = Lane{next_file++, 0, true};
    } else {
      ln.busy = false;
    }
  };
  for (auto& ln : lane) refill(ln);
  uint64_t n = 0;
  bool any = true;
  while (any) {
    any = false;
    for (auto& ln : lane) {
      if (!ln.busy) continue;
      any = true;
      const uint64_t left = sizes[ln.file] - ln.next;
      const uint64_t sz = left < unit_bytes ? left : unit_bytes;
      out[n++] = gfs_unit{ids[ln.file], ln.file, ln.next, sz};
      ln.next += sz;
      if (ln.next >= sizes[ln.file]) refill(ln);
    }
  }
  *nout = n;
  return 0;
}
