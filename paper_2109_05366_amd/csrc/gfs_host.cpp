// Host runtime of the GPU file page cache: context set-up (HBM metadata layout, pinned ring
// and staging), the file registry, statistics, trace, reset and shutdown (Sec. 2.2: the
// GPU page cache and the shared CPU-GPU request queue). The host I/O threads that serve the
// ring are in gfs_hostio.h; the host issues no copy calls: the GPU pulls each request's
// bytes from pinned staging itself.
#include <errno.h>
#include <fcntl.h>
#include <sched.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <time.h>
#include <unistd.h>

#include <algorithm>
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
#include "gfs_hostio.h"
#include "gfs_layout.h"

extern "C" int gfs_internal_zero(void* p, size_t bytes, hipStream_t s);
extern "C" int gfs_internal_resident_blocks(uint32_t threads, uint32_t* blocks);
struct gfs_serve_area;
extern "C" int gfs_internal_serve_setup(int device, gfs_serve_area** out);
extern "C" void gfs_internal_serve_teardown(gfs_serve_area* a);
extern "C" int gfs_internal_purge_file(const gfs_dev* ddev, uint32_t nframes, uint64_t pt_entries, uint32_t file,
                                       hipStream_t s);

namespace {

constexpr uint64_t kAlign = 256;

using gfs_hostio::align_up;
using gfs_hostio::kDirectAlign;
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
  uint64_t off_globals = 0, off_dev = 0, off_files = 0, off_locks = 0, off_lockq = 0, off_claims = 0, off_shadow = 0, off_pslots = 0, off_names = 0, off_fword = 0,
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
  if (c->io_backend != GFS_IO_PREAD && c->io_backend != GFS_IO_PREAD_PARTITIONED && c->io_backend != GFS_IO_URING)
    return -EINVAL;
  if (c->io_depth < 1 || c->io_depth > 256) return -EINVAL;
  if (c->io_backend == GFS_IO_PREAD_PARTITIONED && c->host_threads > c->rpc_slots) return -EINVAL;
  if (c->o_direct > GFS_DIRECT_PREFER) return -EINVAL;
  if (c->trace_level > 2) return -EINVAL;
  if (c->io_chunk_bytes % kDirectAlign || c->io_chunk_bytes < (64u << 10) || c->io_chunk_bytes > (64u << 20))
    return -EINVAL;
  if (c->max_files < 1 || c->max_files > GFS_MAX_FILES) return -EINVAL;
  if (c->ra_recent < 1 || c->ra_recent > GFS_MAX_RECENT) return -EINVAL;
  if (c->ra_near_pages > (1u << 20) || c->ra_near_min < 1 || c->ra_near_min > c->ra_recent + 1) return -EINVAL;
  if (c->ra_async > 1) return -EINVAL;
  if (c->ra_async && c->policy != GFS_POLICY_SHARED) return -EINVAL;   /* markers live in the shared cache */
  if (c->ra_async && c->rpc_slots < 2) return -EINVAL;   /* asynchronous windows need slots of their own */
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
  L->off_shadow = o; o = align_up(o + (uint64_t)(GFS_SHADOW_PAGES / 8) * nf, kAlign);
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
  gfs_hostio::HostFile files[GFS_MAX_FILES];
  gfs_hostio::HostIo io;          // the host I/O threads serving the ring
  bool last_direct = false;
  int clock_khz = 100000;
  gfs_serve_area* serve = nullptr;   // pinned mailbox of gfs_serve_run_noalloc
};

namespace {

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

// clear one file id's miss lock, its queue slots, its window claims and its record of pages
// evicted after use (no kernel running)
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
  if (!rc)
    rc = gfs_internal_zero(c->meta + L.off_shadow + (uint64_t)(GFS_SHADOW_PAGES / 8) * id, GFS_SHADOW_PAGES / 8,
                           c->stream);
  return rc;
}

// zero the dynamic state: counters, hand, ring tail, frames, tags, table, slots, trace
int zero_dynamic(gfs_ctx* c) {
  const Layout& L = c->L;
  int rc = gfs_internal_zero(c->meta + L.off_globals, sizeof(gfs_globals), c->stream);
  // miss locks, their queue slots, window claims, evicted-after-use bits, private slots
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
  cfg->io_depth = 8;
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
  // the io_uring backend needs the kernel's io_uring (a system can switch it off)
  if (cfg->io_backend == GFS_IO_URING) {
    const int rc = gfs_hostio::uring_available();
    if (rc) {
      delete c;
      return rc == -EPERM || rc == -ENOSYS ? -ENOSYS : rc;
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
  // asynchronous windows get a quarter of the ring (at least one slot) to themselves
  h.sync_slots = cfg->ra_async ? cfg->rpc_slots - std::max(1u, cfg->rpc_slots / 4) : cfg->rpc_slots;
  h.max_req_pages = (uint32_t)L.max_req_pages;
  h.trace_level = cfg->trace_level;
  h.trace_cap = cfg->trace_capacity;
  h.max_files = cfg->max_files;
  h.ra_recent = cfg->ra_recent;
  h.ra_near_pages = cfg->ra_near_pages;
  h.ra_near_min = cfg->ra_near_min;
  h.ra_quota_blocks = quota_blocks;
  h.ra_async = cfg->ra_async;
  h.page_timers = cfg->page_timers ? 1u : 0u;
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
  h.shadow = (uint64_t*)(c->meta + L.off_shadow);
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
  // the no-alloc serving entry point: this device's scratch address and the context's mailbox
  rc = gfs_internal_serve_setup(c->device, &c->serve);
  if (rc) {
    (void)hipHostFree(c->staging);
    (void)hipHostFree(c->ring);
    delete c;
    return rc;
  }
  gfs_hostio::HostIo& io = c->io;
  io.rpc_slots = cfg->rpc_slots;
  io.host_threads = cfg->host_threads;
  io.io_backend = cfg->io_backend;
  io.io_depth = cfg->io_depth;
  io.io_chunk_bytes = cfg->io_chunk_bytes;
  io.max_req_bytes = L.max_req_bytes;
  io.ring = c->ring;
  io.staging = c->staging;
  io.files = c->files;
  if (io.init() != 0) {
    gfs_internal_serve_teardown(c->serve);
    (void)hipHostFree(c->staging);
    (void)hipHostFree(c->ring);
    delete c;
    return -ENOMEM;
  }
  gfs_hostio::start_threads(&io);
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
  gfs_hostio::HostFile& hf = c->files[id];
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
  gfs_hostio::HostFile& hf = c->files[file_id];
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
  s.host_requests = c->io.host_requests.load();
  s.host_bytes = c->io.host_bytes.load();
  s.host_read_ns = c->io.host_read_ns.load();
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
  s.ra_async_windows = g.ctr[GFS_C_ADVANCES];
  s.host_errors = c->io.host_errors.load();
  s.host_last_errno = (uint64_t)c->io.host_last_errno.load();
  for (uint32_t i = 0; i < 64; ++i) s.host_spins[i] = c->io.spins[i].load();
  for (uint32_t i = 0; i < 64; ++i) s.host_thread_requests[i] = c->io.thread_requests[i].load();
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
  gfs_hostio::stop_threads(&c->io);
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
  c->io.clear_counters();
  gfs_hostio::start_threads(&c->io);
  return rc;
}

int gfs_shutdown(gfs_ctx* c) {
  if (!c) return -EINVAL;
  gfs_hostio::stop_threads(&c->io);
  for (auto& f : c->files) {
    const int fd = f.fd.exchange(-1);
    if (fd >= 0) close(fd);
  }
  gfs_internal_serve_teardown(c->serve);
  (void)hipHostFree(c->staging);
  (void)hipHostFree(c->ring);
  delete c;
  return 0;
}

gfs_serve_area* gfs_internal_ctx_serve_area(gfs_ctx* c) { return c ? c->serve : nullptr; }

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
