// Serving loop: a stream of whole-file read requests served by one persistent kernel.
//
// The host replays request arrivals on its own clock and admits them in arrival order
// while the cache bytes reserved by unfinished requests stay within a budget; each
// admitted request is appended to a submission array in pinned memory. On the device, the
// persistent blocks take (request, chunk) units oldest request first: a request's chunks
// are handed out by one fetch-and-add counter, so every block that finds work on the
// oldest request helps finish it, and new requests join between chunks. One block at a
// time polls the pinned submissions (so the rest spin on HBM only), copies new requests
// into the device table, and turns the host's close into the exit condition. The block
// that finishes a request's last chunk writes its completion record to pinned memory,
// where the host sees it.
#include <errno.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <deque>
#include <mutex>
#include <new>
#include <vector>

#include <hip/hip_runtime.h>

#include "gfs.h"
#include "gfs_consumers.h"
#include "gfs_device.h"
#include "gfs_layout.h"

extern "C" int gfs_internal_zero(void* p, size_t bytes, hipStream_t s);

namespace {

using gfs_consumers::block_sum_u64;
using gfs_consumers::checksum_part;

/* one admitted request, device memory, indexed by admission order */
struct SrvEntry {
  uint32_t ready;      /* 1 once the poller filled the entry in (release) */
  uint32_t file;
  uint64_t size;
  uint64_t nchunks;
  uint64_t next;       /* chunks handed out */
  uint64_t done;       /* chunks finished */
  uint64_t csum;       /* wrapping sum over finished chunks */
  uint64_t t_first;    /* wall_clock64 when the request's first page was delivered (0: not yet) */
  int64_t err;         /* -errno of the first failed chunk (0: none) */
};
static_assert(sizeof(SrvEntry) == 64, "entry is one 64-byte record");

/* device control words, one 128-byte line each */
struct SrvCtrl {
  uint64_t cursor;      uint64_t pad0[15];   /* entries below it have every chunk handed out */
  uint64_t ingested;    uint64_t pad1[15];   /* entries filled in (written by the poller only) */
  uint64_t poller;      uint64_t pad2[15];   /* 1 while a block polls the host */
  uint64_t final_n;     uint64_t pad3[15];   /* 0 until the host has closed; then requests + 1 */
  uint64_t abort;       uint64_t pad4[15];   /* 1: stop taking work */
  uint64_t progress;    uint64_t pad5[15];   /* wall_clock64 of the last chunk or submission seen */
};

/* pinned host memory */
struct SrvSub {
  uint32_t file;
  uint32_t pad;
  uint64_t size;
};
struct SrvHost {
  uint64_t tail;        uint64_t pad0[15];   /* submissions published (host, release) */
  uint64_t closed;      uint64_t pad1[15];   /* 1: nothing more will be submitted (host) */
  uint64_t abort;       uint64_t pad2[15];   /* 1: stop now (host) */
  uint64_t hello_tick;                       /* device clock when the kernel started */
  uint64_t hello;       uint64_t pad3[14];   /* 1 once hello_tick is written (device) */
};
struct SrvDone {
  uint64_t flag;        /* 1 when the record is complete (device, system-scope release) */
  uint64_t csum;
  int64_t result;
  uint64_t t_first;
  uint64_t t_done;
  uint64_t pad[3];
};
static_assert(sizeof(SrvDone) == 64, "completion record is 64 bytes");

constexpr int kWork = 0, kExit = 1;

/* Idle blocks back off to about 30 us between looks, so that a thousand of them polling
   the table stay a small load on the memory system next to the blocks at work. */
__device__ __forceinline__ void idle_nap(uint32_t& n) {
  const uint32_t reps = n < 4 ? 1 : (n < 16 ? 2 : 8);
  for (uint32_t j = 0; j < reps; ++j) __builtin_amdgcn_s_sleep(127);
  ++n;
}

__device__ __forceinline__ uint64_t ld_sys(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t ld_sys_rlx(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t ld_sys_rlx32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys_rel(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys_rlx(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

/* Write request i's completion record for the host. */
__device__ void complete_entry(SrvEntry* e, SrvDone* dn, uint64_t t_first) {
  const int64_t err = (int64_t)gfsd::ld_acq((uint64_t*)&e->err);
  st_sys_rlx(&dn->csum, gfsd::ld_acq(&e->csum));
  st_sys_rlx((uint64_t*)&dn->result, (uint64_t)(err ? err : (int64_t)e->size));
  st_sys_rlx(&dn->t_first, t_first);
  st_sys_rlx(&dn->t_done, wall_clock64());
  st_sys_rel(&dn->flag, 1);
}

/* The polling block: copy newly submitted requests into the table, and turn the host's
   close (or abort, or a silent host) into the device's exit condition. Thread 0 only. */
__device__ bool poll_host(SrvCtrl* ctl, SrvEntry* tab, uint32_t cap, const SrvSub* subs, SrvHost* host,
                          SrvDone* done, uint64_t chunk, uint64_t idle_ticks) {
  const uint64_t now = wall_clock64();
  if (ld_sys(&host->abort)) {
    gfsd::st_rel(&ctl->abort, 1);
    return false;
  }
  const uint64_t tail = std::min<uint64_t>(ld_sys(&host->tail), cap);
  const uint64_t ing = gfsd::ld_acq(&ctl->ingested);
  if (tail > ing) {
    for (uint64_t k = ing; k < tail; ++k) {
      SrvEntry* e = &tab[k];
      const uint64_t size = ld_sys_rlx(&subs[k].size);
      e->file = ld_sys_rlx32(&subs[k].file);
      e->size = size;
      e->nchunks = (size + chunk - 1) / chunk;
      __hip_atomic_store(&e->ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (size == 0) complete_entry(e, &done[k], now);
    }
    gfsd::st_rel(&ctl->ingested, tail);
    gfsd::st_rlx(&ctl->progress, now);
    return true;
  }
  if (ld_sys(&host->closed) && ld_sys(&host->tail) == ing) {
    gfsd::st_rel(&ctl->final_n, ing + 1);
    return false;
  }
  // other blocks store newer clock values into progress at any time: read the clock after
  // it, and compare signed, so that a value stored after `now` was read is not "idle"
  const uint64_t last = gfsd::ld_rlx(&ctl->progress);
  const uint64_t t = wall_clock64();
  if (last == 0) {
    gfsd::st_rlx(&ctl->progress, t);
  } else if ((int64_t)(t - last) > (int64_t)idle_ticks) {
    gfsd::st_rel(&ctl->abort, 1);
  }
  return false;
}

/* Thread 0: find the next unit, oldest request first, or decide to exit. The flags and
   counters are read relaxed: every block without work runs this loop, and an agent-scope
   acquire would invalidate its XCD's L2 each time; an entry's fields are read after one
   acquire fence, once its ready flag is seen. */
__device__ int pick_unit(SrvCtrl* ctl, SrvEntry* tab, uint32_t cap, const SrvSub* subs, SrvHost* host,
                         SrvDone* done, uint64_t chunk, uint64_t idle_ticks, uint64_t* oi, uint64_t* ok) {
  uint32_t naps = 0;
  while (true) {
    if (gfsd::ld_rlx(&ctl->abort)) return kExit;
    uint64_t c = gfsd::ld_rlx(&ctl->cursor);
    for (uint64_t i = c; i < cap; ++i) {
      SrvEntry* e = &tab[i];
      if (__hip_atomic_load(&e->ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) break;
      gfsd::acquire_agent();   /* the entry's fields, written before ready */
      const uint64_t nch = e->nchunks;
      // look before taking, so that idle blocks only read exhausted entries
      if (gfsd::ld_rlx(&e->next) < nch) {
        const uint64_t k = gfsd::fadd64(&e->next, 1);
        if (k < nch) {
          *oi = i;
          *ok = k;
          return kWork;
        }
      }
      if (i == c) {
        uint64_t expected = c;
        gfsd::cas64(&ctl->cursor, expected, c + 1);   // a failed swap means another block moved it
        c = c + 1;
      }
    }
    const uint64_t fin = gfsd::ld_rlx(&ctl->final_n);
    if (fin && gfsd::ld_rlx(&ctl->cursor) >= fin - 1) return kExit;
    uint64_t free_ = 0;
    if (gfsd::ld_rlx(&ctl->poller) == 0 && gfsd::cas64(&ctl->poller, free_, 1)) {
      const bool fresh = poll_host(ctl, tab, cap, subs, host, done, chunk, idle_ticks);
      gfsd::st_rel(&ctl->poller, 0);
      if (fresh) {
        naps = 0;
        continue;
      }
    }
    idle_nap(naps);
  }
}

__global__ void __launch_bounds__(GFS_MAX_BLOCK_THREADS, 2) serve_kernel(const gfs_dev* d, SrvEntry* tab, uint32_t cap, SrvCtrl* ctl, const SrvSub* subs,
                             SrvHost* host, SrvDone* done, uint8_t* buf, uint64_t chunk, uint64_t idle_ticks,
                             int64_t* status) {
  __shared__ uint64_t red[16];
  __shared__ uint64_t s_i, s_k, s_size;
  __shared__ uint32_t s_file;
  __shared__ int s_cmd;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  uint8_t* mybuf = buf + (uint64_t)blockIdx.x * chunk;
  if (blockIdx.x == 0 && tid == 0) {
    st_sys_rlx(&host->hello_tick, wall_clock64());
    st_sys_rel(&host->hello, 1);
  }
  int fd = -1;
  uint32_t cur_file = 0xffffffffu;
  int64_t err = 0, total = 0;
  while (true) {
    if (tid == 0) {
      uint64_t i = 0, k = 0;
      s_cmd = pick_unit(ctl, tab, cap, subs, host, done, chunk, idle_ticks, &i, &k);
      if (s_cmd == kWork) {
        s_i = i;
        s_k = k;
        s_file = tab[i].file;
        s_size = tab[i].size;
      }
    }
    __syncthreads();
    if (s_cmd == kExit) break;
    const uint64_t i = s_i, k = s_k, size = s_size;
    const uint32_t file = s_file;
    __syncthreads();
    int64_t r = 0;
    if (file != cur_file) {
      if (fd >= 0) gclose(d, fd);
      fd = gopen_id(d, (int)file, GFS_O_RDONLY);
      cur_file = fd >= 0 ? file : 0xffffffffu;
      if (fd < 0) r = fd;
    }
    const uint64_t off = k * chunk;
    const uint64_t len = std::min<uint64_t>(chunk, size - off);
    if (r == 0 && k == 0) {
      // the request's first page on its own, so that its delivery time is the time to
      // first page; then the rest of the chunk
      const uint64_t first = std::min<uint64_t>(len, d->page_size);
      r = gread(d, fd, 0, first, mybuf);
      if (r == (int64_t)first && tid == 0) {
        uint64_t zero = 0;
        gfsd::cas64(&tab[i].t_first, zero, wall_clock64());
      }
      if (r == (int64_t)first && first < len) {
        const int64_t r2 = gread(d, fd, first, len - first, mybuf + first);
        r = r2 < 0 ? r2 : r + r2;
      }
    } else if (r == 0) {
      r = gread(d, fd, off, len, mybuf);
    }
    const uint64_t part = r > 0 ? checksum_part(mybuf, (uint64_t)r, tid, nt) : 0;
    const uint64_t s = block_sum_u64(part, red, tid, nt);
    if (tid == 0) {
      SrvEntry* e = &tab[i];
      if (r < 0) {
        uint64_t zero = 0;
        gfsd::cas64((uint64_t*)&e->err, zero, (uint64_t)r);
        if (!err) err = r;
      } else {
        gfsd::fadd64(&e->csum, s);
        total += r;
      }
      const uint64_t now = wall_clock64();
      gfsd::st_rlx(&ctl->progress, now);
      const uint64_t prev = __hip_atomic_fetch_add(&e->done, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (prev + 1 == e->nchunks) complete_entry(e, &done[i], gfsd::ld_acq(&e->t_first));
    }
    __syncthreads();
  }
  if (fd >= 0) gclose(d, fd);
  if (tid == 0) status[blockIdx.x] = err ? err : total;
}

uint64_t host_ns() {
  timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (uint64_t)t.tv_sec * 1000000000ull + (uint64_t)t.tv_nsec;
}

void nap_ns(uint64_t ns) {
  timespec t{(time_t)(ns / 1000000000ull), (long)(ns % 1000000000ull)};
  nanosleep(&t, nullptr);
}

uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

/* Where one run keeps its state: device memory (request table, control words, block status,
   one chunk buffer per block), pinned host memory (submissions, host control, completion
   records; host and device addresses), and the host's per-request bookkeeping. */
struct ServeMem {
  SrvEntry* tab = nullptr;
  SrvCtrl* ctl = nullptr;
  int64_t* status = nullptr;
  uint8_t* bufs = nullptr;
  uint8_t* dev_clear = nullptr;      /* [tab, ctl, status]: zeroed before the launch */
  uint64_t dev_clear_bytes = 0;
  uint8_t* pin = nullptr;            /* host address of [subs | host control | completions] */
  uint8_t* dpin = nullptr;           /* its device address */
  uint64_t sub_bytes = 0, hc_bytes = 0, dn_bytes = 0;
  uint64_t* size = nullptr;          /* per request: file size */
  uint64_t* resv = nullptr;          /*   cache bytes it reserves */
  uint32_t* seq_req = nullptr;       /* per admission: the request */
  uint8_t* done_seen = nullptr;      /* per request: completion seen */
  uint32_t* queue = nullptr;         /* arrived, not admitted (FIFO; each request once) */
  uint32_t* inflight = nullptr;      /* admitted, not complete */
};

/* device and pinned bytes of a run of n requests on `grid` blocks */
struct ServeSizes {
  uint64_t tab, ctl, st, bufs, sub, hc, dn;
};
ServeSizes serve_sizes(uint32_t n, uint32_t grid, uint64_t chunk) {
  ServeSizes z;
  z.tab = round_up((uint64_t)n * sizeof(SrvEntry), 256);
  z.ctl = round_up(sizeof(SrvCtrl), 256);
  z.st = round_up((uint64_t)grid * 8, 256);
  z.bufs = round_up((uint64_t)grid * chunk, 256);
  z.sub = round_up((uint64_t)n * sizeof(SrvSub), 256);
  z.hc = round_up(sizeof(SrvHost), 256);
  z.dn = round_up((uint64_t)n * sizeof(SrvDone), 256);
  return z;
}

/* Checks shared by both entry points; sets the grid, the device clock rate and the page size. */
int serve_check(gfs_ctx* ctx, const gfs_serve_request* reqs, uint32_t n, const gfs_serve_params* p,
                gfs_serve_record* out, uint32_t* grid_out, int* khz_out, uint64_t* page_out) {
  if (!ctx || !reqs || !p || !out || n == 0 || n > (1u << 20)) return -EINVAL;
  if (p->budget_bytes == 0 || p->chunk_bytes == 0 || p->chunk_bytes % 16 || p->chunk_bytes > (64ull << 20))
    return -EINVAL;
  if (p->threads == 0 || p->threads % 64 || p->threads > GFS_MAX_BLOCK_THREADS) return -EINVAL;
  gfs_config cfg;
  if (gfs_get_config(ctx, &cfg)) return -EINVAL;
  uint32_t grid = p->grid;
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -EIO;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) return -EIO;
  if (grid == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, serve_kernel, (int)p->threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return -EIO;
    grid = (uint32_t)std::max(per_cu, 1) * (uint32_t)cus;
  }
  if (grid > (1u << 16)) return -EINVAL;
  *grid_out = grid;
  *khz_out = khz;
  *page_out = cfg.page_size;
  return 0;
}

/* Run the stream with the state in m (sized for n requests and `grid` blocks). */
int serve_core(gfs_ctx* ctx, const gfs_serve_request* reqs, uint32_t n, const gfs_serve_params* p,
               gfs_serve_record* out, gfs_serve_summary* summary, hipStream_t s, uint32_t grid, int khz,
               uint64_t page, const ServeMem& m) {
  uint64_t* size = m.size;
  uint64_t* resv = m.resv;
  for (uint32_t i = 0; i < n; ++i) {
    if (i && reqs[i].arrival_ns < reqs[i - 1].arrival_ns) return -EINVAL;
    if (gfs_file_size(ctx, (int)reqs[i].file_id, &size[i])) return -EBADF;
    resv[i] = round_up(size[i], page);
  }
  memset(m.pin, 0, m.sub_bytes + m.hc_bytes + m.dn_bytes);
  SrvSub* subs = (SrvSub*)m.pin;
  SrvHost* hc = (SrvHost*)(m.pin + m.sub_bytes);
  SrvDone* dn = (SrvDone*)(m.pin + m.sub_bytes + m.hc_bytes);
  int rc = gfs_internal_zero(m.dev_clear, m.dev_clear_bytes, s);
  if (rc) return rc;
  const uint64_t idle_ns = p->idle_timeout_ns ? p->idle_timeout_ns : 60000000000ull;
  const uint64_t idle_ticks = idle_ns / 1000 * (uint64_t)khz / 1000;
  hipLaunchKernelGGL(serve_kernel, dim3(grid), dim3(p->threads), 0, s, gfs_device_handle(ctx), m.tab, n, m.ctl,
                     (const SrvSub*)m.dpin, (SrvHost*)(m.dpin + m.sub_bytes),
                     (SrvDone*)(m.dpin + m.sub_bytes + m.hc_bytes), m.bufs, p->chunk_bytes, idle_ticks, m.status);
  if (hipGetLastError() != hipSuccess) return -EIO;

  // the host must always let the kernel end: close (or abort) before waiting for it
  auto finish = [&](bool abort) -> int {
    if (abort) __atomic_store_n(&hc->abort, 1ull, __ATOMIC_RELEASE);
    __atomic_store_n(&hc->closed, 1ull, __ATOMIC_RELEASE);
    return hipStreamSynchronize(s) == hipSuccess ? 0 : -EIO;
  };

  // the run's clock starts when the kernel is seen running; the moment the flag was seen
  // fixes the device clock's offset, to within the gap between the last two polls
  uint64_t prev_poll = host_ns(), t0 = 0;
  const uint64_t wait_start = prev_poll;
  while (true) {
    const uint64_t t = host_ns();
    if (__atomic_load_n(&hc->hello, __ATOMIC_ACQUIRE)) {
      t0 = t;
      break;
    }
    prev_poll = t;
    if (t - wait_start > 30000000000ull || hipStreamQuery(s) != hipErrorNotReady) {
      finish(true);
      return -EIO;
    }
  }
  const uint64_t hello_tick = __atomic_load_n(&hc->hello_tick, __ATOMIC_ACQUIRE);
  const double ns_per_tick = 1e6 / (double)khz;
  auto dev_to_run_ns = [&](uint64_t tick) -> uint64_t {
    const double v = ((double)tick - (double)hello_tick) * ns_per_tick;
    return v > 0 ? (uint64_t)v : 0;
  };

  uint32_t* seq_req = m.seq_req;
  uint8_t* done_seen = m.done_seen;
  memset(done_seen, 0, n);
  uint32_t* queue = m.queue;        // arrived requests waiting for admission: [qhead, qtail)
  uint32_t qhead = 0, qtail = 0;
  uint32_t* inflight = m.inflight;  // admission numbers not yet complete: [0, ninflight)
  uint32_t ninflight = 0;
  uint64_t reserved = 0, peak_reserved = 0, delivered = 0, last_query = 0;
  uint32_t next = 0, admitted = 0, completed = 0, peak_pending = 0;
  int err = 0;
  for (uint32_t i = 0; i < n; ++i) out[i] = gfs_serve_record{};
  while (completed < n) {
    uint64_t now = host_ns() - t0;
    while (next < n && reqs[next].arrival_ns <= now) queue[qtail++] = next++;
    peak_pending = std::max<uint32_t>(peak_pending, qtail - qhead);
    while (qhead < qtail) {
      const uint32_t r = queue[qhead];
      if (ninflight && reserved + resv[r] > p->budget_bytes) break;
      const uint32_t q = admitted++;
      subs[q].file = reqs[r].file_id;
      subs[q].size = size[r];
      seq_req[q] = r;
      out[r].arrival_ns = reqs[r].arrival_ns;
      out[r].admit_ns = host_ns() - t0;
      out[r].seq = q;
      out[r].reserved = resv[r];
      __atomic_store_n(&hc->tail, (uint64_t)admitted, __ATOMIC_RELEASE);
      reserved += resv[r];
      peak_reserved = std::max(peak_reserved, reserved);
      inflight[ninflight++] = q;
      ++qhead;
    }
    bool progress = false;
    for (uint32_t j = 0; j < ninflight;) {
      const uint32_t q = inflight[j];
      if (!__atomic_load_n(&dn[q].flag, __ATOMIC_ACQUIRE)) {
        ++j;
        continue;
      }
      const uint32_t r = seq_req[q];
      done_seen[r] = 1;
      out[r].done_ns = host_ns() - t0;
      out[r].csum = dn[q].csum;
      out[r].result = dn[q].result;
      out[r].first_ns = dev_to_run_ns(dn[q].t_first);
      if (out[r].result > 0) delivered += (uint64_t)out[r].result;
      reserved -= resv[r];
      ++completed;
      inflight[j] = inflight[--ninflight];
      progress = true;
    }
    if (progress) continue;
    now = host_ns() - t0;
    if (now - last_query > 1000000ull) {   // the kernel must still be running
      last_query = now;
      if (hipStreamQuery(s) != hipErrorNotReady) {
        err = -ETIMEDOUT;
        break;
      }
    }
    if (qhead == qtail && next < n && reqs[next].arrival_ns > now + 100000ull)
      nap_ns(std::min<uint64_t>(reqs[next].arrival_ns - now - 50000ull, 200000ull));
    else
      nap_ns(2000);
  }
  const uint64_t span = host_ns() - t0;
  const int frc = finish(err != 0);
  if (!err) err = frc;
  // requests the kernel never finished (it stopped early) are reported cancelled
  for (uint32_t i = 0; i < n; ++i)
    if (!done_seen[i]) out[i].result = -ECANCELED;
  if (summary) {
    summary->span_ns = span;
    summary->delivered_bytes = delivered;
    summary->peak_reserved = peak_reserved;
    summary->peak_pending = peak_pending;
    summary->grid = grid;
    summary->clock_skew_ns = t0 - prev_poll;
  }
  return err;
}

/* buffers of one gfs_serve_run; freed on every exit path */
struct ServeBuffers {
  uint8_t* dev = nullptr;    /* table, control, block status */
  uint8_t* bufs = nullptr;   /* one chunk buffer per block */
  uint8_t* pin = nullptr;    /* submissions, host control, completion records (pinned) */
  ~ServeBuffers() {
    if (dev) (void)hipFree(dev);
    if (bufs) (void)hipFree(bufs);
    if (pin) (void)hipHostFree(pin);
  }
};

/* ---- the entry point that allocates nothing ----
 * Its device state lives in `scratch`, one array per GPU the library runs on, held until the
 * process ends. Host code never passes the array's name to a kernel (in host code it is a
 * stand-in, not a device address): the device address comes from hipGetSymbolAddress, taken
 * once per device at gfs_init with that device current, and is used everywhere instead. */
static __device__ __align__(256) uint8_t scratch[GFS_SERVE_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

}  // namespace

/* The pinned mailbox and host bookkeeping of gfs_serve_run_noalloc, allocated once per
   context at gfs_init for GFS_SERVE_NOALLOC_MAX_REQUESTS requests. */
struct gfs_serve_area {
  int device = -1;
  uint8_t* pin = nullptr;    /* host address */
  uint8_t* dpin = nullptr;   /* device address */
  uint64_t* size = nullptr;
  uint64_t* resv = nullptr;
  uint32_t* seq_req = nullptr;
  uint8_t* done_seen = nullptr;
  uint32_t* queue = nullptr;
  uint32_t* inflight = nullptr;
};

extern "C" void gfs_internal_serve_teardown(gfs_serve_area* a) {
  if (!a) return;
  if (a->pin) (void)hipHostFree(a->pin);
  delete[] a->size;
  delete[] a->resv;
  delete[] a->seq_req;
  delete[] a->done_seen;
  delete[] a->queue;
  delete[] a->inflight;
  delete a;
}

/* Called by gfs_init with `device` current: look up this device's scratch address (once per
   device), and allocate the context's mailbox. 0, -ENOMEM or -EIO. */
extern "C" int gfs_internal_serve_setup(int device, gfs_serve_area** out) {
  if (device < 0 || device >= kMaxDevices || !out) return -EINVAL;
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_addr[device]) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return -EIO;
      g_scratch_addr[device] = ptr;
    }
  }
  const uint32_t n = GFS_SERVE_NOALLOC_MAX_REQUESTS;
  const ServeSizes z = serve_sizes(n, 1, 16);
  gfs_serve_area* a = new (std::nothrow) gfs_serve_area;
  if (!a) return -ENOMEM;
  a->device = device;
  a->size = new (std::nothrow) uint64_t[n];
  a->resv = new (std::nothrow) uint64_t[n];
  a->seq_req = new (std::nothrow) uint32_t[n];
  a->done_seen = new (std::nothrow) uint8_t[n];
  a->queue = new (std::nothrow) uint32_t[n];
  a->inflight = new (std::nothrow) uint32_t[n];
  if (!a->size || !a->resv || !a->seq_req || !a->done_seen || !a->queue || !a->inflight ||
      hipHostMalloc((void**)&a->pin, z.sub + z.hc + z.dn, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    a->pin = nullptr;
    gfs_internal_serve_teardown(a);
    return -ENOMEM;
  }
  void* dp = nullptr;
  if (hipHostGetDevicePointer(&dp, a->pin, 0) != hipSuccess) {
    gfs_internal_serve_teardown(a);
    return -EIO;
  }
  a->dpin = (uint8_t*)dp;
  *out = a;
  return 0;
}

extern "C" gfs_serve_area* gfs_internal_ctx_serve_area(gfs_ctx* ctx);

extern "C" int gfs_serve_run(gfs_ctx* ctx, const gfs_serve_request* reqs, uint32_t n,
                             const gfs_serve_params* p, gfs_serve_record* out, gfs_serve_summary* summary,
                             void* hip_stream) {
  uint32_t grid = 0;
  int khz = 0;
  uint64_t page = 0;
  int rc = serve_check(ctx, reqs, n, p, out, &grid, &khz, &page);
  if (rc) return rc;
  const ServeSizes z = serve_sizes(n, grid, p->chunk_bytes);
  ServeBuffers B;
  if (hipMalloc((void**)&B.dev, z.tab + z.ctl + z.st) != hipSuccess) return -ENOMEM;
  if (hipMalloc((void**)&B.bufs, z.bufs) != hipSuccess) return -ENOMEM;
  if (hipHostMalloc((void**)&B.pin, z.sub + z.hc + z.dn, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
    return -ENOMEM;
  void* dpin = nullptr;
  if (hipHostGetDevicePointer(&dpin, B.pin, 0) != hipSuccess) return -EIO;
  std::vector<uint64_t> size(n), resv(n);
  std::vector<uint32_t> seq_req(n), queue(n), inflight(n);
  std::vector<uint8_t> done_seen(n);
  ServeMem m;
  m.tab = (SrvEntry*)B.dev;
  m.ctl = (SrvCtrl*)(B.dev + z.tab);
  m.status = (int64_t*)(B.dev + z.tab + z.ctl);
  m.bufs = B.bufs;
  m.dev_clear = B.dev;
  m.dev_clear_bytes = z.tab + z.ctl + z.st;
  m.pin = B.pin;
  m.dpin = (uint8_t*)dpin;
  m.sub_bytes = z.sub;
  m.hc_bytes = z.hc;
  m.dn_bytes = z.dn;
  m.size = size.data();
  m.resv = resv.data();
  m.seq_req = seq_req.data();
  m.done_seen = done_seen.data();
  m.queue = queue.data();
  m.inflight = inflight.data();
  return serve_core(ctx, reqs, n, p, out, summary, (hipStream_t)hip_stream, grid, khz, page, m);
}

extern "C" int gfs_serve_run_noalloc(gfs_ctx* ctx, const gfs_serve_request* reqs, uint32_t n,
                                     const gfs_serve_params* p, gfs_serve_record* out,
                                     gfs_serve_summary* summary, void* hip_stream) {
  uint32_t grid = 0;
  int khz = 0;
  uint64_t page = 0;
  int rc = serve_check(ctx, reqs, n, p, out, &grid, &khz, &page);
  if (rc) return rc;
  gfs_serve_area* a = gfs_internal_ctx_serve_area(ctx);
  int dev = -1;
  if (!a || hipGetDevice(&dev) != hipSuccess) return -EIO;
  if (dev != a->device) return -EINVAL;   /* the context's device must be current */
  uint8_t* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    base = (uint8_t*)g_scratch_addr[dev];
  }
  if (!base) return -EIO;
  if (n > GFS_SERVE_NOALLOC_MAX_REQUESTS) return -E2BIG;
  const ServeSizes z = serve_sizes(n, grid, p->chunk_bytes);
  if (z.tab + z.ctl + z.st + z.bufs > GFS_SERVE_NOALLOC_SCRATCH_BYTES) return -E2BIG;
  const ServeSizes zmax = serve_sizes(GFS_SERVE_NOALLOC_MAX_REQUESTS, 1, 16);
  ServeMem m;
  m.tab = (SrvEntry*)base;
  m.ctl = (SrvCtrl*)(base + z.tab);
  m.status = (int64_t*)(base + z.tab + z.ctl);
  m.bufs = base + z.tab + z.ctl + z.st;
  m.dev_clear = base;
  m.dev_clear_bytes = z.tab + z.ctl + z.st;
  // the mailbox keeps its full-size layout; this run uses the first n entries of each part
  m.pin = a->pin;
  m.dpin = a->dpin;
  m.sub_bytes = zmax.sub;
  m.hc_bytes = zmax.hc;
  m.dn_bytes = zmax.dn;
  m.size = a->size;
  m.resv = a->resv;
  m.seq_req = a->seq_req;
  m.done_seen = a->done_seen;
  m.queue = a->queue;
  m.inflight = a->inflight;
  return serve_core(ctx, reqs, n, p, out, summary, (hipStream_t)hip_stream, grid, khz, page, m);
}
