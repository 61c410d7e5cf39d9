// Host-only check of the request-ring I/O engine (gfs_hostio.h), built with g++ (under
// ThreadSanitizer by the CPU tests): host threads stand in for GPU blocks and use the real
// ring ABI (gfs_rpc_slot) the way the device does -- a ticket picks the slot and generation,
// the slot is written and its generation published with a release store, the block waits
// for done_seq with an acquire load and a deadline, checks the staged bytes, and frees the
// slot. Every host read backend is driven: the shared ring (any thread takes any posted
// request), the partitioned one (a block posts into its own slot, each host thread serves
// its own range) and the io_uring one (the shared ring with DEPTH reads in flight per host
// thread). Error paths: a request for an unregistered file gets -EBADF, reads that cross the
// end of the file come back short.
//
// usage: hostio_check DIR BACKEND HOST_THREADS SLOTS PRODUCERS REQUESTS DIRECT [DEPTH [CHUNK_KIB MIN_PIECE_KIB]]
// prints one summary line; exit status 0 when every check held, 5 when io_uring is asked for
// and the kernel refuses to create one.
#include <fcntl.h>
#include <stdio.h>
#include <sys/stat.h>

#include <random>

#include "gfs_hostio.h"

namespace {

constexpr uint64_t kPage = 64 << 10;
constexpr uint32_t kMaxPages = 8;                  // pages per request at most
constexpr uint64_t kSizes[2] = {(9ull << 20) + 13, (3ull << 20) + 4101};

uint8_t pattern(int f, uint64_t o) { return (uint8_t)((o >> 2) * 131u + o * 7u + (uint64_t)f * 29u); }

bool write_file(const std::string& path, int f) {
  FILE* fh = fopen(path.c_str(), "wb");
  if (!fh) return false;
  std::vector<uint8_t> buf(1 << 20);
  for (uint64_t o = 0; o < kSizes[f]; o += buf.size()) {
    const uint64_t n = std::min<uint64_t>(buf.size(), kSizes[f] - o);
    for (uint64_t i = 0; i < n; ++i) buf[i] = pattern(f, o + i);
    if (fwrite(buf.data(), 1, n, fh) != n) return false;
  }
  return fclose(fh) == 0;
}

bool wait_u64(const uint64_t* p, uint64_t want, uint64_t deadline_ns) {
  while (__atomic_load_n(p, __ATOMIC_ACQUIRE) != want) {
    if (gfs_hostio::now_ns() > deadline_ns) return false;
    std::this_thread::yield();
  }
  return true;
}

struct Shared {
  gfs_hostio::HostIo* io;
  std::vector<uint64_t> slot_free;       // generation of each slot's last finished use
  std::vector<uint64_t> slot_tail;       // partitioned queue: posts into each slot
  uint64_t ring_tail = 0;
  std::atomic<uint64_t> bytes{0}, requests{0}, failures{0}, ebadf{0}, short_reads{0};
};

void producer(Shared* sh, int id, int nreq, bool partitioned) {
  gfs_hostio::HostIo* io = sh->io;
  std::mt19937_64 rng(1000 + id);
  const uint32_t S = io->rpc_slots;
  for (int r = 0; r < nreq; ++r) {
    // the device's ticket: shared ring or the block's own slot
    uint64_t tk;
    if (partitioned) {
      const uint32_t s = (uint32_t)id % S;
      tk = __atomic_fetch_add(&sh->slot_tail[s], 1, __ATOMIC_RELAXED) * S + s;
    } else {
      tk = __atomic_fetch_add(&sh->ring_tail, 1, __ATOMIC_RELAXED);
    }
    const uint32_t s = (uint32_t)(tk % S);
    const uint64_t gen = tk / S + 1;
    const uint64_t deadline = gfs_hostio::now_ns() + 20000000000ull;
    if (!wait_u64(&sh->slot_free[s], gen - 1, deadline)) {
      sh->failures++;
      return;
    }
    const bool bad = (rng() % 16) == 0;          // a file id that is not registered
    const int f = (int)(rng() % 2);
    const uint64_t npg = (kSizes[f] + kPage - 1) / kPage;
    const uint64_t p0 = rng() % npg;
    const uint32_t np = 1 + (uint32_t)(rng() % kMaxPages);
    const uint64_t off = p0 * kPage;
    uint64_t len = (uint64_t)np * kPage;
    if (off + len > kSizes[f]) len = kSizes[f] - off;
    gfs_rpc_slot* rs = &io->ring[s];
    rs->file_id = bad ? 7u : (uint32_t)f;
    rs->npages = np;
    rs->offset = off;
    rs->length = len;
    rs->ticket = tk;
    __atomic_store_n(&rs->req_seq, gen, __ATOMIC_RELEASE);
    if (!wait_u64(&rs->done_seq, gen, deadline)) {
      sh->failures++;
      return;
    }
    const int64_t res = rs->result;
    const uint8_t* stg = io->staging + (uint64_t)s * io->max_req_bytes;
    if (bad) {
      if (res != -EBADF) sh->failures++;
      sh->ebadf++;
    } else if (res != (int64_t)len) {
      sh->failures++;
    } else {
      for (uint64_t i = 0; i < len; ++i)
        if (stg[i] != pattern(f, off + i)) {
          sh->failures++;
          break;
        }
      sh->bytes += len;
      if (len < (uint64_t)np * kPage) sh->short_reads++;
    }
    sh->requests++;
    __atomic_store_n(&sh->slot_free[s], gen, __ATOMIC_RELEASE);
  }
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 8 && argc != 9 && argc != 11) {
    fprintf(stderr, "usage: %s DIR BACKEND HOST_THREADS SLOTS PRODUCERS REQUESTS DIRECT [DEPTH [CHUNK_KIB MIN_PIECE_KIB]]\n", argv[0]);
    return 2;
  }
  const std::string dir = argv[1];
  const uint32_t backend = (uint32_t)atoi(argv[2]), threads = (uint32_t)atoi(argv[3]), slots = (uint32_t)atoi(argv[4]);
  const int producers = atoi(argv[5]), nreq = atoi(argv[6]);
  const bool direct = atoi(argv[7]) != 0;
  const uint32_t depth = argc >= 9 ? (uint32_t)atoi(argv[8]) : 4u;
  /* optional: piece size and smallest piece in KiB (default 64 and the library's 256: no
     request is then cut finer than its 64 KiB pieces) */
  const uint64_t chunk_kib = argc >= 10 ? (uint64_t)atoi(argv[9]) : 64u;
  const uint64_t min_piece_kib = argc >= 11 ? (uint64_t)atoi(argv[10]) : 256u;
  if (backend == GFS_IO_URING && gfs_hostio::uring_available() != 0) {
    printf("io_uring unavailable\n");
    return 5;
  }
  static gfs_hostio::HostFile files[GFS_MAX_FILES];
  for (int f = 0; f < 2; ++f) {
    const std::string path = dir + "/hostio_" + std::to_string(f) + ".bin";
    if (!write_file(path, f)) return 3;
    int fd = direct ? open(path.c_str(), O_RDONLY | O_DIRECT) : -1;
    files[f].direct = fd >= 0;
    if (fd < 0) fd = open(path.c_str(), O_RDONLY);
    if (fd < 0) return 3;
    files[f].open = true;
    files[f].size = kSizes[f];
    files[f].fd.store(fd);
  }
  gfs_hostio::HostIo io;
  io.rpc_slots = slots;
  io.host_threads = threads;
  io.io_backend = backend;
  io.io_depth = depth;
  io.io_chunk_bytes = chunk_kib << 10;          // pieces smaller than a request: several threads per request
  io.min_piece_bytes = min_piece_kib << 10;
  io.max_req_bytes = kMaxPages * kPage;
  io.ring = (gfs_rpc_slot*)aligned_alloc(128, sizeof(gfs_rpc_slot) * slots);
  io.staging = (uint8_t*)aligned_alloc(4096, io.max_req_bytes * slots);
  io.files = files;
  if (!io.ring || !io.staging || io.init() != 0) return 4;
  memset(io.ring, 0, sizeof(gfs_rpc_slot) * slots);
  Shared sh;
  sh.io = &io;
  sh.slot_free.assign(slots, 0);
  sh.slot_tail.assign(slots, 0);
  gfs_hostio::start_threads(&io);
  std::vector<std::thread> ps;
  for (int i = 0; i < producers; ++i) ps.emplace_back(producer, &sh, i, nreq, backend == GFS_IO_PREAD_PARTITIONED);
  for (auto& t : ps) t.join();
  gfs_hostio::stop_threads(&io);
  const uint64_t want = (uint64_t)producers * nreq;
  uint64_t served = 0;
  for (uint32_t i = 0; i < threads; ++i) served += io.thread_requests[i].load();
  // host_errors counts failed reads, one per piece of a failed request
  const bool ok = sh.failures == 0 && sh.requests == want && io.host_requests.load() == want && served == want &&
                  io.host_bytes.load() == sh.bytes.load() && io.host_errors.load() >= sh.ebadf.load() &&
                  (sh.ebadf == 0 || io.host_last_errno.load() == EBADF);
  printf("requests %llu of %llu, bytes %llu, ebadf %llu, short %llu, failures %llu, host_requests %llu, "
         "host_errors %llu, pieces %llu, direct %d -> %s\n",
         (unsigned long long)sh.requests.load(), (unsigned long long)want, (unsigned long long)sh.bytes.load(),
         (unsigned long long)sh.ebadf.load(), (unsigned long long)sh.short_reads.load(),
         (unsigned long long)sh.failures.load(), (unsigned long long)io.host_requests.load(),
         (unsigned long long)io.host_errors.load(), (unsigned long long)io.host_pieces.load(),
         files[0].direct ? 1 : 0, ok ? "ok" : "FAILED");
  for (int f = 0; f < 2; ++f) close(files[f].fd.load());
  free(io.ring);
  free(io.staging);
  return ok ? 0 : 1;
}
