/* Multi-threaded writer of a SplitMix64 stream file (the synthetic input files).
 *
 * Byte o of the file is byte (o mod 8), little-endian, of output number o/8+1 of
 * SplitMix64 with the given seed (Steele, Lea and Flood 2014). The last output is
 * truncated to the file size. Writes with pwrite from T threads in 8 MiB pieces,
 * fsyncs, then drops the file from the host page cache (POSIX_FADV_DONTNEED).
 *
 * usage: genfile PATH SEED SIZE_BYTES [THREADS]
 */
#define _GNU_SOURCE
#include <errno.h>
#include <fcntl.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define PIECE (8u << 20)

static uint64_t mix(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

typedef struct {
  int fd;
  uint64_t seed, size;
  int tid, nthr;
  int err;
} job_t;

static void* worker(void* arg) {
  job_t* j = (job_t*)arg;
  uint64_t* buf = (uint64_t*)malloc(PIECE);
  if (!buf) { j->err = ENOMEM; return NULL; }
  uint64_t npieces = (j->size + PIECE - 1) / PIECE;
  for (uint64_t p = (uint64_t)j->tid; p < npieces; p += (uint64_t)j->nthr) {
    uint64_t off = p * (uint64_t)PIECE;
    uint64_t len = j->size - off < PIECE ? j->size - off : PIECE;
    uint64_t k0 = off / 8 + 1; /* PIECE is a multiple of 8 */
    uint64_t nw = (len + 7) / 8;
    for (uint64_t i = 0; i < nw; i++) {
      uint64_t w = mix(j->seed + (k0 + i) * 0x9E3779B97F4A7C15ull);
      unsigned char* b = (unsigned char*)&buf[i];
      for (int t = 0; t < 8; t++) b[t] = (unsigned char)(w >> (8 * t)); /* little-endian */
    }
    uint64_t done = 0;
    while (done < len) {
      ssize_t r = pwrite(j->fd, (char*)buf + done, len - done, (off_t)(off + done));
      if (r < 0) { if (errno == EINTR) continue; j->err = errno; free(buf); return NULL; }
      done += (uint64_t)r;
    }
  }
  free(buf);
  return NULL;
}

int main(int argc, char** argv) {
  if (argc < 4) { fprintf(stderr, "usage: %s PATH SEED SIZE [THREADS]\n", argv[0]); return 2; }
  const char* path = argv[1];
  uint64_t seed = strtoull(argv[2], NULL, 0);
  uint64_t size = strtoull(argv[3], NULL, 0);
  int nthr = argc > 4 ? atoi(argv[4]) : 8;
  if (nthr < 1) nthr = 1;
  if (nthr > 64) nthr = 64;
  char tmp[4096];
  if (snprintf(tmp, sizeof tmp, "%s.tmp%d", path, (int)getpid()) >= (int)sizeof tmp) return 2;
  int fd = open(tmp, O_CREAT | O_TRUNC | O_WRONLY, 0644);
  if (fd < 0) { fprintf(stderr, "genfile: open %s: %s\n", tmp, strerror(errno)); return 1; }
  if (size && ftruncate(fd, (off_t)size) != 0) { fprintf(stderr, "genfile: ftruncate: %s\n", strerror(errno)); close(fd); unlink(tmp); return 1; }
  pthread_t th[64];
  job_t jobs[64];
  for (int i = 0; i < nthr; i++) {
    jobs[i] = (job_t){fd, seed, size, i, nthr, 0};
    pthread_create(&th[i], NULL, worker, &jobs[i]);
  }
  int err = 0;
  for (int i = 0; i < nthr; i++) { pthread_join(th[i], NULL); if (jobs[i].err) err = jobs[i].err; }
  if (!err && fsync(fd) != 0) err = errno;
  if (!err) posix_fadvise(fd, 0, 0, POSIX_FADV_DONTNEED);
  close(fd);
  if (err) { fprintf(stderr, "genfile: write: %s\n", strerror(err)); unlink(tmp); return 1; }
  if (rename(tmp, path) != 0) { fprintf(stderr, "genfile: rename: %s\n", strerror(errno)); unlink(tmp); return 1; }
  return 0;
}
