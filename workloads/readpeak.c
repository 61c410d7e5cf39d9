/* Sequential-read throughput of a set of files: the storage bound the benchmarks divide by.
 *
 * T threads read the files back to back in CHUNK-byte pieces (piece i of the concatenated
 * files goes to thread i mod T), each into its own aligned buffer, with O_DIRECT where the
 * file system allows it (else buffered reads after dropping the file from the page
 * cache). Prints bytes read and seconds.
 *
 * usage: readpeak THREADS CHUNK_BYTES LIMIT_BYTES FILE...
 *        (LIMIT_BYTES caps the bytes read from each file; 0 = whole file)
 */
#define _GNU_SOURCE
#include <errno.h>
#include <fcntl.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <time.h>
#include <unistd.h>

typedef struct {
  int fd;
  uint64_t size;
  uint64_t first_piece;   /* index of the file's first piece in the concatenation */
} File;

static File* files;
static int nfiles;
static uint64_t chunk, total_pieces;
static int nthreads;
static uint64_t* got;

static void* worker(void* arg) {
  const int t = (int)(intptr_t)arg;
  void* buf = NULL;
  if (posix_memalign(&buf, 4096, chunk)) return NULL;
  int f = 0;
  for (uint64_t i = (uint64_t)t; i < total_pieces; i += (uint64_t)nthreads) {
    while (f + 1 < nfiles && files[f + 1].first_piece <= i) ++f;
    while (f > 0 && files[f].first_piece > i) --f;
    const uint64_t off = (i - files[f].first_piece) * chunk;
    const uint64_t want = files[f].size - off < chunk ? files[f].size - off : chunk;
    const uint64_t req = (want + 4095) & ~4095ull;   /* O_DIRECT wants whole blocks */
    ssize_t r;
    do {
      r = pread(files[f].fd, buf, req, (off_t)off);
    } while (r < 0 && errno == EINTR);
    if (r > 0) got[t] += (uint64_t)r < want ? (uint64_t)r : want;
  }
  free(buf);
  return NULL;
}

int main(int argc, char** argv) {
  if (argc < 5) {
    fprintf(stderr, "usage: readpeak THREADS CHUNK_BYTES LIMIT_BYTES FILE...\n");
    return 2;
  }
  nthreads = atoi(argv[1]);
  chunk = strtoull(argv[2], NULL, 10);
  const uint64_t limit = strtoull(argv[3], NULL, 10);
  nfiles = argc - 4;
  if (nthreads < 1 || nthreads > 256 || chunk < 4096 || chunk % 4096) {
    fprintf(stderr, "readpeak: bad thread count or chunk size\n");
    return 2;
  }
  files = calloc((size_t)nfiles, sizeof(File));
  got = calloc((size_t)nthreads, sizeof(uint64_t));
  if (!files || !got) return 1;
  for (int i = 0; i < nfiles; ++i) {
    const char* path = argv[4 + i];
    int fd = open(path, O_RDONLY | O_DIRECT);
    if (fd < 0) {
      fd = open(path, O_RDONLY);
      if (fd < 0) {
        perror(path);
        return 1;
      }
      posix_fadvise(fd, 0, 0, POSIX_FADV_DONTNEED);
    }
    struct stat st;
    if (fstat(fd, &st)) {
      perror(path);
      return 1;
    }
    files[i].fd = fd;
    files[i].size = limit && (uint64_t)st.st_size > limit ? limit : (uint64_t)st.st_size;
    files[i].first_piece = total_pieces;
    total_pieces += (files[i].size + chunk - 1) / chunk;
  }
  pthread_t* th = calloc((size_t)nthreads, sizeof(pthread_t));
  if (!th) return 1;
  struct timespec a, b;
  clock_gettime(CLOCK_MONOTONIC, &a);
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, worker, (void*)(intptr_t)t);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  clock_gettime(CLOCK_MONOTONIC, &b);
  uint64_t bytes = 0;
  for (int t = 0; t < nthreads; ++t) bytes += got[t];
  const double secs = (double)(b.tv_sec - a.tv_sec) + 1e-9 * (double)(b.tv_nsec - a.tv_nsec);
  printf("%llu %.6f\n", (unsigned long long)bytes, secs);
  for (int i = 0; i < nfiles; ++i) close(files[i].fd);
  return 0;
}
