// CPU thread model of the device's page-fill protocol, on the library's real layout
// (gfs_layout.h: frame-word bits, the request record gfs_req_dev, the ring slot gfs_rpc_slot),
// built with g++ and run under ThreadSanitizer by the CPU tests. Host threads stand in for GPU
// blocks; one more thread stands in for the host I/O threads. The steps restate the device
// code's atomics with the same orderings, so that a protocol mistake (a frame published twice,
// a slot freed early or never, a helper copying another generation's bytes, a wait that never
// ends) shows up here as a failed check, a data race or a deadline, not on the GPU.
//
// Modes:
//   sync    the synchronous path: a requester takes frames (FILLING, pinned for its demanded
//           page) and shows them to readers, waits for its ring slot's previous generation to
//           be free, posts, waits for the host, publishes the request record, claims the frames
//           no helper has claimed (PULL bit, only while the frame's fill word names the
//           request), copies them from staging, publishes them VALID and counts them off; the
//           block that counts off the last frame frees the slot. Other blocks join frames of
//           the request and, once the record is ready, claim and copy their own.
//   async   mixed: every other request of a block is an asynchronous window. A window takes one
//           of the slots kept for windows without waiting (or is dropped), and its poster does
//           not wait: joiners see the host's completion in the ring slot itself and copy their
//           own frames; some windows lie ahead of every reader (nobody joins them); the poster
//           finishes its window before it posts again, accepting any later generation of the
//           slot (helpers may have published the whole window, and the slot moved on).
//   reserve the lock-free reservation of a page-table entry for a one-page miss: many blocks
//           race to reserve one key in its two 16-entry buckets; after every round exactly one
//           reservation is left.
// Planted mistakes, each of which the deadlines must catch:
//   async-shared-slots  windows take ticketed slots of the shared ring: a requester waits for
//           a slot held by a window that lies ahead of the readers while its poster waits on the
//           requester's own page (the stall seen on the GPU before windows got slots of their
//           own).
//   async-exact-gen     the poster waits for its slot's completion to equal its window's
//           generation; once helpers have published the whole window the slot has moved on and
//           that wait never ends.
// Frame pressure: the frame pool is small, so requesters wait for frames that other requests'
// readers must first let go of.
//
// usage: fill_protocol_model MODE BLOCKS REQUESTS FRAMES SLOTS PAGES
// prints one summary line ending in "-> ok" when every check held; exit status 0.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "gfs_layout.h"

namespace {

constexpr uint64_t kPage = 4096;
double kDeadlineS = 60.0;   // FPM_DEADLINE_S overrides
bool g_planted_shared = false;      // mode "async-shared-slots": a planted protocol mistake
bool g_planted_exact_gen = false;   // mode "async-exact-gen": another one

// ---- atomics with the device's orderings (agent scope -> plain C++ atomics here). The
// device polls with relaxed loads and takes one acquire fence when it sees the awaited value;
// ThreadSanitizer does not follow standalone fences, so the model polls with acquire loads,
// which order the same accesses.
uint64_t ld_rlx(uint64_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
uint64_t ld_acq(uint64_t* p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
void st_rel(uint64_t* p, uint64_t v) { __atomic_store_n(p, v, __ATOMIC_RELEASE); }
void st_rlx(uint64_t* p, uint64_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
bool cas(uint64_t* p, uint64_t& e, uint64_t d) {
  return __atomic_compare_exchange_n(p, &e, d, false, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE);
}
bool cas_rlx(uint64_t* p, uint64_t& e, uint64_t d) {
  return __atomic_compare_exchange_n(p, &e, d, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

std::atomic<int> g_fail{0};
std::mutex g_msg_mu;
void fail(const std::string& m) {
  std::lock_guard<std::mutex> g(g_msg_mu);
  if (g_fail.fetch_add(1) < 5) fprintf(stderr, "FAIL: %s\n", m.c_str());
}
void nap() { std::this_thread::yield(); }

// ---- the shared state, laid out as the library lays it out
struct Model {
  uint32_t nframes, nslots, pages, blocks;
  std::vector<uint64_t> fword, ffill, slot_free, frame_gen_pub;   // frame_gen_pub: checks only
  std::vector<gfs_req_dev> reqd;
  std::vector<gfs_rpc_slot> ring;
  std::vector<uint8_t> frames, staging;
  std::vector<uint64_t> ticket_of_frame;   // the frame's tag: the request its bytes come from
  uint64_t ring_tail = 0;
  std::vector<uint64_t> free_frames;       // frame pool (a stack under a lock: the clock's role)
  std::mutex pool_mu;
  std::atomic<uint64_t> published{0}, freed_slots{0}, joined{0}, helped{0}, posted{0}, dropped{0};
  std::atomic<bool> stop{false};
  uint64_t next_id = 0;            // request ids (the frames' tags)
  uint64_t async_base = 0, async_next = 0;   // frames of asynchronous windows
  uint32_t nsync = 0;              // slots [0, nsync) take ticketed requests
  bool async = false;

  Model(uint32_t b, uint32_t f, uint32_t s, uint32_t p)
      : nframes(f), nslots(s), pages(p), blocks(b), fword(f, 0), ffill(f, 0), slot_free(s, 0),
        frame_gen_pub(f, 0), reqd(s), ring(s), frames((uint64_t)f * kPage), staging((uint64_t)s * p * kPage),
        ticket_of_frame(f, 0) {
    memset(reqd.data(), 0, sizeof(gfs_req_dev) * s);
    memset(ring.data(), 0, sizeof(gfs_rpc_slot) * s);
    for (uint32_t i = 0; i < f; ++i) free_frames.push_back(i);
  }
  // bytes the host writes for page k of request ticket tk
  static uint8_t byte(uint64_t tk, uint32_t k, uint64_t i) { return (uint8_t)(tk * 131u + k * 29u + i * 7u + 1); }
};

// ---- the host: serve posted requests in ring order (any slot), fill staging, publish done
void host_thread(Model* M) {
  std::vector<uint64_t> seen(M->nslots, 0);
  const double t0 = now_s();
  while (!M->stop.load()) {
    bool any = false;
    for (uint32_t s = 0; s < M->nslots; ++s) {
      gfs_rpc_slot* rs = &M->ring[s];
      const uint64_t g = __atomic_load_n(&rs->req_seq, __ATOMIC_ACQUIRE);
      if (g == 0 || g == seen[s]) continue;
      seen[s] = g;
      uint8_t* st = M->staging.data() + (uint64_t)s * M->pages * kPage;
      for (uint32_t k = 0; k < rs->npages; ++k)
        for (uint64_t i = 0; i < kPage; ++i) st[k * kPage + i] = Model::byte(rs->ticket, k, i);
      rs->result = (int64_t)(rs->npages * kPage);
      __atomic_store_n(&rs->done_seq, g, __ATOMIC_RELEASE);
      any = true;
    }
    if (!any) nap();
    if (now_s() - t0 > 4 * kDeadlineS) {
      fail("host: deadline");
      return;
    }
  }
}

// ---- device steps, restated
void publish_frame(Model* M, uint32_t f) {
  uint64_t w = ld_rlx(&M->fword[f]);
  while (true) {
    const uint64_t nw = ((w & ~(GFS_FW_STATE | GFS_FW_PULL)) | GFS_FS_VALID | GFS_FW_REF) + GFS_FW_VER_ONE;
    if (cas(&M->fword[f], w, nw)) break;
  }
  M->published++;
}
void request_done(Model* M, uint32_t s, uint64_t gen, uint32_t cnt) {
  if (cnt == 0) return;
  const uint32_t before = __atomic_fetch_sub(&M->reqd[s].remaining, cnt, __ATOMIC_ACQ_REL);
  if (before < cnt) fail("request counted off below zero");
  if (before == cnt) {
    if (ld_rlx(&M->slot_free[s]) != gen - 1) fail("slot freed out of order");
    st_rel(&M->slot_free[s], gen);
    if (s >= M->nsync) st_rel(&M->reqd[s].busy, 0ull);   /* a window's slot */
    M->freed_slots++;
  }
}
void copy_page(Model* M, uint32_t f, uint32_t s, uint32_t k) {
  memcpy(M->frames.data() + (uint64_t)f * kPage, M->staging.data() + ((uint64_t)s * M->pages + k) * kPage, kPage);
}
void check_page(Model* M, uint32_t f, uint64_t tk, uint32_t k, const char* who) {
  const uint8_t* p = M->frames.data() + (uint64_t)f * kPage;
  for (uint64_t i = 0; i < kPage; i += 509)
    if (p[i] != Model::byte(tk, k, i)) {
      fail(std::string(who) + ": wrong bytes in a frame");
      return;
    }
}

// a joiner: pinned frame f (page k of the request with ticket tk); wait for VALID, helping
// when the request's bytes are staged. Returns false on deadline.
bool join_or_help(Model* M, uint32_t f, uint32_t k, uint64_t tk) {
  const double t0 = now_s();
  while (true) {
    uint64_t w = ld_acq(&M->fword[f]);
    if ((w & GFS_FW_STATE) == GFS_FS_VALID) {
      check_page(M, f, tk, k, "joiner");
      return true;
    }
    if (!(w & GFS_FW_PULL)) {
      const uint64_t ff = ld_rlx(&M->ffill[f]);
      uint32_t s = 0;
      uint64_t gen = 0;
      bool ready = false;
      if (ff >> 63) {   // asynchronous: the host's completion in the ring slot itself
        s = (uint32_t)((ff >> 40) & 0x7fffff) - 1;
        gen = ff & ((1ull << 40) - 1);
        ready = __atomic_load_n(&M->ring[s].done_seq, __ATOMIC_ACQUIRE) == gen;
      } else if (ff) {
        s = (uint32_t)(ff >> 40) - 1;
        gen = ff & ((1ull << 40) - 1);
        const uint64_t r = ld_acq(&M->reqd[s].ready);
        ready = r != 0 && (r & ((1ull << 40) - 1)) == gen;
      }
      if (ready) {
        if (cas(&M->fword[f], w, (w | GFS_FW_PULL) + GFS_FW_VER_ONE)) {
          copy_page(M, f, s, k);
          publish_frame(M, f);   /* a release compare-and-swap */
          request_done(M, s, gen, 1);
          M->helped++;
          continue;
        }
        continue;
      }
    }
    if (now_s() - t0 > kDeadlineS) {
      fail("joiner: deadline");
      return false;
    }
    nap();
  }
}

struct Posted {
  uint32_t slot = 0, n = 0;
  uint64_t gen = 0, tk = 0;   // tk: the request's id (the frames' tag)
  bool async = false;
  uint32_t frames[64];
};

uint64_t fill_of(const Posted& q) {
  return (q.async ? (1ull << 63) : 0ull) | ((uint64_t)(q.slot + 1) << 40) | (q.gen & ((1ull << 40) - 1));
}

// the poster's part after the host is done: publish (sync), claim the rest, copy, publish.
// The slot's generations only grow: done_seq past the request's generation means helpers
// published every frame and the slot went to a later request, so nothing is left to claim.
void finish(Model* M, Posted& q, bool publish_record) {
  gfs_rpc_slot* rs = &M->ring[q.slot];
  const double t0 = now_s();
  uint64_t ds;
  while (true) {
    ds = __atomic_load_n(&rs->done_seq, __ATOMIC_ACQUIRE);
    if (g_planted_exact_gen ? ds == q.gen : (int64_t)(ds - q.gen) >= 0) break;
    if (now_s() - t0 > kDeadlineS) {
      fail("poster: host deadline");
      return;
    }
    nap();
  }
  if (ds != q.gen) return;   /* moved on: every frame was published by helpers */
  if (publish_record) {
    gfs_req_dev* r = &M->reqd[q.slot];
    r->result = rs->result;
    r->first_page = 0;
    __atomic_store_n(&r->remaining, q.n, __ATOMIC_RELAXED);
    st_rel(&r->ready, q.gen);
  }
  const uint64_t fill = fill_of(q);
  uint32_t claimed[64], nc = 0;
  for (uint32_t k = 0; k < q.n; ++k) {
    const uint32_t f = q.frames[k];
    uint64_t w = ld_acq(&M->fword[f]);
    while ((w & GFS_FW_STATE) == GFS_FS_FILLING && !(w & GFS_FW_PULL) && ld_rlx(&M->ffill[f]) == fill)
      if (cas(&M->fword[f], w, (w | GFS_FW_PULL) + GFS_FW_VER_ONE)) {
        claimed[nc++] = k;
        break;
      }
  }
  for (uint32_t c = 0; c < nc; ++c) copy_page(M, q.frames[claimed[c]], q.slot, claimed[c]);
  for (uint32_t c = 0; c < nc; ++c) publish_frame(M, q.frames[claimed[c]]);
  request_done(M, q.slot, q.gen, nc);
}

// board entry of page k of request tk: ((tk << 20 | frame) << 8 | k) << 1 | 1
void advertise(Model* M, const Posted& q, std::vector<std::atomic<uint64_t>>* board) {
  for (uint32_t k = 0; k < q.n; ++k)
    (*board)[(q.tk * M->pages + k) % board->size()].store(((q.tk << 20 | q.frames[k]) << 8 | k) << 1 | 1,
                                                            std::memory_order_release);
}

// pin frame f if it still holds page k of request tk, wait for it (helping), unpin
void join_frame(Model* M, uint32_t f, uint32_t k, uint64_t tk) {
  uint64_t w = __atomic_fetch_add(&M->fword[f], GFS_FW_PIN_ONE, __ATOMIC_ACQUIRE);
  const uint64_t st = w & GFS_FW_STATE;
  if ((st == GFS_FS_FILLING || st == GFS_FS_VALID) && ld_rlx(&M->ticket_of_frame[f]) == tk) {
    M->joined++;
    join_or_help(M, f, k, tk);
  }
  __atomic_fetch_sub(&M->fword[f], GFS_FW_PIN_ONE, __ATOMIC_RELAXED);
}

// join a few frames of other blocks' requests on the board, as a block whose access finds a
// frame being filled does
void join_some(Model* M, std::mt19937_64& rng, std::vector<std::atomic<uint64_t>>* board) {
  for (int j = 0; j < 3; ++j) {
    const uint64_t v = (*board)[rng() % board->size()].load(std::memory_order_acquire);
    if (v & 1) join_frame(M, (uint32_t)((v >> 9) & 0xfffff), (uint32_t)((v >> 1) & 0xff), v >> 29);
  }
}

// join every frame of request tk that the board still shows
void join_ticket(Model* M, uint64_t tk, std::vector<std::atomic<uint64_t>>* board) {
  for (uint32_t k = 0; k < M->pages; ++k) {
    const uint64_t v = (*board)[(tk * M->pages + k) % board->size()].load(std::memory_order_acquire);
    if ((v & 1) && (v >> 29) == tk) join_frame(M, (uint32_t)((v >> 9) & 0xfffff), k, tk);
  }
}

// one block: REQUESTS requests of PAGES pages each. Mode sync: every request synchronous.
// Mixed modes: every other request is an asynchronous window. Synchronous requests take
// frames from the small pool and show them to readers before they get a slot (as the device
// reserves pages before posting); asynchronous windows take frames of their own.
void block_thread(Model* M, uint32_t b, uint32_t nreq, std::vector<std::atomic<uint64_t>>* board) {
  std::mt19937_64 rng(1000 + b);
  Posted pend;
  bool has_pend = false;
  for (uint32_t r = 0; r < nreq && !g_fail.load(); ++r) {
    const bool do_async = M->async && (r & 1);
    // a block that waits for its own synchronous request joins nothing meanwhile; between
    // requests it reads other blocks' pages like any reader
    if (!M->async) join_some(M, rng, board);
    // a poster finishes its outstanding asynchronous window before it posts again
    if (has_pend) {
      finish(M, pend, false);
      has_pend = false;
    }
    Posted q;
    q.n = M->pages;
    q.async = do_async;
    q.tk = __atomic_fetch_add(&M->next_id, 1, __ATOMIC_RELAXED);
    if (do_async) {
      const uint64_t base = M->async_base + __atomic_fetch_add(&M->async_next, q.n, __ATOMIC_RELAXED);
      for (uint32_t k = 0; k < q.n; ++k) q.frames[k] = (uint32_t)(base + k);
    } else {
      const double tf = now_s();
      while (true) {
        {
          std::lock_guard<std::mutex> g(M->pool_mu);
          if (M->free_frames.size() >= q.n) {
            for (uint32_t k = 0; k < q.n; ++k) {
              q.frames[k] = (uint32_t)M->free_frames.back();
              M->free_frames.pop_back();
            }
            break;
          }
        }
        if (now_s() - tf > kDeadlineS) {
          fail("no frames: deadline");
          return;
        }
        nap();
      }
    }
    // CLAIMED -> FILLING, version + 1, the tag (a synchronous request's demanded page, k = 0,
    // pinned by its poster); the fill word is not known yet. An addition, as on the device:
    // a reader holding a stale pin on the frame keeps it (it drops the pin after seeing that
    // the tag is not its page)
    for (uint32_t k = 0; k < q.n; ++k) {
      const uint32_t f = q.frames[k];
      st_rlx(&M->ffill[f], 0ull);
      st_rlx(&M->ticket_of_frame[f], q.tk);
      const uint64_t delta = (GFS_FS_FILLING - GFS_FS_CLAIMED) + GFS_FW_VER_ONE +
                             ((!do_async && k == 0) ? GFS_FW_PIN_ONE : 0);
      __atomic_fetch_add(&M->fword[f], delta, __ATOMIC_RELEASE);
    }
    if (!do_async) advertise(M, q, board);
    if (do_async && !g_planted_shared) {
      // a slot of the windows' own, taken without waiting; none free: the window is dropped
      int32_t s = -1;
      const uint32_t A = M->nslots - M->nsync;
      for (uint32_t i = 0; i < A && s < 0; ++i) {
        const uint32_t c = M->nsync + (b + i) % A;
        uint64_t z = 0;
        if (ld_rlx(&M->reqd[c].busy) == 0 && cas(&M->reqd[c].busy, z, 1ull)) s = (int32_t)c;
      }
      if (s < 0) {
        M->dropped++;
        continue;   /* its frames were never shown to anyone */
      }
      q.slot = (uint32_t)s;
      q.gen = ld_acq(&M->slot_free[q.slot]) + 1;
    } else {
      // ticketed: wait for the slot's previous generation to be free
      const uint64_t t = __atomic_fetch_add(&M->ring_tail, 1, __ATOMIC_RELAXED);
      q.slot = (uint32_t)(t % M->nsync);
      q.gen = t / M->nsync + 1;
      const double ts = now_s();
      while (ld_acq(&M->slot_free[q.slot]) != q.gen - 1) {
        if (now_s() - ts > kDeadlineS) {
          fail("slot: deadline");
          return;
        }
        nap();
      }
    }
    if (do_async) __atomic_store_n(&M->reqd[q.slot].remaining, q.n, __ATOMIC_RELAXED);
    const uint64_t fill = fill_of(q);
    for (uint32_t k = 0; k < q.n; ++k) st_rel(&M->ffill[q.frames[k]], fill);
    // windows that readers reach soon are shown to them (in the mode with adversarial readers,
    // all of them); the rest lie ahead of every reader, like a readahead window
    if (do_async && (g_planted_exact_gen || (rng() & 1))) advertise(M, q, board);
    gfs_rpc_slot* rs = &M->ring[q.slot];
    rs->npages = q.n;
    rs->ticket = q.tk;
    __atomic_store_n(&rs->req_seq, q.gen, __ATOMIC_RELEASE);
    M->posted++;
    if (do_async) {
      pend = q;
      has_pend = true;
      // a block with a window outstanding reads on: it joins frames of others, and in the
      // adversarial mode every frame of the request before its own
      join_some(M, rng, board);
      if (g_planted_exact_gen) {
        // adversarial readers: the poster's own reads reach the whole window, and other
        // windows take its slot before the poster comes back to it
        join_ticket(M, q.tk, board);
        std::this_thread::sleep_for(std::chrono::milliseconds(2));
      }
      continue;
    }
    finish(M, q, true);
    // the demanded page: pulled here or by a helper; wait for it, read it, unpin
    if (join_or_help(M, q.frames[0], 0, q.tk))
      __atomic_fetch_sub(&M->fword[q.frames[0]], GFS_FW_PIN_ONE, __ATOMIC_RELAXED);
    // give back the frames of this block's completed request once nobody pins them (the clock
    // reclaims only unpinned VALID frames)
    for (uint32_t k = 0; k < q.n; ++k) {
      const uint32_t f = q.frames[k];
      const double tr = now_s();
      while (true) {
        uint64_t w = ld_rlx(&M->fword[f]);
        if ((w & GFS_FW_STATE) == GFS_FS_VALID && !(w & GFS_FW_PINS)) {
          const uint64_t claimed = (((w >> GFS_FW_VER_SHIFT) + 1) << GFS_FW_VER_SHIFT) | GFS_FS_CLAIMED;
          if (cas(&M->fword[f], w, claimed)) break;
          continue;
        }
        if (now_s() - tr > kDeadlineS) {
          fail("reclaim: deadline (frame word " + std::to_string(w) + ")");
          return;
        }
        nap();
      }
      std::lock_guard<std::mutex> g(M->pool_mu);
      M->free_frames.push_back(f);
    }
  }
  if (has_pend) finish(M, pend, false);
}

int run_fill(bool async, uint32_t blocks, uint32_t nreq, uint32_t nframes, uint32_t nslots, uint32_t pages) {
  Model M(blocks, nframes, nslots, pages);
  M.async = async;
  // asynchronous windows: a quarter of the slots (at least one) of their own, and frames past
  // the pool (never given back in this model)
  M.nsync = async && !g_planted_shared ? nslots - std::max(1u, nslots / 4) : nslots;
  M.async_base = nframes;
  const uint64_t extra = async ? (uint64_t)blocks * nreq * pages : 0;
  M.frames.assign((nframes + extra) * kPage, 0);
  M.fword.assign(nframes + extra, GFS_FS_CLAIMED);   // every frame starts owned by the pool
  M.ffill.assign(nframes + extra, 0);
  M.ticket_of_frame.assign(nframes + extra, 0);
  std::vector<std::atomic<uint64_t>> board(256);
  for (auto& x : board) x.store(0);
  const uint64_t total = (uint64_t)blocks * nreq;
  std::thread host(host_thread, &M);
  std::vector<std::thread> ts;
  for (uint32_t b = 0; b < blocks; ++b) ts.emplace_back(block_thread, &M, b, nreq, &board);
  for (auto& t : ts) t.join();
  M.stop.store(true);
  host.join();
  // every posted request's frames published exactly once, every slot generation freed
  const uint64_t posted = M.posted.load();
  if (posted + M.dropped.load() != total) fail("requests posted " + std::to_string(posted));
  if (M.published.load() != posted * pages)
    fail("published " + std::to_string(M.published.load()) + " frames, want " + std::to_string(posted * pages));
  if (M.freed_slots.load() != posted) fail("slots freed " + std::to_string(M.freed_slots.load()));
  uint64_t gens = 0;
  for (uint32_t s = 0; s < nslots; ++s) {
    gens += M.slot_free[s];
    if (s >= M.nsync && M.reqd[s].busy) fail("a window's slot is still held");
  }
  if (gens != posted) fail("slot generations " + std::to_string(gens) + " for " + std::to_string(posted) + " requests");
  printf("%s blocks=%u requests=%u frames=%u slots=%u pages=%u posted=%llu dropped=%llu joined=%llu helped=%llu -> %s\n",
         async ? "mixed" : "sync", blocks, nreq, nframes, nslots, pages, (unsigned long long)posted,
         (unsigned long long)M.dropped.load(), (unsigned long long)M.joined.load(), (unsigned long long)M.helped.load(),
         g_fail.load() ? "FAILED" : "ok");
  return g_fail.load() ? 1 : 0;
}

// ---- the one-page reservation without the lock (reserve_unique_wave), 32 "lanes" serial
struct Table {
  uint64_t e[32];
};
int64_t reserve_unique(Table* t, uint64_t key) {
  const uint64_t ent = (key << GFS_ENTRY_FRAME_BITS) | ((1ull << GFS_ENTRY_FRAME_BITS) - 1);
  for (int attempt = 0; attempt < 64; ++attempt) {
    uint64_t e[32];
    for (int i = 0; i < 32; ++i) e[i] = ld_rlx(&t->e[i]);
    for (int i = 0; i < 32; ++i)
      if ((e[i] >> GFS_ENTRY_FRAME_BITS) == key) return -1;
    int used1 = 0, used2 = 0, f1 = -1, f2 = -1;
    for (int i = 0; i < 16; ++i) {
      if (e[i]) ++used1;
      else if (f1 < 0) f1 = i;
      if (e[16 + i]) ++used2;
      else if (f2 < 0) f2 = 16 + i;
    }
    int pick = used2 < used1 ? f2 : f1;
    if (pick < 0) pick = f1 >= 0 ? f1 : f2;
    if (pick < 0) return -2;
    uint64_t z = 0;
    if (!cas_rlx(&t->e[pick], z, ent)) continue;
    // the device waits for the swap to be performed before it looks again (s_waitcnt on the
    // returned atomic); a sequentially consistent fence is the CPU's equivalent
    std::atomic_thread_fence(std::memory_order_seq_cst);
    for (int i = 0; i < 32; ++i) {
      if (i == pick) continue;
      if ((ld_rlx(&t->e[i]) >> GFS_ENTRY_FRAME_BITS) == key) {
        uint64_t x = ent;
        cas_rlx(&t->e[pick], x, 0);
        return -1;
      }
    }
    return pick;
  }
  return -2;
}

int run_reserve(uint32_t blocks, uint32_t rounds) {
  Table t;
  std::atomic<uint32_t> go{0}, done{0};
  std::atomic<int> kept{0};
  uint64_t withdrawn_all = 0;
  std::mt19937_64 rng(7);
  for (uint32_t r = 0; r < rounds && !g_fail.load(); ++r) {
    // other keys fill part of both buckets
    for (int i = 0; i < 32; ++i) t.e[i] = (rng() % 3 == 0) ? ((((uint64_t)(1000 + i)) << GFS_ENTRY_FRAME_BITS) | 5) : 0;
    const uint64_t key = 77 + r;
    kept.store(0);
    int total_kept = 0;
    // until someone keeps a reservation (all may withdraw in a round)
    for (int pass = 0; pass < 100 && total_kept == 0; ++pass) {
      std::vector<std::thread> ts;
      for (uint32_t b = 0; b < blocks; ++b)
        ts.emplace_back([&]() {
          if (reserve_unique(&t, key) >= 0) kept++;
        });
      for (auto& x : ts) x.join();
      total_kept = kept.load();
      if (total_kept == 0) ++withdrawn_all;
    }
    int present = 0;
    for (int i = 0; i < 32; ++i)
      if ((t.e[i] >> GFS_ENTRY_FRAME_BITS) == key) ++present;
    if (total_kept != 1 || present != 1)
      fail("round " + std::to_string(r) + ": kept " + std::to_string(total_kept) + ", entries " + std::to_string(present));
  }
  (void)go;
  (void)done;
  printf("reserve blocks=%u rounds=%u all-withdrew=%llu -> %s\n", blocks, rounds, (unsigned long long)withdrawn_all,
         g_fail.load() ? "FAILED" : "ok");
  return g_fail.load() ? 1 : 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 7) {
    fprintf(stderr, "usage: %s MODE BLOCKS REQUESTS FRAMES SLOTS PAGES\n", argv[0]);
    return 2;
  }
  const std::string mode = argv[1];
  const uint32_t blocks = (uint32_t)atoi(argv[2]), nreq = (uint32_t)atoi(argv[3]), frames = (uint32_t)atoi(argv[4]),
                 slots = (uint32_t)atoi(argv[5]), pages = (uint32_t)atoi(argv[6]);
  if (const char* e = getenv("FPM_DEADLINE_S")) kDeadlineS = atof(e);
  if (mode != "reserve" && (pages == 0 || pages > 64 || blocks == 0 || slots == 0 || frames < pages)) return 2;
  if (mode == "sync") return run_fill(false, blocks, nreq, frames, slots, pages);
  if (const char* e = getenv("FPM_DEADLINE_S")) kDeadlineS = atof(e);
  if (mode == "async") return run_fill(true, blocks, nreq, frames, slots, pages);
  if (mode == "async-shared-slots") {
    g_planted_shared = true;
    return run_fill(true, blocks, nreq, frames, slots, pages);
  }
  if (mode == "async-exact-gen") {
    g_planted_exact_gen = true;
    return run_fill(true, blocks, nreq, frames, slots, pages);
  }
  if (mode == "reserve") return run_reserve(blocks, nreq);
  return 2;
}
