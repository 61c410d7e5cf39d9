"""Step-by-step CPU model of the page cache, readahead detector and clock replacement.

Test infrastructure only (see the package docstring).

What the model follows:

* Sec. 2.2 (GPUfs read path): a threadblock's read is divided into pages; each
  page is looked up in the GPU page cache; a hit is served from the cache, a miss
  becomes a request to the host and the block waits for it.
* Sec. 4.1 (GPU-side mechanism, steps 2, 3, 6 and 7): on a miss the block asks
  the host for the missed page plus a prefetch window, and all of the window's
  pages are placed in the cache. The paper's window is static; the window here
  grows like the Linux readahead the paper describes in Sec. 2.3 (sequentiality
  detected per stream, several streams per file, size doubled on each sequential
  hit up to a maximum). A first read at offset 0 opens a window of ``W0`` pages,
  the Sec. 3.2 example (a 4 KB read at offset 0 prefetches 16 KB) with W0 = 4.
* Sec. 4 (read-only gating, fadvise hint): readahead is on only for read-only
  files and can be switched off per file with the RANDOM hint.
* Sec. 5.1 (replacement): frames are reused in place without being freed and
  re-allocated. The victim is chosen by clock (second chance) over a global
  hand; for read-once streams this evicts in allocation order, like the paper's
  least-recently-allocated queue (pinned in tests against ``oracle.lra``).

Readings where the paper is silent (the same list is in the design notes):
``cap`` below is the configured cap clipped by the thrash guard (``quota_cap``);
window = [s.next, s.next + min(2 s.size, cap)) for a stream s whose zone
[s.next, s.next + s.size) holds the missed page p (lowest slot wins); otherwise a
new stream replaces an empty slot or the least recently used one (lowest index
on ties): if at least ``near_min`` of the file's last ``recent`` misses lie within
``near_pages`` pages of p (defaults 3, 64, 64), many blocks are reading the file in aggregate
(interleaved strides) and the
window is the cap-sized chunk aligned around p; else [p, p + w) with w = min(max(2 h,
r), cap) if the h > r pages right before p are already cached (a history no longer
than the read may be chance next to a random read; h counted up to
max(ceil(cap / 2), r + 1), which decides the comparison and the window exactly; context
readahead: Linux's way of following readers that interleave on one descriptor, Sec.
2.3); else w = min(max(W0 if p == 0 or the file is SEQUENTIAL else 1, r), cap); r is
min(cap, the number of pages of the missing read from p to its end) (a prefetcher reads
at least what the caller asked for, Sec. 2.3). Windows are clamped to EOF; the
block fetches the run of unmapped window pages that contains p (pages beyond a
mapped page are left for later demand, so a request has no holes, and so are pages that
were consumed and then evicted since the cache was set up, unless the demanded page is
one of them: such a page lies behind a reader that has passed it, which is how a stream's
last window reaches into a neighbour's chunk, and a demanded page that is one of them
means the file is being read again; Sec. 5.1 counts prefetched pages evicted unused as
the waste to avoid); the demanded
page is allocated first, then the rest of the run in ascending order; one host
request covers the run; the prefetch is synchronous (the requester waits for the
whole window); a filled frame gets its reference bit set; a pin sets it and
clears the unconsumed-prefetch mark; the hand starts at frame 0, skips frames
that are filling or pinned, clears a set reference bit, and otherwise evicts.

Asynchronous readahead (``ra_async``; Sec. 2.3: Linux issues the next window while the
reader is still consuming the current one). Each decided window sets its stream's marker:
after a demand miss at p, the page p + 1 when the window fetched it; after an
asynchronous window, the window's first page. The marker page's frame carries a mark from
its allocation. A block whose access finds a marked frame (hit or join) clears the mark and,
if a stream's marker still names that page (lowest slot), advances that stream: window
[s.next, s.next + min(2 s.size, cap)), the run from its first page of pages that are
unmapped and, unless the marker page itself was, not consumed and evicted, allocated
ascending and requested from the host, with no page demanded and nobody waiting for it.
A block keeps at most one such request outstanding: it completes the previous one first,
when it reaches a marked page. In serialized runs every request completes by the end of
the read that issued it (the test harness waits for it there). An access that finds a page
still being filled (a later page of the same read, inside the block's own outstanding
request) joins it: the page is filled then.

Events produced (tuples; the GPU trace is decoded into the same vocabulary):

  ("HIT",  block, file, page, frame)
  ("JOIN", block, file, page, frame)          the frame was still being filled
  ("ADV",  block, file, page, ws, wn)         an asynchronous window, triggered at page
  ("MISS", block, file, page, ws, wn)          wn already clamped to EOF
  ("HAND", ticket, frame, action, vfile, vpage, vra, seen)
        action in FREE / SKIP / CLEAR / EVICT; victim fields are -1, -1, 0 unless EVICT;
        seen = what the hand found: ref | pinned << 1 | lost race << 2 | state << 3
        (state 0 free, 2 filling, 3 valid; the model never loses a race)
  ("ALLOC", file, page, frame, ra)             ra = 1 for prefetched (non-demand) pages
  ("REQ",  file, first_page, npages)           one host read of the allocated span
  ("NOFRAME", block, file, page)               no frame for a non-demand page: window cut
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Tuple

FREE, FILLING, VALID = "FREE", "FILLING", "VALID"
# Defaults of the aggregate-reading rule's constants (each is a model parameter):
RECENT = 64          # misses remembered per file
NEAR_MIN = 3         # remembered misses near p that make the file look read in aggregate
NEAR_PAGES = 64      # "near" = within NEAR_PAGES pages
ADV_NORMAL, ADV_SEQUENTIAL, ADV_RANDOM = "normal", "sequential", "random"
# which rule decided a window: readahead off, a stream's zone, aggregate reading, context
# (cached pages right behind p), a new stream (W0 or one page)
RULE_OFF, RULE_ZONE, RULE_AGGREGATE, RULE_CONTEXT, RULE_NEW = 0, 1, 2, 3, 4
# frame states as the trace reports them
STATE_CODE = {"FREE": 0, "FILLING": 2, "VALID": 3}


def quota_cap(cap: int, nframes: int, blocks: int, quota_blocks: int) -> int:
    """The largest window under the thrash guard: the cap, but at most one resident block's
    share of the cache (Sec. 5.1: the cache divided among the threadblocks reading at once,
    the smaller of the launch's blocks and quota_blocks)."""
    r = max(1, min(blocks, quota_blocks))
    return min(cap, max(1, nframes // r))


@dataclasses.dataclass
class Frame:
    state: str = FREE
    file: int = -1
    page: int = -1
    pins: int = 0
    ref: int = 0
    ra: int = 0
    mark: int = 0          # asynchronous readahead: the page is its stream's marker


@dataclasses.dataclass
class Stream:
    valid: bool = False
    next: int = 0
    size: int = 0
    last_use: int = 0
    marker: int = -1       # asynchronous readahead: the page whose access advances the stream


@dataclasses.dataclass
class FileState:
    size: int
    advice: str = ADV_NORMAL
    read_only: bool = True
    streams: List[Stream] = dataclasses.field(default_factory=list)
    clock: int = 0          # per-file count of readahead decisions (stream last_use)
    recent: List[int] = dataclasses.field(default_factory=list)   # the last misses (pages)


class PolicyModel:
    def __init__(self, nframes: int, page_size: int, ra_init_pages: int = 4,
                 ra_cap_pages: int = 0, streams_per_file: int = 8, recent: int = RECENT,
                 near_pages: int = NEAR_PAGES, near_min: int = NEAR_MIN, ra_async: bool = False):
        """ra_cap_pages is the cap after the thrash guard (see ``quota_cap``)."""
        if nframes <= 0 or page_size <= 0:
            raise ValueError("nframes and page_size must be positive")
        self.C = nframes
        self.P = page_size
        self.W0 = ra_init_pages
        self.cap = ra_cap_pages
        self.S = streams_per_file
        self.recent = recent
        self.near_pages = near_pages
        self.near_min = near_min
        self.ra_async = ra_async
        self.pending: Dict[int, List[int]] = {}   # block -> frames of its outstanding request
        self.frames = [Frame() for _ in range(nframes)]
        self.map: Dict[Tuple[int, int], int] = {}
        # (file, page) of every page evicted after it was consumed (a pin cleared its
        # prefetch mark, or it was demanded), since the cache was set up
        self.shadow = set()
        self.hand = 0
        self.files: Dict[int, FileState] = {}
        self.events: List[tuple] = []
        # per miss, in order: (near, h, rule) -- the detector's inputs and the rule it applied
        self.decisions: List[Tuple[int, int, int]] = []
        # counters
        self.hits = 0
        self.joins = 0
        self.advances = 0
        self.misses = 0
        self.evictions = 0
        self.fetched_pages = 0
        self.ra_pages = 0
        self.wasted_pages = 0
        self.fetched_bytes = 0
        self.wasted_bytes = 0
        self.requests = 0
        self.request_bytes = 0
        self.delivered_bytes = 0

    # ---- files ------------------------------------------------------------------------
    def open(self, file_id: int, size: int, advice: str = ADV_NORMAL, read_only: bool = True) -> None:
        self.files[file_id] = FileState(size=size, advice=advice, read_only=read_only,
                                        streams=[Stream() for _ in range(self.S)])

    def npages(self, file_id: int) -> int:
        return (self.files[file_id].size + self.P - 1) // self.P

    def page_bytes(self, file_id: int, page: int) -> int:
        return max(0, min(self.P, self.files[file_id].size - page * self.P))

    # ---- readahead decision (one per miss) -----------------------------------------------
    def ra_decide(self, file_id: int, p: int, req: int = 1) -> Tuple[int, int]:
        """The window for a demand miss at p, made by a read whose pages from p on are `req`;
        the stream it set is left in self.last_stream (None when readahead is off)."""
        fs = self.files[file_id]
        self.last_stream = None
        if self.cap == 0 or fs.advice == ADV_RANDOM or not fs.read_only:
            self.decisions.append((0, 0, RULE_OFF))
            return p, 1
        fs.clock += 1
        near = sum(1 for r in fs.recent if abs(r - p) <= self.near_pages)
        fs.recent.append(p)
        if len(fs.recent) > self.recent:
            fs.recent.pop(0)
        for s in fs.streams:                       # lowest slot index wins
            if s.valid and s.next <= p < s.next + s.size:
                ws = s.next
                wn = min(2 * s.size, self.cap)
                s.next = ws + wn
                s.size = wn
                s.last_use = fs.clock
                self.last_stream = s
                self.decisions.append((near, 0, RULE_ZONE))
                return ws, wn
        # context: the pages right behind p are already cached (read or being read by other
        # blocks), so p continues a sequential stream that no slot tracks; counted up to
        # max(ceil(cap / 2), r + 1), enough to compare with the read's r pages and to size
        # the window min(2 h, cap)
        r = min(req, self.cap)
        hmax = max((self.cap + 1) // 2, r + 1)
        h = 0
        while h < hmax and p - 1 - h >= 0 and (file_id, p - 1 - h) in self.map:
            h += 1
        victim = None
        for s in fs.streams:                       # an empty slot first (lowest index)
            if not s.valid:
                victim = s
                break
        if victim is None:                         # else least recently used, lowest index on ties
            victim = min(fs.streams, key=lambda s: s.last_use)
        if near >= self.near_min:
            # many blocks missing close together: the file is read in aggregate (interleaved
            # strides), take the whole cap-sized aligned chunk around p
            wn = self.cap
            ws = p // wn * wn
            self.decisions.append((near, 0, RULE_AGGREGATE))
        elif h > r:
            # a history longer than the read itself (a shorter one may be a random read next
            # to cached pages); at least the rest of the read that missed (Sec. 2.3: the
            # prefetcher reads more than the caller asked for, never less)
            wn = min(max(2 * h, r), self.cap)
            ws = p
            self.decisions.append((near, h, RULE_CONTEXT))
        else:
            wn = max(self.W0 if (p == 0 or fs.advice == ADV_SEQUENTIAL) else 1, r)
            ws = p
            self.decisions.append((near, h, RULE_NEW))
        wn = max(1, min(wn, self.cap))
        victim.valid = True
        victim.next = ws + wn
        victim.size = wn
        victim.last_use = fs.clock
        self.last_stream = victim
        return ws, wn

    # ---- clock ----------------------------------------------------------------------------
    def alloc(self) -> Optional[int]:
        for _ in range(2 * self.C):
            t = self.hand
            self.hand += 1
            f = t % self.C
            fr = self.frames[f]
            seen = fr.ref | (1 if fr.pins > 0 else 0) << 1 | STATE_CODE[fr.state] << 3
            if fr.state == FREE:
                self.events.append(("HAND", t, f, "FREE", -1, -1, 0, seen))
                return f
            if fr.state == FILLING or fr.pins > 0:
                self.events.append(("HAND", t, f, "SKIP", -1, -1, 0, seen))
                continue
            if fr.ref:
                fr.ref = 0
                self.events.append(("HAND", t, f, "CLEAR", -1, -1, 0, seen))
                continue
            # evict: unmap the old tag, reuse the frame in place
            self.events.append(("HAND", t, f, "EVICT", fr.file, fr.page, fr.ra, seen))
            del self.map[(fr.file, fr.page)]
            self.evictions += 1
            if fr.ra:
                self.wasted_pages += 1
                self.wasted_bytes += self.page_bytes(fr.file, fr.page)
            else:
                self.shadow.add((fr.file, fr.page))
            self.frames[f] = Frame()
            return f
        return None

    def _fetchable(self, file_id: int, q: int, p: int) -> bool:
        """May a window that page p opened fetch page q: q is not cached, and it was not
        consumed and then evicted, unless p was."""
        if (file_id, q) in self.map:
            return False
        return (file_id, q) not in self.shadow or (file_id, p) in self.shadow

    # ---- one page access ------------------------------------------------------------------
    def access(self, block: int, file_id: int, p: int, req: int = 1) -> int:
        """Serve page p of file_id for a block, as page 1 of the `req` pages from p to the end
        of the block's read; returns the frame (pinned, then unpinned)."""
        f = self.map.get((file_id, p))
        if f is not None:
            fr = self.frames[f]
            if fr.state == FILLING:
                # a page of the block's own outstanding request: wait for it, fill it
                self.joins += 1
                self.events.append(("JOIN", block, file_id, p, f))
                fr.state = VALID
                self.pending[block].remove(f)
            else:
                self.hits += 1
                self.events.append(("HIT", block, file_id, p, f))
            fr.pins += 1
            fr.ref = 1
            fr.ra = 0
            fr.pins -= 1
            if self.ra_async and fr.mark:
                fr.mark = 0
                self.advance(block, file_id, p)
            return f
        self.misses += 1
        ws, wn = self.ra_decide(file_id, p, req)
        wn = min(wn, self.npages(file_id) - ws)
        self.events.append(("MISS", block, file_id, p, ws, wn))
        marker = -1
        if self.ra_async and self.last_stream is not None:
            marker = p + 1 if p + 1 < ws + wn else -1
            self.last_stream.marker = marker
        # fetch the run of unmapped window pages that contains p (no holes in a request);
        # consumed-then-evicted pages end it too, unless p is one of them
        a = p
        while a - 1 >= ws and self._fetchable(file_id, a - 1, p):
            a -= 1
        b = p
        while b + 1 < ws + wn and self._fetchable(file_id, b + 1, p):
            b += 1
        order = [p] + [q for q in range(a, b + 1) if q != p]
        allocated = []
        for q in order:
            g = self.alloc()
            if g is None:
                if q == p:
                    raise RuntimeError("no frame for a demanded page: every frame pinned or filling")
                self.events.append(("NOFRAME", block, file_id, q))
                break
            fr = self.frames[g]
            fr.state = FILLING
            fr.file, fr.page = file_id, q
            fr.pins = 1 if q == p else 0
            fr.ref = 0
            fr.ra = 0 if q == p else 1
            fr.mark = 1 if q == marker else 0
            self.map[(file_id, q)] = g
            self.events.append(("ALLOC", file_id, q, g, fr.ra))
            allocated.append((q, g))
            self.fetched_pages += 1
            self.fetched_bytes += self.page_bytes(file_id, q)
            if q != p:
                self.ra_pages += 1
        first = min(q for q, _ in allocated)
        last = max(q for q, _ in allocated)
        self.events.append(("REQ", file_id, first, last - first + 1))
        self.requests += 1
        self.request_bytes += sum(self.page_bytes(file_id, q) for q in range(first, last + 1))
        # synchronous prefetch: the requester waits until the whole window is filled
        for q, g in allocated:
            fr = self.frames[g]
            fr.state = VALID
            fr.ref = 1
        fp = self.map[(file_id, p)]
        self.frames[fp].pins -= 1
        return fp

    # ---- asynchronous readahead ---------------------------------------------------------------
    def complete(self, block: int) -> None:
        """The block's outstanding asynchronous request arrives: its frames become valid."""
        for g in self.pending.pop(block, []):
            fr = self.frames[g]
            fr.state = VALID
            fr.ref = 1

    def advance(self, block: int, file_id: int, p: int) -> None:
        """A block reached marked page p: finish its own outstanding request, then, if a
        stream's marker still names p (lowest slot), issue that stream's next window."""
        self.complete(block)
        fs = self.files[file_id]
        s = next((t for t in fs.streams if t.valid and t.marker == p), None)
        if s is None:
            return
        fs.clock += 1
        ws = s.next
        wn = min(2 * s.size, self.cap)
        s.next = ws + wn
        s.size = wn
        s.last_use = fs.clock
        s.marker = ws
        wn = max(0, min(wn, self.npages(file_id) - ws))
        self.advances += 1
        self.events.append(("ADV", block, file_id, p, ws, wn))
        allocated = []
        q = ws
        while q < ws + wn and self._fetchable(file_id, q, p):
            g = self.alloc()
            if g is None:
                self.events.append(("NOFRAME", block, file_id, q))
                break
            fr = self.frames[g]
            fr.state = FILLING
            fr.file, fr.page = file_id, q
            fr.pins = 0
            fr.ref = 0
            fr.ra = 1
            fr.mark = 1 if q == ws else 0
            self.map[(file_id, q)] = g
            self.events.append(("ALLOC", file_id, q, g, 1))
            allocated.append(g)
            self.fetched_pages += 1
            self.fetched_bytes += self.page_bytes(file_id, q)
            self.ra_pages += 1
            q += 1
        if allocated:
            self.events.append(("REQ", file_id, ws, len(allocated)))
            self.requests += 1
            self.request_bytes += sum(self.page_bytes(file_id, r) for r in range(ws, ws + len(allocated)))
            self.pending[block] = allocated

    # ---- one block-collective read ------------------------------------------------------------
    def gread(self, block: int, file_id: int, offset: int, size: int) -> int:
        """Split [offset, offset+size) into pages (ascending) and access each; returns bytes.
        An asynchronous request the read issued completes when it ends (serialized runs)."""
        fsize = self.files[file_id].size
        if size <= 0 or offset >= fsize:
            return 0
        end = min(offset + size, fsize)
        last = (end - 1) // self.P
        for p in range(offset // self.P, last + 1):
            self.access(block, file_id, p, last - p + 1)
        self.complete(block)
        self.delivered_bytes += end - offset
        return end - offset

    # ---- end of run ---------------------------------------------------------------------------
    def leftover_wasted(self) -> Tuple[int, int]:
        """Prefetched pages still unconsumed in the cache: (pages, bytes)."""
        pages = 0
        nbytes = 0
        for fr in self.frames:
            if fr.state != FREE and fr.ra:
                pages += 1
                nbytes += self.page_bytes(fr.file, fr.page)
        return pages, nbytes

    def check_invariants(self) -> None:
        seen = set()
        for f, fr in enumerate(self.frames):
            assert fr.pins >= 0
            if fr.state == FREE:
                continue
            key = (fr.file, fr.page)
            assert key not in seen, f"{key} mapped twice"
            seen.add(key)
            assert self.map.get(key) == f, f"map/frame disagree for {key}"
        assert len(seen) == len(self.map)


def run_serialized(model: PolicyModel, file_id: int, offsets, read_size: int) -> PolicyModel:
    """Run every block's reads in (round, block) order: round k does read k of blocks 0..B-1."""
    nb, K = offsets.shape
    for k in range(K):
        for b in range(nb):
            model.gread(b, file_id, int(offsets[b, k]), read_size)
    return model
