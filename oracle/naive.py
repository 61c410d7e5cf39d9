"""A second, independently written policy model: plain lists and linear scans.

Test infrastructure only. It exists to cross-check ``oracle.policy`` by brute
force over every interleaving of tiny workloads; it implements the same rules
(page split, lookup, synchronous windowed miss, clock hand, stream detector) from
their statement, without sharing code or data structures with ``policy``.

Frame record: [state, file, page, pins, ref, ra] with state 0 free, 1 filling, 2 valid.
Stream record: [in_use, next, size, last_use].
"""
from __future__ import annotations


def _find(frames, file_id, page):
    for i in range(len(frames)):
        fr = frames[i]
        if fr[0] != 0 and fr[1] == file_id and fr[2] == page:
            return i
    return -1


class NaiveModel:
    def __init__(self, nframes, page_size, w0, cap, nstreams, recent=64, reach=64, enough=3):
        self.frames = [[0, -1, -1, 0, 0, 0] for _ in range(nframes)]
        self.page_size = page_size
        self.w0 = w0
        self.cap = cap
        self.nstreams = nstreams
        self.keep = recent        # misses remembered per file
        self.reach = reach        # how far a remembered miss may be from p and still count
        self.enough = enough      # close misses that mean the file is read in aggregate
        self.hand = 0
        self.size = {}
        self.advice = {}
        self.streams = {}
        self.tick = {}
        self.last_misses = {}
        self.log = []
        self.gone = []            # (file, page) evicted after being read, in eviction order

    def open(self, file_id, size, advice="normal"):
        self.size[file_id] = size
        self.advice[file_id] = advice
        self.streams[file_id] = [[False, 0, 0, 0] for _ in range(self.nstreams)]
        self.tick[file_id] = 0
        self.last_misses[file_id] = []

    def _window(self, file_id, p, want):
        if self.cap == 0 or self.advice[file_id] == "random":
            return p, 1
        self.tick[file_id] = self.tick[file_id] + 1
        now = self.tick[file_id]
        table = self.streams[file_id]
        hist = self.last_misses[file_id]
        reach = self.reach
        close = 0
        for r in hist:
            if p - reach <= r <= p + reach:
                close += 1
        hist.append(p)
        while len(hist) > self.keep:
            del hist[0]
        i = 0
        while i < len(table):
            st = table[i]
            if st[0] and p >= st[1] and p < st[1] + st[2]:
                start = st[1]
                n = 2 * st[2]
                if n > self.cap:
                    n = self.cap
                table[i] = [True, start + n, n, now]
                return start, n
            i += 1
        # the cached pages right behind p, counted up to one past the cap (enough to compare
        # them with a read of up to cap pages and to size the window)
        behind = 0
        q = p - 1
        while q >= 0 and behind <= self.cap and _find(self.frames, file_id, q) >= 0:
            behind += 1
            q -= 1
        asked = want if want < self.cap else self.cap
        slot = -1
        for i in range(len(table)):
            if not table[i][0]:
                slot = i
                break
        if slot < 0:
            slot = 0
            for i in range(1, len(table)):
                if table[i][3] < table[slot][3]:
                    slot = i
        start = p
        if close >= self.enough:
            n = self.cap
            start = p - p % n
        elif behind > asked:      # more cached history than the read itself: a stream
            n = 2 * behind
            if n < asked:         # never less than the rest of the read that missed
                n = asked
        elif p == 0 or self.advice[file_id] == "sequential":
            n = self.w0
            if n < asked:
                n = asked
        else:
            n = asked             # a new stream reads what was asked for, at least one page
        if n > self.cap:
            n = self.cap
        if n < 1:
            n = 1
        table[slot] = [True, start + n, n, now]
        return start, n

    def _take_frame(self):
        C = len(self.frames)
        visits = 0
        while visits < 2 * C:
            t = self.hand
            self.hand = t + 1
            visits += 1
            i = t % C
            fr = self.frames[i]
            # what the hand found: ref bit, pinned, (never a lost race), state 0/2/3
            code = 0 if fr[0] == 0 else (2 if fr[0] == 1 else 3)
            found = fr[4] + 2 * (1 if fr[3] != 0 else 0) + 8 * code
            if fr[0] == 0:
                self.log.append(("HAND", t, i, "FREE", -1, -1, 0, found))
                return i
            if fr[0] == 1 or fr[3] != 0:
                self.log.append(("HAND", t, i, "SKIP", -1, -1, 0, found))
                continue
            if fr[4] == 1:
                fr[4] = 0
                self.log.append(("HAND", t, i, "CLEAR", -1, -1, 0, found))
                continue
            self.log.append(("HAND", t, i, "EVICT", fr[1], fr[2], fr[5], found))
            if fr[5] == 0:
                self.gone.append((fr[1], fr[2]))
            self.frames[i] = [0, -1, -1, 0, 0, 0]
            return i
        return -1

    def read(self, block, file_id, offset, size):
        fsize = self.size[file_id]
        if size <= 0 or offset >= fsize:
            return 0
        last_byte = offset + size
        if last_byte > fsize:
            last_byte = fsize
        P = self.page_size
        npages = (fsize + P - 1) // P
        page = offset // P
        while page * P < last_byte:
            i = _find(self.frames, file_id, page)
            if i >= 0:
                self.frames[i][4] = 1
                self.frames[i][5] = 0
                self.log.append(("HIT", block, file_id, page, i))
            else:
                # pages of this read from `page` to its end
                want = (last_byte - 1) // P - page + 1
                start, n = self._window(file_id, page, want)
                if start + n > npages:
                    n = npages - start
                self.log.append(("MISS", block, file_id, page, start, n))
                # a page read earlier and evicted since is not fetched again for a window,
                # unless the missing page is such a page too (the file is read again)
                again = (file_id, page) in self.gone
                lo = page
                while (lo > start and _find(self.frames, file_id, lo - 1) < 0
                       and (again or (file_id, lo - 1) not in self.gone)):
                    lo -= 1
                hi = page
                while (hi < start + n - 1 and _find(self.frames, file_id, hi + 1) < 0
                       and (again or (file_id, hi + 1) not in self.gone)):
                    hi += 1
                todo = [page]
                for q in range(lo, hi + 1):
                    if q != page:
                        todo.append(q)
                got = []
                for q in todo:
                    i = self._take_frame()
                    if i < 0:
                        if q == page:
                            raise RuntimeError("no frame for demanded page")
                        self.log.append(("NOFRAME", block, file_id, q))
                        break
                    self.frames[i] = [1, file_id, q, 1 if q == page else 0, 0, 0 if q == page else 1]
                    self.log.append(("ALLOC", file_id, q, i, 0 if q == page else 1))
                    got.append(i)
                pages = [self.frames[i][2] for i in got]
                self.log.append(("REQ", file_id, min(pages), max(pages) - min(pages) + 1))
                for i in got:
                    self.frames[i][0] = 2
                    self.frames[i][4] = 1
                j = _find(self.frames, file_id, page)
                self.frames[j][3] = self.frames[j][3] - 1
            page += 1
        return last_byte - offset
