"""The paper's own cache policy: private prefetch buffers and per-block replacement.

Test infrastructure only (see the package docstring).

Sec. 4.1 (GPU-side mechanism), in order:
  1. every threadblock has a private buffer for prefetched data;
  2-3. a read looks in the GPU page cache first and is served from it on a hit;
  4. on a miss the block allocates a new page and looks in its private buffer;
  5. if the page is there, the block fills the cache page from it (no host request);
  6. else it asks the host for PAGE_SIZE + PREFETCH_SIZE bytes (PREFETCH_SIZE static);
  7. the requested page goes into the cache, the rest into the private buffer.
Sec. 5.1 (replacement): each block owns a fixed share of the frames (cache size divided by
the number of concurrently running blocks) and reuses its own least recently allocated
frame in place when the share is used up.

Readings (where the text leaves a choice): a block's share is a contiguous range of frames
(slot s owns [s*quota, (s+1)*quota)) walked in a ring, which is least-recently-allocated
order; the private buffer holds the pages that follow the requested one in the file
(clamped to the end of the file) and is replaced by the next request; a new owner of a slot
starts with an empty buffer, and pages dropped from a buffer without being used are
counted as wasted. Block b uses slot b (the slots outnumber the blocks in every test).

Event tuples, in the order the device records them:
  ("HIT", slot, file, page, frame)
  ("MISS", slot, file, page, window)          window = 1 for a private-buffer fill, else
                                              the pages of the host request
  ("EVICT", slot, frame, vfile, vpage)
  ("ALLOC", slot, file, page, frame)
  ("PBHIT", slot, file, page, frame)
  ("REQ", slot, file, first, npages)
"""
from __future__ import annotations

from typing import Dict, List, Optional, Tuple


class PrivatePolicyModel:
    def __init__(self, nframes: int, page_size: int, prefetch_pages: int, slots: int):
        self.C = nframes
        self.P = page_size
        self.prefetch = prefetch_pages
        self.slots = slots
        self.quota = nframes // slots
        if self.quota < 1:
            raise ValueError("fewer frames than slots")
        self.frames: List[Optional[Tuple[int, int]]] = [None] * nframes
        self.map: Dict[Tuple[int, int], int] = {}
        self.next = [0] * slots
        self.pbuf: List[Optional[Tuple[int, int, int]]] = [None] * slots   # (file, first, n)
        self.used = [0] * slots
        self.sizes: Dict[int, int] = {}
        self.events: List[tuple] = []
        self.hits = self.misses = self.requests = self.request_bytes = 0
        self.evictions = self.pb_hits = self.pb_pages = self.wasted = 0

    def open(self, file_id: int, size: int) -> None:
        self.sizes[file_id] = size

    def npages(self, file_id: int) -> int:
        return -(-self.sizes[file_id] // self.P)

    def _drop_buffer(self, slot: int) -> None:
        if self.pbuf[slot] is not None:
            self.wasted += self.pbuf[slot][2] - self.used[slot]
        self.pbuf[slot] = None
        self.used[slot] = 0

    def begin_block(self, slot: int) -> None:
        """A block takes the slot (gopen): its buffer starts empty."""
        self._drop_buffer(slot)

    def end_block(self, slot: int) -> None:
        """The block gives the slot back (gclose): the buffer is dropped."""
        self._drop_buffer(slot)

    def access(self, slot: int, file_id: int, p: int) -> None:
        key = (file_id, p)
        if key in self.map:                                      # steps 2-3
            self.hits += 1
            self.events.append(("HIT", slot, file_id, p, self.map[key]))
            return
        self.misses += 1
        pb = self.pbuf[slot]
        in_pb = pb is not None and pb[0] == file_id and pb[1] <= p < pb[1] + pb[2]
        span = min(1 + self.prefetch, self.npages(file_id) - p)
        self.events.append(("MISS", slot, file_id, p, 1 if in_pb else span))
        # step 4 with Sec. 5.1: the least recently allocated frame of the block's share
        f = slot * self.quota + self.next[slot]
        self.next[slot] = (self.next[slot] + 1) % self.quota
        old = self.frames[f]
        if old is not None:
            self.evictions += 1
            del self.map[old]
            self.events.append(("EVICT", slot, f, old[0], old[1]))
        self.frames[f] = key
        self.map[key] = f
        self.events.append(("ALLOC", slot, file_id, p, f))
        if in_pb:                                                # step 5
            self.pb_hits += 1
            self.used[slot] += 1
            self.events.append(("PBHIT", slot, file_id, p, f))
            return
        # steps 6-7: one host request for the page and the prefetch behind it
        self.requests += 1
        self.request_bytes += min(span * self.P, self.sizes[file_id] - p * self.P)
        self.events.append(("REQ", slot, file_id, p, span))
        self._drop_buffer(slot)
        self.pbuf[slot] = (file_id, p + 1, span - 1)
        self.pb_pages += span - 1

    def gread(self, slot: int, file_id: int, offset: int, size: int) -> None:
        end = min(offset + size, self.sizes[file_id])
        if size <= 0 or offset >= end:
            return
        for p in range(offset // self.P, (end - 1) // self.P + 1):
            self.access(slot, file_id, p)


def run_serialized(model: PrivatePolicyModel, file_id: int, offsets, read_size: int) -> None:
    """The reads of a list-reader launch in (round, block) order, block b on slot b; every
    block takes its slot first and gives it back after its last read."""
    blocks, reads = offsets.shape
    for b in range(blocks):
        model.begin_block(b)
    for k in range(reads):
        for b in range(blocks):
            model.gread(b, file_id, int(offsets[b, k]), read_size)
    for b in range(blocks):
        model.end_block(b)
