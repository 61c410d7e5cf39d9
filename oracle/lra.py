"""The paper's replacement mechanism: a per-threadblock least-recently-allocated queue.

Test infrastructure only. Sec. 5.1: each threadblock keeps a fixed-size queue of
the pages it allocated in the GPU page cache; the queue size is the cache size
divided by the number of concurrently resident threadblocks. When the block has
no free entry left it evicts the least recently allocated page of its own queue,
reuses that frame in place for the new page (remapping it in the page table) and
puts it back at the head of the queue.

Used to pin the eviction order of the clock model on read-once streams, where
the paper argues every page is used once and local allocation order is the
natural replacement order.
"""
from __future__ import annotations

from collections import deque
from typing import Dict, List, Tuple


class LRACache:
    def __init__(self, nframes: int, resident_blocks: int, page_size: int):
        self.quota = nframes // resident_blocks
        if self.quota < 1:
            raise ValueError("cache smaller than the number of resident blocks")
        self.P = page_size
        self.queues: Dict[int, deque] = {}
        self.pages = set()
        self.evicted: List[Tuple[int, int]] = []   # (file, page) in eviction order
        self.misses = 0
        self.hits = 0

    def read_page(self, block: int, file_id: int, page: int) -> None:
        key = (file_id, page)
        if key in self.pages:
            self.hits += 1
            return
        self.misses += 1
        q = self.queues.setdefault(block, deque())
        if len(q) >= self.quota:
            old = q.popleft()                      # least recently allocated
            self.pages.discard(old)
            self.evicted.append(old)
        q.append(key)                              # head of the queue = most recent
        self.pages.add(key)
