"""Pins for the private-buffer policy model (the paper's Sec. 4.1 prefetcher and Sec. 5.1
replacement), CPU only:

* with no prefetch, one block's misses evict in allocation order, exactly as the
  independent per-block LRA queue of oracle/lra.py does, and a block never evicts
  another block's frames;
* with prefetch k, a block reading a file sequentially makes one host request per
  k + 1 pages and fills the other pages from its private buffer (closed form);
* private buffers are not shared: interleaved blocks reading each other's next pages
  gain nothing from one another's prefetch;
* the last request of a file is clamped to its end, and pages left in a buffer count as
  wasted when the block gives its slot back;
* a hit on a page another block brought in costs no request.
"""
import numpy as np
import pytest

from oracle.lra import LRACache
from oracle.private import PrivatePolicyModel, run_serialized

P = 4096


@pytest.mark.parametrize("quota,npages", [(4, 17), (8, 8), (5, 23)])
def test_no_prefetch_evicts_like_per_block_lra(quota, npages):
    m = PrivatePolicyModel(nframes=quota * 3, page_size=P, prefetch_pages=0, slots=3)
    m.open(0, npages * P)
    lra = LRACache(nframes=quota * 3, resident_blocks=3, page_size=P)
    m.begin_block(1)
    for p in range(npages):
        m.access(1, 0, p)
        lra.read_page(1, 0, p)
    ev = [(e[3], e[4]) for e in m.events if e[0] == "EVICT"]
    assert ev == lra.evicted
    assert m.misses == npages == m.requests
    # slot 1 only ever touched its own share [quota, 2*quota)
    frames = {e[4] for e in m.events if e[0] == "ALLOC"}
    assert frames <= set(range(quota, 2 * quota))


@pytest.mark.parametrize("k,npages", [(3, 40), (7, 64), (1, 9), (15, 16)])
def test_sequential_reader_requests_once_per_window(k, npages):
    m = PrivatePolicyModel(nframes=64, page_size=P, prefetch_pages=k, slots=2)
    m.open(0, npages * P)
    m.begin_block(0)
    m.gread(0, 0, 0, npages * P)
    m.end_block(0)
    assert m.requests == -(-npages // (k + 1))
    assert m.pb_hits == npages - m.requests
    assert m.misses == npages
    assert m.wasted == 0
    reqs = [(e[3], e[4]) for e in m.events if e[0] == "REQ"]
    assert reqs[0] == (0, min(k + 1, npages))
    assert all(first % (k + 1) == 0 for first, _ in reqs)


def test_private_buffers_are_not_shared():
    # two blocks alternate pages 0,1,2,...: each block's prefetch covers pages the other
    # block will read, which the other block cannot use
    m = PrivatePolicyModel(nframes=64, page_size=P, prefetch_pages=4, slots=2)
    m.open(0, 32 * P)
    for s in (0, 1):
        m.begin_block(s)
    for p in range(32):
        m.access(p % 2, 0, p)
    for s in (0, 1):
        m.end_block(s)
    # block 0 at page 0 prefetches 1..4; it uses 2 and 4 (its own), block 1 misses 1 and 3
    assert m.pb_hits > 0
    assert m.requests + m.pb_hits == m.misses == 32
    assert m.wasted > 0
    assert m.hits == 0


def test_end_of_file_clamp_and_wasted_tail():
    m = PrivatePolicyModel(nframes=64, page_size=P, prefetch_pages=8, slots=1)
    size = 10 * P + 123                    # 11 pages, the last one partial
    m.open(0, size)
    m.begin_block(0)
    m.access(0, 0, 0)                      # request pages 0..8
    m.access(0, 0, 9)                      # request 9..10 (clamped)
    m.end_block(0)
    reqs = [(e[3], e[4]) for e in m.events if e[0] == "REQ"]
    assert reqs == [(0, 9), (9, 2)]
    assert m.request_bytes == 9 * P + (P + 123)
    # pages 1..8 were dropped unused when page 9 was requested; page 10 at the end
    assert m.wasted == 8 + 1


def test_hit_on_another_blocks_page():
    m = PrivatePolicyModel(nframes=8, page_size=P, prefetch_pages=2, slots=2)
    m.open(0, 16 * P)
    m.begin_block(0)
    m.begin_block(1)
    m.access(0, 0, 5)
    m.access(1, 0, 5)
    assert m.hits == 1 and m.requests == 1
    assert ("HIT", 1, 0, 5, 0) in m.events


def test_run_serialized_orders_rounds_then_blocks():
    offsets = np.array([[0, 2 * P], [P, 3 * P]], dtype=np.uint64)
    m = PrivatePolicyModel(nframes=8, page_size=P, prefetch_pages=0, slots=2)
    m.open(0, 4 * P)
    run_serialized(m, 0, offsets, P)
    order = [(e[1], e[3]) for e in m.events if e[0] == "MISS"]
    assert order == [(0, 0), (1, 1), (0, 2), (1, 3)]
