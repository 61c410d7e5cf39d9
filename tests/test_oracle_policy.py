"""Pins for the policy half of the oracle (CPU only).

Each test fixes the model against something other than itself:
* the paper's worked readahead example (Sec. 3.2: a 4 KB read at offset 0 makes
  the prefetcher fetch 16 KB) and the doubling-to-a-maximum rule (Sec. 2.3), in
  closed form for a single stream;
* textbook second-chance behaviour on a hand-worked reference string (it differs
  from both FIFO and LRU there);
* the paper's per-threadblock least-recently-allocated replacement (Sec. 5.1) for
  a single read-once stream: same eviction order;
* closed forms: cache >= file gives misses = distinct pages and no evictions;
  a larger-than-cache strided stream gives misses = pages, evictions = pages - frames;
  uniform random pages give a steady-state hit ratio of frames/pages;
* brute force: every interleaving of tiny workloads, against an independently
  written naive model, event for event;
* invariants after every run.
"""
import itertools
import random

import numpy as np
import pytest

from oracle.lra import LRACache
from oracle.naive import NaiveModel
from oracle.policy import PolicyModel, run_serialized
from workloads import configs


def _misses(ev):
    return [e for e in ev if e[0] == "MISS"]


def _evicted(ev):
    return [(e[4], e[5]) for e in ev if e[0] == "HAND" and e[3] == "EVICT"]


def test_paper_example_first_window_is_16KB():
    # Sec. 3.2: 4 KB read at offset 0 -> the prefetcher fetches 16 KB (W0 = 4 pages of 4 KiB).
    m = PolicyModel(nframes=64, page_size=4096, ra_init_pages=4, ra_cap_pages=32)
    m.open(0, 1 << 20)
    m.gread(0, 0, 0, 4096)
    req = [e for e in m.events if e[0] == "REQ"]
    assert req == [("REQ", 0, 0, 4)]
    assert m.request_bytes == 16 * 1024
    # the next 4 KB read is served from the prefetched window
    m.gread(0, 0, 4096, 4096)
    assert m.events[-1][0] == "HIT"


def test_single_stream_window_doubles_to_cap():
    W0, cap, npages = 4, 16, 200
    m = PolicyModel(nframes=512, page_size=1 << 16, ra_init_pages=W0, ra_cap_pages=cap)
    m.open(0, npages << 16)
    for p in range(npages):
        m.gread(0, 0, p << 16, 1 << 16)
    got = [(e[4], e[5]) for e in _misses(m.events)]
    expect = []
    ws, wn = 0, W0
    while ws < npages:
        expect.append((ws, min(wn, npages - ws)))
        ws += wn
        wn = min(2 * wn, cap)
    assert got == expect
    assert m.fetched_pages == npages and m.wasted_pages == 0
    # closed-form request count: W0, 2W0, ... up to cap, then cap
    assert m.requests == len(expect)


def test_textbook_second_chance():
    # hand-worked: 3 frames, RA off, reference string 0 1 2 0 3 1 4 5
    # fills set the reference bit; the hit on page 1 saves it from the next sweep.
    m = PolicyModel(nframes=3, page_size=1, ra_cap_pages=0)
    m.open(0, 100)
    for p in [0, 1, 2, 0, 3, 1, 4, 5]:
        m.gread(0, 0, p, 1)
    assert _evicted(m.events) == [(0, 0), (0, 2), (0, 1)]
    hand = [(e[1], e[2], e[3]) for e in m.events if e[0] == "HAND"]
    assert hand == [(0, 0, "FREE"), (1, 1, "FREE"), (2, 2, "FREE"),
                    (3, 0, "CLEAR"), (4, 1, "CLEAR"), (5, 2, "CLEAR"), (6, 0, "EVICT"),
                    (7, 1, "CLEAR"), (8, 2, "EVICT"),
                    (9, 0, "CLEAR"), (10, 1, "EVICT")]
    # FIFO would evict 0,1,2 and LRU would evict 1 first: second chance is neither
    assert _evicted(m.events) != [(0, 0), (0, 1), (0, 2)]


@pytest.mark.parametrize("nframes,npages", [(8, 40), (16, 16 * 5 + 3)])
def test_single_reader_evicts_in_allocation_order_like_lra(nframes, npages):
    m = PolicyModel(nframes=nframes, page_size=64, ra_cap_pages=0)
    m.open(0, npages * 64)
    lra = LRACache(nframes=nframes, resident_blocks=1, page_size=64)
    for p in range(npages):
        m.gread(0, 0, p * 64, 64)
        lra.read_page(0, 0, p)
    ev = _evicted(m.events)
    assert ev == [(0, q) for q in range(npages - nframes)]
    assert ev == lra.evicted
    assert m.misses == npages == lra.misses


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cache_holds_file_no_evictions_any_order(seed):
    rng = random.Random(seed)
    npages = 50
    m = PolicyModel(nframes=64, page_size=1024, ra_cap_pages=0)
    m.open(0, npages * 1024 - 100)
    order = [rng.randrange(npages) for _ in range(400)]
    for blk, p in enumerate(order):
        m.gread(blk % 7, 0, p * 1024, 1024)
    assert m.misses == len(set(order)) and m.evictions == 0
    m.check_invariants()


def test_strided_larger_than_cache_counts():
    # C2 shape scaled down: 64 blocks, 128 KiB strides, 256 KiB pages, 32 MiB file, 8 MiB cache
    wl = configs.c2_small()
    C = wl.cache_bytes // wl.page_size
    N = wl.file.size // wl.page_size
    m = PolicyModel(nframes=C, page_size=wl.page_size, ra_cap_pages=0)
    m.open(0, wl.file.size)
    run_serialized(m, 0, wl.offsets, wl.read_size)
    assert m.misses == N and m.evictions == N - C and m.fetched_pages == N
    assert m.hits == N  # the second half of every page is a hit for the neighbouring block
    m.check_invariants()


def test_uniform_random_hit_ratio_is_frames_over_pages():
    # independent reference model: any demand policy hits with probability C/N in steady state
    C, N, n = 64, 256, 120_000
    m = PolicyModel(nframes=C, page_size=1, ra_cap_pages=0)
    m.open(0, N)
    rng = np.random.default_rng(12345)
    pages = rng.integers(0, N, size=n)
    for i, p in enumerate(pages):
        m.gread(i % 32, 0, int(p), 1)
    warm = 10_000
    # count hits among the accesses after warm-up
    acc = [e for e in m.events if e[0] in ("HIT", "MISS")]
    steady = acc[warm:]
    ratio = sum(1 for e in steady if e[0] == "HIT") / len(steady)
    assert abs(ratio - C / N) < 0.01, ratio
    assert sum(1 for e in acc if e[0] == "HIT") == m.hits


def test_readahead_accounting_identities():
    wl = configs.c2_small()
    C = wl.cache_bytes // wl.page_size
    m = PolicyModel(nframes=C, page_size=wl.page_size, ra_init_pages=4, ra_cap_pages=16)
    m.open(0, wl.file.size)
    run_serialized(m, 0, wl.offsets, wl.read_size)
    demand = m.misses
    assert m.fetched_pages == demand + m.ra_pages
    left, _ = m.leftover_wasted()
    assert m.wasted_pages + left <= m.ra_pages
    assert m.misses < wl.file.size // wl.page_size   # readahead removed most demand misses
    m.check_invariants()


def test_random_advice_disables_readahead():
    m = PolicyModel(nframes=32, page_size=4096, ra_init_pages=4, ra_cap_pages=16)
    m.open(0, 1 << 20, advice="random")
    for p in range(10):
        m.gread(0, 0, p * 4096, 4096)
    assert [(e[4], e[5]) for e in _misses(m.events)] == [(p, 1) for p in range(10)]
    m2 = PolicyModel(nframes=32, page_size=4096, ra_init_pages=4, ra_cap_pages=16)
    m2.open(0, 1 << 20, advice="sequential")
    m2.gread(0, 0, 5 * 4096, 4096)             # not at offset 0, but SEQUENTIAL opens at W0
    assert _misses(m2.events)[0][4:] == (5, 4)


def test_window_clamped_at_eof_and_partial_page():
    m = PolicyModel(nframes=32, page_size=4096, ra_init_pages=4, ra_cap_pages=16)
    m.open(0, 2 * 4096 + 10)                   # 3 pages, the last one 10 bytes
    assert m.gread(0, 0, 0, 4096 * 8) == 2 * 4096 + 10
    assert _misses(m.events) == [("MISS", 0, 0, 0, 0, 3)]
    assert m.fetched_bytes == 2 * 4096 + 10
    assert m.gread(0, 0, 3 * 4096, 10) == 0    # at/after EOF: nothing


def _interleavings(seqs):
    """Every merge of the per-block sequences that keeps each block's own order."""
    counts = [len(s) for s in seqs]
    labels = []
    for b, c in enumerate(counts):
        labels += [b] * c
    seen = set()
    for perm in itertools.permutations(labels):
        if perm in seen:
            continue
        seen.add(perm)
        yield perm


@pytest.mark.parametrize("case", range(10))
def test_brute_force_against_naive_model(case):
    rng = random.Random(1000 + case)
    # detector constants: the defaults for the first cases, then small ones under which the
    # aggregate rule fires or stays off within a few pages
    det = (64, 64, 3) if case < 4 else (rng.choice([1, 2, 3]), rng.choice([0, 1, 2]), rng.choice([1, 2, 4]))
    nblocks = 3 if case % 2 == 0 else 2
    nacc = 3 if nblocks == 3 else 4
    npages = rng.randint(4, 8)
    nframes = rng.randint(2, 4)
    w0 = rng.randint(1, 2)
    cap = rng.choice([0, 2, 4])
    psz = 8
    fsize = npages * psz - rng.randint(0, 7)
    seqs = [[(rng.randrange(npages), rng.choice([psz, 2 * psz])) for _ in range(nacc)] for _ in range(nblocks)]
    outcomes = set()
    n = 0
    for order in _interleavings(seqs):
        pos = [0] * nblocks
        m = PolicyModel(nframes, psz, ra_init_pages=w0, ra_cap_pages=cap, streams_per_file=2, recent=det[0],
                        near_pages=det[1], near_min=det[2])
        m.open(0, fsize)
        nv = NaiveModel(nframes, psz, w0, cap, 2, recent=det[0], reach=det[1], enough=det[2])
        nv.open(0, fsize)
        for b in order:
            page, size = seqs[b][pos[b]]
            pos[b] += 1
            r1 = m.gread(b, 0, page * psz, size)
            r2 = nv.read(b, 0, page * psz, size)
            assert r1 == r2
        assert m.events == nv.log, (case, order)
        m.check_invariants()
        outcomes.add(tuple(_evicted(m.events)))
        n += 1
    assert n > 1 and len(outcomes) >= 1


def test_a_window_does_not_fetch_again_what_a_reader_consumed_and_the_cache_dropped():
    # hand-worked, 2 frames, one stream slot, aggregate rule off. 5 and 50 are read; 51's
    # window [51, 53) evicts both (consumed, so they leave shadows), then 3 evicts 51 and 4
    # evicts 52, which was prefetched and never read (no shadow). 4 is in 3's zone: window
    # [4, 6), but 5 was consumed and dropped, so only 4 is requested (Sec. 5.1: prefetched
    # pages evicted unused are the waste to avoid; 5 lies behind the reader that read it)
    P = 4096
    m = PolicyModel(nframes=2, page_size=P, ra_init_pages=1, ra_cap_pages=4, streams_per_file=1, near_min=100)
    m.open(0, 64 * P)
    for p in (5, 50, 51, 3, 4):
        m.gread(0, 0, p * P, P)
    assert [(e[4], e[5]) for e in _misses(m.events)] == [(5, 1), (50, 1), (51, 2), (3, 1), (4, 2)]
    assert [e[2:] for e in m.events if e[0] == "REQ"] == [(5, 1), (50, 1), (51, 2), (3, 1), (4, 1)]
    assert [(e[5], e[6]) for e in m.events if e[0] == "HAND" and e[3] == "EVICT"] == \
        [(5, 0), (50, 0), (51, 0), (52, 1)]
    # the same accesses, with 5 never read before: the window fetches both pages
    m2 = PolicyModel(nframes=2, page_size=P, ra_init_pages=1, ra_cap_pages=4, streams_per_file=1, near_min=100)
    m2.open(0, 64 * P)
    for p in (6, 50, 51, 3, 4):
        m2.gread(0, 0, p * P, P)
    assert [e[2:] for e in m2.events if e[0] == "REQ"][-1] == (4, 2)


def test_a_file_read_again_gets_full_windows():
    # a single reader passes twice over a 40-page file through 8 frames: in the second pass
    # every page it misses was consumed and dropped, so the shadows do not cut its windows,
    # and it fetches with the same 4-page requests as the first pass
    P = 4096
    m = PolicyModel(nframes=8, page_size=P, ra_init_pages=4, ra_cap_pages=4, streams_per_file=1)
    m.open(0, 40 * P)
    reqs = []
    for _ in range(2):
        n0 = len(m.events)
        for p in range(40):
            m.gread(0, 0, p * P, P)
        reqs.append([e[2:] for e in m.events[n0:] if e[0] == "REQ"])
    assert reqs[0] == [(q, 4) for q in range(0, 40, 4)]
    assert reqs[1] == reqs[0]
    assert m.fetched_pages == 80 and m.wasted_pages == 0


def test_context_readahead_follows_a_stream_no_slot_tracks():
    # hand-worked, one stream slot: 0 opens [0,4); 100 takes the only slot; 4 is outside every
    # zone, but pages 0..3 right behind it are cached, so it is sequential with history 4:
    # window [4, 4 + min(2*4, cap)) (Sec. 2.3: Linux follows interleaved readers of one file)
    m = PolicyModel(nframes=64, page_size=4096, ra_init_pages=4, ra_cap_pages=16, streams_per_file=1)
    m.open(0, 1 << 20)
    for p in (0, 100, 4):
        m.gread(0, 0, p * 4096, 4096)
    assert [(e[4], e[5]) for e in _misses(m.events)] == [(0, 4), (100, 1), (4, 8)]
    # with no history behind it a page outside every zone is on probation (window 1)
    m.gread(0, 0, 200 * 4096, 4096)
    assert _misses(m.events)[-1][4:] == (200, 1)


def test_a_read_of_several_pages_gets_them_in_one_window():
    # hand-worked, one stream slot, cap 16 (Sec. 2.3: the prefetcher reads at least what the
    # caller asked for): an 8-page read at page 100 opens a new stream with the 8 pages
    # [100, 108) instead of one page on probation, and its other 7 pages are hits (the
    # prefetch is synchronous); the next 8-page read at 108 is in the stream's zone and doubles it to
    # [108, 124); a 40-page read at 300 asks for more than the cap: [300, 316), then the
    # zone takes it on, [316, 332) and [332, 348), three requests for the 40 pages
    m = PolicyModel(nframes=256, page_size=4096, ra_init_pages=4, ra_cap_pages=16, streams_per_file=1)
    m.open(0, 1 << 22)
    m.gread(0, 0, 100 * 4096, 8 * 4096)
    assert [(e[4], e[5]) for e in _misses(m.events)] == [(100, 8)]
    assert [e for e in m.events if e[0] == "REQ"] == [("REQ", 0, 100, 8)]
    assert sum(1 for e in m.events if e[0] == "HIT") == 7
    m.gread(0, 0, 108 * 4096, 8 * 4096)
    assert [(e[4], e[5]) for e in _misses(m.events)][-1] == (108, 16)
    m.gread(0, 0, 300 * 4096, 40 * 4096)
    assert [(e[4], e[5]) for e in _misses(m.events)][-3:] == [(300, 16), (316, 16), (332, 16)]
    assert [r for _, _, r in m.decisions] == [4, 1, 4, 1, 1]   # new, zone, new, zone, zone


def test_context_rule_needs_more_history_than_the_read():
    # hand-worked, one slot, cap 16 (Sec. 2.3; Linux's context readahead): a 4-page read at 0
    # opens [0, 4) (W0 = 4 = the read); a 1-page read at 100 takes the only slot.
    # (a) a 2-page read at 4: history 4 behind it, longer than the read -> context, window
    #     2h = 8: [4, 12)
    # (b) after a 1-page read at 200 takes the slot again, a 12-page read at 12: history 12
    #     (pages 0..11), not longer than the read -> a new stream with the 12 pages asked
    #     for, [12, 24) (the window the context rule would give as well)
    # (c) a 1-page read at 301 with only page 300 cached behind it (read before, its stream
    #     then replaced by a read at 500): a history of 1 is no longer than the read, as
    #     likely a random read as a stream -> one page on probation
    m = PolicyModel(nframes=256, page_size=4096, ra_init_pages=4, ra_cap_pages=16, streams_per_file=1)
    m.open(0, 1 << 22)
    m.gread(0, 0, 0, 4 * 4096)
    m.gread(0, 0, 100 * 4096, 4096)
    m.gread(0, 0, 4 * 4096, 2 * 4096)
    assert [(e[4], e[5]) for e in _misses(m.events)] == [(0, 4), (100, 1), (4, 8)]
    assert m.decisions[-1] == (1, 4, 3)   # one near miss (page 0), history 4, the context rule
    m.gread(0, 0, 200 * 4096, 4096)
    m.gread(0, 0, 12 * 4096, 12 * 4096)
    assert [(e[4], e[5]) for e in _misses(m.events)][-1] == (12, 12)
    assert m.decisions[-1] == (2, 12, 4)   # near misses 0 and 4, history 12, a new stream
    m.gread(0, 0, 300 * 4096, 4096)
    m.gread(0, 0, 500 * 4096, 4096)
    m.gread(0, 0, 301 * 4096, 4096)
    assert [(e[4], e[5]) for e in _misses(m.events)][-1] == (301, 1)
    assert m.decisions[-1][1:] == (1, 4)


def test_aggregate_read_takes_aligned_cap_chunk():
    # hand-worked, one slot, cap 16 (near = within 64 pages): misses at 10, 30, 50 each start a
    # probation stream; at 70 three of the last misses are near, so the block takes the aligned
    # chunk [64, 80) -- the interleaved-strides case where many blocks miss close together
    m = PolicyModel(nframes=256, page_size=4096, ra_init_pages=4, ra_cap_pages=16, streams_per_file=1)
    m.open(0, 1 << 20)
    for p in (10, 30, 50, 70):
        m.gread(0, 0, p * 4096, 4096)
    assert [(e[4], e[5]) for e in _misses(m.events)] == [(10, 1), (30, 1), (50, 1), (64, 16)]
    assert [e for e in m.events if e[0] == "REQ"][-1] == ("REQ", 0, 64, 16)


def test_aggregate_rule_constants_are_parameters():
    # hand-worked with 2 remembered misses, radius 8, 2 near misses needed, cap 16: misses at
    # 10 and 14 open probation streams (10 has no near history, 14 has one: 10); at 18 the
    # ring holds 10 and 14, both within 8 -> aligned chunk [16, 32); at 100 the ring holds
    # 14 and 18 (10 was forgotten), neither near -> probation
    m = PolicyModel(nframes=256, page_size=4096, ra_init_pages=4, ra_cap_pages=16, streams_per_file=1,
                    recent=2, near_pages=8, near_min=2)
    m.open(0, 1 << 20)
    for p in (10, 14, 18, 100):
        m.gread(0, 0, p * 4096, 4096)
    assert [(e[4], e[5]) for e in _misses(m.events)] == [(10, 1), (14, 1), (16, 16), (100, 1)]
    assert [(n, r) for n, _, r in m.decisions] == [(0, 4), (1, 4), (2, 2), (0, 4)]
    # the same reads under the default constants (3 near misses within 64 needed): no chunk
    m2 = PolicyModel(nframes=256, page_size=4096, ra_init_pages=4, ra_cap_pages=16, streams_per_file=1)
    m2.open(0, 1 << 20)
    for p in (10, 14, 18):
        m2.gread(0, 0, p * 4096, 4096)
    assert [(e[4], e[5]) for e in _misses(m2.events)] == [(10, 1), (14, 1), (18, 1)]


def test_thrash_guard_caps_windows_at_one_blocks_share():
    from oracle.policy import quota_cap
    # Sec. 5.1's quota: cache pages over the resident blocks (the smaller of the launch's
    # grid and the resident count)
    assert quota_cap(256, 16384, 1024, 512) == 32
    assert quota_cap(16, 16384, 1024, 512) == 16
    assert quota_cap(64, 8192, 1024, 512) == 16
    assert quota_cap(64, 8192, 8, 512) == 64
    assert quota_cap(16, 64, 1024, 512) == 1
    assert quota_cap(16, 64, 1024, 1) == 16


def test_request_is_the_unmapped_run_around_the_miss():
    # window [0, 8) with page 5 already cached: the miss at 0 fetches the run [0, 5) only
    m = PolicyModel(nframes=64, page_size=4096, ra_init_pages=8, ra_cap_pages=8, streams_per_file=1)
    m.open(0, 1 << 20)
    m.gread(0, 0, 5 * 4096, 4096)                  # page 5: probation window of 1
    m.gread(0, 0, 0, 4096)                         # page 0: W0 = 8 -> [0, 8), run stops at 5
    assert [e for e in m.events if e[0] == "REQ"][-1] == ("REQ", 0, 0, 5)


# ---- asynchronous (marker-triggered) readahead ---------------------------------------------------

def _async_closed_form(npages, W0, cap):
    """Linux-style asynchronous readahead on one stream read page by page from offset 0, in
    closed form (Sec. 2.3): the demand miss at page 0 fetches [0, W0) and marks page 1; each
    marker triggers the next window, twice the last one up to the cap, starting where the last
    one ended, whose first page is the next marker. Returns the (trigger page, start, length)
    of every asynchronous window, lengths cut at the end of the file. (W0 >= 2: a first
    window of one page has no page after the demanded one to mark.)"""
    out = []
    start, size, trigger = W0, min(2 * W0, cap), 1
    while True:
        out.append((trigger, start, max(0, min(size, npages - start))))
        if start >= npages:
            return out
        trigger, start, size = start, start + size, min(2 * size, cap)


@pytest.mark.parametrize("npages,W0,cap", [(100, 4, 16), (37, 2, 8), (5, 4, 4), (64, 2, 64)])
def test_async_single_stream_closed_form(npages, W0, cap):
    m = PolicyModel(nframes=256, page_size=1 << 16, ra_init_pages=W0, ra_cap_pages=cap, ra_async=True)
    m.open(0, npages << 16)
    for p in range(npages):
        m.gread(0, 0, p << 16, 1 << 16)
    adv = [(e[3], e[4], e[5]) for e in m.events if e[0] == "ADV"]
    assert adv == _async_closed_form(npages, W0, cap)
    # one demand miss; every later page was fetched ahead of its reader and hit
    assert m.misses == 1 and m.hits == npages - 1 and m.joins == 0
    assert m.fetched_pages == npages and m.wasted_pages == 0
    reqs = [e for e in m.events if e[0] == "REQ"]
    assert reqs[0] == ("REQ", 0, 0, min(W0, npages))
    assert [(e[2], e[3]) for e in reqs[1:]] == [(s, n) for _, s, n in adv if n > 0]
    m.check_invariants()


def test_async_window_runs_ahead_of_synchronous():
    # the same stream: synchronous readahead waits at the start of every window (a miss
    # each), asynchronous readahead only at page 0
    npages, W0, cap = 200, 4, 16
    counts = {}
    for mode in (False, True):
        m = PolicyModel(nframes=512, page_size=4096, ra_init_pages=W0, ra_cap_pages=cap, ra_async=mode)
        m.open(0, npages * 4096)
        for p in range(npages):
            m.gread(0, 0, p * 4096, 4096)
        counts[mode] = (m.misses, m.requests, m.fetched_pages)
    sync_windows = 1 + (npages - W0 - 8 - 16 + 15) // 16 + 2   # 4, 8, 16, 16, ...
    assert counts[False][0] == counts[False][1] == sync_windows
    assert counts[True][0] == 1 and counts[True][2] == counts[False][2] == npages


def test_async_large_read_joins_its_own_window():
    # one block reading 32 pages at a time (cap 16): the first read's miss at 0 takes the cap,
    # [0, 16) (the read asks for 32); its marker page 1 issues [16, 32); the read reaches that
    # window while it is still being filled, joins its first page, whose mark issues [32, 48)
    m = PolicyModel(nframes=512, page_size=1 << 16, ra_init_pages=4, ra_cap_pages=16, ra_async=True)
    m.open(0, 96 << 16)
    for k in range(3):
        m.gread(0, 0, (32 * k) << 16, 32 << 16)
    ev = [e for e in m.events if e[0] in ("MISS", "ADV", "JOIN")]
    assert ev[:4] == [("MISS", 0, 0, 0, 0, 16), ("ADV", 0, 0, 1, 16, 16), ("JOIN", 0, 0, 16, ev[2][4]),
                      ("ADV", 0, 0, 16, 32, 16)]
    # a read joins only the first page of a window it triggered itself (16 in the first read,
    # whose last window [32, 48) arrives when it ends; 48 and 80 in the later reads, each
    # started by the marker of the window the previous read left behind); all 96 pages
    # delivered, none wasted
    joins = [e[3] for e in m.events if e[0] == "JOIN"]
    assert joins == [16, 48, 80]
    assert m.misses == 1 and m.fetched_pages == 96 and m.wasted_pages == 0
    m.check_invariants()


def test_async_marker_dropped_with_its_stream():
    # one stream slot: a second reader's miss takes the slot, so the first stream's marker page
    # no longer names any stream and its access advances nothing
    m = PolicyModel(nframes=256, page_size=4096, ra_init_pages=4, ra_cap_pages=8, streams_per_file=1,
                    ra_async=True)
    m.open(0, 1000 * 4096)
    m.gread(0, 0, 0, 4096)              # stream at 0: window [0, 4), marker 1
    m.gread(1, 0, 500 * 4096, 4096)     # new stream at 500 takes the only slot
    m.gread(0, 0, 4096, 4096)           # page 1: marked, but no stream names it
    assert [e for e in m.events if e[0] == "ADV"] == []
    assert m.frames[m.map[(0, 1)]].mark == 0


def test_async_off_by_default_and_random_advice():
    m = PolicyModel(nframes=256, page_size=4096, ra_init_pages=4, ra_cap_pages=8, ra_async=True)
    m.open(0, 100 * 4096, advice="random")
    for p in range(20):
        m.gread(0, 0, p * 4096, 4096)
    assert m.advances == 0 and m.misses == 20 and m.fetched_pages == 20
